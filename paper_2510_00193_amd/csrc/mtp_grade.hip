// Neighbourhood-mode extrapolation grade: grade_i = max_k |sum_alpha B[alpha][i] Ainv[alpha][k]|
// on the matrix cores, with the row max-abs taken in the epilogue (the product never leaves
// registers).  B comes in [alpha][atom] layout (one chunk), Ainv is row-major n x n.
//
// A workgroup of several waves stages a panel of Ainv (all rows, up to kPanelBytes of columns,
// zero-padded to whole 16x16 tiles) in LDS once and keeps it there while its waves walk their
// 16-atom tiles (a grid of about one workgroup per CU): every MFMA takes its Ainv operand from
// LDS and the atom operand from B, loaded kRing K steps ahead (global-memory latency is
// several K steps of MFMA work).  Panels after the first fold
// their row maxima into the grades already written.
// V_MFMA_F64_16X16X4F64 operand layout (wave64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; its accumulator register r holds D[4 r + l / 16][l % 16], r = 0..3.  The
// FP32-split variant splits both operands into binary32 hi + lo parts, forms
// hi*hi + hi*lo + lo*hi with V_MFMA_F32_16X16X4F32 (same input layout, but register r holds
// D[4 (l / 16) + r][l % 16]) and adds every K=4 partial into binary64 accumulators.  Both
// output layouts are checked on the device by the grade parity tests.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mtp_device.h"
#include "mtp_internal.h"

namespace mtp {
namespace {

// Workgroup shape per form (measured at 250,000 atoms, level 16): the binary64 form runs four
// waves of one 16-atom tile per SIMD (0.168 ms, against 0.175 ms for two waves of two tiles);
// the split form, with three products per tile, two waves of two tiles (0.375 vs 0.404 ms).
template <bool SPLIT>
struct GradeShape {
  static constexpr int waves = SPLIT ? 8 : 16;  // waves per workgroup
  static constexpr int tpw = SPLIT ? 2 : 1;     // 16-atom tiles per wave
};
constexpr int kMaxTiles = 8;          // 16-column MFMA tiles per column sweep
constexpr int kPanelBytes = 120 * 1024;  // LDS panel of Ainv
constexpr int kRing = 4;              // K steps of atom operands loaded ahead
constexpr int kResMax = 4;            // last columns (beyond whole 16-column tiles) taken on VALU

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double max16(double v) {
  // max over the 16 lanes that share l / 16 (xor shuffles stay inside the 16-lane group)
#pragma unroll
  for (int s = 8; s > 0; s >>= 1) v = fmax(v, __shfl_xor(v, s, 64));
  return v;
}

// One panel: columns [c_lo, c_lo + pw) of Ainv, pw a multiple of 16; kp = na rounded up to 4.
// A wave takes kTpw 16-atom tiles at once, so every Ainv operand read from LDS feeds kTpw MFMAs
// (three per tile in the split form).
// In the split form, when the panel's valid columns end at most kResMax columns past a whole
// 16-column tile, those columns are not padded to a tile of three binary32 products: each lane
// accumulates them with binary64 FMAs over its own K slice (the atom operand it already holds),
// and the four K slices of an atom are summed with lane exchanges after the K loop.  (In the
// binary64 form the padded tile costs less than the VALU columns.)
template <bool SPLIT>
__global__ __launch_bounds__(64 * GradeShape<SPLIT>::waves) void k_grade(const double* __restrict__ B, long ld, int n,
                                                       const double* __restrict__ ainv, int na, int c_lo,
                                                       int pw, int first, double* __restrict__ grade) {
  constexpr int kWaves = GradeShape<SPLIT>::waves, kTpw = GradeShape<SPLIT>::tpw;
  extern __shared__ double sa[];  // [kp][pw]
  const int kp = (na + 3) & ~3;
  for (int idx = threadIdx.x; idx < kp * pw; idx += 64 * kWaves) {
    const int k = idx / pw, c = c_lo + idx % pw;
    sa[idx] = (k < na && c < na) ? ainv[(long)k * na + c] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int row = lane & 15;      // atom row supplied as A operand / column of D
  const int kq = lane >> 4;       // k index inside a K=4 step, and row quad of D
  const int ksteps = kp / 4;
  const int valid = min(pw, na - c_lo);
  int mcols = valid / 16 * 16, nres = valid - mcols;  // matrix-core columns, VALU columns
  if (nres > kResMax || (!SPLIT && nres > 0)) {  // binary64 matrix cores: padding measured faster
    mcols += 16;
    nres = 0;
  }
  const int ngroups = (n + 16 * kTpw - 1) / (16 * kTpw);
  const int stride = gridDim.x * kWaves;
  for (int grp = xcd_logical_block(blockIdx.x, gridDim.x) * kWaves + wave; grp < ngroups; grp += stride) {
    const int i0 = grp * 16 * kTpw;
    bool atom_ok[kTpw];
    const double* bp[kTpw];
#pragma unroll
    for (int h = 0; h < kTpw; ++h) {
      atom_ok[h] = i0 + 16 * h + row < n;
      bp[h] = B + i0 + 16 * h + row;
    }
    double rmax[kTpw][4], res[kTpw][kResMax];
#pragma unroll
    for (int h = 0; h < kTpw; ++h) {
#pragma unroll
      for (int r = 0; r < 4; ++r) rmax[h][r] = 0.0;
#pragma unroll
      for (int c = 0; c < kResMax; ++c) res[h][c] = 0.0;
    }
    // the VALU columns ride along the first column sweep, which loads the atom operands anyway
    for (int c0 = 0; c0 < max(mcols, 1); c0 += 16 * kMaxTiles) {
      const int nt = min(kMaxTiles, (mcols - c0) / 16);
      v4d acc[kTpw][kMaxTiles];
#pragma unroll
      for (int h = 0; h < kTpw; ++h)
#pragma unroll
        for (int t = 0; t < kMaxTiles; ++t) acc[h][t] = v4d{0.0, 0.0, 0.0, 0.0};
      // atom operands of the next kRing K steps in flight (one global load per lane, tile and step)
      double ar[kTpw][kRing];
#pragma unroll
      for (int h = 0; h < kTpw; ++h)
#pragma unroll
        for (int u = 0; u < kRing; ++u) {
          const int k = u * 4 + kq;
          ar[h][u] = (atom_ok[h] && k < na) ? bp[h][(long)k * ld] : 0.0;
        }
      for (int ks0 = 0; ks0 < ksteps; ks0 += kRing) {
#pragma unroll
        for (int u = 0; u < kRing; ++u) {
          const int ks = ks0 + u;
          if (ks < ksteps) {
            double a[kTpw];
            float ah[kTpw], al[kTpw];
            const int kn = (ks + kRing) * 4 + kq;
#pragma unroll
            for (int h = 0; h < kTpw; ++h) {
              a[h] = ar[h][u];
              ar[h][u] = (atom_ok[h] && kn < na) ? bp[h][(long)kn * ld] : 0.0;
              ah[h] = 0.f;
              al[h] = 0.f;
              if (SPLIT) {
                ah[h] = (float)a[h];
                al[h] = (float)(a[h] - (double)ah[h]);
              }
            }
            const double* srow = sa + (ks * 4 + kq) * pw + c0 + row;
            if (c0 == 0 && nres > 0) {
              const double* rrow = sa + (ks * 4 + kq) * pw + mcols;
#pragma unroll
              for (int c = 0; c < kResMax; ++c) {
                if (c < nres) {
                  const double bv = rrow[c];
#pragma unroll
                  for (int h = 0; h < kTpw; ++h) res[h][c] = fma(a[h], bv, res[h][c]);
                }
              }
            }
#pragma unroll
            for (int t = 0; t < kMaxTiles; ++t) {
              if (t < nt) {
                const double b = srow[t * 16];
                if (!SPLIT) {
#pragma unroll
                  for (int h = 0; h < kTpw; ++h)
                    acc[h][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h], b, acc[h][t], 0, 0, 0);
                } else {
                  const float bh = (float)b;
                  const float bl = (float)(b - (double)bh);
#pragma unroll
                  for (int h = 0; h < kTpw; ++h) {
                    v4f p = v4f{0.f, 0.f, 0.f, 0.f};
                    p = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[h], bh, p, 0, 0, 0);
                    v4f q = v4f{0.f, 0.f, 0.f, 0.f};
                    q = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[h], bl, q, 0, 0, 0);
                    q = __builtin_amdgcn_mfma_f32_16x16x4f32(al[h], bh, q, 0, 0, 0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[h][t][r] += (double)p[r] + (double)q[r];
                  }
                }
              }
            }
          }
        }
      }
#pragma unroll
      for (int t = 0; t < kMaxTiles; ++t) {
        if (t < nt) {
          const int col = c_lo + c0 + t * 16 + row;
#pragma unroll
          for (int h = 0; h < kTpw; ++h)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const double v = col < na ? fabs(acc[h][t][r]) : 0.0;
              rmax[h][r] = fmax(rmax[h][r], v);
            }
        }
      }
    }
    // VALU columns: sum the four K slices of each atom (lanes row, row + 16, row + 32, row + 48),
    // then the largest magnitude over the columns, held by every lane of the atom
    double mres[kTpw];
#pragma unroll
    for (int h = 0; h < kTpw; ++h) {
      mres[h] = 0.0;
#pragma unroll
      for (int c = 0; c < kResMax; ++c) {
        double v = res[h][c];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (c < nres) mres[h] = fmax(mres[h], fabs(v));
      }
    }
#pragma unroll
    for (int h = 0; h < kTpw; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = SPLIT ? 4 * kq + r : 4 * r + kq;  // atom of the tile whose row max this is
        const double m = fmax(max16(rmax[h][r]), __shfl(mres[h], a, 64));
        const int out = i0 + 16 * h + a;
        if (row == 0 && out < n) grade[out] = first ? m : fmax(grade[out], m);
      }
  }
}

// max over grade[0..n) into out[0] (order-independent)
__global__ __launch_bounds__(1024) void k_max(const double* __restrict__ x, long n, double* __restrict__ out) {
  __shared__ double sh[1024];
  double m = 0.0;
  for (long i = threadIdx.x; i < n; i += 1024) m = fmax(m, x[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// Configuration-mode grade: out[0] = max_k |sum_alpha b[alpha] ainv[alpha][k]| for one
// descriptor b [na] (one workgroup; each thread owns columns k, reads rows of ainv coalesced).
__global__ __launch_bounds__(1024) void k_cfg_grade(const double* __restrict__ b, const double* __restrict__ ainv,
                                                    int na, double* __restrict__ out) {
  __shared__ double sh[1024];
  double m = 0.0;
  for (int k = threadIdx.x; k < na; k += 1024) {
    double v = 0.0;
    for (int a = 0; a < na; ++a) v = fma(b[a], ainv[(long)a * na + k], v);
    m = fmax(m, fabs(v));
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

}  // namespace

void launch_cfg_grade(const double* b, const double* ainv, int na, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cfg_grade, dim3(1), dim3(1024), 0, s, b, ainv, na, out);
}

void launch_grade(const double* B, long ld, int n, const double* ainv, int na, int split,
                  double* grade, hipStream_t s) {
  if (n <= 0 || na <= 0) return;
  const int kp = (na + 3) & ~3;
  const int ncol = (na + 15) / 16 * 16;
  int pw = (int)(kPanelBytes / (sizeof(double) * kp)) / 16 * 16;
  pw = std::max(16, std::min(pw, ncol));
  const int waves = split ? GradeShape<true>::waves : GradeShape<false>::waves;
  const int tpw = split ? GradeShape<true>::tpw : GradeShape<false>::tpw;
  const int groups = (n + 16 * tpw - 1) / (16 * tpw);
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int nb = std::max(1, std::min((groups + waves - 1) / waves, ncu));
  const size_t lds = sizeof(double) * kp * pw;
  static bool attr_set = false;  // allow the panel beyond the default dynamic LDS limit
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_grade<true>, hipFuncAttributeMaxDynamicSharedMemorySize, kPanelBytes);
    (void)hipFuncSetAttribute((const void*)k_grade<false>, hipFuncAttributeMaxDynamicSharedMemorySize, kPanelBytes);
    attr_set = true;
  }
  for (int c = 0; c < ncol; c += pw) {
    const int w = std::min(pw, ncol - c);
    if (split)
      hipLaunchKernelGGL((k_grade<true>), dim3(nb), dim3(64 * waves), lds, s, B, ld, n, ainv, na, c, w, c == 0, grade);
    else
      hipLaunchKernelGGL((k_grade<false>), dim3(nb), dim3(64 * waves), lds, s, B, ld, n, ainv, na, c, w, c == 0, grade);
  }
}

void launch_max(const double* x, long n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_max, dim3(1), dim3(1024), 0, s, x, n, out);
}

}  // namespace mtp
