// Neighbourhood-mode extrapolation grade: grade_i = max_k |sum_alpha B[alpha][i] Ainv[alpha][k]|
// on the matrix cores, with the row max-abs taken in the epilogue (the product never leaves
// registers).  B comes in [alpha][atom] layout (one chunk), Ainv is row-major n x n.
//
// One wave owns a tile of 16 atoms and sweeps the columns of Ainv in blocks of 8 MFMA tiles
// (128 columns).  V_MFMA_F64_16X16X4F64 operand layout (wave64): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; its accumulator register r holds
// D[4 r + l / 16][l % 16], r = 0..3.  The FP32-split variant splits both operands into
// binary32 hi + lo parts, forms hi*hi + hi*lo + lo*hi with V_MFMA_F32_16X16X4F32 (same input
// layout, but register r holds D[4 (l / 16) + r][l % 16]) and adds every K=4 partial into
// binary64 accumulators.  Both output layouts are checked on the device by the grade parity
// tests.
#include <hip/hip_runtime.h>

#include "mtp_device.h"
#include "mtp_internal.h"

namespace mtp {
namespace {

constexpr int kWaves = 4;           // waves per workgroup, one 16-atom tile each
constexpr int kTilesPerBlock = 8;   // 16-column MFMA tiles per column sweep

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double max16(double v) {
  // max over the 16 lanes that share l / 16 (xor shuffles stay inside the 16-lane group)
#pragma unroll
  for (int s = 8; s > 0; s >>= 1) v = fmax(v, __shfl_xor(v, s, 64));
  return v;
}

template <bool SPLIT>
__global__ __launch_bounds__(64 * kWaves) void k_grade(const double* __restrict__ B, long ld, int n,
                                                       const double* __restrict__ ainv, int na,
                                                       double* __restrict__ grade) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int tile = xcd_logical_block(blockIdx.x, gridDim.x) * kWaves + wave;
  const int i0 = tile * 16;
  if (i0 >= n) return;
  const int row = lane & 15;      // atom row supplied as A operand / column of D
  const int kq = lane >> 4;       // k index inside a K=4 step, and row quad of D
  const int atom = i0 + row;
  const bool atom_ok = atom < n;
  double rmax[4] = {0.0, 0.0, 0.0, 0.0};
  const int ksteps = (na + 3) / 4;
  for (int c0 = 0; c0 < na; c0 += 16 * kTilesPerBlock) {
    v4d acc[kTilesPerBlock];
#pragma unroll
    for (int t = 0; t < kTilesPerBlock; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int ks = 0; ks < ksteps; ++ks) {
      const int k = ks * 4 + kq;
      const double a = (atom_ok && k < na) ? B[(long)k * ld + atom] : 0.0;
      float ah = 0.f, al = 0.f;
      if (SPLIT) {
        ah = (float)a;
        al = (float)(a - (double)ah);
      }
#pragma unroll
      for (int t = 0; t < kTilesPerBlock; ++t) {
        const int col = c0 + t * 16 + row;
        const double b = (k < na && col < na) ? ainv[(long)k * na + col] : 0.0;
        if (!SPLIT) {
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
        } else {
          const float bh = (float)b;
          const float bl = (float)(b - (double)bh);
          v4f p = v4f{0.f, 0.f, 0.f, 0.f};
          p = __builtin_amdgcn_mfma_f32_16x16x4f32(ah, bh, p, 0, 0, 0);
          v4f q = v4f{0.f, 0.f, 0.f, 0.f};
          q = __builtin_amdgcn_mfma_f32_16x16x4f32(ah, bl, q, 0, 0, 0);
          q = __builtin_amdgcn_mfma_f32_16x16x4f32(al, bh, q, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[t][r] += (double)p[r] + (double)q[r];
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kTilesPerBlock; ++t) {
      const int col = c0 + t * 16 + row;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double v = col < na ? fabs(acc[t][r]) : 0.0;
        rmax[r] = fmax(rmax[r], v);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double m = max16(rmax[r]);
    const int out = SPLIT ? i0 + 4 * kq + r : i0 + 4 * r + kq;
    if (row == 0 && out < n) grade[out] = m;
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
  if (n <= 0) return;
  const int tiles = (n + 15) / 16;
  const int nb = (tiles + kWaves - 1) / kWaves;
  if (split)
    hipLaunchKernelGGL((k_grade<true>), dim3(nb), dim3(64 * kWaves), 0, s, B, ld, n, ainv, na, grade);
  else
    hipLaunchKernelGGL((k_grade<false>), dim3(nb), dim3(64 * kWaves), 0, s, B, ld, n, ainv, na, grade);
}

void launch_max(const double* x, long n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_max, dim3(1), dim3(1024), 0, s, x, n, out);
}

}  // namespace mtp
