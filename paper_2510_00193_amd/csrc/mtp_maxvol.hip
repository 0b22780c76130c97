// Active-set update by MaxVol row swaps (the D-optimality / MaxVol basis of the MTP's
// extrapolation grade; the iteration of Goreinov et al. 2010).
//
// One iteration on the device, candidates C [m][n], active set A [n][n], Ainv = A^-1:
//   1. k_rowmax: for every candidate row i, the largest |(c_i Ainv)_k| and the first k reaching
//      it, with the product on binary64 matrix cores (a wave takes 16 rows, column tiles of 16);
//   2. k_argmax_part / k_argmax_final: the first row (row-major order) reaching the largest value;
//   3. k_swap: g = (c_i Ainv)_k; row r = c_i Ainv is formed in LDS, Ainv is updated by
//      Sherman-Morrison for replacing row k of A by c_i,
//        Ainv' = Ainv - Ainv[:, k] (r - e_k) / g,
//      and rows A[k] and C[i] are exchanged.
// The host reads (i, k, g) once per iteration and stops when |g| <= 1 + tol.
#include <hip/hip_runtime.h>
#include <math.h>

#include <cmath>

#include <string>

#include "mtp.h"
#include "mtp_api_internal.h"
#include "mtp_device.h"
#include "mtp_internal.h"

namespace mtp {
namespace {

constexpr int kRowWaves = 4;
constexpr int kNT = 256;
constexpr int kArgParts = 256;

typedef double v4d __attribute__((ext_vector_type(4)));

// (value, index) pair kept by the larger value, then the smaller index
__device__ __forceinline__ void keep_max(double& v, int& k, double v2, int k2) {
  if (v2 > v || (v2 == v && k2 < k)) {
    v = v2;
    k = k2;
  }
}

// V_MFMA_F64_16X16X4F64 layout (wave64): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator register r holds D[4 r + l / 16][l % 16].
__global__ __launch_bounds__(64 * kRowWaves) void k_rowmax(const double* __restrict__ C, int m, int n,
                                                           const double* __restrict__ ainv,
                                                           double* __restrict__ rmax, int* __restrict__ rarg) {
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * kRowWaves + (threadIdx.x >> 6);
  const int i0 = tile * 16;
  if (i0 >= m) return;
  const int row = lane & 15, kq = lane >> 4;
  const int ci = i0 + row;
  double best[4];
  int bk[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    best[r] = -1.0;
    bk[r] = 0x7FFFFFFF;
  }
  for (int c0 = 0; c0 < n; c0 += 16) {
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
    const int col = c0 + row;
    for (int k0 = 0; k0 < n; k0 += 4) {
      const int k = k0 + kq;
      const double a = (ci < m && k < n) ? C[(long)ci * n + k] : 0.0;
      const double b = (k < n && col < n) ? ainv[(long)k * n + col] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // a NaN product counts as the largest magnitude, so that it is selected and reported
      const double v = fabs(acc[r]);
      if (col < n) keep_max(best[r], bk[r], isnan(v) ? INFINITY : v, col);
    }
  }
  // rows 4 r + kq: reduce over the 16 lanes that share kq (the columns)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double v = best[r];
    int k = bk[r];
#pragma unroll
    for (int s = 8; s > 0; s >>= 1) {
      const double v2 = __shfl_xor(v, s, 64);
      const int k2 = __shfl_xor(k, s, 64);
      keep_max(v, k, v2, k2);
    }
    const int out = i0 + 4 * r + kq;
    if (row == 0 && out < m) {
      rmax[out] = v;
      rarg[out] = k;
    }
  }
}

// first row reaching the largest row maximum: per-part (value, row), then one workgroup
__global__ __launch_bounds__(kNT) void k_argmax_part(const double* __restrict__ rmax, int m,
                                                     double* __restrict__ pv, int* __restrict__ pi) {
  __shared__ double sv[kNT];
  __shared__ int si[kNT];
  const long per = (m + kArgParts - 1) / kArgParts;
  const long lo = (long)blockIdx.x * per, hi = min((long)m, lo + per);
  double v = -1.0;
  int id = 0x7FFFFFFF;
  for (long i = lo + threadIdx.x; i < hi; i += kNT) keep_max(v, id, rmax[i], (int)i);
  sv[threadIdx.x] = v;
  si[threadIdx.x] = id;
  __syncthreads();
  for (int s = kNT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      double a = sv[threadIdx.x];
      int b = si[threadIdx.x];
      keep_max(a, b, sv[threadIdx.x + s], si[threadIdx.x + s]);
      sv[threadIdx.x] = a;
      si[threadIdx.x] = b;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = sv[0];
    pi[blockIdx.x] = si[0];
  }
}

// out: [0] = row i, [1] = column k (as doubles), [2] = g = (c_i Ainv)_k (signed).  Every row
// holds a column in [0, n) (column 0 always competes), so i and k are in range; they are still
// clamped, with g set to NaN, should that ever fail.
__global__ __launch_bounds__(kNT) void k_argmax_final(const double* __restrict__ pv, const int* __restrict__ pi,
                                                      const int* __restrict__ rarg, const double* __restrict__ C,
                                                      int m, int n, const double* __restrict__ ainv,
                                                      double* __restrict__ out) {
  __shared__ double sv[kNT];
  __shared__ int si[kNT];
  __shared__ double sg[kNT];
  double v = -1.0;
  int id = 0x7FFFFFFF;
  for (int t = threadIdx.x; t < kArgParts; t += kNT) keep_max(v, id, pv[t], pi[t]);
  sv[threadIdx.x] = v;
  si[threadIdx.x] = id;
  __syncthreads();
  for (int s = kNT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      double a = sv[threadIdx.x];
      int b = si[threadIdx.x];
      keep_max(a, b, sv[threadIdx.x + s], si[threadIdx.x + s]);
      sv[threadIdx.x] = a;
      si[threadIdx.x] = b;
    }
    __syncthreads();
  }
  const bool i_ok = si[0] >= 0 && si[0] < m;
  const int i = i_ok ? si[0] : 0;
  const bool k_ok = i_ok && rarg[i] >= 0 && rarg[i] < n;
  const int k = k_ok ? rarg[i] : 0;
  // signed g = sum_t C[i][t] Ainv[t][k], fixed-order tree over the threads
  double part = 0.0;
  for (int t = threadIdx.x; t < n; t += kNT) part = fma(C[(long)i * n + t], ainv[(long)t * n + k], part);
  const double gs = block_sum<kNT>(part, sg);
  const double g = k_ok ? gs : NAN;
  if (threadIdx.x == 0) {
    out[0] = (double)i;
    out[1] = (double)k;
    out[2] = g;
  }
}

// r = c_i Ainv in LDS; Ainv -= Ainv[:, k] (r - e_k) / g; exchange rows A[k] and C[i].
// One workgroup; the update of Ainv reads column k, which it also writes: the column is staged
// in LDS first.
__global__ __launch_bounds__(1024) void k_swap(double* __restrict__ C, double* __restrict__ A,
                                               double* __restrict__ ainv, int n, const double* __restrict__ sel) {
  extern __shared__ double sm[];  // r [n], column k of Ainv [n]
  double* r = sm;
  double* colk = sm + n;
  const int i = (int)sel[0], k = (int)sel[1];
  const double g = sel[2];
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double s = 0.0;
    for (int t = 0; t < n; ++t) s = fma(C[(long)i * n + t], ainv[(long)t * n + j], s);
    r[j] = s - (j == k ? 1.0 : 0.0);
    colk[j] = ainv[(long)j * n + k];
  }
  __syncthreads();
  const double inv_g = 1.0 / g;
  for (long idx = threadIdx.x; idx < (long)n * n; idx += blockDim.x) {
    const int a = (int)(idx / n), b = (int)(idx % n);
    ainv[idx] = ainv[idx] - colk[a] * (r[b] * inv_g);
  }
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const double x = A[(long)k * n + t];
    A[(long)k * n + t] = C[(long)i * n + t];
    C[(long)i * n + t] = x;
  }
}

}  // namespace
}  // namespace mtp

using namespace mtp;

extern "C" int mtp_maxvol(mtp_model* m, double* cand, int n_cand, int n, double* active, double* ainv, double tol,
                          int max_swaps, int* swaps, double* grades, int* n_swaps, void* stream) {
  if (!m || !n_swaps) return mtp_fail(MTP_ERR_ARG, "null model or swap count");
  *n_swaps = 0;
  if (n < 1 || n > 4096 || n_cand < 0 || max_swaps < 0 || !(tol >= 0.0))
    return mtp_fail(MTP_ERR_ARG, "mtp_maxvol: need 1 <= n <= 4096, n_cand >= 0, max_swaps >= 0, tol >= 0");
  if (!active || !ainv || (n_cand > 0 && !cand)) return mtp_fail(MTP_ERR_ARG, "null matrix");
  if (n_cand == 0 || max_swaps == 0) return MTP_OK;
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if ((rc = m->scratch.reserve((size_t)n_cand * 8 + (size_t)n_cand * 4 + kArgParts * 12 + 64))) return rc;
  double* rmax = (double*)m->scratch.p;
  int* rarg = (int*)(rmax + n_cand);
  double* pv = (double*)((char*)m->scratch.p + (((size_t)n_cand * 12 + 15) & ~(size_t)15));
  int* pi = (int*)(pv + kArgParts);
  double* sel = (double*)(pi + kArgParts + (kArgParts & 1));
  double host[3];
  const int tiles = (n_cand + 15) / 16;
  const int threads = n < 1024 ? ((n + 63) / 64) * 64 : 1024;
  for (int it = 0; it < max_swaps; ++it) {
    hipLaunchKernelGGL(k_rowmax, dim3((tiles + kRowWaves - 1) / kRowWaves), dim3(64 * kRowWaves), 0, s, cand,
                       n_cand, n, ainv, rmax, rarg);
    hipLaunchKernelGGL(k_argmax_part, dim3(kArgParts), dim3(kNT), 0, s, rmax, n_cand, pv, pi);
    hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(kNT), 0, s, pv, pi, rarg, cand, n_cand, n, ainv, sel);
    if (hipGetLastError() != hipSuccess) return mtp_fail(MTP_ERR_HIP, "mtp_maxvol: launch failed");
    if (hipMemcpyAsync(host, sel, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return mtp_fail(MTP_ERR_HIP, "mtp_maxvol: reading the selection failed");
    if (!std::isfinite(host[2]))
      return mtp_fail(MTP_ERR_ARG, "mtp_maxvol: non-finite grade (candidates or inverse not finite)");
    if (!(fabs(host[2]) > 1.0 + tol)) break;
    hipLaunchKernelGGL(k_swap, dim3(1), dim3(threads), 2 * n * sizeof(double), s, cand, active, ainv, n, sel);
    if (hipGetLastError() != hipSuccess) return mtp_fail(MTP_ERR_HIP, "mtp_maxvol: launch failed");
    if (swaps) {
      swaps[2 * it] = (int)host[0];
      swaps[2 * it + 1] = (int)host[1];
    }
    if (grades) grades[it] = host[2];
    *n_swaps = it + 1;
  }
  return MTP_OK;
}
