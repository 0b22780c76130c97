// Level-independent kernels: force gather through the mirrored-pair index and fixed-order
// (deterministic) reductions of site energies and virial partials.
#include <hip/hip_runtime.h>

#include "mtp_device.h"
#include "mtp_internal.h"

namespace mtp {
namespace {

constexpr int kNT = 256;
constexpr int kSumThreads = 1024;

// F_k = sum over row k of (g[p] - g[rev[p]]): the atom's own pair gradients minus the
// gradients of the pairs that have k as neighbour (newton's third law through rev).
__global__ void k_gather(const int* __restrict__ off, const int* __restrict__ rev,
                         const double* __restrict__ g, int n, long long npairs,
                         double* __restrict__ f) {
  const int b = xcd_logical_block(blockIdx.x, gridDim.x);
  const int k = b * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  for (int p = off[k]; p < off[k + 1]; ++p) {
    fx += g[3L * p];
    fy += g[3L * p + 1];
    fz += g[3L * p + 2];
    const long q = rev[p];
    if (q >= 0 && q < npairs) {  // a list not made by this library may lack mirrors
      fx -= g[3 * q];
      fy -= g[3 * q + 1];
      fz -= g[3 * q + 2];
    }
  }
  f[3L * k] = fx;
  f[3L * k + 1] = fy;
  f[3L * k + 2] = fz;
}

// one workgroup: thread t sums x[t], x[t + T], ... then a fixed tree
__global__ __launch_bounds__(kSumThreads) void k_sum(const double* __restrict__ x, long n,
                                                     long stride, double* __restrict__ out) {
  __shared__ double sh[kSumThreads];
  double acc = 0.0;
  for (long i = threadIdx.x; i < n; i += kSumThreads) acc += x[i * stride];
  const double s = block_sum<kSumThreads>(acc, sh);
  if (threadIdx.x == 0) out[0] = s;
}

// out[r * os] = sum_{k < n} x[r * rs + k * es] for each row r (one workgroup per row, fixed order)
__global__ __launch_bounds__(kNT) void k_rowsum(const double* __restrict__ x, long rs, long es, long n,
                                                double* __restrict__ out, long os) {
  __shared__ double sh[kNT];
  const double* row = x + (long)blockIdx.x * rs;
  double acc = 0.0;
  for (long k = threadIdx.x; k < n; k += kNT) acc += row[k * es];
  const double v = block_sum<kNT>(acc, sh);
  if (threadIdx.x == 0) out[(long)blockIdx.x * os] = v;
}

// d(ebar E + fbar.F)/ds_t = ebar * (number of atoms of species t); integer counts are exact
__global__ __launch_bounds__(kNT) void k_species_grad(const int* __restrict__ species, int n, int nsp,
                                                      double ebar, double* __restrict__ out) {
  __shared__ int cnt[16];
  if (threadIdx.x < 16) cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kNT) {
    const int z = species[i];
    if (z >= 0 && z < nsp) atomicAdd(&cnt[z], 1);
  }
  __syncthreads();
  if (threadIdx.x < nsp) out[threadIdx.x] = ebar * (double)cnt[threadIdx.x];
}

}  // namespace

void launch_rowsum(const double* x, long rs, long es, long n, int rows, double* out, long os,
                   hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_rowsum, dim3(rows), dim3(kNT), 0, s, x, rs, es, n, out, os);
}

void launch_species_grad(const int* species, int n, int nsp, double ebar, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_species_grad, dim3(1), dim3(kNT), 0, s, species, n, nsp, ebar, out);
}

void launch_gather_forces(const int* off, const int* rev, const double* g, int n, long long npairs,
                          double* forces, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3((n + kNT - 1) / kNT), dim3(kNT), 0, s, off, rev, g, n, npairs,
                     forces);
}

void launch_sum(const double* x, long n, long stride, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kSumThreads), 0, s, x, n, stride, out);
}

void launch_sum_virial(const double* wpart, long nblocks, double* out, hipStream_t s) {
  for (int k = 0; k < 6; ++k)
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kSumThreads), 0, s, wpart + k, nblocks, 6L, out + k);
}

}  // namespace mtp
