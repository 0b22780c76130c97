// Device helpers shared by the MTP kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Compiler-only memory fence placed between the contraction blocks of the generated
// programs: it keeps the moment loads of a block from being hoisted above earlier blocks,
// which would otherwise make every moment live at once and spill registers.
#define MTP_BLOCK_FENCE() __builtin_amdgcn_sched_barrier(0)

namespace mtp {

constexpr int kMaxCheb = 16;
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies, blocks dispatched round-robin

// Workgroups are dispatched to the XCDs round-robin.  Give each XCD a contiguous range of
// logical blocks so that spatially close atoms (and their shared neighbours) meet in one L2.
__device__ __forceinline__ int xcd_logical_block(int hw, int nb) {
  const int q = nb / kNumXcd, r = nb % kNumXcd;
  const int x = hw % kNumXcd, k = hw / kNumXcd;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Species index kept inside the coefficient tables whatever the input holds (the neighbour
// build rejects out-of-range species; this only guards memory).
__device__ __forceinline__ int clamp_species(int z, int nsp) { return min(max(z, 0), nsp - 1); }

__device__ __forceinline__ void unpack_shift(int w, int& n1, int& n2, int& n3) {
  n1 = (int)(int8_t)(w & 0xFF);
  n2 = (int)(int8_t)((w >> 8) & 0xFF);
  n3 = (int)(int8_t)((w >> 16) & 0xFF);
}

// d = (R_j - R_i) + ((n1 H0 + n2 H1) + n3 H2), binary64 round-to-nearest, no contraction.
// This is the expression of the canonical neighbour predicate; every kernel forms pair
// displacements with it so that mirrored pairs are exact negatives.
__device__ __forceinline__ void pair_displacement(double rix, double riy, double riz, double rjx,
                                                  double rjy, double rjz, int n1, int n2, int n3,
                                                  const double* __restrict__ H, double& dx,
                                                  double& dy, double& dz) {
#pragma clang fp contract(off)
  const double f1 = (double)n1, f2 = (double)n2, f3 = (double)n3;
  const double t0 = (f1 * H[0] + f2 * H[3]) + f3 * H[6];
  const double t1 = (f1 * H[1] + f2 * H[4]) + f3 * H[7];
  const double t2 = (f1 * H[2] + f2 * H[5]) + f3 * H[8];
  dx = (rjx - rix) + t0;
  dy = (rjy - riy) + t1;
  dz = (rjz - riz) + t2;
}

__device__ __forceinline__ double dist2_exact(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}

// Radial functions of one pair: f_mu = w^2 A_mu, f'_mu = w (a w D_mu - 2 A_mu), with
// A_mu = sum_b c_mu,b T_b(u), D_mu = sum_b c_mu,b T'_b(u), w = r_cut - r, u = a r + b0.
// c points at c[z_i][z_j][0][0] (n_mu x n_cheb, row-major).  NC > 0 fixes the Chebyshev count
// at compile time (the recurrence unrolls and the coefficient loads issue together); NC == 0
// takes it from ncheb.  Both forms perform the same operations in the same order.
template <class R, int NMU, int NC = 0>
__device__ __forceinline__ void radial(R r, R sa, R sb, R rcut, const R* __restrict__ c, int ncheb,
                                       R* __restrict__ f, R* __restrict__ fp) {
  const int nc = NC > 0 ? NC : ncheb;
  const R u = fma(sa, r, sb);
  const R w = rcut - r;
  R A[NMU], D[NMU];
#pragma unroll
  for (int mu = 0; mu < NMU; ++mu) {
    A[mu] = c[mu * nc];
    D[mu] = R(0);
  }
  R t_2 = R(1), t_1 = u, d_2 = R(0), d_1 = R(1);
  if (nc > 1) {
#pragma unroll
    for (int mu = 0; mu < NMU; ++mu) {
      A[mu] = fma(c[mu * nc + 1], t_1, A[mu]);
      D[mu] = D[mu] + c[mu * nc + 1];
    }
  }
#pragma unroll
  for (int b = 2; b < nc; ++b) {
    const R t = fma(R(2) * u, t_1, -t_2);
    const R d = fma(R(2) * u, d_1, fma(R(2), t_1, -d_2));
#pragma unroll
    for (int mu = 0; mu < NMU; ++mu) {
      A[mu] = fma(c[mu * nc + b], t, A[mu]);
      D[mu] = fma(c[mu * nc + b], d, D[mu]);
    }
    t_2 = t_1;
    t_1 = t;
    d_2 = d_1;
    d_1 = d;
  }
  const R w2 = w * w;
#pragma unroll
  for (int mu = 0; mu < NMU; ++mu) {
    f[mu] = w2 * A[mu];
    fp[mu] = w * fma(sa * w, D[mu], R(-2) * A[mu]);
  }
}

// Radial function values only.
template <class R, int NMU, int NC = 0>
__device__ __forceinline__ void radial_values(R r, R sa, R sb, R rcut, const R* __restrict__ c,
                                              int ncheb, R* __restrict__ f) {
  const int nc = NC > 0 ? NC : ncheb;
  const R u = fma(sa, r, sb);
  const R w = rcut - r;
  R A[NMU];
#pragma unroll
  for (int mu = 0; mu < NMU; ++mu) A[mu] = c[mu * nc];
  R t_2 = R(1), t_1 = u;
  if (nc > 1) {
#pragma unroll
    for (int mu = 0; mu < NMU; ++mu) A[mu] = fma(c[mu * nc + 1], t_1, A[mu]);
  }
#pragma unroll
  for (int b = 2; b < nc; ++b) {
    const R t = fma(R(2) * u, t_1, -t_2);
#pragma unroll
    for (int mu = 0; mu < NMU; ++mu) A[mu] = fma(c[mu * nc + b], t, A[mu]);
    t_2 = t_1;
    t_1 = t;
  }
  const R w2 = w * w;
#pragma unroll
  for (int mu = 0; mu < NMU; ++mu) f[mu] = w2 * A[mu];
}

// Atom handled by sweep position k, and its cell (kernel-argument copy for one system, the
// configuration's row of the cell table for batches).
template <class A>
__device__ __forceinline__ int atom_at(const A& a, int k) {
  return a.perm ? a.perm[k] : k;
}
template <class A>
__device__ __forceinline__ void load_cell(const A& a, int i, double* H) {
  const double* src = a.cfg ? a.cells + 9L * a.cfg[i] : a.H;
#pragma unroll
  for (int k = 0; k < 9; ++k) H[k] = src[k];
}

// Fixed-order tree sum of a workgroup's values (deterministic); blockDim.x a power of two.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* __restrict__ sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double out = sh[0];
  __syncthreads();
  return out;
}

}  // namespace mtp
