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
// A group of kGatherLanes lanes owns one atom: its row of g is read contiguously, the mirrored
// entries are gathered, and the group sums with a fixed butterfly (deterministic).  With FOWN
// the own sums come precomputed per atom (accumulated by the pair kernel) and only the
// mirrored gradients are read.
constexpr int kGatherLanes = 16;
constexpr int kGatherUnroll = 2;  // 16 x 2 measured 0.248 ms at 1M atoms; 16 x 1 0.255, 32 x 1 0.291, 8 x 4 0.259

template <bool FOWN>
__global__ __launch_bounds__(kNT) void k_gather(const int* __restrict__ off, const int* __restrict__ rev,
                                                const double* __restrict__ g, const double* __restrict__ fown,
                                                int n, long long npairs, double* __restrict__ f) {
  const int b = xcd_logical_block(blockIdx.x, gridDim.x);
  const int k = b * (kNT / kGatherLanes) + threadIdx.x / kGatherLanes;
  const int lane = threadIdx.x % kGatherLanes;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (k < n) {
    // kGatherUnroll strides per iteration: every mirror index of the iteration is loaded before
    // any gather, so a typical row costs one dependent load pair; a lane still adds its pairs in
    // increasing order
    const int end = off[k + 1];
    for (int p = off[k] + lane; p < end; p += kGatherUnroll * kGatherLanes) {
      long q[kGatherUnroll];
#pragma unroll
      for (int u = 0; u < kGatherUnroll; ++u) {
        const int pu = p + u * kGatherLanes;
        q[u] = pu < end ? rev[pu] : -1;  // every mirror exists: built here or validated on entry
      }
#pragma unroll
      for (int u = 0; u < kGatherUnroll; ++u) {
        if (q[u] < 0) continue;
        const long pu = p + u * kGatherLanes;
        if (!FOWN) {
          fx += g[3 * pu];
          fy += g[3 * pu + 1];
          fz += g[3 * pu + 2];
        }
        fx -= g[3 * q[u]];
        fy -= g[3 * q[u] + 1];
        fz -= g[3 * q[u] + 2];
      }
    }
  }
#pragma unroll
  for (int s = kGatherLanes / 2; s > 0; s >>= 1) {
    fx += __shfl_xor(fx, s, kGatherLanes);
    fy += __shfl_xor(fy, s, kGatherLanes);
    fz += __shfl_xor(fz, s, kGatherLanes);
  }
  if (k < n && lane == 0) {
    if (FOWN) {
      fx = fown[3L * k] + fx;
      fy = fown[3L * k + 1] + fy;
      fz = fown[3L * k + 2] + fz;
    }
    f[3L * k] = fx;
    f[3L * k + 1] = fy;
    f[3L * k + 2] = fz;
  }
}

// Two-level fixed-order sum: kPartBlocks workgroups each sum a fixed contiguous slice, then one
// workgroup sums the partials.  out[c] for components c of a strided array (blockIdx.y).
constexpr int kPartBlocks = 256;

__global__ __launch_bounds__(kNT) void k_sum_part(const double* __restrict__ x, long n, long stride,
                                                  double* __restrict__ part) {
  __shared__ double sh[kNT];
  const int c = blockIdx.y;
  const long per = (n + kPartBlocks - 1) / kPartBlocks;
  const long lo = (long)blockIdx.x * per, hi = min(n, lo + per);
  double acc = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += kNT) acc += x[i * stride + c];
  const double v = block_sum<kNT>(acc, sh);
  if (threadIdx.x == 0) part[(long)c * kPartBlocks + blockIdx.x] = v;
}

__global__ __launch_bounds__(kNT) void k_sum_final(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[kNT];
  const int c = blockIdx.x;
  const double v = block_sum<kNT>(threadIdx.x < kPartBlocks ? part[(long)c * kPartBlocks + threadIdx.x] : 0.0, sh);
  if (threadIdx.x == 0) out[c] = v;
}

// The same two-level sums over two strided arrays at once (components c < nc1 of x1, then the
// nc2 components of x2): one launch of partials and one of totals instead of two each; every
// component's slices and order are those of k_sum_part / k_sum_final.
__global__ __launch_bounds__(kNT) void k_sum_part2(const double* __restrict__ x1, long n1, long st1, int nc1,
                                                   const double* __restrict__ x2, long n2, long st2,
                                                   double* __restrict__ part) {
  __shared__ double sh[kNT];
  const int c = blockIdx.y;
  const bool first = c < nc1;
  const double* x = first ? x1 : x2;
  const long n = first ? n1 : n2, stride = first ? st1 : st2;
  const int comp = first ? c : c - nc1;
  const long per = (n + kPartBlocks - 1) / kPartBlocks;
  const long lo = (long)blockIdx.x * per, hi = min(n, lo + per);
  double acc = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += kNT) acc += x[i * stride + comp];
  const double v = block_sum<kNT>(acc, sh);
  if (threadIdx.x == 0) part[(long)c * kPartBlocks + blockIdx.x] = v;
}

__global__ __launch_bounds__(kNT) void k_sum_final2(const double* __restrict__ part, int nc1,
                                                    double* __restrict__ out1, double* __restrict__ out2) {
  __shared__ double sh[kNT];
  const int c = blockIdx.x;
  const double v = block_sum<kNT>(threadIdx.x < kPartBlocks ? part[(long)c * kPartBlocks + threadIdx.x] : 0.0, sh);
  if (threadIdx.x == 0) {
    if (c < nc1) out1[c] = v;
    else out2[c - nc1] = v;
  }
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

// First level of a long row sum: part[r * kRowParts + q] = sum over the q-th contiguous slice of
// row r (grid kRowParts x rows, fixed order inside each slice)
__global__ __launch_bounds__(kNT) void k_rowsum_part(const double* __restrict__ x, long rs, long es, long n,
                                                     double* __restrict__ part) {
  __shared__ double sh[kNT];
  const long per = (n + kRowParts - 1) / kRowParts;
  const long lo = (long)blockIdx.x * per, hi = min(n, lo + per);
  const double* row = x + (long)blockIdx.y * rs;
  double acc = 0.0;
  for (long k = lo + threadIdx.x; k < hi; k += kNT) acc += row[k * es];
  const double v = block_sum<kNT>(acc, sh);
  if (threadIdx.x == 0) part[(long)blockIdx.y * kRowParts + blockIdx.x] = v;
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

// out[seg * os + comp] = sum over atoms i of segment seg of x[i * stride + comp]
// (one workgroup per (segment, component), fixed order)
__global__ __launch_bounds__(kNT) void k_segsum(const double* __restrict__ x, long stride,
                                                const int* __restrict__ seg_off,
                                                double* __restrict__ out, long os) {
  __shared__ double sh[kNT];
  const int seg = blockIdx.x, comp = blockIdx.y;
  double acc = 0.0;
  for (long i = seg_off[seg] + threadIdx.x; i < seg_off[seg + 1]; i += kNT) acc += x[i * stride + comp];
  const double v = block_sum<kNT>(acc, sh);
  if (threadIdx.x == 0) out[(long)seg * os + comp] = v;
}

// Loss (E_c - E0_c)^2 + sum_i |F_i - F0_i|^2 per configuration: cotangents and per-item parts.
__global__ void k_loss_cfg(const double* __restrict__ e, const double* __restrict__ e0, int ncfg,
                           double* __restrict__ ebar, double* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncfg) return;
  const double d = e[c] - e0[c];
  ebar[c] = 2.0 * d;
  part[c] = d * d;
}
__global__ void k_loss_atoms(const double* __restrict__ f, const double* __restrict__ f0, long n,
                             double* __restrict__ fbar, double* __restrict__ part) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double d = f[3 * i + k] - f0[3 * i + k];
    fbar[3 * i + k] = 2.0 * d;
    acc = fma(d, d, acc);
  }
  part[i] = acc;
}

// ds_t = sum_i ebar_{cfg(i)} [z_i = t] (one workgroup per species, fixed order)
// part[t * kRowParts + q] = sum of ebar[cfg[i]] over the atoms i of species t in the q-th slice
// of the atoms (grid kRowParts x nsp); the parts are summed by k_rowsum
__global__ __launch_bounds__(kNT) void k_species_grad_cfg(const int* __restrict__ species,
                                                          const int* __restrict__ cfg,
                                                          const double* __restrict__ ebar, int n,
                                                          double* __restrict__ part) {
  __shared__ double sh[kNT];
  const int t = blockIdx.y;
  const int per = (n + kRowParts - 1) / kRowParts;
  const int lo = blockIdx.x * per, hi = min(n, lo + per);
  double acc = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += kNT)
    if (species[i] == t) acc += ebar[cfg[i]];
  const double v = block_sum<kNT>(acc, sh);
  if (threadIdx.x == 0) part[t * kRowParts + blockIdx.x] = v;
}

// Per-species chains through each CSR row: pfirst[i][t] is the first pair of atom i whose
// neighbour has species t and plink[p] the next pair of the same row and neighbour species
// (-1 ends a chain). One lane per atom walks its row backwards.
__global__ void k_pair_links(const int* __restrict__ off, const int* __restrict__ nj,
                             const int* __restrict__ species, int nsp, int n, int* __restrict__ plink,
                             int* __restrict__ pfirst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int last[kMaxSpecies];
#pragma unroll
  for (int t = 0; t < kMaxSpecies; ++t) last[t] = -1;
  for (int q = off[i + 1] - 1; q >= off[i]; --q) {
    const int z = clamp_species(species[nj[q]], nsp);
    int nxt = -1;
#pragma unroll
    for (int t = 0; t < kMaxSpecies; ++t)
      if (t == z) {
        nxt = last[t];
        last[t] = q;
      }
    plink[q] = nxt;
  }
#pragma unroll
  for (int t = 0; t < kMaxSpecies; ++t)
    if (t < nsp) pfirst[(long)i * nsp + t] = last[t];
}

// Consistency of a caller-supplied CSR list, one lane per atom; any failure sets *bad.
// Checked: off[0] = 0 and off[n] = npairs, each row inside [0, npairs] and non-decreasing,
// 0 <= j < n, species in [0, nsp), and for every pair p of row i the mirror q = rev[p] lies in
// row j[p], points back at i with the negated shift, and has rev[q] = p.  Every read is
// bounds-checked first, so any list is safe to check.
__global__ __launch_bounds__(kNT) void k_check_nlist(const int* __restrict__ off, const int* __restrict__ nj,
                                                     const int* __restrict__ shift, const int* __restrict__ rev,
                                                     const int* __restrict__ species, int n, long long npairs,
                                                     int nsp, int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int err = 0;
  if (i == 0 && (off[0] != 0 || (long long)off[n] != npairs)) err = 1;
  const int z = species[i];
  if (z < 0 || z >= nsp) err = 1;
  const long long p0 = off[i], p1 = off[i + 1];
  if (p0 < 0 || p1 < p0 || p1 > npairs) {
    err = 1;
  } else {
    for (long long p = p0; p < p1; ++p) {
      const int jj = nj[p];
      if (jj < 0 || jj >= n) {
        err = 1;
        break;
      }
      const long long q = rev[p];
      const long long r0 = off[jj], r1 = off[jj + 1];
      if (q < r0 || q >= r1 || q < 0 || q >= npairs) {
        err = 1;
        break;
      }
      int a1, a2, a3, b1, b2, b3;
      unpack_shift(shift[p], a1, a2, a3);
      unpack_shift(shift[q], b1, b2, b3);
      if (nj[q] != i || rev[q] != p || a1 != -b1 || a2 != -b2 || a3 != -b3) {
        err = 1;
        break;
      }
    }
  }
  if (err) atomicOr(bad, 1);
}

__global__ __launch_bounds__(kNT) void k_fill(double* __restrict__ x, long n, double v) {
  const long i = (long)blockIdx.x * kNT + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ __launch_bounds__(kNT) void k_fill_int(int* __restrict__ x, long n, int v) {
  const long i = (long)blockIdx.x * kNT + threadIdx.x;
  if (i < n) x[i] = v;
}

}  // namespace

void launch_fill(double* x, long n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + kNT - 1) / kNT)), dim3(kNT), 0, s, x, n, v);
}

void launch_fill_int(int* x, long n, int v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_int, dim3((unsigned)((n + kNT - 1) / kNT)), dim3(kNT), 0, s, x, n, v);
}

void launch_check_nlist(const int* off, const int* nj, const int* shift, const int* rev, const int* species,
                        int n, long long npairs, int nsp, int* bad, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_check_nlist, dim3((n + kNT - 1) / kNT), dim3(kNT), 0, s, off, nj, shift, rev, species, n,
                     npairs, nsp, bad);
}

void launch_pair_links(const int* off, const int* nj, const int* species, int nsp, int n, int* plink,
                       int* pfirst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pair_links, dim3((n + kNT - 1) / kNT), dim3(kNT), 0, s, off, nj, species, nsp, n, plink,
                     pfirst);
}

void launch_segsum(const double* x, long stride, const int* seg_off, int nseg, int ncomp, double* out,
                   long os, hipStream_t s) {
  if (nseg <= 0) return;
  hipLaunchKernelGGL(k_segsum, dim3(nseg, ncomp), dim3(kNT), 0, s, x, stride, seg_off, out, os);
}

void launch_loss(const double* e, const double* e0, int ncfg, const double* f, const double* f0, long n,
                 double* ebar, double* fbar, double* part_cfg, double* part_atoms, hipStream_t s) {
  if (ncfg > 0) hipLaunchKernelGGL(k_loss_cfg, dim3((ncfg + kNT - 1) / kNT), dim3(kNT), 0, s, e, e0, ncfg, ebar,
                                   part_cfg);
  if (n > 0) hipLaunchKernelGGL(k_loss_atoms, dim3((unsigned)((n + kNT - 1) / kNT)), dim3(kNT), 0, s, f, f0, n,
                                fbar, part_atoms);
}

void launch_species_grad_cfg(const int* species, const int* cfg, const double* ebar, int n, int nsp,
                             double* out, double* tmp, hipStream_t s) {
  hipLaunchKernelGGL(k_species_grad_cfg, dim3(kRowParts, nsp), dim3(kNT), 0, s, species, cfg, ebar, n, tmp);
  hipLaunchKernelGGL(k_rowsum, dim3(nsp), dim3(kNT), 0, s, tmp, (long)kRowParts, 1L, (long)kRowParts, out, 1L);
}

void launch_rowsum(const double* x, long rs, long es, long n, int rows, double* out, long os,
                   hipStream_t s, double* tmp) {
  if (rows <= 0) return;
  if (tmp && n >= kRowSplitMin) {
    // long rows: kRowParts workgroups per row, then one per row over the parts
    hipLaunchKernelGGL(k_rowsum_part, dim3(kRowParts, rows), dim3(kNT), 0, s, x, rs, es, n, tmp);
    hipLaunchKernelGGL(k_rowsum, dim3(rows), dim3(kNT), 0, s, tmp, (long)kRowParts, 1L, (long)kRowParts, out, os);
    return;
  }
  hipLaunchKernelGGL(k_rowsum, dim3(rows), dim3(kNT), 0, s, x, rs, es, n, out, os);
}

void launch_species_grad(const int* species, int n, int nsp, double ebar, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_species_grad, dim3(1), dim3(kNT), 0, s, species, n, nsp, ebar, out);
}

void launch_gather_forces(const int* off, const int* rev, const double* g, const double* fown, int n,
                          long long npairs, double* forces, hipStream_t s) {
  if (n <= 0) return;
  const int per = kNT / kGatherLanes;
  if (fown)
    hipLaunchKernelGGL(k_gather<true>, dim3((n + per - 1) / per), dim3(kNT), 0, s, off, rev, g, fown, n, npairs,
                       forces);
  else
    hipLaunchKernelGGL(k_gather<false>, dim3((n + per - 1) / per), dim3(kNT), 0, s, off, rev, g, fown, n, npairs,
                       forces);
}

// Energy and virial of a small system in one workgroup: energy = sum_i ea[i] (n terms) and
// virial[k] = sum_b wpart[6 b + k] (nb partials).  Each thread sums a strided share of all seven
// quantities, the waves reduce them with a butterfly, and thread 0 adds the waves' sums in
// order (a fixed order throughout).
__global__ __launch_bounds__(kSmallSumThreads) void k_sum_small(const double* __restrict__ ea, long n,
                                                                const double* __restrict__ wpart, long nb,
                                                                double* __restrict__ energy,
                                                                double* __restrict__ virial) {
  constexpr int kW = kSmallSumThreads / 64;
  __shared__ double sh[kW][7];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  if (energy) {
#pragma unroll 4
    for (long i = threadIdx.x; i < n; i += kSmallSumThreads) acc[0] += ea[i];
  }
  if (virial)
    for (long b = threadIdx.x; b < nb; b += kSmallSumThreads)
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[1 + k] += wpart[6 * b + k];
#pragma unroll
  for (int c = 0; c < 7; ++c)
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) acc[c] += __shfl_xor(acc[c], s, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < 7; ++c) sh[wave][c] = acc[c];
  __syncthreads();
  if (threadIdx.x < 7) {
    double v = 0.0;
    for (int w = 0; w < kW; ++w) v += sh[w][threadIdx.x];
    if (threadIdx.x == 0) {
      if (energy) energy[0] = v;
    } else if (virial) {
      virial[threadIdx.x - 1] = v;
    }
  }
}

void launch_sum_small(const double* ea, long n, const double* wpart, long nb, double* energy, double* virial,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_sum_small, dim3(1), dim3(kSmallSumThreads), 0, s, ea, n, wpart, nb, energy, virial);
}

void launch_sum_parts2(const double* x1, long n1, long st1, int nc1, double* out1, const double* x2, long n2,
                       long st2, int nc2, double* out2, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_part2, dim3(kPartBlocks, nc1 + nc2), dim3(kNT), 0, s, x1, n1, st1, nc1, x2, n2, st2,
                     part);
  hipLaunchKernelGGL(k_sum_final2, dim3(nc1 + nc2), dim3(kNT), 0, s, part, nc1, out1, out2);
}

// out[c] = sum_i x[i * stride + c] for c < ncomp; part holds ncomp * kPartBlocks doubles.
void launch_sum_parts(const double* x, long n, long stride, int ncomp, double* part, double* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_sum_part, dim3(kPartBlocks, ncomp), dim3(kNT), 0, s, x, n, stride, part);
  hipLaunchKernelGGL(k_sum_final, dim3(ncomp), dim3(kNT), 0, s, part, out);
}

void launch_sum(const double* x, long n, long stride, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kSumThreads), 0, s, x, n, stride, out);
}

void launch_sum_virial(const double* wpart, long nblocks, double* out, hipStream_t s) {
  for (int k = 0; k < 6; ++k)
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kSumThreads), 0, s, wpart + k, nblocks, 6L, out + k);
}

}  // namespace mtp
