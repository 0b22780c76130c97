// Level-templated MTP kernels.  A translation unit includes one generated level header
// (struct LvXX with the straight-line program) and then this file, and instantiates the
// launchers with MTP_DEFINE_CHAIN / MTP_DEFINE_ADJ / MTP_DEFINE_ADJ_FWD / MTP_DEFINE_ADJ_REV.
//
// Every kernel maps one lane to one atom: the per-atom state (moments, contraction
// outputs, adjoints) lives in registers with compile-time indices, the neighbour loop of
// the lane walks the atom's CSR row.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>

#include "mtp_device.h"
#include "mtp_internal.h"

namespace mtp {

constexpr int kLaneBlock = 64;   // one wave per workgroup for the lane-per-atom kernels

// Tiles of kLaneBlock atoms a workgroup of a pair kernel processes: its own block of the grid
// (PERSIST false: the loop body runs once), or, for a persistent launch, tiles pulled from the
// device counter a.queue until none is left, so that workgroups that finish early take the
// remaining tiles.  Every tile writes its own outputs (per-tile partials included), so the
// result does not depend on which workgroup takes which tile.
template <bool PERSIST>
struct TileLoop {
  int nblocks;
  int* slot;  // LDS word that broadcasts a pulled tile to the workgroup
  __device__ __forceinline__ int pull(int* q) const {
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(q, 1);
    __syncthreads();
    return *slot;
  }
  __device__ __forceinline__ int first(const SysArgs& a) const {
    if constexpr (PERSIST) return pull(a.queue);
    else return xcd_logical_block(blockIdx.x, gridDim.x);
  }
  __device__ __forceinline__ int next(const SysArgs& a) const {
    if constexpr (PERSIST) return pull(a.queue);
    else return nblocks;
  }
};
// K lanes per atom: a tile holds kLaneBlock / K atoms
#define MTP_FOR_TILES_K(a, n, K, b)                                                                    \
  __shared__ int tile_slot_;                                                                           \
  const TileLoop<PERSIST> tiles_{(int)(((long)(n) * (K) + kLaneBlock - 1) / kLaneBlock), &tile_slot_}; \
  for (int b = tiles_.first(a); b < tiles_.nblocks; b = tiles_.next(a))
#define MTP_FOR_TILES(a, n, b) MTP_FOR_TILES_K(a, n, 1, b)

// Sum over the K consecutive lanes of an atom (K = 1, 2, 4, 8) by DPP lane exchanges inside
// quads and half-rows; every lane of the group ends with the same value (each step adds two
// equal partial sums in either order, which is exact commutativity).
template <int CTRL>
__device__ __forceinline__ double dpp_exchange(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_exchange(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int K, class R>
__device__ __forceinline__ R group_sum(R v) {
  static_assert(K == 1 || K == 2 || K == 4 || K == 8, "lanes per atom");
  if constexpr (K >= 2) v += dpp_exchange<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  if constexpr (K >= 4) v += dpp_exchange<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  if constexpr (K >= 8) v += dpp_exchange<0x141>(v);  // row_half_mirror
  return v;
}

inline int pair_grid(const SysArgs& a, int nb) { return a.queue ? std::max(1, std::min(nb, a.pgrid)) : nb; }

// Accessors of [row][atom] arrays in global memory.  The address of a row is the same for the
// whole wave (scalar registers) and each lane adds its byte offset, so a load takes the
// scalar-base form: no per-row 64-bit address is kept in vector registers (the compiler
// otherwise precomputes the addresses of every row a program reads and spills them).
// The host caps a chunk (the atoms of one row) at 2^28, so the byte offset fits 32 bits.
__device__ __forceinline__ unsigned lane_bytes(int li, int size) { return (unsigned)li * (unsigned)size; }

// Moment vector of a lane, [entry][atom] layout.
template <class R>
struct GlobalMoments {
  const R* __restrict__ base;
  long ld;
  unsigned off;  // byte offset of the lane's atom in a row
  __device__ __forceinline__ R operator()(int e) const {
    return *reinterpret_cast<const R*>(reinterpret_cast<const char*>(base + (long)e * ld) + off);
  }
};

// The same with a per-lane 64-bit pointer (vector addresses): measured faster for the forward
// program kernels (k_program, k_program_fwd), whose few spills do not come from addresses.
template <class R>
struct LaneMoments {
  const R* __restrict__ p;
  long ld;
  __device__ __forceinline__ R operator()(int e) const { return p[(long)e * ld]; }
};

// Per-lane vector read from a [component][atom] array in global memory, one load per use.
template <class R>
struct GlobalVector {
  const R* __restrict__ base;
  long ld;
  unsigned off;
  __device__ __forceinline__ R operator[](int q) const {
    return *reinterpret_cast<const R*>(reinterpret_cast<const char*>(base + (long)q * ld) + off);
  }
};

// Per-lane element i of a [row][atom] array written in place (i = row * ld).
template <class R>
struct LaneRows {
  R* __restrict__ base;
  unsigned off;
  __device__ __forceinline__ R& operator[](long i) const {
    return *reinterpret_cast<R*>(reinterpret_cast<char*>(base + i) + off);
  }
};

// Contraction-adjoint vectors longer than this are read from memory where a block needs them
// instead of being loaded into registers up front (which spills at the largest levels).
constexpr int kRegComps = 64;

// Per-lane vector held in LDS in [component][lane] layout (conflict-free across a wave).
template <class R>
struct LaneVector {
  const R* p;
  __device__ __forceinline__ R operator[](int q) const { return p[q * kLaneBlock]; }
};

template <class R>
struct RegMoments {
  const R* m;
  __device__ __forceinline__ R operator()(int e) const { return m[e]; }
};

// radial coefficient table staged in LDS (in the arithmetic type of the kernel)
template <class R>
__device__ __forceinline__ void stage_radial(const SysArgs& a, R* sh) {
  const int n = a.nsp * a.nsp * a.nmu * a.ncheb;
  for (int k = threadIdx.x; k < n; k += blockDim.x) sh[k] = (R)a.radial[k];
  __syncthreads();
}

// Walk the CSR row of atom i with software prefetch: the partner indices are loaded two pairs
// ahead and the partner position/species one pair ahead, so the gather latency overlaps the
// arithmetic of the current pair.  body(p, j, zj, dx, dy, dz, r) sees the exact displacement.
// With K lanes per atom, lane sub of the atom takes pairs sub, sub + K, sub + 2K, ... of the row.
template <int K = 1, class F>
__device__ __forceinline__ void for_pairs(const SysArgs& a, int i, int sub, const double* H, double rix,
                                          double riy, double riz, F&& body) {
  const int p0 = a.off[i] + sub, p1 = a.off[i + 1];
  if (p0 >= p1) return;
  int jA = a.nj[p0], shA = a.shift[p0];
  double xA = a.pos[3 * jA], yA = a.pos[3 * jA + 1], zA = a.pos[3 * jA + 2];
  int sA = a.species[jA];
  int jB = 0, shB = 0;
  if (p0 + K < p1) {
    jB = a.nj[p0 + K];
    shB = a.shift[p0 + K];
  }
  for (int p = p0; p < p1; p += K) {
    const int j = jA, sh = shA, sj = sA;
    const double xj = xA, yj = yA, zj = zA;
    if (p + K < p1) {
      xA = a.pos[3 * jB];
      yA = a.pos[3 * jB + 1];
      zA = a.pos[3 * jB + 2];
      sA = a.species[jB];
      jA = jB;
      shA = shB;
    }
    if (p + 2 * K < p1) {
      jB = a.nj[p + 2 * K];
      shB = a.shift[p + 2 * K];
    }
    int n1, n2, n3;
    unpack_shift(sh, n1, n2, n3);
    double dx, dy, dz;
    pair_displacement(rix, riy, riz, xj, yj, zj, n1, n2, n3, H, dx, dy, dz);
    const double r = sqrt(dist2_exact(dx, dy, dz));
    body(p, j, clamp_species(sj, a.nsp), dx, dy, dz, r);
  }
}

// ---------------------------------------------------------------------------- moments
template <bool BATCH>
__device__ __forceinline__ int sweep_atom(const SysArgs& a, int k) {
  if constexpr (BATCH) return atom_at(a, k);
  else return k;
}
// cell of atom i: the kernel-argument copy (uniform, scalar registers) for one system
template <bool BATCH>
__device__ __forceinline__ void cell_of(const SysArgs& a, int i, double* H) {
  if constexpr (BATCH) {
    load_cell(a, i, H);
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) H[k] = a.H[k];
  }
}

// K lanes per atom (single systems): each accumulates every K-th pair of the row, the partial
// moments are summed over the atom's lanes and its first lane writes them.
template <class L, int G, class R, bool BATCH, int NC, bool PERSIST = false, int K = 1>
__global__ __launch_bounds__(kLaneBlock) void k_moments(SysArgs a, int i0, int n,
                                                        R* __restrict__ mout, long ld) {
  static_assert(K == 1 || !BATCH, "batches take one lane per atom");
  __shared__ R csh[kMaxRadial];
  stage_radial(a, csh);
  MTP_FOR_TILES_K(a, n, K, b) {
  const int li = b * (kLaneBlock / K) + (int)threadIdx.x / K, sub = (int)threadIdx.x % K;
  if (li >= n) continue;
  const int i = sweep_atom<BATCH>(a, i0 + li);
  double H[9];
  cell_of<BATCH>(a, i, H);
  constexpr int LO = L::GROUP_LO[G], HI = L::GROUP_HI[G], NG = HI - LO;
  R m[NG];
#pragma unroll
  for (int e = 0; e < NG; ++e) m[e] = R(0);
  const double rix = a.pos[3 * i], riy = a.pos[3 * i + 1], riz = a.pos[3 * i + 2];
  const int zi = clamp_species(a.species[i], a.nsp);
  const R* cz = csh + zi * a.nsp * L::NMU * a.ncheb;
  for_pairs<K>(a, i, sub, H, rix, riy, riz, [&](int, int, int zj, double dx, double dy, double dz, double r) {
    R f[L::NMU];
    radial_values<R, L::NMU, NC>((R)r, (R)a.sa, (R)a.sb, (R)a.rcut, cz + zj * L::NMU * a.ncheb, a.ncheb, f);
    L::template acc_moments<G>(m, f, (R)dx, (R)dy, (R)dz);
  });
  if constexpr (K > 1) {
#pragma unroll
    for (int e = 0; e < NG; ++e) m[e] = group_sum<K>(m[e]);
  }
  if (sub == 0) {
#pragma unroll
    for (int e = 0; e < NG; ++e) mout[(long)(LO + e) * ld + li] = m[e];
  }
  }
}

// ---------------------------------------------------------------------------- program forward
template <class L, class R>
__global__ __launch_bounds__(kLaneBlock) void k_program_fwd(const R* __restrict__ mom, long ld,
                                                            int i0, int n, const int* __restrict__ perm,
                                                            const int* __restrict__ species,
                                                            const double* __restrict__ xi,
                                                            const double* __restrict__ shift, int nsp,
                                                            double* __restrict__ e_atom,
                                                            R* __restrict__ cbar,
                                                            double* __restrict__ bout) {
  const int b = xcd_logical_block(blockIdx.x, gridDim.x);
  const int li = b * kLaneBlock + threadIdx.x;
  if (li >= n) return;
  LaneMoments<R> M{mom + li, ld};
  R C[L::NCOMP];
  L::template fwd<R>(M, C);
  R Cb[L::NCOMP];
  const double e = bout ? L::template products<true, R>(C, xi, Cb, bout + li, ld)
                        : L::template products<false, R>(C, xi, Cb, nullptr, ld);
  const int i = perm ? perm[i0 + li] : i0 + li;
  e_atom[i] = e + shift[clamp_species(species[i], nsp)];
#pragma unroll
  for (int q = 0; q < L::NCOMP; ++q) cbar[(long)q * ld + li] = Cb[q];
}

// ---------------------------------------------------------------------------- program reverse
template <class L, int G, class R>
__global__ __launch_bounds__(kLaneBlock) void k_program_rev(const R* __restrict__ mom, long ld,
                                                            int n, const R* __restrict__ cbar,
                                                            R* __restrict__ mbar) {
  const int b = xcd_logical_block(blockIdx.x, gridDim.x);
  const int li = b * kLaneBlock + threadIdx.x;
  if (li >= n) return;
  constexpr int LO = L::GROUP_LO[G], HI = L::GROUP_HI[G], NG = HI - LO;
  GlobalMoments<R> M{mom, ld, lane_bytes(li, sizeof(R))};
  R mb[NG];
#pragma unroll
  for (int e = 0; e < NG; ++e) mb[e] = R(0);
  if constexpr (L::NCOMP > kRegComps) {
    L::template rev<G>(M, GlobalVector<R>{cbar, ld, lane_bytes(li, sizeof(R))}, mb);
  } else {
    R Cb[L::NCOMP];
#pragma unroll
    for (int q = 0; q < L::NCOMP; ++q) Cb[q] = cbar[(long)q * ld + li];
    L::template rev<G>(M, Cb, mb);
  }
#pragma unroll
  for (int e = 0; e < NG; ++e) mbar[(long)(LO + e) * ld + li] = mb[e];
}

// ---------------------------------------------------------------------------- fused program
// Forward program, energy and basis products, then the reverse program, in one pass over an
// atom's moments (single-group levels): the contraction adjoints stay in registers instead of
// taking a round trip through memory, and the moments are read by one kernel instead of two.
template <class L, class R>
__global__ __launch_bounds__(kLaneBlock) void k_program(const R* __restrict__ mom, long ld, int i0, int n,
                                                        const int* __restrict__ species,
                                                        const double* __restrict__ xi,
                                                        const double* __restrict__ shift, int nsp,
                                                        double* __restrict__ e_atom, R* __restrict__ mbar) {
  static_assert(L::NGROUP == 1, "the fused program needs all moment entries in one group");
  // contraction adjoints parked in LDS between the two programs (registers are the limit)
  __shared__ R cbs[L::NCOMP * kLaneBlock];
  const int b = xcd_logical_block(blockIdx.x, gridDim.x);
  const int li = b * kLaneBlock + threadIdx.x;
  if (li >= n) return;
  LaneMoments<R> M{mom + li, ld};
  {
    R C[L::NCOMP], Cb[L::NCOMP];
    L::template fwd<R>(M, C);
    const double e = L::template products<false, R>(C, xi, Cb, nullptr, ld);
    const int i = i0 + li;
    e_atom[i] = e + shift[clamp_species(species[i], nsp)];
#pragma unroll
    for (int q = 0; q < L::NCOMP; ++q) cbs[q * kLaneBlock + threadIdx.x] = Cb[q];
  }
  // the reverse program re-reads the moments it needs: no loaded value stays live across
  asm volatile("" ::: "memory");
  R mb[L::NMOM];
#pragma unroll
  for (int e = 0; e < L::NMOM; ++e) mb[e] = R(0);
  L::template rev<0>(M, LaneVector<R>{cbs + threadIdx.x}, mb);
#pragma unroll
  for (int e = 0; e < L::NMOM; ++e) mbar[(long)e * ld + li] = mb[e];
}

// ---------------------------------------------------------------------------- backward pairs
// g[p] (+)= dE_i/dd_ij restricted to the entries of group G; per-workgroup virial partials;
// fown[i] (+)= sum of the atom's own g over its row (the first half of its force), when given.
// K lanes per atom (single systems): each takes every K-th pair of the row; the own sums are
// combined over the atom's lanes, the virial partial over the workgroup as before.
template <class L, int G, class R, bool BATCH, int NC, bool PERSIST = false, int K = 1>
__global__ __launch_bounds__(kLaneBlock) void k_backward(SysArgs a, int i0, int n,
                                                         const R* __restrict__ mbar, long ld,
                                                         double* __restrict__ g, int accumulate,
                                                         double* __restrict__ wpart,
                                                         double* __restrict__ watom,
                                                         double* __restrict__ fown) {
  static_assert(K == 1 || !BATCH, "batches take one lane per atom");
  __shared__ R csh[kMaxRadial];
  __shared__ double red[kLaneBlock];
  stage_radial(a, csh);
  MTP_FOR_TILES_K(a, n, K, b) {
  const int li = b * (kLaneBlock / K) + (int)threadIdx.x / K, sub = (int)threadIdx.x % K;
  constexpr int LO = L::GROUP_LO[G], HI = L::GROUP_HI[G], NG = HI - LO;
  double w[6] = {0, 0, 0, 0, 0, 0};
  double fo[3] = {0, 0, 0};  // sum of the atom's own pair gradients
  if (li < n) {
    const int i = sweep_atom<BATCH>(a, i0 + li);
    double H[9];
    cell_of<BATCH>(a, i, H);
    R mb[NG];
    // adjoints scaled by a! b! c! for the scaled monomials of pair_grad
#pragma unroll
    for (int e = 0; e < NG; ++e) mb[e] = mbar[(long)(LO + e) * ld + li] * R(L::MFACT[LO + e]);
    const double rix = a.pos[3 * i], riy = a.pos[3 * i + 1], riz = a.pos[3 * i + 2];
    const int zi = clamp_species(a.species[i], a.nsp);
    const R* cz = csh + zi * a.nsp * L::NMU * a.ncheb;
    // the gradient of a pair is stored at the start of the next pair's body, after that
    // pair's list and position loads: the wait for those loads at the end of the body then
    // does not also wait for a store issued just before it (one counter covers both)
    int pq = -1;
    double qx = 0.0, qy = 0.0, qz = 0.0;
    for_pairs<K>(a, i, sub, H, rix, riy, riz, [&](int p, int, int zj, double dx, double dy, double dz, double r) {
      if (pq >= 0) {
        g[3L * pq] = qx;
        g[3L * pq + 1] = qy;
        g[3L * pq + 2] = qz;
      }
      R f[L::NMU], fp[L::NMU];
      radial<R, L::NMU, NC>((R)r, (R)a.sa, (R)a.sb, (R)a.rcut, cz + zj * L::NMU * a.ncheb, a.ncheb, f, fp);
      R rgx = R(0), rgy = R(0), rgz = R(0), ru = R(0);
      L::template pair_grad<G>(mb, f, fp, (R)dx, (R)dy, (R)dz, rgx, rgy, rgz, ru);
      const double ur = (double)ru / r;
      const double gx = fma(ur, dx, (double)rgx);
      const double gy = fma(ur, dy, (double)rgy);
      const double gz = fma(ur, dz, (double)rgz);
      if (accumulate) {
        g[3L * p] += gx;
        g[3L * p + 1] += gy;
        g[3L * p + 2] += gz;
      } else {
        pq = p;
        qx = gx;
        qy = gy;
        qz = gz;
      }
      fo[0] += gx;
      fo[1] += gy;
      fo[2] += gz;
      w[0] -= dx * gx;
      w[1] -= dy * gy;
      w[2] -= dz * gz;
      w[3] -= dx * gy;
      w[4] -= dx * gz;
      w[5] -= dy * gz;
    });
    if (pq >= 0) {
      g[3L * pq] = qx;
      g[3L * pq + 1] = qy;
      g[3L * pq + 2] = qz;
    }
    if constexpr (BATCH) {
#pragma unroll
      for (int k = 0; k < 6; ++k) watom[6L * i + k] = accumulate ? watom[6L * i + k] + w[k] : w[k];
    }
    if constexpr (K > 1) {
#pragma unroll
      for (int k = 0; k < 3; ++k) fo[k] = group_sum<K>(fo[k]);
    }
    if (fown && sub == 0) {
#pragma unroll
      for (int k = 0; k < 3; ++k) fown[3L * i + k] = accumulate ? fown[3L * i + k] + fo[k] : fo[k];
    }
  }
  // with accumulate, the launches of the moment groups run one after another on one stream and
  // each adds its share to the same per-workgroup partial
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double s = block_sum<kLaneBlock>(w[k], red);
    if (threadIdx.x == 0) wpart[6L * b + k] = accumulate ? wpart[6L * b + k] + s : s;
  }
  }
}

// ---------------------------------------------------------------------------- parameter adjoint
// Tangent of the moments along delta_ij = fbar_j - fbar_i (the direction in which the
// force-weighted loss term differentiates the energy).
template <class L, int G, bool PERSIST = false>
__global__ __launch_bounds__(kLaneBlock) void k_tan_moments(SysArgs a, const double* __restrict__ fbar,
                                                            int i0, int n, double* __restrict__ mdot,
                                                            long ld) {
  __shared__ double csh[kMaxRadial];
  stage_radial(a, csh);
  MTP_FOR_TILES(a, n, b) {
  const int li = b * kLaneBlock + threadIdx.x;
  if (li >= n) continue;
  const int i = atom_at(a, i0 + li);
  double H[9];
  load_cell(a, i, H);
  constexpr int LO = L::TGROUP_LO[G], HI = L::TGROUP_HI[G], NG = HI - LO;
  double md[NG];
#pragma unroll
  for (int e = 0; e < NG; ++e) md[e] = 0.0;
  const double rix = a.pos[3 * i], riy = a.pos[3 * i + 1], riz = a.pos[3 * i + 2];
  const double fix = fbar[3 * i], fiy = fbar[3 * i + 1], fiz = fbar[3 * i + 2];
  const int zi = clamp_species(a.species[i], a.nsp);
  for_pairs(a, i, 0, H, rix, riy, riz, [&](int, int j, int zj, double dx, double dy, double dz, double r) {
    double f[L::NMU], fp[L::NMU];
    radial<double, L::NMU>(r, a.sa, a.sb, a.rcut, csh + (zi * a.nsp + zj) * L::NMU * a.ncheb, a.ncheb, f, fp);
    const double ex = fbar[3 * j] - fix, ey = fbar[3 * j + 1] - fiy, ez = fbar[3 * j + 2] - fiz;
    const double rdot = (dx * ex + dy * ey + dz * ez) / r;
    L::template tan_moments<G>(md, f, fp, dx, dy, dz, ex, ey, ez, rdot);
  });
#pragma unroll
  for (int e = 0; e < NG; ++e) mdot[(long)(LO + e) * ld + li] = md[e];
  }
}

// Tangents of contractions and basis: out[alpha] = ebar B_alpha - dB_alpha, and dCbar.
template <class L>
__global__ __launch_bounds__(kLaneBlock) void k_tan_forward(const double* __restrict__ mom,
                                                            const double* __restrict__ mdot, long ld,
                                                            int i0, int n, const int* __restrict__ perm,
                                                            const int* __restrict__ cfg,
                                                            const double* __restrict__ ebar_cfg,
                                                            const double* __restrict__ xi,
                                                            double ebar, double* __restrict__ out,
                                                            double* __restrict__ cbard) {
  const int b = xcd_logical_block(blockIdx.x, gridDim.x);
  const int li = b * kLaneBlock + threadIdx.x;
  if (li >= n) return;
  if (ebar_cfg) {
    const int i = perm ? perm[i0 + li] : i0 + li;
    ebar = ebar_cfg[cfg ? cfg[i] : 0];
  }
  const unsigned lo = lane_bytes(li, sizeof(double));
  GlobalMoments<double> M{mom, ld, lo}, Md{mdot, ld, lo};
  double C[L::NCOMP], Cd[L::NCOMP];
  L::template fwd_tan<double>(M, Md, C, Cd);
  double Cb[L::NCOMP], Cbd[L::NCOMP];
  L::template products_tan<double>(C, Cd, xi, ebar, Cb, Cbd, out + li, ld);
#pragma unroll
  for (int q = 0; q < L::NCOMP; ++q) cbard[(long)q * ld + li] = Cbd[q];
}

// Tangent of the moment adjoint: mbd = d(mbar) along the moment tangent.  The reverse program
// is cut into parts of contraction blocks sized for the registers; part P stores or adds the
// entries it touches, so the parts run in order 0, 1, ... on one stream.
template <class L, int P>
__global__ __launch_bounds__(kLaneBlock) void k_tan_reverse(const double* __restrict__ mom,
                                                            const double* __restrict__ mdot, long ld,
                                                            int n, const double* __restrict__ cbar,
                                                            const double* __restrict__ cbard,
                                                            double* __restrict__ mbard) {
  const int b = xcd_logical_block(blockIdx.x, gridDim.x);
  const int li = b * kLaneBlock + threadIdx.x;
  if (li >= n) return;
  const unsigned lo = lane_bytes(li, sizeof(double));
  GlobalMoments<double> M{mom, ld, lo}, Md{mdot, ld, lo};
  if constexpr (L::NCOMP > kRegComps) {
    L::template rev_tan<P, double>(M, Md, GlobalVector<double>{cbar, ld, lo}, GlobalVector<double>{cbard, ld, lo},
                                   LaneRows<double>{mbard, lo}, ld);
  } else {
    double Cb[L::NCOMP], Cbd[L::NCOMP];
#pragma unroll
    for (int q = 0; q < L::NCOMP; ++q) {
      Cb[q] = cbar[(long)q * ld + li];
      Cbd[q] = cbard[(long)q * ld + li];
    }
    L::template rev_tan<P, double>(M, Md, Cb, Cbd, LaneRows<double>{mbard, lo}, ld);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  return v;
}

// Radial-coefficient gradient: per pair (i, j) with species (s, t),
//   dc[s][t][mu][b] += Q_b (ebar S_mu - A_mu) - Q'_b (rhat . delta) S_mu,
// accumulated per lane for one neighbour species at a time (following the per-species pair
// chains) and summed over the wave with a fixed butterfly; one partial per (workgroup, s, t)
// lands in cpart. G is an adjoint group: a
// moment range small enough that its adjoints, their tangents and the sums of its mu values
// [AMU_LO, AMU_HI] stay in registers; the partial rows of the other mu values are written as
// zeros. NC is the compile-time Chebyshev count (0: runtime count up to kMaxCheb); every index
// into the accumulators is a compile-time constant.
template <class L, int G, int NC, bool PERSIST = false>
__global__ __launch_bounds__(kLaneBlock) void k_adj_pairs(SysArgs a, const double* __restrict__ fbar,
                                                          int i0, int n,
                                                          const double* __restrict__ mbar,
                                                          const double* __restrict__ mbard, long ld,
                                                          double ebar, double* __restrict__ cpart) {
  const double ebar0 = ebar;
  MTP_FOR_TILES(a, n, b) {
  ebar = ebar0;
  const int li = b * kLaneBlock + threadIdx.x;
  constexpr int LO = L::AGROUP_LO[G], HI = L::AGROUP_HI[G], NG = HI - LO;
  constexpr int NMU = L::NMU, MLO = L::AMU_LO[G], MHI = L::AMU_HI[G], NM = MHI - MLO + 1;
  constexpr int NQ = NC > 0 ? NC : kMaxCheb;
  const int nq = NC > 0 ? NC : a.ncheb;
  const bool live = li < n;
  const int i = atom_at(a, i0 + (live ? li : 0));
  double H[9];
  load_cell(a, i, H);
  if (a.ebar) ebar = a.ebar[a.cfg ? a.cfg[i] : 0];
  double mb[NG], mbd[NG];
#pragma unroll
  for (int e = 0; e < NG; ++e) {
    mb[e] = live ? mbar[(long)(LO + e) * ld + li] : 0.0;
    mbd[e] = live ? mbard[(long)(LO + e) * ld + li] : 0.0;
  }
  const double rix = a.pos[3 * i], riy = a.pos[3 * i + 1], riz = a.pos[3 * i + 2];
  const double fix = fbar[3 * i], fiy = fbar[3 * i + 1], fiz = fbar[3 * i + 2];
  const int zi = clamp_species(a.species[i], a.nsp);
  const int p0 = live ? a.off[i] : 0, p1 = live ? a.off[i + 1] : 0;
  for (int t = 0; t < a.nsp; ++t) {
    double acc[NM * NQ];
#pragma unroll
    for (int k = 0; k < NM * NQ; ++k) acc[k] = 0.0;
    // each lane follows its row's chain of species-t pairs (the whole row with one species),
    // so the wave runs the pair body max over lanes (not the row length) times per species;
    // the next link and the next pair's list entries are loaded one pair ahead
    auto link = [&](int q) -> int { return a.plink ? a.plink[q] : (q + 1 < p1 ? q + 1 : -1); };
    int p = !live ? -1 : a.pfirst ? a.pfirst[(long)i * a.nsp + t] : (p0 < p1 ? p0 : -1);
    int pn = p >= 0 ? link(p) : -1;
    int j = p >= 0 ? a.nj[p] : 0, sh = p >= 0 ? a.shift[p] : 0;
    for (;;) {
      if (!__any(p >= 0)) break;
      if (p < 0) continue;
      const int pnn = pn >= 0 ? link(pn) : -1;
      const int jn = pn >= 0 ? a.nj[pn] : 0, shn = pn >= 0 ? a.shift[pn] : 0;
      int n1, n2, n3;
      unpack_shift(sh, n1, n2, n3);
      double dx, dy, dz;
      pair_displacement(rix, riy, riz, a.pos[3 * j], a.pos[3 * j + 1], a.pos[3 * j + 2], n1, n2,
                        n3, H, dx, dy, dz);
      const double r = sqrt(dist2_exact(dx, dy, dz));
      const double ex = fbar[3 * j] - fix, ey = fbar[3 * j + 1] - fiy, ez = fbar[3 * j + 2] - fiz;
      const double rdot = (dx * ex + dy * ey + dz * ez) / r;
      double S[NMU], A[NMU];
#pragma unroll
      for (int mu = 0; mu < NMU; ++mu) S[mu] = A[mu] = 0.0;
      L::template adj_pair<G>(mb, mbd, dx, dy, dz, ex, ey, ez, S, A);
      double X[NM], Y[NM];
#pragma unroll
      for (int k = 0; k < NM; ++k) {
        X[k] = fma(ebar, S[MLO + k], -A[MLO + k]);
        Y[k] = -rdot * S[MLO + k];
      }
      // Q_b = T_b(u) w^2, Q'_b = sa T'_b(u) w^2 - 2 T_b(u) w
      const double u = fma(a.sa, r, a.sb), w = a.rcut - r, w2 = w * w;
      double t2 = 1.0, t1 = u, d2 = 0.0, d1 = 1.0;
#pragma unroll
      for (int bq = 0; bq < NQ; ++bq) {
        if (NC == 0 && bq >= nq) break;
        double T, D;
        if (bq == 0) {
          T = 1.0;
          D = 0.0;
        } else if (bq == 1) {
          T = u;
          D = 1.0;
        } else {
          T = fma(2.0 * u, t1, -t2);
          D = fma(2.0 * u, d1, fma(2.0, t1, -d2));
          t2 = t1;
          t1 = T;
          d2 = d1;
          d1 = D;
        }
        const double q = T * w2, qp = fma(a.sa * w2, D, -2.0 * w * T);
#pragma unroll
        for (int k = 0; k < NM; ++k) acc[k * NQ + bq] = fma(q, X[k], fma(qp, Y[k], acc[k * NQ + bq]));
      }
      p = pn;
      pn = pnn;
      j = jn;
      sh = shn;
    }
    for (int sp = 0; sp < a.nsp; ++sp) {
      double* dst = cpart + (long)b * a.nsp * a.nsp * NMU * nq + (long)(sp * a.nsp + t) * NMU * nq;
      for (int k = threadIdx.x; k < NMU * nq; k += kLaneBlock) {
        const int mu = k / nq;
        if (mu < MLO || mu > MHI) dst[k] = 0.0;
      }
#pragma unroll
      for (int k = 0; k < NM; ++k)
#pragma unroll
        for (int bq = 0; bq < NQ; ++bq) {
          if (NC == 0 && bq >= nq) break;
          const double v = wave_sum((live && zi == sp) ? acc[k * NQ + bq] : 0.0);
          if (threadIdx.x == 0) dst[(MLO + k) * nq + bq] = v;
        }
    }
  }
  }
}

// ---------------------------------------------------------------------------- launchers
// The pair kernels come in Chebyshev-count specialisations for the common sizes 8 and 10 and a
// runtime-count form for the rest.
inline int split_tiles(int n, int k) { return (int)(((long)n * k + kLaneBlock - 1) / kLaneBlock); }

template <class L, int G, class R, bool BATCH, bool PERSIST, int K = 1>
void launch_moments_gp(const SysArgs& a, int i0, int n, void* m, long ld, hipStream_t s) {
  const int nb = pair_grid(a, split_tiles(n, K));
  if (a.ncheb == 8)
    hipLaunchKernelGGL((k_moments<L, G, R, BATCH, 8, PERSIST, K>), dim3(nb), dim3(kLaneBlock), 0, s, a, i0, n, (R*)m, ld);
  else if (a.ncheb == 10)
    hipLaunchKernelGGL((k_moments<L, G, R, BATCH, 10, PERSIST, K>), dim3(nb), dim3(kLaneBlock), 0, s, a, i0, n, (R*)m, ld);
  else
    hipLaunchKernelGGL((k_moments<L, G, R, BATCH, 0, PERSIST, K>), dim3(nb), dim3(kLaneBlock), 0, s, a, i0, n, (R*)m, ld);
}
// persistent variants exist for batches only (a single system uses one grid of its tiles);
// split lanes for single systems in binary64 only
template <class L, int G, class R, bool BATCH>
void launch_moments_g(const SysArgs& a, int i0, int n, void* m, long ld, hipStream_t s) {
  if constexpr (BATCH) {
    if (a.queue) return launch_moments_gp<L, G, R, BATCH, true>(a, i0, n, m, ld, s);
  } else if constexpr (std::is_same_v<R, double>) {
    if (a.split == 2) return launch_moments_gp<L, G, R, BATCH, false, 2>(a, i0, n, m, ld, s);
    if (a.split == 4) return launch_moments_gp<L, G, R, BATCH, false, 4>(a, i0, n, m, ld, s);
    if (a.split == 8) return launch_moments_gp<L, G, R, BATCH, false, 8>(a, i0, n, m, ld, s);
  }
  launch_moments_gp<L, G, R, BATCH, false>(a, i0, n, m, ld, s);
}
template <class L, int G, class R>
void launch_rev_g(const void* m, long ld, int n, const void* cb, void* mb, hipStream_t s) {
  const int nb = (n + kLaneBlock - 1) / kLaneBlock;
  hipLaunchKernelGGL((k_program_rev<L, G, R>), dim3(nb), dim3(kLaneBlock), 0, s, (const R*)m, ld, n,
                     (const R*)cb, (R*)mb);
}
template <class L, int G, class R, bool BATCH, bool PERSIST, int K = 1>
void launch_backward_gp(const SysArgs& a, int i0, int n, const void* mb, long ld, double* g,
                        int acc, double* wpart, double* watom, double* fown, hipStream_t s) {
  const int nb = pair_grid(a, split_tiles(n, K));
  if (a.ncheb == 8)
    hipLaunchKernelGGL((k_backward<L, G, R, BATCH, 8, PERSIST, K>), dim3(nb), dim3(kLaneBlock), 0, s, a, i0, n,
                       (const R*)mb, ld, g, acc, wpart, watom, fown);
  else if (a.ncheb == 10)
    hipLaunchKernelGGL((k_backward<L, G, R, BATCH, 10, PERSIST, K>), dim3(nb), dim3(kLaneBlock), 0, s, a, i0, n,
                       (const R*)mb, ld, g, acc, wpart, watom, fown);
  else
    hipLaunchKernelGGL((k_backward<L, G, R, BATCH, 0, PERSIST, K>), dim3(nb), dim3(kLaneBlock), 0, s, a, i0, n,
                       (const R*)mb, ld, g, acc, wpart, watom, fown);
}
// the virial partials: one per workgroup, split_tiles(n, a.split) of them for a single system
template <class L, int G, class R, bool BATCH>
void launch_backward_g(const SysArgs& a, int i0, int n, const void* mb, long ld, double* g,
                       int acc, double* wpart, double* watom, double* fown, hipStream_t s) {
  if constexpr (BATCH) {
    if (a.queue) return launch_backward_gp<L, G, R, BATCH, true>(a, i0, n, mb, ld, g, acc, wpart, watom, fown, s);
  } else if constexpr (std::is_same_v<R, double>) {
    if (a.split == 2) return launch_backward_gp<L, G, R, BATCH, false, 2>(a, i0, n, mb, ld, g, acc, wpart, watom, fown, s);
    if (a.split == 4) return launch_backward_gp<L, G, R, BATCH, false, 4>(a, i0, n, mb, ld, g, acc, wpart, watom, fown, s);
    if (a.split == 8) return launch_backward_gp<L, G, R, BATCH, false, 8>(a, i0, n, mb, ld, g, acc, wpart, watom, fown, s);
  }
  launch_backward_gp<L, G, R, BATCH, false>(a, i0, n, mb, ld, g, acc, wpart, watom, fown, s);
}

template <class L, class R, bool BATCH, size_t... Gs>
void dispatch_moments(int g, const SysArgs& a, int i0, int n, void* m, long ld, hipStream_t s,
                      std::index_sequence<Gs...>) {
  ((g == (int)Gs ? launch_moments_g<L, (int)Gs, R, BATCH>(a, i0, n, m, ld, s) : void()), ...);
}
template <class L, class R, size_t... Gs>
void dispatch_rev(int g, const void* m, long ld, int n, const void* cb, void* mb, hipStream_t s,
                  std::index_sequence<Gs...>) {
  ((g == (int)Gs ? launch_rev_g<L, (int)Gs, R>(m, ld, n, cb, mb, s) : void()), ...);
}
template <class L, class R, bool BATCH, size_t... Gs>
void dispatch_backward(int g, const SysArgs& a, int i0, int n, const void* mb, long ld,
                       double* gout, int acc, double* wpart, double* watom, double* fown, hipStream_t s,
                       std::index_sequence<Gs...>) {
  ((g == (int)Gs ? launch_backward_g<L, (int)Gs, R, BATCH>(a, i0, n, mb, ld, gout, acc, wpart, watom, fown, s)
                 : void()),
   ...);
}

template <class L, class R, bool BATCH>
struct EnergyChain {
  static void moments(int g, const SysArgs& a, int i0, int n, void* m, long ld, hipStream_t s) {
    dispatch_moments<L, R, BATCH>(g, a, i0, n, m, ld, s, std::make_index_sequence<L::NGROUP>{});
  }
  static void prog_fwd(const void* m, long ld, int i0, int n, const int* perm, const int* species,
                       const double* xi, const double* shift, int nsp, double* e_atom, void* cbar,
                       double* bout, hipStream_t s) {
    const int nb = (n + kLaneBlock - 1) / kLaneBlock;
    hipLaunchKernelGGL((k_program_fwd<L, R>), dim3(nb), dim3(kLaneBlock), 0, s, (const R*)m, ld, i0, n,
                       perm, species, xi, shift, nsp, e_atom, (R*)cbar, bout);
  }
  static void prog_rev(int g, const void* m, long ld, int n, const void* cb, void* mb, hipStream_t s) {
    dispatch_rev<L, R>(g, m, ld, n, cb, mb, s, std::make_index_sequence<L::NGROUP>{});
  }
  static void backward(int grp, const SysArgs& a, int i0, int n, const void* mb, long ld, double* gout,
                       int acc, double* wpart, double* watom, double* fown, hipStream_t s) {
    dispatch_backward<L, R, BATCH>(grp, a, i0, n, mb, ld, gout, acc, wpart, watom, fown, s,
                                   std::make_index_sequence<L::NGROUP>{});
  }
  static void program(const void* m, long ld, int i0, int n, const int* species, const double* xi,
                      const double* shift, int nsp, double* e_atom, void* mb, hipStream_t s) {
    if constexpr (L::NGROUP == 1) {
      const int nb = (n + kLaneBlock - 1) / kLaneBlock;
      hipLaunchKernelGGL((k_program<L, R>), dim3(nb), dim3(kLaneBlock), 0, s, (const R*)m, ld, i0, n, species, xi,
                         shift, nsp, e_atom, (R*)mb);
    }
  }
  static ChainOps ops() {
    return ChainOps{&moments, &prog_fwd, &prog_rev, &backward, L::NGROUP == 1 && !BATCH ? &program : nullptr};
  }
};

template <class L>
struct AdjImpl {
  template <int G>
  static void tan_moments_g(const SysArgs& a, const double* fbar, int i0, int n, double* md, long ld,
                            hipStream_t s) {
    const int nb = pair_grid(a, (n + kLaneBlock - 1) / kLaneBlock);
    if (a.queue)
      hipLaunchKernelGGL((k_tan_moments<L, G, true>), dim3(nb), dim3(kLaneBlock), 0, s, a, fbar, i0, n, md, ld);
    else
      hipLaunchKernelGGL((k_tan_moments<L, G, false>), dim3(nb), dim3(kLaneBlock), 0, s, a, fbar, i0, n, md, ld);
  }
  template <size_t... Gs>
  static void tan_moments_d(int g, const SysArgs& a, const double* fbar, int i0, int n, double* md, long ld,
                            hipStream_t s, std::index_sequence<Gs...>) {
    ((g == (int)Gs ? tan_moments_g<(int)Gs>(a, fbar, i0, n, md, ld, s) : void()), ...);
  }
  static void tan_moments(int g, const SysArgs& a, const double* fbar, int i0, int n, double* md, long ld,
                          hipStream_t s) {
    tan_moments_d(g, a, fbar, i0, n, md, ld, s, std::make_index_sequence<L::NTGROUP>{});
  }
  static void tan_forward(const SysArgs& a, const double* m, const double* md, long ld, int i0, int n,
                          const double* xi, double ebar, double* out, double* cbard, hipStream_t s) {
    const int nb = (n + kLaneBlock - 1) / kLaneBlock;
    hipLaunchKernelGGL((k_tan_forward<L>), dim3(nb), dim3(kLaneBlock), 0, s, m, md, ld, i0, n, a.perm, a.cfg,
                       a.ebar, xi, ebar, out, cbard);
  }
  template <int P>
  static void tan_reverse_g(const double* m, const double* md, long ld, int n, const double* cb,
                            const double* cbd, double* mbd, hipStream_t s) {
    const int nb = (n + kLaneBlock - 1) / kLaneBlock;
    hipLaunchKernelGGL((k_tan_reverse<L, P>), dim3(nb), dim3(kLaneBlock), 0, s, m, md, ld, n, cb, cbd, mbd);
  }
  template <int G>
  static void adj_pairs_g(const SysArgs& a, const double* fbar, int i0, int n, const double* mb,
                          const double* mbd, long ld, double ebar, double* cpart, hipStream_t s) {
    const int nb = pair_grid(a, (n + kLaneBlock - 1) / kLaneBlock);
    if (a.queue) adj_pairs_gp<G, true>(nb, a, fbar, i0, n, mb, mbd, ld, ebar, cpart, s);
    else adj_pairs_gp<G, false>(nb, a, fbar, i0, n, mb, mbd, ld, ebar, cpart, s);
  }
  template <int G, bool P>
  static void adj_pairs_gp(int nb, const SysArgs& a, const double* fbar, int i0, int n, const double* mb,
                           const double* mbd, long ld, double ebar, double* cpart, hipStream_t s) {
    if (a.ncheb == 8)
      hipLaunchKernelGGL((k_adj_pairs<L, G, 8, P>), dim3(nb), dim3(kLaneBlock), 0, s, a, fbar, i0, n, mb, mbd, ld,
                         ebar, cpart);
    else if (a.ncheb == 10)
      hipLaunchKernelGGL((k_adj_pairs<L, G, 10, P>), dim3(nb), dim3(kLaneBlock), 0, s, a, fbar, i0, n, mb, mbd, ld,
                         ebar, cpart);
    else
      hipLaunchKernelGGL((k_adj_pairs<L, G, 0, P>), dim3(nb), dim3(kLaneBlock), 0, s, a, fbar, i0, n, mb, mbd, ld,
                         ebar, cpart);
  }
  template <size_t... Gs>
  static void adj_pairs_d(int g, const SysArgs& a, const double* fbar, int i0, int n, const double* mb,
                          const double* mbd, long ld, double ebar, double* cpart, hipStream_t s,
                          std::index_sequence<Gs...>) {
    ((g == (int)Gs ? adj_pairs_g<(int)Gs>(a, fbar, i0, n, mb, mbd, ld, ebar, cpart, s) : void()), ...);
  }
  static void adj_pairs(int g, const SysArgs& a, const double* fbar, int i0, int n, const double* mb,
                        const double* mbd, long ld, double ebar, double* cpart, hipStream_t s) {
    adj_pairs_d(g, a, fbar, i0, n, mb, mbd, ld, ebar, cpart, s, std::make_index_sequence<L::NAGROUP>{});
  }
  static AdjOps ops() {
    AdjOps o{};
    o.tan_moments = &tan_moments;
    o.adj_pairs = &adj_pairs;
    o.nagroup = L::NAGROUP;
    o.ntgroup = L::NTGROUP;
    o.nrtpart = L::NRTPART;
    static_assert(L::NRTPART <= kMaxRevParts, "reverse-tangent parts");
    return o;
  }
};

}  // namespace mtp

// One level is compiled as several translation units (binary64 chain, binary32 chain,
// adjoint, assembly) so that large levels build in parallel.
#define MTP_DEFINE_CHAIN(LV, NUM, TYPE, BATCH, TAG) \
  namespace mtp {                                   \
  ChainOps chain_ops_##NUM##_##TAG() { return EnergyChain<LV, TYPE, BATCH>::ops(); } \
  }
#define MTP_DEFINE_ADJ(LV, NUM) \
  namespace mtp {               \
  AdjOps adj_ops_##NUM() { return AdjImpl<LV>::ops(); } \
  }
#define MTP_DEFINE_ADJ_FWD(LV, NUM) \
  namespace mtp {                   \
  void adj_fwd_##NUM(const SysArgs& a, const double* m, const double* md, long ld, int i0, int n, \
                     const double* xi, double ebar, double* out, double* cbard, hipStream_t s) { \
    AdjImpl<LV>::tan_forward(a, m, md, ld, i0, n, xi, ebar, out, cbard, s);                     \
  }                                                                                             \
  }
#define MTP_DEFINE_ADJ_REV(LV, NUM, G) \
  namespace mtp {                      \
  void adj_rev_##NUM##_##G(const double* m, const double* md, long ld, int n, const double* cb, \
                           const double* cbd, double* mbd, hipStream_t s) {                     \
    AdjImpl<LV>::tan_reverse_g<G>(m, md, ld, n, cb, cbd, mbd, s);                             \
  }                                                                                          \
  }
