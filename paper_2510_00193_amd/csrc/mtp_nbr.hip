// Canonical periodic neighbour list on the GPU.
//
// Output: CSR rows sorted by (j, n1, n2, n3), the mirrored-pair index rev, and the shifts packed
// as three int8.  A pair is kept iff its squared distance, formed by the fixed binary64
// expression of pair_displacement/dist2_exact, is below r_cut^2 (strict).  Two candidate
// generators feed that one predicate:
//   - cells:  atoms binned in fractional coordinates, bins at least r_cut wide in every
//             perpendicular direction, so every pair lies in one of the 27 surrounding bins;
//   - images: every j of the system with the image range that can reach the cutoff,
//             |s_j,k - s_i,k + n_k| < r_cut |b_k| (+ a rounding margin); used for small or
//             thin cells, where an atom may see several images of one partner.
// The candidate sets are supersets of the true set, so both give the same list.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "mtp.h"
#include "mtp_device.h"
#include "mtp_internal.h"

namespace mtp {

namespace {

constexpr int kNT = 256;
constexpr double kImageMargin = 1e-6;  // fractional-coordinate slack of the image ranges

__device__ __forceinline__ long long make_key(int j, int n1, int n2, int n3) {
  return ((long long)j << 24) | ((long long)(n1 + 128) << 16) | ((long long)(n2 + 128) << 8) |
         (long long)(n3 + 128);
}

__device__ __forceinline__ void frac_of(const double* __restrict__ pos, int i,
                                        const double* __restrict__ Hinv, double* s) {
  const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
#pragma unroll
  for (int k = 0; k < 3; ++k) s[k] = x * Hinv[k] + y * Hinv[3 + k] + z * Hinv[6 + k];
}

struct PlanArgs {
  double H[9];
  double Hinv[9];
  double reach[3];
  int nb[3];
  double rc2;
};

// ---------------------------------------------------------------- image path
__global__ void k_frac(const double* __restrict__ pos, const int* __restrict__ species, int nsp, int n,
                       PlanArgs pa, double* __restrict__ s, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) flag[0] = 1;
  if (species[i] < 0 || species[i] >= nsp) flag[1] = 1;
  double f[3];
  frac_of(pos, i, pa.Hinv, f);
  s[3 * i] = f[0];
  s[3 * i + 1] = f[1];
  s[3 * i + 2] = f[2];
}

template <bool FILL>
__device__ __forceinline__ int image_row(int i, const double* __restrict__ pos,
                                         const double* __restrict__ s, int jlo, int jhi,
                                         const double* __restrict__ H, const double* __restrict__ reach,
                                         double rc2, int* __restrict__ nj, int* __restrict__ shift,
                                         long long* __restrict__ key, int base,
                                         int* __restrict__ flag) {
  const double six = s[3 * i], siy = s[3 * i + 1], siz = s[3 * i + 2];
  const double rix = pos[3 * i], riy = pos[3 * i + 1], riz = pos[3 * i + 2];
  const double re0 = reach[0], re1 = reach[1], re2 = reach[2];
  int cnt = 0;
  for (int j = jlo; j < jhi; ++j) {
    const double ds0 = s[3 * j] - six, ds1 = s[3 * j + 1] - siy, ds2 = s[3 * j + 2] - siz;
    const int lo0 = (int)ceil(-re0 - ds0 - kImageMargin);
    const int hi0 = (int)floor(re0 - ds0 + kImageMargin);
    const int lo1 = (int)ceil(-re1 - ds1 - kImageMargin);
    const int hi1 = (int)floor(re1 - ds1 + kImageMargin);
    const int lo2 = (int)ceil(-re2 - ds2 - kImageMargin);
    const int hi2 = (int)floor(re2 - ds2 + kImageMargin);
    if (min(lo0, min(lo1, lo2)) < -127 || max(hi0, max(hi1, hi2)) > 127) {
      // shifts must fit the packed int8 fields; the count pass reports it
      if (!FILL) flag[2] = 1;
      continue;
    }
    const double rjx = pos[3 * j], rjy = pos[3 * j + 1], rjz = pos[3 * j + 2];
    for (int n1 = lo0; n1 <= hi0; ++n1)
      for (int n2 = lo1; n2 <= hi1; ++n2)
        for (int n3 = lo2; n3 <= hi2; ++n3) {
          if (j == i && n1 == 0 && n2 == 0 && n3 == 0) continue;
          double dx, dy, dz;
          pair_displacement(rix, riy, riz, rjx, rjy, rjz, n1, n2, n3, H, dx, dy, dz);
          if (dist2_exact(dx, dy, dz) < rc2) {
            if (FILL) {
              const int p = base + cnt;
              nj[p] = j;
              shift[p] = (n1 & 0xFF) | ((n2 & 0xFF) << 8) | ((n3 & 0xFF) << 16);
              key[p] = make_key(j, n1, n2, n3);
            }
            ++cnt;
          }
        }
  }
  return cnt;
}

__global__ void k_image_count(const double* __restrict__ pos, const double* __restrict__ s, int n,
                              PlanArgs pa, int* __restrict__ counts, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  counts[i] = image_row<false>(i, pos, s, 0, n, pa.H, pa.reach, pa.rc2, nullptr, nullptr, nullptr, 0, flag);
}

__global__ void k_image_fill(const double* __restrict__ pos, const double* __restrict__ s, int n,
                             PlanArgs pa, const int* __restrict__ off, int* __restrict__ nj,
                             int* __restrict__ shift, long long* __restrict__ key) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  image_row<true>(i, pos, s, 0, n, pa.H, pa.reach, pa.rc2, nj, shift, key, off[i], nullptr);
}

// ---------------------------------------------------------------- batches (image path per configuration)
// cells/cinv: [n_cfg][9], reach: [n_cfg][3], atom_off: [n_cfg + 1], cfg: [N]
__global__ void k_batch_frac(const double* __restrict__ pos, const int* __restrict__ species, int nsp,
                             const int* __restrict__ cfg, const double* __restrict__ cinv, int n,
                             double* __restrict__ s, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) flag[0] = 1;
  if (species[i] < 0 || species[i] >= nsp) flag[1] = 1;
  const double* Hinv = cinv + 9L * cfg[i];
  double f[3];
  frac_of(pos, i, Hinv, f);
  s[3 * i] = f[0];
  s[3 * i + 1] = f[1];
  s[3 * i + 2] = f[2];
}

__global__ void k_batch_count(const double* __restrict__ pos, const double* __restrict__ s,
                              const int* __restrict__ cfg, const int* __restrict__ atom_off,
                              const double* __restrict__ cells, const double* __restrict__ reach,
                              double rc2, int n, int* __restrict__ counts, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cfg[i];
  counts[i] = image_row<false>(i, pos, s, atom_off[c], atom_off[c + 1], cells + 9L * c, reach + 3L * c,
                               rc2, nullptr, nullptr, nullptr, 0, flag);
}

__global__ void k_batch_fill(const double* __restrict__ pos, const double* __restrict__ s,
                             const int* __restrict__ cfg, const int* __restrict__ atom_off,
                             const double* __restrict__ cells, const double* __restrict__ reach,
                             double rc2, int n, const int* __restrict__ off, int* __restrict__ nj,
                             int* __restrict__ shift, long long* __restrict__ key) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cfg[i];
  image_row<true>(i, pos, s, atom_off[c], atom_off[c + 1], cells + 9L * c, reach + 3L * c, rc2, nj,
                  shift, key, off[i], nullptr);
}

// ---------------------------------------------------------------- cell path
// counter[key] += 1 for every active lane, with one atomic per distinct key among the lanes of
// the wave: the lowest remaining lane leads its key's lanes, adds their count, and each lane
// gets the old value plus its rank among them in lane order.  (Atoms in index order mostly share
// bins with their neighbours in the wave, so this replaces about eight atomics on one address
// by one: the scatter into bins 72 -> 55 us at 1,024,000 atoms; the plain count, whose result
// is unused, was not faster with it.)
__device__ __forceinline__ int wave_counted_inc(int* counter, int key) {
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(1);
  int result = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lkey = __shfl(key, leader, 64);
    const unsigned long long same = __ballot(key == lkey) & todo;
    int base = 0;
    if (lane == leader) base = atomicAdd(&counter[lkey], __popcll(same));
    base = __shfl(base, leader, 64);
    if (key == lkey) result = base + __popcll(same & ((1ull << lane) - 1ull));
    todo &= ~same;
  }
  return result;
}

__global__ void k_bin(const double* __restrict__ pos, const int* __restrict__ species, int nsp, int n,
                      PlanArgs pa, int* __restrict__ bin, int* __restrict__ img,
                      int* __restrict__ bincount, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (species[i] < 0 || species[i] >= nsp) flag[1] = 1;
  const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
    flag[0] = 1;
    bin[i] = 0;
    img[3 * i] = img[3 * i + 1] = img[3 * i + 2] = 0;
    atomicAdd(&bincount[0], 1);
    return;
  }
  // the staged path's distance filter assumes coordinates below 1e7 (its margin covers the
  // rounding of such magnitudes); larger ones take the unstaged path
  if (fabs(x) > 1e7 || fabs(y) > 1e7 || fabs(z) > 1e7) flag[3] = 1;
  double f[3];
  frac_of(pos, i, pa.Hinv, f);
  int b[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double o = floor(f[k]);
    double w = f[k] - o;
    if (w >= 1.0) {
      w -= 1.0;
      o += 1.0;
    }
    if (fabs(o) > 60.0) {  // image offsets must keep |n| within the packed int8 range
      flag[2] = 1;
      o = 0.0;
    }
    img[3 * i + k] = (int)o;
    b[k] = min((int)(w * pa.nb[k]), pa.nb[k] - 1);
  }
  const int id = (b[0] * pa.nb[1] + b[1]) * pa.nb[2] + b[2];
  bin[i] = id;
  atomicAdd(&bincount[id], 1);
}

// Image offsets of one atom packed as three biased bytes (|offset| <= 60 by the binning check).
__device__ __forceinline__ int pack_img(int o0, int o1, int o2) {
  return ((o0 + 128) << 16) | ((o1 + 128) << 8) | (o2 + 128);
}

// Bin contents: atom index, and (for the staged path) binned copies of the position and of the
// packed image offsets, so that a bin's atoms are contiguous in memory.
__global__ void k_bin_scatter(int n, const int* __restrict__ bin, const int* __restrict__ binstart,
                              int* __restrict__ binfill, int* __restrict__ binatoms,
                              const double* __restrict__ pos, const int* __restrict__ img,
                              double* __restrict__ binpos, int* __restrict__ binimg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int id = bin[i];
  const int q = binstart[id] + wave_counted_inc(binfill, id);
  binatoms[q] = i;
  if (binpos) {
    binpos[3L * q] = pos[3 * i];
    binpos[3L * q + 1] = pos[3 * i + 1];
    binpos[3L * q + 2] = pos[3 * i + 2];
    binimg[q] = pack_img(img[3 * i], img[3 * i + 1], img[3 * i + 2]);
  }
}

template <bool FILL>
__device__ __forceinline__ int cell_row(int i, const double* __restrict__ pos, const PlanArgs& pa,
                                        const int* __restrict__ bin, const int* __restrict__ img,
                                        const int* __restrict__ binstart,
                                        const int* __restrict__ binatoms, long long* __restrict__ key,
                                        int* __restrict__ rowid, int base) {
  const int id = bin[i];
  const int b2 = id % pa.nb[2];
  const int b1 = (id / pa.nb[2]) % pa.nb[1];
  const int b0 = id / (pa.nb[2] * pa.nb[1]);
  const int oi0 = img[3 * i], oi1 = img[3 * i + 1], oi2 = img[3 * i + 2];
  const double rix = pos[3 * i], riy = pos[3 * i + 1], riz = pos[3 * i + 2];
  int cnt = 0;
  for (int d0 = -1; d0 <= 1; ++d0) {
    int c0 = b0 + d0, w0 = 0;
    if (c0 < 0) { c0 += pa.nb[0]; w0 = -1; }
    if (c0 >= pa.nb[0]) { c0 -= pa.nb[0]; w0 = 1; }
    if (pa.nb[0] == 1) { c0 = 0; w0 = d0; }
    for (int d1 = -1; d1 <= 1; ++d1) {
      int c1 = b1 + d1, w1 = 0;
      if (c1 < 0) { c1 += pa.nb[1]; w1 = -1; }
      if (c1 >= pa.nb[1]) { c1 -= pa.nb[1]; w1 = 1; }
      if (pa.nb[1] == 1) { c1 = 0; w1 = d1; }
      for (int d2 = -1; d2 <= 1; ++d2) {
        int c2 = b2 + d2, w2 = 0;
        if (c2 < 0) { c2 += pa.nb[2]; w2 = -1; }
        if (c2 >= pa.nb[2]) { c2 -= pa.nb[2]; w2 = 1; }
        if (pa.nb[2] == 1) { c2 = 0; w2 = d2; }
        const int cid = (c0 * pa.nb[1] + c1) * pa.nb[2] + c2;
        const int q0 = binstart[cid], q1 = binstart[cid + 1];
        for (int q = q0; q < q1; ++q) {
          const int j = binatoms[q];
          const int n1 = w0 + oi0 - img[3 * j];
          const int n2 = w1 + oi1 - img[3 * j + 1];
          const int n3 = w2 + oi2 - img[3 * j + 2];
          if (j == i && n1 == 0 && n2 == 0 && n3 == 0) continue;
          double dx, dy, dz;
          pair_displacement(rix, riy, riz, pos[3 * j], pos[3 * j + 1], pos[3 * j + 2], n1, n2, n3,
                            pa.H, dx, dy, dz);
          if (dist2_exact(dx, dy, dz) < pa.rc2) {
            if (FILL) {
              key[base + cnt] = make_key(j, n1, n2, n3);
              rowid[base + cnt] = i;
            }
            ++cnt;
          }
        }
      }
    }
  }
  return cnt;
}

__global__ void k_cell_count(const double* __restrict__ pos, int n, PlanArgs pa,
                             const int* __restrict__ bin, const int* __restrict__ img,
                             const int* __restrict__ binstart, const int* __restrict__ binatoms,
                             int* __restrict__ counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  counts[i] = cell_row<false>(i, pos, pa, bin, img, binstart, binatoms, nullptr, nullptr, 0);
}

__global__ void k_cell_fill(const double* __restrict__ pos, int n, PlanArgs pa,
                            const int* __restrict__ bin, const int* __restrict__ img,
                            const int* __restrict__ binstart, const int* __restrict__ binatoms,
                            const int* __restrict__ off, long long* __restrict__ key,
                            int* __restrict__ rowid) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cell_row<true>(i, pos, pa, bin, img, binstart, binatoms, key, rowid, off[i]);
}

// rank of each key inside its row (keys are distinct) -> sorted position
__global__ void k_row_sort(long long total, const int* __restrict__ off,
                           const int* __restrict__ rowid, const long long* __restrict__ key,
                           long long* __restrict__ skey, int* __restrict__ nj,
                           int* __restrict__ shift) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  const int i = rowid[p];
  const int q0 = off[i], q1 = off[i + 1];
  const long long k = key[p];
  int rank = 0;
  for (int q = q0; q < q1; ++q) rank += key[q] < k;
  const int dst = q0 + rank;
  skey[dst] = k;
  nj[dst] = (int)(k >> 24);
  const int n1 = (int)((k >> 16) & 0xFF) - 128, n2 = (int)((k >> 8) & 0xFF) - 128,
            n3 = (int)(k & 0xFF) - 128;
  shift[dst] = (n1 & 0xFF) | ((n2 & 0xFF) << 8) | ((n3 & 0xFF) << 16);
}

// row id of every pair (image path writes rows in order; rev needs the centre of each pair)
__global__ void k_rowid(int n, const int* __restrict__ off, int* __restrict__ rowid) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int p = off[i]; p < off[i + 1]; ++p) rowid[p] = i;
}

__global__ void k_rev(long long total, const int* __restrict__ off, const int* __restrict__ rowid,
                      const long long* __restrict__ skey, int* __restrict__ rev) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total) return;
  const long long k = skey[p];
  const int i = rowid[p];
  const int j = (int)(k >> 24);
  const int n1 = (int)((k >> 16) & 0xFF) - 128, n2 = (int)((k >> 8) & 0xFF) - 128,
            n3 = (int)(k & 0xFF) - 128;
  const long long want = make_key(i, -n1, -n2, -n3);
  int lo = off[j], hi = off[j + 1] - 1, found = -1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const long long v = skey[mid];
    if (v == want) {
      found = mid;
      break;
    }
    if (v < want) lo = mid + 1; else hi = mid - 1;
  }
  rev[p] = found;
}

// ---------------------------------------------------------------- cell path, one workgroup per brick
// A workgroup takes a brick of BX x BY x BZ bins and stages the candidates of the brick and
// of its one-bin halo in LDS once: for each, its position shifted by the image the halo bin's
// wrap implies, in binary32 relative to the halo's corner, and its key base (j, wrap - image of
// j).  Every lane then takes one centre atom of the brick; its 27 surrounding bins are 9 runs
// of three z-consecutive halo bins, contiguous in the staged list.
//   1. filter: the binary32 squared distance differs from the canonical binary64 expression
//      (pair_displacement/dist2_exact) by less than a margin the host derives from the brick's
//      extent, so candidates below r_cut^2 minus the margin are hits, those above r_cut^2 plus
//      the margin are not, and only those in between are marked for the canonical test; the
//      staged indices of the survivors go to the lane's list in LDS;
//   2. the survivors' keys (partner index, hit number) are sorted in registers by a bitonic
//      network (every partner appears once in a row when each axis has at least three bins),
//      the marked ones take the canonical test, and the sorted row of keys (j, n1, n2, n3) is
//      written at fixed capacity.
// k_rows_copy then writes the CSR arrays and pairs the mirrors.  A brick whose staged
// candidates exceed MAXC, or a row beyond ROWCAP, sets flag[3] and the caller takes the
// unstaged path.
constexpr int kBrickThreads = 256;
constexpr int kMaxHalo = 512;     // halo bins per brick (two per thread)
constexpr int kMaxInner = 128;    // interior bins per brick
constexpr int kBrickMaxC = 2048;  // staged candidates per brick
constexpr int kFilterStep = 4;    // candidates per step of the filter loop

struct BrickArgs {
  int bx[3];       // brick extent in bins
  int nbk[3];      // bricks per axis
  double margin;   // bound on |binary32 filter distance^2 - canonical distance^2|
};

__device__ __forceinline__ void shift_vec(int n1, int n2, int n3, const double* H, double& tx, double& ty,
                                          double& tz) {
  const double f1 = (double)n1, f2 = (double)n2, f3 = (double)n3;
  tx = (f1 * H[0] + f2 * H[3]) + f3 * H[6];
  ty = (f1 * H[1] + f2 * H[4]) + f3 * H[7];
  tz = (f1 * H[2] + f2 * H[5]) + f3 * H[8];
}

// inclusive scan of v over the workgroup (kBrickThreads lanes), through sh[kBrickThreads / 64]
__device__ __forceinline__ int block_incl_scan(int v, int* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  if (lane == 63) sh[wave] = v;
  __syncthreads();
  int add = 0;
  for (int w = 0; w < wave; ++w) add += sh[w];
  __syncthreads();
  return v + add;
}

// ascending bitonic sort of N values held in registers (N a power of two)
template <int N>
__device__ __forceinline__ void bitonic_sort(unsigned* v) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const unsigned a = v[i], b = v[l];
          const bool up = (i & k) == 0;
          v[i] = up ? min(a, b) : max(a, b);
          v[l] = up ? max(a, b) : min(a, b);
        }
      }
}

template <int MAXC, int ROWCAP>
__global__ __launch_bounds__(kBrickThreads) void k_brick_rows(PlanArgs pa, BrickArgs ba,
                                                              const int* __restrict__ binstart,
                                                              const int* __restrict__ binatoms,
                                                              const double* __restrict__ binpos,
                                                              const int* __restrict__ binimg,
                                                              const double* __restrict__ pos, int cap,
                                                              int* __restrict__ rows_j, int* __restrict__ rows_s,
                                                              int* __restrict__ counts, int* __restrict__ flag) {
  static_assert(ROWCAP <= 64, "hit numbers take six bits of the sort key");
  __shared__ float xs[MAXC + kFilterStep], ys[MAXC + kFilterStep], zs[MAXC + kFilterStep];
  __shared__ long long ckey[MAXC];
  __shared__ unsigned short hl[ROWCAP][kBrickThreads];
  __shared__ int hst[kMaxHalo], hoff[kMaxHalo + 1], hwrap[kMaxHalo];
  __shared__ int ioff[kMaxInner + 1], ihalo[kMaxInner];
  __shared__ int scan_sh[kBrickThreads / 64];
  __shared__ int skip;
  const int bid = blockIdx.x;
  const int k2 = bid % ba.nbk[2], k1 = (bid / ba.nbk[2]) % ba.nbk[1], k0 = bid / (ba.nbk[2] * ba.nbk[1]);
  const int x0 = k0 * ba.bx[0], y0 = k1 * ba.bx[1], z0 = k2 * ba.bx[2];
  const int ex = min(ba.bx[0], pa.nb[0] - x0), ey = min(ba.bx[1], pa.nb[1] - y0), ez = min(ba.bx[2], pa.nb[2] - z0);
  const int hx = ex + 2, hy = ey + 2, hz = ez + 2, nh = hx * hy * hz, ni = ex * ey * ez;
  if (threadIdx.x == 0) skip = flag[3];  // one read: the caller already falls back
  // halo bins in (x, y, z) order with z fastest: physical bin, wrap and atom count; thread t
  // takes halo bins 2t and 2t + 1
  int hc[2] = {0, 0};
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int h = 2 * threadIdx.x + u;
    if (h < nh) {
      const int a2 = h % hz, a1 = (h / hz) % hy, a0 = h / (hz * hy);
      int c0 = x0 - 1 + a0, c1 = y0 - 1 + a1, c2 = z0 - 1 + a2, w0 = 0, w1 = 0, w2 = 0;
      if (c0 < 0) { c0 += pa.nb[0]; w0 = -1; } else if (c0 >= pa.nb[0]) { c0 -= pa.nb[0]; w0 = 1; }
      if (c1 < 0) { c1 += pa.nb[1]; w1 = -1; } else if (c1 >= pa.nb[1]) { c1 -= pa.nb[1]; w1 = 1; }
      if (c2 < 0) { c2 += pa.nb[2]; w2 = -1; } else if (c2 >= pa.nb[2]) { c2 -= pa.nb[2]; w2 = 1; }
      const int cid = (c0 * pa.nb[1] + c1) * pa.nb[2] + c2;
      hst[h] = binstart[cid];
      hc[u] = binstart[cid + 1] - binstart[cid];
      hwrap[h] = pack_img(w0, w1, w2);
    }
  }
  {
    const int incl = block_incl_scan(hc[0] + hc[1], scan_sh);
    if (2 * threadIdx.x < nh) hoff[2 * threadIdx.x + 1] = incl - hc[1];
    if (2 * threadIdx.x + 1 < nh) hoff[2 * threadIdx.x + 2] = incl;
    if (threadIdx.x == 0) hoff[0] = 0;
  }
  __syncthreads();
  const int ncand = hoff[nh];
  if (skip) return;
  if (ncand > MAXC) {
    if (threadIdx.x == 0) flag[3] = 1;
    return;
  }
  // interior bins: halo index and running centre offsets
  {
    int c = 0;
    if (threadIdx.x < ni) {
      const int a2 = threadIdx.x % ez, a1 = (threadIdx.x / ez) % ey, a0 = threadIdx.x / (ez * ey);
      const int h = ((a0 + 1) * hy + (a1 + 1)) * hz + (a2 + 1);
      ihalo[threadIdx.x] = h;
      c = hoff[h + 1] - hoff[h];
    }
    const int incl = block_incl_scan(c, scan_sh);
    if (threadIdx.x < ni) ioff[threadIdx.x + 1] = incl;
    if (threadIdx.x == 0) ioff[0] = 0;
  }
  // halo corner (fractional (x0 - 1, y0 - 1, z0 - 1) / nb): origin of the binary32 coordinates
  double ox0, oy0, oz0;
  {
    const double f0 = (double)(x0 - 1) / pa.nb[0], f1 = (double)(y0 - 1) / pa.nb[1], f2 = (double)(z0 - 1) / pa.nb[2];
    ox0 = (f0 * pa.H[0] + f1 * pa.H[3]) + f2 * pa.H[6];
    oy0 = (f0 * pa.H[1] + f1 * pa.H[4]) + f2 * pa.H[7];
    oz0 = (f0 * pa.H[2] + f1 * pa.H[5]) + f2 * pa.H[8];
  }
  // stage the candidates
  for (int k = threadIdx.x; k < ncand; k += kBrickThreads) {
    int lo = 0, hi = nh - 1;  // halo bin t with hoff[t] <= k < hoff[t + 1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (hoff[mid] <= k) lo = mid; else hi = mid - 1;
    }
    const int q = hst[lo] + (k - hoff[lo]);
    const int j = binatoms[q];
    const int wr = hwrap[lo], im = binimg[q];
    const int c0 = ((wr >> 16) & 0xFF) - ((im >> 16) & 0xFF);
    const int c1 = ((wr >> 8) & 0xFF) - ((im >> 8) & 0xFF);
    const int c2 = (wr & 0xFF) - (im & 0xFF);
    double tx, ty, tz;
    shift_vec(c0, c1, c2, pa.H, tx, ty, tz);
    xs[k] = (float)((binpos[3L * q] + tx) - ox0);
    ys[k] = (float)((binpos[3L * q + 1] + ty) - oy0);
    zs[k] = (float)((binpos[3L * q + 2] + tz) - oz0);
    ckey[k] = make_key(j, c0, c1, c2);
  }
  if (threadIdx.x < kFilterStep) xs[ncand + threadIdx.x] = ys[ncand + threadIdx.x] = zs[ncand + threadIdx.x] = 1e30f;
  __syncthreads();
  const double rc2 = pa.rc2;
  const float rc_hi = (float)(rc2 + ba.margin), rc_lo = (float)(rc2 - ba.margin);
  const int ncent = ioff[ni];
  unsigned short* mylist = &hl[0][threadIdx.x];
  for (int c = threadIdx.x; c < ncent; c += kBrickThreads) {
    int lo = 0, hi = ni - 1;  // interior bin b with ioff[b] <= c < ioff[b + 1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ioff[mid] <= c) lo = mid; else hi = mid - 1;
    }
    const int h = ihalo[lo];
    const int cs = hst[h] + (c - ioff[lo]);  // the centre's slot in the binned arrays
    const int i = binatoms[cs];
    const double rix = pos[3L * i], riy = pos[3L * i + 1], riz = pos[3L * i + 2];
    const int im = binimg[cs];
    const int oi0 = ((im >> 16) & 0xFF) - 128, oi1 = ((im >> 8) & 0xFF) - 128, oi2 = (im & 0xFF) - 128;
    double sx, sy, sz;
    shift_vec(oi0, oi1, oi2, pa.H, sx, sy, sz);
    const float qx = (float)((rix - sx) - ox0), qy = (float)((riy - sy) - oy0), qz = (float)((riz - sz) - oz0);
    const long long self = make_key(i, 0, 0, 0);
    const long long koff = ((long long)oi0 << 16) + ((long long)oi1 << 8) + (long long)oi2;
    const int a2 = h % hz, a1 = (h / hz) % hy, a0 = h / (hz * hy);
    // 1. filter
    int cnt = 0;
    for (int r = 0; r < 9; ++r) {
      const int hb = ((a0 - 1 + r / 3) * hy + (a1 - 1 + r % 3)) * hz + (a2 - 1);
      const int q1 = hoff[hb + 3];
      // four candidates per step: their LDS reads are in flight together (reads past the run
      // stay inside the staged list, which is padded by kFilterStep entries, and are masked)
      for (int q = hoff[hb]; q < q1; q += kFilterStep) {
        float dd[kFilterStep];
#pragma unroll
        for (int u = 0; u < kFilterStep; ++u) {
          const float ex_ = xs[q + u] - qx, ey_ = ys[q + u] - qy, ez_ = zs[q + u] - qz;
          dd[u] = fmaf(ez_, ez_, fmaf(ey_, ey_, ex_ * ex_));
        }
#pragma unroll
        for (int u = 0; u < kFilterStep; ++u) {
          if (q + u < q1 && dd[u] < rc_hi) {
            if (cnt < ROWCAP)
              mylist[cnt * kBrickThreads] = (unsigned short)((q + u) | (dd[u] >= rc_lo ? 0x8000 : 0));
            ++cnt;
          }
        }
      }
    }
    if (cnt > ROWCAP || cnt > cap) {
      flag[3] = 1;
      counts[i] = 0;
      continue;
    }
    // 2. keys (partner << 6 | hit number) of the hits, sorted in registers
    unsigned v[ROWCAP];
#pragma unroll
    for (int t = 0; t < ROWCAP; ++t) {
      v[t] = 0xFFFFFFFFu;
      if (t < cnt) {  // (the bitonic network below only sorts what is set here)
        const unsigned u = mylist[t * kBrickThreads];
        const long long key = ckey[u & 0x7FFF] + koff;
        bool hit = key != self;
        if (hit && (u & 0x8000)) {  // inside the margin: the canonical expression decides
          const int j = (int)(key >> 24);
          const int n1 = (int)((key >> 16) & 0xFF) - 128, n2 = (int)((key >> 8) & 0xFF) - 128,
                    n3 = (int)(key & 0xFF) - 128;
          double dx, dy, dz;
          pair_displacement(rix, riy, riz, pos[3L * j], pos[3L * j + 1], pos[3L * j + 2], n1, n2, n3, pa.H, dx, dy,
                            dz);
          hit = dist2_exact(dx, dy, dz) < rc2;
        }
        if (hit) v[t] = ((unsigned)(key >> 24) << 6) | (unsigned)t;
      }
    }
    // sort the first 32 keys only when no lane of the wave has more hits
    const bool small = __all(cnt <= 32);
    if (small) bitonic_sort<32>(v);
    else bitonic_sort<ROWCAP>(v);
    // the row in registers (partners, packed images; the first 32 partner slots padded with
    // INT_MAX, which k_rows_copy ranks against unmasked), then stored four slots per 16-byte
    // store, as far as the row or the padded slots reach
    int* rj = rows_j + (long)i * cap;
    int* rs = rows_s + (long)i * cap;
    int jv[ROWCAP], sv[ROWCAP];
    int m = 0;
#pragma unroll
    for (int t = 0; t < ROWCAP; ++t) {
      jv[t] = 0x7FFFFFFF;
      sv[t] = 0;
      if ((t < 32 || !small) && v[t] != 0xFFFFFFFFu) {
        const unsigned u = mylist[(v[t] & 63u) * kBrickThreads];
        const long long key = ckey[u & 0x7FFF] + koff;
        const int n1 = (int)((key >> 16) & 0xFF) - 128, n2 = (int)((key >> 8) & 0xFF) - 128,
                  n3 = (int)(key & 0xFF) - 128;
        jv[t] = (int)(key >> 24);
        sv[t] = (n1 & 0xFF) | ((n2 & 0xFF) << 8) | ((n3 & 0xFF) << 16);
        ++m;
      }
    }
#pragma unroll
    for (int g = 0; g < ROWCAP / 4; ++g) {
      if (4 * g < 32 || 4 * g < m) {
        reinterpret_cast<int4*>(rj)[g] = make_int4(jv[4 * g], jv[4 * g + 1], jv[4 * g + 2], jv[4 * g + 3]);
        if (4 * g < m) reinterpret_cast<int4*>(rs)[g] = make_int4(sv[4 * g], sv[4 * g + 1], sv[4 * g + 2], sv[4 * g + 3]);
      }
    }
    counts[i] = m;
  }
}

// Sorted fixed-capacity rows -> CSR j / packed shift, and the mirror index.  Rows built by
// k_brick_rows hold each partner once, sorted by partner, and their first 32 slots are padded
// with INT_MAX, so the mirror of (i, j, n) is entry off[j] + #{u : rows_j[j][u] < i}.
// G lanes per row, E entries per lane (entries t and t + G of the row); a wave holds 64 / G rows
// (one entry per lane measured fastest: two per lane halve the waves but slowed the copy by a third).
// The wave counts cooperatively: in step v of entry slot e, the eight lanes 8k..8k+7 read the
// eight 16-byte pieces of the first 32 slots of the row of lane 8(v % 8) + k's entry e (one
// 128-byte line per eight lanes instead of a line per lane), count the entries below that
// lane's i and sum over the eight lanes; one exchange at the end hands each lane its count (lane
// 8k + m keeps step m's sum).  All exchanges and loads of a lane are issued before
// the first count, so a wave has every load of its rows in flight at once.  A row with all of
// its first 32 entries below i continues alone, four entries at a time, up to counts[j].
constexpr int kCsrThreads = 256;
// sum over the eight lanes 8k..8k+7 with DPP lane exchanges (quads, then half-rows); every lane
// of the eight ends with the same sum
__device__ __forceinline__ int sum8(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1, 0, 3, 2]
  v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2, 3, 0, 1]
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  return v;
}

// i_lane0: the row of lane 0 of the wave; G lanes per row, so lane s's row is i_lane0 + s / G
template <int CAP, int E, int G>
__device__ __forceinline__ void mirror_rank(const int* __restrict__ rows_j, const int* __restrict__ counts,
                                            int i, int i_lane0, const int (&j)[E], int (&rank)[E]) {
  const int l = threadIdx.x & 63;
  int js[E][8], is[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int src = 8 * v + (l >> 3);
    is[v] = i_lane0 + src / G;
#pragma unroll
    for (int e = 0; e < E; ++e) js[e][v] = __shfl(j[e], src, 64);
  }
  int4 q[E][8];
#pragma unroll
  for (int e = 0; e < E; ++e)
#pragma unroll
    for (int v = 0; v < 8; ++v)
      q[e][v] = reinterpret_cast<const int4*>(rows_j + (long)max(js[e][v], 0) * CAP)[l & 7];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    int mine = 0;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int x = is[v];
      const int4 w = q[e][v];
      const int part = sum8(js[e][v] >= 0 ? (w.x < x) + (w.y < x) + (w.z < x) + (w.w < x) : 0);
      if ((l & 7) == v) mine = part;
    }
    rank[e] = __shfl(mine, 8 * (l & 7) + (l >> 3), 64);
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (j[e] >= 0 && rank[e] == 32) {
      const int cj = counts[j[e]];
      const int4* row = reinterpret_cast<const int4*>(rows_j + (long)j[e] * CAP);
      for (int u = 8; 4 * u < cj; ++u) {
        const int4 w = row[u];
        rank[e] += (4 * u + 0 < cj && w.x < i) + (4 * u + 1 < cj && w.y < i) + (4 * u + 2 < cj && w.z < i) +
                   (4 * u + 3 < cj && w.w < i);
      }
    }
  }
}

template <int G, int E, int CAP>
__global__ __launch_bounds__(kCsrThreads) void k_rows_copy(int n, const int* __restrict__ rows_j,
                                                           const int* __restrict__ rows_s,
                                                           const int* __restrict__ counts,
                                                           const int* __restrict__ off, int* __restrict__ nj,
                                                           int* __restrict__ shift, int* __restrict__ rev) {
  static_assert(CAP >= 32 && CAP % 4 == 0 && CAP % (G * E) == 0 && 64 % G == 0, "row layout");
  constexpr int R = kCsrThreads / G;
  const int b = xcd_logical_block(blockIdx.x, gridDim.x);
  const int i = b * R + threadIdx.x / G, lane = threadIdx.x % G;
  // no early exit: the rank count exchanges values across the whole wave
  const int ic = min(i, n - 1);  // rows past the end read row n - 1 and write nothing
  const int cnt = i < n ? counts[i] : 0, o = off[ic];
  for (int t0 = 0; t0 < CAP; t0 += G * E) {
    if (!__any(t0 < cnt)) break;
    int j[E], sr[E], oj[E], rank[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = t0 + lane + e * G;
      const int jr = rows_j[(long)ic * CAP + t];
      sr[e] = rows_s[(long)ic * CAP + t];
      j[e] = t < cnt ? jr : -1;
    }
    if (rev) {
#pragma unroll
      for (int e = 0; e < E; ++e) oj[e] = off[max(j[e], 0)];
      mirror_rank<CAP, E, G>(rows_j, counts, i, b * R + (int)(threadIdx.x & ~63u) / G, j, rank);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = t0 + lane + e * G;
      if (t < cnt) {
        nj[o + t] = j[e];
        shift[o + t] = sr[e];
        if (rev) rev[o + t] = oj[e] + rank[e];
      }
    }
  }
}

// ---------------------------------------------------------------- exclusive scan (int)
constexpr int kScanPer = 8;
constexpr int kScanBlock = kNT * kScanPer;

__global__ void k_scan_local(const int* __restrict__ in, int n, int* __restrict__ out,
                             long long* __restrict__ bsum) {
  __shared__ long long sh[kNT];
  const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
  long long v[kScanPer];
  long long acc = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    acc += v[k];
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 1; s < kNT; s <<= 1) {
    long long t = threadIdx.x >= s ? sh[threadIdx.x - s] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  long long run = sh[threadIdx.x] - acc;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) out[base + k] = (int)run;
    run += v[k];
  }
  if (threadIdx.x == kNT - 1) bsum[blockIdx.x] = sh[kNT - 1];
}

// exclusive scan of the block sums by one workgroup: each thread scans a contiguous run,
// then the run totals are scanned in LDS
constexpr int kScanTop = 1024;
__global__ __launch_bounds__(kScanTop) void k_scan_blocks(long long* __restrict__ bsum, int nb,
                                                          long long* __restrict__ total) {
  __shared__ long long sh[kScanTop];
  const int per = (nb + kScanTop - 1) / kScanTop;
  const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
  long long acc = 0;
  for (int b = b0; b < b1; ++b) acc += bsum[b];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 1; s < kScanTop; s <<= 1) {
    const long long t = threadIdx.x >= s ? sh[threadIdx.x - s] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  long long run = sh[threadIdx.x] - acc;
  for (int b = b0; b < b1; ++b) {
    const long long t = bsum[b];
    bsum[b] = run;
    run += t;
  }
  if (threadIdx.x == kScanTop - 1) total[0] = sh[kScanTop - 1];
}

__global__ void k_scan_add(int* __restrict__ out, int n, const long long* __restrict__ bsum,
                           const long long* __restrict__ total, int write_total) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (int)(out[i] + bsum[i / kScanBlock]);
  if (write_total && i == 0) out[n] = (int)total[0];
}

}  // namespace

// ---------------------------------------------------------------- workspace
struct NbrWork {
  size_t cap[20] = {0};
  void* ptr[20] = {nullptr};
  template <class T>
  T* get(int slot, size_t n) {
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    if (cap[slot] < bytes) {
      if (ptr[slot]) (void)hipFree(ptr[slot]);
      ptr[slot] = nullptr;
      cap[slot] = 0;
      if (hipMalloc(&ptr[slot], bytes) != hipSuccess) return nullptr;
      cap[slot] = bytes;
    }
    return (T*)ptr[slot];
  }
  // pinned host words for the one readback of a build: [0] pair total, [1..4] flags
  long long* host = nullptr;
  long long* host_words() {
    if (!host && hipHostMalloc((void**)&host, 8 * sizeof(long long), hipHostMallocDefault) != hipSuccess)
      host = nullptr;
    return host;
  }
  ~NbrWork();
  PlanArgs pa;
  int row_cap = 0;      // capacity of the staged rows when the workgroup-per-bin path filled them
};

NbrWork::~NbrWork() {
  for (int k = 0; k < 20; ++k)
    if (ptr[k]) (void)hipFree(ptr[k]);
  if (host) (void)hipHostFree(host);
}

NbrWork* nbr_work_create() { return new NbrWork(); }
void nbr_work_destroy(NbrWork* w) { delete w; }

enum Slot { S_FRAC, S_BIN, S_IMG, S_BINCNT, S_BINSTART, S_BINFILL, S_BINATOMS, S_COUNTS, S_BSUM,
            S_TOTAL, S_KEY, S_SKEY, S_ROWID, S_FLAG, S_ROWS, S_ROWS2, S_BINPOS, S_BINIMG, S_NSLOTS };
static_assert(S_NSLOTS <= 20, "workspace slots");

static void inv3(const double* H, double* I, double* det) {
  const double a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7],
               k = H[8];
  const double A = e * k - f * h, B = -(d * k - f * g), C = d * h - e * g;
  *det = a * A + b * B + c * C;
  const double id = 1.0 / *det;
  I[0] = A * id; I[1] = -(b * k - c * h) * id; I[2] = (b * f - c * e) * id;
  I[3] = B * id; I[4] = (a * k - c * g) * id;  I[5] = -(a * f - c * d) * id;
  I[6] = C * id; I[7] = -(a * h - b * g) * id; I[8] = (a * e - b * d) * id;
}

void nbr_plan(const double* H, double rcut, NbrPlan* plan, int* status) {
  double det;
  inv3(H, plan->Hinv, &det);
  *status = 0;
  if (!(fabs(det) > 1e-300) || !isfinite(det)) {
    *status = MTP_ERR_CELL;
    return;
  }
  double width[3];
  for (int k = 0; k < 3; ++k) {
    // b_k = column k of H^-1 (rows of H^-T); perpendicular width 1/|b_k|
    const double bx = plan->Hinv[k], by = plan->Hinv[3 + k], bz = plan->Hinv[6 + k];
    const double bn = sqrt(bx * bx + by * by + bz * bz);
    plan->reach[k] = rcut * bn;
    width[k] = 1.0 / bn;
  }
  const double need = rcut * (1.0 + 1e-9) + 1e-12;
  plan->cells = true;
  long long nbins = 1;
  for (int k = 0; k < 3; ++k) {
    if (width[k] < need) plan->cells = false;
    plan->nb[k] = std::max(1, (int)floor(width[k] / need));
    plan->nb[k] = std::min(plan->nb[k], 1 << 10);
    nbins *= plan->nb[k];
  }
  if (nbins > (1LL << 24)) plan->cells = false;
}

static void fill_args(PlanArgs& pa, const NbrPlan& plan, const double* H, double rcut) {
  for (int k = 0; k < 9; ++k) {
    pa.H[k] = H[k];
    pa.Hinv[k] = plan.Hinv[k];
  }
  for (int k = 0; k < 3; ++k) {
    pa.reach[k] = plan.reach[k];
    pa.nb[k] = plan.nb[k];
  }
  pa.rc2 = rcut * rcut;
}

static int scan_counts(NbrWork* w, const int* counts, int n, int* off, long long* total_host,
                       hipStream_t s) {
  const int nb = (n + kScanBlock - 1) / kScanBlock;
  long long* bsum = w->get<long long>(S_BSUM, nb + 1);
  long long* tot = w->get<long long>(S_TOTAL, 1);
  if (!bsum || !tot) return MTP_ERR_OOM;
  if (n > 0) {
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kNT), 0, s, counts, n, off, bsum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanTop), 0, s, bsum, nb, tot);
    hipLaunchKernelGGL(k_scan_add, dim3((n + kNT - 1) / kNT), dim3(kNT), 0, s, off, n, bsum, tot, 1);
  } else {
    (void)hipMemsetAsync(off, 0, sizeof(int), s);
    (void)hipMemsetAsync(tot, 0, sizeof(long long), s);
  }
  if (total_host) {
    if (hipMemcpyAsync(total_host, tot, sizeof(long long), hipMemcpyDeviceToHost, s) != hipSuccess)
      return MTP_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MTP_ERR_HIP;
  }
  return 0;
}

// One readback per pass: the pair total written by scan_counts and the four flags, through
// pinned host words, then a single stream synchronization.
static int read_back(NbrWork* w, const int* flag, long long* total, int* flags, hipStream_t s) {
  long long* h = w->host_words();
  const long long* tot = w->get<long long>(S_TOTAL, 1);
  if (!h || !tot) return MTP_ERR_OOM;
  if (hipMemcpyAsync(h, tot, sizeof(long long), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(h + 1, flag, 4 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
    return MTP_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return MTP_ERR_HIP;
  *total = h[0];
  const int* f = (const int*)(h + 1);
  for (int k = 0; k < 4; ++k) flags[k] = f[k];
  return 0;
}

// Brick extent (bins per axis) for the staged path: the largest interior whose brick plus halo
// holds on average at most two thirds of the staged capacity, within the halo and interior
// table sizes; false when even a single bin's neighbourhood is too dense.  Also the filter
// margin: binary32 coordinates relative to the halo corner are bounded by the halo's extent
// E = sum_k (bx_k + 2) / nb_k |H_k|, each carries a rounding error below 2^-24 E, so
// |d2_32 - d2| < 2^-24 (7 r E + 3 r^2) for distances r near the cutoff; the margin is four times
// that.
// Brick shape: the least estimated time per centre atom.  A workgroup stages its halo (about
// kStageWeight of a centre pass per staged atom and thread) and then runs ceil(centres /
// kBrickThreads) passes of its lanes over the centres, each pass costing the same whatever the
// number of lanes left busy; so bricks whose centres fit the lanes (with two standard deviations
// to spare) avoid a nearly empty second pass (at 8.2 atoms per bin: 3x3x3 bins, 221 centres,
// instead of 3x3x4, 295).
constexpr double kStageWeight = 0.0143;
static bool brick_shape(const int* nb, double per_bin, const double* H, double rcut, BrickArgs* ba) {
  double best = 0.0;
  for (int x = 1; x <= 8; ++x)
    for (int y = 1; y <= 8; ++y)
      for (int z = 1; z <= 8; ++z) {
        if (x > nb[0] || y > nb[1] || z > nb[2]) continue;
        const int halo = (x + 2) * (y + 2) * (z + 2), inner = x * y * z;
        if (halo > kMaxHalo || inner > kMaxInner) continue;
        if (halo * per_bin > (2.0 / 3.0) * kBrickMaxC) continue;
        const double centres = std::max(inner * per_bin, 1e-9);
        // passes for a brick two standard deviations above the mean count
        const double passes = std::max(1.0, std::ceil((centres + 2.0 * std::sqrt(centres)) / kBrickThreads));
        const double cost = (kStageWeight * halo * per_bin / kBrickThreads + passes) / centres;
        // the cheapest per centre, then the more compact shape among equal costs
        const double score = 1.0 / cost - 1e-9 * halo;
        if (score > best) {
          best = score;
          ba->bx[0] = x;
          ba->bx[1] = y;
          ba->bx[2] = z;
        }
      }
  if (best <= 0.0) return false;
  double ext = 0.0;
  for (int k = 0; k < 3; ++k) {
    ba->nbk[k] = (nb[k] + ba->bx[k] - 1) / ba->bx[k];
    const double len = sqrt(H[3 * k] * H[3 * k] + H[3 * k + 1] * H[3 * k + 1] + H[3 * k + 2] * H[3 * k + 2]);
    ext += (double)(ba->bx[k] + 2) / nb[k] * len;
  }
  ba->margin = 4.0 * ldexp(7.0 * rcut * ext + 3.0 * rcut * rcut, -24);
  return true;
}

int nbr_count(const NbrPlan& plan, const double* pos, const int* species, int nsp, int n,
              const double* H, double rcut, NbrWork* w, int* off, long long* total, int* flags,
              hipStream_t s) {
  PlanArgs& pa = w->pa;
  fill_args(pa, plan, H, rcut);
  int* counts = w->get<int>(S_COUNTS, n);
  int* flag = w->get<int>(S_FLAG, 4);
  if (!counts || !flag) return MTP_ERR_OOM;
  (void)hipMemsetAsync(flag, 0, 4 * sizeof(int), s);
  const int gb = (n + kNT - 1) / kNT;
  if (plan.cells) {
    const int nbins = plan.nb[0] * plan.nb[1] * plan.nb[2];
    int* bin = w->get<int>(S_BIN, n);
    int* img = w->get<int>(S_IMG, 3L * n);
    int* bincnt = w->get<int>(S_BINCNT, nbins);
    int* binstart = w->get<int>(S_BINSTART, nbins + 1);
    int* binfill = w->get<int>(S_BINFILL, nbins);
    int* binatoms = w->get<int>(S_BINATOMS, n);
    if (!bin || !img || !bincnt || !binstart || !binfill || !binatoms) return MTP_ERR_OOM;
    (void)hipMemsetAsync(bincnt, 0, sizeof(int) * nbins, s);
    (void)hipMemsetAsync(binfill, 0, sizeof(int) * nbins, s);
    if (n > 0) hipLaunchKernelGGL(k_bin, dim3(gb), dim3(kNT), 0, s, pos, species, nsp, n, pa, bin, img, bincnt,
                         flag);
    int rc = scan_counts(w, bincnt, nbins, binstart, nullptr, s);
    if (rc) return rc;
    // staged path: bricks of bins sized from the density so that a brick and its halo hold
    // about two thirds of the staged capacity; rows of 64 or 128 keys
    w->row_cap = 0;
    BrickArgs ba{};
    int cap = 0;
    if (n > 0) {
      const double vol = fabs(H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                              H[2] * (H[3] * H[7] - H[4] * H[6]));
      const double expect = 4.18879020478639 * rcut * rcut * rcut * n / vol;
      const double need = 1.25 * expect + 16;
      cap = need <= 64 ? 64 : (need <= 128 ? 128 : 0);
      const double per_bin = (double)n / nbins;
      // sorting by partner index needs every partner once per row (three bins per axis) and
      // partner indices below 2^26 (the sort key)
      if (plan.nb[0] < 3 || plan.nb[1] < 3 || plan.nb[2] < 3 || n >= (1 << 26)) cap = 0;
      if (cap && !brick_shape(plan.nb, per_bin, H, rcut, &ba)) cap = 0;
    }
    double* binpos = cap ? w->get<double>(S_BINPOS, 3L * n) : nullptr;
    int* binimg = cap ? w->get<int>(S_BINIMG, n) : nullptr;
    int* rows_j = cap ? w->get<int>(S_ROWS, (size_t)n * cap) : nullptr;
    int* rows_s = cap ? w->get<int>(S_ROWS2, (size_t)n * cap) : nullptr;
    if (cap && (!binpos || !binimg || !rows_j || !rows_s)) return MTP_ERR_OOM;
    if (n > 0)
      hipLaunchKernelGGL(k_bin_scatter, dim3(gb), dim3(kNT), 0, s, n, bin, binstart, binfill, binatoms, pos, img,
                         binpos, binimg);
    if (cap) {
      const int nbricks = ba.nbk[0] * ba.nbk[1] * ba.nbk[2];
      hipLaunchKernelGGL((k_brick_rows<kBrickMaxC, 64>), dim3(nbricks), dim3(kBrickThreads), 0, s, pa, ba, binstart,
                         binatoms, binpos, binimg, pos, cap, rows_j, rows_s, counts, flag);
      w->row_cap = cap;
    } else if (n > 0) {
      hipLaunchKernelGGL(k_cell_count, dim3(gb), dim3(kNT), 0, s, pos, n, pa, bin, img, binstart, binatoms,
                         counts);
    }
  } else {
    double* sfrac = w->get<double>(S_FRAC, 3L * n);
    if (!sfrac) return MTP_ERR_OOM;
    if (n > 0) {
      hipLaunchKernelGGL(k_frac, dim3(gb), dim3(kNT), 0, s, pos, species, nsp, n, pa, sfrac, flag);
      hipLaunchKernelGGL(k_image_count, dim3(gb), dim3(kNT), 0, s, pos, sfrac, n, pa, counts, flag);
    }
  }
  int rc = scan_counts(w, counts, n, off, nullptr, s);
  if (rc) return rc;
  rc = read_back(w, flag, total, flags, s);
  if (rc) return rc;
  if (w->row_cap > 0 && flags[3]) {
    // a neighbourhood exceeded the staged capacities: count again without staging
    w->row_cap = 0;
    (void)hipMemsetAsync(flag + 3, 0, sizeof(int), s);
    hipLaunchKernelGGL(k_cell_count, dim3(gb), dim3(kNT), 0, s, pos, n, pa, w->get<int>(S_BIN, n),
                       w->get<int>(S_IMG, 3L * n), w->get<int>(S_BINSTART, 1), w->get<int>(S_BINATOMS, n),
                       counts);
    rc = scan_counts(w, counts, n, off, nullptr, s);
    if (rc) return rc;
    rc = read_back(w, flag, total, flags, s);
    if (rc) return rc;
  }
  flags[3] = 0;
  return 0;
}

int nbr_fill(const NbrPlan& plan, const double* pos, int n, const double* H, double rcut,
             NbrWork* w, const int* off, int* nj, int* shift, int* rev, long long total,
             hipStream_t s) {
  PlanArgs& pa = w->pa;
  fill_args(pa, plan, H, rcut);
  const int gb = (n + kNT - 1) / kNT;
  const int gp = (int)((total + kNT - 1) / kNT);
  long long* skey = w->get<long long>(S_SKEY, total);
  int* rowid = w->get<int>(S_ROWID, total);
  if (!skey || !rowid) return MTP_ERR_OOM;
  if (plan.cells && w->row_cap > 0) {
    const int* rows_j = w->get<int>(S_ROWS, 1);
    const int* rows_s = w->get<int>(S_ROWS2, 1);
    int* counts = w->get<int>(S_COUNTS, n);
    if (n > 0) {
      if (w->row_cap == 64)
        hipLaunchKernelGGL((k_rows_copy<32, 1, 64>), dim3((n + 7) / 8), dim3(kCsrThreads), 0, s, n, rows_j, rows_s,
                           counts, off, nj, shift, rev);
      else
        hipLaunchKernelGGL((k_rows_copy<64, 1, 128>), dim3((n + 3) / 4), dim3(kCsrThreads), 0, s, n, rows_j, rows_s,
                           counts, off, nj, shift, rev);
    }
    if (hipGetLastError() != hipSuccess) return MTP_ERR_HIP;
    return 0;
  }
  if (plan.cells) {
    long long* key = w->get<long long>(S_KEY, total);
    if (!key) return MTP_ERR_OOM;
    int* bin = w->get<int>(S_BIN, n);
    int* img = w->get<int>(S_IMG, 3L * n);
    int* binstart = w->get<int>(S_BINSTART, 1);
    int* binatoms = w->get<int>(S_BINATOMS, n);
    if (n > 0) {
      hipLaunchKernelGGL(k_cell_fill, dim3(gb), dim3(kNT), 0, s, pos, n, pa, bin, img, binstart,
                         binatoms, off, key, rowid);
      if (total > 0)
        hipLaunchKernelGGL(k_row_sort, dim3(gp), dim3(kNT), 0, s, total, off, rowid, key, skey, nj,
                           shift);
    }
  } else {
    double* sfrac = w->get<double>(S_FRAC, 3L * n);
    if (n > 0) {
      hipLaunchKernelGGL(k_image_fill, dim3(gb), dim3(kNT), 0, s, pos, sfrac, n, pa, off, nj, shift,
                         skey);
      if (rev) hipLaunchKernelGGL(k_rowid, dim3(gb), dim3(kNT), 0, s, n, off, rowid);
    }
  }
  if (rev && total > 0)
    hipLaunchKernelGGL(k_rev, dim3(gp), dim3(kNT), 0, s, total, off, rowid, skey, rev);
  if (hipGetLastError() != hipSuccess) return MTP_ERR_HIP;
  return 0;
}

int nbr_batch_build(const double* pos, const int* species, int nsp, int n, const int* cfg,
                    const int* atom_off, const double* cells, const double* cinv, const double* reach,
                    double rcut, NbrWork* w, int* off, int** nj, int** shift, int** rev,
                    long long* total, int* flags, int* (*alloc)(void* ctx, int slot, long long n),
                    void* ctx, hipStream_t s) {
  int* counts = w->get<int>(S_COUNTS, n);
  int* flag = w->get<int>(S_FLAG, 4);
  double* sfrac = w->get<double>(S_FRAC, 3L * n);
  if (!counts || !flag || !sfrac) return MTP_ERR_OOM;
  (void)hipMemsetAsync(flag, 0, 4 * sizeof(int), s);
  const double rc2 = rcut * rcut;
  const int gb = (n + kNT - 1) / kNT;
  if (n > 0) {
    hipLaunchKernelGGL(k_batch_frac, dim3(gb), dim3(kNT), 0, s, pos, species, nsp, cfg, cinv, n, sfrac, flag);
    hipLaunchKernelGGL(k_batch_count, dim3(gb), dim3(kNT), 0, s, pos, sfrac, cfg, atom_off, cells, reach,
                       rc2, n, counts, flag);
  }
  int rc = scan_counts(w, counts, n, off, total, s);
  if (rc) return rc;
  if (hipMemcpyAsync(flags, flag, 4 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return MTP_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return MTP_ERR_HIP;
  if (flags[0] || flags[1] || flags[2]) return 0;
  *nj = alloc(ctx, 0, *total);
  *shift = alloc(ctx, 1, *total);
  *rev = alloc(ctx, 2, *total);
  long long* skey = w->get<long long>(S_SKEY, *total);
  int* rowid = w->get<int>(S_ROWID, *total);
  if (!*nj || !*shift || !*rev || !skey || !rowid) return MTP_ERR_OOM;
  const int gp = (int)((*total + kNT - 1) / kNT);
  if (n > 0) {
    hipLaunchKernelGGL(k_batch_fill, dim3(gb), dim3(kNT), 0, s, pos, sfrac, cfg, atom_off, cells, reach,
                       rc2, n, off, *nj, *shift, skey);
    hipLaunchKernelGGL(k_rowid, dim3(gb), dim3(kNT), 0, s, n, off, rowid);
  }
  if (*total > 0) hipLaunchKernelGGL(k_rev, dim3(gp), dim3(kNT), 0, s, *total, off, rowid, skey, *rev);
  if (hipGetLastError() != hipSuccess) return MTP_ERR_HIP;
  return 0;
}

}  // namespace mtp
