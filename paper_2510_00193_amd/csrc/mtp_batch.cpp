// Batched evaluation of many small periodic configurations (training sets).
//
// mtp_batch_create builds the neighbour lists of every configuration once (they are fixed
// for a training set) and reserves all workspace.  mtp_batch_run then enqueues a fixed
// sequence of kernels that covers every configuration in one launch per kernel type:
// forward energies/forces/virials, the loss cotangents on the device, and the parameter
// adjoint.  It allocates nothing and never synchronizes, so it is captured once into a
// hipGraph and replayed (coefficients are updated in place with mtp_set_params).
// mtp_batch_tune times the atom-to-lane schedules and keeps the fastest.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "mtp.h"
#include "mtp_api_internal.h"
#include "mtp_internal.h"

using namespace mtp;

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return mtp_fail(MTP_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_));       \
  } while (0)

struct mtp_batch {
  mtp_model* m = nullptr;
  int ncfg = 0, n = 0;
  long long npairs = 0;
  const double* pos = nullptr;
  const int* species = nullptr;
  DevBuf atom_off, cfg, cells, cinv, reach, off, nj, shift, rev, perm;
  DevBuf plink, pfirst;            // per-species pair chains (fixed with the lists)
  std::vector<int> h_off;          // host copy of the CSR offsets (neighbour counts)
  // workspace
  DevBuf eatom, watom, g, fown, forces, energy, virial, mom, cbar, mbar, mdot, cbard, mbard, xout, dxi_part,
      cpart, wpart, ebar_cfg, fbar, parts, zeros, rsum;
  DevBuf queue;                    // tile counters of the persistent pair-kernel launches
  int pgrid = 0;                   // workgroups of a persistent launch
  // schedule
  int sorted = 0, chunk = 0, persistent = 0;
  // graph
  hipStream_t gs = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> key;
  ~mtp_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (gs) (void)hipStreamDestroy(gs);
  }
};

static int* batch_alloc(void* ctx, int slot, long long count) {
  mtp_batch* b = (mtp_batch*)ctx;
  DevBuf* buf = slot == 0 ? &b->nj : slot == 1 ? &b->shift : &b->rev;
  if (buf->reserve((size_t)std::max<long long>(count, 1) * sizeof(int))) return nullptr;
  return (int*)buf->p;
}

static void inv3(const double* H, double* I, double* det) {
  const double a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7], k = H[8];
  const double A = e * k - f * h, B = -(d * k - f * g), C = d * h - e * g;
  *det = a * A + b * B + c * C;
  const double id = 1.0 / *det;
  I[0] = A * id; I[1] = -(b * k - c * h) * id; I[2] = (b * f - c * e) * id;
  I[3] = B * id; I[4] = (a * k - c * g) * id;  I[5] = -(a * f - c * d) * id;
  I[6] = C * id; I[7] = -(a * h - b * g) * id; I[8] = (a * e - b * d) * id;
}

static long chunk_of(const mtp_batch* b) {
  return std::max(1, std::min(std::min(b->chunk > 0 ? b->chunk : b->n, b->n), kMaxChunk));
}

// Reserve every buffer the run needs for the current schedule (never called during capture).
static int reserve_run(mtp_batch* b) {
  const LevelOps& L = b->m->ops;
  const long n = b->n, ld = chunk_of(b);
  const int nchunks = (int)((n + ld - 1) / ld);
  long nblk = 0;
  for (long i0 = 0; i0 < n; i0 += ld) nblk += (std::min(ld, n - i0) + kLaneBlockHost - 1) / kLaneBlockHost;
  const long K = b->m->nrad;
  int rc;
  if ((rc = b->eatom.reserve(n * 8)) || (rc = b->watom.reserve(6 * n * 8)) ||
      (rc = b->g.reserve(std::max<long long>(b->npairs, 1) * 24)) || (rc = b->forces.reserve(3 * n * 8)) ||
      (rc = b->fown.reserve(3 * n * 8)) ||
      (rc = b->energy.reserve(b->ncfg * 8)) || (rc = b->virial.reserve(6 * b->ncfg * 8)) ||
      (rc = b->mom.reserve(L.nmom * ld * 8)) || (rc = b->cbar.reserve(L.ncomp * ld * 8)) ||
      (rc = b->mbar.reserve(L.nmom * ld * 8)) || (rc = b->mdot.reserve(L.nmom * ld * 8)) ||
      (rc = b->cbard.reserve(L.ncomp * ld * 8)) || (rc = b->mbard.reserve(L.nmom * ld * 8)) ||
      (rc = b->xout.reserve(L.nalpha * ld * 8)) || (rc = b->dxi_part.reserve(L.nalpha * nchunks * 8)) ||
      (rc = b->cpart.reserve(nblk * L.adj.nagroup * K * 8)) || (rc = b->wpart.reserve(nblk * 6 * 8)) ||
      (rc = b->ebar_cfg.reserve(b->ncfg * 8)) || (rc = b->fbar.reserve(3 * n * 8)) ||
      (rc = b->parts.reserve((b->ncfg + n) * 8)) ||
      (rc = b->rsum.reserve(std::max<long>(L.nalpha, K) * kRowParts * 8)))
    return rc;
  return MTP_OK;
}

// Pair-kernel launches of one run (the queue counters a persistent schedule needs).
static long pair_launches(const mtp_batch* b) {
  const LevelOps& L = b->m->ops;
  const long ld = chunk_of(b);
  const long nchunks = ((long)b->n + ld - 1) / ld;
  return nchunks * (3L * L.ngroup + L.adj.ntgroup + L.adj.nagroup) + 1;
}

static int set_schedule(mtp_batch* b, int sorted, int chunk, int persistent) {
  b->sorted = sorted ? 1 : 0;
  b->chunk = chunk > 0 ? std::min(chunk, b->n) : b->n;
  b->persistent = persistent ? 1 : 0;
  if (b->persistent) {
    // one workgroup per SIMD: the lane-per-atom pair kernels run one wave per SIMD
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    b->pgrid = 4 * ncu;
    int rc = b->queue.reserve((size_t)pair_launches(b) * sizeof(int));
    if (rc) return rc;
  }
  std::vector<int> perm(b->n);
  std::iota(perm.begin(), perm.end(), 0);
  if (b->sorted) {
    // atoms with similar neighbour counts share a wave: less divergence in the pair loops
    std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) {
      return b->h_off[x + 1] - b->h_off[x] > b->h_off[y + 1] - b->h_off[y];
    });
  }
  int rc;
  if ((rc = b->perm.reserve((size_t)std::max(b->n, 1) * sizeof(int)))) return rc;
  HIP_TRY(hipMemcpy(b->perm.p, perm.data(), b->n * sizeof(int), hipMemcpyHostToDevice));
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  return reserve_run(b);
}

// The kernel sequence of one batch run (no allocation, no synchronization, no memset).
// With cotangents (ebar_in [n_cfg], fbar_in [N][3]) the adjoint runs on them instead of the loss
// cotangents of targets.
static void run_impl(mtp_batch* b, const double* e_target, const double* f_target, const double* ebar_in,
                     const double* fbar_in, double* energy, double* forces, double* virial, double* loss,
                     double* d_linear, double* d_radial, double* d_shift, hipStream_t s) {
  mtp_model* m = b->m;
  const LevelOps& L = m->ops;
  const ChainOps& K = L.chain[2];
  const int n = b->n;
  const long ld = chunk_of(b);
  const long KR = m->nrad;
  SysArgs a{};
  a.pos = b->pos;
  a.species = b->species;
  a.off = (const int*)b->off.p;
  a.nj = (const int*)b->nj.p;
  a.shift = (const int*)b->shift.p;
  a.radial = (const double*)m->radial.p;
  a.cells = (const double*)b->cells.p;
  a.cfg = (const int*)b->cfg.p;
  a.perm = (const int*)b->perm.p;
  a.ebar = nullptr;
  a.plink = b->plink.p ? (const int*)b->plink.p : nullptr;
  a.pfirst = b->pfirst.p ? (const int*)b->pfirst.p : nullptr;
  a.sa = 2.0 / (m->rcut - m->rmin);
  a.sb = -(m->rmin + m->rcut) / (m->rcut - m->rmin);
  a.rcut = m->rcut;
  a.nsp = m->nsp;
  a.nmu = L.nmu;
  a.ncheb = m->ncheb;
  a.queue = nullptr;
  a.pgrid = b->pgrid;
  a.split = 1;
  // persistent schedule: one zeroed tile counter per pair-kernel launch (a kernel, not a memset,
  // so that the sequence can be captured into a graph)
  int* qbase = b->persistent ? (int*)b->queue.p : nullptr;
  int qslot = 0;
  if (qbase) launch_fill_int(qbase, pair_launches(b), 0, s);
  auto q = [&]() { return qbase ? qbase + qslot++ : nullptr; };
  double* ea = (double*)b->eatom.p;
  double* wa = (double*)b->watom.p;
  double* g = (double*)b->g.p;
  double* wpart = (double*)b->wpart.p;
  long blk = 0;
  // ---- forward: energies, pair gradients, per-atom virials
  for (long i0 = 0; i0 < n; i0 += ld) {
    const int cn = (int)std::min(ld, (long)n - i0);
    for (int gi = 0; gi < L.ngroup; ++gi) {
      ProfScope ps(&m->prof, P_MOMENTS, s);
      a.queue = q();
      K.moments(gi, a, (int)i0, cn, b->mom.p, ld, s);
    }
    {
      ProfScope ps(&m->prof, P_PROG_FWD, s);
      K.prog_fwd(b->mom.p, ld, (int)i0, cn, a.perm, b->species, (const double*)m->linear.p,
                 (const double*)m->shift.p, m->nsp, ea, b->cbar.p, nullptr, s);
    }
    for (int gi = 0; gi < L.ngroup; ++gi) {
      ProfScope ps(&m->prof, P_PROG_REV, s);
      K.prog_rev(gi, b->mom.p, ld, cn, b->cbar.p, b->mbar.p, s);
    }
    for (int gi = 0; gi < L.ngroup; ++gi) {
      ProfScope ps(&m->prof, P_BACKWARD, s);
      a.queue = q();
      K.backward(gi, a, (int)i0, cn, b->mbar.p, ld, g, gi > 0, wpart + 6 * blk, wa, (double*)b->fown.p, s);
    }
    blk += (cn + kLaneBlockHost - 1) / kLaneBlockHost;
  }
  double* F = forces ? forces : (double*)b->forces.p;
  double* E = energy ? energy : (double*)b->energy.p;
  {
    ProfScope ps(&m->prof, P_GATHER, s);
    launch_gather_forces(a.off, (const int*)b->rev.p, g, (const double*)b->fown.p, n, b->npairs, F, s);
  }
  {
    ProfScope ps(&m->prof, P_REDUCE, s);
    launch_segsum(ea, 1, (const int*)b->atom_off.p, b->ncfg, 1, E, 1, s);
    launch_segsum(wa, 6, (const int*)b->atom_off.p, b->ncfg, 6, virial ? virial : (double*)b->virial.p, 6, s);
  }
  const bool vjp = ebar_in && fbar_in;
  if (!vjp && (!e_target || !f_target)) return;
  const double* ebar = ebar_in;
  const double* fbar = fbar_in;
  if (!vjp) {
    // ---- loss cotangents on the device
    double* eb = (double*)b->ebar_cfg.p;
    double* fb = (double*)b->fbar.p;
    double* parts = (double*)b->parts.p;
    ProfScope ps(&m->prof, P_REDUCE, s);
    launch_loss(E, e_target, b->ncfg, F, f_target, n, eb, fb, parts, parts + b->ncfg, s);
    if (loss) launch_sum(parts, (long)b->ncfg + n, 1, loss, s);
    ebar = eb;
    fbar = fb;
  }
  // ---- adjoint
  a.ebar = ebar;
  const int nchunks = (int)((n + ld - 1) / ld);
  double* dxp = (double*)b->dxi_part.p;
  double* cpart = (double*)b->cpart.p;
  long part = 0;
  int c = 0;
  for (long i0 = 0; i0 < n; i0 += ld, ++c) {
    const int cn = (int)std::min(ld, (long)n - i0);
    const long cblk = (cn + kLaneBlockHost - 1) / kLaneBlockHost;
    if (ld < n) {  // the forward state of this chunk was overwritten by later chunks
      for (int gi = 0; gi < L.ngroup; ++gi) {
        ProfScope ps(&m->prof, P_MOMENTS, s);
        a.queue = q();
        K.moments(gi, a, (int)i0, cn, b->mom.p, ld, s);
      }
      {
        ProfScope ps(&m->prof, P_PROG_FWD, s);
        K.prog_fwd(b->mom.p, ld, (int)i0, cn, a.perm, b->species, (const double*)m->linear.p,
                   (const double*)m->shift.p, m->nsp, ea, b->cbar.p, nullptr, s);
      }
    }
    for (int gi = 0; ld < n && gi < L.ngroup; ++gi) {
      ProfScope ps(&m->prof, P_PROG_REV, s);
      K.prog_rev(gi, b->mom.p, ld, cn, b->cbar.p, b->mbar.p, s);
    }
    for (int gi = 0; gi < L.adj.ntgroup; ++gi) {
      ProfScope ps(&m->prof, P_TANGENT, s);
      a.queue = q();
      L.adj.tan_moments(gi, a, fbar, (int)i0, cn, (double*)b->mdot.p, ld, s);
    }
    {
      ProfScope ps(&m->prof, P_TANGENT, s);
      L.adj.tan_forward(a, (const double*)b->mom.p, (const double*)b->mdot.p, ld, (int)i0, cn,
                    (const double*)m->linear.p, 0.0, (double*)b->xout.p, (double*)b->cbard.p, s);
    }
    for (int gi = 0; gi < L.adj.nrtpart; ++gi) {
      ProfScope ps(&m->prof, P_TANGENT, s);
      L.adj.tan_reverse[gi]((const double*)b->mom.p, (const double*)b->mdot.p, ld, cn, (const double*)b->cbar.p,
                    (const double*)b->cbard.p, (double*)b->mbard.p, s);
    }
    for (int gi = 0; gi < L.adj.nagroup; ++gi) {
      ProfScope ps(&m->prof, P_ADJ_PAIRS, s);
      a.queue = q();
      L.adj.adj_pairs(gi, a, fbar, (int)i0, cn, (const double*)b->mbar.p, (const double*)b->mbard.p, ld, 0.0,
                  cpart + part * KR, s);
      part += cblk;
    }
    ProfScope ps(&m->prof, P_REDUCE, s);
    launch_rowsum((const double*)b->xout.p, ld, 1, cn, L.nalpha, dxp + c, nchunks, s, (double*)b->rsum.p);
  }
  ProfScope ps(&m->prof, P_REDUCE, s);
  launch_rowsum(dxp, nchunks, 1, nchunks, L.nalpha, d_linear, 1, s);
  launch_rowsum(cpart, 1, KR, part, (int)KR, d_radial, 1, s, (double*)b->rsum.p);
  launch_species_grad_cfg(b->species, (const int*)b->cfg.p, ebar, n, m->nsp, d_shift, (double*)b->rsum.p, s);
}

static int launch_run(mtp_batch* b, const double* e_target, const double* f_target, const double* ebar,
                      const double* fbar, double* energy, double* forces, double* virial, double* loss,
                      double* d_linear, double* d_radial, double* d_shift, int use_graph, hipStream_t s);

extern "C" {

int mtp_batch_create(mtp_model* m, int n_cfg, const int* atom_off, const double* pos, const int* species,
                     const double* cells, mtp_batch** out, void* stream) {
  if (!m || !atom_off || !cells || !out || n_cfg < 1) return mtp_fail(MTP_ERR_ARG, "null argument or n_cfg < 1");
  *out = nullptr;
  if (atom_off[0] != 0) return mtp_fail(MTP_ERR_ARG, "atom_off[0] must be 0");
  for (int c = 0; c < n_cfg; ++c)
    if (atom_off[c + 1] < atom_off[c]) return mtp_fail(MTP_ERR_ARG, "atom_off must be non-decreasing");
  const int n = atom_off[n_cfg];
  if (n > 0 && (!pos || !species)) return mtp_fail(MTP_ERR_ARG, "null positions or species");
  hipStream_t s = (hipStream_t)stream;
  std::vector<double> cinv(9L * n_cfg), reach(3L * n_cfg);
  for (int c = 0; c < n_cfg; ++c) {
    double det;
    for (int k = 0; k < 9; ++k)
      if (!isfinite(cells[9L * c + k])) return mtp_fail(MTP_ERR_CELL, "non-finite cell");
    inv3(cells + 9L * c, &cinv[9L * c], &det);
    if (!(fabs(det) > 1e-300)) return mtp_fail(MTP_ERR_CELL, "singular cell " + std::to_string(c));
    for (int k = 0; k < 3; ++k) {
      const double bx = cinv[9L * c + k], by = cinv[9L * c + 3 + k], bz = cinv[9L * c + 6 + k];
      reach[3L * c + k] = m->rcut * sqrt(bx * bx + by * by + bz * bz);
    }
  }
  std::vector<int> cfg(n);
  for (int c = 0; c < n_cfg; ++c)
    for (int i = atom_off[c]; i < atom_off[c + 1]; ++i) cfg[i] = c;
  mtp_batch* b = new mtp_batch();
  b->m = m;
  b->ncfg = n_cfg;
  b->n = n;
  b->pos = pos;
  b->species = species;
  int rc;
  if ((rc = b->atom_off.reserve((n_cfg + 1) * sizeof(int))) || (rc = b->cfg.reserve(std::max(n, 1) * sizeof(int))) ||
      (rc = b->cells.reserve(9L * n_cfg * 8)) || (rc = b->cinv.reserve(9L * n_cfg * 8)) ||
      (rc = b->reach.reserve(3L * n_cfg * 8)) || (rc = b->off.reserve((n + 1) * sizeof(int)))) {
    delete b;
    return rc;
  }
  if (hipMemcpy(b->atom_off.p, atom_off, (n_cfg + 1) * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->cfg.p, cfg.data(), n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->cells.p, cells, 9L * n_cfg * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->cinv.p, cinv.data(), 9L * n_cfg * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->reach.p, reach.data(), 3L * n_cfg * 8, hipMemcpyHostToDevice) != hipSuccess) {
    delete b;
    return mtp_fail(MTP_ERR_HIP, "copying batch tables failed");
  }
  int* nj = nullptr;
  int* sh = nullptr;
  int* rv = nullptr;
  long long total = 0;
  int flags[4] = {0, 0, 0, 0};
  rc = nbr_batch_build(pos, species, m->nsp, n, (const int*)b->cfg.p, (const int*)b->atom_off.p,
                       (const double*)b->cells.p, (const double*)b->cinv.p, (const double*)b->reach.p, m->rcut,
                       m->nbr, (int*)b->off.p, &nj, &sh, &rv, &total, flags, batch_alloc, b, s);
  if (rc) {
    delete b;
    return mtp_fail(rc, "batched neighbour build failed");
  }
  if (flags[0] || flags[1] || flags[2]) {
    delete b;
    return flags[0] ? mtp_fail(MTP_ERR_NONFINITE, "non-finite position")
                    : flags[1] ? mtp_fail(MTP_ERR_ARG, "species outside [0, n_species)")
                               : mtp_fail(MTP_ERR_CELL, "an image shift does not fit in int8");
  }
  b->npairs = total;
  if (m->nsp > 1 && total > 0) {
    if ((rc = b->plink.reserve((size_t)total * 4)) || (rc = b->pfirst.reserve((size_t)n * m->nsp * 4))) {
      delete b;
      return mtp_fail(rc, "allocating the pair species chains failed");
    }
    launch_pair_links((const int*)b->off.p, nj, species, m->nsp, (int)n, (int*)b->plink.p, (int*)b->pfirst.p, s);
  }
  b->h_off.resize(n + 1);
  if (hipMemcpy(b->h_off.data(), b->off.p, (n + 1) * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
    delete b;
    return mtp_fail(MTP_ERR_HIP, "reading neighbour offsets failed");
  }
  if ((rc = set_schedule(b, 0, 0, 0))) {
    delete b;
    return rc;
  }
  *out = b;
  return MTP_OK;
}

void mtp_batch_destroy(mtp_batch* b) { delete b; }

int mtp_batch_sizes(const mtp_batch* b, int* n_atoms, long long* n_pairs, int* sorted, int* chunk_atoms,
                    int* persistent) {
  if (!b) return mtp_fail(MTP_ERR_ARG, "null batch");
  if (n_atoms) *n_atoms = b->n;
  if (n_pairs) *n_pairs = b->npairs;
  if (sorted) *sorted = b->sorted;
  if (chunk_atoms) *chunk_atoms = (int)chunk_of(b);
  if (persistent) *persistent = b->persistent;
  return MTP_OK;
}

int mtp_batch_neighbors(const mtp_batch* b, const int** off, const int** j, const int** shift, const int** rev) {
  if (!b) return mtp_fail(MTP_ERR_ARG, "null batch");
  if (off) *off = (const int*)b->off.p;
  if (j) *j = (const int*)b->nj.p;
  if (shift) *shift = (const int*)b->shift.p;
  if (rev) *rev = (const int*)b->rev.p;
  return MTP_OK;
}

int mtp_batch_schedule(mtp_batch* b, int sorted, int chunk_atoms, int persistent) {
  if (!b || chunk_atoms < 0) return mtp_fail(MTP_ERR_ARG, "null batch or negative chunk");
  return set_schedule(b, sorted, chunk_atoms, persistent);
}

int mtp_batch_run(mtp_batch* b, const double* e_target, const double* f_target, double* energy, double* forces,
                  double* virial, double* loss, double* d_linear, double* d_radial, double* d_shift, int use_graph,
                  void* stream) {
  if (!b) return mtp_fail(MTP_ERR_ARG, "null batch");
  const bool adj = e_target || f_target;
  if (adj && (!e_target || !f_target || !d_linear || !d_radial || !d_shift))
    return mtp_fail(MTP_ERR_ARG, "the loss gradient needs both targets and all three gradient outputs");
  if (b->n == 0) return mtp_fail(MTP_ERR_ARG, "empty batch");
  return launch_run(b, e_target, f_target, nullptr, nullptr, energy, forces, virial, loss, d_linear, d_radial,
                    d_shift, use_graph, (hipStream_t)stream);
}

int mtp_batch_vjp(mtp_batch* b, const double* ebar, const double* fbar, double* d_linear, double* d_radial,
                  double* d_shift, int use_graph, void* stream) {
  if (!b) return mtp_fail(MTP_ERR_ARG, "null batch");
  if (!ebar || !fbar || !d_linear || !d_radial || !d_shift)
    return mtp_fail(MTP_ERR_ARG, "the product needs both cotangents and all three gradient outputs");
  if (b->n == 0) return mtp_fail(MTP_ERR_ARG, "empty batch");
  return launch_run(b, nullptr, nullptr, ebar, fbar, nullptr, nullptr, nullptr, nullptr, d_linear, d_radial,
                    d_shift, use_graph, (hipStream_t)stream);
}

}  // extern "C"

// Enqueue run_impl directly, or as the replay of a graph captured once per set of pointers.
static int launch_run(mtp_batch* b, const double* e_target, const double* f_target, const double* ebar,
                      const double* fbar, double* energy, double* forces, double* virial, double* loss,
                      double* d_linear, double* d_radial, double* d_shift, int use_graph, hipStream_t s) {
  if (!use_graph) {
    run_impl(b, e_target, f_target, ebar, fbar, energy, forces, virial, loss, d_linear, d_radial, d_shift, s);
    HIP_TRY(hipGetLastError());
    return MTP_OK;
  }
  std::vector<const void*> key = {e_target, f_target, ebar, fbar, energy, forces, virial, loss, d_linear, d_radial,
                                  d_shift};
  if (!b->gs) {
    HIP_TRY(hipStreamCreateWithFlags(&b->gs, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
  }
  if (!b->exec || key != b->key) {
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    const bool prof = b->m->prof.on;
    b->m->prof.on = false;  // no event records inside the graph
    HIP_TRY(hipStreamBeginCapture(b->gs, hipStreamCaptureModeThreadLocal));
    run_impl(b, e_target, f_target, ebar, fbar, energy, forces, virial, loss, d_linear, d_radial, d_shift, b->gs);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->gs, &graph);
    b->m->prof.on = prof;
    if (e != hipSuccess) return mtp_fail(MTP_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return mtp_fail(MTP_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    b->key = key;
  }
  HIP_TRY(hipEventRecord(b->ev_in, s));
  HIP_TRY(hipStreamWaitEvent(b->gs, b->ev_in, 0));
  {
    ProfScope ps(&b->m->prof, P_BATCH, b->gs);
    HIP_TRY(hipGraphLaunch(b->exec, b->gs));
  }
  HIP_TRY(hipEventRecord(b->ev_out, b->gs));
  HIP_TRY(hipStreamWaitEvent(s, b->ev_out, 0));
  return MTP_OK;
}

extern "C" {

// Autotuner: time every (order, chunk) schedule on this batch (forward + loss gradient, zero
// targets), keep the fastest; cache_path (text lines "key sorted chunk") makes the pick
// reproducible across processes.  choice (may be NULL) receives {sorted, chunk}.
int mtp_batch_tune(mtp_batch* b, const char* cache_path, int* choice, void* stream) {
  if (!b) return mtp_fail(MTP_ERR_ARG, "null batch");
  hipStream_t s = (hipStream_t)stream;
  const mtp_model* m = b->m;
  const int bucket = b->n < 4096 ? 4096 : b->n < 65536 ? 65536 : b->n < 1048576 ? 1048576 : 1 << 30;
  char key[160];
  snprintf(key, sizeof(key), "gfx950-L%d-sp%d-q%d-n%d", m->ops.level, m->nsp, m->ncheb, bucket);
  auto report = [&]() {
    if (choice) {
      choice[0] = b->sorted;
      choice[1] = (int)chunk_of(b);
      choice[2] = b->persistent;
    }
  };
  if (cache_path) {
    FILE* fh = fopen(cache_path, "r");
    if (fh) {
      char line[256];
      while (fgets(line, sizeof(line), fh)) {
        char k[160];
        int so = 0, ch = 0, pe = 0;
        if (sscanf(line, "%159s %d %d %d", k, &so, &ch, &pe) == 4 && strcmp(k, key) == 0) {
          fclose(fh);
          int rc = set_schedule(b, so, ch > 0 ? ch : 0, pe);
          if (!rc) report();
          return rc;
        }
      }
      fclose(fh);
    }
  }
  // schedules: atom order (natural / sorted by neighbour count, longest rows first), chunk of
  // atoms per pass, and static grids or persistent pair kernels pulling tiles from a queue
  std::vector<int> chunks = {0, 262144, 65536};
  int best_sorted = 0, best_chunk = 0, best_pers = 0;
  float best_ms = -1.f;
  int rc;
  if ((rc = b->zeros.reserve(std::max<long>(3L * b->n, b->ncfg) * 8))) return rc;
  HIP_TRY(hipMemsetAsync(b->zeros.p, 0, std::max<long>(3L * b->n, b->ncfg) * 8, s));
  DevBuf dl, dr, ds;
  if ((rc = dl.reserve(m->ops.nalpha * 8)) || (rc = dr.reserve(m->nrad * 8)) || (rc = ds.reserve(m->nsp * 8)))
    return rc;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  for (int so = 0; so < 2; ++so) {
    for (int ch : chunks) {
      if (ch > 0 && ch >= b->n) continue;
      for (int pe = 0; pe < 2; ++pe) {
        if ((rc = set_schedule(b, so, ch, pe))) return rc;
        const double* z = (const double*)b->zeros.p;
        run_impl(b, z, z, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, (double*)dl.p, (double*)dr.p,
                 (double*)ds.p, s);
        HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < 2; ++r)
          run_impl(b, z, z, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, (double*)dl.p, (double*)dr.p,
                   (double*)ds.p, s);
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (best_ms < 0.f || ms < best_ms) {
          best_ms = ms;
          best_sorted = so;
          best_chunk = ch;
          best_pers = pe;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if ((rc = set_schedule(b, best_sorted, best_chunk, best_pers))) return rc;
  if (cache_path) {
    FILE* fh = fopen(cache_path, "a");
    if (fh) {
      fprintf(fh, "%s %d %d %d\n", key, best_sorted, best_chunk, best_pers);
      fclose(fh);
    }
  }
  report();
  return MTP_OK;
}

}  // extern "C"
