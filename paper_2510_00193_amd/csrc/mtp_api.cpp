// C ABI of the MTP library: argument checking, workspace, and the launch sequence of the
// hot path (neighbour list -> moments -> contractions -> adjoint -> pair gradients ->
// force gather and fixed-order sums).  All device work goes to the caller's stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <string>
#include <vector>

#include "mtp.h"
#include "mtp_internal.h"
#include "mtp_api_internal.h"

namespace mtp {
#define MTP_LEVEL(N) LevelOps level_ops_##N();
#include "gen/levels.inc"
#undef MTP_LEVEL

static bool find_level(int level, LevelOps* out) {
  switch (level) {
#define MTP_LEVEL(N) \
  case N:            \
    *out = level_ops_##N(); \
    return true;
#include "gen/levels.inc"
#undef MTP_LEVEL
    default:
      return false;
  }
}
}  // namespace mtp

using namespace mtp;

static thread_local std::string g_err;

int mtp_fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) return mtp_fail(MTP_ERR_HIP, std::string(#expr ": ") +   \
                                                           hipGetErrorString(e_)); \
  } while (0)

DevBuf::~DevBuf() {
  if (p) (void)hipFree(p);
}

int DevBuf::reserve(size_t n) {
  if (bytes >= n) return MTP_OK;
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
  if (n == 0) return MTP_OK;
  if (hipMalloc(&p, n) != hipSuccess) {
    (void)hipGetLastError();
    return mtp_fail(MTP_ERR_OOM, "device allocation of " + std::to_string(n) + " bytes failed");
  }
  bytes = n;
  return MTP_OK;
}

hipEvent_t Profiler::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

Profiler::~Profiler() {
  for (auto& r : pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

ProfScope::ProfScope(Profiler* p_, int cls_, hipStream_t s_) : p(p_), cls(cls_), s(s_) {
  if (p && p->on) {
    a = p->take();
    if (a) (void)hipEventRecord(a, s);
  }
}

ProfScope::~ProfScope() {
  if (!a) return;
  hipEvent_t b = p->take();
  if (!b) return;
  (void)hipEventRecord(b, s);
  p->pending.push_back({cls, a, b});
}

static const char* kProfNames[P_NCLASS] = {"neighbor_build", "moments", "program_forward",
                                           "program_reverse", "pair_backward", "force_gather",
                                           "reductions", "grade_gemm", "tangent", "adjoint_pairs",
                                           "batch", "program"};

extern "C" {

const char* mtp_last_error(void) { return g_err.c_str(); }

int mtp_level_info(int level, int* info, int n_info) {
  LevelOps ops;
  if (!find_level(level, &ops))
    return mtp_fail(MTP_ERR_LEVEL, "level " + std::to_string(level) + " is not compiled");
  if (!info || n_info < 0) return mtp_fail(MTP_ERR_ARG, "null info");
  const int vals[7] = {ops.nalpha, ops.nmu, ops.nmom, ops.ncomp, ops.triples, ops.maxnu, ops.ngroup};
  for (int k = 0; k < n_info && k < 7; ++k) info[k] = vals[k];
  return MTP_OK;
}

int mtp_profile(mtp_model* m, int enable) {
  if (!m) return mtp_fail(MTP_ERR_ARG, "null model");
  m->prof.on = enable != 0;
  return MTP_OK;
}

int mtp_profile_reset(mtp_model* m) {
  if (!m) return mtp_fail(MTP_ERR_ARG, "null model");
  for (auto& r : m->prof.pending) {
    (void)hipEventSynchronize(r.b);
    m->prof.pool.push_back(r.a);
    m->prof.pool.push_back(r.b);
  }
  m->prof.pending.clear();
  for (int k = 0; k < P_NCLASS; ++k) {
    m->prof.ms[k] = 0.0;
    m->prof.launches[k] = 0;
  }
  return MTP_OK;
}

int mtp_profile_read(mtp_model* m, int k, const char** name, double* total_ms, long long* launches) {
  if (!m) return mtp_fail(MTP_ERR_ARG, "null model");
  if (k < 0 || k >= P_NCLASS) return mtp_fail(MTP_ERR_ARG, "no such kernel class");
  for (auto& r : m->prof.pending) {
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    m->prof.ms[r.cls] += ms;
    m->prof.launches[r.cls] += 1;
    m->prof.pool.push_back(r.a);
    m->prof.pool.push_back(r.b);
  }
  m->prof.pending.clear();
  if (name) *name = kProfNames[k];
  if (total_ms) *total_ms = m->prof.ms[k];
  if (launches) *launches = m->prof.launches[k];
  return MTP_OK;
}

int mtp_levels(int* n, int* levels) {
  if (!n) return mtp_fail(MTP_ERR_ARG, "n is NULL");
  int k = 0;
#define MTP_LEVEL(N) \
  if (levels) levels[k] = N; \
  ++k;
#include "gen/levels.inc"
#undef MTP_LEVEL
  *n = k;
  return MTP_OK;
}

int mtp_create(const mtp_params* p, mtp_model** out) {
  if (!p || !out) return mtp_fail(MTP_ERR_ARG, "null argument");
  *out = nullptr;
  LevelOps ops;
  if (!find_level(p->level, &ops))
    return mtp_fail(MTP_ERR_LEVEL, "level " + std::to_string(p->level) + " is not compiled");
  if (p->n_species < 1 || p->n_species > kMaxSpecies)
    return mtp_fail(MTP_ERR_ARG, "n_species must be in [1, " + std::to_string(kMaxSpecies) + "]");
  if (p->n_cheb < 1 || p->n_cheb > kMaxChebHost)
    return mtp_fail(MTP_ERR_ARG, "n_cheb must be in [1, 16]");
  if (!(p->r_min >= 0.0) || !(p->r_cut > p->r_min) || !isfinite(p->r_cut))
    return mtp_fail(MTP_ERR_ARG, "need 0 <= r_min < r_cut");
  if (!p->radial || !p->linear || !p->shift) return mtp_fail(MTP_ERR_ARG, "null coefficients");
  if (p->precision != MTP_FP64 && p->precision != MTP_FP32_MOMENTS)
    return mtp_fail(MTP_ERR_ARG, "unknown precision");
  if (p->chunk_atoms < 0 || p->chunk_atoms > kMaxChunk) return mtp_fail(MTP_ERR_ARG, "chunk_atoms outside [0, 2^28]");
  if (p->lanes_per_atom != 0 && p->lanes_per_atom != 1 && p->lanes_per_atom != 2 && p->lanes_per_atom != 4 &&
      p->lanes_per_atom != 8)
    return mtp_fail(MTP_ERR_ARG, "lanes_per_atom must be 0, 1, 2, 4 or 8");
  if (p->precision == MTP_FP32_MOMENTS && !ops.chain[1].moments)
    return mtp_fail(MTP_ERR_LEVEL, "the binary32 form is not compiled for level " + std::to_string(p->level));
  const long nrad = (long)p->n_species * p->n_species * ops.nmu * p->n_cheb;
  if (nrad > kMaxRadial) return mtp_fail(MTP_ERR_ARG, "radial table too large");
  mtp_model* m = new mtp_model();
  m->ops = ops;
  m->nsp = p->n_species;
  m->ncheb = p->n_cheb;
  m->rmin = p->r_min;
  m->rcut = p->r_cut;
  m->precision = p->precision;
  m->chunk = p->chunk_atoms > 0 ? p->chunk_atoms : kDefaultChunk;
  m->grade_select = p->grade_select;
  m->grade_break = p->grade_break;
  m->split = p->lanes_per_atom;
  {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&m->ncu, hipDeviceAttributeMultiprocessorCount, dev);
  }
  m->nrad = nrad;
  int rc = MTP_OK;
  if ((rc = m->radial.reserve(nrad * sizeof(double))) || (rc = m->linear.reserve(ops.nalpha * sizeof(double))) ||
      (rc = m->shift.reserve(m->nsp * sizeof(double)))) {
    delete m;
    return rc;
  }
  if (hipMemcpy(m->radial.p, p->radial, nrad * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->linear.p, p->linear, ops.nalpha * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->shift.p, p->shift, m->nsp * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    delete m;
    return mtp_fail(MTP_ERR_HIP, "copying coefficients failed");
  }
  m->nbr = nbr_work_create();
  if ((rc = static_scratch_resolve(&m->static_scratch))) {
    mtp_destroy(m);
    return rc;
  }
  *out = m;
  return MTP_OK;
}

void mtp_destroy(mtp_model* m) {
  if (!m) return;
  nbr_work_destroy(m->nbr);
  delete m;
}

int mtp_sizes(const mtp_model* m, int* n_alpha, int* n_mu, int* n_moments, int* n_components) {
  if (!m) return mtp_fail(MTP_ERR_ARG, "null model");
  if (n_alpha) *n_alpha = m->ops.nalpha;
  if (n_mu) *n_mu = m->ops.nmu;
  if (n_moments) *n_moments = m->ops.nmom;
  if (n_components) *n_components = m->ops.ncomp;
  return MTP_OK;
}

int mtp_set_params(mtp_model* m, const double* radial, const double* linear, const double* shift,
                   int on_device, void* stream) {
  if (!m) return mtp_fail(MTP_ERR_ARG, "null model");
  hipStream_t s = (hipStream_t)stream;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (radial) HIP_TRY(hipMemcpyAsync(m->radial.p, radial, m->nrad * sizeof(double), kind, s));
  if (linear) HIP_TRY(hipMemcpyAsync(m->linear.p, linear, m->ops.nalpha * sizeof(double), kind, s));
  if (shift) HIP_TRY(hipMemcpyAsync(m->shift.p, shift, m->nsp * sizeof(double), kind, s));
  if (!on_device) HIP_TRY(hipStreamSynchronize(s));
  return MTP_OK;
}

}  // extern "C"

int check_system(const mtp_model* m, const mtp_system* sys) {
  if (!m || !sys) return mtp_fail(MTP_ERR_ARG, "null model or system");
  if (sys->n_atoms < 0) return mtp_fail(MTP_ERR_ARG, "n_atoms < 0");
  if (sys->n_atoms > 0 && (!sys->pos || !sys->species))
    return mtp_fail(MTP_ERR_ARG, "null positions or species");
  for (int k = 0; k < 9; ++k)
    if (!isfinite(sys->cell[k])) return mtp_fail(MTP_ERR_CELL, "non-finite cell");
  return MTP_OK;
}

// Build the canonical list into the given buffers (or the model's own when off is NULL).
int build_neighbors(mtp_model* m, const mtp_system* sys, int* off, int* nj, int* shift, int* rev,
                    long long cap, long long* n_pairs, bool own, hipStream_t s) {
  NbrPlan plan;
  int st = 0;
  nbr_plan(sys->cell, m->rcut, &plan, &st);
  if (st) return mtp_fail(MTP_ERR_CELL, "singular cell");
  const int n = sys->n_atoms;
  int rc;
  if (own) {
    if ((rc = m->nl_off.reserve((n + 1) * sizeof(int)))) return rc;
    off = (int*)m->nl_off.p;
  }
  if (!plan.cells && n > kMaxAllPairsAtoms)
    return mtp_fail(MTP_ERR_CELL, "cell thinner than r_cut for a system too large for the all-pairs search");
  ProfScope ps(&m->prof, P_NBR, s);
  long long total = 0;
  int flags[4] = {0, 0, 0, 0};
  rc = nbr_count(plan, sys->pos, sys->species, m->nsp, n, sys->cell, m->rcut, m->nbr, off, &total,
                 flags, s);
  if (rc) return mtp_fail(rc, "neighbour count failed");
  if (flags[0]) return mtp_fail(MTP_ERR_NONFINITE, "non-finite position");
  if (flags[1]) return mtp_fail(MTP_ERR_ARG, "species outside [0, n_species)");
  if (flags[2]) return mtp_fail(MTP_ERR_CELL, "an image shift does not fit in int8");
  if (total >= (1LL << 31)) return mtp_fail(MTP_ERR_CAPACITY, "more than 2^31 - 1 pairs");
  *n_pairs = total;
  if (own) {
    if ((rc = m->nl_j.reserve(total * sizeof(int))) || (rc = m->nl_shift.reserve(total * sizeof(int))) ||
        (rc = m->nl_rev.reserve(total * sizeof(int))))
      return rc;
    nj = (int*)m->nl_j.p;
    shift = (int*)m->nl_shift.p;
    rev = (int*)m->nl_rev.p;
  } else if (total > cap) {
    return mtp_fail(MTP_ERR_CAPACITY, "pair capacity " + std::to_string(cap) + " < " +
                                          std::to_string(total));
  }
  rc = nbr_fill(plan, sys->pos, n, sys->cell, m->rcut, m->nbr, off, nj, shift, rev, total, s);
  if (rc) return mtp_fail(rc, "neighbour fill failed");
  return MTP_OK;
}

extern "C" int mtp_neighbors(mtp_model* m, const mtp_system* sys, int* off, int* j, int* shift,
                             int* rev, long long cap, long long* n_pairs, void* stream) {
  int rc = check_system(m, sys);
  if (rc) return rc;
  if (!off || !n_pairs || (cap > 0 && (!j || !shift)) || cap < 0)
    return mtp_fail(MTP_ERR_ARG, "null output buffer or negative capacity");
  return build_neighbors(m, sys, off, j, shift, rev, cap, n_pairs, false, (hipStream_t)stream);
}

// Resolve the list to use: the caller's, or a freshly built internal one.  flag: a device word
// for the check of a caller's list, or NULL to use the model's own.
int resolve_nlist(mtp_model* m, const mtp_system* sys, const mtp_nlist* nl, mtp_nlist* out,
                  hipStream_t s, int* flag) {
  if (nl) {
    if (!nl->off || (nl->n_pairs > 0 && (!nl->j || !nl->shift || !nl->rev)) || nl->n_pairs < 0)
      return mtp_fail(MTP_ERR_ARG, "incomplete neighbour list");
    if (nl->n_pairs >= (1LL << 31)) return mtp_fail(MTP_ERR_ARG, "more than 2^31 - 1 pairs");
    if (!nl->checked) {
      if (sys->n_atoms == 0 && nl->n_pairs != 0) return mtp_fail(MTP_ERR_ARG, "pairs in an empty system");
      if (sys->n_atoms > 0) {
        if (!flag) {
          int rc = m->flag.reserve(sizeof(int));
          if (rc) return rc;
          flag = (int*)m->flag.p;
        }
        int bad = 0;
        launch_fill_int(flag, 1, 0, s);
        launch_check_nlist(nl->off, nl->j, nl->shift, nl->rev, sys->species, sys->n_atoms, nl->n_pairs, m->nsp,
                           flag, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (bad)
          return mtp_fail(MTP_ERR_ARG, "inconsistent neighbour list (offsets, partner index, mirror or shift) "
                                       "or species outside [0, n_species)");
      }
    }
    *out = *nl;
    return MTP_OK;
  }
  long long total = 0;
  int rc = build_neighbors(m, sys, nullptr, nullptr, nullptr, nullptr, 0, &total, true, s);
  if (rc) return rc;
  out->off = (const int*)m->nl_off.p;
  out->j = (const int*)m->nl_j.p;
  out->shift = (const int*)m->nl_shift.p;
  out->rev = (const int*)m->nl_rev.p;
  out->n_pairs = total;
  out->checked = 1;
  return MTP_OK;
}

SysArgs make_sys_args(const mtp_model* m, const mtp_system* sys, const mtp_nlist& nl) {
  SysArgs a;
  a.pos = sys->pos;
  a.species = sys->species;
  a.off = nl.off;
  a.nj = nl.j;
  a.shift = nl.shift;
  a.radial = (const double*)m->radial.p;
  for (int k = 0; k < 9; ++k) a.H[k] = sys->cell[k];
  a.cells = nullptr;
  a.cfg = nullptr;
  a.perm = nullptr;
  a.ebar = nullptr;
  a.plink = nullptr;
  a.pfirst = nullptr;
  a.sa = 2.0 / (m->rcut - m->rmin);
  a.sb = -(m->rmin + m->rcut) / (m->rcut - m->rmin);
  a.rcut = m->rcut;
  a.nsp = m->nsp;
  a.nmu = m->ops.nmu;
  a.ncheb = m->ncheb;
  a.queue = nullptr;
  a.pgrid = 0;
  a.split = pair_split(m, sys->n_atoms);
  return a;
}

// Small systems leave SIMDs idle with one lane per atom (a wave per 64 atoms, one wave per
// SIMD at these register counts): the lanes per atom double while the waves still fit on the
// SIMDs (4 per compute unit) at once.
int pair_split(const mtp_model* m, int n) {
  if (m->precision != MTP_FP64) return 1;
  if (m->split > 0) return m->split;
  int k = 1;
  while (k < 8 && (long)n * 2 * k <= (long)kLaneBlockHost * 4 * m->ncu) k *= 2;
  return k;
}

long pair_blocks(int n, int split) { return ((long)n * split + kLaneBlockHost - 1) / kLaneBlockHost; }

long chain_wpart_blocks(int n, int chunk, int split) {
  return pair_blocks(n, split) + (n / std::max(chunk, 1) + 1);
}

int chain_work_reserve(mtp_model* m, int n, long long npairs, bool backward, ChainWork* w) {
  const LevelOps& L = m->ops;
  const int chunk = std::max(1, std::min(m->chunk, std::max(n, 1)));
  int rc;
  if ((rc = m->mom.reserve((size_t)L.nmom * chunk * sizeof(double))) ||
      (rc = m->cbar.reserve((size_t)L.ncomp * chunk * sizeof(double))))
    return rc;
  *w = ChainWork{};
  w->chunk = chunk;
  w->mom = m->mom.p;
  w->cbar = m->cbar.p;
  if (backward) {
    if ((rc = m->mbar.reserve((size_t)L.nmom * chunk * sizeof(double))) ||
        (rc = m->g.reserve((size_t)std::max<long long>(npairs, 1) * 3 * sizeof(double))) ||
        (rc = m->fown.reserve((size_t)std::max(n, 1) * 3 * sizeof(double))) ||
        (rc = m->wpart.reserve((size_t)chain_wpart_blocks(n, chunk, pair_split(m, n)) * 6 * sizeof(double))))
      return rc;
    w->mbar = m->mbar.p;
    w->g = (double*)m->g.p;
    w->fown = (double*)m->fown.p;
    w->wpart = (double*)m->wpart.p;
  }
  return MTP_OK;
}

// Forward (moments, contractions, energies) and optionally the adjoint chain down to the
// per-pair gradients g and per-workgroup virial partials, chunk by chunk, in the buffers of w.
int run_energy_chain(mtp_model* m, const mtp_system* sys, const mtp_nlist& nl, double* e_atom,
                     bool backward, double* bvals, hipStream_t s,
                     const std::function<void(int, int)>& after_forward, ChainWork& w) {
  const LevelOps& L = m->ops;
  const ChainOps& K = L.chain[m->precision == MTP_FP32_MOMENTS ? 1 : 0];
  const int n = sys->n_atoms;
  const int chunk = w.chunk;
  const long ld = chunk;
  SysArgs a = make_sys_args(m, sys, nl);
  void* mom = w.mom;
  void* cbar = w.cbar;
  void* mbar = w.mbar;
  long blk = 0;
  for (int i0 = 0; i0 < n; i0 += chunk) {
    const int cn = std::min(chunk, n - i0);
    for (int g = 0; g < L.ngroup; ++g) {
      ProfScope ps(&m->prof, P_MOMENTS, s);
      K.moments(g, a, i0, cn, mom, ld, s);
    }
    if (backward && K.program && !bvals && !after_forward) {
      // energies and moment adjoints in one kernel
      {
        ProfScope ps(&m->prof, P_PROGRAM, s);
        K.program(mom, ld, i0, cn, sys->species, (const double*)m->linear.p, (const double*)m->shift.p, m->nsp,
                  e_atom, mbar, s);
      }
      {
        ProfScope ps(&m->prof, P_BACKWARD, s);
        K.backward(0, a, i0, cn, mbar, ld, w.g, 0, w.wpart + 6 * blk, nullptr, w.fown, s);
      }
      blk += pair_blocks(cn, a.split);
      continue;
    }
    {
      ProfScope ps(&m->prof, P_PROG_FWD, s);
      K.prog_fwd(mom, ld, i0, cn, nullptr, sys->species, (const double*)m->linear.p,
                 (const double*)m->shift.p, m->nsp, e_atom, cbar, bvals, s);
    }
    if (after_forward) after_forward(i0, cn);
    if (backward) {
      for (int g = 0; g < L.ngroup; ++g) {
        ProfScope ps(&m->prof, P_PROG_REV, s);
        K.prog_rev(g, mom, ld, cn, cbar, mbar, s);
      }
      for (int g = 0; g < L.ngroup; ++g) {
        ProfScope ps(&m->prof, P_BACKWARD, s);
        K.backward(g, a, i0, cn, mbar, ld, w.g, g > 0, w.wpart + 6 * blk, nullptr, w.fown, s);
      }
      blk += pair_blocks(cn, a.split);
    }
  }
  w.wblocks = blk;
  HIP_TRY(hipGetLastError());
  return MTP_OK;
}

// Energy reduction, force gather and virial reduction after the chain (part: 7 kSumParts doubles).
int finish_compute(mtp_model* m, const mtp_nlist& nl, int n, const double* ea, const ChainWork& w,
                   double* part, double* energy, double* forces, double* virial, hipStream_t s) {
  if (forces && n > 0) {
    ProfScope ps(&m->prof, P_GATHER, s);
    launch_gather_forces(nl.off, nl.rev, w.g, w.fown, n, nl.n_pairs, forces, s);
  }
  if (!energy && !virial) {
    HIP_TRY(hipGetLastError());
    return MTP_OK;
  }
  ProfScope ps(&m->prof, P_REDUCE, s);
  // small systems: energy and virial in one launch (latency); otherwise both two-level sums
  // share their launches
  const bool small = n > 0 && n <= kSmallSumMax && w.wblocks <= kSmallSumMax;
  if (small) {
    launch_sum_small(ea, n, virial ? w.wpart : nullptr, virial ? w.wblocks : 0, energy, virial, s);
  } else if (n > 0 && energy && virial) {
    launch_sum_parts2(ea, n, 1, 1, energy, w.wpart, w.wblocks, 6, 6, virial, part, s);
  } else {
    if (energy) launch_sum_parts(ea, n, 1, 1, part, energy, s);
    if (virial) {
      if (n > 0)
        launch_sum_parts(w.wpart, w.wblocks, 6, 6, part, virial, s);
      else
        launch_fill(virial, 6, 0.0, s);
    }
  }
  HIP_TRY(hipGetLastError());
  return MTP_OK;
}

extern "C" int mtp_compute(mtp_model* m, const mtp_system* sys, const mtp_nlist* nl,
                           double* energy, double* e_atom, double* forces, double* virial,
                           void* stream) {
  int rc = check_system(m, sys);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int n = sys->n_atoms;
  mtp_nlist use;
  if ((rc = resolve_nlist(m, sys, nl, &use, s))) return rc;
  double* ea = e_atom;
  if (!ea) {
    if ((rc = m->eatom.reserve((size_t)std::max(n, 1) * sizeof(double)))) return rc;
    ea = (double*)m->eatom.p;
  }
  const bool backward = forces || virial;
  ChainWork w;
  if ((rc = chain_work_reserve(m, n, use.n_pairs, backward, &w))) return rc;
  if (n > 0) {
    if ((rc = run_energy_chain(m, sys, use, ea, backward, nullptr, s, nullptr, w))) return rc;
  }
  if ((rc = m->scratch.reserve(7 * kSumParts * sizeof(double)))) return rc;
  return finish_compute(m, use, n, ea, w, (double*)m->scratch.p, energy, forces, virial, s);
}

extern "C" int mtp_grade(mtp_model* m, const mtp_system* sys, const mtp_nlist* nl, const double* ainv,
                         int mode, double* grade, double* grade_max, void* stream) {
  int rc = check_system(m, sys);
  if (rc) return rc;
  if (!ainv || (sys->n_atoms > 0 && !grade) || !grade_max)
    return mtp_fail(MTP_ERR_ARG, "null grade buffers or inverse active-set matrix");
  if (mode != MTP_GRADE_FP64 && mode != MTP_GRADE_FP32SPLIT) return mtp_fail(MTP_ERR_ARG, "unknown grade mode");
  hipStream_t s = (hipStream_t)stream;
  const int n = sys->n_atoms;
  mtp_nlist use;
  if ((rc = resolve_nlist(m, sys, nl, &use, s))) return rc;
  const int na = m->ops.nalpha;
  const long ld = std::max(1, std::min(m->chunk, std::max(n, 1)));
  if ((rc = m->bvals.reserve((size_t)na * ld * sizeof(double))) ||
      (rc = m->eatom.reserve((size_t)std::max(n, 1) * sizeof(double))))
    return rc;
  double* bv = (double*)m->bvals.p;
  if (n > 0) {
    ChainWork w;
    if ((rc = chain_work_reserve(m, n, use.n_pairs, false, &w))) return rc;
    rc = run_energy_chain(m, sys, use, (double*)m->eatom.p, false, bv, s, [&](int i0, int cn) {
      ProfScope ps(&m->prof, P_GRADE, s);
      launch_grade(bv, ld, cn, ainv, na, mode == MTP_GRADE_FP32SPLIT, grade + i0, s);
    }, w);
    if (rc) return rc;
    ProfScope ps(&m->prof, P_REDUCE, s);
    launch_max(grade, n, grade_max, s);
  } else {
    HIP_TRY(hipMemsetAsync(grade_max, 0, sizeof(double), s));
  }
  HIP_TRY(hipGetLastError());
  if (m->grade_select > 0.0 || m->grade_break > 0.0) {
    double gm = 0.0;
    HIP_TRY(hipMemcpyAsync(&gm, grade_max, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (m->grade_break > 0.0 && gm > m->grade_break) return MTP_GRADE_BREAK;
    if (m->grade_select > 0.0 && gm > m->grade_select) return MTP_GRADE_SELECT;
  }
  return MTP_OK;
}

extern "C" int mtp_grade_config(mtp_model* m, const mtp_system* sys, const mtp_nlist* nl, const double* ainv,
                                double* descriptor, double* grade, void* stream) {
  int rc = check_system(m, sys);
  if (rc) return rc;
  if (!ainv || !grade) return mtp_fail(MTP_ERR_ARG, "null grade output or inverse active-set matrix");
  hipStream_t s = (hipStream_t)stream;
  const int n = sys->n_atoms;
  mtp_nlist use;
  if ((rc = resolve_nlist(m, sys, nl, &use, s))) return rc;
  const int na = m->ops.nalpha;
  const long ld = std::max(1, std::min(m->chunk, std::max(n, 1)));
  const long nchunks = ((long)n + ld - 1) / ld;
  // per-chunk descriptor partials [chunk][na], then the descriptor itself
  if ((rc = m->bvals.reserve((size_t)na * ld * sizeof(double))) ||
      (rc = m->eatom.reserve((size_t)std::max(n, 1) * sizeof(double))) ||
      (rc = m->dxi_part.reserve((size_t)(nchunks + 1) * na * sizeof(double))) ||
      (rc = m->rsum.reserve((size_t)na * kRowParts * sizeof(double))))
    return rc;
  double* bv = (double*)m->bvals.p;
  double* part = (double*)m->dxi_part.p;
  double* desc = descriptor ? descriptor : part + nchunks * na;
  if (n > 0) {
    long chunk = 0;
    ChainWork w;
    if ((rc = chain_work_reserve(m, n, use.n_pairs, false, &w))) return rc;
    rc = run_energy_chain(m, sys, use, (double*)m->eatom.p, false, bv, s, [&](int, int cn) {
      ProfScope ps(&m->prof, P_REDUCE, s);
      launch_rowsum(bv, ld, 1, cn, na, part + chunk * na, 1, s, (double*)m->rsum.p);
      ++chunk;
    }, w);
    if (rc) return rc;
    ProfScope ps(&m->prof, P_REDUCE, s);
    launch_rowsum(part, 1, na, nchunks, na, desc, 1, s);
  } else {
    HIP_TRY(hipMemsetAsync(desc, 0, (size_t)na * sizeof(double), s));
  }
  {
    ProfScope ps(&m->prof, P_GRADE, s);
    launch_cfg_grade(desc, ainv, na, grade, s);
  }
  HIP_TRY(hipGetLastError());
  if (m->grade_select > 0.0 || m->grade_break > 0.0) {
    double gm = 0.0;
    HIP_TRY(hipMemcpyAsync(&gm, grade, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (m->grade_break > 0.0 && gm > m->grade_break) return MTP_GRADE_BREAK;
    if (m->grade_select > 0.0 && gm > m->grade_select) return MTP_GRADE_SELECT;
  }
  return MTP_OK;
}

extern "C" int mtp_param_grad(mtp_model* m, const mtp_system* sys, const mtp_nlist* nl, double ebar,
                              const double* fbar, double* d_linear, double* d_radial, double* d_shift,
                              void* stream) {
  int rc = check_system(m, sys);
  if (rc) return rc;
  if ((sys->n_atoms > 0 && !fbar) || !d_linear || !d_radial || !d_shift)
    return mtp_fail(MTP_ERR_ARG, "null fbar or gradient outputs");
  if (!isfinite(ebar)) return mtp_fail(MTP_ERR_ARG, "non-finite ebar");
  hipStream_t s = (hipStream_t)stream;
  const LevelOps& L = m->ops;
  const int n = sys->n_atoms;
  const int na = L.nalpha;
  const long K = m->nrad;  // nsp^2 * nmu * ncheb
  if (n == 0) {
    HIP_TRY(hipMemsetAsync(d_linear, 0, na * sizeof(double), s));
    HIP_TRY(hipMemsetAsync(d_radial, 0, K * sizeof(double), s));
    HIP_TRY(hipMemsetAsync(d_shift, 0, m->nsp * sizeof(double), s));
    return MTP_OK;
  }
  mtp_nlist use;
  if ((rc = resolve_nlist(m, sys, nl, &use, s))) return rc;
  const int chunk = std::max(1, std::min(m->chunk, n));
  const long ld = chunk;
  const int nchunks = (n + chunk - 1) / chunk;
  long nblk = 0;
  for (int i0 = 0; i0 < n; i0 += chunk) nblk += (std::min(chunk, n - i0) + kLaneBlockHost - 1) / kLaneBlockHost;
  const long nparts = nblk * L.adj.nagroup;
  if ((rc = m->mom.reserve((size_t)L.nmom * ld * 8)) || (rc = m->cbar.reserve((size_t)L.ncomp * ld * 8)) ||
      (rc = m->mbar.reserve((size_t)L.nmom * ld * 8)) || (rc = m->mdot.reserve((size_t)L.nmom * ld * 8)) ||
      (rc = m->cbard.reserve((size_t)L.ncomp * ld * 8)) || (rc = m->mbard.reserve((size_t)L.nmom * ld * 8)) ||
      (rc = m->xout.reserve((size_t)na * ld * 8)) || (rc = m->eatom.reserve((size_t)n * 8)) ||
      (rc = m->dxi_part.reserve((size_t)na * nchunks * 8)) || (rc = m->cpart.reserve((size_t)nparts * K * 8)) ||
      (rc = m->rsum.reserve((size_t)std::max<long>(na, K) * kRowParts * 8)))
    return rc;
  SysArgs a = make_sys_args(m, sys, use);
  if (m->nsp > 1 && use.n_pairs > 0) {
    // neighbour species per pair, for the per-species passes of the adjoint pair kernel
    if ((rc = m->plink.reserve((size_t)use.n_pairs * 4)) || (rc = m->pfirst.reserve((size_t)n * m->nsp * 4)))
      return rc;
    launch_pair_links(use.off, use.j, sys->species, m->nsp, n, (int*)m->plink.p, (int*)m->pfirst.p, s);
    a.plink = (const int*)m->plink.p;
    a.pfirst = (const int*)m->pfirst.p;
  }
  double *mom = (double*)m->mom.p, *cbar = (double*)m->cbar.p, *mbar = (double*)m->mbar.p;
  double *mdot = (double*)m->mdot.p, *cbard = (double*)m->cbard.p, *mbard = (double*)m->mbard.p;
  double *xout = (double*)m->xout.p, *dxp = (double*)m->dxi_part.p, *cpart = (double*)m->cpart.p;
  long part = 0;
  int c = 0;
  for (int i0 = 0; i0 < n; i0 += chunk, ++c) {
    const int cn = std::min(chunk, n - i0);
    const long cblk = (cn + kLaneBlockHost - 1) / kLaneBlockHost;
    for (int g = 0; g < L.ngroup; ++g) {
      ProfScope ps(&m->prof, P_MOMENTS, s);
      L.chain[0].moments(g, a, i0, cn, mom, ld, s);
    }
    {
      ProfScope ps(&m->prof, P_PROG_FWD, s);
      L.chain[0].prog_fwd(mom, ld, i0, cn, nullptr, sys->species, (const double*)m->linear.p,
                          (const double*)m->shift.p, m->nsp, (double*)m->eatom.p, cbar, nullptr, s);
    }
    for (int g = 0; g < L.ngroup; ++g) {
      ProfScope ps(&m->prof, P_PROG_REV, s);
      L.chain[0].prog_rev(g, mom, ld, cn, cbar, mbar, s);
    }
    for (int g = 0; g < L.adj.ntgroup; ++g) {
      ProfScope ps(&m->prof, P_TANGENT, s);
      L.adj.tan_moments(g, a, fbar, i0, cn, mdot, ld, s);
    }
    {
      ProfScope ps(&m->prof, P_TANGENT, s);
      L.adj.tan_forward(a, mom, mdot, ld, i0, cn, (const double*)m->linear.p, ebar, xout, cbard, s);
    }
    for (int g = 0; g < L.adj.nrtpart; ++g) {
      ProfScope ps(&m->prof, P_TANGENT, s);
      L.adj.tan_reverse[g](mom, mdot, ld, cn, cbar, cbard, mbard, s);
    }
    for (int g = 0; g < L.adj.nagroup; ++g) {
      ProfScope ps(&m->prof, P_ADJ_PAIRS, s);
      L.adj.adj_pairs(g, a, fbar, i0, cn, mbar, mbard, ld, ebar, cpart + part * K, s);
      part += cblk;
    }
    ProfScope ps(&m->prof, P_REDUCE, s);
    launch_rowsum(xout, ld, 1, cn, na, dxp + c, nchunks, s, (double*)m->rsum.p);
  }
  {
    ProfScope ps(&m->prof, P_REDUCE, s);
    launch_rowsum(dxp, nchunks, 1, nchunks, na, d_linear, 1, s);
    launch_rowsum(cpart, 1, K, part, (int)K, d_radial, 1, s, (double*)m->rsum.p);
    launch_species_grad(sys->species, n, m->nsp, ebar, d_shift, s);
  }
  HIP_TRY(hipGetLastError());
  return MTP_OK;
}
