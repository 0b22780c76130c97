// Host/device declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

namespace mtp {

constexpr int kMaxSpecies = 8;
constexpr int kMaxMu = 8;
constexpr int kMaxGroups = 4;    // moment groups per level
constexpr int kMaxRevParts = 16;  // parts of the reverse-tangent program per level
constexpr int kMaxRadial = 1024;  // doubles of the staged c[z_i][z_j][mu][b] table
constexpr int kMaxChebHost = 16;

// Per-system arguments of the pair kernels (passed by value: lands in kernel-argument SGPRs).
struct SysArgs {
  const double* pos;      // [N][3]
  const int* species;     // [N]
  const int* off;         // [N+1]
  const int* nj;          // [P]
  const int* shift;       // [P] packed int8 x3
  const double* radial;   // [nsp][nsp][nmu][ncheb]
  double H[9];            // rows = lattice vectors (single system)
  const double* cells;    // [n_cfg][9] per-configuration cells (batches), or null
  const int* cfg;         // [N] configuration of each atom (batches), or null
  const int* perm;        // [N] processing order: lane k of the sweep takes atom perm[k], or null
  const double* ebar;     // [n_cfg] per-configuration energy cotangent (batches), or null
  // per-species chains through the rows (launch_pair_links), or null for one species
  const int* plink;       // [P] next pair of the same row and neighbour species, -1 at the end
  const int* pfirst;      // [N][nsp] first pair of each neighbour species, -1 if none
  double sa, sb, rcut;    // u = sa r + sb
  int nsp, nmu, ncheb;
  // persistent launches of the pair kernels: a device counter from which workgroups pull their
  // 64-atom tiles (zeroed before the launch), and the number of workgroups; null for a grid of
  // one workgroup per tile
  int* queue;
  int pgrid;
  // lanes per atom of the single-system pair kernels (1, 2, 4 or 8): with more than one, the
  // lanes of an atom take every split-th pair of its row and combine their sums
  int split;
};

// Energy/force chain of one level in one arithmetic type (per-atom buffers m, cbar, mbar are
// arrays of that type; energies, pair gradients and virial partials stay binary64).
struct ChainOps {
  void (*moments)(int g, const SysArgs& a, int i0, int n, void* m, long ld, hipStream_t s);
  void (*prog_fwd)(const void* m, long ld, int i0, int n, const int* perm, const int* species,
                   const double* xi, const double* shift, int nsp, double* e_atom, void* cbar,
                   double* bout, hipStream_t s);
  void (*prog_rev)(int g, const void* m, long ld, int n, const void* cb, void* mb, hipStream_t s);
  // fown (optional, [atom][3]): (+)= the atom's own pair-gradient sum, for launch_gather_forces
  void (*backward)(int grp, const SysArgs& a, int i0, int n, const void* mb, long ld, double* g,
                   int acc, double* wpart, double* watom, double* fown, hipStream_t s);
  // forward + products + reverse in one kernel (single-group levels, one system; else null):
  // writes e_atom[i0 + k] and the moment adjoints
  void (*program)(const void* m, long ld, int i0, int n, const int* species, const double* xi,
                  const double* shift, int nsp, double* e_atom, void* mb, hipStream_t s);
};

// Parameter-adjoint launchers of one level (binary64).
struct AdjOps {
  void (*tan_moments)(int grp, const SysArgs& a, const double* fbar, int i0, int n, double* md,
                      long ld, hipStream_t s);
  void (*tan_forward)(const SysArgs& a, const double* m, const double* md, long ld, int i0, int n,
                      const double* xi, double ebar, double* out, double* cbard, hipStream_t s);
  // one launcher per part of the reverse-tangent program (compiled in separate units); the
  // parts store or add their entries of mbd and run in order 0 .. nrtpart - 1 on one stream
  void (*tan_reverse[kMaxRevParts])(const double* m, const double* md, long ld, int n, const double* cb,
                                    const double* cbd, double* mbd, hipStream_t s);
  int nrtpart;
  // grp is one of the nagroup adjoint groups (moment ranges sized for the pair kernel's
  // registers, independent of the chain's groups)
  void (*adj_pairs)(int grp, const SysArgs& a, const double* fbar, int i0, int n, const double* mb,
                    const double* mbd, long ld, double ebar, double* cpart, hipStream_t s);
  int nagroup;
  int ntgroup;  // moment ranges of tan_moments (the adjoint ranges or the chain's groups)
};

// Launchers of one compiled level (assembled from the level's translation units).
struct LevelOps {
  int level, nmom, ncomp, nalpha, nmu, maxnu, ngroup, triples;
  ChainOps chain[3];  // [0] binary64, [1] binary32 moments (null when not compiled),
                      // [2] binary64 for batches (per-atom cells, atom permutation, per-atom virials)
  AdjOps adj;
};

// neighbour list (mtp_nbr.hip)
struct NbrWork;
struct NbrPlan {
  bool cells;              // cell-list path (else all-pairs with per-pair image ranges)
  int nb[3];               // bins per axis (cell path)
  double Hinv[9];
  double reach[3];         // r_cut |b_k|
};
void nbr_plan(const double* H, double rcut, NbrPlan* plan, int* status);
// Counting pass: writes off[0..N] (exclusive scan of counts) and returns the pair total
// through the host pointer (synchronizes).  Host flags[4]: [0] a non-finite position,
// [1] a species outside [0, nsp), [2] an image index outside the packed int8 range.
int nbr_count(const NbrPlan& plan, const double* pos, const int* species, int nsp, int n,
              const double* H, double rcut, NbrWork* w, int* off, long long* total, int* flags,
              hipStream_t s);
int nbr_fill(const NbrPlan& plan, const double* pos, int n, const double* H, double rcut,
             NbrWork* w, const int* off, int* nj, int* shift, int* rev, long long total,
             hipStream_t s);
// Batched build (image path per configuration): counts (synchronizes), then asks alloc for the
// j/shift/rev arrays of *total pairs (slots 0, 1, 2) and fills them.  flags as for nbr_count;
// when a flag is set nothing is filled.
int nbr_batch_build(const double* pos, const int* species, int nsp, int n, const int* cfg,
                    const int* atom_off, const double* cells, const double* cinv, const double* reach,
                    double rcut, NbrWork* w, int* off, int** nj, int** shift, int** rev,
                    long long* total, int* flags, int* (*alloc)(void* ctx, int slot, long long n),
                    void* ctx, hipStream_t s);
NbrWork* nbr_work_create();
void nbr_work_destroy(NbrWork* w);

// level-independent kernels (mtp_common.hip)
// x[0..n) = v by a kernel (no memset node when a caller captures the stream into a graph)
void launch_fill(double* x, long n, double v, hipStream_t s);
void launch_fill_int(int* x, long n, int v, hipStream_t s);
// forces = (fown ? fown : own row sums of g) - mirrored gradients g[rev[p]]
void launch_gather_forces(const int* off, const int* rev, const double* g, const double* fown, int n,
                          long long npairs, double* forces, hipStream_t s);
void launch_sum(const double* x, long n, long stride, double* out, hipStream_t s);
// Two-level deterministic sums of ncomp strided components (part: ncomp * kSumParts doubles).
constexpr int kSumParts = 256;
// energy (ea over n atoms) and virial (nb per-workgroup partials) of a small system in one
// launch; either output may be null.  For n and nb up to kSmallSumMax.
constexpr int kSmallSumThreads = 1024;
constexpr long kSmallSumMax = 32768;
void launch_sum_small(const double* ea, long n, const double* wpart, long nb, double* energy, double* virial,
                      hipStream_t s);
// launch_sum_parts over two arrays in one pair of launches (part: (nc1 + nc2) * kSumParts
// doubles); each output equals what launch_sum_parts gives for its array
void launch_sum_parts2(const double* x1, long n1, long st1, int nc1, double* out1, const double* x2, long n2,
                       long st2, int nc2, double* out2, double* part, hipStream_t s);
void launch_sum_parts(const double* x, long n, long stride, int ncomp, double* part, double* out,
                      hipStream_t s);
void launch_sum_virial(const double* wpart, long nblocks, double* out, hipStream_t s);

// out[r * os] = sum_{k < n} x[r * rs + k * es], r < rows (deterministic: the order depends on n
// and on whether tmp is given).  tmp (optional, rows * kRowParts doubles) lets rows of at least
// kRowSplitMin terms be summed by kRowParts workgroups each.
constexpr int kRowParts = 64;
constexpr long kRowSplitMin = 16384;
void launch_rowsum(const double* x, long rs, long es, long n, int rows, double* out, long os,
                   hipStream_t s, double* tmp = nullptr);
void launch_species_grad(const int* species, int n, int nsp, double ebar, double* out, hipStream_t s);
void launch_segsum(const double* x, long stride, const int* seg_off, int nseg, int ncomp, double* out,
                   long os, hipStream_t s);
void launch_loss(const double* e, const double* e0, int ncfg, const double* f, const double* f0, long n,
                 double* ebar, double* fbar, double* part_cfg, double* part_atoms, hipStream_t s);
// d/ds_t of sum_c ebar_c E_c over a batch; tmp holds nsp * kRowParts doubles
void launch_species_grad_cfg(const int* species, const int* cfg, const double* ebar, int n, int nsp,
                             double* out, double* tmp, hipStream_t s);

// grade (mtp_grade.hip)
void launch_grade(const double* B, long ld, int n, const double* ainv, int na, int split,
                  double* grade, hipStream_t s);
void launch_max(const double* x, long n, double* out, hipStream_t s);
// zp[p] = species of neighbour nj[p], clamped to [0, nsp)
// *bad |= 1 when the CSR list (off, nj, shift, rev) of n atoms and npairs pairs is inconsistent
// or a species lies outside [0, nsp) (*bad is not cleared here)
void launch_check_nlist(const int* off, const int* nj, const int* shift, const int* rev, const int* species,
                        int n, long long npairs, int nsp, int* bad, hipStream_t s);
void launch_pair_links(const int* off, const int* nj, const int* species, int nsp, int n, int* plink,
                       int* pfirst, hipStream_t s);
// out[0] = max_k |(b . ainv)_k| for one descriptor b [na]
void launch_cfg_grade(const double* b, const double* ainv, int na, double* out, hipStream_t s);

}  // namespace mtp
