/*
 * mtp.h - C ABI of the MI355X Moment Tensor Potential library (libmtp.so).
 *
 * The library evaluates the Moment Tensor Potential, the model the paper
 * accelerates inside LAMMPS (Section 2.1: inference yields energies, forces
 * and stresses; active learning adds an extrapolation grade in neighbourhood
 * or configuration mode).  The potential itself is defined by the MTP
 * formulation the paper cites in Section 1:
 *
 *   u       = (2 r - (r_min + r_cut)) / (r_cut - r_min)
 *   Q_b(r)  = T_b(u) (r_cut - r)^2                   Chebyshev T_b, b < n_cheb
 *   f_mu    = sum_b c[z_i][z_j][mu][b] Q_b(r_ij)
 *   M_mu,nu = sum_j f_mu(r_ij) d_ij^(x nu)           d_ij = R_j + n.H - R_i (full vector)
 *   B_alpha = full contraction of moments (every contraction multigraph of level <= L,
 *             moment level 2 + 4 mu + nu, disconnected products included)
 *   E_i     = s[z_i] + sum_alpha xi_alpha B_alpha(i),  E = sum_i E_i
 *   F_k     = -dE/dR_k,   W = -sum_{i,j} d_ij (x) dE_i/dd_ij
 *   grade_i = max_k |sum_alpha B_alpha(i) Ainv[alpha][k]|
 *
 * Conventions shared by every call:
 *   - Device pointers are caller-owned device memory (for instance torch
 *     tensors); host pointers are said to be host.  Arrays are C-contiguous.
 *   - stream is a hipStream_t passed as void*; NULL means the null stream.
 *     Work is enqueued on it; calls return before the GPU finishes unless a
 *     call says it synchronizes.
 *   - Every call returns an MTP_* status and never aborts; mtp_last_error()
 *     gives a message for the calling thread.
 *   - A handle is not thread-safe; use one handle per stream.
 *   - The basis order (index alpha of the linear coefficients) is: total
 *     level, then moment labels (mu, nu) sorted ascending, then the smallest
 *     row-major upper-triangle tuple of the contraction matrix.
 */
#ifndef MTP_H
#define MTP_H

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MTP_OK 0
#define MTP_ERR_ARG 1         /* invalid argument (null pointer, bad size, species out of range) */
#define MTP_ERR_CELL 2        /* singular cell, or a shift outside the packed range */
#define MTP_ERR_CAPACITY 3    /* caller buffer too small; the required size is reported */
#define MTP_ERR_NONFINITE 4   /* a non-finite position was found */
#define MTP_ERR_HIP 5         /* a HIP runtime call failed */
#define MTP_ERR_OOM 6         /* device allocation failed */
#define MTP_ERR_LEVEL 7       /* this level is not compiled into the library */
#define MTP_GRADE_BREAK 8     /* grade_max exceeded grade_break; outputs are still written */
#define MTP_GRADE_SELECT 9    /* grade_max exceeded grade_select (but not grade_break) */

/* precision of the moment/contraction arithmetic */
#define MTP_FP64 0            /* everything in binary64 */
#define MTP_FP32_MOMENTS 1    /* radial functions, moments, contractions and pair gradients in
                                 binary32; displacements, energies, virial and force sums in binary64 */

/* grade product */
#define MTP_GRADE_FP64 0      /* B . Ainv on binary64 matrix cores */
#define MTP_GRADE_FP32SPLIT 1 /* hi/lo binary32 split, three binary32 matrix-core products,
                                 binary64 accumulation of the tile partials */

typedef struct mtp_model mtp_model;

typedef struct {
  int level;             /* MTP level L (even, compiled set reported by mtp_levels) */
  int n_species;         /* number of species, >= 1 */
  int n_cheb;            /* Chebyshev basis size n_cheb, 1..16 */
  double r_min, r_cut;   /* radial interval (Angstrom), 0 <= r_min < r_cut */
  const double* radial;  /* host [n_species][n_species][n_mu][n_cheb], c[z_i][z_j][mu][b] */
  const double* linear;  /* host [n_alpha], xi in the basis order above */
  const double* shift;   /* host [n_species], per-species energy constant s */
  int precision;         /* MTP_FP64 or MTP_FP32_MOMENTS */
  int chunk_atoms;       /* atoms evaluated per chunk (bounds workspace, cf. the paper's
                            chunksize, Section 2.3); 0 = library default (1,048,576 atoms,
                            about 2 KB of workspace per atom at level 16); at most 2^28,
                            else MTP_ERR_ARG */
  double grade_select;   /* grade_max above this returns MTP_GRADE_SELECT; <= 0 disables */
  double grade_break;    /* grade_max above this returns MTP_GRADE_BREAK; <= 0 disables */
  int lanes_per_atom;    /* lanes that share one atom's neighbour loop in the binary64 pair
                            kernels (moments, pair gradients) of a single system: 1, 2, 4 or 8,
                            or 0 = chosen from the system size so that the waves cover the
                            GPU's SIMDs (small systems; cf. the paper's block-parallel variant
                            for small atom counts, Section 2.1).  The binary32 form and batches
                            use one lane per atom. */
} mtp_params;

typedef struct {
  int n_atoms;           /* N >= 0 */
  const double* pos;     /* device [N][3] Cartesian positions, used as given (not wrapped) */
  const int* species;    /* device [N], values in [0, n_species) */
  double cell[9];        /* host copy of H, rows are the lattice vectors (row-major) */
} mtp_system;

/* Canonical full neighbour list in CSR form (all device memory).
 * Row i holds every (j, n) with 0 < |R_j - R_i + n.H|^2 < r_cut^2, j = i allowed when n != 0,
 * sorted by (j, n1, n2, n3).  The squared distance is evaluated in binary64 round-to-nearest
 * without fused multiply-add as
 *     t_a = (n1 H[0][a] + n2 H[1][a]) + n3 H[2][a],  d_a = (R_j[a] - R_i[a]) + t_a,
 *     dd  = (d_0 d_0 + d_1 d_1) + d_2 d_2,  test dd < r_cut * r_cut.
 * shift packs n: byte k (k = 0, 1, 2) holds n_{k+1} as a two's-complement int8.
 * rev[p] is the index of the mirrored pair (j, i, -n). */
typedef struct {
  const int* off;        /* [N + 1] */
  const int* j;          /* [n_pairs] */
  const int* shift;      /* [n_pairs] */
  const int* rev;        /* [n_pairs] */
  long long n_pairs;
  int checked;           /* 1: written by mtp_neighbors for these positions and cell and not
                            modified since, used as is.  0: validated before use (one pass over
                            the list on the device and one synchronization): off[0] = 0,
                            off[N] = n_pairs, rows non-decreasing, 0 <= j < N, every rev[p] a pair
                            of row j[p] whose partner is the row's atom, with the negated shift,
                            and rev[rev[p]] = p; species in [0, n_species).  A list that fails
                            returns MTP_ERR_ARG and nothing else is enqueued. */
} mtp_nlist;

/* Number of compiled levels and their values (host array of at least 32 ints). */
int mtp_levels(int* n, int* levels);

/* Sizes of a compiled level without creating a model.  info (host, n_info ints) receives
 * [n_alpha, n_mu, n_moments, n_components, n_products, max_nu, n_groups]: basis functions,
 * radial functions, stored moment components, connected contractions, weighted products
 * of the compiled contraction program, largest tensor rank, moment groups per pass. */
int mtp_level_info(int level, int* info, int n_info);

/* Create a model: copies the parameters to the device.  Synchronizes. */
int mtp_create(const mtp_params* p, mtp_model** out);
void mtp_destroy(mtp_model* m);
const char* mtp_last_error(void);

/* Sizes of the model: basis functions, radial functions, stored moment components,
 * connected contractions (any pointer may be NULL). */
int mtp_sizes(const mtp_model* m, int* n_alpha, int* n_mu, int* n_moments, int* n_components);

/* Replace the coefficients in place.  Pointers are device memory when on_device != 0,
 * else host; NULL keeps the current value.  Enqueued on stream (graph-safe when on_device). */
int mtp_set_params(mtp_model* m, const double* radial, const double* linear, const double* shift,
                   int on_device, void* stream);

/* Build the canonical neighbour list of a system into caller buffers (device).  The paper's
 * variants read LAMMPS half lists (the Kokkos flags of Section 2.3, newton on, neigh half); this
 * library builds a full list itself so that every row is complete and the result is
 * reproducible bit for bit.
 * off must hold N + 1 ints; j, shift and rev must hold cap ints each (rev may be NULL).
 * *n_pairs (host) receives the pair count.  If it exceeds cap, nothing but off is written
 * and MTP_ERR_CAPACITY is returned.  Synchronizes the stream once (to read the count). */
int mtp_neighbors(mtp_model* m, const mtp_system* sys, int* off, int* j, int* shift, int* rev,
                  long long cap, long long* n_pairs, void* stream);

/* Energy, forces and virial (device outputs; any may be NULL), the inference use case of
 * Section 2.1 (energies, forces and stresses):
 *   energy [1], e_atom [N], forces [N][3], virial [6] as xx, yy, zz, xy, xz, yz with
 *   W_ab = -sum_pairs d_a g_b (g = dE_i/dd_ij), positive under repulsion.
 * nl: a list for these positions (see mtp_nlist.checked), or NULL to build one internally
 * (then the call synchronizes once).  Results are deterministic run to run. */
int mtp_compute(mtp_model* m, const mtp_system* sys, const mtp_nlist* nl, double* energy,
                double* e_atom, double* forces, double* virial, void* stream);

/* mtp_compute without allocation, for callers that cannot allocate device memory (code under
 * stream capture into a graph, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments and results as mtp_compute (bit-identical), except:
 *   - nl is required (building a list allocates); an unchecked list is validated as in
 *     mtp_compute, which synchronizes, so callers that capture pass a checked list;
 *   - every intermediate lives in one fixed 64 MiB device scratch area per GPU, reserved when
 *     the library is loaded and held until the process ends.  At level 16 that is about
 *     20,000 atoms in one chunk; larger systems run in smaller chunks of the model's atoms down
 *     to 64, and a system whose pair gradients and per-atom sums alone do not fit (about
 *     90,000 atoms at level 16) returns MTP_ERR_CAPACITY before anything is enqueued;
 *   - all calls on one GPU share the area and it keeps the last call's contents: calls that
 *     overlap on one GPU (two streams, two threads, two models) race and must be serialized
 *     by the caller;
 *   - profiling (mtp_profile) does not time this call.
 * No hipMalloc, hipFree or memset is issued; the work is kernel launches on the stream. */
int mtp_compute_static(mtp_model* m, const mtp_system* sys, const mtp_nlist* nl, double* energy,
                       double* e_atom, double* forces, double* virial, void* stream);

/* Neighbourhood-mode extrapolation grade (Section 2.3 of the paper):
 *   grade [N] (device) = max_k |(B_i Ainv)_k|, grade_max [1] (device) = max_i grade_i.
 * ainv: device [n_alpha][n_alpha] row-major.  mode: MTP_GRADE_FP64 or MTP_GRADE_FP32SPLIT.
 * When grade_select or grade_break is set in the parameters the call synchronizes, compares
 * grade_max and returns MTP_GRADE_SELECT / MTP_GRADE_BREAK (outputs written either way). */
int mtp_grade(mtp_model* m, const mtp_system* sys, const mtp_nlist* nl, const double* ainv,
              int mode, double* grade, double* grade_max, void* stream);

/* Configuration-mode extrapolation grade (the second active-learning mode of Section 2.1; the
 * definition is MLIP-3's): descriptor b [n_alpha] = sum_i B_i (= dE/dxi), reduced over atoms in
 * a fixed order, and grade [1] (device) = max_k |(b Ainv)_k|.  ainv: device [n_alpha][n_alpha]
 * row-major.  descriptor: device [n_alpha] output, or NULL.  Thresholds as for mtp_grade, with
 * the configuration's grade in place of grade_max. */
int mtp_grade_config(mtp_model* m, const mtp_system* sys, const mtp_nlist* nl, const double* ainv,
                     double* descriptor, double* grade, void* stream);

/* Active-set update by MaxVol row swaps.  The paper bases the extrapolation grade on
 * D-optimality and the MaxVol algorithm (Section 1): the active set is the n x n matrix A
 * whose rows are the basis vectors of selected neighbourhoods (or configuration descriptors),
 * a candidate row c has grade max_k |(c A^-1)_k|, and replacing active row k by candidate i
 * multiplies |det A| by |(c_i A^-1)_k|.  The call runs the MaxVol iteration (Goreinov et al.,
 * 2010): take the candidate entry of largest |(c_i A^-1)_k| (the first in row-major order
 * among equal values); if it exceeds 1 + tol, exchange active row k and candidate row i and
 * update A^-1 by the Sherman-Morrison formula; repeat, at most max_swaps times.
 *   cand  device [n_cand][n], active device [n][n], ainv device [n][n] = active^-1, row-major,
 *         all updated in place (rows exchanged, ainv kept as the inverse).
 *   swaps host [2 * max_swaps] or NULL: the (i, k) of every swap in order; grades host
 *         [max_swaps] or NULL: the signed (c_i A^-1)_k of every swap; *n_swaps (host) swaps done.
 * 1 <= n <= 4096.  Synchronizes once per iteration (the host decides whether to continue).
 * Returns MTP_ERR_ARG for bad sizes or null matrices, and when the selected entry is not finite
 * (NaN or infinite candidates or inverse): the swaps done before stay applied and counted. */
int mtp_maxvol(mtp_model* m, double* cand, int n_cand, int n, double* active, double* ainv, double tol,
               int max_swaps, int* swaps, double* grades, int* n_swaps, void* stream);

/* Vector-Jacobian product of (E, F) with respect to the coefficients.  The paper keeps MLIP-3's
 * potential files and its fitting (Section 1 and Section 2.3); this call is the gradient a fit
 * needs, computed on the device:
 *   d_linear [n_alpha], d_radial [n_species^2 n_mu n_cheb], d_shift [n_species] (device) =
 *   ebar dE/dtheta + sum_k fbar_k . dF_k/dtheta,  fbar device [N][3].
 * For the loss (E - E0)^2 + sum |F - F0|^2 pass ebar = 2 (E - E0), fbar = 2 (F - F0). */
int mtp_param_grad(mtp_model* m, const mtp_system* sys, const mtp_nlist* nl, double ebar,
                   const double* fbar, double* d_linear, double* d_radial, double* d_shift,
                   void* stream);

/* ---- Batched training over many small configurations ------------------------------------
 * Not in the paper, which evaluates one configuration per MD step; this is the batched form
 * of the same path for fitting on a training set.  The batch always runs in binary64.
 *
 * mtp_batch_create: configurations c = 0..n_cfg-1 hold atoms atom_off[c] .. atom_off[c+1]-1
 *   (host int array, atom_off[0] = 0, non-decreasing); pos (device [N][3]) and species
 *   (device [N]) are referenced, not copied, and must stay valid for the batch's lifetime;
 *   cells (host [n_cfg][9], rows = lattice vectors) are copied.  Builds every
 *   configuration's canonical neighbour list once (synchronizes) and reserves all workspace.
 * mtp_batch_run: energies [n_cfg], forces [N][3], virials [n_cfg][6] (device, any may be
 *   NULL) of every configuration; with targets e_target [n_cfg] and f_target [N][3] also the
 *   loss L = sum_c (E_c - E0_c)^2 + sum_i |F_i - F0_i|^2 (loss [1], may be NULL) and its
 *   gradient d_linear [n_alpha], d_radial [n_sp^2 n_mu n_cheb], d_shift [n_sp] (device).
 *   One launch per kernel type covers all configurations.  It allocates nothing and never
 *   synchronizes; with use_graph != 0 the sequence is captured once into a hipGraph (per set
 *   of output pointers) and replayed on an internal stream ordered after and before the
 *   caller's stream.  Coefficient updates through mtp_set_params(on_device = 1) reach the
 *   replays without re-capture.
 * mtp_batch_tune: times the schedules on this batch and keeps the fastest: atom order (natural,
 *   or sorted by neighbour count so that a wave's lanes do similar work and the longest tiles
 *   come first), chunk of atoms per pass, and static grids or persistent pair kernels (one
 *   workgroup per SIMD pulling 64-atom tiles from a device counter inside the same launch
 *   sequence, zeroed by a kernel so that graph capture stays valid); with cache_path (text
 *   file) the pick is read back for the same level, species, Chebyshev count and size bucket.
 *   choice (host [3], may be NULL) receives {sorted, chunk_atoms, persistent}.  Synchronizes.
 * mtp_batch_schedule: sets a schedule explicitly (sorted 0/1, chunk_atoms 0 = all atoms,
 *   persistent 0/1).
 * mtp_batch_neighbors: device pointers of the batch's CSR list (global atom indices). */
typedef struct mtp_batch mtp_batch;
int mtp_batch_create(mtp_model* m, int n_cfg, const int* atom_off, const double* pos, const int* species,
                     const double* cells, mtp_batch** out, void* stream);
int mtp_batch_run(mtp_batch* b, const double* e_target, const double* f_target, double* energy,
                  double* forces, double* virial, double* loss, double* d_linear, double* d_radial,
                  double* d_shift, int use_graph, void* stream);
int mtp_batch_tune(mtp_batch* b, const char* cache_path, int* choice, void* stream);
/* mtp_batch_vjp: the vector-Jacobian product of every configuration's (E_c, F) for any
 *   cotangents: d_linear [n_alpha], d_radial [n_sp^2 n_mu n_cheb], d_shift [n_sp] (device) =
 *   sum_c ebar_c dE_c/dtheta + sum_i fbar_i . dF_i/dtheta, with ebar device [n_cfg] and fbar
 *   device [N][3].  The forward state is recomputed (nothing is kept from an earlier run).
 *   Allocates nothing, never synchronizes; use_graph as for mtp_batch_run. */
int mtp_batch_vjp(mtp_batch* b, const double* ebar, const double* fbar, double* d_linear, double* d_radial,
                  double* d_shift, int use_graph, void* stream);
int mtp_batch_schedule(mtp_batch* b, int sorted, int chunk_atoms, int persistent);
int mtp_batch_sizes(const mtp_batch* b, int* n_atoms, long long* n_pairs, int* sorted, int* chunk_atoms,
                    int* persistent);
int mtp_batch_neighbors(const mtp_batch* b, const int** off, const int** j, const int** shift,
                        const int** rev);
void mtp_batch_destroy(mtp_batch* b);

/* Per-kernel timing with HIP events recorded on the caller's stream around every launch of the
 * hot path (for benchmarks; off by default).  mtp_profile_read synchronizes the recorded
 * events, adds them to the totals, and reports kernel class k: its name (static string),
 * accumulated milliseconds and launch count; MTP_ERR_ARG past the last class.
 * mtp_profile_reset clears the totals. */
int mtp_profile(mtp_model* m, int enable);
int mtp_profile_read(mtp_model* m, int k, const char** name, double* total_ms, long long* launches);
int mtp_profile_reset(mtp_model* m);

#ifdef __cplusplus
}
#endif
#endif /* MTP_H */
