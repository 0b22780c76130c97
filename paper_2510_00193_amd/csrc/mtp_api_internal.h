// Host-side model and workspace shared by the library's API translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "mtp.h"
#include "mtp_internal.h"

constexpr int kMaxChunk = 1 << 28;  // atoms per chunk at most: per-lane byte offsets in a row fit 32 bits
constexpr int kDefaultChunk = 1 << 20;  // atoms per chunk: bounds the per-atom workspace (~2 KB/atom at level 16)
constexpr int kLaneBlockHost = 64;     // workgroup size of the lane-per-atom kernels
constexpr int kMaxAllPairsAtoms = 200000;  // largest system searched pair by pair (thin cells)

// Grow-only device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf();
  int reserve(size_t n);
};

// Kernel classes timed by the profiler.
enum ProfClass { P_NBR = 0, P_MOMENTS, P_PROG_FWD, P_PROG_REV, P_BACKWARD, P_GATHER, P_REDUCE, P_GRADE,
                 P_TANGENT, P_ADJ_PAIRS, P_BATCH, P_PROGRAM, P_NCLASS };

struct Profiler {
  bool on = false;
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<hipEvent_t> pool;
  std::vector<Rec> pending;
  double ms[P_NCLASS] = {0};
  long long launches[P_NCLASS] = {0};
  hipEvent_t take();
  ~Profiler();
};

// Brackets the launches of one kernel class with events when profiling is on.
struct ProfScope {
  Profiler* p;
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(Profiler* p_, int cls_, hipStream_t s_);
  ~ProfScope();
};

struct mtp_model {
  mtp::LevelOps ops;
  int nsp = 0, ncheb = 0, precision = 0, chunk = 0;
  int split = 0, ncu = 256;  // lanes per atom (0 = by system size), compute units of the device
  long nrad = 0;
  double rmin = 0, rcut = 0, grade_select = 0, grade_break = 0;
  DevBuf radial, linear, shift;                        // coefficients (device)
  DevBuf nl_off, nl_j, nl_shift, nl_rev;               // internally built neighbour list
  DevBuf mom, cbar, mbar, bvals, g, fown, eatom, wpart;  // per-chunk / per-pair workspace
  DevBuf mdot, cbard, mbard, xout, dxi_part, cpart;   // parameter-adjoint workspace
  DevBuf plink, pfirst;                                 // per-species pair chains (adjoint)
  DevBuf rsum;                                          // partials of long row sums
  DevBuf scratch;
  DevBuf flag;                                          // status word of the list check
  void* static_scratch = nullptr;                       // device address of the fixed scratch area
  mtp::NbrWork* nbr = nullptr;
  Profiler prof;
};

int mtp_fail(int code, const std::string& msg);
int resolve_nlist(mtp_model* m, const mtp_system* sys, const mtp_nlist* nl, mtp_nlist* out,
                  hipStream_t s, int* flag = nullptr);
mtp::SysArgs make_sys_args(const mtp_model* m, const mtp_system* sys, const mtp_nlist& nl);
// Buffers of the energy chain: moments, contraction adjoints and moment adjoints per chunk atom
// ([entry][chunk] layout), per-pair gradients g [P][3], own force sums [N][3] and the
// per-workgroup virial partials; wblocks is the number of partials the chain wrote.
struct ChainWork {
  void* mom = nullptr;
  void* cbar = nullptr;
  void* mbar = nullptr;
  double* g = nullptr;
  double* fown = nullptr;
  double* wpart = nullptr;
  int chunk = 1;
  long wblocks = 0;
};
// lanes per atom of the binary64 single-system pair kernels for a system of n atoms
int pair_split(const mtp_model* m, int n);
// workgroups of a pair kernel over n atoms with `split` lanes per atom (one virial partial each)
long pair_blocks(int n, int split);
// upper bound of the virial partials the chain writes for n atoms in chunks of `chunk`
long chain_wpart_blocks(int n, int chunk, int split);
// chain buffers from the model's grow-only workspace
int chain_work_reserve(mtp_model* m, int n, long long npairs, bool backward, ChainWork* w);
int run_energy_chain(mtp_model* m, const mtp_system* sys, const mtp_nlist& nl, double* e_atom,
                     bool backward, double* bvals, hipStream_t s,
                     const std::function<void(int, int)>& after_forward, ChainWork& w);
int finish_compute(mtp_model* m, const mtp_nlist& nl, int n, const double* ea, const ChainWork& w,
                   double* part, double* energy, double* forces, double* virial, hipStream_t s);
int check_system(const mtp_model* m, const mtp_system* sys);
// device address of the library's fixed scratch area on the current device (resolved once per
// device), and its size in bytes
int static_scratch_resolve(void** ptr);
size_t static_scratch_bytes();
