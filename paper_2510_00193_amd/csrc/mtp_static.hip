// Energy, forces and virial from a fixed scratch area, for callers that cannot allocate device
// memory (code under stream capture, serving loops, harnesses that forbid allocation).
//
// The scratch area is one file-scope device array per GPU.  Its device address is resolved once
// per device (mtp_create, with the model's device current) and kept in a per-device table; host
// code uses that address, never the array's name.  The entry point carves the energy chain's
// buffers out of it, so it calls no allocator; every call on one GPU shares the area, and calls
// that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "mtp.h"
#include "mtp_api_internal.h"
#include "mtp_internal.h"

using namespace mtp;

namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU, held until the process ends
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;
constexpr int kMinChunk = 64;                       // chunks are whole workgroups of 64 atoms

void* g_scratch_addr[kMaxDevices] = {nullptr};
std::mutex g_scratch_mu;

size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

int static_scratch_resolve(void** ptr) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return mtp_fail(MTP_ERR_HIP, "hipGetDevice failed");
  }
  if (dev < 0 || dev >= kMaxDevices) return mtp_fail(MTP_ERR_HIP, "device index outside the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return mtp_fail(MTP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_addr[dev] = p;
  }
  *ptr = g_scratch_addr[dev];
  return MTP_OK;
}

size_t static_scratch_bytes() { return kScratchBytes; }

namespace {
// Byte layout of the scratch area for one call; total() is what it needs.
struct StaticLayout {
  size_t part = 0, flag = 0, eatom = 0, g = 0, fown = 0, wpart = 0, mom = 0, cbar = 0, mbar = 0, end = 0;
};

StaticLayout layout_for(const LevelOps& L, int n, long long npairs, bool need_eatom, bool backward, int chunk,
                        int split) {
  StaticLayout s;
  size_t o = 0;
  s.part = o;
  o += align_up(7 * kSumParts * sizeof(double));
  s.flag = o;
  o += kAlign;
  s.eatom = o;
  if (need_eatom) o += align_up((size_t)std::max(n, 1) * sizeof(double));
  s.mom = o;
  o += align_up((size_t)L.nmom * chunk * sizeof(double));
  s.cbar = o;
  o += align_up((size_t)L.ncomp * chunk * sizeof(double));
  if (backward) {
    s.mbar = o;
    o += align_up((size_t)L.nmom * chunk * sizeof(double));
    s.g = o;
    o += align_up((size_t)std::max<long long>(npairs, 1) * 3 * sizeof(double));
    s.fown = o;
    o += align_up((size_t)std::max(n, 1) * 3 * sizeof(double));
    s.wpart = o;
    o += align_up((size_t)chain_wpart_blocks(n, chunk, split) * 6 * sizeof(double));
  }
  s.end = o;
  return s;
}
}  // namespace

extern "C" int mtp_compute_static(mtp_model* m, const mtp_system* sys, const mtp_nlist* nl, double* energy,
                                  double* e_atom, double* forces, double* virial, void* stream) {
  int rc = check_system(m, sys);
  if (rc) return rc;
  if (!nl) return mtp_fail(MTP_ERR_ARG, "mtp_compute_static needs a neighbour list (building one allocates)");
  if (!m->static_scratch) return mtp_fail(MTP_ERR_HIP, "scratch area not resolved for this model's device");
  hipStream_t s = (hipStream_t)stream;
  const int n = sys->n_atoms;
  const bool backward = forces || virial;
  // the model's chunk, shrunk in whole workgroups until the buffers fit: per-atom results and
  // the per-workgroup virial partials do not depend on the chunk when it is a multiple of 64
  int chunk = std::max(1, std::min(m->chunk, std::max(n, 1)));
  const int split = pair_split(m, n);
  StaticLayout lay = layout_for(m->ops, n, nl->n_pairs, !e_atom, backward, chunk, split);
  while (lay.end > kScratchBytes && chunk > kMinChunk) {
    chunk = std::max(kMinChunk, (chunk / 2 + kMinChunk - 1) / kMinChunk * kMinChunk);
    lay = layout_for(m->ops, n, nl->n_pairs, !e_atom, backward, chunk, split);
  }
  if (lay.end > kScratchBytes)
    return mtp_fail(MTP_ERR_CAPACITY, "mtp_compute_static: " + std::to_string(n) + " atoms and " +
                                          std::to_string(nl->n_pairs) + " pairs need " + std::to_string(lay.end) +
                                          " bytes of scratch, the fixed area holds " +
                                          std::to_string(kScratchBytes));
  unsigned char* base = (unsigned char*)m->static_scratch;
  mtp_nlist use;
  if ((rc = resolve_nlist(m, sys, nl, &use, s, (int*)(base + lay.flag)))) return rc;
  double* ea = e_atom ? e_atom : (double*)(base + lay.eatom);
  ChainWork w;
  w.chunk = chunk;
  w.mom = base + lay.mom;
  w.cbar = base + lay.cbar;
  if (backward) {
    w.mbar = base + lay.mbar;
    w.g = (double*)(base + lay.g);
    w.fown = (double*)(base + lay.fown);
    w.wpart = (double*)(base + lay.wpart);
  }
  // timing events would be created on first use: no profiling inside this call
  const bool prof = m->prof.on;
  m->prof.on = false;
  if (n > 0) rc = run_energy_chain(m, sys, use, ea, backward, nullptr, s, nullptr, w);
  if (!rc) rc = finish_compute(m, use, n, ea, w, (double*)(base + lay.part), energy, forces, virial, s);
  m->prof.on = prof;
  return rc;
}
