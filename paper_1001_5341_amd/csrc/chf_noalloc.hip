// chf_forward_scratch: the full forward run of a plan inside a static device array, for callers
// that cannot allocate device memory (code under graph capture, tight serving loops, harnesses
// that forbid allocation).  The plan's own workspace binding and state are left untouched.
#include <hip/hip_runtime.h>

#include <mutex>

#include "chf_internal.h"

namespace {

constexpr uint64_t kScratchBytes = (uint64_t)CHF_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per GPU, resident until the process ends.  In host code `scratch` is a host-side
// stand-in: only the address hipGetSymbolAddress returns for the current device may reach a
// kernel or a copy.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch` per device, set on first use

// Device address of the current device's copy (looked up once per device, that device current).
hipError_t scratch_ptr(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || (uintptr_t)p % 256) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

uint64_t chf_scratch_bytes(void) { return kScratchBytes; }

chf_status chf_forward_scratch(chf_plan *p, void *stream, const double *q_bins_dev, double *w_dev) {
  if (!p) {
    chf::set_error("NULL plan");
    return CHF_EINVAL;
  }
  if (p->dev.n_obs > 0 && !w_dev) {
    chf::set_error("waveforms_dev is NULL");
    return CHF_EINVAL;
  }
  if (p->ws_bytes > kScratchBytes) {
    chf::set_error("plan needs " + std::to_string(p->ws_bytes) + " bytes of workspace, above the " +
                   std::to_string(kScratchBytes) + "-byte static scratch (use chf_forward with a bound workspace)");
    return CHF_ENOMEM;
  }
  void *sp = nullptr;
  hipError_t e = scratch_ptr(&sp);
  if (e != hipSuccess) {
    chf::set_error(std::string("scratch lookup: ") + hipGetErrorString(e));
    return CHF_EHIP;
  }
  hipStream_t s = (hipStream_t)stream;
  // the plan's own binding and step state, restored once the run is enqueued (kernels take their
  // parameter block by value)
  char *ws0 = p->ws;
  const chf::Dev dev0 = p->dev;
  const int par0 = p->parity, done0 = p->n_done, adj0 = p->adj_next, ls0 = p->lev_swap, ps0 = p->pe_swap;
  hipStream_t aux0 = p->aux;
  p->aux = nullptr;  // no side stream: the boundary sweep runs in order on `stream`
  e = chf::bind_tables(p, (char *)sp, s);
  if (e == hipSuccess) e = chf::launch_zero(*p, s);
  p->parity = 0;
  p->n_done = 0;
  if (e == hipSuccess) e = chf::advance(*p, s, q_bins_dev, w_dev, 0, p->grid.n_steps, p->grid.n_steps);
  p->ws = ws0;
  p->dev = dev0;
  p->parity = par0;
  p->n_done = done0;
  p->adj_next = adj0;
  p->lev_swap = ls0;
  p->pe_swap = ps0;
  p->aux = aux0;
  if (e != hipSuccess) {
    chf::set_error(std::string("scratch forward: ") + hipGetErrorString(e));
    return CHF_EHIP;
  }
  return CHF_OK;
}

}  // extern "C"
