// Preconditioner application that allocates no device memory.
//
// For callers that cannot allocate (code under HIP graph capture, tight
// serving loops): the scratch of one application (task descriptors, sync
// words, strip buffers, complex64 staging, exchange areas) lives in one
// static device array of HH_NOALLOC_SCRATCH bytes, which every GPU that runs
// the library holds until the process ends.  Host code never uses the
// array's name as an address: its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and that pointer is
// what the kernels receive.  Calls that overlap on one GPU share the array
// and race; each call clears what has to start at zero (the sync words).
#include <mutex>

#include "hh_internal.h"

namespace hh {

namespace {

constexpr size_t HH_NOALLOC_SCRATCH = size_t(64) << 20;
constexpr int HH_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[HH_NOALLOC_SCRATCH];

std::mutex g_scratch_mu;
void* g_scratch_ptr[HH_MAX_DEVICES] = {};

// Device address of this device's scratch (looked up on first use).
char* scratch_ptr(int device) {
  if (device < 0 || device >= HH_MAX_DEVICES) {
    set_error("device %d is beyond the %d devices the no-allocation scratch tracks", device,
              HH_MAX_DEVICES);
    throw ArgError();
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    HH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = p;
  }
  return (char*)g_scratch_ptr[device];
}

}  // namespace

void sweep_apply_noalloc(hh_problem* pb, int i, int mode, int nvec, const c128* r, c128* z) {
  if (nvec == 0) return;
  int cur = -1;
  HH_HIP(hipGetDevice(&cur));
  if (cur != pb->device) {
    set_error("the problem lives on device %d but device %d is current", pb->device, cur);
    throw ArgError();
  }
  const int plan = sweep_plan_of(pb, nvec);
  size_t need = 0;
  sweep_layout(pb, nvec, plan, nullptr, &need);
  if (need > HH_NOALLOC_SCRATCH) {
    set_error("%d vectors need %zu bytes of scratch; the no-allocation entry point holds %zu",
              nvec, need, HH_NOALLOC_SCRATCH);
    throw ArgError();
  }
  if (plan != HH_PLAN_WIDE && !pb->fs.batch_maps) {
    set_error("the batch plans' maps are not built: apply the preconditioner once with the "
              "allocating entry point first");
    throw ArgError();
  }
  char* base = scratch_ptr(cur);
  sweep_apply_core(pb, i, mode, nvec, r, z, plan, sweep_layout(pb, nvec, plan, base, &need));
}

}  // namespace hh
