// Host runtime of the library: error reporting, the caching device
// allocator and the per-family kernel timers.
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>

#include "hh_internal.h"

namespace hh {

// ------------------------------------------------------------ errors
namespace {
thread_local char g_err[1024] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

const char* last_error() { return g_err; }

// ------------------------------------------------------------ allocator
// Exact-size caching of device blocks: repeated solves of the same shapes
// reuse memory without calling hipMalloc.  Sizes are rounded up to 2 MiB
// above 2 MiB and to 256 B below.
namespace {
std::mutex g_mem_mu;
std::multimap<size_t, void*> g_free;
std::map<void*, size_t> g_live;
// caller's allocator (hh_set_allocator): blocks go straight to and from it
void* (*g_user_alloc)(size_t, void*) = nullptr;
void (*g_user_free)(void*, void*) = nullptr;
void* g_user_ctx = nullptr;

size_t round_size(size_t b) {
  const size_t big = size_t(2) << 20;
  if (b >= big) return (b + big - 1) / big * big;
  return (b + 255) & ~size_t(255);
}
}  // namespace

void* dev_alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  size_t sz = round_size(bytes);
  void* (*ua)(size_t, void*) = nullptr;
  void* uctx = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    ua = g_user_alloc;
    uctx = g_user_ctx;
  }
  if (ua) {
    // the caller's allocator, called outside the library's lock
    void* p = ua(sz, uctx);
    if (!p) {
      set_error("the caller's allocator returned no memory for %zu bytes", sz);
      throw MemError();
    }
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_live[p] = sz;
    return p;
  }
  std::lock_guard<std::mutex> lk(g_mem_mu);
  auto it = g_free.find(sz);
  void* p = nullptr;
  if (it != g_free.end()) {
    p = it->second;
    g_free.erase(it);
  } else {
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
      // release cached blocks and retry once
      (void)hipGetLastError();
      for (auto& kv : g_free) (void)hipFree(kv.second);
      g_free.clear();
      e = hipMalloc(&p, sz);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation of %zu bytes failed: %s", sz, hipGetErrorString(e));
        throw MemError();
      }
    }
  }
  g_live[p] = sz;
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  void (*uf)(void*, void*) = nullptr;
  void* uctx = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    const size_t sz = it->second;
    g_live.erase(it);
    if (g_user_free) {
      uf = g_user_free;
      uctx = g_user_ctx;
    } else {
      g_free.emplace(sz, p);
    }
  }
  if (uf) uf(p, uctx);
}

// Installs (or with null functions removes) the caller's allocator.  Only
// while the library holds no device memory, so that every block returns to
// the allocator it came from; the library's cached blocks are released.
bool set_allocator(void* (*alloc)(size_t, void*), void (*free_fn)(void*, void*), void* ctx) {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  if (!g_live.empty()) return false;
  for (auto& kv : g_free) (void)hipFree(kv.second);
  g_free.clear();
  g_user_alloc = alloc;
  g_user_free = alloc ? free_fn : nullptr;
  g_user_ctx = alloc ? ctx : nullptr;
  return true;
}

size_t dev_live_bytes() {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  size_t s = 0;
  for (auto& kv : g_live) s += kv.second;
  return s;
}

namespace {
std::mutex g_st_mu;
hipStream_t g_caller_st[2] = {nullptr, nullptr};
}  // namespace

void set_caller_streams(hipStream_t x, hipStream_t y) {
  std::lock_guard<std::mutex> lk(g_st_mu);
  g_caller_st[0] = x;
  g_caller_st[1] = y;
}

bool caller_streams(hipStream_t& x, hipStream_t& y) {
  std::lock_guard<std::mutex> lk(g_st_mu);
  x = g_caller_st[0];
  y = g_caller_st[1];
  return x != nullptr || y != nullptr;
}

void dev_trim() {
  std::lock_guard<std::mutex> lk(g_mem_mu);
  for (auto& kv : g_free) (void)hipFree(kv.second);
  g_free.clear();
}

// ------------------------------------------------------------ timing
namespace {
std::mutex g_t_mu;
bool g_t_on = false;
TimingFamily g_fam[FAM_COUNT];
struct Pending {
  int fam;
  hipEvent_t e0, e1;
  double bytes;
};
std::vector<Pending> g_pending;
// Events are reused rather than created per region (creation costs host time
// inside the iteration loop).  They only time work, so they skip the
// system-scope fence: no cache write-back and invalidation at each record.
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event() {
  {
    std::lock_guard<std::mutex> lk(g_t_mu);
    if (!g_event_pool.empty()) {
      hipEvent_t e = g_event_pool.back();
      g_event_pool.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool timing_on() { return g_t_on; }

void runtime_release_caches() {
  timing_flush();
  {
    std::lock_guard<std::mutex> lk(g_t_mu);
    for (hipEvent_t e : g_event_pool) (void)hipEventDestroy(e);
    g_event_pool.clear();
  }
  dev_trim();
}

TimedRegion::TimedRegion(int family, hipStream_t s, double b) : fam(family), st(s), bytes(b) {
  if (!g_t_on) return;
  e0 = take_event();
  e1 = take_event();
  if (!e0 || !e1) {
    std::lock_guard<std::mutex> lk(g_t_mu);
    for (hipEvent_t e : {e0, e1})
      if (e) g_event_pool.push_back(e);
    e0 = e1 = nullptr;
    return;
  }
  (void)hipEventRecord(e0, st);
}

TimedRegion::~TimedRegion() {
  if (!e0) return;
  (void)hipEventRecord(e1, st);
  std::lock_guard<std::mutex> lk(g_t_mu);
  g_pending.push_back({fam, e0, e1, bytes});
}

void timing_flush() {
  std::lock_guard<std::mutex> lk(g_t_mu);
  for (auto& p : g_pending) {
    float ms = 0;
    if (hipEventSynchronize(p.e1) == hipSuccess && hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
      g_fam[p.fam].launches += 1;
      g_fam[p.fam].ms += ms;
      g_fam[p.fam].bytes += p.bytes;
    }
    g_event_pool.push_back(p.e0);
    g_event_pool.push_back(p.e1);
  }
  g_pending.clear();
}

void timing_set(bool on) { g_t_on = on; }

void timing_reset_all() {
  timing_flush();
  std::lock_guard<std::mutex> lk(g_t_mu);
  for (auto& f : g_fam) f = TimingFamily();
}

TimingFamily timing_get(int fam) {
  timing_flush();
  std::lock_guard<std::mutex> lk(g_t_mu);
  return g_fam[fam];
}

// ------------------------------------------------------------ sizes
size_t FactorSet::bytes() const {
  size_t es = precision == HH_FP64 ? sizeof(c128) : sizeof(c64);
  return band_elems * es + img_elems * es + piv_elems * sizeof(int) + tr_elems * es +
         strips.size() * sizeof(StripDesc) + 2 * sizeof(int);
}

}  // namespace hh

size_t hh_problem::bytes() const {
  return (size_t)4 * n * n * sizeof(hh::c128) + c.size() * sizeof(double) + fs.bytes();
}
