// C ABI entry points (include/hh.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "engine.h"
#include "hh_internal.h"
#include "krylov.h"

namespace hh {
void timing_set(bool on);
void timing_reset_all();
TimingFamily timing_get(int fam);
}  // namespace hh

using namespace hh;

namespace {

template <class F>
int guard(F&& f) {
  try {
    return f();
  } catch (const ArgError&) {
    return HH_EINVAL;
  } catch (const MemError&) {
    return HH_ENOMEM;
  } catch (const DeviceError&) {
    return HH_EDEVICE;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HH_ENOMEM;
  } catch (...) {
    set_error("unexpected exception");
    return HH_EDEVICE;
  }
}

#define REQUIRE(cond, ...)      \
  do {                          \
    if (!(cond)) {              \
      set_error(__VA_ARGS__);   \
      throw ArgError();         \
    }                           \
  } while (0)

void free_factors(FactorSet& fs) {
  dev_free(fs.band);
  dev_free(fs.img);
  dev_free(fs.piv);
  dev_free(fs.tr);
  dev_free(fs.d_strips);
  dev_free(fs.d_err);
  dev_free(fs.d_pflag);
  fs = FactorSet();
}

int dir_slot(const hh_problem* pb, unsigned dir) {
  REQUIRE(dir == HH_DIR_X || dir == HH_DIR_Y, "direction must be HH_DIR_X or HH_DIR_Y");
  const int d = dir == HH_DIR_X ? 0 : 1;
  for (int i = 0; i < pb->fs.nd; ++i)
    if (pb->fs.dir_id[i] == d) return i;
  set_error("direction %u has not been factored", dir);
  throw ArgError();
}

}  // namespace

namespace hh {

void factor_setup(hh_problem* pb, unsigned dirs, int nstrips, int precision) {
  REQUIRE(dirs >= 1 && dirs <= 3, "dirs must be HH_DIR_X, HH_DIR_Y or both");
  REQUIRE(precision == HH_FP64 || precision == HH_FP32, "precision must be HH_FP64 or HH_FP32");
  const int n = pb->n, N = nstrips;
  REQUIRE(N >= 1 && (n - 1) % N == 0, "(n-1) = %d is not divisible by nstrips = %d", n - 1, N);
  const int m = (n - 1) / N;
  REQUIRE(N == 1 || m >= 2, "each strip needs at least 2 intervals (nstrips <= (n-1)/2)");
  free_factors(pb->fs);
  FactorSet& fs = pb->fs;
  fs.N = N;
  fs.dirs = dirs;
  fs.precision = precision;
  if (dirs & HH_DIR_X) fs.dir_id[fs.nd++] = 0;
  if (dirs & HH_DIR_Y) fs.dir_id[fs.nd++] = 1;
  long long band = 0, img = 0, piv = 0, tr = 0;
  int kl_max = 0;
  for (int s = 0; s < N; ++s) {
    const int a = std::max(0, s * m - 1), b = std::min(n - 1, (s + 1) * m + 1);
    kl_max = std::max(kl_max, b - a + 2);
  }
  REQUIRE(kl_max <= 63, "strip band half-width %d exceeds 63 (strips too wide)", kl_max);
  const int S = 2 * kl_max + 1 <= 64 ? 1 : 2;
  const int P = sweep_segments(map_dim(blocked_kp(kl_max)), n,
                               precision == HH_FP64 ? sizeof(c128) : sizeof(c64));
  // the wide segment plan's maps are built only where that plan can run
  const bool wide = sweep_wide_fits(precision, P, kl_max, n);
  for (int i = 0; i < fs.nd; ++i) {
    for (int s = 0; s < N; ++s) {
      StripDesc sd{};
      sd.dir = fs.dir_id[i];
      sd.s = s;
      sd.a = std::max(0, s * m - 1);
      const int b = std::min(n - 1, (s + 1) * m + 1);
      sd.w = b - sd.a + 1;
      sd.ns = n * sd.w;
      sd.kl = sd.w + 1;
      sd.ldab = 3 * sd.kl + 1;
      sd.has1 = s > 0;
      sd.has2 = s < N - 1;
      sd.S = S;
      sd.KP = blocked_kp(kl_max);
      sd.gid = (int)fs.strips.size();
      const long long NP = sd.ns + HH_PAD;
      sd.band_off = band;
      band += (long long)sd.ns * sd.ldab;
      sd.segs = P;
      sd.wide = wide;
      plan_layout(sd);
      for (int p = 0; p < HH_NPLAN; ++p)
        REQUIRE(sd.pseg[p] >= sd.kl, "segment of %d rows is shorter than the band half-width %d",
                sd.pseg[p], sd.kl);
      sd.img_off = img;
      sd.t_off = img + 2 * blocked_blocks(sd.ns) * sd.KP * 64;
      sd.phi_off = sd.t_off + 2LL * sd.tmaps * map_dim(sd.KP) * map_dim(sd.KP);
      img += strip_image_elems(sd.ns, S, sd.KP, sd.kl, P, wide);
      sd.piv_off = piv;
      piv += NP;
      sd.tr1_off = sd.has1 ? tr : -1;
      if (sd.has1) tr += 7LL * n;
      sd.tr2_off = sd.has2 ? tr : -1;
      if (sd.has2) tr += 7LL * n;
      fs.max_ns = std::max(fs.max_ns, sd.ns);
      fs.max_kl = std::max(fs.max_kl, sd.kl);
      fs.strips.push_back(sd);
    }
  }
  const size_t es = precision == HH_FP64 ? sizeof(c128) : sizeof(c64);
  fs.band_elems = band;
  fs.img_elems = img;
  fs.piv_elems = piv;
  fs.tr_elems = std::max(tr, 1LL);
  fs.band = dev_alloc(fs.band_elems * es);
  fs.img = dev_alloc(fs.img_elems * es);
  fs.piv = (int*)dev_alloc(fs.piv_elems * sizeof(int));
  fs.tr = dev_alloc(fs.tr_elems * es);
  fs.d_strips = (StripDesc*)dev_alloc(fs.strips.size() * sizeof(StripDesc));
  fs.d_err = (int*)dev_alloc(2 * sizeof(int));
  fs.d_pflag = (int*)dev_alloc(fs.strips.size() * sizeof(int));
  fs.h_err = {0, 0};
}

// Queues the strip packing, the batched LU and the image build on st; the
// zero-pivot flag is copied back asynchronously (read by factor_finish).
void factor_launch(hh_problem* pb, hipStream_t st) {
  FactorSet& fs = pb->fs;
  HH_HIP(hipMemcpyAsync(fs.d_strips, fs.strips.data(), fs.strips.size() * sizeof(StripDesc),
                        hipMemcpyHostToDevice, st));
  HH_HIP(hipMemsetAsync(fs.d_err, 0, 2 * sizeof(int), st));
  HH_HIP(hipMemsetAsync(fs.d_pflag, 0, fs.strips.size() * sizeof(int), st));
  fs.batch_maps = fs.eager_batch_maps || !fs.strips[0].wide;
  launch_pack_strips(pb, st);
  launch_band_lu(pb, st);
  HH_HIP(hipMemcpyAsync(fs.h_err.data(), fs.d_err, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  fs.h_pflag.assign(fs.strips.size(), 0);
  HH_HIP(hipMemcpyAsync(fs.h_pflag.data(), fs.d_pflag, fs.strips.size() * sizeof(int),
                        hipMemcpyDeviceToHost, st));
}

// After the factorisation stream has completed: releases the LU work buffer
// and reports a zero pivot.
int factor_finish(hh_problem* pb) {
  FactorSet& fs = pb->fs;
  if (fs.batch_maps) {
    dev_free(fs.band);
    fs.band = nullptr;
  }
  fs.any_pivot = std::any_of(fs.h_pflag.begin(), fs.h_pflag.end(), [](int f) { return f != 0; });
  if (fs.h_err[0]) {
    const StripDesc& sd = fs.strips[fs.h_err[0] - 1];
    set_error("zero pivot in the LU of strip %d of direction %c", sd.s + 1, sd.dir == 0 ? 'x' : 'y');
    return HH_ESINGULAR;
  }
  return HH_OK;
}

void ensure_batch_maps(hh_problem* pb, hipStream_t st) {
  FactorSet& fs = pb->fs;
  if (fs.batch_maps) return;
  launch_transfer(fs, 1, st);
  HH_HIP(hipStreamSynchronize(st));
  dev_free(fs.band);
  fs.band = nullptr;
  fs.batch_maps = true;
}

// New problem handle with the operator assembled asynchronously on its stream.
hh_problem* problem_create(double omega, int nlayers, const double* c_layers, int n) {
  REQUIRE(std::isfinite(omega) && omega > 0, "omega must be positive and finite");
  REQUIRE(n >= 3 && n <= 8193, "n must be in [3, 8193]");
  REQUIRE(nlayers >= 1 && c_layers != nullptr, "need at least one layer speed");
  for (int l = 0; l < nlayers; ++l)
    REQUIRE(std::isfinite(c_layers[l]) && c_layers[l] > 0, "layer speed %d is not positive", l);
  std::unique_ptr<hh_problem> pb(new hh_problem());
  pb->n = n;
  pb->omega = omega;
  pb->c.assign(c_layers, c_layers + nlayers);
  HH_HIP(hipGetDevice(&pb->device));
  HH_HIP(hipStreamCreate(&pb->st[0]));
  HH_HIP(hipStreamCreate(&pb->st[1]));
  pb->d_c = (double*)dev_alloc(nlayers * sizeof(double));
  pb->d_A = (c128*)dev_alloc((size_t)4 * n * n * sizeof(c128));
  HH_HIP(hipMemcpyAsync(pb->d_c, pb->c.data(), nlayers * sizeof(double), hipMemcpyHostToDevice,
                        pb->st[0]));
  {
    TimedRegion tr(FAM_ASSEMBLE, pb->st[0], (double)n * n * 64.0);
    launch_assemble(n, omega, nlayers, pb->d_c, pb->d_A, pb->st[0]);
  }
  return pb.release();
}

void problem_destroy(hh_problem* pb) {
  if (!pb) return;
  (void)hipStreamSynchronize(pb->st[0]);
  (void)hipStreamSynchronize(pb->st[1]);
  free_factors(pb->fs);
  dev_free(pb->d_A);
  dev_free(pb->d_c);
  (void)hipStreamDestroy(pb->st[0]);
  (void)hipStreamDestroy(pb->st[1]);
  delete pb;
}

}  // namespace hh

extern "C" {

const char* hh_last_error(void) { return last_error(); }

int hh_assemble(double omega, int nlayers, const double* c_layers, int n, hh_problem** out) {
  return guard([&]() {
    REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    hh_problem* pb = problem_create(omega, nlayers, c_layers, n);
    hipError_t e = hipStreamSynchronize(pb->st[0]);
    if (e != hipSuccess) {
      problem_destroy(pb);
      set_error("assembly failed: %s", hipGetErrorString(e));
      return HH_EDEVICE;
    }
    *out = pb;
    return HH_OK;
  });
}

int hh_load_vector(hh_problem* pb, int nvec, const hh_c128* f, hh_c128* b) {
  return guard([&]() {
    REQUIRE(pb && f && b && nvec >= 0, "invalid arguments");
    launch_load_vector(pb->n, nvec, (const c128*)f, (c128*)b, pb->st[0]);
    HH_HIP(hipStreamSynchronize(pb->st[0]));
    return HH_OK;
  });
}

int hh_factor_sweeps(hh_problem* pb, unsigned dirs, int nstrips, int precision) {
  return guard([&]() {
    REQUIRE(pb != nullptr, "problem is NULL");
    factor_setup(pb, dirs, nstrips, precision);
    factor_launch(pb, pb->st[0]);
    HH_HIP(hipStreamSynchronize(pb->st[0]));
    return factor_finish(pb);
  });
}

int hh_strip_info(const hh_problem* pb, unsigned dir, int s, int* a, int* w, int* kl) {
  return guard([&]() {
    REQUIRE(pb != nullptr, "problem is NULL");
    const int i = dir_slot(pb, dir);
    REQUIRE(s >= 1 && s <= pb->fs.N, "strip index out of range");
    const StripDesc& sd = pb->fs.strips[(size_t)i * pb->fs.N + s - 1];
    if (a) *a = sd.a;
    if (w) *w = sd.w;
    if (kl) *kl = sd.kl;
    return HH_OK;
  });
}

int hh_strip_solve(hh_problem* pb, unsigned dir, int s, const hh_c128* rhs, hh_c128* x) {
  return guard([&]() {
    REQUIRE(pb && rhs && x, "invalid arguments");
    const int i = dir_slot(pb, dir);
    REQUIRE(s >= 1 && s <= pb->fs.N, "strip index out of range");
    const int si = i * pb->fs.N + s - 1;
    const size_t es = pb->fs.precision == HH_FP64 ? sizeof(c128) : sizeof(c64);
    ensure_batch_maps(pb, pb->st[0]);  // the strip solve runs segment plan 0
    void* work = dev_alloc(pb->fs.strips[si].ns * es);
    launch_strip_solve(pb, si, (const c128*)rhs, (c128*)x, work, pb->st[0]);
    HH_HIP(hipStreamSynchronize(pb->st[0]));
    dev_free(work);
    return HH_OK;
  });
}

int hh_sweep_apply(hh_problem* pb, unsigned dir, int nvec, const hh_c128* r, hh_c128* z) {
  return guard([&]() {
    REQUIRE(pb && r && z && nvec >= 0, "invalid arguments");
    const int i = dir_slot(pb, dir);
    if (nvec == 0) return HH_OK;
    const FactorSet& fs = pb->fs;
    const long long len = (long long)pb->n * pb->n;
    const size_t es = fs.precision == HH_FP64 ? sizeof(c128) : sizeof(c64);
    void* rho = dev_alloc((size_t)nvec * fs.max_ns * es);
    void* g1 = dev_alloc((size_t)nvec * fs.N * pb->n * es);
    void* zs = fs.precision == HH_FP64 ? (void*)z : dev_alloc((size_t)nvec * len * es);
    // one chain per right-hand side, one or plan_width(plan) workgroups per chain
    const int ntask = nvec;
    const int plan = sweep_plan_for(ntask, fs.precision, fs.strips[0].segs, fs.max_kl, pb->n,
                                    fs.any_pivot, fs.strips[0].wide != 0);
    const int G = plan_width(plan);
    hipStream_t st = pb->st[0];
    if (plan == 0) ensure_batch_maps(pb, st);
    // sync words: [0] abort, then one 128-byte line per chain
    unsigned* sync = (unsigned*)dev_alloc((size_t)(ntask + 1) * 128);
    void* xch = plan > 0 ? dev_alloc((size_t)ntask * G * 64 * es) : nullptr;
    HH_HIP(hipMemsetAsync(sync, 0, (size_t)(ntask + 1) * 128, st));
    std::vector<SweepTask> tasks(ntask);
    for (int v = 0; v < nvec; ++v) {
      SweepTask& tk = tasks[v];
      tk.ch.strips = fs.d_strips + (size_t)i * fs.N;
      tk.ch.r = (const c128*)r + v * len;
      tk.ch.z = (char*)zs + v * len * es;
      tk.ch.rho = (char*)rho + (size_t)v * fs.max_ns * es;
      tk.ch.g1 = (char*)g1 + (size_t)v * fs.N * pb->n * es;
      tk.img = fs.img;
      tk.piv = fs.piv;
      tk.pflag = fs.d_pflag;
      tk.tr = fs.tr;
      tk.n = pb->n;
      tk.N = fs.N;
      tk.xch = xch ? (char*)xch + (size_t)v * G * 64 * es : nullptr;
      tk.bar = sync + 32 * (v + 1);
    }
    SweepTask* d_tasks = (SweepTask*)dev_alloc(ntask * sizeof(SweepTask));
    HH_HIP(hipMemcpyAsync(d_tasks, tasks.data(), ntask * sizeof(SweepTask), hipMemcpyHostToDevice, st));
    {
      double bytes = 0;
      for (int q = 0; q < fs.N; ++q) {
        const StripDesc& sd = fs.strips[(size_t)i * fs.N + q];
        const double solves = q == fs.N - 1 ? 1.0 : 2.0;
        bytes += solves * ((double)sd.ns * sd.ldab * es + nvec * (double)sd.ns * (sizeof(c128) + es));
      }
      TimedRegion tr(FAM_SWEEP, st, bytes);
      launch_sweep(d_tasks, ntask, fs.precision, fs.strips[0].KP, fs.strips[0].segs, fs.max_kl,
                   pb->n, fs.any_pivot, plan, sync, st);
    }
    if (fs.precision != HH_FP64) launch_widen((const c64*)zs, (c128*)z, nvec * len, st);
    unsigned aborted = 0;
    HH_HIP(hipMemcpyAsync(&aborted, sync, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HH_HIP(hipStreamSynchronize(st));
    dev_free(d_tasks);
    dev_free(rho);
    dev_free(g1);
    dev_free(xch);
    dev_free(sync);
    if (zs != (void*)z) dev_free(zs);
    if (aborted) {
      set_error("sweep workgroups of one chain did not meet within the time limit");
      throw DeviceError();
    }
    return HH_OK;
  });
}

int hh_spmv(hh_problem* pb, int nvec, const hh_c128* x, hh_c128* y) {
  return guard([&]() {
    REQUIRE(pb && x && y && nvec >= 0, "invalid arguments");
    if (nvec == 0) return HH_OK;
    SpmvTask tk{};
    tk.A = pb->d_A;
    tk.x = x;
    tk.y = (c128*)y;
    tk.n = pb->n;
    tk.nvec = nvec;
    SpmvTask* d = (SpmvTask*)dev_alloc(sizeof(SpmvTask));
    hipStream_t st = pb->st[0];
    HH_HIP(hipMemcpyAsync(d, &tk, sizeof(tk), hipMemcpyHostToDevice, st));
    {
      const double len = (double)pb->n * pb->n;
      TimedRegion tr(FAM_SPMV, st, len * (64.0 + nvec * 32.0));
      launch_spmv(d, 1, (long long)pb->n * pb->n, HH_FP64, st);
    }
    HH_HIP(hipStreamSynchronize(st));
    dev_free(d);
    return HH_OK;
  });
}

int hh_get_operator(const hh_problem* pb, hh_c128* diag) {
  return guard([&]() {
    REQUIRE(pb && diag, "invalid arguments");
    HH_HIP(hipMemcpy(diag, pb->d_A, (size_t)4 * pb->n * pb->n * sizeof(c128), hipMemcpyDeviceToHost));
    return HH_OK;
  });
}

int hh_mpgmres(hh_problem* pb, int nrhs, const hh_c128* b, double tol, int maxit, hh_c128* x,
               hh_stats* stats) {
  return guard([&]() {
    REQUIRE(pb && b && x && nrhs >= 0, "invalid arguments");
    REQUIRE(pb->fs.precision >= 0, "hh_factor_sweeps has not been called");
    REQUIRE(std::isfinite(tol) && tol > 0, "tol must be positive");
    REQUIRE(maxit >= 1, "maxit must be >= 1");
    if (nrhs == 0) return HH_OK;
    const long long len = (long long)pb->n * pb->n;
    std::vector<Solve> solves(nrhs);
    std::vector<Solve*> ptr(nrhs);
    for (int r = 0; r < nrhs; ++r) {
      Solve& s = solves[r];
      s.pb = pb;
      s.b = (const c128*)b + r * len;
      s.x = (c128*)x + r * len;
      s.len = len;
      s.tol = tol;
      s.maxit = maxit;
      ptr[r] = &s;
    }
    Engine eng(pb->st[0]);
    int rc = HH_OK;
    try {
      eng.begin(ptr);
      for (;;) {
        bool any = false;
        for (Solve* s : ptr) any |= !s->done;
        if (!any) break;
        eng.step(ptr);
      }
      eng.finish(ptr);
    } catch (...) {
      for (Solve* s : ptr) Engine::release(s);
      throw;
    }
    for (int r = 0; r < nrhs; ++r) {
      Solve& s = solves[r];
      if (!s.converged) rc = HH_ENOCONV;
      if (stats) {
        stats[r].iterations = s.k;
        stats[r].converged = s.converged ? 1 : 0;
        stats[r].res_est = s.res_est;
        stats[r].res_true = s.res_true;
        stats[r].basis_size = s.m - s.deflated;
        stats[r].deflated = s.deflated;
      }
      Engine::release(&s);
    }
    if (rc == HH_ENOCONV) set_error("MPGMRES did not reach the tolerance within maxit for some RHS");
    return rc;
  });
}

int hh_free(hh_problem* pb) {
  if (!pb) return HH_OK;
  return guard([&]() {
    problem_destroy(pb);
    return HH_OK;
  });
}

int hh_timing_enable(int on) {
  timing_set(on != 0);
  return HH_OK;
}

int hh_timing_reset(void) {
  return guard([&]() {
    timing_reset_all();
    return HH_OK;
  });
}

int hh_timing_get(const char* family, long long* launches, double* total_ms, double* bytes) {
  return guard([&]() {
    REQUIRE(family != nullptr, "family is NULL");
    static const char* names[FAM_COUNT] = {"sweep", "spmv", "factor", "orth", "assemble"};
    int f = -1;
    for (int i = 0; i < FAM_COUNT; ++i)
      if (std::strcmp(family, names[i]) == 0) f = i;
    REQUIRE(f >= 0, "unknown timing family '%s'", family);
    TimingFamily t = timing_get(f);
    if (launches) *launches = t.launches;
    if (total_ms) *total_ms = t.ms;
    if (bytes) *bytes = t.bytes;
    return HH_OK;
  });
}

}  // extern "C"
