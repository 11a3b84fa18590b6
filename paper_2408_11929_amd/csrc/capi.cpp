// C ABI entry points (include/hh.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "engine.h"
#include "hh_internal.h"
#include "krylov.h"
#include "tune.h"

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

// Factored slot and sweep order of a preconditioner kind (HH_PRE_*).
void kind_slot(const hh_problem* pb, int kind, int& slot, int& mode) {
  REQUIRE(kind >= HH_PRE_LRL && kind <= HH_PRE_TB, "unknown preconditioner kind %d", kind);
  const bool y = kind == HH_PRE_BTB || kind == HH_PRE_BT || kind == HH_PRE_TB;
  slot = dir_slot(pb, y ? HH_DIR_Y : HH_DIR_X);
  mode = kind == HH_PRE_LRL || kind == HH_PRE_BTB ? SWEEP_DOUBLE
         : kind == HH_PRE_LR || kind == HH_PRE_BT ? SWEEP_FORWARD
                                                  : SWEEP_REVERSE;
}

// z = M^{-1} r for nvec vectors with the strips of factored slot i in the
// given sweep order (one chain per vector), on scratch from the allocator.
void sweep_apply(hh_problem* pb, int i, int mode, int nvec, const c128* r, c128* z) {
  if (nvec == 0) return;
  const int plan = sweep_plan_of(pb, nvec);
  size_t bytes = 0;
  sweep_layout(pb, nvec, plan, nullptr, &bytes);
  void* base = dev_alloc(bytes);
  try {
    sweep_apply_core(pb, i, mode, nvec, r, z, plan, sweep_layout(pb, nvec, plan, (char*)base, &bytes));
  } catch (...) {
    (void)hipStreamSynchronize(pb->st[0]);
    dev_free(base);
    throw;
  }
  dev_free(base);
}

}  // namespace

namespace hh {

// Sub-blocks of every strip for recursive strip solves: nsub per strip along
// its length, the outer strips' rule (one extra line past each internal
// boundary), each ordered by its narrower side; lane-major factors only.
static void sub_block_setup(FactorSet& fs, int n, int nsub, long long& band, long long& img,
                            long long& piv, long long& tr) {
  const int m2 = (n - 1) / nsub;
  const int nouter = (int)fs.strips.size();
  fs.first_sub = nouter;
  int kl_max = 0, ns_sub = 0, w_max = 0;
  // one window slot count for all sub-blocks (the sweep kernel's template)
  for (int o = 0; o < nouter; ++o)
    for (int t = 0; t < nsub; ++t) {
      const int len = std::min(n - 1, (t + 1) * m2 + 1) - std::max(0, t * m2 - 1) + 1;
      kl_max = std::max(kl_max, std::min(fs.strips[o].w, len) + 1);
    }
  REQUIRE(kl_max <= HH_KL_MAX, "sub-block band half-width %d exceeds %d", kl_max, HH_KL_MAX);
  const int SL = lane_slots(kl_max);
  fs.strips.reserve((size_t)nouter * (1 + nsub));
  for (int o = 0; o < nouter; ++o) {
    // a copy: the push_backs below may move the vector's storage
    fs.strips[o].sub = (int)fs.strips.size() - o;  // relative to the strip's own descriptor
    fs.strips[o].nsub = nsub;
    const StripDesc sd = fs.strips[o];
    w_max = std::max(w_max, sd.w);
    for (int t = 0; t < nsub; ++t) {
      StripDesc u{};
      u.dir = sd.dir;
      u.s = sd.s;
      u.a = sd.a;
      u.w = sd.w;
      u.c0 = std::max(0, t * m2 - 1);
      u.len = std::min(n - 1, (t + 1) * m2 + 1) - u.c0 + 1;
      u.orient = sd.w <= u.len ? 0 : 1;
      u.ns = sd.w * u.len;
      u.nr = u.ns;
      u.kl = (u.orient == 0 ? sd.w : u.len) + 1;
      u.ldab = 3 * u.kl + 1;
      u.has1 = t > 0;
      u.has2 = t < nsub - 1;
      u.SL = SL;
      u.S = 2 * SL;
      u.KP = sd.KP;
      u.segs = sd.segs;
      u.gid = (int)fs.strips.size();
      u.sub = -1;
      u.band_off = band;
      band += (long long)u.ns * u.ldab;
      u.img_off = img;
      img += (long long)(u.ns + HH_PAD) * (64LL * 3 * u.SL + 1);
      u.piv_off = piv;
      piv += u.ns + HH_PAD;
      u.tr1_off = u.has1 ? tr : -1;
      if (u.has1) tr += 7LL * sd.w;
      u.tr2_off = u.has2 ? tr : -1;
      if (u.has2) tr += 7LL * sd.w;
      ns_sub = std::max(ns_sub, u.ns);
      fs.strips.push_back(u);
    }
  }
  // every sub-block inside its strip, with the geometry the kernels index by
  for (int o = 0; o < nouter; ++o) {
    const StripDesc& sd = fs.strips[o];
    REQUIRE(sd.sub == (int)fs.strips.size() - nouter * nsub + o * (nsub - 1) && sd.nsub == nsub,
            "sub-block layout of strip %d", o);
    for (int t = 0; t < nsub; ++t) {
      const StripDesc& u = fs.strips[o + sd.sub + t];
      REQUIRE(u.w == sd.w && u.a == sd.a && u.dir == sd.dir && u.c0 >= 0 && u.len >= 3 &&
                  u.c0 + u.len <= n && u.ns == u.w * u.len && u.ns <= sd.ns &&
                  u.kl == (u.orient ? u.len : u.w) + 1 && u.kl <= kl_max && u.SL == SL &&
                  u.band_off >= 0 && u.img_off >= 0 && u.piv_off >= 0,
              "sub-block %d of strip %d is inconsistent", t, o);
    }
  }
  fs.max_kl = kl_max;
  // per chain: the strip right-hand side, the inner solution and the
  // sub-block work vector (ns of the strip each), the inner Gamma_1 data
  // (nsub x w)
  fs.rho_elems = 3LL * fs.max_ns + (long long)nsub * w_max + 64;
}

void factor_setup(hh_problem* pb, unsigned dirs, int nstrips, int precision, int nsub) {
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
  fs.npre = fs.nd;  // LRL, then BTB: the ordered combination of Sec. 4
  for (int i = 0; i < fs.nd; ++i) {
    fs.pre_slot[i] = i;
    fs.pre_mode[i] = SWEEP_DOUBLE;
  }
  long long band = 0, img = 0, piv = 0, tr = 0;
  int kl_max = 0;
  for (int s = 0; s < N; ++s) {
    const int a = std::max(0, s * m - 1), b = std::min(n - 1, (s + 1) * m + 1);
    kl_max = std::max(kl_max, b - a + 2);
  }
  const bool rec = nsub > 1;
  if (rec) {
    REQUIRE((n - 1) % nsub == 0, "(n-1) = %d is not divisible by nsub = %d", n - 1, nsub);
    REQUIRE((n - 1) / nsub >= 2, "each sub-block needs at least 2 intervals (nsub <= (n-1)/2)");
  } else {
    REQUIRE(kl_max <= HH_KL_MAX, "strip band half-width %d exceeds %d (strips too wide)", kl_max,
            HH_KL_MAX);
  }
  const bool lane_major = !rec && kl_max > HH_KL_WINDOW;  // blocked MFMA LU, lane-major substitution
  const int SL = lane_major ? lane_slots(kl_max) : 1;
  const int S = lane_major ? 2 * SL : 2 * kl_max + 1 <= 64 ? 1 : 2;
  const int P = sweep_segments(map_dim(blocked_kp(kl_max)), n,
                               precision == HH_FP64 ? sizeof(c128) : sizeof(c64));
  // the wide segment plan's maps are built only where that plan can run
  const bool wide = !rec && !lane_major && sweep_wide_fits(precision, P, kl_max, n);
  for (int i = 0; i < fs.nd; ++i) {
    for (int s = 0; s < N; ++s) {
      StripDesc sd{};
      sd.dir = fs.dir_id[i];
      sd.s = s;
      sd.a = std::max(0, s * m - 1);
      const int b = std::min(n - 1, (s + 1) * m + 1);
      sd.w = b - sd.a + 1;
      sd.nr = n * sd.w;
      // strips whose sweeps may take the wide plan get identity rows up to a
      // whole number of its segment groups, so that a workgroup's rows of
      // the back substitution are its own of the forward one (mirror); not
      // where plan 0 is the one taken (eager_batch_maps: the server)
      sd.ns = sd.nr;
      if (wide && !fs.eager_batch_maps) {
        const long long grp = (long long)P * plan_seg(sd.nr, P, HH_PLAN_WIDE, sd.w + 1);
        sd.ns = (int)((sd.nr + grp - 1) / grp * grp);
      }
      sd.kl = sd.w + 1;
      sd.ldab = 3 * sd.kl + 1;
      sd.has1 = s > 0;
      sd.has2 = s < N - 1;
      sd.S = S;
      sd.SL = SL;
      sd.KP = blocked_kp(kl_max);
      sd.gid = (int)fs.strips.size();
      sd.sub = -1;
      sd.nsub = 1;
      const long long NP = sd.ns + HH_PAD;
      sd.band_off = band;
      if (!rec) band += (long long)sd.ns * sd.ldab;  // recursive: the sub-blocks hold the factors
      sd.segs = P;
      sd.wide = wide;
      plan_layout(sd);
      sd.mirror = 0;
      for (int p = 1; p < HH_NPLAN && wide; ++p)
        if (plan_width(p) > 1 && sd.ns % ((long long)P * sd.pseg[p]) == 0) sd.mirror |= 1 << p;
      REQUIRE(!wide || fs.eager_batch_maps || (sd.mirror >> HH_PLAN_WIDE & 1),
              "strip %d: %d rows are not whole segment groups of the wide plan", s, sd.ns);
      for (int p = 0; p < HH_NPLAN && !lane_major; ++p)
        REQUIRE(sd.pseg[p] >= sd.kl, "segment of %d rows is shorter than the band half-width %d",
                sd.pseg[p], sd.kl);
      sd.img_off = img;
      sd.t_off = img + 2 * blocked_blocks(sd.ns) * sd.KP * 64;
      long long po = sd.t_off + 2LL * sd.tmaps * map_dim(sd.KP) * map_dim(sd.KP);
      for (int p = 0; p < HH_NPLAN; ++p) {
        sd.phi_off[p] = po;
        if (p == 0 || wide) po += 2 * plan_phi_elems(sd.ns, P, sd.kl, map_dim(sd.KP), p);
      }
      if (!rec) img += strip_image_elems(sd.ns, S, sd.KP, sd.kl, P, wide);
      sd.piv_off = piv;
      if (!rec) piv += NP;
      sd.tr1_off = sd.has1 ? tr : -1;
      if (sd.has1) tr += 7LL * n;
      sd.tr2_off = sd.has2 ? tr : -1;
      if (sd.has2) tr += 7LL * n;
      fs.max_ns = std::max(fs.max_ns, sd.ns);
      fs.max_kl = std::max(fs.max_kl, sd.kl);
      fs.strips.push_back(sd);
    }
  }
  fs.nsub = rec ? nsub : 1;
  fs.first_sub = (int)fs.strips.size();
  fs.rho_elems = 2LL * fs.max_ns;  // the strip vector and the back substitution's scratch
  if (rec) sub_block_setup(fs, n, nsub, band, img, piv, tr);
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
    // the LU launch of recursive solves covers the sub-blocks only
    const int e = fs.h_err[0] - 1 + (fs.nsub > 1 ? fs.first_sub : 0);
    const StripDesc& sd = fs.strips[e];
    set_error("zero or non-finite pivot in the LU of strip %d of direction %c (in complex%d)", sd.s + 1,
              sd.dir == 0 ? 'x' : 'y', fs.precision == HH_FP64 ? 128 : 64);
    return HH_ESINGULAR;
  }
  return HH_OK;
}

void ensure_batch_maps(hh_problem* pb, hipStream_t st) {
  FactorSet& fs = pb->fs;
  if (fs.batch_maps) return;
  launch_transfer(fs, HH_BATCH_PLANS, st);
  launch_products(fs, HH_BATCH_PLANS, st);
  HH_HIP(hipStreamSynchronize(st));
  dev_free(fs.band);
  fs.band = nullptr;
  fs.batch_maps = true;
}

int sweep_plan_of(const hh_problem* pb, int nvec) {
  const FactorSet& fs = pb->fs;
  if (fs.nsub > 1) return HH_PLAN_REC;
  const int KP = fs.strips[0].KP, P = fs.strips[0].segs;
  const bool wide = fs.strips[0].wide != 0;
  int p = 0;
  if (!std::getenv("HH_SWEEP_PLAN") &&
      tune_lookup(TuneKey{fs.precision, KP, P, fs.max_kl, pb->n, fs.N, tune_bucket(nvec)}, p) &&
      sweep_plan_fits(p, nvec, fs.precision, KP, P, fs.max_kl, pb->n, fs.any_pivot, wide))
    return p;
  return sweep_plan_for(nvec, fs.precision, P, fs.max_kl, pb->n, fs.any_pivot, wide);
}

SweepBuffers sweep_layout(const hh_problem* pb, int nvec, int plan, char* base, size_t* total) {
  const FactorSet& fs = pb->fs;
  const size_t es = fs.precision == HH_FP64 ? sizeof(c128) : sizeof(c64);
  const size_t len = (size_t)pb->n * pb->n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  SweepBuffers b{};
  b.tasks = (SweepTask*)take((size_t)nvec * sizeof(SweepTask));
  b.sync = (unsigned*)take((size_t)(nvec + 1) * 128);  // [0] abort, then a line per chain
  b.rho = take((size_t)nvec * fs.rho_elems * es);
  b.g1 = take((size_t)nvec * fs.N * pb->n * es);
  b.zs = fs.precision == HH_FP64 ? nullptr : take((size_t)nvec * len * es);
  // the exchange areas of the forward and the back substitution
  b.xch = plan == HH_PLAN_WIDE || plan == HH_PLAN_PAIR
              ? take((size_t)nvec * plan_width(plan) * HH_XCH_BYTES_PER_WG)
              : nullptr;
  b.xch_bytes = b.xch ? (size_t)nvec * plan_width(plan) * HH_XCH_BYTES_PER_WG : 0;
  *total = off;
  return b;
}

void sweep_apply_core(hh_problem* pb, int i, int mode, int nvec, const c128* r, c128* z,
                      int plan, const SweepBuffers& b) {
  const FactorSet& fs = pb->fs;
  const long long len = (long long)pb->n * pb->n;
  const size_t es = fs.precision == HH_FP64 ? sizeof(c128) : sizeof(c64);
  void* zs = fs.precision == HH_FP64 ? (void*)z : b.zs;
  const int G = plan_width(plan);
  hipStream_t st = pb->st[0];
  if (plan != HH_PLAN_WIDE) ensure_batch_maps(pb, st);
  launch_zero(b.sync, (size_t)(nvec + 1) * 128, st);
  if (b.xch) launch_zero(b.xch, b.xch_bytes, st);  // no tail stamp is zero
  // descriptors staged on the stack for up to 64 chains (no host allocation)
  SweepTask few[64];
  std::vector<SweepTask> many(nvec > 64 ? nvec : 0);
  SweepTask* tasks = nvec > 64 ? many.data() : few;
  for (int v = 0; v < nvec; ++v) {
    SweepTask& tk = tasks[v];
    tk = SweepTask{};
    tk.ch.strips = fs.d_strips + (size_t)i * fs.N;
    tk.ch.r = r + v * len;
    tk.ch.z = (char*)zs + v * len * es;
    tk.ch.rho = (char*)b.rho + (size_t)v * fs.rho_elems * es;
    tk.ch.g1 = (char*)b.g1 + (size_t)v * fs.N * pb->n * es;
    tk.img = fs.img;
    tk.piv = fs.piv;
    tk.pflag = fs.d_pflag;
    tk.tr = fs.tr;
    tk.n = pb->n;
    tk.N = fs.N;
    tk.xch = b.xch ? (char*)b.xch + (size_t)v * G * HH_XCH_BYTES_PER_WG : nullptr;
    tk.bar = b.sync + 32 * (v + 1);
    tk.mode = mode;
  }
  // tiles of two vectors: consecutive pairs, a last single one repeated
  int nlaunch = nvec;
  if (plan == HH_PLAN_TILE) {
    nlaunch = (nvec + 1) / 2;
    for (int q = 0; q < nlaunch; ++q) {
      SweepTask tl = tasks[2 * q];
      tl.ch2 = tasks[2 * q + 1 < nvec ? 2 * q + 1 : 2 * q].ch;
      tasks[q] = tl;
    }
  }
  HH_HIP(hipMemcpyAsync(b.tasks, tasks, nlaunch * sizeof(SweepTask), hipMemcpyHostToDevice, st));
  {
    double bytes = 0;
    for (int q = 0; q < fs.N; ++q) {
      const StripDesc& sd = fs.strips[(size_t)i * fs.N + q];
      const double solves = mode != SWEEP_DOUBLE ? 1.0 : q == fs.N - 1 ? 1.0 : 2.0;
      bytes += solves * ((double)sd.nr * sd.ldab * es + nvec * (double)sd.nr * (sizeof(c128) + es));
    }
    TimedRegion tr(FAM_SWEEP, st, bytes);
    if (plan == HH_PLAN_TILE)
      launch_sweep_tiles(b.tasks, nlaunch, fs.precision, fs.strips[0].KP, fs.strips[0].segs,
                         pb->n, fs.any_pivot, st);
    else
      launch_sweep(b.tasks, nvec, fs.precision, fs.strips[0].KP, fs.strips[0].segs, fs.max_kl,
                   pb->n, fs.any_pivot, plan, b.sync, st);
  }
  if (fs.precision != HH_FP64) launch_widen((const c64*)zs, z, nvec * len, st);
  unsigned aborted = 0;
  HH_HIP(hipMemcpyAsync(&aborted, b.sync, sizeof(unsigned), hipMemcpyDeviceToHost, st));
  HH_HIP(hipStreamSynchronize(st));
  if (aborted) {
    set_error("sweep workgroups of one chain did not meet within the time limit");
    throw DeviceError();
  }
}

namespace {
// A problem handle with its streams (the caller's, if hh_set_streams gave
// any) and the operator storage; the caller fills the medium and assembles.
std::unique_ptr<hh_problem> problem_shell(double omega, int n) {
  REQUIRE(std::isfinite(omega) && omega > 0, "omega must be positive and finite");
  REQUIRE(n >= 3 && n <= 8193, "n must be in [3, 8193]");
  std::unique_ptr<hh_problem> pb(new hh_problem());
  pb->n = n;
  pb->omega = omega;
  HH_HIP(hipGetDevice(&pb->device));
  hipStream_t x = nullptr, y = nullptr;
  if (caller_streams(x, y)) {
    pb->own_streams = false;
    pb->st[0] = x ? x : y;
    pb->st[1] = y ? y : x;
  } else {
    HH_HIP(hipStreamCreate(&pb->st[0]));
    HH_HIP(hipStreamCreate(&pb->st[1]));
  }
  return pb;
}

void problem_assemble(hh_problem* pb) {
  const int n = pb->n;
  pb->d_A = (c128*)dev_alloc((size_t)4 * n * n * sizeof(c128));
  TimedRegion tr(FAM_ASSEMBLE, pb->st[0], (double)n * n * 64.0);
  launch_assemble(n, medium_of(pb), pb->d_A, pb->st[0]);
}
}  // namespace

// New problem handle with the operator assembled asynchronously on its stream.
hh_problem* problem_create(double omega, int nlayers, const double* c_layers, int n, int scheme) {
  REQUIRE(scheme == HH_SCHEME_P1 || scheme == HH_SCHEME_FD5, "unknown scheme %d", scheme);
  REQUIRE(nlayers >= 1 && c_layers != nullptr, "need at least one layer speed");
  for (int l = 0; l < nlayers; ++l)
    REQUIRE(std::isfinite(c_layers[l]) && c_layers[l] > 0, "layer speed %d is not positive", l);
  std::unique_ptr<hh_problem> pb = problem_shell(omega, n);
  pb->scheme = scheme;
  try {
    pb->c.assign(c_layers, c_layers + nlayers);
    pb->d_c = (double*)dev_alloc(nlayers * sizeof(double));
    HH_HIP(hipMemcpyAsync(pb->d_c, pb->c.data(), nlayers * sizeof(double), hipMemcpyHostToDevice,
                          pb->st[0]));
    problem_assemble(pb.get());
  } catch (...) {
    problem_destroy(pb.release());
    throw;
  }
  return pb.release();
}

// Wave numbers omega / c of a speed field sampled on the host at the triangle
// centroids and the edge midpoints (the layout of hh_problem::d_kt, d_kv, d_kh).
hh_problem* problem_create_field(double omega, double (*speed)(double, double, void*), void* ctx,
                                 int n, int scheme) {
  REQUIRE(speed != nullptr, "the speed field has no function");
  REQUIRE(scheme == HH_SCHEME_P1 || scheme == HH_SCHEME_FD5, "unknown scheme %d", scheme);
  REQUIRE(std::isfinite(omega) && omega > 0, "omega must be positive and finite");
  REQUIRE(n >= 3 && n <= 8193, "n must be in [3, 8193]");
  const double h = 1.0 / (n - 1);
  const long long m = n - 1;
  std::vector<double> kt(2 * m * m), kv((size_t)m * n), kh((size_t)m * n), kn((size_t)n * n);
  auto k_at = [&](double x, double y) {
    const double c = speed(x, y, ctx);
    REQUIRE(std::isfinite(c) && c > 0, "the speed field is not positive and finite at (%g, %g)", x, y);
    return omega / c;
  };
  for (long long cj = 0; cj < m; ++cj)
    for (long long ci = 0; ci < m; ++ci) {
      // lower {(i,j),(i+1,j),(i+1,j+1)} and upper {(i,j),(i+1,j+1),(i,j+1)}
      kt[2 * (cj * m + ci)] = k_at((3 * ci + 2) * h / 3.0, (3 * cj + 1) * h / 3.0);
      kt[2 * (cj * m + ci) + 1] = k_at((3 * ci + 1) * h / 3.0, (3 * cj + 2) * h / 3.0);
    }
  for (long long j = 0; j < m; ++j)
    for (long long i = 0; i < n; ++i) kv[j * n + i] = k_at(i * h, (j + 0.5) * h);
  for (long long j = 0; j < n; ++j)
    for (long long i = 0; i < m; ++i) kh[j * m + i] = k_at((i + 0.5) * h, j * h);
  for (long long j = 0; j < n; ++j)
    for (long long i = 0; i < n; ++i) kn[j * n + i] = k_at(i * h, j * h);
  std::unique_ptr<hh_problem> pb = problem_shell(omega, n);
  pb->scheme = scheme;
  try {
    pb->c.assign(1, 1.0);
    pb->d_kn = (double*)dev_alloc(kn.size() * sizeof(double));
    HH_HIP(hipMemcpyAsync(pb->d_kn, kn.data(), kn.size() * sizeof(double), hipMemcpyHostToDevice, pb->st[0]));
    pb->d_kt = (double*)dev_alloc(kt.size() * sizeof(double));
    pb->d_kv = (double*)dev_alloc(kv.size() * sizeof(double));
    pb->d_kh = (double*)dev_alloc(kh.size() * sizeof(double));
    HH_HIP(hipMemcpyAsync(pb->d_kt, kt.data(), kt.size() * sizeof(double), hipMemcpyHostToDevice, pb->st[0]));
    HH_HIP(hipMemcpyAsync(pb->d_kv, kv.data(), kv.size() * sizeof(double), hipMemcpyHostToDevice, pb->st[0]));
    HH_HIP(hipMemcpyAsync(pb->d_kh, kh.data(), kh.size() * sizeof(double), hipMemcpyHostToDevice, pb->st[0]));
    problem_assemble(pb.get());
    HH_HIP(hipStreamSynchronize(pb->st[0]));  // the host tables go out of scope
  } catch (...) {
    problem_destroy(pb.release());
    throw;
  }
  return pb.release();
}

void problem_destroy(hh_problem* pb) {
  if (!pb) return;
  for (hipStream_t s : pb->st)
    if (s) (void)hipStreamSynchronize(s);
  free_factors(pb->fs);
  dev_free(pb->d_A);
  dev_free(pb->d_c);
  dev_free(pb->d_kt);
  dev_free(pb->d_kv);
  dev_free(pb->d_kh);
  dev_free(pb->d_kn);
  dev_free(pb->d_b);
  if (pb->own_streams)
    for (hipStream_t s : pb->st)
      if (s) (void)hipStreamDestroy(s);
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

int hh_assemble_field(double omega, const hh_cfield* c, int n, const hh_c128* f,
                      hh_problem** out) {
  return guard([&]() {
    REQUIRE(out != nullptr && c != nullptr, "out or c is NULL");
    *out = nullptr;
    hh_problem* pb = c->speed ? problem_create_field(omega, c->speed, c->ctx, n, c->scheme)
                              : problem_create(omega, c->nlayers, c->c_layers, n, c->scheme);
    try {
      if (f) {
        pb->d_b = (c128*)dev_alloc((size_t)n * n * sizeof(c128));
        launch_load_vector(n, 1, (const c128*)f, pb->d_b, pb->st[0],
                           pb->scheme == HH_SCHEME_FD5);
      }
      HH_HIP(hipStreamSynchronize(pb->st[0]));
    } catch (...) {
      problem_destroy(pb);
      throw;
    }
    *out = pb;
    return HH_OK;
  });
}

int hh_set_allocator(void* (*alloc)(size_t bytes, void* ctx), void (*free_fn)(void* p, void* ctx),
                     void* ctx) {
  return guard([&]() {
    REQUIRE((alloc == nullptr) == (free_fn == nullptr), "give both functions or neither");
    REQUIRE(set_allocator(alloc, free_fn, ctx),
            "the library still holds device memory: free every problem and server first");
    return HH_OK;
  });
}

int hh_set_streams(void* x, void* y) {
  set_caller_streams((hipStream_t)x, (hipStream_t)y);
  return HH_OK;
}

int hh_autotune(int on) {
  tune_set_enabled(on != 0);
  return HH_OK;
}

int hh_tune_save(const char* path) {
  return guard([&]() {
    REQUIRE(path != nullptr, "path is NULL");
    REQUIRE(tune_save(path), "cannot write %s", path);
    return HH_OK;
  });
}

int hh_tune_load(const char* path) {
  return guard([&]() {
    REQUIRE(path != nullptr, "path is NULL");
    REQUIRE(tune_load(path), "cannot read tuning choices from %s", path);
    return HH_OK;
  });
}

int hh_tune_clear(void) {
  tune_clear();
  return HH_OK;
}

int hh_release_caches(void) {
  return guard([&]() {
    runtime_release_caches();
    return HH_OK;
  });
}

int hh_load_vector(hh_problem* pb, int nvec, const hh_c128* f, hh_c128* b) {
  return guard([&]() {
    REQUIRE(pb && f && b && nvec >= 0, "invalid arguments");
    launch_load_vector(pb->n, nvec, (const c128*)f, (c128*)b, pb->st[0],
                       pb->scheme == HH_SCHEME_FD5);
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

int hh_factor_sweeps_inner(hh_problem* pb, unsigned dirs, int nstrips, int nsub, int precision) {
  return guard([&]() {
    REQUIRE(pb != nullptr, "problem is NULL");
    REQUIRE(nsub >= 1, "nsub must be >= 1");
    factor_setup(pb, dirs, nstrips, precision, nsub);
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
    REQUIRE(pb->fs.nsub <= 1, "the strips of this factorisation are solved by inner sweeps");
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
    sweep_apply(pb, dir_slot(pb, dir), SWEEP_DOUBLE, nvec, (const c128*)r, (c128*)z);
    return HH_OK;
  });
}

int hh_precond_apply(hh_problem* pb, int kind, int nvec, const hh_c128* r, hh_c128* z) {
  return guard([&]() {
    REQUIRE(pb && r && z && nvec >= 0, "invalid arguments");
    int slot = 0, mode = 0;
    kind_slot(pb, kind, slot, mode);
    sweep_apply(pb, slot, mode, nvec, (const c128*)r, (c128*)z);
    return HH_OK;
  });
}

int hh_precond_apply_noalloc(hh_problem* pb, int kind, int nvec, const hh_c128* r, hh_c128* z) {
  return guard([&]() {
    REQUIRE(pb && r && z && nvec >= 0, "invalid arguments");
    int slot = 0, mode = 0;
    kind_slot(pb, kind, slot, mode);
    sweep_apply_noalloc(pb, slot, mode, nvec, (const c128*)r, (c128*)z);
    return HH_OK;
  });
}

int hh_set_preconditioners(hh_problem* pb, int t, const int* kinds) {
  return guard([&]() {
    REQUIRE(pb != nullptr && kinds != nullptr, "invalid arguments");
    REQUIRE(pb->fs.precision >= 0, "hh_factor_sweeps has not been called");
    REQUIRE(t >= 1 && t <= HH_MAXPRE, "t = %d preconditioners: between 1 and %d", t, HH_MAXPRE);
    int slot[HH_MAXPRE], mode[HH_MAXPRE];
    for (int i = 0; i < t; ++i) kind_slot(pb, kinds[i], slot[i], mode[i]);
    FactorSet& fs = pb->fs;
    fs.npre = t;
    for (int i = 0; i < t; ++i) {
      fs.pre_slot[i] = slot[i];
      fs.pre_mode[i] = mode[i];
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
  return hh_mpgmres_x0(pb, nrhs, b, nullptr, tol, maxit, x, stats);
}

int hh_mpgmres_x0(hh_problem* pb, int nrhs, const hh_c128* b, const hh_c128* x0, double tol,
                  int maxit, hh_c128* x, hh_stats* stats) {
  return guard([&]() {
    REQUIRE(pb && x && nrhs >= 0, "invalid arguments");
    if (!b) {
      REQUIRE(pb->d_b != nullptr && nrhs == 1,
              "b is NULL: only one right-hand side, given to hh_assemble_field, can be implied");
      b = (const hh_c128*)pb->d_b;
    }
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
      s.x0 = x0 ? (const c128*)x0 + r * len : nullptr;
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
    int bad = -1;
    for (int r = 0; r < nrhs; ++r) {
      Solve& s = solves[r];
      if (s.fail == HH_EINVAL && bad < 0) bad = r;
      if (!s.converged && rc == HH_OK) rc = HH_ENOCONV;
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
    if (bad >= 0) {
      set_error("right-hand side %d (or b - A x0) is not finite: no iteration was run for it", bad);
      return HH_EINVAL;
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
