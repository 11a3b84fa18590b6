// Batched selective MPGMRES (Sec. 3) with the Sec. 4 selection rule.
#include "engine.h"
#include "tune.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <tuple>
#include <type_traits>

namespace hh {

// ------------------------------------------------------------ least squares
void LeastSquares::init(double beta) {
  R_.clear();
  piv_.clear();
  rots_.clear();
  g_.assign(1, zd(beta, 0.0));
  rank_ = 0;
}

void LeastSquares::add_rows(int count) { g_.resize(g_.size() + count, zd(0.0, 0.0)); }

void LeastSquares::add_column(std::vector<zd> h) {
  h.resize(g_.size(), zd(0.0, 0.0));
  double nrm = 0;
  for (auto& v : h) nrm += std::norm(v);
  nrm = std::sqrt(nrm);
  for (const Rot& r : rots_) {
    zd a = h[r.i], b = h[r.k];
    h[r.i] = r.c * a + r.s * b;
    h[r.k] = -std::conj(r.s) * a + r.c * b;
  }
  const int pr = rank_;
  for (int row = pr + 1; row < (int)h.size(); ++row) {
    zd a = h[pr], b = h[row];
    if (b == zd(0.0, 0.0)) continue;
    Rot r;
    r.i = pr;
    r.k = row;
    double aa = std::abs(a), bb = std::abs(b);
    double rho = std::hypot(aa, bb);
    if (aa == 0.0) {
      r.c = 0.0;
      r.s = zd(1.0, 0.0);
    } else {
      r.c = aa / rho;
      r.s = (a / aa) * std::conj(b) / rho;
    }
    h[pr] = r.c * a + r.s * b;
    h[row] = zd(0.0, 0.0);
    zd ga = g_[pr], gb = g_[row];
    g_[pr] = r.c * ga + r.s * gb;
    g_[row] = -std::conj(r.s) * ga + r.c * gb;
    rots_.push_back(r);
  }
  if (pr < (int)h.size() && std::abs(h[pr]) > 1e-14 * nrm && nrm > 0) {
    piv_.push_back(pr);
    ++rank_;
  } else {
    piv_.push_back(-1);
  }
  R_.push_back(std::move(h));
}

double LeastSquares::residual() const {
  double s = 0;
  for (int i = rank_; i < (int)g_.size(); ++i) s += std::norm(g_[i]);
  return std::sqrt(s);
}

std::vector<zd> LeastSquares::solve() const {
  const int nc = (int)R_.size();
  std::vector<zd> y(nc, zd(0.0, 0.0));
  for (int j = nc - 1; j >= 0; --j) {
    const int pr = piv_[j];
    if (pr < 0) continue;
    zd acc = g_[pr];
    for (int jj = j + 1; jj < nc; ++jj)
      if (piv_[jj] >= 0) acc -= R_[jj][pr] * y[jj];
    y[j] = acc / R_[j][pr];
  }
  return y;
}

// ------------------------------------------------------------ layout
HdLayout::HdLayout(int m, int t) {
  size_t o = 0;
  g1 = o;
  o += (size_t)(m + t) * t;
  g2 = o;
  o += (size_t)m * t;
  r1 = o;
  o += (size_t)t * t;
  r2 = o;
  o += (size_t)t * t;
  rd = o;
  o += t;
  nr = o;
  o += t;
  total = o;
}

namespace {
size_t esz_of(int prec) { return prec == HH_FP64 ? sizeof(c128) : sizeof(c64); }
// Row blocks of the Gram products with nlive solves in the launch: about
// 512 rows each (two rows per thread) for up to eight solves, so that a
// single solve spreads over the chip, proportionally longer blocks for more
// (a batch fills the chip with its solves); at most 256 blocks.  nblk_for(len)
// (nlive = 1) sizes the partial-sum buffers.
int nblk_for(long long len, size_t nlive = 1) {
  const long long rows = 512LL * (long long)std::max<size_t>(1, nlive / 8);
  const long long b = (len + rows - 1) / rows;
  return (int)std::max(1LL, std::min(b, 256LL));
}
}  // namespace

void PinnedBuf::reserve(size_t n, bool keep) {
  if (n <= cap) return;
  const size_t nc = std::max<size_t>(n * 2, 4096);
  void* q = nullptr;
  HH_HIP(hipHostMalloc(&q, nc, hipHostMallocDefault));
  if (keep && p) std::memcpy(q, p, cap);
  if (p) {
    HH_HIP(hipDeviceSynchronize());  // no copy may still use the old buffer (grows are rare)
    HH_HIP(hipHostFree(p));
  }
  p = (unsigned char*)q;
  cap = nc;
}
PinnedBuf::~PinnedBuf() {
  if (p) (void)hipHostFree(p);
}

Engine::Engine(hipStream_t st) : st_(st) {}
Engine::~Engine() {
  if (task_dev_) dev_free(task_dev_);
  if (sync_) dev_free(sync_);
  if (xch_) dev_free(xch_);
  if (ones_) dev_free(ones_);
  if (dl_dev_) dev_free(dl_dev_);
}

template <class TT>
TT* Engine::stage(const std::vector<TT>& v, size_t& off) {
  size_t bytes = (v.size() * sizeof(TT) + 255) & ~size_t(255);
  task_host_.reserve(off + bytes, true);
  std::memcpy(task_host_.p + off, v.data(), v.size() * sizeof(TT));
  TT* d = reinterpret_cast<TT*>(off);  // resolved in upload()
  off += bytes;
  return d;
}

// Makes the device area hold the staged bytes (its address is final from
// here until the next stage() beyond it).
void Engine::reserve_dev() {
  task_host_.reserve(staged_, true);
  if (staged_ > task_cap_) {
    HH_HIP(hipStreamSynchronize(st_));
    if (task_dev_) dev_free(task_dev_);
    task_cap_ = staged_ * 2;
    task_dev_ = dev_alloc(task_cap_);
  }
}

// Copies the staged host descriptors to the device in one transfer.
void Engine::upload() {
  reserve_dev();
  if (staged_) HH_HIP(hipMemcpyAsync(task_dev_, task_host_.p, staged_, hipMemcpyHostToDevice, st_));
}

// Makes the device area hold dl bytes of gathered results (and the pinned
// host area as many).
void Engine::reserve_dl(size_t dl) {
  if (dl > dl_dev_cap_) {
    HH_HIP(hipStreamSynchronize(st_));
    if (dl_dev_) dev_free(dl_dev_);
    dl_dev_ = nullptr;
    dl_dev_cap_ = 0;
    dl_dev_ = static_cast<unsigned char*>(dev_alloc(dl * 2));
    dl_dev_cap_ = dl * 2;
  }
  dl_host_.reserve(dl, false);
}

#define DEV(ptr) reinterpret_cast<std::remove_reference_t<decltype(ptr)>>((char*)task_dev_ + (size_t)(ptr))

size_t Engine::footprint(const hh_problem* pb, int t, int prec, int maxit) {
  const long long len = (long long)pb->n * pb->n;
  const int cols = 1 + (maxit + 1) * t;
  size_t b = (size_t)len * cols * sizeof(c128);                  // V
  b += (size_t)len * (size_t)maxit * t * esz_of(prec);           // Z
  HdLayout L(cols, t);
  b += L.total * sizeof(c128);
  b += (size_t)nblk_for(len) * (cols + t) * t * sizeof(c128);    // partial sums
  b += (size_t)t * (pb->fs.rho_elems + (size_t)pb->fs.N * pb->n) * esz_of(prec);
  if (t > 2) b += (size_t)len * sizeof(c128);                    // summed sweep input
  return b;
}

void Engine::release(Solve* s) {
  dev_free(s->V);
  dev_free(s->Z);
  dev_free(s->Hd);
  dev_free(s->part);
  dev_free(s->flags);
  dev_free(s->rho);
  dev_free(s->g1);
  dev_free(s->sumv);
  s->sumv = nullptr;
  s->V = nullptr;
  s->Z = nullptr;
  s->Hd = nullptr;
  s->part = nullptr;
  s->flags = nullptr;
  s->rho = s->g1 = nullptr;
}

size_t Engine::iteration_bytes(const Solve* s) {
  return (size_t)s->len * s->t * (sizeof(c128) + esz_of(s->prec));
}

struct GrowRefused {};

// Grows V, Z and the coefficient scratch so that the next iteration fits.
void Engine::ensure_capacity(Solve* s) {
  const int t = s->t;
  const size_t es = esz_of(s->prec);
  const int need_v = s->m + t, need_z = (s->k + 1) * t;
  if (need_v > s->vcap || need_z > s->zcap) {
    int it_cap = std::max(16, 2 * (s->k + 1));
    it_cap = std::min(it_cap, s->maxit);
    it_cap = std::max(it_cap, s->k + 1);
    int vcap = 1 + it_cap * t, zcap = it_cap * t;
    // budget: iterations beyond the charged ones, and while the old bases are
    // copied, the old bases a second time
    const long long old_bytes =
        s->V ? (long long)(s->len * s->vcap * sizeof(c128) + s->len * s->zcap * es) : 0;
    const long long extra =
        it_cap > s->charged_its ? (long long)(it_cap - s->charged_its) * (long long)iteration_bytes(s) : 0;
    if (grow_ && (extra > 0 || old_bytes > 0)) {
      if (!grow_(s, extra + old_bytes)) throw GrowRefused();
    }
    c128* V = nullptr;
    void* Z = nullptr;
    try {
      V = (c128*)dev_alloc((size_t)s->len * vcap * sizeof(c128));
      Z = dev_alloc((size_t)s->len * zcap * es);
    } catch (...) {
      dev_free(V);
      if (grow_ && (extra > 0 || old_bytes > 0)) grow_(s, -(extra + old_bytes));
      throw;
    }
    s->charged_its = std::max(s->charged_its, it_cap);
    if (s->V) {
      HH_HIP(hipMemcpyAsync(V, s->V, (size_t)s->len * s->m * sizeof(c128), hipMemcpyDeviceToDevice, st_));
      HH_HIP(hipMemcpyAsync(Z, s->Z, (size_t)s->len * s->k * t * es, hipMemcpyDeviceToDevice, st_));
      HH_HIP(hipStreamSynchronize(st_));
      dev_free(s->V);
      dev_free(s->Z);
    }
    if (grow_ && old_bytes > 0) grow_(s, -old_bytes);
    s->V = V;
    s->Z = Z;
    s->vcap = vcap;
    s->zcap = zcap;
  }
  if (s->m + t > s->hcap || !s->Hd) {
    if (s->Hd) dev_free(s->Hd);
    if (s->part) dev_free(s->part);
    s->hcap = s->vcap;
    HdLayout L(s->hcap, t);
    s->Hd = (c128*)dev_alloc(L.total * sizeof(c128));
    s->part_elems = (size_t)nblk_for(s->len) * (s->hcap + t) * t;
    s->part = (c128*)dev_alloc(s->part_elems * sizeof(c128));
  }
}

void Engine::ensure_all(std::vector<Solve*>& solves) {
  for (Solve* s : solves) {
    if (s->done) continue;
    try {
      ensure_capacity(s);
    } catch (const GrowRefused&) {
      set_error("a solve's Krylov bases would exceed the HBM budget");
      s->fail = HH_EBUDGET;
      s->done = true;
    } catch (const MemError&) {
      s->fail = HH_ENOMEM;
      s->done = true;
    }
  }
}

// ------------------------------------------------------------ begin
void Engine::begin(std::vector<Solve*>& solves) {
  std::vector<Solve*> live;
  for (Solve* s : solves) {
    s->k = 0;
    s->m = 1;
    s->done = s->converged = s->breakdown = s->finalized = false;
    s->deflated = 0;
    s->fail = 0;
    const FactorSet& fs = s->pb->fs;
    s->t = fs.npre;
    s->prec = fs.precision;
    s->sum_input = false;
    const size_t es = esz_of(s->prec);
    ensure_capacity(s);  // the first bases fit the iterations charged at admission
    if (!s->flags) s->flags = (int*)dev_alloc(4 * sizeof(int));
    if (!s->rho) s->rho = dev_alloc((size_t)s->t * fs.rho_elems * es + 256);
    if (!s->g1) s->g1 = dev_alloc((size_t)s->t * fs.N * s->pb->n * es + 256);
    if (s->t > 2 && !s->sumv) s->sumv = (c128*)dev_alloc((size_t)s->len * sizeof(c128));
    live.push_back(s);
  }
  if (live.empty()) return;
  if (sync_) HH_HIP(hipMemsetAsync(sync_, 0, sizeof(unsigned), st_));  // clear a past abort
  staged_ = 256;  // offset 0 is reserved so that no staged array aliases nullptr
  long long maxlen = 0;
  int maxblk = 1;
  // with a starting guess: v1 = b - A x0 and ||b||^2 into the (still unused) G1 slot
  std::vector<SpmvTask> sp0;
  std::vector<ResTask> rt0;
  std::vector<GramTask> gb;
  for (Solve* s : live) {
    maxlen = std::max(maxlen, s->len);
    if (!s->x0) continue;
    SpmvTask tk{};
    tk.A = s->pb->d_A;
    tk.x = s->x0;
    tk.y = s->V;
    tk.n = s->pb->n;
    tk.nvec = 1;
    sp0.push_back(tk);
    rt0.push_back(ResTask{s->b, s->V, s->len});
    HdLayout L(s->hcap, s->t);
    GramTask g{};
    g.X = s->b;
    g.Y = s->b;
    g.out = s->Hd + L.g1;
    g.part = s->part;
    g.len = s->len;
    g.ldx = g.ldy = s->len;
    g.ldo = 1;
    g.px = 1;
    g.ty = 1;
    g.nblk = nblk_for(s->len, live.size());
    maxblk = std::max(maxblk, g.nblk);
    gb.push_back(g);
  }
  if (!sp0.empty()) {
    SpmvTask* dsp = stage(sp0, staged_);
    ResTask* drt = stage(rt0, staged_);
    GramTask* dgb = stage(gb, staged_);
    upload();
    launch_spmv(DEV(dsp), (int)sp0.size(), maxlen, HH_FP64, st_);
    launch_residual(DEV(drt), (int)rt0.size(), maxlen, st_);
    launch_gram(DEV(dgb), (int)gb.size(), maxblk, 1, 1, st_);
    staged_ = 256;
  }
  // beta^2 = r0^H r0 into NR slot 0, then v1 = r0 / beta, with r0 = b (read
  // in place) or b - A x0 (formed in v1's column above)
  std::vector<GramTask> gt;
  std::vector<NormTask> nt;
  for (Solve* s : live) {
    HdLayout L(s->hcap, s->t);
    const c128* r0 = s->x0 ? s->V : s->b;
    GramTask g{};
    g.X = r0;
    g.Y = r0;
    g.out = s->Hd + L.nr;
    g.part = s->part;
    g.len = s->len;
    g.ldx = g.ldy = s->len;
    g.ldo = 1;
    g.px = 1;
    g.ty = 1;
    g.nblk = nblk_for(s->len, live.size());
    g.accumulate = 0;
    gt.push_back(g);
    NormTask q{};
    q.y = s->V;
    q.x = r0;
    q.nrm2 = s->Hd + L.nr;
    q.ref2 = s->Hd + L.nr;
    q.rdiag = s->Hd + L.rd;
    q.flag = s->flags;
    q.len = s->len;
    q.tol = 0.0;
    nt.push_back(q);
    maxlen = std::max(maxlen, s->len);
    maxblk = std::max(maxblk, g.nblk);
  }
  GramTask* dg = stage(gt, staged_);
  NormTask* dn = stage(nt, staged_);
  // per solve beta, its square and ||b||^2 to the host in one transfer
  std::vector<CopyTask> dlt;
  constexpr long long zw = sizeof(zd) / 4;
  for (size_t q = 0; q < live.size(); ++q) {
    const Solve* s = live[q];
    HdLayout L(s->hcap, s->t);
    const long long o = (long long)(q * 3 * sizeof(zd));
    dlt.push_back({s->Hd + L.rd, o, zw});
    dlt.push_back({s->Hd + L.nr, o + (long long)sizeof(zd), zw});
    if (s->x0) dlt.push_back({s->Hd + L.g1, o + 2 * (long long)sizeof(zd), zw});
  }
  CopyTask* ddl = stage(dlt, staged_);
  const size_t dl = live.size() * 3 * sizeof(zd);
  reserve_dl(dl);
  upload();
  launch_gram(DEV(dg), (int)gt.size(), maxblk, 1, 1, st_);
  launch_normalize(DEV(dn), (int)nt.size(), maxlen, st_);
  launch_gather(DEV(ddl), (int)dlt.size(), dl_dev_, st_);
  HH_HIP(hipMemcpyAsync(dl_host_.p, dl_dev_, dl, hipMemcpyDeviceToHost, st_));
  HH_HIP(hipStreamSynchronize(st_));
  for (size_t q = 0; q < live.size(); ++q) {
    Solve* s = live[q];
    zd r[3];
    std::memcpy(r, dl_host_.p + q * 3 * sizeof(zd), sizeof(r));
    const double v = r[0].real(), v2 = r[1].real(), bb = s->x0 ? r[2].real() : 0.0;
    // the normalisation deflates a NaN norm to zero: the raw square tells
    s->beta = std::isfinite(v2) ? v : v2;
    s->bnorm = s->x0 ? (std::isfinite(bb) ? std::sqrt(std::max(0.0, bb)) : bb) : s->beta;
  }
  for (Solve* s : live) {
    s->ls.init(s->beta);
    for (int i = 0; i < s->t; ++i) s->inputs[i] = 0;
    s->res_est = 1.0;
    if (!std::isfinite(s->beta) || !std::isfinite(s->bnorm)) {
      // a NaN or Inf in b (or in A x0): no iteration; x = 0 or x0
      s->done = true;
      s->fail = HH_EINVAL;
      s->res_est = std::numeric_limits<double>::quiet_NaN();
    } else if (s->bnorm == 0.0) {
      s->done = true;  // b = 0: x = 0 whatever x0
      s->converged = true;
      s->res_est = 0.0;
      s->x0 = nullptr;
    } else if (s->beta <= s->tol * s->bnorm) {
      s->done = true;  // x0 (or x = 0 when tol >= 1) already meets the tolerance
      s->converged = true;
      s->res_est = s->beta / s->bnorm;
    }
  }
}

// ------------------------------------------------------------ step
void Engine::step(std::vector<Solve*>& solves) {
  ensure_all(solves);
  std::vector<Solve*> live;
  for (Solve* s : solves)
    if (!s->done) live.push_back(s);
  if (live.empty()) return;
  staged_ = 256;  // offset 0 is reserved so that no staged array aliases nullptr

  // 1. sweeps: every preconditioner of every solve, one chain each.  Launch
  // kinds are keyed by (precision, blocked term count KP, segments P, presence
  // of pivoted strips); each kind then takes its segment plan.
  struct Kind {
    std::vector<SweepTask> tasks;
    int prec, KP, P, kmax, nmax;
    bool piv;
    int plan;
    bool wide;  // the maps of plans 1 and 2 exist
    bool rec = false;              // recursive strip solves (k_sweep_rec)
    std::vector<hh_problem*> pbs;  // problems with tasks in this kind
    bool tune = false;             // measure the plans that fit before the launch
    TuneKey key{};
  };
  std::vector<Kind> kinds;
  for (Solve* s : live) {
    const hh_problem* pb = s->pb;
    const FactorSet& fs = pb->fs;
    const size_t es = esz_of(fs.precision);
    const int KP = fs.strips[0].KP, P = fs.strips[0].segs;
    const bool wide = fs.strips[0].wide != 0;
    const bool rec = fs.nsub > 1;
    auto it = std::find_if(kinds.begin(), kinds.end(), [&](const Kind& k) {
      return k.prec == fs.precision && k.KP == KP && k.P == P && k.piv == fs.any_pivot &&
             k.wide == wide && k.rec == rec;
    });
    if (it == kinds.end()) {
      kinds.push_back({{}, fs.precision, KP, P, 0, 0, fs.any_pivot, 0, wide, rec, {}});
      it = kinds.end() - 1;
    }
    if (std::find(it->pbs.begin(), it->pbs.end(), s->pb) == it->pbs.end()) it->pbs.push_back(s->pb);
    it->kmax = std::max(it->kmax, fs.max_kl);
    it->nmax = std::max(it->nmax, pb->n);
    for (int i = 0; i < s->t; ++i) {
      SweepTask tk{};
      tk.ch.strips = fs.d_strips + (size_t)fs.pre_slot[i] * fs.N;
      tk.mode = fs.pre_mode[i];
      tk.ch.r = s->sum_input ? s->sumv : s->V + (size_t)s->inputs[i] * s->len;
      tk.ch.z = (char*)s->Z + ((size_t)s->k * s->t + i) * s->len * es;
      tk.ch.rho = (char*)s->rho + (size_t)i * fs.rho_elems * es;
      tk.ch.g1 = (char*)s->g1 + (size_t)i * fs.N * pb->n * es;
      tk.img = fs.img;
      tk.piv = fs.piv;
      tk.pflag = fs.d_pflag;
      tk.tr = fs.tr;
      tk.n = pb->n;
      tk.N = fs.N;
      it->tasks.push_back(tk);
    }
  }
  size_t wide_chains = 0;
  {
    size_t chains = 0, xbytes = 0;
    for (Kind& k : kinds) {
      const int nt = (int)k.tasks.size();
      k.plan = 0;
      k.tune = false;
      if (k.rec) {
        k.plan = HH_PLAN_REC;
        continue;
      }
      if (!wide_ok_) {
        // plan 0's results whatever the mix: plan 0, or its tiles (the same
        // bits) when the chains outnumber the compute units
        const int p = sweep_plan_for(nt, k.prec, k.P, k.kmax, k.nmax, k.piv, false);
        k.plan = p == HH_PLAN_TILE ? p : 0;
      } else {
        k.key = TuneKey{k.prec, k.KP, k.P, k.kmax, k.nmax, k.pbs[0]->fs.N, tune_bucket(nt)};
        int p = 0;
        if (!std::getenv("HH_SWEEP_PLAN") && tune_lookup(k.key, p) &&
            sweep_plan_fits(p, nt, k.prec, k.KP, k.P, k.kmax, k.nmax, k.piv, k.wide)) {
          k.plan = p;
        } else {
          k.plan = sweep_plan_for(nt, k.prec, k.P, k.kmax, k.nmax, k.piv, k.wide);
          k.tune = !std::getenv("HH_SWEEP_PLAN") && tune_enabled() && !k.piv &&
                   ((k.wide && sweep_wide_fits(k.prec, k.P, k.kmax, k.nmax)) ||
                    sweep_plan_fits(HH_PLAN_TILE, nt, k.prec, k.KP, k.P, k.kmax, k.nmax, k.piv,
                                    true));
        }
      }
      if (k.plan != HH_PLAN_WIDE || k.tune)
        for (hh_problem* q : k.pbs) ensure_batch_maps(q, st_);
      if ((k.plan == 0 || k.plan == HH_PLAN_TILE) && !k.tune) continue;
      chains += k.tasks.size();
      // a tuned kind may run any plan: room for the widest
      xbytes += k.tasks.size() * (size_t)plan_width(k.tune ? HH_PLAN_WIDE : k.plan) *
                HH_XCH_BYTES_PER_WG;
    }
    if (chains > 0) {
      const size_t sbytes = (chains + 1) * 128;
      if (sbytes > sync_cap_) {
        HH_HIP(hipStreamSynchronize(st_));
        if (sync_) dev_free(sync_);
        sync_cap_ = sbytes * 2;
        sync_ = (unsigned*)dev_alloc(sync_cap_);
        HH_HIP(hipMemsetAsync(sync_, 0, sync_cap_, st_));
        sync_clear_ = sync_cap_ / 128 - 1;
      }
      if (xbytes > xch_cap_) {
        HH_HIP(hipStreamSynchronize(st_));
        if (xch_) dev_free(xch_);
        xch_cap_ = xbytes * 2;
        xch_ = dev_alloc(xch_cap_);
        launch_zero(xch_, xch_cap_, st_);  // no tail stamp is zero
      }
      // arrival counters start from zero in every launch; normally the
      // previous launch's lines were cleared behind it (below)
      if (chains > sync_clear_) HH_HIP(hipMemsetAsync(sync_ + 32, 0, chains * 128, st_));
      sync_clear_ = 0;
      wide_chains = chains;
      size_t ci = 0, xo = 0;
      for (Kind& k : kinds) {
        if ((k.plan == 0 || k.plan == HH_PLAN_TILE || k.plan == HH_PLAN_REC) && !k.tune) continue;
        for (SweepTask& tk : k.tasks) {
          tk.bar = sync_ + 32 * (1 + ci++);
          tk.xch = (char*)xch_ + xo;
          xo += (size_t)plan_width(k.tune ? HH_PLAN_WIDE : k.plan) * HH_XCH_BYTES_PER_WG;
        }
      }
    }
  }
  // tiles of two right-hand sides (choice HH_PLAN_TILE): tasks of the same
  // strips, image and sweep mode in pairs, a last single one repeated
  std::vector<std::vector<SweepTask>> tiles(kinds.size());
  for (size_t q = 0; q < kinds.size(); ++q) {
    Kind& k = kinds[q];
    if (k.plan != HH_PLAN_TILE && !k.tune) continue;
    std::vector<int> order(k.tasks.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      const SweepTask &x = k.tasks[a], &y = k.tasks[b];
      return std::make_tuple((uintptr_t)x.ch.strips, x.mode) <
             std::make_tuple((uintptr_t)y.ch.strips, y.mode);
    });
    for (size_t i = 0; i < order.size();) {
      SweepTask tl = k.tasks[order[i]];
      const bool pair = i + 1 < order.size() &&
                        k.tasks[order[i + 1]].ch.strips == tl.ch.strips &&
                        k.tasks[order[i + 1]].mode == tl.mode;
      tl.ch2 = pair ? k.tasks[order[i + 1]].ch : tl.ch;
      tiles[q].push_back(tl);
      i += pair ? 2 : 1;
    }
    // a rule-based choice of tiles needs pairs: with few of them the repeated
    // singles would cost more than plan 0's second round
    if (k.plan == HH_PLAN_TILE && !k.tune && tiles[q].size() * 4 > k.tasks.size() * 3) {
      k.plan = 0;
      tiles[q].clear();
    }
  }
  std::vector<SweepTask*> dsw(kinds.size()), dtl(kinds.size(), nullptr);
  for (size_t q = 0; q < kinds.size(); ++q) {
    dsw[q] = stage(kinds[q].tasks, staged_);
    if (!tiles[q].empty()) dtl[q] = stage(tiles[q], staged_);
  }
  // one launch of kind q with choice c (a segment plan, or tiles)
  auto launch_kind = [&](size_t q, int c) {
    const Kind& k = kinds[q];
    if (c == HH_PLAN_TILE)
      launch_sweep_tiles(DEV(dtl[q]), (int)tiles[q].size(), k.prec, k.KP, k.P, k.nmax, k.piv, st_);
    else
      launch_sweep(DEV(dsw[q]), (int)k.tasks.size(), k.prec, k.KP, k.P, k.kmax, k.nmax, k.piv, c,
                   sync_, st_);
  };

  // 0. t > 2 (sum rule): the sweeps' input is the sum of the previous
  // iteration's t new basis vectors (deflated ones are zero)
  std::vector<CombTask> sums;
  long long sumlen = 0;
  for (Solve* s : live) {
    if (!s->sum_input) continue;
    CombTask c{};
    c.Z = s->V + (size_t)(s->m - s->t) * s->len;
    c.y = nullptr;  // the staged ones, below
    c.x = s->sumv;
    c.len = s->len;
    c.ncols = s->t;
    sums.push_back(c);
    sumlen = std::max(sumlen, s->len);
  }
  CombTask* dsums = nullptr;
  if (!sums.empty()) {
    if (!ones_) {
      ones_ = (c128*)dev_alloc(HH_MAXPRE * sizeof(c128));
      const std::vector<c128> h(HH_MAXPRE, mk(1.0, 0.0));
      HH_HIP(hipMemcpyAsync(ones_, h.data(), HH_MAXPRE * sizeof(c128), hipMemcpyHostToDevice, st_));
      HH_HIP(hipStreamSynchronize(st_));
    }
    for (CombTask& c : sums) c.y = ones_;
    dsums = stage(sums, staged_);
  }

  // 2. SpMV: W = A Z_k into the basis slots m..m+t-1
  std::vector<SpmvTask> sp[2];
  long long maxlen = 0;
  for (Solve* s : live) {
    SpmvTask tk{};
    tk.A = s->pb->d_A;
    tk.x = (char*)s->Z + (size_t)s->k * s->t * s->len * esz_of(s->prec);
    tk.y = s->V + (size_t)s->m * s->len;
    tk.n = s->pb->n;
    tk.nvec = s->t;
    sp[s->prec == HH_FP64 ? 0 : 1].push_back(tk);
    maxlen = std::max(maxlen, s->len);
  }
  SpmvTask* dsp[2];
  for (int a = 0; a < 2; ++a) dsp[a] = sp[a].empty() ? nullptr : stage(sp[a], staged_);

  // 3-6. two passes of block CGS against the basis
  std::vector<GramTask> g1, g2;
  std::vector<UpdTask> u1, u2;
  int maxblk = 1, maxpx = 1, maxt = 1;
  for (Solve* s : live) {
    HdLayout L(s->hcap, s->t);
    const int m = s->m, t = s->t;
    c128* W = s->V + (size_t)m * s->len;
    GramTask g{};
    g.X = s->V;
    g.Y = W;
    g.out = s->Hd + L.g1;
    g.part = s->part;
    g.len = s->len;
    g.ldx = g.ldy = s->len;
    g.ldo = m + t;
    g.px = m + t;
    g.ty = t;
    g.nblk = nblk_for(s->len, live.size());
    g.accumulate = 0;
    g1.push_back(g);
    g.px = m;
    g.ldo = m;
    g.out = s->Hd + L.g2;
    g2.push_back(g);
    UpdTask u{};
    u.X = s->V;
    u.Y = W;
    u.C = s->Hd + L.g1;
    u.len = s->len;
    u.ldx = u.ldy = s->len;
    u.ldc = m + t;
    u.px = m;
    u.ty = t;
    u1.push_back(u);
    u.C = s->Hd + L.g2;
    u.ldc = m;
    u2.push_back(u);
    maxblk = std::max(maxblk, g.nblk);
    maxpx = std::max(maxpx, m + t);
    maxt = std::max(maxt, t);
  }
  GramTask* dg1 = stage(g1, staged_);
  UpdTask* du1 = stage(u1, staged_);
  GramTask* dg2 = stage(g2, staged_);
  UpdTask* du2 = stage(u2, staged_);

  // 7. QR of the new block: modified Gram-Schmidt with two passes per column,
  // then normalisation, in fused steps (k_qr_step; bitwise the separate
  // kernels): the first column's norm; per column c the step that normalises
  // it and forms the first pass's products of column c + 1, then that pass's
  // update with the second pass's products, then the second update with the
  // norm of c + 1.  A solve of t columns takes 3t - 1 steps; step k of every
  // solve is one launch.  Consecutive steps use two halves of the partial
  // sums' scratch, since a step reads its predecessor's while writing its own.
  std::vector<std::vector<QrTask>> qs(3 * HH_MAXPRE - 1);
  int maxqblk = 1;
  for (Solve* s : live) {
    HdLayout L(s->hcap, s->t);
    const int m = s->m, t = s->t, nb = nblk_for(s->len, live.size());
    maxqblk = std::max(maxqblk, nb);
    c128* W = s->V + (size_t)m * s->len;
    auto col = [&](int c) { return W + (size_t)c * s->len; };
    auto step = [&]() {
      QrTask q{};
      q.len = s->len;
      q.ld = s->len;
      q.nblk = nb;
      q.cnblk = nb;
      q.xg_is_y = -1;
      q.tol = 1e-12;
      return q;
    };
    std::vector<QrTask> chain;
    QrTask q = step();
    q.Xg = col(0);
    q.gy = col(0);
    q.gpx = 1;
    chain.push_back(q);
    for (int c = 0; c < t; ++c) {
      q = step();  // normalise c; the first pass's products of c + 1
      q.cpx = 1;
      q.cout = s->Hd + L.nr + c;
      q.op = QR_NORMALIZE;
      q.y = col(c);
      q.ref2 = s->Hd + L.g1 + (size_t)(m + c) + (size_t)c * (m + t);  // ||A z_c||^2
      q.rdiag = s->Hd + L.rd + c;
      q.flag = s->flags + c;
      if (c + 1 < t) {
        q.Xg = W;
        q.gy = col(c + 1);
        q.gpx = c + 1;
        q.xg_is_y = c;
      }
      chain.push_back(q);
      if (c + 1 == t) break;
      for (int pass = 0; pass < 2; ++pass) {
        q = step();  // the pass's update of c + 1; the next pass's products or its norm
        q.cpx = c + 1;
        q.cout = s->Hd + (pass == 0 ? L.r1 : L.r2) + (size_t)(c + 1) * t;
        q.op = QR_UPDATE;
        q.y = col(c + 1);
        q.Xop = W;
        q.Xg = pass == 0 ? W : col(c + 1);
        q.gy = col(c + 1);
        q.gpx = pass == 0 ? c + 1 : 1;
        q.xg_is_y = pass == 0 ? -1 : 0;
        q.gy_is_y = 1;
        chain.push_back(q);
      }
    }
    for (size_t k = 0; k < chain.size(); ++k) {
      chain[k].gpart = s->part + (k % 2) * (size_t)nb * 4;
      chain[k].cpart = s->part + ((k + 1) % 2) * (size_t)nb * 4;
      qs[k].push_back(chain[k]);
    }
  }
  std::vector<QrTask*> dqs(qs.size(), nullptr);
  for (size_t k = 0; k < qs.size(); ++k)
    if (!qs[k].empty()) dqs[k] = stage(qs[k], staged_);
  // the iteration's results for the host, gathered into one device area and
  // sent in one transfer: per solve its coefficients and flags, then the
  // abort word
  std::vector<size_t> hoff(live.size()), foff(live.size());
  std::vector<CopyTask> dlt;
  size_t dl = 0;
  for (size_t q = 0; q < live.size(); ++q) {
    Solve* s = live[q];
    const size_t hb = HdLayout(s->hcap, s->t).total * sizeof(c128);
    hoff[q] = dl;
    dlt.push_back({s->Hd, (long long)dl, (long long)(hb / 4)});
    dl += hb;
    foff[q] = dl;
    dlt.push_back({s->flags, (long long)dl, (long long)s->t});
    dl += (s->t * sizeof(int) + 15) & ~size_t(15);
  }
  const size_t aoff = dl;
  if (sync_) dlt.push_back({sync_, (long long)aoff, 1});
  dl += sizeof(unsigned);
  CopyTask* ddl = stage(dlt, staged_);
  reserve_dl(dl);
  upload();

  // ---- launches
  if (dsums) launch_combine(DEV(dsums), (int)sums.size(), sumlen, HH_FP64, st_);
  // first launch of a shape with tuning on: time every plan that fits (best of
  // two launches each, arrival counters cleared before each), keep the
  // fastest; the launch below then writes the outputs with it
  for (size_t q = 0; q < kinds.size(); ++q) {
    Kind& k = kinds[q];
    if (!k.tune) continue;
    const int nt = (int)k.tasks.size();
    TuneEntry best;
    double best_ms = -1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HH_HIP(hipEventCreate(&e0));
    HH_HIP(hipEventCreate(&e1));
    for (int p = 0; p < HH_NCHOICE; ++p) {
      if (!sweep_plan_fits(p, nt, k.prec, k.KP, k.P, k.kmax, k.nmax, k.piv, true)) continue;
      double ms_best = -1;
      for (int rep = 0; rep < 2; ++rep) {
        if (wide_chains) launch_zero(sync_ + 32, wide_chains * 128, st_);
        HH_HIP(hipEventRecord(e0, st_));
        launch_kind(q, p);
        HH_HIP(hipEventRecord(e1, st_));
        HH_HIP(hipEventSynchronize(e1));
        float ms = 0;
        HH_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms_best < 0 || ms < ms_best) ms_best = ms;
      }
      best.ms[p] = ms_best;
      if (best_ms < 0 || ms_best < best_ms) {
        best_ms = ms_best;
        best.plan = p;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    k.plan = best.plan;
    tune_store(k.key, best);
    if (wide_chains) launch_zero(sync_ + 32, wide_chains * 128, st_);
    sync_clear_ = wide_chains;
  }
  {
    // algorithmic bytes: each (problem, direction) factor read once per strip
    // solve of the launch, plus FP64 input and sweep-precision output per task
    double bytes = 0;
    std::vector<const hh_problem*> seen;
    for (Solve* s : live) {
      const FactorSet& fs = s->pb->fs;
      const size_t es = esz_of(s->prec);
      const bool first = std::find(seen.begin(), seen.end(), s->pb) == seen.end();
      if (first) seen.push_back(s->pb);
      for (int i = 0; i < s->t; ++i)
        for (int q = 0; q < fs.N; ++q) {
          const StripDesc& sd = fs.strips[(size_t)fs.pre_slot[i] * fs.N + q];
          const double solves = fs.pre_mode[i] != SWEEP_DOUBLE ? 1.0 : q == fs.N - 1 ? 1.0 : 2.0;
          if (first) bytes += solves * (double)sd.nr * sd.ldab * es;
          bytes += solves * (double)sd.nr * (sizeof(c128) + es);
        }
    }
    TimedRegion tr(FAM_SWEEP, st_, bytes);
    for (size_t q = 0; q < kinds.size(); ++q) launch_kind(q, kinds[q].plan);
  }
  if (wide_chains > 0) {
    // zero the counters for the next launch now, behind this one on the
    // stream, rather than between the host's update and the next sweep
    HH_HIP(hipMemsetAsync(sync_ + 32, 0, wide_chains * 128, st_));
    sync_clear_ = wide_chains;
  }
  {
    double bytes = 0;
    for (Solve* s : live) bytes += (double)s->len * (64.0 + s->t * (esz_of(s->prec) + 16.0));
    TimedRegion tr(FAM_SPMV, st_, bytes);
    for (int a = 0; a < 2; ++a)
      if (dsp[a]) launch_spmv(DEV(dsp[a]), (int)sp[a].size(), maxlen, a == 0 ? HH_FP64 : HH_FP32, st_);
  }
  {
    double bytes = 0;
    for (Solve* s : live) bytes += (double)s->len * 16.0 * (4.0 * s->m + 8.0 * s->t);
    TimedRegion tr(FAM_ORTH, st_, bytes);
    const int n = (int)live.size();
    launch_gram(DEV(dg1), n, maxblk, maxpx, maxt, st_);
    launch_block_update(DEV(du1), n, maxlen, maxt, st_);
    launch_gram(DEV(dg2), n, maxblk, maxpx, maxt, st_);
    launch_block_update(DEV(du2), n, maxlen, maxt, st_);
    for (size_t k = 0; k < qs.size(); ++k)
      if (dqs[k]) launch_qr_step(DEV(dqs[k]), (int)qs[k].size(), maxqblk, st_);
  }

  // ---- coefficients to the host, least squares, selection
  launch_gather(DEV(ddl), (int)dlt.size(), dl_dev_, st_);
  HH_HIP(hipMemcpyAsync(dl_host_.p, dl_dev_, dl, hipMemcpyDeviceToHost, st_));
  HH_HIP(hipStreamSynchronize(st_));
  std::vector<std::vector<int>> flags(live.size());
  for (size_t q = 0; q < live.size(); ++q) {
    Solve* s = live[q];
    HdLayout L(s->hcap, s->t);
    s->hbuf.resize(L.total);
    std::memcpy(s->hbuf.data(), dl_host_.p + hoff[q], L.total * sizeof(c128));
    flags[q].resize(s->t);
    std::memcpy(flags[q].data(), dl_host_.p + foff[q], s->t * sizeof(int));
  }
  unsigned abort_host = 0;
  if (sync_) std::memcpy(&abort_host, dl_host_.p + aoff, sizeof(unsigned));
  if (sync_ && abort_host) {
    set_error("sweep workgroups of one chain did not meet within the time limit");
    throw DeviceError();
  }
  for (size_t q = 0; q < live.size(); ++q) {
    Solve* s = live[q];
    HdLayout L(s->hcap, s->t);
    const int m = s->m, t = s->t;
    const zd* H = s->hbuf.data();
    s->ls.add_rows(t);
    for (int c = 0; c < t; ++c) {
      std::vector<zd> col(m + t, zd(0.0, 0.0));
      for (int i = 0; i < m; ++i) col[i] = H[L.g1 + i + (size_t)c * (m + t)] + H[L.g2 + i + (size_t)c * m];
      for (int i = 0; i < c; ++i) col[m + i] = H[L.r1 + i + (size_t)c * t] + H[L.r2 + i + (size_t)c * t];
      col[m + c] = H[L.rd + c];
      s->ls.add_column(col);
    }
    std::vector<int> kept;
    for (int c = 0; c < t; ++c) {
      if (flags[q][c]) ++s->deflated;
      else kept.push_back(m + c);
    }
    s->k += 1;
    s->m += t;
    s->res_est = s->ls.residual() / s->bnorm;
    s->sum_input = false;
    if (s->res_est <= s->tol) {
      s->done = true;
      s->converged = true;
    } else if (kept.empty()) {
      s->done = true;
      s->breakdown = true;
    } else if (s->k >= s->maxit) {
      s->done = true;
    } else if (t == 2 && kept.size() == 2) {
      s->inputs[0] = kept[1];  // LRL gets the vector from BTB's column (Sec. 4)
      s->inputs[1] = kept[0];
    } else if (t > 2 && kept.size() >= 2) {
      s->sum_input = true;     // every M_i gets the sum of the new vectors (Sec. 4)
    } else {
      for (int i = 0; i < t; ++i) s->inputs[i] = kept[0];
    }
  }
}

// ------------------------------------------------------------ finish
void Engine::finish(std::vector<Solve*>& solves) {
  std::vector<Solve*> fin;
  for (Solve* s : solves)
    if (s->done && !s->finalized) fin.push_back(s);
  if (fin.empty()) return;
  staged_ = 256;  // offset 0 is reserved so that no staged array aliases nullptr
  std::vector<CombTask> ct[2];
  std::vector<SpmvTask> sp;
  std::vector<ResTask> rt;
  std::vector<GramTask> gt;
  long long maxlen = 0;
  int maxblk = 1;
  // the coefficients y travel with the descriptors: c.y holds the staged
  // offset until the device area's address is known
  for (Solve* s : fin) {
    const std::vector<zd> y = s->ls.solve();
    const int nc = (int)y.size();
    CombTask c{};
    c.Z = s->Z;
    c.y = nc > 0 ? reinterpret_cast<c128*>(stage(y, staged_)) : nullptr;
    c.x0 = s->x0;
    c.x = s->x;
    c.len = s->len;
    c.ncols = nc;
    ct[s->prec == HH_FP64 ? 0 : 1].push_back(c);
    // residual scratch: basis slot m (free after the last iteration) when capacity allows
    c128* r = s->V + (size_t)std::min(s->m, s->vcap - 1) * s->len;
    SpmvTask tk{};
    tk.A = s->pb->d_A;
    tk.x = s->x;
    tk.y = r;
    tk.n = s->pb->n;
    tk.nvec = 1;
    sp.push_back(tk);
    ResTask rs{};
    rs.b = s->b;
    rs.r = r;
    rs.len = s->len;
    rt.push_back(rs);
    HdLayout L(s->hcap, s->t);
    GramTask g{};
    g.X = r;
    g.Y = r;
    g.out = s->Hd + L.nr;
    g.part = s->part;
    g.len = s->len;
    g.ldx = g.ldy = s->len;
    g.ldo = 1;
    g.px = 1;
    g.ty = 1;
    g.nblk = nblk_for(s->len, fin.size());
    gt.push_back(g);
    maxlen = std::max(maxlen, s->len);
    maxblk = std::max(maxblk, g.nblk);
  }
  CombTask* dct[2];
  for (int a = 0; a < 2; ++a) dct[a] = ct[a].empty() ? nullptr : stage(ct[a], staged_);
  SpmvTask* dsp = stage(sp, staged_);
  ResTask* drt = stage(rt, staged_);
  GramTask* dgt = stage(gt, staged_);
  std::vector<CopyTask> dlt;
  for (size_t q = 0; q < fin.size(); ++q) {
    const Solve* s = fin[q];
    HdLayout L(s->hcap, s->t);
    dlt.push_back({s->Hd + L.nr, (long long)(q * sizeof(zd)), (long long)(sizeof(zd) / 4)});
  }
  CopyTask* ddl = stage(dlt, staged_);
  const size_t dl = fin.size() * sizeof(zd);
  reserve_dl(dl);
  reserve_dev();
  for (int a = 0; a < 2; ++a) {
    if (!dct[a]) continue;
    CombTask* hc = reinterpret_cast<CombTask*>(task_host_.p + reinterpret_cast<size_t>(dct[a]));
    for (size_t i = 0; i < ct[a].size(); ++i)
      if (hc[i].y) hc[i].y = DEV(hc[i].y);
  }
  upload();
  for (int a = 0; a < 2; ++a)
    if (dct[a]) launch_combine(DEV(dct[a]), (int)ct[a].size(), maxlen, a == 0 ? HH_FP64 : HH_FP32, st_);
  launch_spmv(DEV(dsp), (int)sp.size(), maxlen, HH_FP64, st_);
  launch_residual(DEV(drt), (int)rt.size(), maxlen, st_);
  launch_gram(DEV(dgt), (int)gt.size(), maxblk, 1, 1, st_);
  launch_gather(DEV(ddl), (int)dlt.size(), dl_dev_, st_);
  HH_HIP(hipMemcpyAsync(dl_host_.p, dl_dev_, dl, hipMemcpyDeviceToHost, st_));
  HH_HIP(hipStreamSynchronize(st_));
  for (size_t q = 0; q < fin.size(); ++q) {
    Solve* s = fin[q];
    zd nr;
    std::memcpy(&nr, dl_host_.p + q * sizeof(zd), sizeof(zd));
    s->res_true = s->bnorm > 0 ? std::sqrt(std::max(0.0, nr.real())) / s->bnorm : 0.0;
    if (s->fail == HH_EINVAL) s->res_true = std::numeric_limits<double>::quiet_NaN();
    s->finalized = true;
  }
}

}  // namespace hh
