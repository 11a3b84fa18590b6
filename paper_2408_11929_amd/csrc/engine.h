// Batched selective MPGMRES engine (Sec. 3, selection rule of Sec. 4).
//
// A Solve is one right-hand side of one problem.  The engine advances any set
// of solves (of one or several problems) by one outer iteration with batched
// launches: the sweeps of every preconditioner of every solve in one launch,
// one SpMV launch, and the block Gram-Schmidt kernels over all bases at once.
// The only host synchronisation per iteration is the copy of the new
// Hessenberg block columns to the host, where the small least-squares problem
// is updated with Givens rotations in FP64.
#pragma once

#include <complex>
#include <functional>
#include <vector>

#include "hh_internal.h"
#include "krylov.h"

namespace hh {

using zd = std::complex<double>;

// Incremental QR (Givens) of the block Hessenberg matrix Hbar: rows are basis
// vectors, columns are preconditioned vectors.  Columns found dependent (zero
// pivot after rotation) get a zero coefficient.
class LeastSquares {
 public:
  void init(double beta);
  void add_rows(int count);
  void add_column(std::vector<zd> h);  // h.size() == rows()
  int rows() const { return (int)g_.size(); }
  int cols() const { return (int)R_.size(); }
  double residual() const;
  std::vector<zd> solve() const;

 private:
  struct Rot {
    int i, k;
    double c;
    zd s;
  };
  std::vector<std::vector<zd>> R_;
  std::vector<int> piv_;
  std::vector<Rot> rots_;
  std::vector<zd> g_;
  int rank_ = 0;
};

struct Solve {
  hh_problem* pb = nullptr;
  const c128* b = nullptr;  // device
  c128* x = nullptr;        // device
  const c128* x0 = nullptr; // device starting guess (nullptr: x0 = 0); may equal x
  long long len = 0;
  int t = 0;
  int prec = HH_FP64;
  double tol = 1e-6;
  int maxit = 200;
  // state
  double beta = 0;   // ||b - A x0||_2, the Krylov space's starting norm
  double bnorm = 0;  // ||b||_2: tolerances and reported residuals are relative to it
  int k = 0;        // completed iterations
  int m = 0;        // basis columns in use (1 + k t)
  int vcap = 0, zcap = 0;
  c128* V = nullptr;
  void* Z = nullptr;
  c128* Hd = nullptr;     // device scratch for one iteration's coefficients
  int hcap = 0;           // basis capacity Hd was sized for
  c128* part = nullptr;   // partial sums
  size_t part_elems = 0;
  int* flags = nullptr;   // t deflation flags
  void* rho = nullptr;    // sweep scratch, t chains
  void* g1 = nullptr;
  c128* sumv = nullptr;   // t > 2: the sum of the new basis vectors (sweep input)
  int inputs[4] = {0, 0, 0, 0};
  bool sum_input = false; // the next sweeps read sumv (formed at the next step)
  LeastSquares ls;
  bool done = false, converged = false, breakdown = false, finalized = false;
  int fail = 0;           // stopped early: HH_EBUDGET (growth refused), HH_ENOMEM, or
                          // HH_EINVAL (b or b - A x0 not finite)
  void* owner = nullptr;  // the caller's tag (the server's request)
  int charged_its = 0;    // iterations of Krylov memory charged to the owner's budget
  int deflated = 0;
  double res_est = 0, res_true = 0;
  std::vector<zd> hbuf;   // host copy of Hd
};

// Layout of Solve::Hd for an iteration with basis size m and block width t:
//   G1 : (m+t) x t, ld m+t   (X^H W against [V, W] before any update)
//   G2 : m x t, ld m          (second CGS pass)
//   R1 : t x t, R2 : t x t    (in-block MGS, two passes)
//   RD : t                    (norms after in-block orthogonalisation)
//   NR : t                    (squared norms before normalisation)
struct HdLayout {
  size_t g1, g2, r1, r2, rd, nr, total;
  HdLayout(int m, int t);
};

// Growable pinned host buffer, so that copies to and from it run as direct
// transfers.  A grow waits for the device before it frees the old buffer;
// keep copies the old contents.
struct PinnedBuf {
  unsigned char* p = nullptr;
  size_t cap = 0;
  void reserve(size_t n, bool keep);
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf();
};

class Engine {
 public:
  explicit Engine(hipStream_t st);
  ~Engine();
  // Prepares solves (allocates, beta = ||b||, v1 = b / beta).
  void begin(std::vector<Solve*>& solves);
  // One outer iteration for every solve that is not done.
  void step(std::vector<Solve*>& solves);
  // x = Z y and the FP64 residual for solves that are done but not finalised.
  void finish(std::vector<Solve*>& solves);
  static void release(Solve* s);
  static size_t footprint(const hh_problem* pb, int t, int prec, int maxit);
  // Whether sweeps may run on several workgroups per chain (the wide segment
  // plan); engines that share the device with other engines keep it off.
  void set_wide(bool on) { wide_ok_ = on; }
  // Budget hook for the growth of a solve's Krylov bases past the iterations
  // charged to it (Solve::charged_its): called with the extra device bytes
  // (negative to give some back); false refuses the growth, and that solve
  // alone stops with fail = HH_EBUDGET.  Without a hook growth is unlimited.
  void set_grow_hook(std::function<bool(Solve*, long long)> h) { grow_ = std::move(h); }
  // Device bytes of one iteration's Krylov columns (V and Z) of a solve.
  static size_t iteration_bytes(const Solve* s);

 private:
  hipStream_t st_;
  void* task_dev_ = nullptr;
  size_t task_cap_ = 0;
  PinnedBuf task_host_;  // staged descriptors
  PinnedBuf dl_host_;    // one iteration's coefficients, flags and abort word
  unsigned char* dl_dev_ = nullptr;  // the same gathered on the device, one transfer
  size_t dl_dev_cap_ = 0;
  template <class TT>
  TT* stage(const std::vector<TT>& v, size_t& off);
  void upload();
  void reserve_dev();
  void reserve_dl(size_t dl);
  void ensure_capacity(Solve* s);
  // ensure_capacity for every solve, stopping (fail) the ones whose growth
  // is refused or cannot be allocated, without touching the others.
  void ensure_all(std::vector<Solve*>& solves);
  std::function<bool(Solve*, long long)> grow_;
  size_t staged_ = 0;
  // wide plan: sync words (word 0: abort, sticky until begin(); then one
  // 128-byte line per chain) and the chains' exchange areas
  bool wide_ok_ = true;
  unsigned* sync_ = nullptr;
  size_t sync_cap_ = 0;
  size_t sync_clear_ = 0;  // chain lines zeroed since their last launch
  void* xch_ = nullptr;
  size_t xch_cap_ = 0;
  c128* ones_ = nullptr;  // HH_MAXPRE ones: coefficients of the sum rule's combination
};

}  // namespace hh
