// Internal declarations shared by the HIP kernels, the MPGMRES engine and the
// C ABI.  Nothing here is part of the public interface (include/hh.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <array>
#include <mutex>
#include <string>
#include <vector>

#include "hh.h"

namespace hh {

// ---------------------------------------------------------------- complex
template <class T>
struct cx {
  T re, im;
};

template <class T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) {
  cx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
template <class T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return mk(a.re + b.re, a.im + b.im);
}
template <class T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return mk(a.re - b.re, a.im - b.im);
}
template <class T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class T>
__host__ __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) {
  return mk(a.re * s, a.im * s);
}
// a - b * c
template <class T>
__host__ __device__ __forceinline__ cx<T> cfms(cx<T> a, cx<T> b, cx<T> c) {
  return mk(a.re - b.re * c.re + b.im * c.im, a.im - b.re * c.im - b.im * c.re);
}
// c ? a : b on the components.  (A conditional between two complex lvalues
// would select between their addresses and load through the result; with
// one of them in LDS or on the stack that becomes a flat load.)
template <class T>
__host__ __device__ __forceinline__ cx<T> csel(bool c, cx<T> a, cx<T> b) {
  return mk(c ? a.re : b.re, c ? a.im : b.im);
}
// a + b * c as four fused multiply-adds
__host__ __device__ __forceinline__ float fmac_(float x, float y, float z) { return __builtin_fmaf(x, y, z); }
__host__ __device__ __forceinline__ double fmac_(double x, double y, double z) { return __builtin_fma(x, y, z); }
template <class T>
__host__ __device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {
  return mk(fmac_(-b.im, c.im, fmac_(b.re, c.re, a.re)), fmac_(b.im, c.re, fmac_(b.re, c.im, a.im)));
}
// conj(a) * b
template <class T>
__host__ __device__ __forceinline__ cx<T> cdotc(cx<T> a, cx<T> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <class T>
__host__ __device__ __forceinline__ cx<T> cinv(cx<T> a) {
  // 1/a with scaling to avoid overflow in |a|^2
  T s = fabs(a.re) > fabs(a.im) ? fabs(a.re) : fabs(a.im);
  if (s == T(0)) return mk(T(0), T(0));
  T ar = a.re / s, ai = a.im / s;
  T d = (ar * ar + ai * ai) * s;
  return mk(ar / d, -ai / d);
}
template <class T>
__host__ __device__ __forceinline__ T cabs1(cx<T> a) {
  return fabs(a.re) + fabs(a.im);
}
template <class To, class Ti>
__host__ __device__ __forceinline__ cx<To> ccast(cx<Ti> a) {
  return mk((To)a.re, (To)a.im);
}

using c64 = cx<float>;
using c128 = cx<double>;

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
const char* last_error();

#define HH_HIP(call)                                                               \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::hh::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call, hipGetErrorString(e_)); \
      throw ::hh::DeviceError();                                                   \
    }                                                                              \
  } while (0)

struct DeviceError {};
struct ArgError {};
struct MemError {};

// ---------------------------------------------------------------- geometry
// Segment plans of the parallel substitution (see sweep.hip): plan p spreads
// each triangular substitution of a strip over plan_width(p) workgroups.
// Plan 0: one workgroup per chain; plan 1 (HH_PLAN_WIDE): sixteen, for a few
// chains; plan 2 (HH_PLAN_PAIR): two, for batches of up to one chain per two
// compute units.  Plans 1 and 2 share the kernel and the kinds of maps
// (segment responses and map products), each with its own segment cut.
constexpr int HH_NPLAN = 3;
constexpr int HH_PLAN_WIDE = 1;
constexpr int HH_PLAN_PAIR = 2;
// A launch's choice is a segment plan, or HH_PLAN_TILE: plan 0's segments
// with tiles of two right-hand sides per chain (k_sweep_n).
constexpr int HH_PLAN_TILE = 3;
constexpr int HH_NCHOICE = 4;
// The launch of a factorisation with recursive strip solves (k_sweep_rec);
// not a choice the tuner makes.
constexpr int HH_PLAN_REC = 4;
// One strip of one sweep direction (0 = x / LRL, 1 = y / BTB).
struct StripDesc {
  int dir;        // 0 x, 1 y
  int s;          // 0-based position in the sweep
  int a;          // first node line across the strip
  int w;          // width in node lines
  int ns;         // rows of the factored system: the nr unknowns, then ns - nr identity rows
  int nr;         // unknowns n*w, local order q = long*w + short
  int kl;         // band half-width w + 1 (ku = kl)
  int ldab;       // band column stride 3*kl + 1
  int has1;       // interface Gamma_{s,1} (short index 0) present
  int has2;       // interface Gamma_{s,2} (short index w-1) present
  int S;          // lane slots of the back-substitution window (2 kl + 1 <= 64 S)
  int SL;         // lane slots of the forward-substitution window (kl + 1 <= 64 SL)
  int KP;         // terms per lane of the blocked substitution (see factor.hip)
  int gid;        // index of this strip in FactorSet::strips
  long long band_off;  // complex elements into the LU work buffer (factorisation only)
  long long img_off;   // complex elements into the solve image (see factor.hip)
  long long piv_off;   // ints into the pivot buffer (ns + HH_PAD entries)
  long long tr1_off;   // complex elements into the transmission buffer (n*7), or -1
  long long tr2_off;
  int segs;            // segments of the parallel substitution (waves of a sweep workgroup)
  int seg;             // rows per segment of plan 0 (a multiple of 64); the last may be shorter
  int tmaps;           // transfer maps per triangle, all plans together
  int pseg[HH_NPLAN];  // rows per segment of each plan
  int pmap[HH_NPLAN];  // index of the plan's first segment map among the triangle's maps
  int pwmap[HH_NPLAN]; // index of the plan's first workgroup map
  // plans p >= 1: slots of the products of maps (see plan_layout; index 0 unused)
  int pi_map[HH_NPLAN], a1_map[HH_NPLAN], a2_map[HH_NPLAN], ps_map[HH_NPLAN];
  int wide;            // the maps and responses of plans 1 and 2 exist (sweep_wide_fits)
  // bit p: ns is a whole number of plan p's segment groups (P pseg[p] rows),
  // so that workgroup g's rows of the forward substitution are those of the
  // back substitution's workgroup gu - 1 - g (gu: workgroups holding segments)
  int mirror;
  long long t_off;     // complex elements into the solve image: transfer maps (L, then U)
  long long phi_off[HH_NPLAN];  // complex elements into the solve image of the segment
                                // responses of plan p (L, then U; see plan_phi_elems)
  // Recursive strip solves (hh_factor_sweeps_inner): an outer strip names its
  // nsub sub-blocks (the descriptors this + sub .. this + sub + nsub - 1) and carries no
  // factors; a sub-block of the strip of width w (its a, w, dir are the
  // strip's) covers the strip's lines c0 .. c0+len-1 along its length, in the
  // order q' = (l - c0) w + t (orient 0) or q' = t len + (l - c0) (orient 1),
  // with has1/has2 and tr1_off/tr2_off for its own interfaces (w nodes each).
  int sub;
  int nsub;
  int c0, len, orient;
};

// Band half-widths: the one-wave LU window, the blocked substitution and the
// segment plans take kl <= HH_KL_WINDOW; wider strips (up to HH_KL_MAX) are
// factored by the blocked MFMA LU and solved by the lane-major substitution
// alone, with SL = ceil((kl + 1) / 64) and S = 2 SL window slots.
constexpr int HH_KL_WINDOW = 63;
constexpr int HH_KL_MAX = 191;
inline int lane_slots(int kl) { return (kl + 64) / 64; }

// Zero steps appended to every strip's solve image and pivot list, so that the
// substitution loops may run and prefetch past the end without bounds checks.
constexpr int HH_PAD = 64;

// Strip factors of every strip of every factored direction.
// Sweep orders of a preconditioner (Sec. 2 and Sec. 4): the double sweep
// (LRL, BTB), the forward single sweep (LR, BT) and the reverse single sweep
// (RL, TB).
enum SweepMode { SWEEP_DOUBLE = 0, SWEEP_FORWARD = 1, SWEEP_REVERSE = 2 };
constexpr int HH_MAXPRE = 4;  // preconditioners of one MPGMRES (t)

struct FactorSet {
  int N = 0;
  unsigned dirs = 0;
  int precision = -1;       // HH_FP64 / HH_FP32, -1 = not factored
  int nd = 0;               // number of factored directions
  int dir_id[2] = {-1, -1}; // direction (0/1) of factored slot 0/1 (strips[slot*N + s])
  // The preconditioners M_1..M_t of MPGMRES in order: the factored slot whose
  // strips they use and their sweep order.  hh_factor_sweeps sets the double
  // sweeps of the factored directions (LRL, then BTB).
  int npre = 0;
  int pre_slot[HH_MAXPRE] = {0, 0, 0, 0};
  int pre_mode[HH_MAXPRE] = {0, 0, 0, 0};
  std::vector<StripDesc> strips;  // dir-major: strips[d*N + s]
  StripDesc* d_strips = nullptr;  // device copy
  void* band = nullptr;            // LU work buffer, freed once every map is built
  void* img = nullptr;             // solve image, complex<precision> elements
  int* piv = nullptr;
  void* tr = nullptr;              // transmission stencils, complex<precision>
  int* d_err = nullptr;            // [0] = 1 + strip index of first zero pivot, [1] = column
  int* d_pflag = nullptr;          // per strip: 1 if the LU interchanged any rows
  std::array<int, 2> h_err{{0, 0}};  // host copy, valid once the factor stream completed
  std::vector<int> h_pflag;           // host copy of d_pflag, likewise
  bool any_pivot = false;             // some strip pivoted (set by factor_finish)
  // The maps of segment plans 0 and 2 (one and two workgroups per chain)
  // serve batched sweeps only; where plans 1 and 2 exist they are built from
  // the kept band when a launch first takes plan 0 or 2 (ensure_batch_maps),
  // unless eager_batch_maps asks for them with the factorisation.
  bool eager_batch_maps = false;
  bool batch_maps = true;             // the maps of plans 0 and 2 are built or queued
  size_t band_elems = 0, img_elems = 0, piv_elems = 0, tr_elems = 0;
  int max_ns = 0, max_kl = 0;
  int nsub = 1;       // sub-blocks per strip (> 1: recursive strip solves)
  int first_sub = 0;  // index of the first sub-block in strips
  long long rho_elems = 0;  // per-chain strip scratch of a sweep (elements)
  size_t bytes() const;
};

}  // namespace hh

struct hh_problem {
  int n = 0;
  double omega = 0;
  std::vector<double> c;
  double* d_c = nullptr;           // layer speeds on the device
  // A sampled speed field (hh_assemble_field): wave numbers omega / c of the
  // triangles (2 per cell, lower then upper, cell (ci, cj) at 2 (cj (n-1) + ci)),
  // of the edges (i, j)-(i, j+1) at j n + i and of the edges (i, j)-(i+1, j) at
  // j (n-1) + i; null for a layered medium.
  double* d_kt = nullptr;
  double* d_kv = nullptr;
  double* d_kh = nullptr;
  double* d_kn = nullptr;          // ... and at the nodes (j n + i)
  int scheme = 0;                  // HH_SCHEME_P1 or HH_SCHEME_FD5
  hh::c128* d_b = nullptr;         // right-hand side b = -M f given at assembly, or null
  hh::c128* d_A = nullptr;         // 4 * n*n upper diagonals
  hh::FactorSet fs;
  hipStream_t st[2] = {nullptr, nullptr};
  bool own_streams = true;         // false: the caller's (hh_set_streams), not destroyed
  hipEvent_t ev[2] = {nullptr, nullptr};
  int device = 0;
  size_t bytes() const;
};

namespace hh {

// ---------------------------------------------------------------- timing
struct TimingFamily {
  long long launches = 0;
  double ms = 0;
  double bytes = 0;
};
bool timing_on();
// Records (start, stop) events around a launch; resolved lazily.
struct TimedRegion {
  int fam;
  hipStream_t st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double bytes;
  TimedRegion(int family, hipStream_t s, double b);
  ~TimedRegion();
};
enum { FAM_SWEEP = 0, FAM_SPMV, FAM_FACTOR, FAM_ORTH, FAM_ASSEMBLE, FAM_COUNT };
void timing_flush();

// ---------------------------------------------------------------- media
// What the assembly kernels need to know of the wave speed (eq. (1), k = omega
// / c): the layer table, or the sampled wave numbers of a speed field (see
// hh_problem::d_kt, d_kv, d_kh; when kt is set, kv and kh are too).
struct Medium {
  double omega;
  int L;
  const double* c;
  const double* kt;
  const double* kv;
  const double* kh;
  const double* kn;  // sampled field: wave numbers at the nodes (five-point scheme)
  int fd5;           // the five-point scheme of Sec. 4 instead of P1 (see assemble.hip)
};

// ---------------------------------------------------------------- problems
// Internal halves of hh_assemble / hh_factor_sweeps / hh_free (capi.cpp),
// also driven asynchronously by the serving loop.
void factor_setup(hh_problem* pb, unsigned dirs, int nstrips, int precision, int nsub = 1);
void factor_launch(hh_problem* pb, hipStream_t st);
int factor_finish(hh_problem* pb);
hh_problem* problem_create(double omega, int nlayers, const double* c_layers, int n,
                           int scheme = 0);
// The same for a speed field sampled by a host callback at the triangle
// centroids, edge midpoints and nodes.
hh_problem* problem_create_field(double omega, double (*speed)(double, double, void*), void* ctx,
                                 int n, int scheme = 0);
void problem_destroy(hh_problem* pb);

// ---------------------------------------------------------------- memory
void* dev_alloc(size_t bytes);
void dev_free(void* p);
size_t dev_live_bytes();
bool set_allocator(void* (*alloc)(size_t, void*), void (*free_fn)(void*, void*), void* ctx);
// Releases the cached free blocks and the pooled timing events.
void runtime_release_caches();
// Streams for problems created from now on (hh_set_streams): both null means
// the problems create and own their streams.
void set_caller_streams(hipStream_t x, hipStream_t y);
bool caller_streams(hipStream_t& x, hipStream_t& y);

// ---------------------------------------------------------------- kernels
// assemble.hip
Medium medium_of(const hh_problem* pb);
void launch_assemble(int n, const Medium& md, c128* d_A, hipStream_t st);
// b = -M f (P1) or b = -h^2 w f (five-point scheme, fd5).
void launch_load_vector(int n, int nvec, const c128* f, c128* b, hipStream_t st, int fd5 = 0);
void launch_pack_strips(const hh_problem* pb, hipStream_t st);
// Zeroes and packs again the bands of the strips whose pflag is 2 (marked by
// the LU that assumes no interchange).
void launch_repack_marked(const hh_problem* pb, hipStream_t st);
// HH_LU_INTERCHANGE=1: factor every strip with the interchanging LU kernel.
bool lu_interchanging_only();

// factor.hip
void launch_band_lu(const hh_problem* pb, hipStream_t st);
void launch_transfer(const FactorSet& fs, int planmask, hipStream_t st);
// Map products of the plans p >= 1 in planmask (bit p: plan p).
void launch_products(const FactorSet& fs, int planmask, hipStream_t st);
// Plans whose maps a factorisation builds at once (the rest, plans 0 and 2,
// when a batch first needs them): bit p for plan p.
constexpr int HH_EAGER_PLANS = 1 << HH_PLAN_WIDE;
constexpr int HH_BATCH_PLANS = (1 << 0) | (1 << HH_PLAN_PAIR);
// Builds the maps of plans 0 and 2 on st if the factorisation left them out,
// waits for them and frees the band.
void ensure_batch_maps(hh_problem* pb, hipStream_t st);

// sweep.hip
// One preconditioner application (one direction, one right-hand side).
struct SweepChain {
  const StripDesc* strips;  // N descriptors of the direction (device)
  const c128* r;            // FP64 input, n*n
  void* z;                  // output in sweep precision, n*n
  void* rho;                // scratch, >= 2 max ns elements of sweep precision (FactorSet::rho_elems)
  void* g1;                 // scratch, N*n elements of sweep precision
};
// One double sweep: one chain over the N strips of a direction.
struct SweepTask {
  SweepChain ch;
  SweepChain ch2;  // the second right-hand side of a tile (launch_sweep with nr = 2)
  const void* img;
  const int* piv;
  const int* pflag;
  const void* tr;
  int n;
  int N;
  void* xch;      // wide plan: HH_XCH_BYTES_PER_WG bytes per workgroup (G * 64 stamped
                  // tail entries of the forward substitution, then as many of the back one)
  unsigned* bar;  // wide plan: arrival counter of the chain's workgroups, zero at launch
  int mode;       // SweepMode: double sweep, forward or reverse single sweep
};
// All tasks share the precision, the blocked-term count KP (which fixes the
// slot count S of the pivoted path) and the segment count P (waves per
// workgroup); kmax and nmax = largest band half-width and n among the tasks
// (they size the LDS); pivots: some strip of some task pivoted (selects the
// kernel that carries the pivoted path).  plan: segment plan (0: one
// workgroup per chain; otherwise plan_width(plan) workgroups per chain, which
// needs pivots == false, xch and bar in every task, and abort: a device word
// that a workgroup raises when its partners fail to arrive in time).
void launch_sweep(const SweepTask* d_tasks, int ntasks, int precision, int KP, int P, int kmax,
                  int nmax, bool pivots, int plan, unsigned* abort, hipStream_t st);
// Tiles of two right-hand sides of the same preconditioner per chain
// (k_sweep_n, segment plan 0): task t holds its two chains in ch and ch2.
// They need complex64 strips none of which pivoted and a workgroup's LDS for
// two rings per wave (sweep_tiles_fit).  The results are bitwise those of
// launch_sweep on plan 0.
bool sweep_tiles_fit(int precision, int KP, int P, int nmax, bool pivots);
void launch_sweep_tiles(const SweepTask* d_tiles, int ntiles, int precision, int KP, int P,
                        int nmax, bool pivots, hipStream_t st);
// Whether the wide plan can run a factorisation (complex64 strips, band
// half-width at most 31, at most two workgroup tails per wave, LDS).
bool sweep_wide_fits(int precision, int P, int kmax, int nmax);
// Choice for a launch of ntasks chains (without a tuned one): the
// HH_SWEEP_PLAN environment variable (0-3) when set and possible; else the
// sixteen-workgroup plan while ntasks times sixteen workgroups fit the
// device at once, the two-workgroup plan while its workgroups fit the device
// at once (built: its maps exist), tiles of two right-hand sides beyond one
// chain per compute unit, and plan 0 otherwise (always where a strip pivoted).
int sweep_plan_for(int ntasks, int precision, int P, int kmax, int nmax, bool pivots, bool built);
// Whether plan p can run a launch of ntasks chains: plan 0 always; plans 1
// and 2 on complex64 strips none of which pivoted (sweep_wide_fits), when all
// ntasks * plan_width(p) workgroups fit the device at once (occupancy), plan 2
// once its maps are built (built = the batch maps).
bool sweep_plan_fits(int plan, int ntasks, int precision, int KP, int P, int kmax, int nmax,
                     bool pivots, bool built);
// Blocked substitution: block size and terms per lane for band half-width kl.
// KP terms per lane cover the K + HH_BLK columns of a block map over the 64/HH_BLK
// lanes of one output row; KP <= 12 exactly when 2 kl + 1 <= 64 (one lane-major
// row of the pivoted image).
constexpr int HH_BLK = 16;
inline int blocked_kp(int kl) {
  return kl <= 16 ? 8 : kl <= 24 ? 10 : kl <= 31 ? 12 : kl <= 48 ? 16 : 20;
}
// Blocks stored per triangle: whole 64-row chunks plus sixteen zero blocks, so
// the substitution (steps of up to four blocks, rounded up to a multiple of
// three, maps requested up to two steps ahead) reads no bounds-tested memory.
__host__ __device__ inline long long blocked_blocks(long long ns) { return 4 * ((ns + 63) / 64) + 16; }
// Rows per segment when a strip's substitutions are split over P waves.
__host__ __device__ inline int segment_rows(int ns, int P) {
  const int per = (ns + P - 1) / P;
  return (per + 63) / 64 * 64;
}
// Plan p: a triangle of ns rows (band half-width K) is cut into segments of
// plan_seg rows, P per workgroup over plan_width(p) workgroups.  Plan 0 is
// the one-workgroup split (segments a multiple of 64 rows); the wide plan cuts
// 16-row aligned segments.  Either way a segment is at least K rows long, so
// that a segment's state (the K outputs before it) lies in the segment before
// it, and every segment after the first starts at row K or later.
// Exchange area of a wide-plan chain, per workgroup: 64 tail entries for each
// of the two substitutions, each entry two 64-bit words (value half, stamp).
constexpr size_t HH_XCH_BYTES_PER_WG = 2 * 64 * 16;
__host__ __device__ inline int plan_width(int p) {
  return p == HH_PLAN_WIDE ? 16 : p == HH_PLAN_PAIR ? 2 : 1;
}
__host__ __device__ inline int plan_seg(int ns, int P, int p, int K) {
  if (p == 0) return segment_rows(ns, P);
  const int S = plan_width(p) * P, per = (ns + S - 1) / S, least = (K + 15) / 16 * 16;
  const int seg = (per + 15) / 16 * 16;
  return seg > least ? seg : least;
}
__host__ __device__ inline int plan_nseg(int ns, int seg) { return (ns + seg - 1) / seg; }
// Segment transfer maps: segments 1 .. nseg-2 (segment 0 starts from the
// true zero state and the state after the last one is never needed).
__host__ __device__ inline int plan_seg_maps(int ns, int seg) {
  const int v = plan_nseg(ns, seg) - 2;
  return v > 0 ? v : 0;
}
// Workgroup transfer maps (over the P segments of workgroup g, g = 1 .. gu-2
// with gu the workgroups that hold segments); only plans of more than two
// workgroups need them.
__host__ __device__ inline int plan_wg_maps(int ns, int seg, int P, int G) {
  if (G <= 2) return 0;
  const int gu = (plan_nseg(ns, seg) + P - 1) / P, v = gu - 2;
  return v > 0 ? v : 0;
}
// Transfer maps and segment responses are stored zero-padded to KM = map_dim
// state entries (KM >= K for every strip of a factorisation, fixed by its
// blocked term count KP): a map is KM x KM, column-major.
__host__ __device__ constexpr int map_dim(int KP) {
  return KP <= 8 ? 16 : KP <= 10 ? 24 : KP <= 12 ? 32 : KP <= 16 ? 48 : 64;
}
// Segment responses of plan p (one triangle): for segments c = 1 ..
// nseg-1, the outputs of the segment's rows started from the unit state e_k
// with zero inputs, Phi_c[k][i] at ((c - 1) KM + k) seg + i (zero for k >= K).
__host__ __device__ inline long long plan_phi_elems(int ns, int P, int K, int KM, int p) {
  const int seg = plan_seg(ns, P, p, K), nseg = plan_nseg(ns, seg);
  return nseg > 1 ? (long long)(nseg - 1) * seg * KM : 0;
}
// Fills the plan fields of sd (ns, kl and segs set) and returns the maps per
// triangle.  Map slots of a triangle: per plan its segment maps T_c (slot
// pmap + c - 1) and workgroup maps W_g (pwmap + g - 1); then, per plan p >= 1,
// products of consecutive segment maps within a workgroup, slot + c - 1 for
// segment c = g P + w:
//   pi_map: Pi_c = T_{c-1} ... T_{gP} (w >= 1), the map from the workgroup's
//           start state to segment c's start state;
//   a1_map: T_c T_{c-1} (w >= 2);  a2_map: T_c ... T_{c-3} (w >= 4);
// and ps_map + g G + j: Psi_{j,g} = W_{g-1} ... W_{j+1} (0 <= j <= g-2).
inline int plan_layout(StripDesc& sd) {
  int m = 0;
  for (int p = 0; p < HH_NPLAN; ++p) {
    const bool on = p == 0 || sd.wide;  // plans 1 and 2 only where they can run
    sd.pseg[p] = plan_seg(sd.ns, sd.segs, p, sd.kl);
    sd.pmap[p] = m;
    if (on) m += plan_seg_maps(sd.ns, sd.pseg[p]);
    sd.pwmap[p] = m;
    if (on) m += plan_wg_maps(sd.ns, sd.pseg[p], sd.segs, plan_width(p));
  }
  sd.pi_map[0] = sd.a1_map[0] = sd.a2_map[0] = sd.ps_map[0] = 0;
  for (int p = 1; p < HH_NPLAN; ++p) {
    const int nseg = plan_nseg(sd.ns, sd.pseg[p]), G = plan_width(p);
    const int per = sd.wide && nseg > 1 ? nseg - 1 : 0;
    sd.pi_map[p] = m;
    sd.a1_map[p] = m + per;
    sd.a2_map[p] = m + 2 * per;
    sd.ps_map[p] = m + 3 * per;
    m += 3 * per + (sd.wide && G >= 3 && nseg > 1 ? G * G : 0);
  }
  sd.seg = sd.pseg[0];
  sd.tmaps = m;
  return m;
}
// LDS of a wide-plan workgroup (complex elements): the rings (640 P), three
// vectors per wave (tails and states, scan exchange, partial sums: 64 each,
// one more for the scan) and two node lines of transmission data.
inline long long sweep_lds_elems_wide(int P, int n) {
  return 640LL * P + 64LL * (3 * P + 1) + 2LL * n;
}
// LDS of a sweep workgroup of P waves (complex elements): per-wave rings
// (phase 1 and 3) sharing space with the staged transfer maps (phase 2), the
// segment tails and states, and two node lines of transmission data.
inline long long sweep_lds_elems(int P, int KM, int n) {
  const long long work = std::max(640LL * P, (long long)std::max(P - 2, 0) * KM * KM);
  return work + 2LL * 64 * P + 2LL * n;
}
// Segments of the parallel substitution: the most (up to 8) whose workgroup
// fits the LDS.
inline int sweep_segments(int KM, int n, size_t esz) {
  for (int P : {8, 6, 4, 3, 2})
    if (sweep_lds_elems(P, KM, n) * (long long)esz <= 150 * 1024) return P;
  return 1;
}
// Image elements of one strip: the larger of the pivoted (lane-major) and the
// unpivoted (blocked maps plus segment transfer maps) layouts; which one is
// built is decided by the LU.
inline long long strip_image_elems(long long ns, int S, int KP, int K, int P, bool wide) {
  const long long lane_major = (ns + HH_PAD) * (64LL * (1 + S) + 1);
  if (K > HH_KL_WINDOW) return (ns + HH_PAD) * (64LL * 3 * lane_slots(K) + 1);
  StripDesc sd{};
  sd.ns = (int)ns;
  sd.kl = K;
  sd.segs = P;
  sd.wide = wide;
  const int KM = map_dim(KP);
  long long phi = 0;
  for (int p = 0; p < HH_NPLAN; ++p)
    if (p == 0 || wide) phi += 2 * plan_phi_elems((int)ns, P, K, KM, p);
  const long long blocked = 2 * blocked_blocks(ns) * KP * 64 + 2LL * plan_layout(sd) * KM * KM + phi;
  return lane_major > blocked ? lane_major : blocked;
}
// Scratch of one preconditioner application (sweep_apply_core): the task
// descriptors, the sync words ([0] abort, then one 128-byte line per chain),
// the strip buffers rho and g1, the complex64 staging of z (complex64 strips
// only) and the wide plan's exchange areas.
struct SweepBuffers {
  SweepTask* tasks;
  unsigned* sync;
  void* rho;
  void* g1;
  void* zs;
  void* xch;
  size_t xch_bytes;
};
// Segment plan of an application to nvec vectors.
int sweep_plan_of(const hh_problem* pb, int nvec);
// The buffers carved from base (256-byte aligned parts); *total receives the
// bytes they take (base may be nullptr to size them only).
SweepBuffers sweep_layout(const hh_problem* pb, int nvec, int plan, char* base, size_t* total);
// z = M^{-1} r for nvec vectors with the strips of factored slot i in sweep
// order mode, on the given scratch; waits for the stream.  Allocates nothing
// unless the plan-0 transfer maps have to be built first (ensure_batch_maps).
void sweep_apply_core(hh_problem* pb, int i, int mode, int nvec, const c128* r, c128* z,
                      int plan, const SweepBuffers& b);
// The no-allocation variant (noalloc.hip): the same application on the
// library's static device scratch.
void sweep_apply_noalloc(hh_problem* pb, int i, int mode, int nvec, const c128* r, c128* z);
// Zeroes bytes (a multiple of 4) with a fill kernel on st.
void launch_zero(void* p, size_t bytes, hipStream_t st);

// Single strip solve (test hook): rhs/x in FP64, strip-local order.
void launch_strip_solve(const hh_problem* pb, int strip_index, const c128* rhs, c128* x,
                        void* scratch, hipStream_t st);

// krylov.hip: see krylov.h

}  // namespace hh
