// Double-sweep preconditioner application (Sec. 2, eqs. (2)-(4)).
//
// One 64-lane workgroup runs one whole double sweep: forward over strips
// 1..N (eq. (2), zero data on Gamma_{s,2}), backward over N-1..1 (eq. (3),
// reusing the Gamma_{s,1} data of v_{s-1} formed in the forward pass and
// taking the Gamma_{s,2} data from u_{s+1}); u_N = v_N, so 2N-1 strip solves.
// Every strip solve forms the strip right-hand side R_s r + g, runs the
// forward substitution with L and the back substitution with U, and writes
// the strip solution over the global vector (the most recent solve wins in
// the overlaps).  Other workgroups run the other directions and right-hand
// sides, so one launch covers a whole batch of applications.
//
// Transmission data (eq. (4), zeroth-order Robin): for an interface node,
// g = sum_d coef_d z[p + off_d] over the 7-point stencil, with coef = (A_s - A)
// on that row, precomputed at factorisation time.
//
// Substitutions.  A strip whose factorisation made no row interchange (the
// usual case) uses the blocked row recurrence of solve_blocked, with block
// maps built at factorisation time.  A strip that pivoted uses the lane-major
// recurrence of solve_lower / solve_upper:
//     out_e = b_e (times 1/U_ee for U),  b_{e+c} -= coef(e, c) b_e,  c = 1..K
// over e = 0..ns-1 (reversed order for U), K = kl for L and 2 kl for U.
// Element e of the sliding window lives in lane e mod 64 (slot k holds the
// element 64k further on).  A step is: read the pivot and the current element
// from their lanes (v_readlane), apply the interchange and record the output
// (v_writelane), switch the finished lane to its next element, and one
// complex multiply-subtract per lane with that lane's coefficient, which the
// solve image provides as one coalesced 64-lane row per step.  Coefficient
// rows are prefetched D steps ahead, window elements one 64-block ahead.
#include <atomic>
#include <cstdlib>
#include <map>

#include "hh_internal.h"

namespace hh {

namespace {

template <class T>
using gptr = T __attribute__((address_space(1)))*;

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni(long long v) {
  int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffLL));
  int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((long long)hi << 32) | (unsigned int)lo;
}
template <class P>
__device__ __forceinline__ P* uniptr(P* p) {
  return (P*)(uintptr_t)uni((long long)(uintptr_t)p);
}

__device__ __forceinline__ float rl(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rl(double v, int l) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <class T>
__device__ __forceinline__ cx<T> rlc(cx<T> v, int l) {
  return mk(rl(v.re, l), rl(v.im, l));
}
// v_writelane_b32: lane l of `old` takes the wave-uniform value v.
__device__ int writelane_i32(int v, int l, int old) __asm("llvm.amdgcn.writelane.i32");

__device__ __forceinline__ float wl(float v, int l, float old) {
  return __int_as_float(writelane_i32(__float_as_int(v), l, __float_as_int(old)));
}
__device__ __forceinline__ double wl(double v, int l, double old) {
  long long b = __double_as_longlong(v), o = __double_as_longlong(old);
  int lo = writelane_i32((int)(b & 0xffffffffLL), l, (int)(o & 0xffffffffLL));
  int hi = writelane_i32((int)(b >> 32), l, (int)(o >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <class T>
__device__ __forceinline__ cx<T> wlc(cx<T> v, int l, cx<T> old) {
  return mk(wl(v.re, l, old.re), wl(v.im, l, old.im));
}
template <class T>
__device__ __forceinline__ cx<T> ld(gptr<const cx<T>> p, long long i) {
  return mk(p[i].re, p[i].im);
}
template <class T>
__device__ __forceinline__ cx<T> ld(gptr<cx<T>> p, long long i) {
  return mk(p[i].re, p[i].im);
}
template <class T>
__device__ __forceinline__ void st(gptr<cx<T>> p, long long i, cx<T> v) {
  p[i].re = v.re;
  p[i].im = v.im;
}
template <class T>
__device__ __forceinline__ cx<T> sel(bool c, cx<T> a, cx<T> b) {
  return mk(c ? a.re : b.re, c ? a.im : b.im);
}
// a b with the rounding of each component fixed (a product, then one fused
// multiply-add), so that every kernel forms it bit for bit alike whatever the
// compiler would otherwise contract
template <class T>
__device__ __forceinline__ cx<T> cmulx(cx<T> a, cx<T> b) {
  return mk(fmac_(a.re, b.re, -(a.im * b.im)), fmac_(a.re, b.im, a.im * b.re));
}

// Access policies for vectors that workgroups of one chain share.  Plain:
// ordinary loads and stores (one workgroup per chain).  Agent: complex64
// loads and stores coherent at agent scope (relaxed atomics, one 64-bit
// access each), so that a store is visible to every other workgroup once it
// has completed and a load never returns a line cached before: the meetings
// of a chain then order them with a wait for the stores and the arrival
// counter alone, without writing back or invalidating the L2 caches.
struct PlainAcc {
  template <class T>
  static __device__ __forceinline__ cx<T> load(gptr<const cx<T>> p, long long i) {
    return ld<T>(p, i);
  }
  template <class T>
  static __device__ __forceinline__ void store(gptr<cx<T>> p, long long i, cx<T> v) {
    st<T>(p, i, v);
  }
};
struct AgentAcc {
  using u64g = unsigned long long __attribute__((address_space(1)))*;
  using cu64g = const unsigned long long __attribute__((address_space(1)))*;
  static __device__ __forceinline__ c64 load(gptr<const c64> p, long long i) {
    const unsigned long long b =
        __hip_atomic_load((cu64g)(p + i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return mk(__uint_as_float((unsigned)b), __uint_as_float((unsigned)(b >> 32)));
  }
  static __device__ __forceinline__ void store(gptr<c64> p, long long i, c64 v) {
    const unsigned long long b =
        ((unsigned long long)__float_as_uint(v.im) << 32) | __float_as_uint(v.re);
    __hip_atomic_store((u64g)(p + i), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

// Forward substitution with the row interchanges of partial pivoting for C
// chains: y = L^{-1} P b in place on x[c][0..ns).  Lm: solve-image rows
// (64 per step, padded), piv: padded pivot lists.  ns is wave-uniform and
// equal for all chains.
template <class T, int C, int D>
__device__ __forceinline__ void solve_lower(gptr<cx<T>> (&x)[C], gptr<const cx<T>> (&Lm)[C],
                                            gptr<const int> (&piv)[C], int ns, int lane) {
  const cx<T> zero = mk((T)0, (T)0);
  cx<T> b[C], nxtA[C], nxt[C], yout[C], cc[C][D], cn[C][D];
  int pc[C], pn[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    b[c] = csel(lane < ns, ld<T>(x[c], lane < ns ? lane : 0), zero);
    nxtA[c] = csel(64 + lane < ns, ld<T>(x[c], 64 + lane < ns ? 64 + lane : 0), zero);
    nxt[c] = yout[c] = zero;
    pc[c] = lane < D ? piv[c][lane] : 0;
#pragma unroll
    for (int u = 0; u < D; ++u) cc[c][u] = ld<T>(Lm[c], (long long)u * 64 + lane);
  }
  for (int j0 = 0; j0 < ns; j0 += D) {
    if ((j0 & 63) == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        nxt[c] = nxtA[c];
        const int e = j0 + 128 + lane;
        nxtA[c] = csel(e < ns, ld<T>(x[c], e < ns ? e : 0), zero);
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      gptr<const cx<T>> row = Lm[c] + (long long)(j0 + D) * 64 + lane;
#pragma unroll
      for (int u = 0; u < D; ++u) cn[c][u] = ld<T>(row, (long long)u * 64);
      pn[c] = lane < D ? piv[c][j0 + D + lane] : 0;
    }
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int lj = (j0 + u) & 63;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int lp = __builtin_amdgcn_readlane(pc[c], u) & 63;
        const cx<T> bj = rlc(b[c], lp);
        const cx<T> bp = rlc(b[c], lj);
        b[c] = wlc(bp, lp, b[c]);              // interchange: element p takes element j
        yout[c] = wlc(bj, lj, yout[c]);        // y_j, stored with its 64-block
        b[c] = sel(lane == lj, nxt[c], b[c]);  // lane lj moves on to element j + 64
        b[c] = cfms(b[c], cc[c][u], bj);
      }
    }
    if (((j0 + D) & 63) == 0) {
      const int e = j0 + D - 64 + lane;
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (e < ns) st<T>(x[c], e, yout[c]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
      for (int u = 0; u < D; ++u) cc[c][u] = cn[c][u];
      pc[c] = pn[c];
    }
  }
  const int jend = (ns + D - 1) / D * D;
  if (jend & 63) {
    const int e = (jend & ~63) + lane;
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (e < ns) st<T>(x[c], e, yout[c]);
  }
}

// solve_lower for one chain with a window of SL 64-element slots, for band
// half-widths up to 64 SL - 1: slot k of lane l holds the element 64 k past
// that of its slot 0, and the pivot row of a step may sit in any slot.  The
// coefficient row of step j is SL x 64 wide (Lm[j][k][l], c = 64 k + ((l -
// j) mod 64)).  The update is applied before the finished lane moves on, so
// that each slot meets the coefficient of the element it holds.
template <class T, int D, int SL>
__device__ __forceinline__ void solve_lower_w(gptr<cx<T>> x, gptr<const cx<T>> Lm,
                                              gptr<const int> piv, int ns, int lane) {
  const cx<T> zero = mk((T)0, (T)0);
  cx<T> b[SL], cc[SL][D], cn[SL][D];
#pragma unroll
  for (int k = 0; k < SL; ++k) {
    const int e = 64 * k + lane;
    b[k] = csel(e < ns, ld<T>(x, e < ns ? e : 0), zero);
  }
  const int e0 = 64 * SL + lane;
  cx<T> nxtA = csel(e0 < ns, ld<T>(x, e0 < ns ? e0 : 0), zero), nxt = zero, yout = zero;
  int pc = lane < D ? piv[lane] : 0, pn = 0;
#pragma unroll
  for (int u = 0; u < D; ++u)
#pragma unroll
    for (int k = 0; k < SL; ++k) cc[k][u] = ld<T>(Lm, ((long long)u * SL + k) * 64 + lane);
  for (int j0 = 0; j0 < ns; j0 += D) {
    if ((j0 & 63) == 0) {
      nxt = nxtA;
      const int e = j0 + 64 * SL + 64 + lane;
      nxtA = csel(e < ns, ld<T>(x, e < ns ? e : 0), zero);
    }
    gptr<const cx<T>> row = Lm + (long long)(j0 + D) * SL * 64 + lane;
#pragma unroll
    for (int u = 0; u < D; ++u)
#pragma unroll
      for (int k = 0; k < SL; ++k) cn[k][u] = ld<T>(row, ((long long)u * SL + k) * 64);
    pn = lane < D ? piv[j0 + D + lane] : 0;
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int j = j0 + u, lj = j & 63;
      const int p = __builtin_amdgcn_readlane(pc, u), lp = p & 63;
      const int kp = (p - j - ((lp - lj) & 63)) >> 6;  // slot of element p in lane lp
      const cx<T> bj0 = rlc(b[0], lj);                  // element j
      cx<T> bj = zero;                                  // element p: y_j
#pragma unroll
      for (int k = 0; k < SL; ++k)
        if (k == kp) bj = rlc(b[k], lp);
#pragma unroll
      for (int k = 0; k < SL; ++k)
        if (k == kp) b[k] = wlc(bj0, lp, b[k]);  // interchange: element p takes element j
      yout = wlc(bj, lj, yout);
#pragma unroll
      for (int k = 0; k < SL; ++k) b[k] = cfms(b[k], cc[k][u], bj);
#pragma unroll
      for (int k = 0; k + 1 < SL; ++k) b[k] = sel(lane == lj, b[k + 1], b[k]);
      b[SL - 1] = sel(lane == lj, nxt, b[SL - 1]);
    }
    if (((j0 + D) & 63) == 0) {
      const int e = j0 + D - 64 + lane;
      if (e < ns) st<T>(x, e, yout);
    }
#pragma unroll
    for (int u = 0; u < D; ++u)
#pragma unroll
      for (int k = 0; k < SL; ++k) cc[k][u] = cn[k][u];
    pc = pn;
  }
  const int jend = (ns + D - 1) / D * D;
  if (jend & 63) {
    const int e = (jend & ~63) + lane;
    if (e < ns) st<T>(x, e, yout);
  }
}

// Back substitution with the solve image for C chains: on entry x holds y,
// on exit U^{-1} y.  Reversed indices E = ns-1-e; S lane slots.
template <class T, int C, int D, int S>
__device__ __forceinline__ void solve_upper(gptr<cx<T>> (&x)[C], gptr<const cx<T>> (&Um)[C],
                                            gptr<const cx<T>> (&rdg)[C], int ns, int lane) {
  const cx<T> zero = mk((T)0, (T)0);
  cx<T> b[C][S], nxtA[C], nxt[C], braw[C], rd[C], cc[C][S][D], cn[C][S][D];
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const int E = 64 * k + lane;
      b[c][k] = csel(E < ns, ld<T>(x[c], E < ns ? ns - 1 - E : 0), zero);
    }
    const int E = 64 * S + lane;
    nxtA[c] = csel(E < ns, ld<T>(x[c], E < ns ? ns - 1 - E : 0), zero);
    nxt[c] = braw[c] = rd[c] = zero;
#pragma unroll
    for (int u = 0; u < D; ++u)
#pragma unroll
      for (int k = 0; k < S; ++k) cc[c][k][u] = ld<T>(Um[c], ((long long)u * S + k) * 64 + lane);
  }
  for (int J0 = 0; J0 < ns; J0 += D) {
    if ((J0 & 63) == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        nxt[c] = nxtA[c];
        const int E = J0 + 64 * S + 64 + lane;
        nxtA[c] = csel(E < ns, ld<T>(x[c], E < ns ? ns - 1 - E : 0), zero);
        rd[c] = ld<T>(rdg[c], J0 + lane);
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      gptr<const cx<T>> row = Um[c] + (long long)(J0 + D) * S * 64 + lane;
#pragma unroll
      for (int u = 0; u < D; ++u)
#pragma unroll
        for (int k = 0; k < S; ++k) cn[c][k][u] = ld<T>(row, ((long long)u * S + k) * 64);
    }
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int lJ = (J0 + u) & 63;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const cx<T> bJ = rlc(b[c][0], lJ);
        braw[c] = wlc(bJ, lJ, braw[c]);
#pragma unroll
        for (int k = 0; k < S; ++k) b[c][k] = cfms(b[c][k], cc[c][k][u], bJ);
#pragma unroll
        for (int k = 0; k + 1 < S; ++k) b[c][k] = sel(lane == lJ, b[c][k + 1], b[c][k]);
        b[c][S - 1] = sel(lane == lJ, nxt[c], b[c][S - 1]);
      }
    }
    if (((J0 + D) & 63) == 0) {  // x_j = b_j / U_jj for a complete 64-block
      const int E = J0 + D - 64 + lane;
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (E < ns) st<T>(x[c], ns - 1 - E, braw[c] * rd[c]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int u = 0; u < D; ++u)
#pragma unroll
        for (int k = 0; k < S; ++k) cc[c][k][u] = cn[c][k][u];
  }
  const int Jend = (ns + D - 1) / D * D;
  if (Jend & 63) {
    const int E = (Jend & ~63) + lane;
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (E < ns) st<T>(x[c], ns - 1 - E, braw[c] * rd[c]);
  }
}

// Sum of a complex partial over the four 16-lane groups of the wave, both
// parts in one pass.  v_permlane16_swap exchanges rows 1 and 3 of its first
// operand with rows 0 and 2 of its second, so with (re, im) as operands the
// two results hold the real parts of rows 0/2 and the imaginary parts of rows
// 1/3, and the real parts of rows 1/3 and the imaginary parts of rows 0/2;
// v_permlane32_swap then does the same with the two halves of the wave.  Lane
// r + 16 p ends with the real part of the sum when p is even and the imaginary
// part when p is odd, (g0 + g1) + (g2 + g3) in every lane.
__device__ __forceinline__ float sum4c(float re, float im) {
  const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(re), __float_as_uint(im), false,
                                                  false);
  const float s = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  const unsigned w = __float_as_uint(s);
  const auto b = __builtin_amdgcn_permlane32_swap(w, w, false, false);
  return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}
__device__ __forceinline__ double sum4c(double re, double im) {
  const unsigned long long ur = __double_as_longlong(re), ui = __double_as_longlong(im);
  const auto al = __builtin_amdgcn_permlane16_swap((unsigned)ur, (unsigned)ui, false, false);
  const auto ah = __builtin_amdgcn_permlane16_swap((unsigned)(ur >> 32), (unsigned)(ui >> 32), false,
                                                   false);
  const double s = __longlong_as_double(((long long)ah[0] << 32) | al[0]) +
                   __longlong_as_double(((long long)ah[1] << 32) | al[1]);
  const unsigned long long w = __double_as_longlong(s);
  const unsigned wl = (unsigned)w, wh = (unsigned)(w >> 32);
  const auto bl = __builtin_amdgcn_permlane32_swap(wl, wl, false, false);
  const auto bh = __builtin_amdgcn_permlane32_swap(wh, wh, false, false);
  return __longlong_as_double(((long long)bh[0] << 32) | bl[0]) +
         __longlong_as_double(((long long)bh[1] << 32) | bl[1]);
}

// Blocked row substitution for an unpivoted strip (image layout in
// factor.hip): out_i = d_i (in_i - sum_{c=1..K} T(i, c) out_{i-c}) in blocks
// of B = 16 outputs, each a dense map of the K previous outputs and the 16
// block inputs.  Lane l = r + 16 p accumulates KP terms of output r, and the
// four partial sums of a row are combined by lane swaps (sum4c), after which
// lanes with even p hold the real and lanes with odd p the imaginary part.
//
// Only the four terms of a lane that involve the previous block's outputs lie
// on the chain from block to block; the other KP - 4 terms of block b+1
// (its inputs and the outputs older than block b) are accumulated while block
// b completes.  Outputs and inputs live in two 256-entry LDS rings (position i
// at slot i & 255) whose first 64 slots are mirrored into slots 256..319, so
// that the consecutive reads of a lane (at most 20) never wrap and use
// immediate offsets.  init (LDS, K entries, or null for zeros) holds the
// outputs of positions -K..-1, i.e. the state the recurrence starts from.
//
// The loop runs in steps of U blocks (R = 16 U rows).  Everything a step
// needs from memory is requested NB - 1 steps earlier, at the start of a
// previous step: the maps of its U blocks (NB register buffers, the loop
// unrolled by NB steps so that the buffers keep fixed registers) and 64
// inputs, which enter the input ring at its own start (step j commits rows
// jR + 128 .. jR + 191, so the ring spans at most 192 rows).  The outputs of
// a step are written back at the start of the next one.  Issuing all memory
// traffic of a step together keeps the loop-carried waits short: whatever the
// hardware counters make the loop head wait for was requested at least one
// whole step before.  The map array ends
// in zero blocks and reads past the end are clamped, so the body is free of
// bounds tests (positions past ns meet only zero map entries: rows >= ns of a
// map are zero and no row < ns depends on a later position).  Single wave:
// the LDS accesses of one wave are performed in order, no barrier is needed.
// Rows are read through src and written through dst (lanes past the end
// write row ns-1 again, with the same value, so the write needs no branch).
//
// The reads that start the recurrence (the first 128 input rows, the inputs
// and maps of the first NB - 1 steps) can be issued ahead, into a
// BlockedPre, by blocked_fetch_maps and blocked_fetch_inputs; solve_blocked
// issues them itself, solve_blocked_run takes them prefetched.
template <class T, int KP, int U, int NB, class Src>
struct BlockedPre {
  typename Src::P in0, in1;  // rows lane and 64 + lane
  typename Src::P pend[NB];  // pend[j % NB]: input rows jR + 128 + lane until step j
  cx<T> g[NB][U][KP];
  gptr<const cx<T>> gp;      // maps of the next step to request
};

template <class T, int KP, int U, int NB, class Src>
__device__ __forceinline__ void blocked_fetch_maps(BlockedPre<T, KP, U, NB, Src>& pre,
                                                   gptr<const cx<T>> G, int lane) {
  pre.gp = G + lane;
#pragma unroll
  for (int b = 0; b + 1 < NB; ++b) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < KP; ++t) pre.g[b][u][t] = ld<T>(pre.gp, (long long)(u * KP + t) * 64);
    pre.gp = pre.gp + (long long)U * KP * 64;
  }
}

template <class T, int KP, int U, int NB, class Src>
__device__ __forceinline__ void blocked_fetch_inputs(BlockedPre<T, KP, U, NB, Src>& pre,
                                                     const Src& src, int lane) {
  constexpr int R = U * 16;
  pre.in0 = src.load(lane);
  pre.in1 = src.load(64 + lane);
#pragma unroll
  for (int b = 0; b + 1 < NB; ++b) pre.pend[b] = src.load(b * R + 128 + lane);
}

template <class T, int KP, int U, int NB, class Src, class Dst>
__device__ __forceinline__ void solve_blocked_run(BlockedPre<T, KP, U, NB, Src>& pre,
                                                  const Src& src, const Dst& dst, int ns, int K,
                                                  cx<T>* ring, const cx<T>* init, int lane) {
  static_assert(HH_BLK == 16 && KP >= 8, "four lane groups of 16 rows, four chain terms each");
  constexpr int R = U * 16, KO = KP - 8;
  static_assert(R <= 64 && 64 % R == 0 && NB >= 2, "a step divides 64 rows");
  cx<T>* oring = ring;
  cx<T>* iring = ring + 320;
  const cx<T> zero = mk((T)0, (T)0);
  const int r = lane & 15, p = lane >> 4;
  const int nst = (ns + R - 1) / R;
  auto put = [&](cx<T>* rg, int i, cx<T> v) {
    const int k = i & 255;
    rg[k] = v;
    rg[k < 64 ? k + 256 : k] = v;
  };
  auto put_part = [&](cx<T>* rg, int i, int part, T v) {  // one component of entry i
    const int k = i & 255;
    T* base = reinterpret_cast<T*>(rg) + part;
    base[2 * k] = v;
    base[2 * (k < 64 ? k + 256 : k)] = v;
  };
#pragma unroll
  for (int q = 0; q < 10; ++q) ring[64 * q + lane] = zero;
  if (init && lane < K) put(oring, lane - K, init[lane]);
  put(iring, lane, src.get(pre.in0));
  put(iring, 64 + lane, src.get(pre.in1));
  auto& pend = pre.pend;
  auto& g = pre.g;
  auto& gp = pre.gp;
  // terms of block i0 that do not involve the outputs of the block before it
  auto rest = [&](const cx<T>(&gb)[KP], int i0) -> cx<T> {
    const cx<T>* in = iring + ((i0 + 4 * p) & 255);
    const cx<T>* old = oring + ((i0 - K + p * KO) & 255);
    cx<T> a0 = cmulx(gb[4], in[0]), a1 = cmulx(gb[5], in[1]);
    a0 = cfma(a0, gb[6], in[2]);
    a1 = cfma(a1, gb[7], in[3]);
#pragma unroll
    for (int t = 0; t < KO; t += 2) {
      a0 = cfma(a0, gb[8 + t], old[t]);
      if (t + 1 < KO) a1 = cfma(a1, gb[9 + t], old[t + 1]);
    }
    return a0 + a1;
  };
  cx<T> rst = rest(g[0][0], 0);
  const int nstr = (nst + NB - 1) / NB * NB;
  for (int j0 = 0; j0 < nstr; j0 += NB) {
#pragma unroll
    for (int h = 0; h < NB; ++h) {
      const int j = j0 + h;
      if (j >= nst) break;  // the unrolled group may overrun the last step
      // requests NB-1 steps ahead: maps and inputs; write-back of the last step
      const int hn = (h + NB - 1) % NB;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < KP; ++t) g[hn][u][t] = ld<T>(gp, (long long)(u * KP + t) * 64);
      gp = gp + (long long)U * KP * 64;
      put(iring, j * R + 128 + lane, src.get(pend[h]));
      pend[hn] = src.load((j + NB - 1) * R + 128 + lane);
      if (j > 0) {
        const int q = (j - 1) * R + (lane & (R - 1)), qs = q < ns ? q : ns - 1;
        dst.put(qs, oring[qs & 255]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i0 = j * R + 16 * u;
        const cx<T>* pv = oring + ((i0 - 16 + 4 * p) & 255);
        cx<T> a0 = cfma(rst, g[h][u][0], pv[0]), a1 = cmulx(g[h][u][1], pv[1]);
        a0 = cfma(a0, g[h][u][2], pv[2]);
        a1 = cfma(a1, g[h][u][3], pv[3]);
        const cx<T> part = a0 + a1;
        const T half = sum4c(part.re, part.im);  // real part (p even) or imaginary part (p odd)
        if (u + 1 < U)
          rst = rest(g[h][u + 1 < U ? u + 1 : u], i0 + 16);
        else
          rst = rest(g[(h + 1) % NB][0], i0 + 16);
        put_part(oring, i0 + r, p & 1, half);
      }
    }
  }
  const int q = (nst - 1) * R + (lane & (R - 1)), qs = q < ns ? q : ns - 1;
  dst.put(qs, oring[qs & 255]);
}

template <class T, int KP, int U, int NB, class Src, class Dst>
__device__ __forceinline__ void solve_blocked(const Src& src, const Dst& dst, gptr<const cx<T>> G,
                                              int ns, int K, cx<T>* ring, const cx<T>* init,
                                              int lane) {
  BlockedPre<T, KP, U, NB, Src> pre;
  blocked_fetch_inputs(pre, src, lane);
  blocked_fetch_maps(pre, G, lane);
  solve_blocked_run(pre, src, dst, ns, K, ring, init, lane);
}

// g = sum_d coef_d z[p + off_d] on interface node (i, j) = p.
template <class T, class A = PlainAcc>
__device__ __forceinline__ cx<T> transmission(gptr<const cx<T>> coef, gptr<cx<T>> z, int i, int j,
                                              int n) {
  const int di[7] = {-1, 0, -1, 0, 1, 0, 1};
  const int dj[7] = {-1, -1, 0, 0, 0, 1, 1};
  cx<T> g = mk((T)0, (T)0);
#pragma unroll
  for (int d = 0; d < 7; ++d) {
    const int ii = i + di[d], jj = j + dj[d];
    if (ii < 0 || ii >= n || jj < 0 || jj >= n) continue;
    g = cfma(g, ld<T>(coef, d), A::load((gptr<const cx<T>>)z, (long long)jj * n + ii));
  }
  return g;
}

// q = l w + t with 0 <= t < w, from a float estimate of q / w: the estimate is
// off by at most one for q < 2^22, which one correction step absorbs.
__device__ __forceinline__ void line_of(int q, int w, float winv, int& l, int& t) {
  l = (int)((float)q * winv);
  t = q - l * w;
  if (t < 0) {
    --l;
    t += w;
  } else if (t >= w) {
    ++l;
    t -= w;
  }
}

// Streams of the blocked substitution.  load(i) issues the memory reads of
// row i (clamped to the last row) and returns them raw; get() forms the value
// when the row enters the ring, one step later.
template <class T, class A = PlainAcc>
struct SrcVec {  // x[i] (rev: x[ns-1-i]) in the working precision
  gptr<const cx<T>> x;
  int ns;
  bool rev;
  using P = cx<T>;
  __device__ P load(int i) const {
    i = i < ns ? i : ns - 1;
    return A::load(x, rev ? ns - 1 - i : i);
  }
  __device__ cx<T> get(const P& v) const { return v; }
};
template <class T>
struct SrcC128 {  // strip-local FP64 right-hand side (nr rows), forward order
  gptr<const c128> b;
  int nr;
  using P = c128;
  __device__ P load(int i) const {  // zero on the identity rows past nr
    const int q = i < nr ? i : nr - 1;
    const c128 v = mk(b[q].re, b[q].im);
    return i < nr ? v : mk(0.0, 0.0);
  }
  __device__ cx<T> get(const P& v) const { return mk((T)v.re, (T)v.im); }
};
// Strip right-hand side R_s r + g, forward order: local row q = l w + t is the
// global node (a + t, l) of an x strip or (l, a + t) of a y strip; the
// transmission data of node line l sit in LDS (e1 on t = 0 where the strip has
// a Gamma_{s,1} side, e2 on t = w - 1 where Gamma_{s,2} data apply).  Rows
// past the nr unknowns (identity rows) read zero.
template <class T>
struct SrcGather {
  gptr<const c128> r;
  const cx<T>* gl1;
  const cx<T>* gl2;
  int nr, w, n, a, dir;
  bool use1, use2;
  struct P {
    c128 v;
    int l;
    bool f1, f2;
  };
  float winv;  // 1 / w
  // the global read is issued at load, the transmission data (LDS) are read
  // at get, so that loads may run ahead of the transmission data
  __device__ P load(int i) const {
    const bool in = i < nr;
    const int q = in ? i : nr - 1;
    int l, t;
    line_of(q, w, winv, l, t);
    const long long p = dir == 0 ? (long long)l * n + a + t : (long long)(a + t) * n + l;
    const c128 v = mk(r[p].re, r[p].im);
    P o;
    o.v = in ? v : mk(0.0, 0.0);
    o.l = l;
    o.f1 = in && use1 && t == 0;
    o.f2 = in && use2 && t == w - 1;
    return o;
  }
  __device__ cx<T> get(const P& o) const {
    const cx<T> v = mk((T)o.v.re, (T)o.v.im);
    const cx<T> e = csel(o.f1, gl1[o.l], gl2[o.l]);
    return o.f1 || o.f2 ? v + e : v;
  }
};
template <class T, class A = PlainAcc>
struct DstVec {  // x[i] (rev: x[ns-1-i])
  gptr<cx<T>> x;
  int ns;
  bool rev;
  __device__ void put(int i, cx<T> v) const { A::store(x, rev ? ns - 1 - i : i, v); }
  __device__ cx<T> get(int i) const { return A::load((gptr<const cx<T>>)x, rev ? ns - 1 - i : i); }
};
template <class T>
struct DstC128 {  // strip-local FP64 output (nr rows), reversed order over ns rows
  gptr<c128> x;
  int ns, nr;
  __device__ void put(int i, cx<T> v) const {  // identity rows (q >= nr) are dropped
    const int q = ns - 1 - i;
    if (q >= nr) return;
    x[q].re = (double)v.re;
    x[q].im = (double)v.im;
  }
  __device__ cx<T> get(int i) const {  // exact: the value put was of this precision
    const int q = ns - 1 - i;
    if (q >= nr) return mk((T)0, (T)0);
    return mk((T)x[q].re, (T)x[q].im);
  }
};
// Scatter of the strip solution over the global vector, reversed order (the
// back substitution produces the last local row first); the identity rows
// (q >= nr, which come first) are dropped and read back as zero, their value.
template <class T, class A = PlainAcc>
struct DstScatter {
  gptr<cx<T>> z;
  int ns, nr, w, n, a, dir;
  float winv;  // 1 / w
  __device__ long long pos(int q) const {
    int l, t;
    line_of(q, w, winv, l, t);
    return dir == 0 ? (long long)l * n + a + t : (long long)(a + t) * n + l;
  }
  __device__ void put(int i, cx<T> v) const {
    const int q = ns - 1 - i;
    if (q < nr) A::store(z, pos(q), v);
  }
  __device__ cx<T> get(int i) const {
    const int q = ns - 1 - i;
    const cx<T> v = A::load((gptr<const cx<T>>)z, pos(q < nr ? q : 0));
    return q < nr ? v : mk((T)0, (T)0);
  }
};

// Rows base .. base + cnt - 1 of a strip vector held in LDS (the wide plan's
// forward outputs of one workgroup): DstLds in forward order, SrcLdsRev as
// the back substitution reads them (x[ns - 1 - i]).
template <class T>
struct DstLds {
  cx<T>* v;
  int base;
  __device__ void put(int i, cx<T> x) const { v[i - base] = x; }
  __device__ cx<T> get(int i) const { return v[i - base]; }
};
template <class T>
struct SrcLdsRev {
  const cx<T>* v;
  int ns, base;
  using P = cx<T>;
  __device__ P load(int i) const { return v[ns - 1 - i - base]; }
  __device__ cx<T> get(const P& x) const { return x; }
};

// Segment views for the parallel substitution: rows off..off+len-1 of a
// stream as rows 0..len-1 (reads past the end clamped to the last row).
template <class Src>
struct SegSrc {
  const Src& b;
  int off, len;
  using P = typename Src::P;
  __device__ P load(int i) const { return b.load(off + (i < len ? i : len - 1)); }
  __device__ auto get(const P& v) const { return b.get(v); }
};
template <class T, class Dst>
struct SegDst {
  const Dst& b;
  int off;
  __device__ void put(int i, cx<T> v) const { b.put(off + i, v); }
  __device__ cx<T> get(int i) const { return b.get(off + i); }
};
template <class T, class Dst>
struct SegDstIf {  // SegDst whose stores are dropped unless on
  const Dst& b;
  int off;
  bool on;
  __device__ void put(int i, cx<T> v) const {
    if (on) b.put(off + i, v);
  }
  __device__ cx<T> get(int i) const { return b.get(off + i); }
};
template <class T>
struct DstTail {  // keeps only the last K rows of a segment (in LDS)
  cx<T>* yt;
  int len, K;
  __device__ void put(int i, cx<T> v) const {
    const int c = i - (len - K);
    if (c >= 0) yt[c] = v;
  }
};

// v = y + M x in lane c < K (row c; zero in the other lanes), y being the
// lane's own entry: M is KM x KM, column-major (element (c, c') at c' KM + c)
// and zero beyond K, x is zero beyond K (both in LDS).  With KM <= 32 two
// lanes share a row (lane c + 32 h sums the columns c' = h mod 2) and one lane
// swap adds the halves.  Unrolled in chunks of columns (sized for the
// register file): every LDS read has a fixed offset and a chunk's reads are
// issued before its products.
template <class T, int KM>
__device__ __forceinline__ cx<T> map_apply(const cx<T>* M, const cx<T>* x, cx<T> y, int K,
                                           int lane) {
  constexpr int H = KM <= 32 ? 2 : 1, NC = KM / H;
  constexpr int CH = sizeof(T) == 8 ? 4 : (NC <= 16 ? NC : 16);
  static_assert(NC % CH == 0, "column chunks");
  const cx<T> zero = mk((T)0, (T)0);
  const int c = H == 2 ? (lane & 31) : lane, h = H == 2 ? (lane >> 5) : 0;
  const cx<T>* Mb = M + h * KM + (c < KM ? c : 0);
  const cx<T>* xb = x + h;
  cx<T> a[4] = {zero, zero, zero, zero};
  for (int q0 = 0; q0 < NC; q0 += CH) {
#pragma unroll
    for (int q = 0; q < CH; ++q)
      a[q & 3] = cfma(a[q & 3], Mb[(q0 + q) * H * KM], xb[(q0 + q) * H]);
  }
  cx<T> v = (a[0] + a[1]) + (a[2] + a[3]);
  if (H == 2) v = v + mk(__shfl_xor(v.re, 32), __shfl_xor(v.im, 32));
  return csel(lane < K, v + y, zero);
}

// outputs += Phi_c s_c over the rows 0..len-1 of a segment (lane = row), RB
// blocks of 64 rows at a time with all their response loads issued together
// (the correction is bound by those loads' latency), each row's KM terms
// into four partial sums in a fixed order, so that the tiles of k_sweep_n and
// plan 0 agree bit for bit.  Phi_c[k][i] at k seg + i, zero-padded to KM rows
// (the padding adds exact zeros); sc: the state (LDS, zero beyond K).  The
// zero-start outputs come from in (the destination itself where that is a
// contiguous vector, else a contiguous scratch, so that a scattered
// destination is written once).
// KC terms of RB row blocks in flight, sized to what the kernels' register
// files leave (KC a multiple of four dividing KM: the order of a row's terms
// is the same whatever the shape, so plan 0 and the tiles still agree).  The
// loop over chunks stays rolled: unrolled, the scheduler hoists every chunk's
// loads to the top and the kernels spill.
template <class T, int KM, int NR>
struct ResponseShape {
  static constexpr bool dbl = sizeof(T) == 8;
  static constexpr int KC = dbl ? (KM == 24 ? 8 : 16)
                                : NR == 1 ? (KM == 48 ? 16 : KM == 64 ? 32 : KM)
                                          : (KM <= 24 ? KM : 16);
  static constexpr int RB = dbl ? (KM == 24 ? 2 : 1)
                                : NR == 1 ? (KM == 16 ? 4 : KM == 24 || KM == 48 ? 2 : 1)
                                          : (KM == 16 ? 2 : 1);
  static_assert(KC % 4 == 0 && KM % KC == 0, "whole chunks of four terms");
};
template <class T, int KM, class Out, class In>
__device__ __forceinline__ void add_response(const Out& out, const In& in, int len, int seg,
                                             gptr<const cx<T>> Ph, const cx<T>* sc, int lane) {
  constexpr int KC = ResponseShape<T, KM, 1>::KC, RB = ResponseShape<T, KM, 1>::RB;
  const cx<T> zero = mk((T)0, (T)0);
  for (int i0 = 0; i0 < len; i0 += 64 * RB) {
    int ic[RB];
    cx<T> a[RB][4];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int i = i0 + 64 * b + lane;
      ic[b] = i < len ? i : len - 1;
      a[b][0] = in.get(ic[b]);
      a[b][1] = a[b][2] = a[b][3] = zero;
    }
#pragma unroll 1
    for (int k0 = 0; k0 < KM; k0 += KC) {
      cx<T> pv[RB][KC];
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int q = 0; q < KC; ++q) pv[b][q] = ld<T>(Ph, (long long)(k0 + q) * seg + ic[b]);
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int q = 0; q < KC; ++q) a[b][q & 3] = cfma(a[b][q & 3], pv[b][q], sc[k0 + q]);
    }
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int i = i0 + 64 * b + lane;
      if (i < len) out.put(i, (a[b][0] + a[b][1]) + (a[b][2] + a[b][3]));
    }
  }
}

// add_response for the NR right-hand sides of a tile: per right-hand side the
// same operations in the same order, the responses read once for all, and
// every zero-start output read before any corrected one is written (a tile
// of one repeats its chain: both then read the same value and write the same
// result).
template <class T, int KM, int NR, class Out, class In>
__device__ __forceinline__ void add_response_n(const Out (&out)[NR], const In (&in)[NR], int len,
                                               int seg, gptr<const cx<T>> Ph,
                                               const cx<T>* const (&sc)[NR], int lane) {
  constexpr int KC = ResponseShape<T, KM, NR>::KC, RB = ResponseShape<T, KM, NR>::RB;
  const cx<T> zero = mk((T)0, (T)0);
  for (int i0 = 0; i0 < len; i0 += 64 * RB) {
    int ic[RB];
    cx<T> a[RB][NR][4];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int i = i0 + 64 * b + lane;
      ic[b] = i < len ? i : len - 1;
#pragma unroll
      for (int v = 0; v < NR; ++v) {
        a[b][v][0] = in[v].get(ic[b]);
        a[b][v][1] = a[b][v][2] = a[b][v][3] = zero;
      }
    }
#pragma unroll 1
    for (int k0 = 0; k0 < KM; k0 += KC) {
      cx<T> pv[RB][KC];
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int q = 0; q < KC; ++q) pv[b][q] = ld<T>(Ph, (long long)(k0 + q) * seg + ic[b]);
#pragma unroll
      for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int v = 0; v < NR; ++v)
#pragma unroll
          for (int q = 0; q < KC; ++q)
            a[b][v][q & 3] = cfma(a[b][v][q & 3], pv[b][q], sc[v][k0 + q]);
    }
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const int i = i0 + 64 * b + lane;
      if (i < len) {
#pragma unroll
        for (int v = 0; v < NR; ++v)
          out[v].put(i, (a[b][v][0] + a[b][v][1]) + (a[b][v][2] + a[b][v][3]));
      }
    }
  }
}

// One triangular substitution of a strip by all P waves of the workgroup,
// segment plan 0 (the recurrence is linear, so it splits exactly over
// segments of seg rows):
//  1. every segment runs from a zero state and writes its outputs (segment
//     0's state is the true one, so its outputs are final); the tails (last
//     K outputs) of all but the last go to yt;
//  2. wave 0 propagates the true states, state_{s+1} = tail_s + T_s state_s,
//     with the transfer maps T_s staged into LDS;
//  3. segments 1.. add their response Phi_s times their state (the outputs of
//     the segment started from the unit states with zero inputs).
// The chain of one strip is one blocked substitution of seg rows, about ns / P
// (a second substitution in place of phase 3 would double it).  work: the
// LDS shared by the rings (phase 1, 640 entries per wave) and the staged maps
// (phase 2, KM x KM each); yt, stt: 64 entries per segment.
template <class T, int KP, int U, int NB, class Src, class Dst, class Tmp>
__device__ __forceinline__ void solve_triangle(const Src& src, const Dst& dst, const Tmp& tmp,
                                               const cx<T>* G, const cx<T>* Tm, const cx<T>* Ph,
                                               int ns, int K, int seg, cx<T>* work, cx<T>* yt,
                                               cx<T>* stt) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nthr = blockDim.x;
  const int nseg = (ns + seg - 1) / seg;
  cx<T>* ring = work + 640 * wv;
  const int off = wv * seg, len = ns - off < seg ? ns - off : seg;
  gptr<const cx<T>> Gw = (gptr<const cx<T>>)(G + (long long)(off / 16) * KP * 64);
  if (wv == 0) {
    solve_blocked<T, KP, U, NB>(SegSrc<Src>{src, 0, len}, SegDst<T, Dst>{dst, 0}, Gw, len, K, ring,
                            (const cx<T>*)nullptr, lane);
  } else if (wv < nseg) {
    solve_blocked<T, KP, U, NB>(SegSrc<Src>{src, off, len}, SegDst<T, Tmp>{tmp, off}, Gw, len, K,
                            ring, (const cx<T>*)nullptr, lane);
  }
  if (wv < nseg - 1 && lane < K) yt[64 * wv + lane] = ring[(len - K + lane) & 255];
  if (nseg == 1) return;
  __syncthreads();
  constexpr int KM = map_dim(KP);
  const int nT = (nseg - 2) * KM * KM;
  gptr<const cx<T>> Tg = (gptr<const cx<T>>)Tm;
  for (int e0 = 0; e0 < nT; e0 += 8 * nthr) {
    cx<T> v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + q * nthr + tid;
      v[q] = ld<T>(Tg, e < nT ? e : nT - 1);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + q * nthr + tid;
      if (e < nT) work[e] = v[q];
    }
  }
  __syncthreads();
  if (wv == 0) {
    for (int s = 1; s < nseg; ++s) {
      const cx<T> y = lane < K ? yt[64 * (s - 1) + lane] : mk((T)0, (T)0);
      stt[64 * s + lane] =
          s >= 2 ? map_apply<T, KM>(work + (s - 2) * KM * KM, stt + 64 * (s - 1), y, K, lane) : y;
    }
  }
  __syncthreads();
  // the rings were overwritten by the staged maps: the zero-start outputs
  // come back from tmp
  if (wv >= 1 && wv < nseg)
    add_response<T, KM>(SegDst<T, Dst>{dst, off}, SegDst<T, Tmp>{tmp, off}, len, seg,
                        (gptr<const cx<T>>)(Ph + (long long)(wv - 1) * seg * KM), stt + 64 * wv,
                        lane);
}

// ---------------------------------------------------------------- RHS tiles
// The blocked substitution for NR right-hand sides at once (one wave, the
// same strip): every map row the wave reads feeds all NR of them, and their
// NR independent recurrences fill the wave's latency.  Per right-hand side
// the operations are those of solve_blocked_run in the same order, so the
// results are bitwise those of NR separate substitutions.  ring: NR rings of
// 640 entries; init[v]: state of right-hand side v (LDS) or null.
template <class T, int KP, int U, int NB, int NR, class Src>
struct BlockedPreN {
  typename Src::P in0[NR], in1[NR];
  typename Src::P pend[NB][NR];
  cx<T> g[NB][U][KP];
  gptr<const cx<T>> gp;
};

template <class T, int KP, int U, int NB, int NR, class Src, class Dst>
__device__ __forceinline__ void solve_blocked_n(const Src (&src)[NR], const Dst (&dst)[NR],
                                                gptr<const cx<T>> G, int ns, int K, cx<T>* ring,
                                                const cx<T>* const (&init)[NR], int lane) {
  static_assert(HH_BLK == 16 && KP >= 8, "four lane groups of 16 rows, four chain terms each");
  constexpr int R = U * 16, KO = KP - 8;
  static_assert(R <= 64 && 64 % R == 0 && NB >= 2, "a step divides 64 rows");
  BlockedPreN<T, KP, U, NB, NR, Src> pre;
#pragma unroll
  for (int v = 0; v < NR; ++v) {
    pre.in0[v] = src[v].load(lane);
    pre.in1[v] = src[v].load(64 + lane);
#pragma unroll
    for (int b = 0; b + 1 < NB; ++b) pre.pend[b][v] = src[v].load(b * R + 128 + lane);
  }
  pre.gp = G + lane;
#pragma unroll
  for (int b = 0; b + 1 < NB; ++b) {
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < KP; ++t) pre.g[b][u][t] = ld<T>(pre.gp, (long long)(u * KP + t) * 64);
    pre.gp = pre.gp + (long long)U * KP * 64;
  }
  const cx<T> zero = mk((T)0, (T)0);
  const int r = lane & 15, p = lane >> 4;
  const int nst = (ns + R - 1) / R;
  auto put = [&](cx<T>* rg, int i, cx<T> v) {
    const int k = i & 255;
    rg[k] = v;
    rg[k < 64 ? k + 256 : k] = v;
  };
  auto put_part = [&](cx<T>* rg, int i, int part, T v) {
    const int k = i & 255;
    T* base = reinterpret_cast<T*>(rg) + part;
    base[2 * k] = v;
    base[2 * (k < 64 ? k + 256 : k)] = v;
  };
#pragma unroll
  for (int v = 0; v < NR; ++v) {
    cx<T>* oring = ring + 640 * v;
    cx<T>* iring = oring + 320;
#pragma unroll
    for (int q = 0; q < 10; ++q) oring[64 * q + lane] = zero;
    if (init[v] && lane < K) put(oring, lane - K, init[v][lane]);
    put(iring, lane, src[v].get(pre.in0[v]));
    put(iring, 64 + lane, src[v].get(pre.in1[v]));
  }
  auto& pend = pre.pend;
  auto& g = pre.g;
  auto& gp = pre.gp;
  auto rest = [&](const cx<T>(&gb)[KP], int i0, int v) -> cx<T> {
    const cx<T>* oring = ring + 640 * v;
    const cx<T>* in = oring + 320 + ((i0 + 4 * p) & 255);
    const cx<T>* old = oring + ((i0 - K + p * KO) & 255);
    cx<T> a0 = cmulx(gb[4], in[0]), a1 = cmulx(gb[5], in[1]);
    a0 = cfma(a0, gb[6], in[2]);
    a1 = cfma(a1, gb[7], in[3]);
#pragma unroll
    for (int t = 0; t < KO; t += 2) {
      a0 = cfma(a0, gb[8 + t], old[t]);
      if (t + 1 < KO) a1 = cfma(a1, gb[9 + t], old[t + 1]);
    }
    return a0 + a1;
  };
  cx<T> rst[NR];
#pragma unroll
  for (int v = 0; v < NR; ++v) rst[v] = rest(g[0][0], 0, v);
  const int nstr = (nst + NB - 1) / NB * NB;
  for (int j0 = 0; j0 < nstr; j0 += NB) {
#pragma unroll
    for (int h = 0; h < NB; ++h) {
      const int j = j0 + h;
      if (j >= nst) break;
      const int hn = (h + NB - 1) % NB;
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < KP; ++t) g[hn][u][t] = ld<T>(gp, (long long)(u * KP + t) * 64);
      gp = gp + (long long)U * KP * 64;
#pragma unroll
      for (int v = 0; v < NR; ++v) {
        cx<T>* iring = ring + 640 * v + 320;
        put(iring, j * R + 128 + lane, src[v].get(pend[h][v]));
        pend[hn][v] = src[v].load((j + NB - 1) * R + 128 + lane);
        if (j > 0) {
          const int q = (j - 1) * R + (lane & (R - 1)), qs = q < ns ? q : ns - 1;
          dst[v].put(qs, ring[640 * v + (qs & 255)]);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i0 = j * R + 16 * u;
#pragma unroll
        for (int v = 0; v < NR; ++v) {
          cx<T>* oring = ring + 640 * v;
          const cx<T>* pv = oring + ((i0 - 16 + 4 * p) & 255);
          cx<T> a0 = cfma(rst[v], g[h][u][0], pv[0]), a1 = cmulx(g[h][u][1], pv[1]);
          a0 = cfma(a0, g[h][u][2], pv[2]);
          a1 = cfma(a1, g[h][u][3], pv[3]);
          const cx<T> part = a0 + a1;
          const T half = sum4c(part.re, part.im);
          if (u + 1 < U)
            rst[v] = rest(g[h][u + 1 < U ? u + 1 : u], i0 + 16, v);
          else
            rst[v] = rest(g[(h + 1) % NB][0], i0 + 16, v);
          put_part(oring, i0 + r, p & 1, half);
        }
      }
    }
  }
  const int q = (nst - 1) * R + (lane & (R - 1)), qs = q < ns ? q : ns - 1;
#pragma unroll
  for (int v = 0; v < NR; ++v) dst[v].put(qs, ring[640 * v + (qs & 255)]);
}

// solve_triangle for NR right-hand sides of the same strip (segment plan 0):
// the same three phases, each wave carrying its segment for all NR; the
// transfer maps are staged once, the responses read once per 64 rows for
// both.  work: max(640 P NR, (P - 2) KM^2) entries; yt, stt: 64 P entries per
// right-hand side (right-hand side v at 64 P v).
template <class T, int KP, int U, int NB, int NR, class Src, class Dst, class Tmp>
__device__ __forceinline__ void solve_triangle_n(const Src (&src)[NR], const Dst (&dst)[NR],
                                                 const Tmp (&tmp)[NR], const cx<T>* G,
                                                 const cx<T>* Tm, const cx<T>* Ph, int ns, int K,
                                                 int seg, cx<T>* work, cx<T>* yt, cx<T>* stt) {
  static_assert(NR == 2, "tiles of two right-hand sides (what the register budget allows)");
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nthr = blockDim.x;
  const int P = nthr >> 6;
  const int nseg = (ns + seg - 1) / seg;
  cx<T>* ring = work + 640 * NR * wv;
  const int off = wv * seg, len = ns - off < seg ? ns - off : seg;
  gptr<const cx<T>> Gw = (gptr<const cx<T>>)(G + (long long)(off / 16) * KP * 64);
  const cx<T>* none[NR];
#pragma unroll
  for (int v = 0; v < NR; ++v) none[v] = nullptr;
  if (wv == 0) {
    SegSrc<Src> ss[NR] = {SegSrc<Src>{src[0], 0, len}, SegSrc<Src>{src[NR - 1], 0, len}};
    SegDst<T, Dst> sd[NR] = {SegDst<T, Dst>{dst[0], 0}, SegDst<T, Dst>{dst[NR - 1], 0}};
    solve_blocked_n<T, KP, U, NB, NR>(ss, sd, Gw, len, K, ring, none, lane);
  } else if (wv < nseg) {
    SegSrc<Src> ss[NR] = {SegSrc<Src>{src[0], off, len}, SegSrc<Src>{src[NR - 1], off, len}};
    SegDst<T, Tmp> sd[NR] = {SegDst<T, Tmp>{tmp[0], off}, SegDst<T, Tmp>{tmp[NR - 1], off}};
    solve_blocked_n<T, KP, U, NB, NR>(ss, sd, Gw, len, K, ring, none, lane);
  }
  if (wv < nseg - 1 && lane < K) {
#pragma unroll
    for (int v = 0; v < NR; ++v)
      yt[64 * P * v + 64 * wv + lane] = ring[640 * v + ((len - K + lane) & 255)];
  }
  if (nseg == 1) return;
  __syncthreads();
  constexpr int KM = map_dim(KP);
  const int nT = (nseg - 2) * KM * KM;
  gptr<const cx<T>> Tg = (gptr<const cx<T>>)Tm;
  for (int e0 = 0; e0 < nT; e0 += 8 * nthr) {
    cx<T> v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + q * nthr + tid;
      v[q] = ld<T>(Tg, e < nT ? e : nT - 1);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + q * nthr + tid;
      if (e < nT) work[e] = v[q];
    }
  }
  __syncthreads();
  if (wv == 0) {
    for (int s = 1; s < nseg; ++s) {
#pragma unroll
      for (int v = 0; v < NR; ++v) {
        cx<T>* ytv = yt + 64 * P * v;
        cx<T>* sttv = stt + 64 * P * v;
        const cx<T> y = lane < K ? ytv[64 * (s - 1) + lane] : mk((T)0, (T)0);
        sttv[64 * s + lane] =
            s >= 2 ? map_apply<T, KM>(work + (s - 2) * KM * KM, sttv + 64 * (s - 1), y, K, lane) : y;
      }
    }
  }
  __syncthreads();
  if (wv >= 1 && wv < nseg) {
    const SegDst<T, Dst> sd[NR] = {SegDst<T, Dst>{dst[0], off}, SegDst<T, Dst>{dst[NR - 1], off}};
    const SegDst<T, Tmp> st[NR] = {SegDst<T, Tmp>{tmp[0], off}, SegDst<T, Tmp>{tmp[NR - 1], off}};
    const cx<T>* const sc[NR] = {stt + 64 * wv, stt + 64 * P * (NR - 1) + 64 * wv};
    add_response_n<T, KM, NR>(sd, st, len, seg,
                              (gptr<const cx<T>>)(Ph + (long long)(wv - 1) * seg * KM), sc, lane);
  }
}

// Transmission data of strip s, node lines l = 0..n-1, into LDS (all
// threads of the workgroup): gl1 = Gamma_{s,1} data where has1 (forward:
// formed from the current z and, if keep, stored to g1 for the backward
// pass; backward: the stored data), gl2 = Gamma_{s,2} data from the current z
// where use2.
template <class T, class A = PlainAcc>
__device__ __forceinline__ void strip_data(cx<T>* gl1, cx<T>* gl2, gptr<cx<T>> z, gptr<cx<T>> g1,
                                           const cx<T>* trb, int s, int n, int a, int w, int dir,
                                           bool has1, bool use2, bool fwd, bool keep,
                                           long long t1off, long long t2off) {
  const cx<T> zero = mk((T)0, (T)0);
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    cx<T> e1 = zero, e2 = zero;
    if (has1) {
      if (fwd) {
        const int i = dir == 0 ? a : l, j = dir == 0 ? l : a;
        e1 = transmission<T, A>((gptr<const cx<T>>)(trb + t1off + 7LL * l), z, i, j, n);
        if (keep) A::store(g1, (long long)s * n + l, e1);
      } else {
        e1 = A::load((gptr<const cx<T>>)g1, (long long)s * n + l);
      }
    }
    if (use2) {
      const int at = a + w - 1;
      const int i = dir == 0 ? at : l, j = dir == 0 ? l : at;
      e2 = transmission<T, A>((gptr<const cx<T>>)(trb + t2off + 7LL * l), z, i, j, n);
    }
    gl1[l] = e1;
    gl2[l] = e2;
  }
}

// Strip order of a sweep (Sec. 2, eqs. (2)-(3); single sweeps of Sec. 4):
// the double sweep solves s = 0..N-1 forward, then N-2..0 backward (u_N =
// v_N), 2N - 1 steps; the forward single sweep s = 0..N-1 and the reverse
// single sweep s = N-1..0, N steps each.  data1/data2: whether the step takes
// transmission data on Gamma_{s,1} / Gamma_{s,2} (where the strip has that
// side; the other side gets zero data); fwd: Gamma_{s,1} data are formed from
// the current z (otherwise the ones kept by the forward pass are read); keep:
// they are kept for the backward pass.
struct SweepStep {
  int s;
  bool fwd, data1, data2, keep;
};
__device__ __forceinline__ int sweep_steps(int mode, int N) {
  return mode == SWEEP_DOUBLE ? 2 * N - 1 : N;
}
__device__ __forceinline__ SweepStep sweep_step(int mode, int N, int step) {
  SweepStep o;
  if (mode == SWEEP_REVERSE) {
    o.s = N - 1 - step;
    o.fwd = false;
    o.data1 = false;
    o.data2 = true;
    o.keep = false;
  } else {
    o.fwd = step < N;
    o.s = o.fwd ? step : 2 * N - 2 - step;
    o.data1 = true;
    o.data2 = !o.fwd;
    o.keep = o.fwd && mode == SWEEP_DOUBLE;
  }
  return o;
}

// One workgroup of P waves runs one double sweep.  Per strip: the
// transmission data of its interfaces go to LDS (forward: g_{s,1} from the
// current z, also kept for the backward pass; backward: the kept g_{s,1} and
// g_{s,2} from the current z), then the forward substitution streams the
// gathered right-hand side into the strip buffer and the back substitution
// streams the solution from it into z.  Strips whose factorisation pivoted
// take the lane-major path on wave 0, with explicit gather and scatter passes.
// Dynamic LDS (complex elements): two node lines of transmission data, the
// segment tails and states (64 P each), then the work area of solve_triangle.
template <class T, int D, int S, int KP, int U, int NB, bool PIV>
__global__ __launch_bounds__(512) void k_sweep(const SweepTask* __restrict__ tasks) {
  extern __shared__ char smem_raw[];
  const SweepTask& tk = tasks[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nthr = blockDim.x;
  const int P = nthr >> 6;
  const int n = uni(tk.n), N = uni(tk.N);
  cx<T>* gl1 = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* gl2 = gl1 + n;
  cx<T>* yt = gl2 + n;
  cx<T>* stt = yt + 64 * P;
  cx<T>* work = stt + 64 * P;
  const cx<T>* img = uniptr((const cx<T>*)tk.img);
  const int* pivb = uniptr(tk.piv);
  const cx<T>* trb = uniptr((const cx<T>*)tk.tr);
  const int* pflag = uniptr(tk.pflag);
  gptr<cx<T>> z = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch.z);
  gptr<cx<T>> rho = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch.rho);
  gptr<cx<T>> g1 = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch.g1);
  gptr<const c128> r = (gptr<const c128>)uniptr(tk.ch.r);
  const StripDesc* strips = uniptr(tk.ch.strips);
  const int mode = uni(tk.mode);
  const int nsteps = sweep_steps(mode, N);
  for (int step = 0; step < nsteps; ++step) {
    const SweepStep ss = sweep_step(mode, N, step);
    const bool fwd = ss.fwd;
    const int s = ss.s;
    const StripDesc* sp = strips + s;
    const int ns = uni(sp->ns), nr = uni(sp->nr), w = uni(sp->w), kl = uni(sp->kl);
    const int dir = uni(sp->dir), a = uni(sp->a), has1 = uni(sp->has1), has2 = uni(sp->has2);
    const long long img_off = uni(sp->img_off), piv_off = uni(sp->piv_off);
    const long long t1off = uni(sp->tr1_off), t2off = uni(sp->tr2_off);
    const int pivoted = PIV ? uni(pflag[uni(sp->gid)]) : 0;
    const bool use1 = has1 && ss.data1;
    const bool use2 = has2 && ss.data2;
    strip_data<T>(gl1, gl2, z, g1, trb, s, n, a, w, dir, use1, use2, fwd, ss.keep, t1off, t2off);
    __syncthreads();
    const float winv = 1.0f / (float)w;
    const SrcGather<T> gather{r, gl1, gl2, nr, w, n, a, dir, use1, use2, winv};
    if (!pivoted) {
      const int seg = uni(sp->seg);
      const cx<T>* GL = img + img_off;
      const cx<T>* GU = GL + blocked_blocks(ns) * KP * 64;
      constexpr long long KM2 = (long long)map_dim(KP) * map_dim(KP);
      const cx<T>* TL = img + uni(sp->t_off) + uni(sp->pmap[0]) * KM2;
      const cx<T>* TU = TL + uni(sp->tmaps) * KM2;
      const cx<T>* PL = img + uni(sp->phi_off[0]);
      const cx<T>* PU = PL + plan_phi_elems(ns, uni(sp->segs), kl, map_dim(KP), 0);
      // the forward substitution ends at the last unknown (the identity rows
      // past it feed nothing) and the back substitution reads those rows as
      // zero; its later segments keep their zero-start outputs in the second
      // half of the chain's scratch, so that z (a scatter) is written once
      for (int q = nr + tid; q < ns; q += nthr) st<T>(rho, q, mk((T)0, (T)0));
      const DstVec<T> drho{rho, ns, false};
      solve_triangle<T, KP, U, NB>(gather, drho, drho, GL, TL, PL, nr, kl, seg, work, yt, stt);
      __syncthreads();
      solve_triangle<T, KP, U, NB>(SrcVec<T>{(gptr<const cx<T>>)rho, ns, true},
                               DstScatter<T>{z, ns, nr, w, n, a, dir, winv},
                               DstVec<T>{rho + ns, ns, false}, GU, TU, PU, ns, kl, seg, work, yt,
                               stt);
    } else if (PIV && wv == 0) {
      // single wave: its memory accesses are performed in order, the fences
      // only keep the compiler from reordering them
      for (int q = lane; q < ns; q += 64) st<T>(rho, q, gather.get(gather.load(q)));
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      gptr<cx<T>> x[1] = {rho};
      gptr<const cx<T>> Lm[1] = {(gptr<const cx<T>>)(img + img_off)};
      gptr<const int> pv[1] = {(gptr<const int>)(pivb + piv_off)};
      solve_lower<T, 1, D>(x, Lm, pv, ns, lane);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      const long long NP = ns + HH_PAD;
      gptr<const cx<T>> Um[1] = {(gptr<const cx<T>>)(img + img_off + NP * 64)};
      gptr<const cx<T>> rdg[1] = {(gptr<const cx<T>>)(img + img_off + NP * 64 * (1 + S))};
      solve_upper<T, 1, D, S>(x, Um, rdg, ns, lane);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      const DstScatter<T> out{z, ns, nr, w, n, a, dir, winv};
      for (int q = lane; q < ns; q += 64) out.put(ns - 1 - q, ld<T>(rho, q));
    }
    __syncthreads();
  }
}

// k_sweep for factorisations of wide strips (kl > HH_KL_WINDOW): one wave per
// chain, every strip through the lane-major substitution (solve_lower_w with
// SL slots, solve_upper with S = 2 SL).  Dynamic LDS: two node lines of
// transmission data.
template <class T, int D, int SL>
__global__ __launch_bounds__(64) void k_sweep_lm(const SweepTask* __restrict__ tasks) {
  constexpr int S = 2 * SL;
  extern __shared__ char smem_raw[];
  const SweepTask& tk = tasks[blockIdx.x];
  const int lane = threadIdx.x;
  const int n = uni(tk.n), N = uni(tk.N);
  cx<T>* gl1 = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* gl2 = gl1 + n;
  const cx<T>* img = uniptr((const cx<T>*)tk.img);
  const int* pivb = uniptr(tk.piv);
  const cx<T>* trb = uniptr((const cx<T>*)tk.tr);
  gptr<cx<T>> z = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch.z);
  gptr<cx<T>> rho = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch.rho);
  gptr<cx<T>> g1 = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch.g1);
  gptr<const c128> r = (gptr<const c128>)uniptr(tk.ch.r);
  const StripDesc* strips = uniptr(tk.ch.strips);
  const int mode = uni(tk.mode);
  const int nsteps = sweep_steps(mode, N);
  for (int step = 0; step < nsteps; ++step) {
    const SweepStep ss = sweep_step(mode, N, step);
    const int s = ss.s;
    const StripDesc* sp = strips + s;
    const int ns = uni(sp->ns), nr = uni(sp->nr), w = uni(sp->w);
    const int dir = uni(sp->dir), a = uni(sp->a), has1 = uni(sp->has1), has2 = uni(sp->has2);
    const long long img_off = uni(sp->img_off), piv_off = uni(sp->piv_off);
    const long long t1off = uni(sp->tr1_off), t2off = uni(sp->tr2_off);
    const bool use1 = has1 && ss.data1;
    const bool use2 = has2 && ss.data2;
    strip_data<T>(gl1, gl2, z, g1, trb, s, n, a, w, dir, use1, use2, ss.fwd, ss.keep, t1off, t2off);
    __syncthreads();
    const float winv = 1.0f / (float)w;
    const SrcGather<T> gather{r, gl1, gl2, nr, w, n, a, dir, use1, use2, winv};
    // a single wave: its memory accesses are performed in order, the fences
    // only keep the compiler from reordering them
    for (int q = lane; q < ns; q += 64) st<T>(rho, q, gather.get(gather.load(q)));
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const long long NP = ns + HH_PAD;
    solve_lower_w<T, D, SL>(rho, (gptr<const cx<T>>)(img + img_off),
                            (gptr<const int>)(pivb + piv_off), ns, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    gptr<cx<T>> x[1] = {rho};
    gptr<const cx<T>> Um[1] = {(gptr<const cx<T>>)(img + img_off + NP * 64 * SL)};
    gptr<const cx<T>> rdg[1] = {(gptr<const cx<T>>)(img + img_off + NP * 64 * (SL + S))};
    solve_upper<T, 1, D, S>(x, Um, rdg, ns, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const DstScatter<T> out{z, ns, nr, w, n, a, dir, winv};
    for (int q = lane; q < ns; q += 64) out.put(ns - 1 - q, ld<T>(rho, q));
    __syncthreads();
  }
}

// Inner transmission data of a sub-block interface node (strip-local line l,
// position t across the strip): g = sum_d coef_d U[neighbour d] over the
// seven stencil neighbours in the strip's local order q = l w + t (x strips:
// t along x, l along y; y strips: l along x, t along y).  Neighbours outside
// the strip have zero coefficients and are skipped.
template <class T>
__device__ __forceinline__ cx<T> inner_transmission(gptr<const cx<T>> coef, gptr<cx<T>> U, int l,
                                                    int t, int w, int n, int dir) {
  const int di[7] = {-1, 0, -1, 0, 1, 0, 1};
  const int dj[7] = {-1, -1, 0, 0, 0, 1, 1};
  cx<T> g = mk((T)0, (T)0);
#pragma unroll
  for (int d = 0; d < 7; ++d) {
    const int ll = l + (dir == 0 ? dj[d] : di[d]), tt = t + (dir == 0 ? di[d] : dj[d]);
    if (ll < 0 || ll >= n || tt < 0 || tt >= w) continue;
    g = cfma(g, ld<T>(coef, d), ld<T>(U, (long long)ll * w + tt));
  }
  return g;
}

// Double sweeps whose strip solves are inner double sweeps (recursive strip
// solves, Sec. 4 closing discussion): one wave per chain.  Per outer step the
// strip right-hand side R_s r + g (outer transmission data as in k_sweep) goes
// to scratch A, the inner solution U starts from zero, and sub-blocks t = 1..N2
// then N2-1..1 are solved with the lane-major substitution: right-hand side
// A restricted to the sub-block plus its inner transmission data (formed from
// U, the Gamma_1 data kept for the backward pass), solution written over U.
// U then goes over z.  Scratch per chain (rho): A, U and the sub-block vector
// (ns of the strip each), then the inner Gamma_1 data (N2 x w).  Dynamic LDS:
// the outer data (2n) and the inner data (2n).
template <class T, int D, int SL>
__global__ __launch_bounds__(64) void k_sweep_rec(const SweepTask* __restrict__ tasks) {
  constexpr int S = 2 * SL;
  extern __shared__ char smem_raw[];
  const SweepTask& tk = tasks[blockIdx.x];
  const int lane = threadIdx.x;
  const int n = uni(tk.n), N = uni(tk.N);
  cx<T>* gl1 = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* gl2 = gl1 + n;
  cx<T>* gi1 = gl2 + n;
  cx<T>* gi2 = gi1 + n;
  const cx<T>* img = uniptr((const cx<T>*)tk.img);
  const int* pivb = uniptr(tk.piv);
  const cx<T>* trb = uniptr((const cx<T>*)tk.tr);
  const cx<T> zero = mk((T)0, (T)0);
  gptr<cx<T>> z = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch.z);
  gptr<cx<T>> rho = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch.rho);
  gptr<cx<T>> g1 = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch.g1);
  gptr<const c128> r = (gptr<const c128>)uniptr(tk.ch.r);
  const StripDesc* strips = uniptr(tk.ch.strips);
  const int mode = uni(tk.mode);
  const int nsteps = sweep_steps(mode, N);
  for (int step = 0; step < nsteps; ++step) {
    const SweepStep ss = sweep_step(mode, N, step);
    const int s = ss.s;
    const StripDesc* sp = strips + s;
    const int ns = uni(sp->ns), nr = uni(sp->nr), w = uni(sp->w);
    const int dir = uni(sp->dir), a = uni(sp->a), has1 = uni(sp->has1), has2 = uni(sp->has2);
    const long long t1off = uni(sp->tr1_off), t2off = uni(sp->tr2_off);
    const bool use1 = has1 && ss.data1;
    const bool use2 = has2 && ss.data2;
    strip_data<T>(gl1, gl2, z, g1, trb, s, n, a, w, dir, use1, use2, ss.fwd, ss.keep, t1off, t2off);
    __syncthreads();
    gptr<cx<T>> A = rho, U = rho + ns, C = rho + 2LL * ns, G1 = rho + 3LL * ns;
    const float winv = 1.0f / (float)w;
    const SrcGather<T> gather{r, gl1, gl2, nr, w, n, a, dir, use1, use2, winv};
    // a single wave: its memory accesses are performed in order, the fences
    // only keep the compiler from reordering them
    for (int q = lane; q < ns; q += 64) {
      st<T>(A, q, gather.get(gather.load(q)));
      st<T>(U, q, zero);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const StripDesc* subs = sp + uni(sp->sub);
    const int N2 = uni(sp->nsub);
    for (int it = 0; it < 2 * N2 - 1; ++it) {
      const SweepStep is = sweep_step(SWEEP_DOUBLE, N2, it);
      const StripDesc* up = subs + is.s;
      const int c0 = uni(up->c0), len = uni(up->len), orient = uni(up->orient), nsu = uni(up->ns);
      const bool u1 = uni(up->has1) && is.data1, u2 = uni(up->has2) && is.data2;
      const long long i1 = uni(up->tr1_off), i2 = uni(up->tr2_off);
      for (int t = lane; t < w; t += 64) {
        cx<T> e1 = zero, e2 = zero;
        if (u1) {
          if (is.fwd) {
            e1 = inner_transmission<T>((gptr<const cx<T>>)(trb + i1 + 7LL * t), U, c0, t, w, n, dir);
            if (is.keep) st<T>(G1, (long long)is.s * w + t, e1);
          } else {
            e1 = ld<T>(G1, (long long)is.s * w + t);
          }
        }
        if (u2)
          e2 = inner_transmission<T>((gptr<const cx<T>>)(trb + i2 + 7LL * t), U, c0 + len - 1, t, w,
                                     n, dir);
        gi1[t] = e1;
        gi2[t] = e2;
      }
      __syncthreads();
      for (int q = lane; q < nsu; q += 64) {
        const int L = orient == 0 ? q / w : q % len, Tt = orient == 0 ? q % w : q / len;
        cx<T> v = ld<T>(A, (long long)(c0 + L) * w + Tt);
        if (u1 && L == 0) v = v + gi1[Tt];
        if (u2 && L == len - 1) v = v + gi2[Tt];
        st<T>(C, q, v);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      const long long ioff = uni(up->img_off), NP = nsu + HH_PAD;
      solve_lower_w<T, D, SL>(C, (gptr<const cx<T>>)(img + ioff),
                              (gptr<const int>)(pivb + uni(up->piv_off)), nsu, lane);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      gptr<cx<T>> x[1] = {C};
      gptr<const cx<T>> Um[1] = {(gptr<const cx<T>>)(img + ioff + NP * 64 * SL)};
      gptr<const cx<T>> rdg[1] = {(gptr<const cx<T>>)(img + ioff + NP * 64 * (SL + S))};
      solve_upper<T, 1, D, S>(x, Um, rdg, nsu, lane);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      for (int q = lane; q < nsu; q += 64) {
        const int L = orient == 0 ? q / w : q % len, Tt = orient == 0 ? q % w : q / len;
        st<T>(U, (long long)(c0 + L) * w + Tt, ld<T>(C, q));
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __syncthreads();
    }
    const DstScatter<T> out{z, ns, nr, w, n, a, dir, winv};
    for (int q = lane; q < ns; q += 64) out.put(ns - 1 - q, ld<T>(U, q));
    __syncthreads();
  }
}

// k_sweep for tiles of NR = 2 right-hand sides of the same preconditioner
// (unpivoted strips, segment plan 0): task t carries its two chains in ch and
// ch2 (the same strips and sweep mode; a tile of one repeats its chain in
// ch2, whose identical stores are harmless).  Dynamic LDS (complex elements):
// two node lines of transmission data per right-hand side, yt and stt (64 P
// each per right-hand side), then the work area max(640 P NR, (P - 2) KM^2).
template <class T, int KP, int U, int NB>
__global__ __launch_bounds__(512) void k_sweep_n(const SweepTask* __restrict__ tasks) {
  constexpr int NR = 2;
  extern __shared__ char smem_raw[];
  const SweepTask& tk = tasks[blockIdx.x];
  const int nthr = blockDim.x;
  const int P = nthr >> 6;
  const int n = uni(tk.n), N = uni(tk.N);
  cx<T>* gl = reinterpret_cast<cx<T>*>(smem_raw);  // gl1, gl2 of v at gl + 2 n v
  cx<T>* yt = gl + 2 * n * NR;
  cx<T>* stt = yt + 64 * P * NR;
  cx<T>* work = stt + 64 * P * NR;
  const cx<T>* img = uniptr((const cx<T>*)tk.img);
  const cx<T>* trb = uniptr((const cx<T>*)tk.tr);
  const SweepChain* chs[NR] = {&tk.ch, &tk.ch2};
  gptr<cx<T>> z[NR], rho[NR], g1[NR];
  gptr<const c128> r[NR];
#pragma unroll
  for (int v = 0; v < NR; ++v) {
    z[v] = (gptr<cx<T>>)uniptr((cx<T>*)chs[v]->z);
    rho[v] = (gptr<cx<T>>)uniptr((cx<T>*)chs[v]->rho);
    g1[v] = (gptr<cx<T>>)uniptr((cx<T>*)chs[v]->g1);
    r[v] = (gptr<const c128>)uniptr(chs[v]->r);
  }
  const StripDesc* strips = uniptr(tk.ch.strips);
  const int mode = uni(tk.mode);
  const int nsteps = sweep_steps(mode, N);
  for (int step = 0; step < nsteps; ++step) {
    const SweepStep ss = sweep_step(mode, N, step);
    const bool fwd = ss.fwd;
    const int s = ss.s;
    const StripDesc* sp = strips + s;
    const int ns = uni(sp->ns), nr = uni(sp->nr), w = uni(sp->w), kl = uni(sp->kl);
    const int dir = uni(sp->dir), a = uni(sp->a), has1 = uni(sp->has1), has2 = uni(sp->has2);
    const long long img_off = uni(sp->img_off);
    const long long t1off = uni(sp->tr1_off), t2off = uni(sp->tr2_off);
    const bool use1 = has1 && ss.data1;
    const bool use2 = has2 && ss.data2;
#pragma unroll
    for (int v = 0; v < NR; ++v)
      strip_data<T>(gl + 2 * n * v, gl + 2 * n * v + n, z[v], g1[v], trb, s, n, a, w, dir, use1, use2,
                    fwd, ss.keep, t1off, t2off);
    __syncthreads();
    const float winv = 1.0f / (float)w;
    const SrcGather<T> gather[NR] = {
        SrcGather<T>{r[0], gl, gl + n, nr, w, n, a, dir, use1, use2, winv},
        SrcGather<T>{r[1], gl + 2 * n, gl + 3 * n, nr, w, n, a, dir, use1, use2, winv}};
    const int seg = uni(sp->seg);
    const cx<T>* GL = img + img_off;
    const cx<T>* GU = GL + blocked_blocks(ns) * KP * 64;
    constexpr long long KM2 = (long long)map_dim(KP) * map_dim(KP);
    const cx<T>* TL = img + uni(sp->t_off) + uni(sp->pmap[0]) * KM2;
    const cx<T>* TU = TL + uni(sp->tmaps) * KM2;
    const cx<T>* PL = img + uni(sp->phi_off[0]);
    const cx<T>* PU = PL + plan_phi_elems(ns, uni(sp->segs), kl, map_dim(KP), 0);
    // the forward substitution ends at the last unknown; the back
    // substitution reads the identity rows past it as zero
#pragma unroll
    for (int v = 0; v < NR; ++v)
      for (int q = nr + (int)threadIdx.x; q < ns; q += nthr) st<T>(rho[v], q, mk((T)0, (T)0));
    const DstVec<T> drho[NR] = {DstVec<T>{rho[0], ns, false}, DstVec<T>{rho[1], ns, false}};
    solve_triangle_n<T, KP, U, NB, NR>(gather, drho, drho, GL, TL, PL, nr, kl, seg, work, yt, stt);
    __syncthreads();
    const SrcVec<T> srho[NR] = {SrcVec<T>{(gptr<const cx<T>>)rho[0], ns, true},
                                SrcVec<T>{(gptr<const cx<T>>)rho[1], ns, true}};
    const DstScatter<T> dz[NR] = {DstScatter<T>{z[0], ns, nr, w, n, a, dir, winv},
                                  DstScatter<T>{z[1], ns, nr, w, n, a, dir, winv}};
    const DstVec<T> dtmp[NR] = {DstVec<T>{rho[0] + ns, ns, false}, DstVec<T>{rho[1] + ns, ns, false}};
    solve_triangle_n<T, KP, U, NB, NR>(srho, dz, dtmp, GU, TU, PU, ns, kl, seg, work, yt, stt);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- wide plan
// A chain on G workgroups (complex64 strips).  The rows of a triangle split
// into G P segments (wave w of workgroup g solves segment c = g P + w).  The
// recurrence is linear: the outputs of segment c are its zero-start outputs
// plus Phi_c s_c, where s_c is the segment's true state (the K outputs
// before it) and Phi_c its response to that state; the state after segment c
// is tail_c + T_c s_c (T_c: the last K rows of Phi_c).  Phi, T and the
// products of consecutive T's named below are formed at factorisation time.
//  1. every segment runs from a zero state and writes its outputs (segment 0
//     is then final); it keeps its tail;
//  2. the zero-start states after each segment of a workgroup follow from an
//     inclusive scan over its P segments (steps of distance 1, 2, 4 with the
//     maps T_c, T_c T_{c-1} and T_c ... T_{c-3}, all waves at once); the last
//     one, the workgroup's tail, goes to the chain's exchange area, stamped
//     (tail_put);
//  3. workgroup g waits for the stamped tails of workgroups j < g (tail_get:
//     no meeting of the chain) and forms its true start
//     state S_g = sum_{j<g} Psi_{j,g} tail_j (Psi_{j,g} = W_{g-1} ... W_{j+1},
//     W the workgroup maps, Psi_{g-1,g} = I; one product per wave), and the
//     true states s_c = z_c + Pi_c S_g (z_c the zero-start state, Pi_c the
//     product of the workgroup's maps before segment c);
//  4. every segment but segment 0 adds Phi_c s_c to its outputs.
// The maps of steps 2 and 3 are read into registers (one row per lane), those
// of step 3 and the first rows of Phi_c before the tails.  The workgroups
// meet when the strip's solution is complete (the next strip's transmission
// data read it), and, unless the strip is whole segment groups of the plan
// (then each workgroup's back substitution takes its own forward rows, from
// its LDS), when the forward output is complete: a strip solve is one
// meeting, or two.  A workgroup rewrites its tail in an exchange area only
// in the next strip, after a meeting that every reader of the old tail
// reaches only once it has read it.

// Meeting of the G workgroups of one chain, in two halves so that work can
// go between them.  Everything the workgroups exchange goes through AgentAcc
// (agent-coherent loads and stores).  chain_arrive: every wave waits until
// its stores have completed, the workgroup synchronises and thread 0 counts
// it in.  chain_wait: thread 0 waits until all G have arrived, then the
// workgroup synchronises.  The wait is bounded: after `limit` ticks of the
// constant-rate clock, or as soon as another workgroup has given up, thread 0
// raises *abort and gives up.  Returns false once the chain is aborted, the
// same answer in every thread.
struct ChainBar {
  unsigned* cnt;    // arrivals so far (zero at launch)
  unsigned* abort;  // raised by a workgroup that gave up
  unsigned need;    // arrivals that complete the current meeting
  unsigned G;
  long long limit;
  int* ok;       // LDS word (1 until the chain gives up)
  unsigned tag;  // stamp of the current triangle's tails (tail_put / tail_get)
};

__device__ __forceinline__ void chain_arrive(ChainBar& b) {
  __builtin_amdgcn_s_waitcnt(0);  // every memory access of this wave has completed
  __syncthreads();
  b.need += b.G;
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(b.cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool chain_wait(ChainBar& b) {
  if (threadIdx.x == 0) {
    const long long t0 = wall_clock64();
    int ok = 1;
    // a poll is one round trip to L2; the abort word and the clock are
    // looked at every eighth poll only, so that they do not double it
    for (unsigned it = 0;
         __hip_atomic_load(b.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < b.need; ++it) {
      if ((it & 7) == 0 &&
          (__hip_atomic_load(b.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
           wall_clock64() - t0 > b.limit)) {
        __hip_atomic_store(b.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    *b.ok = ok;
  }
  __syncthreads();
  return *b.ok != 0;
}

__device__ __forceinline__ bool chain_meet(ChainBar& b) {
  chain_arrive(b);
  return chain_wait(b);
}

// The workgroup tails of a triangle travel without a meeting: entry i of the
// exchange area is two agent-scope 64-bit words, the real and the imaginary
// part each in the low half of its word beside the triangle's stamp in the
// high half.  A word is written whole (single-copy atomic), so a reader that
// finds the stamp in both words holds the value; a stale entry carries
// another stamp (a stamp names the launch and the triangle).
__device__ __forceinline__ void tail_put(gptr<c64> x, long long i, c64 v, unsigned tag) {
  const AgentAcc::u64g p = (AgentAcc::u64g)x + 2 * i;
  const unsigned long long t = (unsigned long long)tag << 32;
  __hip_atomic_store(p, t | __float_as_uint(v.re), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 1, t | __float_as_uint(v.im), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Entry i as soon as it carries the stamp (lanes with need false read
// nothing and get zero).  The wait is bounded as chain_wait's: past the
// limit, or once another workgroup has given up, the wave raises the abort
// word and returns false (the same answer in every lane).
__device__ __forceinline__ bool tail_get(gptr<const c64> x, long long i, bool need, c64& v,
                                         const ChainBar& b) {
  const AgentAcc::cu64g p = (AgentAcc::cu64g)x + 2 * (need ? i : 0);
  unsigned long long re = 0, im = 0;
  bool have = !need;
  long long t0 = 0;
  for (unsigned it = 0;; ++it) {
    if (!have) {
      re = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      im = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      have = (unsigned)(re >> 32) == b.tag && (unsigned)(im >> 32) == b.tag;
    }
    if (__all(have)) break;
    if (it == 0) t0 = wall_clock64();
    if ((it & 7) == 7 &&
        __any(__hip_atomic_load(b.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
              wall_clock64() - t0 > b.limit)) {
      __hip_atomic_store(b.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  v = need ? mk(__uint_as_float((unsigned)re), __uint_as_float((unsigned)im)) : mk(0.0f, 0.0f);
  return true;
}

// One row of a KM x KM map (KM <= 32, column-major, zero beyond K) held in
// registers: lane c + 32 h holds the entries (c, h + 2 q), q < KM / 2.
template <class T, int KM>
struct MapRow {
  static_assert(KM <= 32, "two lanes per row");
  cx<T> v[KM / 2];
};

template <class T, int KM>
__device__ __forceinline__ void map_row_load(MapRow<T, KM>& m, const cx<T>* M, int lane) {
  gptr<const cx<T>> Mg = (gptr<const cx<T>>)M;
  const int c = lane & 31, h = lane >> 5, cr = c < KM ? c : 0;
#pragma unroll
  for (int q = 0; q < KM / 2; ++q) m.v[q] = ld<T>(Mg, (long long)(h + 2 * q) * KM + cr);
}

// v = y + M x in lane c < K (zero in the other lanes), y being the lane's
// own entry, M from registers, x in LDS and zero beyond K; the two halves of
// a row are added by one lane swap.
template <class T, int KM>
__device__ __forceinline__ cx<T> map_apply_r(const MapRow<T, KM>& m, const cx<T>* x, cx<T> y,
                                             int K, int lane) {
  static_assert(sizeof(T) == 4, "complex64 maps");
  const cx<T> zero = mk((T)0, (T)0);
  const cx<T>* xb = x + (lane >> 5);
  cx<T> a[4] = {zero, zero, zero, zero};
#pragma unroll
  for (int q = 0; q < KM / 2; ++q) a[q & 3] = cfma(a[q & 3], m.v[q], xb[2 * q]);
  const cx<T> v = (a[0] + a[1]) + (a[2] + a[3]);
  // v_permlane32_swap gives every lane the row's entries of both halves
  const auto sr = __builtin_amdgcn_permlane32_swap(__float_as_uint(v.re), __float_as_uint(v.re), false, false);
  const auto si = __builtin_amdgcn_permlane32_swap(__float_as_uint(v.im), __float_as_uint(v.im), false, false);
  const cx<T> sum = mk(__uint_as_float(sr[0]) + __uint_as_float(sr[1]),
                       __uint_as_float(si[0]) + __uint_as_float(si[1]));
  return csel(lane < K, sum + y, zero);
}

// Map slots of one triangle for the wide plan (see plan_layout): maps[s] is
// slot s; T_c at t0 + c, Pi_c at pi + c - 1, T_c T_{c-1} at a1 + c - 1,
// T_c ... T_{c-3} at a2 + c - 1, Psi_{j,g} at ps + g G + j.
struct WideMaps {
  const cx<float>* maps;
  int t0, pi, a1, a2, ps;
};

// One triangular substitution of a strip by workgroup g of the chain's G
// (steps 1-4 above), after before() and after() (see step 1).  Phi: the segment
// responses (plan_phi_elems layout),
// xch: exchange area (64 stamped entries per workgroup).  LDS: the wave's ring (640
// entries from ring), yt, kb, pw (64 entries per wave each: tails and
// states, scan exchange, partial sums).  Returns false when the chain was
// aborted.
template <int KP, int U, int NB, bool EARLY_INPUTS, class Src, class Dst, class Before,
          class After>
__device__ __forceinline__ bool solve_triangle_wide(
    const Src& src, const Dst& dst, const c64* G, const Before& before, const After& after,
    const WideMaps& mp, const c64* Phi, int ns, int K, int seg, int g, int Gw, c64* ring, c64* yt,
    c64* kb, c64* pw, gptr<c64> xch, ChainBar& bar) {
  using T = float;
  constexpr int KM = map_dim(KP);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, P = blockDim.x >> 6;
  const int nseg = (ns + seg - 1) / seg, gu = (nseg + P - 1) / P;
  const int c = g * P + w;
  const c64 zero = mk(0.0f, 0.0f);
  const int off = c * seg, len = c < nseg ? (ns - off < seg ? ns - off : seg) : 0;
  const SegDst<T, Dst> out{dst, off};
  auto mslot = [&](int s) { return mp.maps + (long long)s * KM * KM; };
  // 1. zero-start solve.  Its first reads go out between before() and
  // after() (the caller's work that the triangle waits for: the maps always,
  // the inputs when they do not depend on that work), so that their round
  // trip overlaps it; a meeting's arrival, which waits for every access of
  // the wave, belongs in before().
  if (!before()) return false;
  const SegSrc<Src> ssrc{src, off, len};
  BlockedPre<T, KP, U, NB, SegSrc<Src>> pre;
  if (c < nseg) {
    blocked_fetch_maps(pre, (gptr<const c64>)(G + (long long)(off / 16) * KP * 64), lane);
    if (EARLY_INPUTS) blocked_fetch_inputs(pre, ssrc, lane);
  }
  if (!after()) return false;
  if (c < nseg) {
    if (!EARLY_INPUTS) blocked_fetch_inputs(pre, ssrc, lane);
    // a segment that step 4 corrects from its ring keeps its zero-start
    // outputs there only: their stores would be overwritten unread, and the
    // next meeting's arrival would wait for them
    const SegDstIf<T, Dst> zout{dst, off, c == 0 || len > 256};
    solve_blocked_run(pre, ssrc, zout, len, K, ring, (const c64*)nullptr, lane);
    if (c < nseg - 1 && lane < K) yt[64 * w + lane] = ring[(len - K + lane) & 255];
  }
  if (nseg == 1) return true;
  // 2. scan of the zero-start states over the workgroup's segments
  const bool has_t = c <= nseg - 2;  // segment c has a tail and (c >= 1) a map T_c
  MapRow<T, KM> A0, A1, A2;
  if (has_t && w >= 1) map_row_load(A0, mslot(mp.t0 + c), lane);
  if (has_t && w >= 2) map_row_load(A1, mslot(mp.a1 + c - 1), lane);
  if (has_t && w >= 4) map_row_load(A2, mslot(mp.a2 + c - 1), lane);
  c64 b = has_t && lane < K ? yt[64 * w + lane] : zero;
  for (int d = 1, lev = 0; d < P; d *= 2, ++lev) {
    kb[64 * w + lane] = b;
    __syncthreads();
    if (has_t && w >= d) {
      const c64* x = kb + 64 * (w - d);
      b = lev == 0 ? map_apply_r(A0, x, b, K, lane)
                   : (lev == 1 ? map_apply_r(A1, x, b, K, lane) : map_apply_r(A2, x, b, K, lane));
    }
    __syncthreads();
  }
  kb[64 * w + lane] = b;  // zero-start state after segment c
  if (w == P - 1 && g < gu - 1 && lane < K) tail_put(xch, (long long)g * 64 + lane, b, bar.tag);
  __syncthreads();  // the states in kb
  // maps of step 3 and the first rows of the correction, read before the
  // other workgroups' tails; wave w takes the tails of workgroups w and w + P
  // (G - 1 <= 2 P)
  MapRow<T, KM> PI, PS0, PS1;
  if (g >= 1 && w >= 1 && c <= nseg - 1) map_row_load(PI, mslot(mp.pi + c - 1), lane);
  if (g >= 2 && w <= g - 2) map_row_load(PS0, mslot(mp.ps + g * Gw + w), lane);
  if (g >= 2 && w + P <= g - 2) map_row_load(PS1, mslot(mp.ps + g * Gw + w + P), lane);
  const bool corr = c >= 1 && c < nseg;
  gptr<const c64> Ph = (gptr<const c64>)(Phi + (long long)(corr ? c - 1 : 0) * seg * KM);
  c64 ph0[KM];
  {
    const int ic = lane < len ? lane : (len > 0 ? len - 1 : 0);
#pragma unroll
    for (int k = 0; k < KM; ++k) ph0[k] = corr ? ld<T>(Ph, (long long)k * seg + ic) : zero;
  }
  // 3. true states
  c64 s = zero;
  if (g == 0) {
    if (w >= 1 && c < nseg) s = kb[64 * (w - 1) + lane];
  } else if (g < gu) {
    if (w < g) {
      c64 t[2] = {zero, zero};
      bool got = true;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int j = w + P * k;
        got = got && tail_get((gptr<const c64>)xch, (long long)j * 64 + lane, lane < K && j < g,
                              t[k], bar);
      }
      if (!got) *bar.ok = 0;
      c64 v = zero;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int j = w + P * k;
        if (j < g) {
          c64 vj = t[k];
          if (j <= g - 2) {
            yt[64 * w + lane] = t[k];
            vj = map_apply_r(k == 0 ? PS0 : PS1, yt + 64 * w, zero, K, lane);
          }
          v = v + vj;
        }
      }
      pw[64 * w + lane] = v;
    }
    __syncthreads();
    if (*bar.ok == 0) return false;
    c64 S = zero;
    for (int j = 0; j < (g < P ? g : P); ++j) S = S + pw[64 * j + lane];
    if (w == 0) {
      s = S;
    } else if (c < nseg) {
      yt[64 * w + lane] = S;
      s = map_apply_r(PI, yt + 64 * w, kb[64 * (w - 1) + lane], K, lane);
    }
  }
  // 4. outputs += Phi_c s_c, 64 rows at a time (lane = row); the zero-start
  // outputs come from the ring while the segment fits it
  if (corr) {
    yt[64 * w + lane] = s;
    const c64* sc = yt + 64 * w;
    for (int i0 = 0; i0 < len; i0 += 64) {
      const int i = i0 + lane, ic = i < len ? i : len - 1;
      c64 a[4] = {len <= 256 ? ring[ic & 255] : out.get(ic), zero, zero, zero};
      if (i0 == 0) {
#pragma unroll
        for (int k = 0; k < KM; ++k) a[k & 3] = cfma(a[k & 3], ph0[k], sc[k]);
      } else {
        c64 pv[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) pv[k] = ld<T>(Ph, (long long)k * seg + ic);
#pragma unroll
        for (int k = 0; k < KM; ++k) a[k & 3] = cfma(a[k & 3], pv[k], sc[k]);
      }
      if (i < len) out.put(i, (a[0] + a[1]) + (a[2] + a[3]));
    }
  }
  return true;
}

// The double sweep of k_sweep on G workgroups per chain (complex64,
// unpivoted strips): workgroup g = blockIdx.x % G of chain blockIdx.x / G.
// Every workgroup forms the transmission data of all node lines itself
// (workgroup 0 keeps the forward ones for the backward pass).  Dynamic LDS
// (complex elements): two node lines, yt, kb, pw (64 P each), the rings
// (640 P), then lo_cap entries for the workgroup's forward outputs where a
// strip is whole segment groups of the plan and they fit.
template <int KP, int U, int NB>
__global__ __launch_bounds__(512) void k_sweep_wide(const SweepTask* __restrict__ tasks, int plan,
                                                    unsigned* abort, long long limit,
                                                    int lo_cap, unsigned epoch) {
  using T = float;
  extern __shared__ char smem_raw[];
  __shared__ int ok;
  if (threadIdx.x == 0) ok = 1;  // read after the first strip's barriers
  const int G = plan_width(plan);
  const SweepTask& tk = tasks[blockIdx.x / G];
  const int g = uni((int)(blockIdx.x % G));
  const int P = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = uni(tk.n), N = uni(tk.N);
  c64* gl1 = reinterpret_cast<c64*>(smem_raw);
  c64* gl2 = gl1 + n;
  c64* yt = gl2 + n;
  c64* kb = yt + 64 * P;
  c64* pw = kb + 64 * P;
  c64* ring = pw + 64 * P + 640 * w;
  c64* lo = pw + 64 * P + 640 * P;  // lo_cap entries: a workgroup's forward outputs
  const c64* img = uniptr((const c64*)tk.img);
  const c64* trb = uniptr((const c64*)tk.tr);
  gptr<c64> z = (gptr<c64>)uniptr((c64*)tk.ch.z);
  gptr<c64> rho = (gptr<c64>)uniptr((c64*)tk.ch.rho);
  gptr<c64> g1 = (gptr<c64>)uniptr((c64*)tk.ch.g1);
  gptr<c64> xch = (gptr<c64>)uniptr((c64*)tk.xch);
  gptr<const c128> r = (gptr<const c128>)uniptr(tk.ch.r);
  const StripDesc* strips = uniptr(tk.ch.strips);
  ChainBar bar{uniptr(tk.bar), abort, 0u, (unsigned)G, limit, &ok, 0u};
  constexpr long long K2 = (long long)map_dim(KP) * map_dim(KP);
  const int mode = uni(tk.mode);
  const int nsteps = sweep_steps(mode, N);
  for (int step = 0; step < nsteps; ++step) {
    const SweepStep ss = sweep_step(mode, N, step);
    const bool fwd = ss.fwd;
    const int s = ss.s;
    const StripDesc* sp = strips + s;
    const int ns = uni(sp->ns), nr = uni(sp->nr), wd = uni(sp->w), kl = uni(sp->kl);
    const int dir = uni(sp->dir), a = uni(sp->a), has1 = uni(sp->has1), has2 = uni(sp->has2);
    const long long img_off = uni(sp->img_off);
    const long long t1off = uni(sp->tr1_off), t2off = uni(sp->tr2_off);
    const bool use1 = has1 && ss.data1;
    const bool use2 = has2 && ss.data2;
    const float winv = 1.0f / (float)wd;
    const SrcGather<T> gather{r, gl1, gl2, nr, wd, n, a, dir, use1, use2, winv};
    const int seg = uni(sp->pseg[plan]);
    // local: the strip is whole segment groups (mirror), so this workgroup's
    // rows of the back substitution (role gu - 1 - g) are its own rows of the
    // forward one; where they fit the LDS its forward outputs stay there, and
    // the back substitution reads them after a workgroup barrier instead of a
    // meeting of the chain
    const int gu = (plan_nseg(ns, seg) + P - 1) / P;
    const bool local = (uni(sp->mirror) >> plan & 1) != 0 && P * seg <= lo_cap;
    const int gb = local && g < gu ? gu - 1 - g : g;
    const int base = g * P * seg;
    const long long tm = uni(sp->tmaps);
    const c64* GL = img + img_off;
    const c64* GU = GL + blocked_blocks(ns) * KP * 64;
    const c64* T0 = img + uni(sp->t_off);
    const WideMaps mL{T0, uni(sp->pmap[plan]) - 1, uni(sp->pi_map[plan]), uni(sp->a1_map[plan]),
                      uni(sp->a2_map[plan]), uni(sp->ps_map[plan])};
    WideMaps mU = mL;
    mU.maps = T0 + tm * K2;
    const c64* PL = img + uni(sp->phi_off[plan]);
    const c64* PU = PL + plan_phi_elems(ns, uni(sp->segs), kl, map_dim(KP), plan);
    // forward substitution: its first reads (maps, residual) go out before
    // the wait for the previous strip's meeting, the transmission data that
    // need that strip's solution after it
    auto none = []() { return true; };
    auto form_data = [&]() {
      if (step > 0 && !chain_wait(bar)) return false;
      strip_data<T, AgentAcc>(gl1, gl2, z, g1, trb, s, n, a, wd, dir, use1, use2, fwd,
                              ss.keep && g == 0, t1off, t2off);
      __syncthreads();
      return true;
    };
    bar.tag = epoch << 16 | (unsigned)(2 * step);  // stamps of this launch: (epoch, triangle)
    if (local) {
      if (!solve_triangle_wide<KP, U, NB, true>(gather, DstLds<T>{lo, base}, GL, none, form_data, mL,
                                                PL, ns, kl, seg, g, G, ring, yt, kb, pw, xch, bar))
        return;
    } else if (!solve_triangle_wide<KP, U, NB, true>(gather, DstVec<T, AgentAcc>{rho, ns, false}, GL,
                                                     none, form_data, mL, PL, ns, kl, seg, g, G,
                                                     ring, yt, kb, pw, xch, bar)) {
      return;
    }
    // back substitution, with the second exchange area (a workgroup may start
    // it while another still reads the forward one's tails): its inputs come
    // from the LDS after a workgroup barrier (local) or from every
    // workgroup's stores after a meeting; its maps go out before either
    const SrcVec<T, AgentAcc> bin{(gptr<const c64>)rho, ns, true};
    const DstScatter<T, AgentAcc> bout{z, ns, nr, wd, n, a, dir, winv};
    const gptr<c64> xchb = xch + (long long)G * 128;  // 64 two-word entries per workgroup
    bar.tag = epoch << 16 | (unsigned)(2 * step + 1);
    if (local) {
      auto sync = []() {
        __syncthreads();
        return true;
      };
      if (!solve_triangle_wide<KP, U, NB, false>(SrcLdsRev<T>{lo, ns, base}, bout, GU, none, sync,
                                                 mU, PU, ns, kl, seg, gb, G, ring, yt, kb, pw, xchb,
                                                 bar))
        return;
    } else {
      auto arrive = [&]() {
        chain_arrive(bar);
        return true;
      };
      auto wait = [&]() { return chain_wait(bar); };
      if (!solve_triangle_wide<KP, U, NB, false>(bin, bout, GU, arrive, wait, mU, PU, ns, kl, seg,
                                                 gb, G, ring, yt, kb, pw, xchb, bar))
        return;
    }
    // the strip's outputs are complete: the next strip waits for this
    // arrival in its forward substitution; the last needs no meeting
    if (step < nsteps - 1) chain_arrive(bar);
  }
}

// One strip solve in FP64 in/out (test hook) by a workgroup of P waves, the
// same substitutions as the sweep; work: ns elements of scratch.  Dynamic
// LDS: tails, states and work area as in k_sweep.
template <class T, int D, int S, int KP, int U, int NB>
__global__ __launch_bounds__(512) void k_strip_solve(const StripDesc* __restrict__ strips, int si,
                                                     const void* __restrict__ img,
                                                     const int* __restrict__ pivb,
                                                     const int* __restrict__ pflag,
                                                     const c128* __restrict__ rhs,
                                                     c128* __restrict__ x,
                                                     cx<T>* __restrict__ work) {
  extern __shared__ char smem_raw[];
  const int P = blockDim.x >> 6, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  cx<T>* yt = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* stt = yt + 64 * P;
  cx<T>* lds = stt + 64 * P;
  const StripDesc* sp = strips + si;
  const int ns = uni(sp->ns), nr = uni(sp->nr), kl = uni(sp->kl);
  const long long ioff = uni(sp->img_off), poff = uni(sp->piv_off);
  const int pivoted = uni(pflag[si]);
  const cx<T>* im = (const cx<T>*)img;
  gptr<cx<T>> wk = (gptr<cx<T>>)work;
  const SrcC128<T> in{(gptr<const c128>)rhs, nr};
  if (!pivoted) {
    const int seg = uni(sp->seg);
    const cx<T>* GL = im + ioff;
    const cx<T>* GU = GL + blocked_blocks(ns) * KP * 64;
    constexpr long long KM2 = (long long)map_dim(KP) * map_dim(KP);
    const cx<T>* TL = im + uni(sp->t_off) + uni(sp->pmap[0]) * KM2;
    const cx<T>* TU = TL + uni(sp->tmaps) * KM2;
    const cx<T>* PL = im + uni(sp->phi_off[0]);
    const cx<T>* PU = PL + plan_phi_elems(ns, uni(sp->segs), kl, map_dim(KP), 0);
    const DstVec<T> dwk{wk, ns, false};
    const DstC128<T> dx{(gptr<c128>)x, ns, nr};
    for (int q = nr + (int)threadIdx.x; q < ns; q += (int)blockDim.x) st<T>(wk, q, mk((T)0, (T)0));
    solve_triangle<T, KP, U, NB>(in, dwk, dwk, GL, TL, PL, nr, kl, seg, lds, yt, stt);
    __syncthreads();
    solve_triangle<T, KP, U, NB>(SrcVec<T>{(gptr<const cx<T>>)wk, ns, true}, dx, dx, GU, TU, PU, ns,
                             kl, seg, lds, yt, stt);
  } else if (wv == 0) {
    for (int q = lane; q < ns; q += 64) st<T>(wk, q, in.get(in.load(q)));
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    gptr<cx<T>> xs[1] = {wk};
    gptr<const cx<T>> Lm[1] = {(gptr<const cx<T>>)(im + ioff)};
    gptr<const int> pv[1] = {(gptr<const int>)(pivb + poff)};
    solve_lower<T, 1, D>(xs, Lm, pv, ns, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    const long long NP = ns + HH_PAD;
    gptr<const cx<T>> Um[1] = {(gptr<const cx<T>>)(im + ioff + NP * 64)};
    gptr<const cx<T>> rdg[1] = {(gptr<const cx<T>>)(im + ioff + NP * 64 * (1 + S))};
    solve_upper<T, 1, D, S>(xs, Um, rdg, ns, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    for (int q = lane; q < nr; q += 64) {
      const cx<T> v = ld<T>(wk, q);
      x[q] = mk((double)v.re, (double)v.im);
    }
  }
}

// Strip solve of a wide strip (test hook): lane-major substitutions on one wave.
template <class T, int D, int SL>
__global__ __launch_bounds__(64) void k_strip_solve_lm(const StripDesc* __restrict__ strips, int si,
                                                       const void* __restrict__ img,
                                                       const int* __restrict__ pivb,
                                                       const c128* __restrict__ rhs,
                                                       c128* __restrict__ x,
                                                       cx<T>* __restrict__ work) {
  constexpr int S = 2 * SL;
  const int lane = threadIdx.x;
  const StripDesc* sp = strips + si;
  const int ns = uni(sp->ns), nr = uni(sp->nr);
  const long long ioff = uni(sp->img_off), poff = uni(sp->piv_off), NP = ns + HH_PAD;
  const cx<T>* im = (const cx<T>*)img;
  gptr<cx<T>> wk = (gptr<cx<T>>)work;
  const SrcC128<T> in{(gptr<const c128>)rhs, nr};
  for (int q = lane; q < ns; q += 64) st<T>(wk, q, in.get(in.load(q)));
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  solve_lower_w<T, D, SL>(wk, (gptr<const cx<T>>)(im + ioff), (gptr<const int>)(pivb + poff), ns,
                          lane);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  gptr<cx<T>> xs[1] = {wk};
  gptr<const cx<T>> Um[1] = {(gptr<const cx<T>>)(im + ioff + NP * 64 * SL)};
  gptr<const cx<T>> rdg[1] = {(gptr<const cx<T>>)(im + ioff + NP * 64 * (SL + S))};
  solve_upper<T, 1, D, S>(xs, Um, rdg, ns, lane);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  for (int q = lane; q < nr; q += 64) {
    const cx<T> v = ld<T>(wk, q);
    x[q] = mk((double)v.re, (double)v.im);
  }
}

}  // namespace

// Template choice.  D: coefficient prefetch depth of the pivoted path (deep
// enough to cover memory latency, small enough to fit the register file);
// KP: terms per lane of the blocked path (fixes S: KP <= 12 <=> kl <= 31);
// U: blocks per step of the blocked path, NB: steps of maps held in registers
// (requests run NB - 1 steps ahead).
template <class T, int KP>
struct SweepShape {
  static constexpr bool dbl = sizeof(T) == 8;
  static constexpr int S = KP <= 12 ? 1 : 2;
  static constexpr int D = S == 1 ? (dbl ? 16 : 32) : (dbl ? 8 : 16);
  static constexpr int U = !dbl && KP <= 12 ? 2 : 1;
  static constexpr int NB = dbl && KP > 10 ? 2 : 3;
};

template <class T, int KP, bool PIV>
static void launch_sweep_kp(const SweepTask* d, int ntasks, int P, int kmax, int nmax,
                            hipStream_t st) {
  using Sh = SweepShape<T, KP>;
  const void* fn = (const void*)k_sweep<T, Sh::D, Sh::S, KP, Sh::U, Sh::NB, PIV>;
  const size_t lds = (size_t)sweep_lds_elems(P, map_dim(KP), nmax) * sizeof(cx<T>);
  if (lds > 64 * 1024)
    HH_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_sweep<T, Sh::D, Sh::S, KP, Sh::U, Sh::NB, PIV>), dim3(ntasks), dim3(64 * P),
                     lds, st, d);
}

template <class T, int KP>
static void launch_sweep_kp(const SweepTask* d, int ntasks, int P, int kmax, int nmax, bool piv,
                            hipStream_t st) {
  if (piv)
    launch_sweep_kp<T, KP, true>(d, ntasks, P, kmax, nmax, st);
  else
    launch_sweep_kp<T, KP, false>(d, ntasks, P, kmax, nmax, st);
}

template <class T>
static void launch_sweep_t(const SweepTask* d, int ntasks, int KP, int P, int kmax, int nmax,
                           bool piv, hipStream_t st) {
  switch (KP) {
    case 8: launch_sweep_kp<T, 8>(d, ntasks, P, kmax, nmax, piv, st); break;
    case 10: launch_sweep_kp<T, 10>(d, ntasks, P, kmax, nmax, piv, st); break;
    case 12: launch_sweep_kp<T, 12>(d, ntasks, P, kmax, nmax, piv, st); break;
    case 16: launch_sweep_kp<T, 16>(d, ntasks, P, kmax, nmax, piv, st); break;
    case 20: launch_sweep_kp<T, 20>(d, ntasks, P, kmax, nmax, piv, st); break;
    default: set_error("unsupported blocked term count %d", KP); throw ArgError();
  }
}

// Device properties the wide plan needs: compute units and the rate of the
// constant clock that bounds the waits of chain_wait (kHz).
struct WideDev {
  int cus = 0, khz = 0;
};
static WideDev wide_dev() {
  int dev = 0;
  HH_HIP(hipGetDevice(&dev));
  static WideDev cache[64];
  WideDev& d = cache[dev & 63];
  if (d.cus == 0) {
    HH_HIP(hipDeviceGetAttribute(&d.khz, hipDeviceAttributeWallClockRate, dev));
    HH_HIP(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  return d;
}

// Entries of LDS for a workgroup's forward outputs (plans whose strips are
// whole segment groups): as many as fit beside the rest under 150 KB, at most
// 4096 (P pseg of the 321 x 321 benchmark: 512 on sixteen workgroups, 3840 on
// two).
static int wide_lo_cap(int P, int nmax) {
  const long long room = 150LL * 1024 / (long long)sizeof(c64) - sweep_lds_elems_wide(P, nmax);
  return (int)std::max(0LL, std::min(4096LL, room));
}

static size_t wide_lds_bytes(int P, int nmax) {
  return (size_t)(sweep_lds_elems_wide(P, nmax) + wide_lo_cap(P, nmax)) * sizeof(c64);
}

// Plans 1 and 2 run complex64 strips whose maps fit two lanes per row, with
// at most two workgroup tails per wave in step 3 (G - 1 <= 2 P).
bool sweep_wide_fits(int precision, int P, int kmax, int nmax) {
  return precision == HH_FP32 && map_dim(blocked_kp(kmax)) <= 32 &&
         plan_width(HH_PLAN_WIDE) - 1 <= 2 * P && wide_lds_bytes(P, nmax) <= 150 * 1024;
}

template <int KP>
static const void* wide_kernel() {
  using Sh = SweepShape<float, KP>;
  return (const void*)k_sweep_wide<KP, Sh::U, Sh::NB>;
}

// Workgroups of k_sweep_wide that fit the device at once (a cooperative launch
// must not exceed it): its occupancy per compute unit, for the launch's
// workgroup size and LDS, times the compute units.
static long long wide_capacity(int KP, int P, int nmax) {
  int dev = 0;
  HH_HIP(hipGetDevice(&dev));
  const size_t lds = wide_lds_bytes(P, nmax);
  static std::mutex mu;
  static std::map<std::array<long long, 4>, long long> cache;
  const std::array<long long, 4> key{dev, KP, P, (long long)lds};
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  const void* fn = KP == 8 ? wide_kernel<8>() : KP == 10 ? wide_kernel<10>() : wide_kernel<12>();
  if (lds > 64 * 1024)
    HH_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int per_cu = 0;
  HH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * P, lds));
  const long long c = (long long)std::max(per_cu, 0) * wide_dev().cus;
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = c;
  return c;
}

bool sweep_plan_fits(int plan, int ntasks, int precision, int KP, int P, int kmax, int nmax,
                     bool pivots, bool built) {
  if (plan == 0) return true;
  if (plan == HH_PLAN_TILE) return ntasks >= 2 && sweep_tiles_fit(precision, KP, P, nmax, pivots);
  if (pivots || !sweep_wide_fits(precision, P, kmax, nmax)) return false;
  if (KP != 8 && KP != 10 && KP != 12) return false;
  if (plan == HH_PLAN_PAIR && !built) return false;
  return (long long)ntasks * plan_width(plan) <= wide_capacity(KP, P, nmax);
}

int sweep_plan_for(int ntasks, int precision, int P, int kmax, int nmax, bool pivots, bool built) {
  const char* tenv = std::getenv("HH_SWEEP_PLAN");
  if (tenv && std::atoi(tenv) == HH_PLAN_TILE)
    return sweep_plan_fits(HH_PLAN_TILE, ntasks, precision, blocked_kp(kmax), P, kmax, nmax,
                           pivots, true)
               ? HH_PLAN_TILE
               : 0;
  // more chains than compute units: plan 0 would take two rounds of
  // workgroups, tiles of two right-hand sides take one (same results)
  const int KPt = blocked_kp(kmax);
  const bool many = ntasks > wide_dev().cus &&
                    sweep_plan_fits(HH_PLAN_TILE, ntasks, precision, KPt, P, kmax, nmax, pivots, true);
  if (pivots || !sweep_wide_fits(precision, P, kmax, nmax)) return many ? HH_PLAN_TILE : 0;
  const int KP = blocked_kp(kmax);
  const char* env = std::getenv("HH_SWEEP_PLAN");
  if (env && *env) {
    const int p = std::atoi(env);
    if (p == HH_PLAN_TILE)
      return sweep_plan_fits(p, ntasks, precision, KP, P, kmax, nmax, pivots, true) ? p : 0;
    if (p == HH_PLAN_PAIR)
      return sweep_plan_fits(p, ntasks, precision, KP, P, kmax, nmax, pivots, true) ? p : 0;
    return p > 0 && sweep_plan_fits(HH_PLAN_WIDE, ntasks, precision, KP, P, kmax, nmax, pivots,
                                    built)
               ? HH_PLAN_WIDE
               : 0;
  }
  // a few chains: sixteen workgroups each while they all fit the device at
  // once (16 chains of the 801 x 801 medium: 66.6 ms of sweeps per batch
  // against 243 ms on two workgroups each); up to one chain per two compute
  // units: two workgroups each; more: plan 0, or its tiles beyond one chain
  // per compute unit (the autotuner measures instead where it is on)
  if ((long long)ntasks * plan_width(HH_PLAN_WIDE) <= wide_dev().cus &&
      sweep_plan_fits(HH_PLAN_WIDE, ntasks, precision, KP, P, kmax, nmax, pivots, built))
    return HH_PLAN_WIDE;
  if (built && sweep_plan_fits(HH_PLAN_PAIR, ntasks, precision, KP, P, kmax, nmax, pivots, true))
    return HH_PLAN_PAIR;
  return many ? HH_PLAN_TILE : 0;
}

// The launch's part of its tails' stamps, one count over every wide launch
// of the process (every instantiation, every exchange area): 16 bits, never
// 0, so that the zeros of a fresh exchange area match no stamp and a stamp
// comes back only after 65535 launches.
static std::atomic<unsigned> g_wide_launches{0};
static unsigned next_wide_epoch() {
  unsigned e = 0;
  while (e == 0) e = ++g_wide_launches & 0xffffu;
  return e;
}

template <int KP>
static void launch_wide_kp(const SweepTask* d, int ntasks, int P, int nmax, int plan,
                           unsigned* abort, hipStream_t st) {
  using Sh = SweepShape<float, KP>;
  const int G = plan_width(plan);
  const void* fn = (const void*)k_sweep_wide<KP, Sh::U, Sh::NB>;
  const size_t lds = wide_lds_bytes(P, nmax);
  if (lds > 64 * 1024)
    HH_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  // bound of each wait: HH_SWEEP_WAIT_US microseconds when set, else 250 ms
  const char* env = std::getenv("HH_SWEEP_WAIT_US");
  const long long us = env && *env ? std::atoll(env) : 250000LL;
  long long limit = (long long)wide_dev().khz * us / 1000;
  int lo_cap = wide_lo_cap(P, nmax);
  unsigned epoch = next_wide_epoch();
  void* args[] = {(void*)&d,     (void*)&plan,   (void*)&abort,
                  (void*)&limit, (void*)&lo_cap, (void*)&epoch};
  HH_HIP(hipLaunchCooperativeKernel(fn, dim3((unsigned)(ntasks * G)), dim3(64 * P), args,
                                    (unsigned)lds, st));
}

static void launch_wide(const SweepTask* d, int ntasks, int KP, int P, int nmax, int plan,
                        unsigned* abort, hipStream_t st) {
  switch (KP) {
    case 8: launch_wide_kp<8>(d, ntasks, P, nmax, plan, abort, st); break;
    case 10: launch_wide_kp<10>(d, ntasks, P, nmax, plan, abort, st); break;
    case 12: launch_wide_kp<12>(d, ntasks, P, nmax, plan, abort, st); break;
    default: set_error("the wide segment plan does not take %d blocked terms", KP); throw ArgError();
  }
}

// Tiles of two right-hand sides (k_sweep_n): complex64 strips with the
// one-workgroup plan's segments, when the workgroup's LDS fits.
static size_t tile_lds_bytes(int P, int KP, int nmax) {
  constexpr int NR = 2;
  const long long KM = map_dim(KP);
  const long long work = std::max(640LL * P * NR, (long long)std::max(P - 2, 0) * KM * KM);
  return (size_t)(2LL * nmax * NR + 2LL * 64 * P * NR + work) * sizeof(c64);
}

bool sweep_tiles_fit(int precision, int KP, int P, int nmax, bool pivots) {
  return precision == HH_FP32 && !pivots && (KP == 8 || KP == 10 || KP == 12 || KP == 16) &&
         tile_lds_bytes(P, KP, nmax) <= 160 * 1024;
}

template <int KP>
static void launch_tiles_kp(const SweepTask* d, int ntiles, int P, int nmax, hipStream_t st) {
  using Sh = SweepShape<float, KP>;
  const void* fn = (const void*)k_sweep_n<float, KP, Sh::U, 2>;
  const size_t lds = tile_lds_bytes(P, KP, nmax);
  if (lds > 64 * 1024)
    HH_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_sweep_n<float, KP, Sh::U, 2>), dim3(ntiles), dim3(64 * P), lds, st, d);
}

void launch_sweep_tiles(const SweepTask* d_tiles, int ntiles, int precision, int KP, int P,
                        int nmax, bool pivots, hipStream_t st) {
  if (ntiles <= 0) return;
  if (!sweep_tiles_fit(precision, KP, P, nmax, pivots) || P < 1 || P > 8) {
    set_error("right-hand-side tiles do not fit this factorisation");
    throw ArgError();
  }
  switch (KP) {
    case 8: launch_tiles_kp<8>(d_tiles, ntiles, P, nmax, st); break;
    case 10: launch_tiles_kp<10>(d_tiles, ntiles, P, nmax, st); break;
    case 12: launch_tiles_kp<12>(d_tiles, ntiles, P, nmax, st); break;
    default: launch_tiles_kp<16>(d_tiles, ntiles, P, nmax, st); break;
  }
  HH_HIP(hipGetLastError());
}

// Wide strips: prefetch depth D of the lane-major rows (registers: 2 (SL + S) D
// complex coefficients per lane, S = 2 SL; D divides 64).  Four rows ahead in
// FP64 and eight in FP32 fit without scratch (a few values go to the
// accumulation registers at SL = 3).
template <class T>
struct LaneMajorShape {
  static constexpr int D = sizeof(T) == 8 ? 4 : 8;
};
template <class T, int SL>
static void launch_sweep_lm_t(const SweepTask* d, int ntasks, int nmax, hipStream_t st) {
  const size_t lds = (size_t)2 * nmax * sizeof(cx<T>);
  const void* fn = (const void*)k_sweep_lm<T, LaneMajorShape<T>::D, SL>;
  if (lds > 64 * 1024)
    HH_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_sweep_lm<T, LaneMajorShape<T>::D, SL>), dim3(ntasks), dim3(64), lds, st,
                     d);
}
template <class T, int SL>
static void launch_sweep_rec_t(const SweepTask* d, int ntasks, int nmax, hipStream_t st) {
  const size_t lds = (size_t)4 * nmax * sizeof(cx<T>);
  const void* fn = (const void*)k_sweep_rec<T, LaneMajorShape<T>::D, SL>;
  if (lds > 64 * 1024)
    HH_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_sweep_rec<T, LaneMajorShape<T>::D, SL>), dim3(ntasks), dim3(64), lds, st,
                     d);
}
static void launch_sweep_rec(const SweepTask* d, int ntasks, int precision, int kmax, int nmax,
                             hipStream_t st) {
  const int SL = lane_slots(kmax);
  if (kmax > HH_KL_MAX || SL < 1 || SL > 3) {
    set_error("no recursive sweep for sub-block band half-width %d", kmax);
    throw ArgError();
  }
  if (precision == HH_FP64) {
    if (SL == 1) launch_sweep_rec_t<double, 1>(d, ntasks, nmax, st);
    else if (SL == 2) launch_sweep_rec_t<double, 2>(d, ntasks, nmax, st);
    else launch_sweep_rec_t<double, 3>(d, ntasks, nmax, st);
  } else {
    if (SL == 1) launch_sweep_rec_t<float, 1>(d, ntasks, nmax, st);
    else if (SL == 2) launch_sweep_rec_t<float, 2>(d, ntasks, nmax, st);
    else launch_sweep_rec_t<float, 3>(d, ntasks, nmax, st);
  }
  HH_HIP(hipGetLastError());
}
static void launch_sweep_lm(const SweepTask* d, int ntasks, int precision, int kmax, int nmax,
                            hipStream_t st) {
  const int SL = lane_slots(kmax);
  if (kmax > HH_KL_MAX || SL < 2 || SL > 3) {
    set_error("no lane-major sweep for band half-width %d", kmax);
    throw ArgError();
  }
  if (precision == HH_FP64) {
    if (SL == 2) launch_sweep_lm_t<double, 2>(d, ntasks, nmax, st);
    else launch_sweep_lm_t<double, 3>(d, ntasks, nmax, st);
  } else {
    if (SL == 2) launch_sweep_lm_t<float, 2>(d, ntasks, nmax, st);
    else launch_sweep_lm_t<float, 3>(d, ntasks, nmax, st);
  }
  HH_HIP(hipGetLastError());
}

void launch_sweep(const SweepTask* d_tasks, int ntasks, int precision, int KP, int P, int kmax,
                  int nmax, bool pivots, int plan, unsigned* abort, hipStream_t st) {
  if (ntasks <= 0) return;
  if (plan == HH_PLAN_REC) {
    launch_sweep_rec(d_tasks, ntasks, precision, kmax, nmax, st);
    return;
  }
  if (kmax > HH_KL_WINDOW) {
    if (plan != 0) {
      set_error("strips of band half-width %d run on segment plan 0 only", kmax);
      throw ArgError();
    }
    launch_sweep_lm(d_tasks, ntasks, precision, kmax, nmax, st);
    return;
  }
  if (P < 1 || P > 8) {
    set_error("unsupported segment count %d", P);
    throw ArgError();
  }
  if (plan == HH_PLAN_TILE) {
    set_error("tiles of right-hand sides are launched with launch_sweep_tiles");
    throw ArgError();
  }
  if (plan < 0 || plan >= HH_NPLAN || (plan > 0 && (pivots || !abort))) {
    set_error("segment plan %d cannot run here", plan);
    throw ArgError();
  }
  if (plan > 0) {
    if (!sweep_plan_fits(plan, ntasks, precision, KP, P, kmax, nmax, pivots, true)) {
      set_error("segment plan %d does not fit this factorisation or launch", plan);
      throw ArgError();
    }
    launch_wide(d_tasks, ntasks, KP, P, nmax, plan, abort, st);
  } else if (precision == HH_FP64) {
    launch_sweep_t<double>(d_tasks, ntasks, KP, P, kmax, nmax, pivots, st);
  } else {
    launch_sweep_t<float>(d_tasks, ntasks, KP, P, kmax, nmax, pivots, st);
  }
  HH_HIP(hipGetLastError());
}

template <class T, int KP>
static void launch_strip_kp(const hh_problem* pb, int si, const c128* rhs, c128* x, void* scratch,
                            hipStream_t st) {
  using Sh = SweepShape<T, KP>;
  const FactorSet& fs = pb->fs;
  const int P = fs.strips[si].segs;
  const void* fn = (const void*)k_strip_solve<T, Sh::D, Sh::S, KP, Sh::U, Sh::NB>;
  const size_t lds = (size_t)sweep_lds_elems(P, map_dim(KP), 0) * sizeof(cx<T>);
  if (lds > 64 * 1024)
    HH_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_strip_solve<T, Sh::D, Sh::S, KP, Sh::U, Sh::NB>), dim3(1), dim3(64 * P), lds, st,
                     fs.d_strips, si, fs.img, fs.piv, fs.d_pflag, rhs, x, (cx<T>*)scratch);
}

template <class T>
static void launch_strip_t(const hh_problem* pb, int si, const c128* rhs, c128* x, void* scratch,
                           hipStream_t st) {
  switch (pb->fs.strips[si].KP) {
    case 8: launch_strip_kp<T, 8>(pb, si, rhs, x, scratch, st); break;
    case 10: launch_strip_kp<T, 10>(pb, si, rhs, x, scratch, st); break;
    case 12: launch_strip_kp<T, 12>(pb, si, rhs, x, scratch, st); break;
    case 16: launch_strip_kp<T, 16>(pb, si, rhs, x, scratch, st); break;
    case 20: launch_strip_kp<T, 20>(pb, si, rhs, x, scratch, st); break;
    default: set_error("unsupported blocked term count"); throw ArgError();
  }
}

void launch_strip_solve(const hh_problem* pb, int si, const c128* rhs, c128* x, void* scratch,
                        hipStream_t st) {
  const FactorSet& fs = pb->fs;
  if (fs.max_kl > HH_KL_WINDOW) {
    const int SL = fs.strips[si].SL;
    const bool dbl = fs.precision == HH_FP64;
    const void* img = fs.img;
    if (dbl && SL == 2)
      hipLaunchKernelGGL((k_strip_solve_lm<double, LaneMajorShape<double>::D, 2>), dim3(1), dim3(64), 0,
                         st, fs.d_strips, si, img, fs.piv, rhs, x, (c128*)scratch);
    else if (dbl)
      hipLaunchKernelGGL((k_strip_solve_lm<double, LaneMajorShape<double>::D, 3>), dim3(1), dim3(64), 0,
                         st, fs.d_strips, si, img, fs.piv, rhs, x, (c128*)scratch);
    else if (SL == 2)
      hipLaunchKernelGGL((k_strip_solve_lm<float, LaneMajorShape<float>::D, 2>), dim3(1), dim3(64), 0,
                         st, fs.d_strips, si, img, fs.piv, rhs, x, (c64*)scratch);
    else
      hipLaunchKernelGGL((k_strip_solve_lm<float, LaneMajorShape<float>::D, 3>), dim3(1), dim3(64), 0,
                         st, fs.d_strips, si, img, fs.piv, rhs, x, (c64*)scratch);
    HH_HIP(hipGetLastError());
    return;
  }
  if (pb->fs.precision == HH_FP64)
    launch_strip_t<double>(pb, si, rhs, x, scratch, st);
  else
    launch_strip_t<float>(pb, si, rhs, x, scratch, st);
  HH_HIP(hipGetLastError());
}

}  // namespace hh
