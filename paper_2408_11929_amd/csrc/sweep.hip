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
    b[c] = lane < ns ? ld<T>(x[c], lane) : zero;
    nxtA[c] = 64 + lane < ns ? ld<T>(x[c], 64 + lane) : zero;
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
        nxtA[c] = e < ns ? ld<T>(x[c], e) : zero;
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
      b[c][k] = E < ns ? ld<T>(x[c], ns - 1 - E) : zero;
    }
    const int E = 64 * S + lane;
    nxtA[c] = E < ns ? ld<T>(x[c], ns - 1 - E) : zero;
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
        nxtA[c] = E < ns ? ld<T>(x[c], ns - 1 - E) : zero;
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

// Blocked row substitution for an unpivoted strip (image layout in
// factor.hip): out_i = d_i (in_i - sum_{c=1..K} T(i, c) out_{i-c}) in blocks
// of B = HH_BLK outputs, each a dense map of the K previous outputs and the B
// block inputs.  Lane l = r + B p accumulates KP terms of output r; the P = 64/B
// partial sums are combined by lane shuffles, after which all P lanes of a row
// hold the same (bitwise) sum.
//
// The K previous outputs and the upcoming inputs live in a 256-entry LDS ring
// (position i at slot i & 255) mirrored into slots 256..511, so the KP
// consecutive reads of a lane never wrap and use immediate offsets.  The loop
// runs in steps of U blocks (R = U B rows).  Everything a step needs from
// memory is requested one step earlier, at the start of the previous step:
// the maps of its U blocks (two register buffers, the loop unrolled by two
// steps so that the buffers keep fixed registers) and 64 more inputs, which
// enter the ring one step later (the ring then holds inputs up to row
// jR + 191 - R, and no live position is 256 or more rows behind that).  The outputs of a step are written back at
// the start of the next one.  Issuing all memory traffic of a step together
// keeps the loop-carried waits short: whatever the hardware counters make the
// loop head wait for was requested a whole step before.  The map array ends
// in zero blocks and reads past the end are clamped, so the body is free of
// bounds tests (positions past ns meet only zero map entries: rows >= ns of a
// map are zero and no row < ns depends on a later position).  Single wave:
// the LDS accesses of one wave are performed in order, no barrier is needed.
// Rows are read through src and written through dst (lanes past the end
// write row ns-1 again, with the same value, so the write needs no branch).
template <class T, int KP, int U, class Src, class Dst>
__device__ __forceinline__ void solve_blocked(const Src& src, const Dst& dst, gptr<const cx<T>> G,
                                              int ns, int K, cx<T>* ring, int lane) {
  constexpr int B = HH_BLK, R = U * HH_BLK;
  static_assert(R <= 64 && 64 % R == 0, "a step must divide 64 rows");
  const cx<T> zero = mk((T)0, (T)0);
  const int r = lane % B, p = lane / B;
  const int nst = (ns + R - 1) / R;
  auto put = [&](int i, cx<T> v) {
    ring[i & 255] = v;
    ring[(i & 255) + 256] = v;
  };
#pragma unroll
  for (int q = 0; q < 8; ++q) ring[64 * q + lane] = zero;
  put(lane, src.get(src.load(lane)));
  put(64 + lane, src.get(src.load(64 + lane)));
  // before step j, pend holds rows jR + 128 - R + lane
  typename Src::P pend = src.load(128 - R + lane);
  cx<T> g[2][U][KP];
  gptr<const cx<T>> gp = G + lane;
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int t = 0; t < KP; ++t) g[0][u][t] = ld<T>(gp, (long long)(u * KP + t) * 64);
  gp = gp + (long long)U * KP * 64;
  for (int j0 = 0; j0 < nst; j0 += 2) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = j0 + h;
      // requests for the next step: maps, inputs; write-back of the last step
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int t = 0; t < KP; ++t) g[1 - h][u][t] = ld<T>(gp, (long long)(u * KP + t) * 64);
      gp = gp + (long long)U * KP * 64;
      put(j * R + 128 - R + lane, src.get(pend));
      pend = src.load(j * R + 128 + lane);
      if (j > 0) {
        const int q = (j - 1) * R + lane % R, qs = q < ns ? q : ns - 1;
        dst.put(qs, ring[qs & 255]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i0 = j * R + B * u;
        const cx<T>* win = ring + ((i0 - K + p * KP) & 255);
        cx<T> a0 = zero, a1 = zero;
#pragma unroll
        for (int t = 0; t < KP; t += 2) {
          a0 = a0 + g[h][u][t] * win[t];
          if (t + 1 < KP) a1 = a1 + g[h][u][t + 1] * win[t + 1];
        }
        cx<T> acc = a0 + a1;
#pragma unroll
        for (int off = B; off < 64; off <<= 1)
          acc = acc + mk(__shfl_xor(acc.re, off, 64), __shfl_xor(acc.im, off, 64));
        put(i0 + r, acc);
      }
    }
  }
  const int q = (((nst + 1) & ~1) - 1) * R + lane % R, qs = q < ns ? q : ns - 1;
  dst.put(qs, ring[qs & 255]);
}

// g = sum_d coef_d z[p + off_d] on interface node (i, j) = p.
template <class T>
__device__ __forceinline__ cx<T> transmission(gptr<const cx<T>> coef, gptr<cx<T>> z, int i, int j,
                                              int n) {
  const int di[7] = {-1, 0, -1, 0, 1, 0, 1};
  const int dj[7] = {-1, -1, 0, 0, 0, 1, 1};
  cx<T> g = mk((T)0, (T)0);
#pragma unroll
  for (int d = 0; d < 7; ++d) {
    const int ii = i + di[d], jj = j + dj[d];
    if (ii < 0 || ii >= n || jj < 0 || jj >= n) continue;
    g = g + ld<T>(coef, d) * ld<T>(z, (long long)jj * n + ii);
  }
  return g;
}

// Streams of the blocked substitution.  load(i) issues the memory reads of
// row i (clamped to the last row) and returns them raw; get() forms the value
// when the row enters the ring, one step later.
template <class T>
struct SrcVec {  // x[i] (rev: x[ns-1-i]) in the working precision
  gptr<const cx<T>> x;
  int ns;
  bool rev;
  using P = cx<T>;
  __device__ P load(int i) const {
    i = i < ns ? i : ns - 1;
    return ld<T>(x, rev ? ns - 1 - i : i);
  }
  __device__ cx<T> get(const P& v) const { return v; }
};
template <class T>
struct SrcC128 {  // strip-local FP64 right-hand side, forward order
  gptr<const c128> b;
  int ns;
  using P = c128;
  __device__ P load(int i) const {
    const int q = i < ns ? i : ns - 1;
    return mk(b[q].re, b[q].im);
  }
  __device__ cx<T> get(const P& v) const { return mk((T)v.re, (T)v.im); }
};
// Strip right-hand side R_s r + g, forward order: local row q = l w + t is the
// global node (a + t, l) of an x strip or (l, a + t) of a y strip; the
// transmission data of node line l sit in LDS (e1 on t = 0 where the strip has
// a Gamma_{s,1} side, e2 on t = w - 1 where Gamma_{s,2} data apply).
template <class T>
struct SrcGather {
  gptr<const c128> r;
  const cx<T>* gl1;
  const cx<T>* gl2;
  int ns, w, n, a, dir;
  bool use1, use2;
  struct P {
    c128 v;
    cx<T> e1, e2;
    bool f1, f2;
  };
  __device__ P load(int i) const {
    const int q = i < ns ? i : ns - 1;
    const int l = q / w, t = q - l * w;
    const long long p = dir == 0 ? (long long)l * n + a + t : (long long)(a + t) * n + l;
    P o;
    o.v = mk(r[p].re, r[p].im);
    o.e1 = gl1[l];
    o.e2 = gl2[l];
    o.f1 = use1 && t == 0;
    o.f2 = use2 && t == w - 1;
    return o;
  }
  __device__ cx<T> get(const P& o) const {
    const cx<T> v = mk((T)o.v.re, (T)o.v.im);
    return o.f1 ? v + o.e1 : (o.f2 ? v + o.e2 : v);
  }
};
template <class T>
struct DstVec {  // x[i] (rev: x[ns-1-i])
  gptr<cx<T>> x;
  int ns;
  bool rev;
  __device__ void put(int i, cx<T> v) const { st<T>(x, rev ? ns - 1 - i : i, v); }
};
template <class T>
struct DstC128 {  // strip-local FP64 output, reversed order
  gptr<c128> x;
  int ns;
  __device__ void put(int i, cx<T> v) const {
    const int q = ns - 1 - i;
    x[q].re = (double)v.re;
    x[q].im = (double)v.im;
  }
};
// Scatter of the strip solution over the global vector, reversed order (the
// back substitution produces the last local row first).
template <class T>
struct DstScatter {
  gptr<cx<T>> z;
  int ns, w, n, a, dir;
  __device__ void put(int i, cx<T> v) const {
    const int q = ns - 1 - i;
    const int l = q / w, t = q - l * w;
    const long long p = dir == 0 ? (long long)l * n + a + t : (long long)(a + t) * n + l;
    st<T>(z, p, v);
  }
};

// One workgroup (one wave) runs one double sweep.  Per strip: the
// transmission data of its interfaces go to LDS (forward: g_{s,1} from the
// current z, also kept for the backward pass; backward: the kept g_{s,1} and
// g_{s,2} from the current z), then the forward substitution streams the
// gathered right-hand side into the strip buffer and the back substitution
// streams the solution from it into z.  Strips whose factorisation pivoted
// take the lane-major path with explicit gather and scatter passes.
// Dynamic LDS: the 512-entry ring and two node lines of transmission data.
template <class T, int D, int S, int KP, int U>
__global__ __launch_bounds__(64) void k_sweep(const SweepTask* __restrict__ tasks) {
  extern __shared__ char smem_raw[];
  const SweepTask& tk = tasks[blockIdx.x];
  const int lane = threadIdx.x;
  const int n = uni(tk.n), N = uni(tk.N);
  cx<T>* ring = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* gl1 = ring + 512;
  cx<T>* gl2 = gl1 + n;
  const cx<T>* img = uniptr((const cx<T>*)tk.img);
  const int* pivb = uniptr(tk.piv);
  const cx<T>* trb = uniptr((const cx<T>*)tk.tr);
  const int* pflag = uniptr(tk.pflag);
  gptr<cx<T>> z = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch.z);
  gptr<cx<T>> rho = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch.rho);
  gptr<cx<T>> g1 = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch.g1);
  gptr<const c128> r = (gptr<const c128>)uniptr(tk.ch.r);
  const StripDesc* strips = uniptr(tk.ch.strips);
  const cx<T> zero = mk((T)0, (T)0);
  for (int step = 0; step < 2 * N - 1; ++step) {
    const bool fwd = step < N;
    const int s = fwd ? step : 2 * N - 2 - step;
    const StripDesc* sp = strips + s;
    const int ns = uni(sp->ns), w = uni(sp->w), kl = uni(sp->kl);
    const int dir = uni(sp->dir), a = uni(sp->a), has1 = uni(sp->has1), has2 = uni(sp->has2);
    const long long img_off = uni(sp->img_off), piv_off = uni(sp->piv_off);
    const long long t1off = uni(sp->tr1_off), t2off = uni(sp->tr2_off);
    const int pivoted = uni(pflag[uni(sp->gid)]);
    const bool use2 = has2 && !fwd;
    for (int l = lane; l < n; l += 64) {
      cx<T> e1 = zero, e2 = zero;
      if (has1) {
        if (fwd) {
          const int i = dir == 0 ? a : l, j = dir == 0 ? l : a;
          e1 = transmission<T>((gptr<const cx<T>>)(trb + t1off + 7LL * l), z, i, j, n);
          st<T>(g1, (long long)s * n + l, e1);
        } else {
          e1 = ld<T>(g1, (long long)s * n + l);
        }
      }
      if (use2) {
        const int at = a + w - 1;
        const int i = dir == 0 ? at : l, j = dir == 0 ? l : at;
        e2 = transmission<T>((gptr<const cx<T>>)(trb + t2off + 7LL * l), z, i, j, n);
      }
      gl1[l] = e1;
      gl2[l] = e2;
    }
    __syncthreads();
    const SrcGather<T> gather{r, gl1, gl2, ns, w, n, a, dir, has1 != 0, use2};
    if (!pivoted) {
      const cx<T>* GL = img + img_off;
      const cx<T>* GU = GL + blocked_blocks(ns) * KP * 64;
      solve_blocked<T, KP, U>(gather, DstVec<T>{rho, ns, false}, (gptr<const cx<T>>)GL, ns, kl,
                              ring, lane);
      __syncthreads();
      solve_blocked<T, KP, U>(SrcVec<T>{(gptr<const cx<T>>)rho, ns, true},
                              DstScatter<T>{z, ns, w, n, a, dir}, (gptr<const cx<T>>)GU, ns, kl,
                              ring, lane);
    } else {
      for (int q = lane; q < ns; q += 64) st<T>(rho, q, gather.get(gather.load(q)));
      __syncthreads();
      gptr<cx<T>> x[1] = {rho};
      gptr<const cx<T>> Lm[1] = {(gptr<const cx<T>>)(img + img_off)};
      gptr<const int> pv[1] = {(gptr<const int>)(pivb + piv_off)};
      solve_lower<T, 1, D>(x, Lm, pv, ns, lane);
      __syncthreads();
      const long long NP = ns + HH_PAD;
      gptr<const cx<T>> Um[1] = {(gptr<const cx<T>>)(img + img_off + NP * 64)};
      gptr<const cx<T>> rdg[1] = {(gptr<const cx<T>>)(img + img_off + NP * 64 * (1 + S))};
      solve_upper<T, 1, D, S>(x, Um, rdg, ns, lane);
      __syncthreads();
      const DstScatter<T> out{z, ns, w, n, a, dir};
      for (int q = lane; q < ns; q += 64) out.put(ns - 1 - q, ld<T>(rho, q));
    }
    __syncthreads();
  }
}

// One strip solve in FP64 in/out (test hook); work: ns elements of scratch.
template <class T, int D, int S, int KP, int U>
__global__ __launch_bounds__(64) void k_strip_solve(const StripDesc* __restrict__ strips, int si,
                                                    const void* __restrict__ img,
                                                    const int* __restrict__ pivb,
                                                    const int* __restrict__ pflag,
                                                    const c128* __restrict__ rhs, c128* __restrict__ x,
                                                    cx<T>* __restrict__ work) {
  __shared__ cx<T> ring[512];
  const StripDesc* sp = strips + si;
  const int ns = uni(sp->ns), kl = uni(sp->kl);
  const long long ioff = uni(sp->img_off), poff = uni(sp->piv_off);
  const int pivoted = uni(pflag[si]);
  const int lane = threadIdx.x;
  const cx<T>* im = (const cx<T>*)img;
  gptr<cx<T>> wk = (gptr<cx<T>>)work;
  const SrcC128<T> in{(gptr<const c128>)rhs, ns};
  if (!pivoted) {
    const cx<T>* GL = im + ioff;
    const cx<T>* GU = GL + blocked_blocks(ns) * KP * 64;
    solve_blocked<T, KP, U>(in, DstVec<T>{wk, ns, false}, (gptr<const cx<T>>)GL, ns, kl, ring, lane);
    __syncthreads();
    solve_blocked<T, KP, U>(SrcVec<T>{(gptr<const cx<T>>)wk, ns, true},
                            DstC128<T>{(gptr<c128>)x, ns}, (gptr<const cx<T>>)GU, ns, kl, ring,
                            lane);
  } else {
    for (int q = lane; q < ns; q += 64) st<T>(wk, q, in.get(in.load(q)));
    __syncthreads();
    gptr<cx<T>> xs[1] = {wk};
    gptr<const cx<T>> Lm[1] = {(gptr<const cx<T>>)(im + ioff)};
    gptr<const int> pv[1] = {(gptr<const int>)(pivb + poff)};
    solve_lower<T, 1, D>(xs, Lm, pv, ns, lane);
    __syncthreads();
    const long long NP = ns + HH_PAD;
    gptr<const cx<T>> Um[1] = {(gptr<const cx<T>>)(im + ioff + NP * 64)};
    gptr<const cx<T>> rdg[1] = {(gptr<const cx<T>>)(im + ioff + NP * 64 * (1 + S))};
    solve_upper<T, 1, D, S>(xs, Um, rdg, ns, lane);
    __syncthreads();
    for (int q = lane; q < ns; q += 64) {
      const cx<T> v = ld<T>(wk, q);
      x[q] = mk((double)v.re, (double)v.im);
    }
  }
}

}  // namespace

// Template choice.  D: coefficient prefetch depth of the pivoted path (deep
// enough to cover memory latency, small enough to fit the register file);
// KP: terms per lane of the blocked path (fixes S: KP <= 12 <=> kl <= 31);
// U: blocks per step of the blocked path (two steps of maps are held in
// registers).
template <class T, int KP>
struct SweepShape {
  static constexpr bool dbl = sizeof(T) == 8;
  static constexpr int S = KP <= 12 ? 1 : 2;
  static constexpr int D = S == 1 ? (dbl ? 16 : 32) : (dbl ? 8 : 16);
  static constexpr int U = dbl ? (KP <= 10 ? 2 : 1) : (KP <= 10 ? 4 : 2);
};

template <class T, int KP>
static void launch_sweep_kp(const SweepTask* d, int ntasks, int nmax, hipStream_t st) {
  using Sh = SweepShape<T, KP>;
  const void* fn = (const void*)k_sweep<T, Sh::D, Sh::S, KP, Sh::U>;
  const size_t lds = (512 + 2 * (size_t)nmax) * sizeof(cx<T>);
  if (lds > 64 * 1024)
    HH_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_sweep<T, Sh::D, Sh::S, KP, Sh::U>), dim3(ntasks), dim3(64), lds, st, d);
}

template <class T>
static void launch_sweep_t(const SweepTask* d, int ntasks, int KP, int nmax, hipStream_t st) {
  switch (KP) {
    case 8: launch_sweep_kp<T, 8>(d, ntasks, nmax, st); break;
    case 10: launch_sweep_kp<T, 10>(d, ntasks, nmax, st); break;
    case 12: launch_sweep_kp<T, 12>(d, ntasks, nmax, st); break;
    case 16: launch_sweep_kp<T, 16>(d, ntasks, nmax, st); break;
    case 20: launch_sweep_kp<T, 20>(d, ntasks, nmax, st); break;
    default: set_error("unsupported blocked term count %d", KP); throw ArgError();
  }
}

void launch_sweep(const SweepTask* d_tasks, int ntasks, int precision, int KP, int nmax,
                  hipStream_t st) {
  if (ntasks <= 0) return;
  if (precision == HH_FP64)
    launch_sweep_t<double>(d_tasks, ntasks, KP, nmax, st);
  else
    launch_sweep_t<float>(d_tasks, ntasks, KP, nmax, st);
  HH_HIP(hipGetLastError());
}

template <class T, int KP>
static void launch_strip_kp(const hh_problem* pb, int si, const c128* rhs, c128* x, void* scratch,
                            hipStream_t st) {
  using Sh = SweepShape<T, KP>;
  const FactorSet& fs = pb->fs;
  hipLaunchKernelGGL((k_strip_solve<T, Sh::D, Sh::S, KP, Sh::U>), dim3(1), dim3(64), 0, st,
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
  if (pb->fs.precision == HH_FP64)
    launch_strip_t<double>(pb, si, rhs, x, scratch, st);
  else
    launch_strip_t<float>(pb, si, rhs, x, scratch, st);
  HH_HIP(hipGetLastError());
}

}  // namespace hh
