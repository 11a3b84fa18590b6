// Double-sweep preconditioner application (Sec. 2, eqs. (2)-(4)).
//
// One 64-lane workgroup runs whole double sweeps: forward over strips 1..N
// (eq. (2), zero data on Gamma_{s,2}), backward over N-1..1 (eq. (3), reusing
// the Gamma_{s,1} data of v_{s-1} formed in the forward pass and taking the
// Gamma_{s,2} data from u_{s+1}); u_N = v_N, so 2N-1 strip solves.  Every
// strip solve gathers the strip right-hand side R_s r + g, runs the pivoted
// forward substitution with L and the back substitution with U from the solve
// image of factor.hip, and scatters the strip solution over the global vector
// (the most recent solve wins in the overlaps).
//
// A workgroup carries C independent chains (C = 2: typically the x and the y
// sweep of one right-hand side, which walk strips of identical sizes) and
// interleaves their steps, so that the dependency latency of one chain is
// hidden behind the other's instructions.  Other workgroups handle the other
// right-hand sides, so one launch covers a whole batch of applications.
//
// Transmission data (eq. (4), zeroth-order Robin): for an interface node,
// g = sum_d coef_d z[p + off_d] over the 7-point stencil, with coef = (A_s - A)
// on that row, precomputed at factorisation time.
//
// Band substitution.  Both triangular solves are the recurrence
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

struct ChainView {
  int dir, a, has1, has2;
  long long img_off, piv_off, t1off, t2off;
};

template <class T, int C, int D, int S>
__global__ __launch_bounds__(64) void k_sweep(const SweepTask* __restrict__ tasks) {
  const SweepTask& tk = tasks[blockIdx.x];
  const int lane = threadIdx.x;
  const int n = uni(tk.n), N = uni(tk.N);
  const cx<T>* img = uniptr((const cx<T>*)tk.img);
  const int* pivb = uniptr(tk.piv);
  const cx<T>* trb = uniptr((const cx<T>*)tk.tr);
  gptr<cx<T>> z[C], rho[C], g1[C];
  gptr<const c128> r[C];
  const StripDesc* strips[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    z[c] = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch[c].z);
    rho[c] = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch[c].rho);
    g1[c] = (gptr<cx<T>>)uniptr((cx<T>*)tk.ch[c].g1);
    r[c] = (gptr<const c128>)uniptr(tk.ch[c].r);
    strips[c] = uniptr(tk.ch[c].strips);
  }
  for (int step = 0; step < 2 * N - 1; ++step) {
    const bool fwd = step < N;
    const int s = fwd ? step : 2 * N - 2 - step;
    const int ns = uni(strips[0][s].ns), w = uni(strips[0][s].w);
    ChainView cv[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const StripDesc* sp = strips[c] + s;
      cv[c].dir = uni(sp->dir);
      cv[c].a = uni(sp->a);
      cv[c].has1 = uni(sp->has1);
      cv[c].has2 = uni(sp->has2);
      cv[c].img_off = uni(sp->img_off);
      cv[c].piv_off = uni(sp->piv_off);
      cv[c].t1off = uni(sp->tr1_off);
      cv[c].t2off = uni(sp->tr2_off);
    }
    // gather R_s r into the strip buffer (local q = l*w + t)
    {
      int l = lane / w, t = lane - (lane / w) * w;
      const int dl = 64 / w, dt = 64 - (64 / w) * w;
      for (int q = lane; q < ns; q += 64) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const long long p = cv[c].dir == 0 ? (long long)l * n + cv[c].a + t
                                             : (long long)(cv[c].a + t) * n + l;
          const c128 rv = mk(r[c][p].re, r[c][p].im);
          st<T>(rho[c], q, mk((T)rv.re, (T)rv.im));
        }
        l += dl;
        t += dt;
        if (t >= w) {
          t -= w;
          l += 1;
        }
      }
    }
    __syncthreads();
    // add the transmission data on Gamma_{s,1} (stored from v_{s-1}) and Gamma_{s,2}
    for (int l = lane; l < n; l += 64) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        if (cv[c].has1) {
          cx<T> g;
          if (fwd) {
            const int i = cv[c].dir == 0 ? cv[c].a : l, j = cv[c].dir == 0 ? l : cv[c].a;
            g = transmission<T>((gptr<const cx<T>>)(trb + cv[c].t1off + 7LL * l), z[c], i, j, n);
            st<T>(g1[c], (long long)s * n + l, g);
          } else {
            g = ld<T>(g1[c], (long long)s * n + l);
          }
          const long long q = (long long)l * w;
          st<T>(rho[c], q, ld<T>(rho[c], q) + g);
        }
        if (cv[c].has2 && !fwd) {
          const int at = cv[c].a + w - 1;
          const int i = cv[c].dir == 0 ? at : l, j = cv[c].dir == 0 ? l : at;
          const cx<T> g = transmission<T>((gptr<const cx<T>>)(trb + cv[c].t2off + 7LL * l), z[c], i, j, n);
          const long long q = (long long)l * w + w - 1;
          st<T>(rho[c], q, ld<T>(rho[c], q) + g);
        }
      }
    }
    __syncthreads();
    {
      gptr<const cx<T>> Lm[C];
      gptr<const int> pv[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        Lm[c] = (gptr<const cx<T>>)(img + cv[c].img_off);
        pv[c] = (gptr<const int>)(pivb + cv[c].piv_off);
      }
      solve_lower<T, C, D>(rho, Lm, pv, ns, lane);
    }
    __syncthreads();
    {
      gptr<const cx<T>> Um[C], rdg[C];
      const long long NP = ns + HH_PAD;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        Um[c] = (gptr<const cx<T>>)(img + cv[c].img_off + NP * 64);
        rdg[c] = (gptr<const cx<T>>)(img + cv[c].img_off + NP * 64 * (1 + S));
      }
      solve_upper<T, C, D, S>(rho, Um, rdg, ns, lane);
    }
    __syncthreads();
    {
      int l = lane / w, t = lane - (lane / w) * w;
      const int dl = 64 / w, dt = 64 - (64 / w) * w;
      for (int q = lane; q < ns; q += 64) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const long long p = cv[c].dir == 0 ? (long long)l * n + cv[c].a + t
                                             : (long long)(cv[c].a + t) * n + l;
          st<T>(z[c], p, ld<T>(rho[c], q));
        }
        l += dl;
        t += dt;
        if (t >= w) {
          t -= w;
          l += 1;
        }
      }
    }
    __syncthreads();
  }
}

// One strip solve in FP64 in/out (test hook).
template <class T, int D, int S>
__global__ __launch_bounds__(64) void k_strip_solve(const StripDesc* __restrict__ strips, int si,
                                                    const void* __restrict__ img,
                                                    const int* __restrict__ pivb,
                                                    const c128* __restrict__ rhs, c128* __restrict__ x,
                                                    cx<T>* __restrict__ work) {
  const StripDesc* sp = strips + si;
  const int ns = uni(sp->ns);
  const long long ioff = uni(sp->img_off), poff = uni(sp->piv_off);
  const long long NP = ns + HH_PAD;
  const int lane = threadIdx.x;
  gptr<cx<T>> wk[1] = {(gptr<cx<T>>)work};
  for (int q = lane; q < ns; q += 64) st<T>(wk[0], q, mk((T)rhs[q].re, (T)rhs[q].im));
  __syncthreads();
  gptr<const cx<T>> Lm[1] = {(gptr<const cx<T>>)((const cx<T>*)img + ioff)};
  gptr<const int> pv[1] = {(gptr<const int>)(pivb + poff)};
  solve_lower<T, 1, D>(wk, Lm, pv, ns, lane);
  __syncthreads();
  gptr<const cx<T>> Um[1] = {(gptr<const cx<T>>)((const cx<T>*)img + ioff + NP * 64)};
  gptr<const cx<T>> rdg[1] = {(gptr<const cx<T>>)((const cx<T>*)img + ioff + NP * 64 * (1 + S))};
  solve_upper<T, 1, D, S>(wk, Um, rdg, ns, lane);
  __syncthreads();
  for (int q = lane; q < ns; q += 64) {
    const cx<T> v = ld<T>(wk[0], q);
    x[q] = mk((double)v.re, (double)v.im);
  }
}

}  // namespace

// Prefetch depth D: deep enough to cover memory latency, small enough that
// C chains' coefficient buffers fit the register file.
void launch_sweep(const SweepTask* d_tasks, int ntasks, int precision, int S, int C,
                  hipStream_t st) {
  if (ntasks <= 0) return;
  if (S < 1 || S > 2 || C < 1 || C > 2) {
    set_error("unsupported sweep configuration S=%d C=%d", S, C);
    throw ArgError();
  }
  dim3 g(ntasks), b(64);
  if (precision == HH_FP64) {
    if (C == 1 && S == 1) hipLaunchKernelGGL((k_sweep<double, 1, 16, 1>), g, b, 0, st, d_tasks);
    if (C == 1 && S == 2) hipLaunchKernelGGL((k_sweep<double, 1, 8, 2>), g, b, 0, st, d_tasks);
    if (C == 2 && S == 1) hipLaunchKernelGGL((k_sweep<double, 2, 8, 1>), g, b, 0, st, d_tasks);
    if (C == 2 && S == 2) hipLaunchKernelGGL((k_sweep<double, 2, 4, 2>), g, b, 0, st, d_tasks);
  } else {
    if (C == 1 && S == 1) hipLaunchKernelGGL((k_sweep<float, 1, 32, 1>), g, b, 0, st, d_tasks);
    if (C == 1 && S == 2) hipLaunchKernelGGL((k_sweep<float, 1, 16, 2>), g, b, 0, st, d_tasks);
    if (C == 2 && S == 1) hipLaunchKernelGGL((k_sweep<float, 2, 16, 1>), g, b, 0, st, d_tasks);
    if (C == 2 && S == 2) hipLaunchKernelGGL((k_sweep<float, 2, 8, 2>), g, b, 0, st, d_tasks);
  }
  HH_HIP(hipGetLastError());
}

void launch_strip_solve(const hh_problem* pb, int si, const c128* rhs, c128* x, void* scratch,
                        hipStream_t st) {
  const FactorSet& fs = pb->fs;
  const int S = fs.strips[si].S;
  if (fs.precision == HH_FP64) {
    if (S == 1)
      hipLaunchKernelGGL((k_strip_solve<double, 16, 1>), dim3(1), dim3(64), 0, st, fs.d_strips, si,
                         fs.img, fs.piv, rhs, x, (c128*)scratch);
    else
      hipLaunchKernelGGL((k_strip_solve<double, 8, 2>), dim3(1), dim3(64), 0, st, fs.d_strips, si,
                         fs.img, fs.piv, rhs, x, (c128*)scratch);
  } else {
    if (S == 1)
      hipLaunchKernelGGL((k_strip_solve<float, 32, 1>), dim3(1), dim3(64), 0, st, fs.d_strips, si,
                         fs.img, fs.piv, rhs, x, (c64*)scratch);
    else
      hipLaunchKernelGGL((k_strip_solve<float, 16, 2>), dim3(1), dim3(64), 0, st, fs.d_strips, si,
                         fs.img, fs.piv, rhs, x, (c64*)scratch);
  }
  HH_HIP(hipGetLastError());
}

}  // namespace hh
