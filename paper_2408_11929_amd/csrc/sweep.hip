// Double-sweep preconditioner application (Sec. 2, eqs. (2)-(4)).
//
// One 64-lane workgroup runs the whole double sweep of one direction for one
// right-hand side: forward over strips 1..N (eq. (2), zero data on
// Gamma_{s,2}), backward over N-1..1 (eq. (3), reusing the Gamma_{s,1} data
// of v_{s-1} formed in the forward pass and taking the Gamma_{s,2} data from
// u_{s+1}); u_N = v_N, so 2N-1 strip solves.  Every strip solve gathers the
// strip right-hand side R_s r + g, runs the pivoted forward substitution with
// L and the back substitution with U from the factor format of factor.hip,
// and scatters the strip solution over the global vector (the most recent
// solve wins in the overlaps).  Independent workgroups handle the other
// direction and the other right-hand sides, so one launch covers a whole
// batch of preconditioner applications.
//
// Transmission data (eq. (4), zeroth-order Robin): for an interface node,
// g = sum_d coef_d z[p + off_d] over the 7-point stencil, with coef = (A_s - A)
// on that row, precomputed at factorisation time.
//
// Band substitution.  Both triangular solves are the recurrence
//     out_e = b_e (times 1/U_ee for U),  b_{e+c} -= coef(e, c) b_e,  c = 1..K
// over e = 0..ns-1 (reversed order for U), K = kl for L and 2 kl for U.
// Element e of the sliding window lives in lane e mod 64 (slot k holds the
// element 64k further on), so a step is two lane reads and one complex
// multiply-subtract per lane; the coefficients of the next D steps and the
// elements of the next 64-step block are prefetched so that no step waits
// on memory.
#include "hh_internal.h"

namespace hh {

namespace {

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

// Forward substitution with the row interchanges of partial pivoting:
// y = L^{-1} P b in place on x[0..ns).
template <class T, int D>
__device__ void solve_lower(cx<T>* __restrict__ x, const cx<T>* __restrict__ ab,
                            const int* __restrict__ piv, int ns, int kl, int ldab, int lane) {
  const int kv = 2 * kl;
  const cx<T> zero = mk((T)0, (T)0);
  auto elem = [&](int e) -> cx<T> { return e < ns ? x[e] : zero; };
  auto coef = [&](int j) -> cx<T> {
    int c = (lane - (j & 63)) & 63;
    if (j < ns && c >= 1 && c <= kl && j + c < ns) return ab[(long long)j * ldab + kv + c];
    return zero;
  };
  cx<T> b = elem(lane);
  cx<T> nxtA = elem(64 + lane);
  cx<T> nxt = zero, yout = zero;
  cx<T> cc[D], cn[D];
  int pc = lane < D && lane < ns ? piv[lane] : 0, pn = 0;
#pragma unroll
  for (int u = 0; u < D; ++u) cc[u] = coef(u);
  for (int j0 = 0; j0 < ns; j0 += D) {
    if ((j0 & 63) == 0) {
      nxt = nxtA;
      nxtA = elem(j0 + 128 + lane);
    }
#pragma unroll
    for (int u = 0; u < D; ++u) cn[u] = coef(j0 + D + u);
    pn = (lane < D && j0 + D + lane < ns) ? piv[j0 + D + lane] : 0;
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int j = j0 + u;
      if (j < ns) {
        const int lj = j & 63;
        const int lp = __builtin_amdgcn_readlane(pc, u) & 63;
        const cx<T> bj = rlc(b, lp);
        const cx<T> bp = rlc(b, lj);
        if (lane == lp) b = bp;
        if (lane == lj) {
          yout = bj;
          b = nxt;
        }
        b = cfms(b, cc[u], bj);
        if (lj == 63 || j == ns - 1) {
          int e = (j & ~63) + lane;
          if (lane <= lj) x[e] = yout;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < D; ++u) cc[u] = cn[u];
    pc = pn;
  }
}

// Back substitution with the scaled U of factor.hip: on entry x holds y, on
// exit U^{-1} y.  Works on reversed indices E = ns-1-e.  S slots per lane
// (window 2 kl + 1 <= 64 S).
template <class T, int D, int S>
__device__ void solve_upper(cx<T>* __restrict__ x, const cx<T>* __restrict__ ab, int ns, int kl,
                            int ldab, int lane) {
  const int kv = 2 * kl;
  const cx<T> zero = mk((T)0, (T)0);
  auto elem = [&](int E) -> cx<T> { return E < ns ? x[ns - 1 - E] : zero; };
  // coefficient of slot k at step J: row E + c of column j = ns-1-J, c = 64k + ((lane - lJ) & 63)
  auto coef = [&](int J, int k) -> cx<T> {
    int c = 64 * k + ((lane - (J & 63)) & 63);
    if (J < ns && c <= kv && J + c < ns) return ab[(long long)(ns - 1 - J) * ldab + kv - c];
    return zero;
  };
  cx<T> b[S];
#pragma unroll
  for (int k = 0; k < S; ++k) b[k] = elem(64 * k + lane);
  cx<T> nxtA = elem(64 * S + lane);
  cx<T> nxt = zero, xout = zero;
  cx<T> cc[S][D], cn[S][D];
#pragma unroll
  for (int u = 0; u < D; ++u)
#pragma unroll
    for (int k = 0; k < S; ++k) cc[k][u] = coef(u, k);
  for (int J0 = 0; J0 < ns; J0 += D) {
    if ((J0 & 63) == 0) {
      nxt = nxtA;
      nxtA = elem(J0 + 64 * S + 64 + lane);
    }
#pragma unroll
    for (int u = 0; u < D; ++u)
#pragma unroll
      for (int k = 0; k < S; ++k) cn[k][u] = coef(J0 + D + u, k);
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int J = J0 + u;
      if (J < ns) {
        const int lJ = J & 63;
        const cx<T> bJ = rlc(b[0], lJ);
        if (lane == lJ) xout = bJ * cc[0][u];  // slot-0 coefficient of lane lJ is 1/U_jj
#pragma unroll
        for (int k = 0; k < S; ++k) b[k] = cfms(b[k], cc[k][u], bJ);
        if (lane == lJ) {
#pragma unroll
          for (int k = 0; k + 1 < S; ++k) b[k] = b[k + 1];
          b[S - 1] = nxt;
        }
        if (lJ == 63 || J == ns - 1) {
          int E = (J & ~63) + lane;
          if (lane <= lJ) x[ns - 1 - E] = xout;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < D; ++u)
#pragma unroll
      for (int k = 0; k < S; ++k) cc[k][u] = cn[k][u];
  }
}

template <class T>
__device__ __forceinline__ long long global_index(const StripDesc& sd, int n, int l, int t) {
  return sd.dir == 0 ? (long long)l * n + sd.a + t : (long long)(sd.a + t) * n + l;
}

// g = sum_d coef_d z[p + off_d] on interface node (i, j) = p.
template <class T>
__device__ cx<T> transmission(const cx<T>* __restrict__ coef, const cx<T>* __restrict__ z,
                              long long p, int n) {
  const int i = (int)(p % n), j = (int)(p / n);
  const int di[7] = {-1, 0, -1, 0, 1, 0, 1};
  const int dj[7] = {-1, -1, 0, 0, 0, 1, 1};
  cx<T> g = mk((T)0, (T)0);
#pragma unroll
  for (int d = 0; d < 7; ++d) {
    int ii = i + di[d], jj = j + dj[d];
    if (ii < 0 || ii >= n || jj < 0 || jj >= n) continue;
    cx<T> cf = coef[d];
    if (cf.re == (T)0 && cf.im == (T)0) continue;
    g = g + cf * z[(long long)jj * n + ii];
  }
  return g;
}

template <class T, int D, int S>
__global__ __launch_bounds__(64) void k_sweep(const SweepTask* __restrict__ tasks) {
  const SweepTask tk = tasks[blockIdx.x];
  const int lane = threadIdx.x;
  const int n = tk.n, N = tk.N;
  cx<T>* z = (cx<T>*)tk.z;
  cx<T>* rho = (cx<T>*)tk.rho;
  cx<T>* g1 = (cx<T>*)tk.g1;
  const cx<T>* trb = (const cx<T>*)tk.tr;
  for (int step = 0; step < 2 * N - 1; ++step) {
    const bool fwd = step < N;
    const int s = fwd ? step : 2 * N - 2 - step;
    const StripDesc sd = tk.strips[s];
    const cx<T>* ab = (const cx<T>*)tk.band + sd.band_off;
    // gather R_s r + g_{s,1} (+ g_{s,2} on the way back)
    for (int q = lane; q < sd.ns; q += 64) {
      const int l = q / sd.w, t = q - l * sd.w;
      const long long p = global_index<T>(sd, n, l, t);
      c128 rv = tk.r[p];
      cx<T> v = mk((T)rv.re, (T)rv.im);
      if (t == 0 && sd.has1) {
        cx<T> g;
        if (fwd) {
          g = transmission<T>(trb + sd.tr1_off + 7LL * l, z, p, n);
          g1[(long long)s * n + l] = g;
        } else {
          g = g1[(long long)s * n + l];
        }
        v = v + g;
      }
      if (t == sd.w - 1 && sd.has2 && !fwd) v = v + transmission<T>(trb + sd.tr2_off + 7LL * l, z, p, n);
      rho[q] = v;
    }
    __syncthreads();
    solve_lower<T, D>(rho, ab, tk.piv + sd.piv_off, sd.ns, sd.kl, sd.ldab, lane);
    __syncthreads();
    solve_upper<T, D, S>(rho, ab, sd.ns, sd.kl, sd.ldab, lane);
    __syncthreads();
    for (int q = lane; q < sd.ns; q += 64) {
      const int l = q / sd.w, t = q - l * sd.w;
      z[global_index<T>(sd, n, l, t)] = rho[q];
    }
    __syncthreads();
  }
}

// One strip solve in FP64 in/out (test hook).
template <class T, int D, int S>
__global__ __launch_bounds__(64) void k_strip_solve(const StripDesc* __restrict__ strips, int si,
                                                    const void* __restrict__ band,
                                                    const int* __restrict__ pivb,
                                                    const c128* __restrict__ rhs, c128* __restrict__ x,
                                                    cx<T>* __restrict__ work) {
  const StripDesc sd = strips[si];
  const int lane = threadIdx.x;
  const cx<T>* ab = (const cx<T>*)band + sd.band_off;
  for (int q = lane; q < sd.ns; q += 64) work[q] = mk((T)rhs[q].re, (T)rhs[q].im);
  __syncthreads();
  solve_lower<T, D>(work, ab, pivb + sd.piv_off, sd.ns, sd.kl, sd.ldab, lane);
  __syncthreads();
  solve_upper<T, D, S>(work, ab, sd.ns, sd.kl, sd.ldab, lane);
  __syncthreads();
  for (int q = lane; q < sd.ns; q += 64) x[q] = mk((double)work[q].re, (double)work[q].im);
}

}  // namespace

void launch_sweep(const SweepTask* d_tasks, int ntasks, int precision, int klmax, hipStream_t st) {
  if (ntasks <= 0) return;
  if (klmax > 63) {
    set_error("strip band half-width %d exceeds the supported maximum 63", klmax);
    throw ArgError();
  }
  const bool one = 2 * klmax + 1 <= 64;
  if (precision == HH_FP64) {
    if (one)
      hipLaunchKernelGGL((k_sweep<double, 8, 1>), dim3(ntasks), dim3(64), 0, st, d_tasks);
    else
      hipLaunchKernelGGL((k_sweep<double, 8, 2>), dim3(ntasks), dim3(64), 0, st, d_tasks);
  } else {
    if (one)
      hipLaunchKernelGGL((k_sweep<float, 16, 1>), dim3(ntasks), dim3(64), 0, st, d_tasks);
    else
      hipLaunchKernelGGL((k_sweep<float, 16, 2>), dim3(ntasks), dim3(64), 0, st, d_tasks);
  }
  HH_HIP(hipGetLastError());
}

void launch_strip_solve(const hh_problem* pb, int si, const c128* rhs, c128* x, void* scratch,
                        hipStream_t st) {
  const FactorSet& fs = pb->fs;
  const bool one = 2 * fs.strips[si].kl + 1 <= 64;
  if (fs.precision == HH_FP64) {
    if (one)
      hipLaunchKernelGGL((k_strip_solve<double, 8, 1>), dim3(1), dim3(64), 0, st, fs.d_strips, si,
                         fs.band, fs.piv, rhs, x, (c128*)scratch);
    else
      hipLaunchKernelGGL((k_strip_solve<double, 8, 2>), dim3(1), dim3(64), 0, st, fs.d_strips, si,
                         fs.band, fs.piv, rhs, x, (c128*)scratch);
  } else {
    if (one)
      hipLaunchKernelGGL((k_strip_solve<float, 16, 1>), dim3(1), dim3(64), 0, st, fs.d_strips, si,
                         fs.band, fs.piv, rhs, x, (c64*)scratch);
    else
      hipLaunchKernelGGL((k_strip_solve<float, 16, 2>), dim3(1), dim3(64), 0, st, fs.d_strips, si,
                         fs.band, fs.piv, rhs, x, (c64*)scratch);
  }
  HH_HIP(hipGetLastError());
}

}  // namespace hh
