// Batched band LU with partial pivoting of every strip matrix (Sec. 2: the
// sweep is a block LU forward/backward substitution; Sec. 4 solves each
// strip problem directly).  One workgroup per strip, all strips of all
// directions in one launch.
//
// Storage (per strip, column-major, ldab = 3 kl + 1, kv = 2 kl): on entry,
// A_s(i, j) sits at column j, position kv + i - j (general band storage with
// kl rows of fill space on top).  The elimination keeps the active
// (kl+1) x (kv+1) window in LDS as a circular buffer, so each column step
// touches HBM only to retire one row of U and one column of L and to bring
// in the one row of A that enters the window.
//
// Pivot rule: largest |Re| + |Im| in the column, first index on ties.
//
// After the elimination a second pass writes the "solve image" the sweep
// kernels stream through, one 64-lane row per substitution step so that a step
// is one coalesced load (NP = ns + HH_PAD steps, zero rows past the end):
//   Lm[j][k][l]    multiplier L(j+c, j), c = 64 k + ((l - j) mod 64), if
//                  1 <= c <= kl   (k < SL: one slot unless kl >= 64)
//   Um[J][k][l]    U(j-c, j) / U(j, j) for column j = ns-1-J,
//                  c = 64 k + ((l - J) mod 64), if 1 <= c <= 2 kl   (k < S)
//   rd[J]          1 / U(j, j)
// Lane l then always holds the coefficient of the window element it owns.
// The pivot list is padded with identity interchanges.
#include <algorithm>

#include "hh_internal.h"

namespace hh {

namespace {

constexpr int LU_WAVES = 4;
constexpr int LU_THREADS = 64 * LU_WAVES;
constexpr int LU_ROWS = (63 + LU_WAVES - 1) / LU_WAVES;  // rows of the window per wave (kl <= 63)
constexpr int LU_CH = 16;  // column steps per staged chunk of entering rows

// A pivot the elimination cannot divide by: zero, not finite, or so large
// that its squared modulus overflows the strip precision.
template <class T>
__device__ __forceinline__ bool bad_pivot(T pd) {
  return !(pd > (T)0) || __builtin_isinf(pd);
}

template <class T>
__device__ __forceinline__ void wave_argmax(T& v, int& idx) {
  for (int off = 32; off >= 1; off >>= 1) {
    T v2 = __shfl_xor(v, off, 64);
    int i2 = __shfl_xor(idx, off, 64);
    if (v2 > v || (v2 == v && i2 < idx)) {
      v = v2;
      idx = i2;
    }
  }
}
__device__ __forceinline__ float rdl(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rdl(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <class T>
__device__ __forceinline__ cx<T> rdlc(cx<T> v, int l) {
  return mk(rdl(v.re, l), rdl(v.im, l));
}
// Lanes of one wave exchange data through LDS here.  Without this, such an
// exchange is a data race to the compiler, which may then keep a lane's own
// stores in registers and never load what other lanes wrote.  The fences
// stop it from moving or forwarding LDS accesses across the point; at
// wavefront scope they cost no wait, a wave's LDS accesses completing in
// order.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Column step j works on the (kl+1) x (2kl+1) window of rows j..j+kl and
// columns j..j+2kl, kept in LDS with rotating physical rows and columns
// (logical row r at (j + r) mod R, logical column c at (j + c) mod C).  Lane l
// of every wave owns the physical columns l and l + 64; the window rows are
// dealt out to the waves (row 1 + w + 8 i to wave w).  A step: every wave
// reads the pivot column (lane r holds row r) and picks the pivot -- a
// ballot against the diagonal settles the usual no-interchange case, only a
// real interchange runs the shuffle reduction; lane r forms the multiplier of
// row r; each wave updates its rows of the trailing window into registers
// (row rp takes the old row 0: the interchange), retires the pivot row as a
// row of U and the multipliers as a column of L, and after a barrier writes
// them back, the retired column slot becoming the next fill column and the
// retired row slot the entering row j+kl+1 (prefetched four steps ahead).
template <class T>
using lds_ptr = T __attribute__((address_space(3)))*;
template <class T>
__device__ __forceinline__ cx<T> ldw(lds_ptr<cx<T>> W, int i) {
  return mk(W[i].re, W[i].im);
}
template <class T>
__device__ __forceinline__ void stw(lds_ptr<cx<T>> W, int i, cx<T> v) {
  W[i].re = v.re;
  W[i].im = v.im;
}

template <class T, int NSL>
__global__ __launch_bounds__(LU_THREADS) void k_band_lu(const StripDesc* __restrict__ strips,
                                                        cx<T>* __restrict__ band,
                                                        int* __restrict__ pivbuf, int* err,
                                                        int* __restrict__ pflag) {
  extern __shared__ unsigned char smem_raw[];
  lds_ptr<cx<T>> W = (lds_ptr<cx<T>>)smem_raw;
  const StripDesc sd = strips[blockIdx.x];
  const int kl = sd.kl, kv = 2 * kl, R = kl + 1, C = kv + 1, ldab = sd.ldab, ns = sd.ns;
  cx<T>* ab = band + sd.band_off;
  int* piv = pivbuf + sd.piv_off;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform, so readlane(r) is scalar
  const cx<T> zero = mk((T)0, (T)0);

  // window at j = 0: logical (r, c) = physical (r, c)
  for (int e = tid; e < R * C; e += LU_THREADS) {
    const int r = e / C, c = e - r * C;
    cx<T> v = zero;
    if (r < ns && c < ns && r - c <= kl && c - r <= kl) v = ab[(long long)c * ldab + kv + r - c];
    stw(W, r * C + c, v);
  }
  // entering row of step j (row j+kl+1) at physical column pc: after the
  // step that slot holds logical column (pc - c0 - 1) mod C, c0 = j mod C
  // (the load is unconditional, from a clamped address: a select between a
  // global element and a local zero would become a flat load, which the LDS
  // waits of every step would then have to wait for)
  auto fetch = [&](int j, int c0, int pc) -> cx<T> {
    const int i = j + kl + 1;
    int cl = pc - c0 - 1;
    cl = cl < 0 ? cl + C : cl;
    const int col = j + 1 + cl;
    const bool in = pc < C && i < ns && col < ns;
    const long long at = in ? (long long)col * ldab + kv + i - col : 0;
    const cx<T> v = ab[at];
    return csel(in, v, zero);
  };
  auto wrap = [](int x, int m) { return x >= m ? x - m : x; };
  // Entering rows are staged through LDS in chunks of LU_CH steps: the rows
  // of chunk k+1 are loaded into registers (wave w: rows q = w mod LU_WAVES)
  // while chunk k runs, so the column steps themselves issue no global loads
  // and never wait for memory.
  constexpr int QW = LU_CH / LU_WAVES;
  lds_ptr<cx<T>> Sg = W + R * C;
  cx<T> stg[QW][NSL];
  auto load_chunk = [&](int jc, int cq) {
#pragma unroll
    for (int k = 0; k < QW; ++k) {
      const int q = wv + LU_WAVES * k;
      const int c0q = wrap(cq + q % C, C);
#pragma unroll
      for (int s = 0; s < NSL; ++s) stg[k][s] = fetch(jc + q, c0q, lane + 64 * s);
    }
  };
  load_chunk(0, 0);
  int r0 = 0, c0 = 0, cn = LU_CH % C;  // cn = (jc + LU_CH) mod C
  __syncthreads();

  for (int jc = 0; jc < ns; jc += LU_CH) {
#pragma unroll
    for (int k = 0; k < QW; ++k) {
      const int q = wv + LU_WAVES * k;
#pragma unroll
      for (int s = 0; s < NSL; ++s) {
        const int pc = lane + 64 * s;
        if (pc < C) stw(Sg, q * C + pc, stg[k][s]);
      }
    }
    load_chunk(jc + LU_CH, cn);
    cn = wrap(cn + LU_CH % C, C);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < LU_CH; ++u) {
      const int j = jc + u;
      if (j >= ns) break;
      auto prow = [&](int r) { return wrap(r0 + r, R); };
      // ---- pivot column, pivot choice (redundantly in every wave)
      const int rmax = min(kl, ns - 1 - j);
      const cx<T> val = csel(lane <= kl, ldw(W, prow(lane <= kl ? lane : kl) * C + c0), zero);
      const T av = lane <= rmax ? cabs1(val) : (T)-1;
      const T ad = rdl(av, 0);
      int rp = 0;
      if (__ballot(av > ad)) {  // a real interchange (rare): first index of the maximum
        T v = av;
        int idx = lane <= rmax ? lane : 64;
        wave_argmax(v, idx);
        rp = __builtin_amdgcn_readfirstlane(idx);
      }
      const int prp = prow(rp);
      const cx<T> pv = rdlc(val, rp);
      const T pd = pv.re * pv.re + pv.im * pv.im;
      const bool singular = bad_pivot(pd);
      const T ipd = singular ? (T)0 : (T)1 / pd;
      const cx<T> ipv = mk(pv.re * ipd, -pv.im * ipd);
      // multiplier of (new) row r, which is the old row 0 if r == rp
      const cx<T> v0 = rdlc(val, 0);
      const cx<T> Lr = csel(lane >= 1 && lane <= rmax, csel(lane == rp, v0, val) * ipv, zero);
      // pivot row (the new row of U) in the lane's columns
      cx<T> ucol[NSL];
#pragma unroll
      for (int s = 0; s < NSL; ++s) {
        const int pc = lane + 64 * s;
        ucol[s] = csel(pc < C, ldw(W, prp * C + (pc < C ? pc : C - 1)), zero);
      }
      if (wv == 0) {
        if (lane == 0) {
          piv[j] = j + rp;
          if (rp != 0) pflag[blockIdx.x] = 1;
          if (singular) atomicCAS(err, 0, (int)blockIdx.x + 1);
        }
        if (lane >= 1 && lane <= rmax) ab[(long long)j * ldab + kv + lane] = Lr;
#pragma unroll
        for (int s = 0; s < NSL; ++s) {
          const int pc = lane + 64 * s;
          int c = pc - c0;
          c = c < 0 ? c + C : c;
          if (pc < C && j + c < ns) ab[(long long)(j + c) * ldab + kv - c] = ucol[s];
        }
      }
      // ---- trailing update of this wave's rows, into registers
      cx<T> keep[LU_ROWS][NSL];
#pragma unroll
      for (int i = 0; i < LU_ROWS; ++i) {
        const int r = 1 + wv + LU_WAVES * i;
        if (r <= kl) {
          const int src = prow(r == rp ? 0 : r);
          const cx<T> l = rdlc(Lr, r);
#pragma unroll
          for (int s = 0; s < NSL; ++s) {
            const int pc = lane + 64 * s;
            const cx<T> w = csel(pc < C, ldw(W, src * C + (pc < C ? pc : C - 1)), zero);
            keep[i][s] = csel(pc == c0, zero, cfms(w, l, ucol[s]));
          }
        }
      }
      __syncthreads();
      // ---- write back; the retired row slot takes the entering row
#pragma unroll
      for (int i = 0; i < LU_ROWS; ++i) {
        const int r = 1 + wv + LU_WAVES * i;
        if (r <= kl) {
          const int pr = prow(r);
#pragma unroll
          for (int s = 0; s < NSL; ++s) {
            const int pc = lane + 64 * s;
            if (pc < C) stw(W, pr * C + pc, keep[i][s]);
          }
        }
      }
      if (wv == LU_WAVES - 1) {
#pragma unroll
        for (int s = 0; s < NSL; ++s) {
          const int pc = lane + 64 * s;
          if (pc < C) stw(W, r0 * C + pc, ldw(Sg, u * C + pc));
        }
      }
      r0 = wrap(r0 + 1, R);
      c0 = wrap(c0 + 1, C);
      __syncthreads();
    }
  }
}

// The same elimination by one wave with the window in registers, for
// 2 kl + 1 <= 64 and kl < KR.  Lane l owns the physical column slot l of the
// window of step j (logical column c = (l - c0) mod C, c0 = j mod C) and holds
// its rows j + r in a[r], r <= kl.  A step:
//  - lane c0 passes the pivot column through LDS so that lane r holds row r;
//    the pivot test and the multipliers are as in k_band_lu, and the
//    multipliers go back through LDS to every lane;
//  - every lane swaps its rows 0 and rp when the step interchanges, stores
//    its row-0 entry as the new row of U, and updates and shifts its rows at
//    once: a[r-1] = a[r] - L_r a[0], which keeps every register index fixed;
//  - the retired slot (lane c0) becomes column j + C, zero in the window but
//    for the entering row j + kl + 1.
// The registers past the window (r = kl+1 .. KR-1, whose multipliers are
// zero) carry the entering rows of the next steps: the row entering at step
// j + D, D = KR - 1 - kl, is put in a[KR-1] at step j and reaches a[kl]
// when it enters, so no register is chosen by kl.  Entering rows are read
// one chunk of CH steps ahead and pass through LDS.
// With redo set, only the strips that k_band_lu_h marked (pflag = 2, band
// packed again since) are factored.
template <class T, int KR, int CH>
__global__ __launch_bounds__(64) void k_band_lu_w(const StripDesc* __restrict__ strips,
                                                  cx<T>* __restrict__ band,
                                                  int* __restrict__ pivbuf, int* err,
                                                  int* __restrict__ pflag, int redo) {
  __shared__ cx<T> colb[64];      // pivot column, lane r = row r
  __shared__ cx<T> lbuf[64];      // multipliers
  __shared__ cx<T> ebuf[CH][64];  // entering rows of the current chunk
  __shared__ cx<T> xbuf[KR][64];  // the window, for an interchange
  if (redo) {
    if (pflag[blockIdx.x] != 2) return;
    if (threadIdx.x == 0) pflag[blockIdx.x] = 0;
  }
  const StripDesc sd = strips[blockIdx.x];
  const int kl = sd.kl, kv = 2 * kl, C = kv + 1, ldab = sd.ldab, ns = sd.ns;
  const int D = KR - 1 - kl;
  cx<T>* ab = band + sd.band_off;
  int* piv = pivbuf + sd.piv_off;
  const int lane = threadIdx.x;
  const cx<T> zero = mk((T)0, (T)0);
  auto wrap = [](int x, int m) { return x >= m ? x - m : x; };
  // entering row of step j (row j+kl+1) in this lane's slot, whose logical
  // column after the step is (lane - c0 - 1) mod C (clamped load, then a select)
  auto fetch = [&](int j) -> cx<T> {
    const int i = j + kl + 1, c0j = j % C;
    int cl = lane - c0j - 1;
    cl = cl < 0 ? cl + C : cl;
    const int col = j + 1 + cl;
    const bool in = lane < C && i < ns && col < ns;
    const cx<T> v = ab[in ? (long long)col * ldab + kv + i - col : 0];
    return csel(in, v, zero);
  };
  cx<T> a[KR];
#pragma unroll
  for (int r = 0; r < KR; ++r) {
    // rows of the first window, then the entering rows of steps 0 .. D-1
    const bool in = lane < C && r <= kl && r < ns && lane < ns && r - lane <= kl && lane - r <= kl;
    const cx<T> v = ab[in ? (long long)lane * ldab + kv + r - lane : 0];
    a[r] = r <= kl ? csel(in, v, zero) : fetch(r - kl - 1);
  }
  cx<T> nxt[CH];
#pragma unroll
  for (int u = 0; u < CH; ++u) nxt[u] = fetch(D + u);
  int c0 = 0;
  for (int jc = 0; jc < ns; jc += CH) {
    wave_lds_sync();
#pragma unroll
    for (int u = 0; u < CH; ++u) ebuf[u][lane] = nxt[u];
#pragma unroll
    for (int u = 0; u < CH; ++u) nxt[u] = fetch(jc + CH + D + u);
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int j = jc + u;
      if (j >= ns) break;
      const int rmax = min(kl, ns - 1 - j);
      const cx<T> ein = ebuf[u][lane];  // enters a[KR-1] after this step
      wave_lds_sync();
      if (lane == c0) {
#pragma unroll
        for (int r = 0; r < KR; ++r) colb[r] = a[r];
      }
      wave_lds_sync();
      const cx<T> val = csel(lane <= kl, colb[lane <= kl ? lane : 0], zero);
      const T av = lane <= rmax ? cabs1(val) : (T)-1;
      const T ad = rdl(av, 0);
      int rp = 0;
      if (__ballot(av > ad)) {  // a real interchange (rare): first index of the maximum
        T v = av;
        int idx = lane <= rmax ? lane : 64;
        wave_argmax(v, idx);
        rp = __builtin_amdgcn_readfirstlane(idx);
      }
      const cx<T> pv = rdlc(val, rp);
      const T pd = pv.re * pv.re + pv.im * pv.im;
      const bool singular = bad_pivot(pd);
      const T ipd = singular ? (T)0 : (T)1 / pd;
      const cx<T> ipv = mk(pv.re * ipd, -pv.im * ipd);
      const cx<T> v0 = rdlc(val, 0);
      const cx<T> Lr = csel(lane >= 1 && lane <= rmax, csel(lane == rp, v0, val) * ipv, zero);
      lbuf[lane] = Lr;
      wave_lds_sync();
      if (lane == 0) {
        piv[j] = j + rp;
        if (rp != 0) pflag[blockIdx.x] = 1;
        if (singular) atomicCAS(err, 0, (int)blockIdx.x + 1);
      }
      if (lane >= 1 && lane <= rmax) ab[(long long)j * ldab + kv + lane] = Lr;
      if (rp != 0) {  // interchange rows 0 and rp in every column (rare), through LDS
#pragma unroll
        for (int r = 0; r < KR; ++r) xbuf[r][lane] = a[r];
        wave_lds_sync();
        const cx<T> t = xbuf[rp][lane];
        xbuf[rp][lane] = xbuf[0][lane];
        xbuf[0][lane] = t;
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < KR; ++r) a[r] = xbuf[r][lane];
      }
      const cx<T> u0 = a[0];
      {
        int c = lane - c0;
        c = c < 0 ? c + C : c;
        if (lane < C && j + c < ns) ab[(long long)(j + c) * ldab + kv - c] = u0;
      }
      const bool ret = lane == c0;
#pragma unroll
      for (int r = 1; r < KR; ++r) {
        const cx<T> v = cfms(a[r], lbuf[r], u0);
        a[r - 1] = csel(ret && r - 1 < kl, zero, v);
      }
      a[KR - 1] = ein;
      c0 = wrap(c0 + 1, C);
    }
  }
}

// Band LU of a strip whose partial pivoting makes no interchange, by one wave
// with two lanes per column.  Without interchanges U keeps kl
// superdiagonals, so step j only touches the M = kl + 1 columns j .. j + kl:
// slot s (lanes s and s + 32) holds column j + ((s - c0) mod M), c0 = j mod M,
// and half h of the wave holds window rows h R .. h R + R - 1 in a[0..R-1]
// (rows j .. j + 2R - 1, 2R > kl; the rows past kl have not entered yet and
// their multipliers are zero).  A step:
//  - the pivot slot passes its column through LDS so that lane r holds row
//    r; a ballot against the diagonal finds a step where partial pivoting
//    (largest |Re| + |Im|, first index on ties) would interchange.  The strip
//    is then marked (pflag = 2) and left at the end of the chunk; its band is
//    packed again and k_band_lu_w factors it with interchanges;
//  - lane r forms the multiplier of row r, stores it as L(j + r, j) and
//    passes it through LDS to the half that holds row r;
//  - half 0 stores its row 0 as row j of U; v_permlane32_swap hands that row
//    to half 1, every lane updates and shifts its rows at once (a[k-1] =
//    a[k] - L a[0]), a second swap moves row R from half 1 to half 0, and
//    half 1 takes the row entering at the bottom;
//  - the pivot slot takes column j + M, untouched by every earlier step: its
//    rows j + 1 .. j + 2R come from the band, like the entering rows staged
//    in LDS one chunk of CH steps ahead.
// The stores of a step never overlap what later steps read from the band:
// U rows and L columns lie at or left of the current step.
template <class T>
__device__ __forceinline__ cx<T> half0_to_both(cx<T> v);
template <>
__device__ __forceinline__ c64 half0_to_both(c64 v) {
  const unsigned r = __float_as_uint(v.re), i = __float_as_uint(v.im);
  return mk(__uint_as_float(__builtin_amdgcn_permlane32_swap(r, r, false, false)[0]),
            __uint_as_float(__builtin_amdgcn_permlane32_swap(i, i, false, false)[0]));
}
template <>
__device__ __forceinline__ c128 half0_to_both(c128 v) {
  const unsigned long long r = __double_as_longlong(v.re), i = __double_as_longlong(v.im);
  const unsigned rl = (unsigned)r, rh = (unsigned)(r >> 32), il = (unsigned)i, ih = (unsigned)(i >> 32);
  const unsigned a = __builtin_amdgcn_permlane32_swap(rl, rl, false, false)[0];
  const unsigned b = __builtin_amdgcn_permlane32_swap(rh, rh, false, false)[0];
  const unsigned c = __builtin_amdgcn_permlane32_swap(il, il, false, false)[0];
  const unsigned d = __builtin_amdgcn_permlane32_swap(ih, ih, false, false)[0];
  return mk(__longlong_as_double(((long long)b << 32) | a), __longlong_as_double(((long long)d << 32) | c));
}
template <class T>
__device__ __forceinline__ cx<T> half1_to_both(cx<T> v);
template <>
__device__ __forceinline__ c64 half1_to_both(c64 v) {
  const unsigned r = __float_as_uint(v.re), i = __float_as_uint(v.im);
  return mk(__uint_as_float(__builtin_amdgcn_permlane32_swap(r, r, false, false)[1]),
            __uint_as_float(__builtin_amdgcn_permlane32_swap(i, i, false, false)[1]));
}
template <>
__device__ __forceinline__ c128 half1_to_both(c128 v) {
  const unsigned long long r = __double_as_longlong(v.re), i = __double_as_longlong(v.im);
  const unsigned rl = (unsigned)r, rh = (unsigned)(r >> 32), il = (unsigned)i, ih = (unsigned)(i >> 32);
  const unsigned a = __builtin_amdgcn_permlane32_swap(rl, rl, false, false)[1];
  const unsigned b = __builtin_amdgcn_permlane32_swap(rh, rh, false, false)[1];
  const unsigned c = __builtin_amdgcn_permlane32_swap(il, il, false, false)[1];
  const unsigned d = __builtin_amdgcn_permlane32_swap(ih, ih, false, false)[1];
  return mk(__longlong_as_double(((long long)b << 32) | a), __longlong_as_double(((long long)d << 32) | c));
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

template <class T, int R, int CH>
__global__ __launch_bounds__(64) void k_band_lu_h(const StripDesc* __restrict__ strips,
                                                  cx<T>* __restrict__ band,
                                                  int* __restrict__ pivbuf, int* err,
                                                  int* __restrict__ pflag) {
  constexpr int R2 = 2 * R;
  constexpr int NE = CH / 2;              // staged entering-row entries per lane (M <= 32)
  constexpr int NB = (CH * R2 + 63) / 64;  // staged entering-column entries per lane
  __shared__ cx<T> colb[32];               // pivot column, entry r = window row r
  __shared__ cx<T> ebuf[CH * 32 + 64];     // entering rows [step][logical column], spill slots
  __shared__ cx<T> nbuf[NB * 64];          // entering columns [step][window row]
  const StripDesc sd = strips[blockIdx.x];
  const int kl = sd.kl, kv = 2 * kl, M = kl + 1, ldab = sd.ldab, ns = sd.ns;
  cx<T>* ab = band + sd.band_off;
  int* piv = pivbuf + sd.piv_off;
  const int lane = threadIdx.x, h = lane >> 5, s = lane & 31;
  const bool act = s < M;
  const cx<T> zero = mk((T)0, (T)0);
  auto wrap = [](int x, int m) { return x >= m ? x - m : x; };
  // Staging of the chunk that starts at step jn: entry (u, c) of the entering
  // rows is A(jn + u + 2R, jn + u + 1 + c), the row that enters after step
  // jn + u in logical column c of the next step (zero left of the band);
  // entry (u, r) of the entering columns is A(jn + u + 1 + r, jn + u + M).
  // Each is A at band position jn ldab + off, so the offsets, the last row
  // or column an entry needs and its LDS slot are fixed per lane.
  int eoff[NE], elast[NE], epos[NE], noff[NB], nlast[NB];
#pragma unroll
  for (int t = 0; t < NE; ++t) {
    const int e = lane + 64 * t, u = e / M, c = e - u * M;
    const bool ok = u < CH && c >= R2 - 1 - kl;  // row - column = 2R - 1 - c <= kl
    eoff[t] = (u + 1 + c) * (ldab - 1) + kv + u + R2;
    elast[t] = ok ? u + R2 : 1 << 30;           // the row; the column is left of it
    epos[t] = u < CH ? u * 32 + c : CH * 32 + lane;
  }
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int e = lane + 64 * t, u = e / R2, r = e - u * R2;
    const bool ok = u < CH && r <= 2 * kl;  // row - column = 1 + r - M <= kl
    noff[t] = (u + M) * (ldab - 1) + kv + u + 1 + r;
    nlast[t] = ok ? max(u + 1 + r, u + M) : 1 << 30;
  }
  cx<T> ne[NE], nn[NB];
  auto fetch = [&](int jn) {
    const long long base = (long long)jn * ldab;
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const bool in = jn + elast[t] < ns;
      const cx<T> v = ab[in ? base + eoff[t] : 0];
      ne[t] = csel(in, v, zero);
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const bool in = jn + nlast[t] < ns;
      const cx<T> v = ab[in ? base + noff[t] : 0];
      nn[t] = csel(in, v, zero);
    }
  };
  cx<T> a[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = h * R + k;
    const bool in = act && i < ns && s < ns && i - s <= kl && s - i <= kl;
    const cx<T> v = ab[in ? (long long)s * ldab + kv + i - s : 0];
    a[k] = csel(in, v, zero);
  }
  fetch(0);
  // the pivot slot, the column of this slot and its U-row offset (row 0 at
  // ab[uoff + j]), its logical column after the step
  int c0 = 0, col = s, lcn = !act || s == 0 ? (act ? M - 1 : 0) : s - 1;
  long long uoff = (long long)col * (ldab - 1) + kv;
  // positive once this lane saw a step that needs an interchange or a zero pivot
  T badm = (T)-1;
  if (s == 0) {
#pragma unroll
    for (int k = 0; k < R; ++k) colb[h * R + k] = a[k];
  }
  // steps past ns change nothing; nor do those past the unknowns (sd.nr): the
  // identity rows after them are packed as their own factors, and no
  // earlier step reaches their columns
  const int nsteps = (sd.nr + CH - 1) / CH * CH;
  for (int j = nsteps + lane; j < ns; j += 64) piv[j] = j;
  for (int jc = 0; jc < nsteps; jc += CH) {
    wave_lds_sync();
#pragma unroll
    for (int t = 0; t < NE; ++t) ebuf[epos[t]] = ne[t];
#pragma unroll
    for (int t = 0; t < NB; ++t) nbuf[lane + 64 * t] = nn[t];
    fetch(jc + CH);
    // four steps per unrolled body: a whole chunk keeps so many per-step
    // constants alive that they spill to lanes of a VGPR
#pragma unroll 4
    for (int u = 0; u < CH; ++u) {
      const int j = jc + u;
      const int rmax = min(kl, ns - 1 - j);
      wave_lds_sync();
      // the pivot column as written by its slot: the pivot, lane r's row,
      // and every row of this lane's half
      const cx<T> pv = colb[0];
      const cx<T> val = colb[s];
      cx<T> lr[R];
#pragma unroll
      for (int k = 0; k < R; ++k) lr[k] = colb[h * R + k];
      const T pd = pv.re * pv.re + pv.im * pv.im;
      const T ipd = bad_pivot(pd) ? (T)0 : recip(pd);
      const cx<T> ipv = mk(pv.re * ipd, -pv.im * ipd);
      // row k of the half loses L(k) u0 = col(k) (u0 / pivot): the pivot
      // column is zero in the rows that have not entered and past the matrix
      const cx<T> a0 = a[0];
      const cx<T> w = half0_to_both(a0) * ipv;
      cx<T> t[R];
#pragma unroll
      for (int k = 0; k < R; ++k) t[k] = cfms(a[k], lr[k], w);
      const cx<T> up = half1_to_both(t[0]);
      const cx<T> ein = ebuf[u * 32 + lcn];
#pragma unroll
      for (int k = 0; k + 1 < R; ++k) a[k] = t[k + 1];
      a[R - 1] = csel(h == 0, up, ein);
      // the next pivot slot passes its column before the retired slot
      // reloads, so that the reload's wait overlaps the next step's; the
      // stores and the pivot test are off that chain
      const int c1 = wrap(c0 + 1, M);
      if (s == c1) {
#pragma unroll
        for (int k = 0; k < R; ++k) colb[h * R + k] = a[k];
      }
      if (s == c0) {
#pragma unroll
        for (int k = 0; k < R; ++k) a[k] = nbuf[u * R2 + h * R + k];
      }
      const T av = lane <= rmax ? cabs1(val) : (T)-1;
      // a running maximum, which the compiler keeps as one accumulator (an
      // OR of the steps' comparisons it would keep alive to the chunk end)
      const T d = bad_pivot(pd) && j < ns ? (T)1 : av - cabs1(pv);
      badm = fmax(badm, d);
      if (lane >= 1 && lane <= rmax) ab[(long long)j * ldab + kv + lane] = val * ipv;
      if (h == 0 && act && col < ns && j < ns) ab[uoff + j] = a0;
      if (s == c0) {
        col += M;
        uoff += (long long)M * (ldab - 1);
      }
      c0 = c1;
      lcn = lcn == 0 ? M - 1 : lcn - 1;
    }
    if (lane < CH && jc + lane < ns) piv[jc + lane] = jc + lane;
    if (__any(badm > (T)0)) {
      if (lane == 0) pflag[blockIdx.x] = 2;
      return;
    }
  }
}

// ---- wide bands (kl >= 64): blocked elimination with MFMA trailing updates
//
// Beyond the one-wave window of the kernels above, a strip is factored by a
// blocked right-looking band LU (the same pivot rule and the same storage;
// the multipliers of a column stay in the row order of its own step, so the
// lane-major substitution applies the interchanges as it goes).  One
// workgroup of four waves per strip:
//   1. the panel of LU_NB columns j0.. and the rows j0 .. j0+LU_NB-1+kl that
//      they reach are loaded to LDS and eliminated column by column
//      (pivot search, interchange within the panel, multipliers, rank-1
//      update of the panel's remaining columns);
//   2. L11^{-1} (unit lower, LU_NB x LU_NB) is formed in LDS;
//   3. the trailing columns j0+LU_NB .. j0+LU_NB-1+2kl (where U's fill can
//      reach) go through LDS LU_NB at a time: the panel's interchanges in
//      order, U12 = L11^{-1} A12 and A22 -= L21 U12, both products of 16 x 16
//      complex tiles on the matrix cores (four real f64 16x16x4 MFMAs per
//      complex step).
// The elimination runs in FP64 for either storage precision: a complex64
// strip is widened on load and its factors rounded once on store, so that
// the explicit L11^{-1} and the blocked updates do not lose accuracy against
// the column-by-column elimination (their complex64 rounding, step by step,
// gave three times the solve error of LAPACK's on a kl = 131 strip).
// Entries outside the band are zero in exact arithmetic (U's rows reach 2kl
// columns past the diagonal, L's columns kl rows below it), so the loads
// fill them with zeros and the stores skip them.
constexpr int LU_NB = 16;

template <class T>
struct MfmaT;
// Both take A as lane l = row l mod 16, k = l / 16 of a 4-wide k slice and B
// as lane l = k l / 16, column l mod 16; the accumulator's entry i of lane l
// is column l mod 16 and row row(l, i): 4 (l / 16) + i for f32, l / 16 + 4 i
// for f64 (rows interleaved), as measured on gfx950.
template <>
struct MfmaT<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};
template <>
struct MfmaT<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};

// C += sg A B for 16 x 16 complex tiles in LDS (row-major, strides lda, ldb),
// C held as two accumulators (real and imaginary parts) in the layout above.
template <class T>
__device__ __forceinline__ void ctile_mma(typename MfmaT<T>::v4& cre, typename MfmaT<T>::v4& cim,
                                          const cx<T>* A, int lda, const cx<T>* B, int ldb,
                                          int lane, T sg) {
#pragma unroll
  for (int k0 = 0; k0 < 16; k0 += 4) {
    const cx<T> a = A[(lane & 15) * lda + k0 + (lane >> 4)];
    const cx<T> b = B[(k0 + (lane >> 4)) * ldb + (lane & 15)];
    const T are = sg * a.re, aim = sg * a.im;
    cre = MfmaT<T>::op(are, b.re, cre);
    cre = MfmaT<T>::op(-aim, b.im, cre);
    cim = MfmaT<T>::op(are, b.im, cim);
    cim = MfmaT<T>::op(aim, b.re, cim);
  }
}

// Rows of the LDS panel and chunk: LU_NB + kl rounded up to whole tiles.
__host__ __device__ inline int lu_blk_rows(int kl) { return (LU_NB + kl + 15) / 16 * 16; }
__host__ inline size_t lu_blk_lds(int kl) {
  return (size_t)(2 * lu_blk_rows(kl) * LU_NB + LU_NB * LU_NB) * sizeof(c128) + 4 * sizeof(double) +
         (4 + LU_NB) * sizeof(int);
}

template <class T>
__global__ __launch_bounds__(256) void k_band_lu_blk(const StripDesc* __restrict__ strips,
                                                     cx<T>* __restrict__ band,
                                                     int* __restrict__ piv, int* __restrict__ err,
                                                     int* __restrict__ pflag) {
  using W = double;  // the elimination runs in FP64 whatever the storage
  using V4 = typename MfmaT<W>::v4;
  extern __shared__ unsigned char smem_raw[];
  const StripDesc sd = strips[blockIdx.x];
  const int ns = sd.ns, kl = sd.kl, kv = 2 * kl, ldab = sd.ldab;
  const int RM = lu_blk_rows(kl);
  cx<T>* ab = band + sd.band_off;
  int* pv = piv + sd.piv_off;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  cx<W>* Pn = reinterpret_cast<cx<W>*>(smem_raw);  // RM x LU_NB, row-major
  cx<W>* Ch = Pn + RM * LU_NB;                      // RM x LU_NB, row-major
  cx<W>* Li = Ch + RM * LU_NB;                      // LU_NB x LU_NB, row-major
  W* redv = reinterpret_cast<W*>(Li + LU_NB * LU_NB);
  int* redi = reinterpret_cast<int*>(redv + 4);
  int* pl = redi + 4;  // the panel's pivot rows, relative to j0
  const cx<W> zero = mk(0.0, 0.0);
  auto at = [&](int i, int j) { return (long long)j * ldab + kv + i - j; };
  if (tid == 0) pflag[blockIdx.x] = 1;  // every strip takes the lane-major substitution
  for (int j0 = 0; j0 < ns; j0 += LU_NB) {
    const int nb = min(LU_NB, ns - j0);
    const int R = min(nb + kl, ns - j0);
    // ---- 1. the panel (consecutive threads read consecutive rows of a column)
    for (int e = tid; e < RM * LU_NB; e += 256) {
      const int c = e / RM, r = e - c * RM, i = j0 + r, j = j0 + c;
      const bool in = r < R && c < nb && i - j <= kl && j - i <= kv;
      Pn[r * LU_NB + c] = in ? ccast<W>(ab[at(i, j)]) : zero;
    }
    __syncthreads();
    for (int jj = 0; jj < nb; ++jj) {
      const int j = j0 + jj, km = min(kl, ns - 1 - j);
      W v = -1.0;
      int idx = 1 << 20;
      if (tid <= km) {
        v = cabs1(Pn[(jj + tid) * LU_NB + jj]);
        idx = tid;
      }
      wave_argmax(v, idx);
      if (lane == 0) {
        redv[wv] = v;
        redi[wv] = idx;
      }
      __syncthreads();
      // largest |Re| + |Im|, first index on ties (wave 0 always holds row jj)
      W bv = redv[0];
      int p = redi[0];
      for (int w = 1; w < 4; ++w)
        if (redv[w] > bv || (redv[w] == bv && redi[w] < p)) {
          bv = redv[w];
          p = redi[w];
        }
      const cx<W> pvv = Pn[(jj + p) * LU_NB + jj];
      const W pd = pvv.re * pvv.re + pvv.im * pvv.im;
      // the stored pivot must be usable in the strip precision too
      const cx<T> pvs = ccast<T>(pvv);
      const T pds = pvs.re * pvs.re + pvs.im * pvs.im;
      if (tid == 0) {
        pv[j] = j + p;
        pl[jj] = jj + p;
        if (bad_pivot(pd) || bad_pivot(pds)) atomicCAS(err, 0, (int)blockIdx.x + 1);
      }
      if (p != 0 && tid < nb) {  // whole rows: L11 and L21 in the final row order
        const cx<W> t0 = Pn[jj * LU_NB + tid];
        Pn[jj * LU_NB + tid] = Pn[(jj + p) * LU_NB + tid];
        Pn[(jj + p) * LU_NB + tid] = t0;
      }
      __syncthreads();
      const W ipd = bad_pivot(pd) ? 0.0 : 1.0 / pd;
      const cx<W> ipv = mk(pvv.re * ipd, -pvv.im * ipd);
      if (tid >= 1 && tid <= km) {
        const int r = jj + tid;
        const cx<W> m = Pn[r * LU_NB + jj] * ipv;
        Pn[r * LU_NB + jj] = m;
        for (int c = jj + 1; c < nb; ++c)
          Pn[r * LU_NB + c] = cfms(Pn[r * LU_NB + c], m, Pn[jj * LU_NB + c]);
      }
      __syncthreads();
    }
    const int j1 = j0 + nb, jmax = min(j0 + nb - 1 + kv, ns - 1);
    // ---- 2. L11^{-1}, column tid (a full panel: nb == LU_NB wherever j1 <= jmax)
    if (j1 <= jmax && tid < LU_NB) {
      cx<W> xc[LU_NB];
#pragma unroll
      for (int r = 0; r < LU_NB; ++r) xc[r] = r == tid ? mk(1.0, 0.0) : zero;
#pragma unroll
      for (int c = 0; c < LU_NB; ++c)
#pragma unroll
        for (int r = c + 1; r < LU_NB; ++r) xc[r] = cfms(xc[r], Pn[r * LU_NB + c], xc[c]);
#pragma unroll
      for (int r = 0; r < LU_NB; ++r) Li[r * LU_NB + tid] = xc[r];
    }
    __syncthreads();
    // ---- 3. trailing columns, LU_NB at a time
    const int ntile = (R - nb + 15) / 16;
    for (int c0 = j1; c0 <= jmax; c0 += LU_NB) {
      const int cw = min(LU_NB, jmax - c0 + 1);
      for (int e = tid; e < RM * LU_NB; e += 256) {
        const int c = e / RM, r = e - c * RM, i = j0 + r, j = c0 + c;
        const bool in = r < R && c < cw && i - j <= kl && j - i <= kv;
        Ch[r * LU_NB + c] = in ? ccast<W>(ab[at(i, j)]) : zero;
      }
      __syncthreads();
      if (tid < cw) {
        for (int jj = 0; jj < nb; ++jj) {
          const int p = pl[jj];
          if (p != jj) {
            const cx<W> t0 = Ch[jj * LU_NB + tid];
            Ch[jj * LU_NB + tid] = Ch[p * LU_NB + tid];
            Ch[p * LU_NB + tid] = t0;
          }
        }
      }
      __syncthreads();
      if (wv == 0) {  // U12 = L11^{-1} A12 (the wave reads all of A12 before it writes)
        V4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
        ctile_mma<W>(cre, cim, Li, LU_NB, Ch, LU_NB, lane, 1.0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          Ch[MfmaT<W>::row(lane, i) * LU_NB + (lane & 15)] = mk(cre[i], cim[i]);
      }
      __syncthreads();
      for (int t = wv; t < ntile; t += 4) {  // A22 -= L21 U12, one 16-row tile per wave
        const int r0 = nb + 16 * t;
        V4 cre, cim;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const cx<W> c = Ch[(r0 + MfmaT<W>::row(lane, i)) * LU_NB + (lane & 15)];
          cre[i] = c.re;
          cim[i] = c.im;
        }
        ctile_mma<W>(cre, cim, Pn + r0 * LU_NB, LU_NB, Ch, LU_NB, lane, -1.0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          Ch[(r0 + MfmaT<W>::row(lane, i)) * LU_NB + (lane & 15)] = mk(cre[i], cim[i]);
      }
      __syncthreads();
      for (int e = tid; e < RM * LU_NB; e += 256) {
        const int c = e / RM, r = e - c * RM, i = j0 + r, j = c0 + c;
        if (r < R && c < cw && i - j <= kl && j - i <= kv) ab[at(i, j)] = ccast<T>(Ch[r * LU_NB + c]);
      }
      __syncthreads();
    }
    // ---- 4. the panel back to the band, each column's multipliers in the
    // row order of its own step (later interchanges undone on the L part)
    for (int jj = nb - 1; jj >= 1; --jj) {
      const int p = pl[jj];
      if (p != jj && tid < jj) {
        const cx<W> t0 = Pn[jj * LU_NB + tid];
        Pn[jj * LU_NB + tid] = Pn[p * LU_NB + tid];
        Pn[p * LU_NB + tid] = t0;
      }
      __syncthreads();
    }
    for (int e = tid; e < RM * LU_NB; e += 256) {
      const int c = e / RM, r = e - c * RM, i = j0 + r, j = j0 + c;
      if (r < R && c < nb && i - j <= kl && j - i <= kv) ab[at(i, j)] = ccast<T>(Pn[r * LU_NB + c]);
    }
    __syncthreads();
  }
}

// Solve image of every strip (layout above).  grid = (NP*64 / 256, strips).
template <class T>
__global__ void k_build_image(const StripDesc* __restrict__ strips, const cx<T>* __restrict__ band,
                              cx<T>* __restrict__ img, int* __restrict__ pivbuf,
                              const int* __restrict__ pflag) {
  if (!pflag[blockIdx.y]) return;  // unpivoted strips use the blocked image
  const StripDesc sd = strips[blockIdx.y];
  const int ns = sd.ns, NP = ns + HH_PAD, kl = sd.kl, kv = 2 * kl, S = sd.S, SL = sd.SL;
  const int ldab = sd.ldab;
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= (long long)NP * 64) return;
  const int j = (int)(e >> 6), l = (int)(e & 63);
  const cx<T> zero = mk((T)0, (T)0);
  const cx<T>* ab = band + sd.band_off;
  cx<T>* Lm = img + sd.img_off;
  cx<T>* Um = Lm + (long long)NP * 64 * SL;
  cx<T>* rdg = Um + (long long)NP * 64 * S;
  int c;
  for (int k = 0; k < SL; ++k) {
    c = 64 * k + ((l - (j & 63)) & 63);
    const bool inl = j < ns && c >= 1 && c <= kl && j + c < ns;
    Lm[((long long)j * SL + k) * 64 + l] = csel(inl, ab[inl ? (long long)j * ldab + kv + c : 0], zero);
  }
  const int col = ns - 1 - j;  // step J = j of the back substitution
  cx<T> rd = zero;
  if (j < ns) {
    const cx<T> d = ab[(long long)col * ldab + kv];
    rd = csel(d.re == (T)0 && d.im == (T)0, zero, cinv(d));
  }
  for (int k = 0; k < S; ++k) {
    c = 64 * k + ((l - (j & 63)) & 63);
    cx<T> v = zero;
    if (j < ns && c >= 1 && c <= kv && j + c < ns) v = ab[(long long)col * ldab + kv - c] * rd;
    Um[((long long)j * S + k) * 64 + l] = v;
  }
  if (l == 0) {
    rdg[j] = rd;
    if (j >= ns) pivbuf[sd.piv_off + j] = j;
  }
}

// Blocked image of an unpivoted strip.  Without interchanges L is unit lower
// and U upper triangular, both with half-bandwidth K = kl, and each
// substitution is the row recurrence
//     out_i = d_i (in_i - sum_{c=1..K} T(i, c) out_{i-c})
// (L: T(i, c) = L(i, i-c), d = 1; U in reversed order E = ns-1-j:
// T(E, c) = U(j, j+c), d = 1/U(j, j)).  For a block of HH_BLK outputs
// i0..i0+B-1 the outputs are a fixed linear map G of the K previous outputs
// and the B block inputs: out = G [out_{i0-K..i0-1}; in_{i0..i0+B-1}].
// Column k of G is obtained by running the block's recurrence on the k-th
// unit input, in FP64 from the stored factors.  Stored per block as KP rows
// of 64 lanes; lane l = r + 16 p holds coefficients of output r, and the four
// lanes of a row split the columns so that each holds four of the previous
// block's outputs (row t = 0..3: out_{i0-16+4p+t}), four block inputs
// (t = 4..7: in_{i0+4p+t-4}) and KO = KP - 8 of the older outputs
// (t = 8..: out_{i0-K+p KO+t-8}, zero where that lies at or past i0-16).
// One wave per (block, strip, triangle): the block's coefficients T(i, c) go
// to LDS, lane l runs the recurrences of columns l and l + 64; a unit
// "previous output" enters each row once, the rest is the block's own
// recurrence (at most 15 terms per row).
template <class T>
__global__ __launch_bounds__(64) void k_build_blocked(const StripDesc* __restrict__ strips,
                                                      const cx<T>* __restrict__ band,
                                                      cx<T>* __restrict__ img,
                                                      const int* __restrict__ pflag) {
  constexpr int B = HH_BLK;
  static_assert(HH_BLK == 16, "the column split assumes four lane groups of 16 rows");
  __shared__ c128 cf[B][64];  // cf[r][c - 1] = T(i0 + r, c), zero where undefined
  __shared__ c128 dv[B];      // row scale d (1 for L, 1/U(j, j) for U, 0 past the end)
  if (pflag[blockIdx.y]) return;
  const StripDesc sd = strips[blockIdx.y];
  const int ns = sd.ns, K = sd.kl, kv = 2 * sd.kl, ldab = sd.ldab, KP = sd.KP;
  const int nb = (ns + B - 1) / B, b = blockIdx.x;
  if (b >= nb) return;
  const int lane = threadIdx.x;
  const bool upper = blockIdx.z == 1;
  const cx<T>* ab = band + sd.band_off;
  cx<T>* G = img + sd.img_off + (upper ? blocked_blocks(ns) * KP * 64 : 0);
  const int i0 = b * B;
  for (int r = 0; r < B; ++r) {
    const int g = i0 + r, c = lane + 1;
    c128 v = mk(0.0, 0.0);
    if (c <= K && g < ns && g - c >= 0) {
      const cx<T> x = upper ? ab[(long long)(ns - 1 - g + c) * ldab + kv - c]
                            : ab[(long long)(g - c) * ldab + kv + c];
      v = mk((double)x.re, (double)x.im);
    }
    cf[r][lane] = v;
  }
  if (lane < B) {
    const int g = i0 + lane;
    c128 d = mk(g < ns ? 1.0 : 0.0, 0.0);
    if (upper && g < ns) {
      const cx<T> x = ab[(long long)(ns - 1 - g) * ldab + kv];
      d = cinv(mk((double)x.re, (double)x.im));
    }
    dv[lane] = d;
  }
  __syncthreads();
  const int KO = KP - 8;
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int k = lane + 64 * sl;
    if (k >= K + B) break;
    c128 out[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
      c128 acc = mk((k >= K && k - K == r) ? 1.0 : 0.0, 0.0);
      if (k < K) {  // the unit previous output sits c = K + r - k rows back
        const int c = K + r - k;
        if (c <= K) acc = acc - cf[r][c - 1];
      }
#pragma unroll
      for (int c = 1; c <= r; ++c)
        if (c <= K) acc = cfms(acc, cf[r][c - 1], out[r - c]);
      out[r] = acc * dv[r];
    }
    // lane group p and row t of column k (see above)
    int p, t;
    if (k >= K) {  // block input k - K
      p = (k - K) / 4;
      t = 4 + (k - K) % 4;
    } else if (k >= K - B) {  // output of the previous block, i0 - K + k = i0 - 16 + j
      const int j = k - (K - B);
      p = j / 4;
      t = j % 4;
    } else {  // older output
      p = k / KO;
      t = 8 + k % KO;
    }
#pragma unroll
    for (int r = 0; r < B; ++r)
      G[((long long)b * KP + t) * 64 + r + B * p] = mk((T)out[r].re, (T)out[r].im);
  }
}

// Rows of k_build_transfer's output window: a power of two above the band.
__host__ __device__ inline int transfer_ring(int kl) { return kl < 32 ? 32 : 64; }

// Segments that k_build_transfer runs for plan p: those with a tail map
// (1..nseg-2), and for plans 1 and 2 also the last one (its response only).
__host__ __device__ inline int transfer_jobs(const StripDesc& sd, int p) {
  const int nseg = plan_nseg(sd.ns, sd.pseg[p]);
  if (p >= 1 && !sd.wide) return 0;
  return nseg > 1 ? nseg - 1 : 0;  // segments 1 .. nseg-1: responses, maps for all but the last
}

// Both halves of the wave get v(l mod 32) + v(l mod 32 + 32), summed in that
// order.
__device__ __forceinline__ c128 halves_sum(c128 v) {
  const unsigned long long r = __double_as_longlong(v.re), m = __double_as_longlong(v.im);
  const auto rl = __builtin_amdgcn_permlane32_swap((unsigned)r, (unsigned)r, false, false);
  const auto rh = __builtin_amdgcn_permlane32_swap((unsigned)(r >> 32), (unsigned)(r >> 32), false,
                                                   false);
  const auto ml = __builtin_amdgcn_permlane32_swap((unsigned)m, (unsigned)m, false, false);
  const auto mh = __builtin_amdgcn_permlane32_swap((unsigned)(m >> 32), (unsigned)(m >> 32), false,
                                                   false);
  auto d = [](unsigned lo, unsigned hi) {
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
  };
  return mk(d(rl[0], rh[0]) + d(rl[1], rh[1]), d(ml[0], mh[0]) + d(ml[1], mh[1]));
}

// Segment transfer maps of an unpivoted strip.  The substitutions split a
// strip's rows into segments (one cut per segment plan) that are solved in
// parallel from a zero state; the true state of segment s+1 (the K outputs
// before it) is then the zero-state tail of segment s plus T_s times the state
// of segment s, where column c' of T_s is the tail of the recurrence over
// segment s started from the unit state e_c' with zero inputs.  A triangle's
// maps are numbered plan by plan (segments 1..nseg-2 of plan p from
// sd.pmap[p] on) and stored column-major zero-padded to KM = map_dim(KP)
// (map m at (m KM + c') KM + c = tail row c), the U maps sd.tmaps maps after
// the L maps.  One wave per (map,
// strip, triangle; the map is the slowest grid dimension, so that the long
// segments of plan 0 are dispatched first), lane c' runs column c' in FP64
// from the stored factors
// (same conventions as the blocked maps) with its window of the last 64
// outputs in LDS; the coefficients of the next row are fetched while a row is
// computed.
template <class T>
__global__ __launch_bounds__(64) void k_build_transfer(const StripDesc* __restrict__ strips,
                                                       const cx<T>* __restrict__ band,
                                                       cx<T>* __restrict__ img,
                                                       const int* __restrict__ pflag,
                                                       int wstride, int planmask) {
  // win[(i mod RS) W + c'] = out_i of column c' < K, W = max_kl + 1, then
  // the coefficients of CR rows, row u at cb[u W ..] (entry K: the scale d)
  // (dynamic LDS, (RS + CR) W entries)
  extern __shared__ c128 win[];
  const int W = wstride;
  if (pflag[blockIdx.x]) return;
  const StripDesc sd = strips[blockIdx.x];
  const int ns = sd.ns, K = sd.kl, kv = 2 * sd.kl, ldab = sd.ldab;
  int m = blockIdx.z, plan = 0;
  for (; plan < HH_NPLAN; ++plan) {
    const int c = transfer_jobs(sd, plan);
    if (m < c) break;
    m -= c;
  }
  if (plan == HH_NPLAN || !(planmask >> plan & 1)) return;
  // (plan is not known at compile time: these come from global memory rather
  // than from a private copy indexed at run time)
  const int seg = strips[blockIdx.x].pseg[plan], pmap = strips[blockIdx.x].pmap[plan];
  const int s = 1 + m, nseg = plan_nseg(ns, seg);
  const int lane = threadIdx.x;
  const bool upper = blockIdx.y == 1;
  const cx<T>* ab = band + sd.band_off;
  // the tail map T_s exists for s <= nseg-2; every row of the segment (its
  // response Phi_s) is kept too, the last segment included
  const bool tmap = s <= nseg - 2;
  const int KM = map_dim(sd.KP);
  cx<T>* Tm = img + sd.t_off +
              ((upper ? (long long)sd.tmaps : 0LL) + pmap + m) * KM * KM;
  cx<T>* Ph = img + strips[blockIdx.x].phi_off[plan] +
              (upper ? plan_phi_elems(ns, sd.segs, K, KM, plan) : 0LL) +
              (long long)(s - 1) * seg * KM;
  const int s0 = s * seg, s1 = s0 + seg < ns ? s0 + seg : ns;
  // lane c < K fetches T(i, c + 1)
  auto coef = [&](int i) -> c128 {
    const int j = ns - 1 - i, c = lane + 1;
    if (lane < K) {
      const cx<T> x = upper ? ab[(long long)(j + c) * ldab + kv - c]
                            : ab[(long long)(i - c) * ldab + kv + c];
      return mk((double)x.re, (double)x.im);
    }
    return mk(0.0, 0.0);
  };
  // the diagonal U(j, j) of row i, j = ns - 1 - i (U only)
  auto diag = [&](int i) -> c128 {
    const cx<T> x = ab[(long long)(ns - 1 - i) * ldab + kv];
    return mk((double)x.re, (double)x.im);
  };
  // Each lane's recurrence touches only its own column of the window, so
  // the rows run without barriers; the coefficients come CR rows at a time
  // through cb, loaded one chunk ahead: lane c < K the row's T(i, c + 1),
  // lane u < CR the scale of row i0 + u (the reciprocal of the diagonal for
  // U, all CR of them at once; 1 for L).
  constexpr int CR = 16;
  const int RS = transfer_ring(W - 1), rm = RS - 1;
  c128* cb = win + RS * W;
  c128 cr[CR], dg;
  auto fetch = [&](int i0) {
#pragma unroll
    for (int u = 0; u < CR; ++u) cr[u] = i0 + u < s1 ? coef(i0 + u) : mk(0.0, 0.0);
    dg = upper && lane < CR && i0 + lane < s1 ? diag(i0 + lane) : mk(1.0, 0.0);
  };
  // The response rows of a chunk go out from the window once the chunk is
  // done, sixteen lanes per column so that each column's rows are written as
  // one contiguous run (rows f0 .. f0 + fn - 1; the ring keeps a chunk's rows
  // until the chunk after next).
  auto flush = [&](int f0, int fn) {
    for (int e = lane; e < K * CR; e += 64) {
      const int c = e / CR, u = e % CR;
      if (u < fn) {
        const c128 v = win[((f0 + u) & rm) * W + c];
        Ph[(long long)c * seg + (f0 + u - s0)] = mk((T)v.re, (T)v.im);
      }
    }
  };
  for (int q = 0; q < RS; ++q)
    if (lane < W) win[q * W + lane] = mk(0.0, 0.0);
  if (lane < K) win[((s0 - K + lane) & rm) * W + lane] = mk(1.0, 0.0);
  fetch(s0);
  // The workgroup is one wave (64 threads), so ordering its LDS accesses
  // needs no barrier: wave_lds_sync keeps the coefficient loads of the next
  // chunk and the stores in flight while the rows run.
  for (int i0 = s0; i0 < s1; i0 += CR) {
    wave_lds_sync();  // the previous chunk's coefficients and rows are done
    if (lane < K) {
#pragma unroll
      for (int u = 0; u < CR; ++u) cb[u * W + lane] = cr[u];
    }
    if (lane < CR) cb[lane * W + K] = upper ? cinv(dg) : dg;
    // after the coefficient registers are consumed, so that waiting for
    // them does not wait for these stores as well
    if (Ph && i0 > s0) flush(i0 - CR, CR);
    fetch(i0 + CR);
    wave_lds_sync();
    const int un = s1 - i0 < CR ? s1 - i0 : CR;
    if (K <= 32) {
      // two lanes per column: lane c + 32 h sums the terms of its half (h = 0:
      // rows 1 .. H back, h = 1: H + 1 .. K back), one swap of the halves
      // gives both lanes the same total, and both write it to the window, so
      // that each lane reads back only rows it wrote itself
      const int col = lane & 31, h = lane >> 5, H = (K + 1) >> 1;
      const int cb0 = h ? H + 1 : 1, ce = h ? K : H;
      if (col < K) {
        for (int u = 0; u < un; ++u) {
          const int i = i0 + u;
          const c128* cf = cb + u * W;
          c128 a[4] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
          int c = cb0;
          for (; c + 3 <= ce; c += 4) {
            c128 wv[4], fv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              wv[q] = win[((i - c - q) & rm) * W + col];
              fv[q] = cf[c - 1 + q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = cfms(a[q], fv[q], wv[q]);
          }
          for (; c <= ce; ++c) a[0] = cfms(a[0], cf[c - 1], win[((i - c) & rm) * W + col]);
          const c128 acc = halves_sum((a[0] + a[1]) + (a[2] + a[3])) * cf[K];
          win[(i & rm) * W + col] = acc;
          if (h == 0 && tmap && i >= s1 - K)
            Tm[(long long)col * KM + (i - (s1 - K))] = mk((T)acc.re, (T)acc.im);
        }
      }
      continue;
    }
    // lanes past K have no column: they stay out of the rows, which keeps the
    // LDS reads to the K live lanes
    if (lane < K) {
      for (int u = 0; u < un; ++u) {
        const int i = i0 + u;
        const c128* cf = cb + u * W;
        // eight terms at a time, their LDS reads issued together, into four
        // partial sums
        c128 a[4] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
        int c = 1;
        for (; c + 7 <= K; c += 8) {
          c128 wv[8], fv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            wv[q] = win[((i - c - q) & rm) * W + lane];
            fv[q] = cf[c - 1 + q];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) a[q & 3] = cfms(a[q & 3], fv[q], wv[q]);
        }
        for (; c <= K; ++c) a[0] = cfms(a[0], cf[c - 1], win[((i - c) & rm) * W + lane]);
        const c128 acc = ((a[0] + a[1]) + (a[2] + a[3])) * cf[K];
        win[(i & rm) * W + lane] = acc;
        if (tmap && i >= s1 - K)
          Tm[(long long)lane * KM + (i - (s1 - K))] = mk((T)acc.re, (T)acc.im);
      }
    }
  }
  if (Ph) {
    wave_lds_sync();
    const int fl = s0 + (s1 - s0 - 1) / CR * CR;  // the last chunk
    flush(fl, s1 - fl);
  }
}

// Products of segment maps for plan p >= 1 (slots in plan_layout), formed
// in FP64 from the stored maps.  Stage 0, for workgroup g (segments c = g P
// + w): the running product T_{gP+q-1} ... T_{gP}, stored as Pi_{gP+q} for
// q < P and as W_g for q = P (the chain of workgroup g), and A1_c = T_c
// T_{c-1} (w >= 2).  Stage 1: A2_c = A1_c A1_{c-2} (w >= 4) and, for
// workgroup g, the running product W_{g-1} ... W_{j+1} = Psi_{j,g} for j =
// g-2 down to 0 (its chain).  One workgroup of 256 threads per (strip,
// triangle, job); jobs 0 .. G-1 of a stage are the chains, so that with the
// job as the slowest grid index every chain is dispatched before the single
// products.  The maps involved are copied into LDS (three KM x KM buffers in
// FP64, column-major like the stored maps) and the 256 threads share the
// entries of a product.
template <class T>
__global__ __launch_bounds__(256) void k_build_products(const StripDesc* __restrict__ strips,
                                                        cx<T>* __restrict__ img,
                                                        const int* __restrict__ pflag, int stage,
                                                        int plan) {
  extern __shared__ c128 sh[];  // 3 KM^2
  if (pflag[blockIdx.x]) return;
  const StripDesc sd = strips[blockIdx.x];
  if (!sd.wide) return;
  const int G = plan_width(plan);
  const int pi_map = sd.pi_map[plan], a1_map = sd.a1_map[plan], a2_map = sd.a2_map[plan];
  const int ps_map = sd.ps_map[plan];
  const int ns = sd.ns, K = sd.kl, P = sd.segs, KM = map_dim(sd.KP), K2 = KM * KM;
  const int nseg = plan_nseg(ns, sd.pseg[plan]), gu = (nseg + P - 1) / P;
  const int t0 = sd.pmap[plan] - 1;  // slot of T_c is t0 + c
  const int m = blockIdx.z, tid = threadIdx.x;
  const long long tri = blockIdx.y == 1 ? (long long)sd.tmaps : 0LL;
  const cx<T>* maps = img + sd.t_off + tri * K2;
  cx<T>* outm = img + sd.t_off + tri * K2;
  c128* X = sh;
  c128* Y = sh + K2;
  c128* Z = sh + 2 * K2;
  auto load = [&](c128* d, int slot) {
    const cx<T>* src = maps + (long long)slot * K2;
    for (int e0 = 0; e0 < K2; e0 += 4 * 256) {
      cx<T> v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + q * 256 + tid;
        v[q] = src[e < K2 ? e : K2 - 1];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + q * 256 + tid;
        if (e < K2) d[e] = mk((double)v[q].re, (double)v[q].im);
      }
    }
    __syncthreads();
  };
  auto store = [&](int slot, const c128* src) {  // the K x K block; the padding stays zero
    cx<T>* d = outm + (long long)slot * K2;
    for (int e = tid; e < K2; e += 256)
      if (e % KM < K && e / KM < K) d[e] = mk((T)src[e].re, (T)src[e].im);
  };
  // d = A B over the K x K blocks (d distinct from A, B): thread e % 256
  // forms entry (e mod K, e / K)
  auto mul = [&](c128* d, const c128* A, const c128* B) {
    for (int e = tid; e < K * K; e += 256) {
      const int c = e / K, r = e - c * K;
      c128 acc = mk(0.0, 0.0);
      for (int cc = 0; cc < K; ++cc) acc = cfma(acc, A[cc * KM + r], B[c * KM + cc]);
      d[c * KM + r] = acc;
    }
    __syncthreads();
  };
  if (stage == 0) {
    // job m < G: the chain of workgroup m (k = 0); else A1 job k = 1 + (m - G) mod P
    const int g = m < G ? m : (m - G) / P, k = m < G ? 0 : 1 + (m - G) % P;
    if (g >= gu) return;
    if (k == 0) {
      if (g == 0 || g * P > nseg - 2) return;
      c128* cur = X;
      c128* nxt = Y;
      load(cur, t0 + g * P);
      for (int q = 1;; ++q) {  // cur = T_{gP+q-1} ... T_{gP}
        if (q < P) {
          if (g * P + q > nseg - 1) break;
          store(pi_map + g * P + q - 1, cur);
        } else {
          if (g <= gu - 2) store(sd.pwmap[plan] + g - 1, cur);
          break;
        }
        const int c = g * P + q;
        if (c > nseg - 2) break;
        load(Z, t0 + c);
        mul(nxt, Z, cur);
        c128* tmp = cur;
        cur = nxt;
        nxt = tmp;
      }
    } else {
      const int w = k - 1, c = g * P + w;
      if (w < 2 || c > nseg - 2) return;
      load(X, t0 + c);
      load(Y, t0 + c - 1);
      mul(Z, X, Y);
      store(a1_map + c - 1, Z);
    }
  } else if (m >= G) {
    const int g = (m - G) / P, w = (m - G) % P, c = g * P + w;
    if (g >= gu || w < 4 || c > nseg - 2) return;
    load(X, a1_map + c - 1);
    load(Y, a1_map + c - 3);
    mul(Z, X, Y);
    store(a2_map + c - 1, Z);
  } else {
    const int g = m;
    if (G < 3 || g < 2 || g > gu - 1) return;
    c128* cur = X;
    c128* nxt = Y;
    load(cur, sd.pwmap[plan] + g - 2);  // W_{g-1}
    store(ps_map + g * G + g - 2, cur);
    for (int j = g - 3; j >= 0; --j) {
      load(Z, sd.pwmap[plan] + j);  // W_{j+1}
      mul(nxt, cur, Z);
      c128* tmp = cur;
      cur = nxt;
      nxt = tmp;
      store(ps_map + g * G + j, cur);
    }
  }
}

}  // namespace

dim3 blocked_grid(const FactorSet& fs) {
  int blocks = 1;
  for (auto& sd : fs.strips) blocks = std::max(blocks, (sd.ns + HH_BLK - 1) / HH_BLK);
  return dim3((unsigned)blocks, (unsigned)fs.strips.size(), 2);
}

static dim3 transfer_grid(const FactorSet& fs) {
  int maps = 1;
  for (auto& sd : fs.strips) {
    int m = 0;
    for (int p = 0; p < HH_NPLAN; ++p) m += transfer_jobs(sd, p);
    maps = std::max(maps, m);
  }
  return dim3((unsigned)fs.strips.size(), 2, (unsigned)maps);
}

static dim3 product_grid(const FactorSet& fs, int stage, int plan) {
  int jobs = 0;
  for (auto& sd : fs.strips) {
    const int G = plan_width(plan);
    jobs = std::max(jobs, stage == 0 ? G * (sd.segs + 1) : G * sd.segs + G);
  }
  return dim3((unsigned)fs.strips.size(), 2, (unsigned)jobs);
}

template <class T>
static void launch_products_t(const FactorSet& fs, int planmask, hipStream_t st) {
  if (!fs.strips[0].wide) return;
  const int KM = map_dim(fs.strips[0].KP);
  const size_t lds = 3 * (size_t)KM * KM * sizeof(c128);
  const void* fn = (const void*)k_build_products<T>;
  if (lds > 64 * 1024)
    HH_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  for (int plan = 1; plan < HH_NPLAN; ++plan) {
    if (!(planmask >> plan & 1)) continue;
    for (int stage = 0; stage < 2; ++stage)
      hipLaunchKernelGGL(k_build_products<T>, product_grid(fs, stage, plan), dim3(256), lds, st,
                         fs.d_strips, (cx<T>*)fs.img, fs.d_pflag, stage, plan);
  }
}

void launch_products(const FactorSet& fs, int planmask, hipStream_t st) {
  if (fs.precision == HH_FP64)
    launch_products_t<double>(fs, planmask, st);
  else
    launch_products_t<float>(fs, planmask, st);
  HH_HIP(hipGetLastError());
}

// kl < 32: the two-lanes-per-column kernel on every strip; the strips it
// marks are packed again and factored with interchanges by the one-wave
// register kernel (kl < KR); the launches find nothing to do when no strip
// was marked.  Larger bands: the LDS window on four waves (one or two column
// slots per lane: 2 kl + 1 <= 64 needs one).
template <class T, int R>
static void launch_lu_h(const FactorSet& fs, hipStream_t st) {
  constexpr int CH = sizeof(T) == 8 ? 8 : 16;
  hipLaunchKernelGGL((k_band_lu_h<T, R, CH>), dim3((unsigned)fs.strips.size()), dim3(64), 0, st,
                     fs.d_strips, (cx<T>*)fs.band, fs.piv, fs.d_err, fs.d_pflag);
}
template <class T, int KR>
static void launch_lu_w(const FactorSet& fs, hipStream_t st, int redo) {
  constexpr int CH = sizeof(T) == 8 ? 8 : 16;
  hipLaunchKernelGGL((k_band_lu_w<T, KR, CH>), dim3((unsigned)fs.strips.size()), dim3(64), 0, st,
                     fs.d_strips, (cx<T>*)fs.band, fs.piv, fs.d_err, fs.d_pflag, redo);
}
template <class T>
static void launch_lu_h_any(const FactorSet& fs, hipStream_t st) {
  switch ((fs.max_kl + 2) / 2) {  // smallest R with 2 R > kl
    case 1: return launch_lu_h<T, 1>(fs, st);
    case 2: return launch_lu_h<T, 2>(fs, st);
    case 3: return launch_lu_h<T, 3>(fs, st);
    case 4: return launch_lu_h<T, 4>(fs, st);
    case 5: return launch_lu_h<T, 5>(fs, st);
    case 6: return launch_lu_h<T, 6>(fs, st);
    case 7: return launch_lu_h<T, 7>(fs, st);
    case 8: return launch_lu_h<T, 8>(fs, st);
    case 9: return launch_lu_h<T, 9>(fs, st);
    case 10: return launch_lu_h<T, 10>(fs, st);
    case 11: return launch_lu_h<T, 11>(fs, st);
    case 12: return launch_lu_h<T, 12>(fs, st);
    case 13: return launch_lu_h<T, 13>(fs, st);
    case 14: return launch_lu_h<T, 14>(fs, st);
    case 15: return launch_lu_h<T, 15>(fs, st);
    default: return launch_lu_h<T, 16>(fs, st);
  }
}
template <class T>
static void launch_lu_w_any(const FactorSet& fs, hipStream_t st, int redo) {
  const int kl = fs.max_kl;
  if (kl < 8) return launch_lu_w<T, 8>(fs, st, redo);
  if (kl < 12) return launch_lu_w<T, 12>(fs, st, redo);
  if (kl < 16) return launch_lu_w<T, 16>(fs, st, redo);
  if (kl < 20) return launch_lu_w<T, 20>(fs, st, redo);
  if (kl < 24) return launch_lu_w<T, 24>(fs, st, redo);
  if (kl < 28) return launch_lu_w<T, 28>(fs, st, redo);
  return launch_lu_w<T, 32>(fs, st, redo);
}

template <class T>
static void launch_lu(const hh_problem* pb, size_t lds, hipStream_t st) {
  const FactorSet& fs = pb->fs;
  const int nstr = (int)fs.strips.size();
  if (fs.max_kl > HH_KL_WINDOW) {
    const size_t bl = lu_blk_lds(fs.max_kl);
    HH_HIP(hipFuncSetAttribute((const void*)k_band_lu_blk<T>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bl));
    hipLaunchKernelGGL(k_band_lu_blk<T>, dim3(nstr), dim3(256), bl, st, fs.d_strips,
                       (cx<T>*)fs.band, fs.piv, fs.d_err, fs.d_pflag);
    return;
  }
  if (fs.max_kl < 32) {
    if (lu_interchanging_only()) return launch_lu_w_any<T>(fs, st, 0);
    launch_lu_h_any<T>(fs, st);
    launch_repack_marked(pb, st);
    return launch_lu_w_any<T>(fs, st, 1);
  }
  const bool one = 2 * fs.max_kl + 1 <= 64;
  const void* fn = one ? (const void*)k_band_lu<T, 1> : (const void*)k_band_lu<T, 2>;
  HH_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (one)
    hipLaunchKernelGGL((k_band_lu<T, 1>), dim3(nstr), dim3(LU_THREADS), lds, st, fs.d_strips,
                       (cx<T>*)fs.band, fs.piv, fs.d_err, fs.d_pflag);
  else
    hipLaunchKernelGGL((k_band_lu<T, 2>), dim3(nstr), dim3(LU_THREADS), lds, st, fs.d_strips,
                       (cx<T>*)fs.band, fs.piv, fs.d_err, fs.d_pflag);
}

// Transfer maps of the segment plans in planmask (bit p: plan p).
void launch_transfer(const FactorSet& fs, int planmask, hipStream_t st) {
  const size_t lds = (size_t)(transfer_ring(fs.max_kl) + 16) * (fs.max_kl + 1) * sizeof(c128);
  if (fs.precision == HH_FP64) {
    HH_HIP(hipFuncSetAttribute((const void*)k_build_transfer<double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_build_transfer<double>, transfer_grid(fs), dim3(64), lds, st,
                       fs.d_strips, (const c128*)fs.band, (c128*)fs.img, fs.d_pflag,
                       fs.max_kl + 1, planmask);
  } else {
    HH_HIP(hipFuncSetAttribute((const void*)k_build_transfer<float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_build_transfer<float>, transfer_grid(fs), dim3(64), lds, st,
                       fs.d_strips, (const c64*)fs.band, (c64*)fs.img, fs.d_pflag,
                       fs.max_kl + 1, planmask);
  }
  HH_HIP(hipGetLastError());
}

void launch_band_lu(const hh_problem* pb, hipStream_t st) {
  const FactorSet& fs = pb->fs;
  HH_HIP(hipMemsetAsync(fs.img, 0, fs.img_elems * (fs.precision == HH_FP64 ? sizeof(c128) : sizeof(c64)), st));
  int nstr = (int)fs.strips.size();
  size_t esz = fs.precision == HH_FP64 ? sizeof(c128) : sizeof(c64);
  size_t lds = (size_t)(fs.max_kl + 1 + LU_CH) * (2 * fs.max_kl + 1) * esz;
  double bytes = 0;
  for (size_t u = fs.nsub > 1 ? fs.first_sub : 0; u < fs.strips.size(); ++u)
    bytes += 2.0 * (double)fs.strips[u].nr * fs.strips[u].ldab * esz;
  TimedRegion tr(FAM_FACTOR, st, bytes);
  if (fs.nsub > 1) {
    // recursive strip solves: the sub-blocks, by the blocked LU (any band
    // half-width) and the lane-major image
    const int nsubs = (int)fs.strips.size() - fs.first_sub;
    int ns_sub = 0;
    for (size_t u = fs.first_sub; u < fs.strips.size(); ++u) ns_sub = std::max(ns_sub, fs.strips[u].ns);
    const StripDesc* ds = fs.d_strips + fs.first_sub;
    int* pf = fs.d_pflag + fs.first_sub;
    const size_t bl = lu_blk_lds(fs.max_kl);
    const dim3 gi((unsigned)(((long long)(ns_sub + HH_PAD) * 64 + 255) / 256), (unsigned)nsubs);
    if (fs.precision == HH_FP64) {
      HH_HIP(hipFuncSetAttribute((const void*)k_band_lu_blk<double>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bl));
      hipLaunchKernelGGL(k_band_lu_blk<double>, dim3(nsubs), dim3(256), bl, st, ds, (c128*)fs.band,
                         fs.piv, fs.d_err, pf);
      hipLaunchKernelGGL(k_build_image<double>, gi, dim3(256), 0, st, ds, (const c128*)fs.band,
                         (c128*)fs.img, fs.piv, pf);
    } else {
      HH_HIP(hipFuncSetAttribute((const void*)k_band_lu_blk<float>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bl));
      hipLaunchKernelGGL(k_band_lu_blk<float>, dim3(nsubs), dim3(256), bl, st, ds, (c64*)fs.band,
                         fs.piv, fs.d_err, pf);
      hipLaunchKernelGGL(k_build_image<float>, gi, dim3(256), 0, st, ds, (const c64*)fs.band,
                         (c64*)fs.img, fs.piv, pf);
    }
    HH_HIP(hipGetLastError());
    return;
  }
  if (fs.precision == HH_FP64) {
    launch_lu<double>(pb, lds, st);
    HH_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_build_image<double>, dim3((unsigned)(((long long)(fs.max_ns + HH_PAD) * 64 + 255) / 256), nstr),
                       dim3(256), 0, st, fs.d_strips, (const c128*)fs.band, (c128*)fs.img, fs.piv,
                       fs.d_pflag);
    if (fs.max_kl <= HH_KL_WINDOW) {  // wide bands take the lane-major substitution only
      hipLaunchKernelGGL(k_build_blocked<double>, blocked_grid(fs), dim3(64), 0, st, fs.d_strips,
                         (const c128*)fs.band, (c128*)fs.img, fs.d_pflag);
      launch_transfer(fs, HH_EAGER_PLANS | (fs.batch_maps ? HH_BATCH_PLANS : 0), st);
      launch_products(fs, HH_EAGER_PLANS | (fs.batch_maps ? HH_BATCH_PLANS : 0), st);
    }
  } else {
    launch_lu<float>(pb, lds, st);
    HH_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_build_image<float>, dim3((unsigned)(((long long)(fs.max_ns + HH_PAD) * 64 + 255) / 256), nstr),
                       dim3(256), 0, st, fs.d_strips, (const c64*)fs.band, (c64*)fs.img, fs.piv,
                       fs.d_pflag);
    if (fs.max_kl <= HH_KL_WINDOW) {  // wide bands take the lane-major substitution only
      hipLaunchKernelGGL(k_build_blocked<float>, blocked_grid(fs), dim3(64), 0, st, fs.d_strips,
                         (const c64*)fs.band, (c64*)fs.img, fs.d_pflag);
      launch_transfer(fs, HH_EAGER_PLANS | (fs.batch_maps ? HH_BATCH_PLANS : 0), st);
      launch_products(fs, HH_EAGER_PLANS | (fs.batch_maps ? HH_BATCH_PLANS : 0), st);
    }
  }
  HH_HIP(hipGetLastError());
}

}  // namespace hh
