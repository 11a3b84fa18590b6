// FP64 kernels of the MPGMRES outer loop (Sec. 3): the sparse product with
// the P1 operator, block classical Gram-Schmidt (tall-skinny Gram products
// and rank-t updates), normalisation with deflation, the solution update
// x = Z y and the residual.  Every kernel takes an array of task descriptors
// so that one launch serves a whole batch of independent solves, possibly of
// different sizes.  All reductions are two-stage and deterministic.
#include "hh_internal.h"
#include "krylov.h"

namespace hh {

namespace {

template <class T>
__device__ __forceinline__ c128 ld_c128(const void* base, long long idx) {
  const cx<T> v = ((const cx<T>*)base)[idx];
  return mk((double)v.re, (double)v.im);
}

// y = A x with A complex symmetric, stored as its upper diagonals
// d0 = A[p][p], d1 = A[p][p+1], dn = A[p][p+n], dn1 = A[p][p+n+1].
template <class T>
__global__ __launch_bounds__(256) void k_spmv(const SpmvTask* __restrict__ tasks) {
  const SpmvTask tk = tasks[blockIdx.y];
  const int n = tk.n;
  const long long nn = (long long)n * n;
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  if (p >= nn) return;
  const c128* A = tk.A;
  const c128 a0 = A[p], a1 = A[nn + p], an = A[2 * nn + p], an1 = A[3 * nn + p];
  const c128 zero = mk(0.0, 0.0);
  // (the loads stay inside A for every p; the selects act on values)
  const c128 b1 = csel(p >= 1, A[nn + p - 1], zero);
  const c128 bn = csel(p >= n, A[2 * nn + p - n], zero);
  const c128 bn1 = csel(p >= n + 1, A[3 * nn + p - n - 1], zero);
  for (int v = 0; v < tk.nvec; ++v) {
    const long long o = v * nn;
    c128 acc = a0 * ld_c128<T>(tk.x, o + p);
    if (p + 1 < nn) acc = acc + a1 * ld_c128<T>(tk.x, o + p + 1);
    if (p + n < nn) acc = acc + an * ld_c128<T>(tk.x, o + p + n);
    if (p + n + 1 < nn) acc = acc + an1 * ld_c128<T>(tk.x, o + p + n + 1);
    if (p >= 1) acc = acc + b1 * ld_c128<T>(tk.x, o + p - 1);
    if (p >= n) acc = acc + bn * ld_c128<T>(tk.x, o + p - n);
    if (p >= n + 1) acc = acc + bn1 * ld_c128<T>(tk.x, o + p - n - 1);
    tk.y[o + p] = acc;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Partial sums of X^H Y over one block of rows and one chunk of CH columns of X.
// grid = (row blocks, column chunks, tasks); part[(blk * px + i) * ty + c].
template <int CH, int TY>
__global__ __launch_bounds__(256) void k_gram_partial(const GramTask* __restrict__ tasks) {
  const GramTask tk = tasks[blockIdx.z];
  const int blk = blockIdx.x, i0 = blockIdx.y * CH;
  if (blk >= tk.nblk || i0 >= tk.px) return;
  const long long rows_per = (tk.len + tk.nblk - 1) / tk.nblk;
  const long long r0 = blk * rows_per;
  const long long r1 = min((long long)tk.len, r0 + rows_per);
  double acc_re[CH][TY], acc_im[CH][TY];
#pragma unroll
  for (int a = 0; a < CH; ++a)
#pragma unroll
    for (int c = 0; c < TY; ++c) acc_re[a][c] = acc_im[a][c] = 0.0;
  const int ni = min(CH, tk.px - i0);
  for (long long p = r0 + threadIdx.x; p < r1; p += 256) {
    c128 y[TY];
#pragma unroll
    for (int c = 0; c < TY; ++c) y[c] = c < tk.ty ? tk.Y[c * (long long)tk.ldy + p] : mk(0.0, 0.0);
#pragma unroll
    for (int a = 0; a < CH; ++a) {
      if (a < ni) {
        const c128 x = tk.X[(i0 + a) * (long long)tk.ldx + p];
#pragma unroll
        for (int c = 0; c < TY; ++c) {
          const c128 d = cdotc(x, y[c]);
          acc_re[a][c] += d.re;
          acc_im[a][c] += d.im;
        }
      }
    }
  }
  __shared__ double red[4][CH * TY * 2];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
  for (int a = 0; a < CH; ++a)
#pragma unroll
    for (int c = 0; c < TY; ++c) {
      double sr = wave_sum(acc_re[a][c]);
      double si = wave_sum(acc_im[a][c]);
      if (ln == 0) {
        red[wv][(a * TY + c) * 2] = sr;
        red[wv][(a * TY + c) * 2 + 1] = si;
      }
    }
  __syncthreads();
  for (int e = threadIdx.x; e < ni * tk.ty; e += 256) {
    const int a = e / tk.ty, c = e - a * tk.ty;
    const int k = (a * TY + c) * 2;
    double sr = red[0][k] + red[1][k] + red[2][k] + red[3][k];
    double si = red[0][k + 1] + red[1][k + 1] + red[2][k + 1] + red[3][k + 1];
    tk.part[((long long)blk * tk.px + i0 + a) * tk.ty + c] = mk(sr, si);
  }
}

// out[i + c*ldo] (=|+=) sum over blocks of part: one wave per entry, lane l
// summing blocks l, l + 64, ..., then a fixed-order wave sum.
// grid = (ceil(px*ty/4), tasks)
__global__ __launch_bounds__(256) void k_gram_reduce(const GramTask* __restrict__ tasks) {
  const GramTask tk = tasks[blockIdx.y];
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6), ln = threadIdx.x & 63;
  if (e >= tk.px * tk.ty) return;
  const int i = e / tk.ty, c = e - i * tk.ty;
  double sr = 0.0, si = 0.0;
  for (int b = ln; b < tk.nblk; b += 64) {
    const c128 v = tk.part[((long long)b * tk.px + i) * tk.ty + c];
    sr += v.re;
    si += v.im;
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (ln == 0) {
    c128* o = tk.out + i + (long long)c * tk.ldo;
    *o = tk.accumulate ? *o + mk(sr, si) : mk(sr, si);
  }
}

// Y[:, c] -= X C[:, c]; C (px x ty, column stride ldc) on the device.
template <int TY>
__global__ __launch_bounds__(256) void k_block_update(const UpdTask* __restrict__ tasks) {
  const UpdTask tk = tasks[blockIdx.y];
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  if (p >= tk.len) return;
  c128 y[TY];
#pragma unroll
  for (int c = 0; c < TY; ++c) y[c] = c < tk.ty ? tk.Y[c * (long long)tk.ldy + p] : mk(0.0, 0.0);
  for (int i = 0; i < tk.px; ++i) {
    const c128 x = tk.X[i * (long long)tk.ldx + p];
#pragma unroll
    for (int c = 0; c < TY; ++c)
      if (c < tk.ty) y[c] = cfms(y[c], x, tk.C[i + (long long)c * tk.ldc]);
  }
#pragma unroll
  for (int c = 0; c < TY; ++c)
    if (c < tk.ty) tk.Y[c * (long long)tk.ldy + p] = y[c];
}

// y = x / the norm whose square is nrm2->re (x = y when not given); deflate
// (zero y, flag) when the norm is at most tol times sqrt(ref2->re).
// grid = (row blocks, tasks).
__global__ __launch_bounds__(256) void k_normalize(const NormTask* __restrict__ tasks) {
  const NormTask tk = tasks[blockIdx.y];
  const double nrm = sqrt(fmax(tk.nrm2->re, 0.0));
  const double ref = sqrt(fmax(tk.ref2->re, 0.0));
  const bool defl = !(nrm > tk.tol * ref) || nrm == 0.0;
  const double s = defl ? 0.0 : 1.0 / nrm;
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *tk.rdiag = mk(defl ? 0.0 : nrm, 0.0);
    *tk.flag = defl ? 1 : 0;
  }
  if (p < tk.len) tk.y[p] = cscale(tk.x ? tk.x[p] : tk.y[p], s);
}

// One fused step of the block's QR (QrTask).  Rows as k_gram_partial's: row
// block blk of the task, thread tid taking rows r0 + tid, r0 + tid + 256, ...
// in order; every row of y lies in exactly one block, so the op is applied
// once per row.  Reductions in the orders of k_gram_reduce (one wave per
// entry) and k_gram_partial (wave sums, then the four waves in turn).
__global__ __launch_bounds__(256) void k_qr_step(const QrTask* __restrict__ tasks) {
  constexpr int CX = 4;
  const QrTask tk = tasks[blockIdx.y];
  const int blk = blockIdx.x, tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  if (blk >= tk.nblk) return;
  __shared__ c128 coef[CX];
  __shared__ double red[4][CX * 2];
  // 1. the previous Gram's coefficients
  if (wv < tk.cpx) {
    double sr = 0.0, si = 0.0;
    for (int b = ln; b < tk.cnblk; b += 64) {
      const c128 v = tk.cpart[(long long)b * tk.cpx + wv];
      sr += v.re;
      si += v.im;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (ln == 0) {
      coef[wv] = mk(sr, si);
      if (blk == 0) tk.cout[wv] = mk(sr, si);
    }
  }
  __syncthreads();
  double scale = 1.0;
  if (tk.op == QR_NORMALIZE) {
    const double nrm = sqrt(fmax(coef[0].re, 0.0));
    const double ref = sqrt(fmax(tk.ref2->re, 0.0));
    const bool defl = !(nrm > tk.tol * ref) || nrm == 0.0;
    scale = defl ? 0.0 : 1.0 / nrm;
    if (blk == 0 && tid == 0) {
      *tk.rdiag = mk(defl ? 0.0 : nrm, 0.0);
      *tk.flag = defl ? 1 : 0;
    }
  }
  // 2. the op and the next Gram's partial sums, row by row
  const long long rows_per = (tk.len + tk.nblk - 1) / tk.nblk;
  const long long r0 = blk * rows_per;
  const long long r1 = min(tk.len, r0 + rows_per);
  double acc_re[CX], acc_im[CX];
#pragma unroll
  for (int a = 0; a < CX; ++a) acc_re[a] = acc_im[a] = 0.0;
  for (long long p = r0 + tid; p < r1; p += 256) {
    c128 v = mk(0.0, 0.0);
    if (tk.op == QR_UPDATE) {
      v = tk.y[p];
      for (int i = 0; i < tk.cpx; ++i) v = cfms(v, tk.Xop[i * tk.ld + p], coef[i]);
      tk.y[p] = v;
    } else if (tk.op == QR_NORMALIZE) {
      v = cscale(tk.y[p], scale);
      tk.y[p] = v;
    }
    if (tk.gpx > 0) {
      const c128 y = tk.gy_is_y ? v : tk.gy[p];
#pragma unroll
      for (int a = 0; a < CX; ++a) {
        if (a < tk.gpx) {
          const c128 x = a == tk.xg_is_y ? v : tk.Xg[a * tk.ld + p];
          const c128 d = cdotc(x, y);
          acc_re[a] += d.re;
          acc_im[a] += d.im;
        }
      }
    }
  }
  if (tk.gpx <= 0) return;
#pragma unroll
  for (int a = 0; a < CX; ++a) {
    const double sr = wave_sum(acc_re[a]);
    const double si = wave_sum(acc_im[a]);
    if (ln == 0) {
      red[wv][a * 2] = sr;
      red[wv][a * 2 + 1] = si;
    }
  }
  __syncthreads();
  if (tid < tk.gpx) {
    const int k = tid * 2;
    const double sr = red[0][k] + red[1][k] + red[2][k] + red[3][k];
    const double si = red[0][k + 1] + red[1][k + 1] + red[2][k + 1] + red[3][k + 1];
    tk.gpart[(long long)blk * tk.gpx + tid] = mk(sr, si);
  }
}

// x = Z y (plus x0 if add); Z columns contiguous with stride len.
template <class T>
__global__ __launch_bounds__(256) void k_combine(const CombTask* __restrict__ tasks) {
  const CombTask tk = tasks[blockIdx.y];
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  if (p >= tk.len) return;
  c128 acc = mk(0.0, 0.0);
  for (int j = 0; j < tk.ncols; ++j) acc = acc + ld_c128<T>(tk.Z, j * (long long)tk.len + p) * tk.y[j];
  tk.x[p] = tk.x0 ? tk.x0[p] + acc : acc;
}

// r = b - Ab (elementwise), in place on ab.
__global__ __launch_bounds__(256) void k_residual(const ResTask* __restrict__ tasks) {
  const ResTask tk = tasks[blockIdx.y];
  const long long p = blockIdx.x * 256LL + threadIdx.x;
  if (p >= tk.len) return;
  tk.r[p] = tk.b[p] - tk.r[p];
}

}  // namespace

void launch_spmv(const SpmvTask* d_tasks, int ntasks, long long max_rows, int xprec,
                 hipStream_t st) {
  if (ntasks <= 0) return;
  dim3 grid((unsigned)((max_rows + 255) / 256), (unsigned)ntasks);
  if (xprec == HH_FP64)
    hipLaunchKernelGGL(k_spmv<double>, grid, dim3(256), 0, st, d_tasks);
  else
    hipLaunchKernelGGL(k_spmv<float>, grid, dim3(256), 0, st, d_tasks);
  HH_HIP(hipGetLastError());
}

void launch_gram(const GramTask* d_tasks, int ntasks, int max_nblk, int max_px, int max_ty,
                 hipStream_t st) {
  if (ntasks <= 0) return;
  if (max_ty <= 1) {
    dim3 grid((unsigned)max_nblk, (unsigned)((max_px + 15) / 16), (unsigned)ntasks);
    hipLaunchKernelGGL((k_gram_partial<16, 1>), grid, dim3(256), 0, st, d_tasks);
  } else if (max_ty <= 2) {
    dim3 grid((unsigned)max_nblk, (unsigned)((max_px + 7) / 8), (unsigned)ntasks);
    hipLaunchKernelGGL((k_gram_partial<8, 2>), grid, dim3(256), 0, st, d_tasks);
  } else if (max_ty <= 4) {
    dim3 grid((unsigned)max_nblk, (unsigned)((max_px + 3) / 4), (unsigned)ntasks);
    hipLaunchKernelGGL((k_gram_partial<4, 4>), grid, dim3(256), 0, st, d_tasks);
  } else {
    set_error("block width %d exceeds 4", max_ty);
    throw ArgError();
  }
  HH_HIP(hipGetLastError());
  dim3 g2((unsigned)((max_px * max_ty + 3) / 4), (unsigned)ntasks);
  hipLaunchKernelGGL(k_gram_reduce, g2, dim3(256), 0, st, d_tasks);
  HH_HIP(hipGetLastError());
}

void launch_qr_step(const QrTask* d_tasks, int ntasks, int max_nblk, hipStream_t st) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_qr_step, dim3((unsigned)max_nblk, (unsigned)ntasks), dim3(256), 0, st,
                     d_tasks);
  HH_HIP(hipGetLastError());
}

void launch_block_update(const UpdTask* d_tasks, int ntasks, long long max_len, int max_ty,
                         hipStream_t st) {
  if (ntasks <= 0) return;
  dim3 grid((unsigned)((max_len + 255) / 256), (unsigned)ntasks);
  if (max_ty <= 1)
    hipLaunchKernelGGL(k_block_update<1>, grid, dim3(256), 0, st, d_tasks);
  else if (max_ty <= 2)
    hipLaunchKernelGGL(k_block_update<2>, grid, dim3(256), 0, st, d_tasks);
  else
    hipLaunchKernelGGL(k_block_update<4>, grid, dim3(256), 0, st, d_tasks);
  HH_HIP(hipGetLastError());
}

void launch_normalize(const NormTask* d_tasks, int ntasks, long long max_len, hipStream_t st) {
  if (ntasks <= 0) return;
  dim3 grid((unsigned)((max_len + 255) / 256), (unsigned)ntasks);
  hipLaunchKernelGGL(k_normalize, grid, dim3(256), 0, st, d_tasks);
  HH_HIP(hipGetLastError());
}

void launch_combine(const CombTask* d_tasks, int ntasks, long long max_len, int zprec,
                    hipStream_t st) {
  if (ntasks <= 0) return;
  dim3 grid((unsigned)((max_len + 255) / 256), (unsigned)ntasks);
  if (zprec == HH_FP64)
    hipLaunchKernelGGL(k_combine<double>, grid, dim3(256), 0, st, d_tasks);
  else
    hipLaunchKernelGGL(k_combine<float>, grid, dim3(256), 0, st, d_tasks);
  HH_HIP(hipGetLastError());
}

void launch_residual(const ResTask* d_tasks, int ntasks, long long max_len, hipStream_t st) {
  if (ntasks <= 0) return;
  dim3 grid((unsigned)((max_len + 255) / 256), (unsigned)ntasks);
  hipLaunchKernelGGL(k_residual, grid, dim3(256), 0, st, d_tasks);
  HH_HIP(hipGetLastError());
}

}  // namespace hh

namespace hh {
namespace {
__global__ void k_widen(const c64* __restrict__ a, c128* __restrict__ b, long long n) {
  long long p = blockIdx.x * 256LL + threadIdx.x;
  if (p < n) b[p] = mk((double)a[p].re, (double)a[p].im);
}

__global__ __launch_bounds__(256) void k_gather(const CopyTask* __restrict__ tasks,
                                                unsigned char* __restrict__ dst) {
  const CopyTask t = tasks[blockIdx.x];
  const unsigned* __restrict__ src = static_cast<const unsigned*>(t.src);
  unsigned* __restrict__ out = reinterpret_cast<unsigned*>(dst + t.dst);
  for (long long i = threadIdx.x; i < t.words; i += blockDim.x) out[i] = src[i];
}
}  // namespace

__global__ __launch_bounds__(256) void k_zero(unsigned* __restrict__ p, long long n) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i < n) p[i] = 0u;
}

void launch_zero(void* p, size_t bytes, hipStream_t st) {
  const long long n = (long long)(bytes / 4);
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (unsigned*)p, n);
  HH_HIP(hipGetLastError());
}

void launch_gather(const CopyTask* d_tasks, int ntasks, unsigned char* dst, hipStream_t st) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)ntasks), dim3(256), 0, st, d_tasks, dst);
  HH_HIP(hipGetLastError());
}

void launch_widen(const c64* a, c128* b, long long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_widen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
  HH_HIP(hipGetLastError());
}
}  // namespace hh
