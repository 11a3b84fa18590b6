// Task descriptors and launchers of the batched FP64 Krylov kernels.
#pragma once

#include "hh_internal.h"

namespace hh {

// y = A x for nvec vectors of one problem.
struct SpmvTask {
  const c128* A;   // 4 n*n upper diagonals
  const void* x;   // nvec vectors, stride n*n (complex of the launch's xprec)
  c128* y;         // nvec vectors, stride n*n
  int n;
  int nvec;
};

// out (px x ty, column stride ldo) (=|+=) X^H Y, X: px columns, Y: ty columns.
struct GramTask {
  const c128* X;
  const c128* Y;
  c128* out;
  c128* part;      // >= nblk * px * ty scratch
  long long len;
  long long ldx, ldy;
  int ldo;
  int px;
  int ty;
  int nblk;
  int accumulate;
};

// Y[:, c] -= X C[:, c].
struct UpdTask {
  const c128* X;
  c128* Y;
  const c128* C;
  long long len;
  long long ldx, ldy;
  int ldc;
  int px;
  int ty;
};

// y /= ||y|| unless ||y|| <= tol * ref (then y = 0 and *flag = 1).
struct NormTask {
  c128* y;
  const c128* x;     // the vector normalised into y (null: y itself)
  const c128* nrm2;  // .re = ||y||^2
  const c128* ref2;  // .re = reference norm squared
  c128* rdiag;       // receives ||y|| (0 if deflated)
  int* flag;
  long long len;
  double tol;
};

// One step of the QR of a solve's new block (modified Gram-Schmidt, two
// passes per column, then normalisation), fused: the previous step's Gram
// partial sums (cpx entries over cnblk row blocks) are reduced into cout, the
// column op is applied to y (QR_UPDATE: y -= Xop[:, 0..cpx) cout;
// QR_NORMALIZE: y /= ||y|| with ||y||^2 = cout[0], deflated as NormTask),
// then the next step's Gram partial sums Xg[:, 0..gpx)^H gy go to gpart
// (gpx = 0: none).  Every value is formed
// as by k_gram_reduce, k_block_update, k_normalize and k_gram_partial in
// turn, so the results are bitwise theirs.
enum QrOp { QR_NONE = 0, QR_UPDATE = 1, QR_NORMALIZE = 2 };
struct QrTask {
  const c128* cpart;
  c128* cout;
  int cpx, cnblk;
  int op;
  c128* y;
  const c128* Xop;
  const c128* ref2;
  c128* rdiag;
  int* flag;
  double tol;
  const c128* Xg;
  const c128* gy;
  c128* gpart;
  int gpx;
  int xg_is_y;  // column of Xg that is y (-1: none)
  int gy_is_y;  // gy is y
  int nblk;     // row blocks of the Gram (the op covers the same rows)
  long long len, ld;
};

// x = Z y.
struct CombTask {
  const void* Z;
  const c128* y;
  const c128* x0;  // added to Z y when not null (may equal x)
  c128* x;
  long long len;
  int ncols;
};

// r = b - r.
struct ResTask {
  const c128* b;
  c128* r;
  long long len;
};

// One region of a gather into a contiguous buffer: `words` 4-byte words from
// src to byte offset dst (a multiple of 4) of the destination.
struct CopyTask {
  const void* src;
  long long dst;
  long long words;
};

void launch_spmv(const SpmvTask* d_tasks, int ntasks, long long max_rows, int xprec,
                 hipStream_t st);
void launch_gram(const GramTask* d_tasks, int ntasks, int max_nblk, int max_px, int max_ty,
                 hipStream_t st);
void launch_block_update(const UpdTask* d_tasks, int ntasks, long long max_len, int max_ty,
                         hipStream_t st);
void launch_normalize(const NormTask* d_tasks, int ntasks, long long max_len, hipStream_t st);
void launch_combine(const CombTask* d_tasks, int ntasks, long long max_len, int zprec,
                    hipStream_t st);
void launch_residual(const ResTask* d_tasks, int ntasks, long long max_len, hipStream_t st);
// One fused QR step for ntasks solves (grid: max_nblk row blocks x tasks).
void launch_qr_step(const QrTask* d_tasks, int ntasks, int max_nblk, hipStream_t st);
// The regions of ntasks copy tasks into dst, one workgroup per task (so that
// an iteration's small results leave the device in one transfer).
void launch_gather(const CopyTask* d_tasks, int ntasks, unsigned char* dst, hipStream_t st);

}  // namespace hh

namespace hh {
// b = (complex128) a, elementwise.
void launch_widen(const c64* a, c128* b, long long n, hipStream_t st);
}  // namespace hh
