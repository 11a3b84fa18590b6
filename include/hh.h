/*
 * hh.h -- C ABI of the MI355X multipreconditioned sweeping Helmholtz solver.
 *
 * Solves the impedance Helmholtz problem of Bootland & Rees (arXiv 2408.11929),
 * eq. (1):  Delta u + k^2 u = f in (0,1)^2,  du/dn - i k u = 0 on the boundary,
 * k = omega / c, discretised with continuous P1 triangles, by selective
 * multipreconditioned GMRES (Sec. 3) whose preconditioners are directional
 * double sweeps over overlapping strips with zeroth-order Robin transmission
 * (Sec. 2, eqs. (2)-(4)); the x sweep is "LRL", the y sweep "BTB" (Sec. 4).
 *
 * Conventions shared by every entry point
 *   - Grid: n x n nodes at (i h, j h), h = 1/(n-1); node index p = j*n + i.
 *   - Complex numbers are interleaved (re, im) pairs: hh_c128 is two doubles,
 *     layout-compatible with C99 double _Complex and numpy/torch complex128.
 *   - "device pointer" means memory allocated on the current HIP device
 *     (hipMalloc or any allocator over it); "host pointer" means ordinary
 *     CPU memory.  Arrays are only read or written during the call unless an
 *     entry point says otherwise; the library keeps no reference to them.
 *   - Every call returns an int status: HH_OK (0), HH_PENDING (1), or a
 *     negative error code.  hh_last_error() returns a message for the last
 *     failing call of the calling thread.  On error, output arrays may be
 *     partially written; handles stay valid.
 *   - All work runs on the library's own HIP streams (default priority) and
 *     every call is synchronous with respect to the host unless it says
 *     otherwise.  One problem handle must not be used from two threads at
 *     once; different handles may.
 */
#ifndef HH_H
#define HH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HH_OK 0
#define HH_PENDING 1
#define HH_EINVAL (-1)     /* invalid argument or state                      */
#define HH_ENOMEM (-2)     /* device memory allocation failed                */
#define HH_ESINGULAR (-3)  /* zero or non-finite pivot in a strip factorisation */
#define HH_ENOCONV (-4)    /* MPGMRES hit maxit before reaching the tolerance */
#define HH_EDEVICE (-5)    /* HIP runtime error                              */
#define HH_EBUDGET (-6)    /* request can never fit the server's HBM budget  */

#define HH_DIR_X 1u        /* LRL: strips in x, swept left to right and back  */
#define HH_DIR_Y 2u        /* BTB: strips in y, swept bottom to top and back  */

/* Preconditioner kinds (Sec. 4, Table 1): double sweeps and single sweeps. */
#define HH_PRE_LRL 1       /* x: left to right, then back to the left        */
#define HH_PRE_BTB 2       /* y: bottom to top, then back to the bottom      */
#define HH_PRE_LR 3        /* x: one forward sweep, left to right            */
#define HH_PRE_RL 4        /* x: one forward sweep, right to left            */
#define HH_PRE_BT 5        /* y: one forward sweep, bottom to top            */
#define HH_PRE_TB 6        /* y: one forward sweep, top to bottom            */

#define HH_FP64 0          /* strip factors and sweeps in complex128          */
#define HH_FP32 1          /* strip factors and sweeps in complex64           */

typedef struct {
  double re, im;
} hh_c128;

typedef struct hh_problem hh_problem;

/* Per right-hand-side result of hh_mpgmres. */
typedef struct {
  int iterations;        /* outer MPGMRES iterations (each applies all t sweeps) */
  int converged;         /* 1 if the least-squares residual reached tol           */
  double res_est;        /* least-squares residual estimate, relative to ||b||    */
  double res_true;       /* ||b - A x||_2 / ||b||_2 recomputed in FP64             */
  int basis_size;        /* number of orthonormal basis vectors built              */
  int deflated;          /* Z columns whose A z added no new basis direction       */
} hh_stats;

/* ---- assembly: eq. (1) ------------------------------------------------------
 * Builds the P1 operator A = K - M_{k^2} - i M_{Gamma,k} of eq. (1) on the
 * n x n grid and keeps it on the device (four upper diagonals of the complex
 * symmetric matrix, complex128).  The wave speed c is piecewise constant on
 * nlayers equal horizontal layers (layer 0 at the bottom); the wave number of a
 * triangle is omega / c at its centroid, that of a boundary edge omega / c at
 * its midpoint, with the layer of a height y = P / (6(n-1)) computed in exact
 * integer arithmetic as min(floor(P nlayers / (6(n-1))), nlayers - 1).
 *   omega      angular frequency (> 0, finite); with c = 1, k = omega
 *   nlayers    >= 1;  c_layers: host pointer, nlayers positive finite speeds
 *   n          nodes per side, 3 <= n <= 8193
 *   out        receives a new problem handle (free with hh_free)
 * Errors: HH_EINVAL for bad arguments, HH_ENOMEM, HH_EDEVICE. */
int hh_assemble(double omega, int nlayers, const double* c_layers, int n, hh_problem** out);

/* Wave-speed field of eq. (1) (k = omega / c) for hh_assemble_field: either
 * a function c(x, y) that the library samples on the host at every triangle
 * centroid and every mesh-edge midpoint (4 n^2 calls or so; it must return a
 * positive finite speed), or, with speed == NULL, the layer table of
 * hh_assemble. */
typedef double (*hh_speed_fn)(double x, double y, void* ctx);
typedef struct {
  hh_speed_fn speed;        /* or NULL: use nlayers / c_layers                */
  void* ctx;                /* passed to speed                                */
  int nlayers;              /* equal horizontal layers, layer 0 at the bottom */
  const double* c_layers;   /* host pointer, nlayers speeds                   */
  int scheme;               /* HH_SCHEME_P1 or HH_SCHEME_FD5                  */
} hh_cfield;

/* Discretisations of eq. (1) on the n x n grid: continuous P1 triangles (the
 * "/" diagonal in every cell), or the five-point finite differences of Sec. 4
 * with the impedance condition imposed through an eliminated ghost node at
 * each boundary side (central difference), rows scaled by h^2 times the node
 * weight (1/2 on a side, 1/4 at a corner) so that A stays complex symmetric:
 * A = K - h^2 diag(k^2 w) - i h diag(k on the boundary), k at the nodes, and
 * b = -h^2 w f.  The strips of the sweeps get the same scheme on their
 * rectangles. */
#define HH_SCHEME_P1 0
#define HH_SCHEME_FD5 1

/* hh_assemble for a general speed field (eq. (1)): the P1 operator with the
 * wave number omega / c(centroid) on each triangle and omega / c(midpoint) on
 * each edge (boundary edges in A, interface edges in the strip operators of
 * eq. (4)), or with c->scheme == HH_SCHEME_FD5 the five-point operator with
 * omega / c at the nodes (layers: the node's layer).  f: NULL, or a device pointer to n*n hh_c128 nodal source values;
 * then b = -M f is formed and kept with the problem, and hh_mpgmres with
 * b == NULL and nrhs == 1 solves for it.  Errors: HH_EINVAL (also for a
 * speed that is not positive and finite at a sample point), HH_ENOMEM,
 * HH_EDEVICE. */
int hh_assemble_field(double omega, const hh_cfield* c, int n, const hh_c128* f,
                      hh_problem** out);

/* Right-hand side of eq. (1) for nodal sources: b = -M f (P1 mass matrix M;
 * b = -h^2 w f for the five-point scheme), impedance data g = 0.  f and b are device pointers to nvec x n*n hh_c128
 * (vector v at offset v*n*n); f and b must not overlap. */
int hh_load_vector(hh_problem* pb, int nvec, const hh_c128* f, hh_c128* b);

/* ---- strip factorisation: Sec. 2 (Fig. 1) and Sec. 4 setup -----------------
 * Decomposes the square into nstrips overlapping strips per selected
 * direction (one extra mesh line per internal boundary, overlap 2h) and
 * factors every strip matrix (P1 operator of the strip with the impedance
 * operator of eq. (4) on its artificial sides) by band LU with partial
 * pivoting, all strips of all directions in one launch.  Replaces any
 * previous factorisation of the handle.
 *   dirs       HH_DIR_X, HH_DIR_Y or both; with both, the preconditioner order
 *              is M_1 = LRL, M_2 = BTB (the ordered combination of Sec. 4)
 *   nstrips    N >= 1 with (n-1) % N == 0 and (n-1)/N >= 2 when N > 1; the
 *              band half-width of a strip, kl = (strip width in node lines)
 *              + 1, must be at most 191.  Up to kl = 63 the strips get the
 *              one-wave LU and the blocked substitution with its segment plans;
 *              wider strips (e.g. N = 4 and 8 at n = 513: kl = 132 and 68) are
 *              factored by a blocked band LU whose trailing updates run on the
 *              matrix cores and are swept by the lane-major substitution on
 *              one wave per chain (one workgroup per chain, no tiles; the
 *              server refuses them).
 *   precision  HH_FP64 or HH_FP32 (factors, transmission data and sweeps)
 * Errors: HH_EINVAL, HH_ENOMEM, HH_ESINGULAR (a zero pivot, or one that is not
 * finite in the strip precision, as when omega / c is so large that strip
 * entries overflow complex64; the message names the strip), HH_EDEVICE. */
int hh_factor_sweeps(hh_problem* pb, unsigned dirs, int nstrips, int precision);

/* Recursive strip solves (Sec. 4, closing discussion: the strip problems
 * decomposed again in the perpendicular direction and solved approximately):
 * as hh_factor_sweeps, but every strip is cut along its length into nsub
 * sub-blocks by the same rule as the strips ((n-1) % nsub == 0, (n-1)/nsub
 * >= 2, one extra mesh line past each internal boundary), only the
 * sub-blocks are factored, and each strip solve of a sweep becomes one inner
 * double sweep over them, with the strip operator A_s in the role of A: the
 * sub-block operators carry the impedance condition on all four sides and
 * their transmission data are A_{s,t} R_t u - R_t A_s u on their interface
 * lines.  A sub-block is ordered by its narrower side, so wide strips get
 * narrow bands (at most 191).  nsub = 1 is hh_factor_sweeps with the strip
 * solves done this way (the exact strip solve).  The preconditioner, sweep
 * and MPGMRES entry points then apply these inexact sweeps (one wave per
 * chain, lane-major substitutions); hh_strip_solve is refused.
 * Errors: as hh_factor_sweeps. */
int hh_factor_sweeps_inner(hh_problem* pb, unsigned dirs, int nstrips, int nsub, int precision);

/* ---- preconditioner application: eqs. (2)-(4) -------------------------------
 * z = M_dir^{-1} r for nvec vectors: forward sweep over strips 1..N, backward
 * sweep over N-1..1, 2N-1 strip solves, overlap values from the most recent
 * solve.  r, z: device pointers, nvec x n*n hh_c128 (non-overlapping).  With
 * HH_FP32 factors, r is rounded to complex64 and z holds the complex64 result
 * exactly.  dir is HH_DIR_X or HH_DIR_Y (must have been factored).
 * Each vector is one sweep chain.  Few chains (at most half the compute units
 * at sixteen workgroups each) of complex64 strips none of which pivoted run on
 * sixteen workgroups per chain that meet four times per strip solve; the
 * environment variable HH_SWEEP_PLAN=0/1 forces one or sixteen (where
 * possible), and
 * HH_SWEEP_WAIT_US bounds each meeting (default 250000): a chain whose
 * workgroups do not meet in time stops, and the call returns HH_EDEVICE. */
int hh_sweep_apply(hh_problem* pb, unsigned dir, int nvec, const hh_c128* r, hh_c128* z);

/* z = M^{-1} r for the preconditioner `kind` (HH_PRE_*): the double sweeps
 * as in hh_sweep_apply, or a single sweep (Sec. 4, the LR, RL, BT and TB of
 * Table 1): one pass of eq. (2), N strip solves, each strip taking the
 * transmission data of the previous solve on the interface that faces it and
 * zero data on the other; in the overlaps the most recent solve wins.  LR and
 * BT go from strip 1 to N, RL and TB from N to 1.  The kind's direction must
 * have been factored; r, z, nvec and errors as in hh_sweep_apply. */
int hh_precond_apply(hh_problem* pb, int kind, int nvec, const hh_c128* r, hh_c128* z);

/* hh_precond_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with the call's scratch (descriptors, sync
 * words, strip buffers, complex64 staging, exchange areas) in one static
 * device array of 64 MiB that each GPU running the library holds until the
 * process ends.  It calls no hipMalloc/hipFree.  Calls on one GPU share that
 * array: calls that overlap in time on the same GPU race (serialise them);
 * the array keeps the last call's contents, and each call clears what must
 * start at zero.  The problem's device must be current.
 * Errors: HH_EINVAL when the call needs more than 64 MiB of scratch (about
 * 0.93 MiB per vector at n = 321 with complex64 strips), when the problem's
 * device is not current, or when a complex64 batch of more than eight
 * vectors needs the one-workgroup transfer maps and no allocating
 * application has built them yet; otherwise as hh_precond_apply. */
int hh_precond_apply_noalloc(hh_problem* pb, int kind, int nvec, const hh_c128* r, hh_c128* z);

/* Chooses the t preconditioners M_1..M_t that hh_mpgmres combines, in order
 * (Sec. 3; the combinations of Sec. 4 such as LRL+BTB, LR+RL or
 * LR+BT+RL+TB).  kinds: host pointer to t HH_PRE_* values, 1 <= t <= 4, each
 * of a factored direction (a kind may repeat).  hh_factor_sweeps resets the
 * choice to the double sweeps of its directions (LRL, then BTB).
 * Errors: HH_EINVAL. */
int hh_set_preconditioners(hh_problem* pb, int t, const int* kinds);

/* One strip solve x = A_s^{-1} rhs with the stored factors (strip s is
 * 1-based, vectors in the strip's local order q = long*w + short, where w is
 * the strip width in mesh lines).  rhs, x: device pointers of
 * n*w hh_c128 each.  Test hook for the factorisation. */
int hh_strip_solve(hh_problem* pb, unsigned dir, int s, const hh_c128* rhs, hh_c128* x);

/* Geometry of strip s (1-based): first node line a, width w (node lines),
 * band half-width kl. Host pointers; any may be NULL. */
int hh_strip_info(const hh_problem* pb, unsigned dir, int s, int* a, int* w, int* kl);

/* ---- operator products ------------------------------------------------------
 * y = A x for nvec vectors (device pointers, nvec x n*n, non-overlapping). */
int hh_spmv(hh_problem* pb, int nvec, const hh_c128* x, hh_c128* y);

/* Copies the assembled operator to host memory: diag is 4 x n*n hh_c128 with
 * rows A[p][p], A[p][p+1], A[p][p+n], A[p][p+n+1] (zero where the neighbour
 * does not exist); the lower part follows from A = A^T. */
int hh_get_operator(const hh_problem* pb, hh_c128* diag);

/* ---- selective MPGMRES: Sec. 3 with the selection rule of Sec. 4 -----------
 * Solves A x = b for nrhs independent right-hand sides that share the
 * factored sweeps (one MPGMRES per RHS, batched on the device).  x0 = 0, no
 * restart; iteration k applies each of the t chosen preconditioners once
 * (hh_set_preconditioners; by default the double sweeps of the factored
 * directions).  Selection (Sec. 4): for t = 2 the cross rule (M_1 is applied
 * to the basis vector that came from M_2's column and vice versa); for t > 2
 * every M_i is applied to the sum of the new basis vectors; t = 1 is
 * right-preconditioned GMRES.  The new block is
 * orthogonalised by two passes of block classical Gram-Schmidt and a
 * reorthogonalised modified Gram-Schmidt inside the block; the small least
 * squares problem is solved on the host in FP64.  Stops when the
 * least-squares residual is <= tol ||b||_2.  SpMV, Gram-Schmidt, least
 * squares and the final residual check are FP64 whatever the strip precision.
 *   b, x       device pointers, nrhs x n*n hh_c128 (x is overwritten); b may
 *              be NULL for the one right-hand side given to hh_assemble_field
 *   tol        > 0;  maxit >= 1
 *   stats      host pointer to nrhs hh_stats (may be NULL)
 * The sweeps of every RHS and direction run in one launch per iteration, one
 * chain each, on one or sixteen workgroups per chain as in hh_sweep_apply.
 * Returns HH_ENOCONV (x and stats still filled) if any RHS did not converge,
 * HH_EINVAL if one holds a NaN or Inf (see hh_mpgmres_x0). */
int hh_mpgmres(hh_problem* pb, int nrhs, const hh_c128* b, double tol, int maxit,
               hh_c128* x, hh_stats* stats);

/* hh_mpgmres from a starting guess x0 (Sec. 3 with a non-zero initial
 * iterate): the Krylov space is built on r0 = b - A x0 (FP64), the result is
 * x = x0 + Z y, and the stopping test and the reported residuals stay relative
 * to ||b||_2, so that a solve resumed from a saved x stops where an
 * uninterrupted one would.  x0 is a device pointer of nrhs x n*n hh_c128 or
 * NULL (= hh_mpgmres); it may be the same array as x (resume in place) but
 * must not overlap it otherwise.  A right-hand side with b = 0 gets x = 0;
 * one whose b or A x0 holds a NaN or Inf is not iterated (x = x0, or 0, and
 * res_true = NaN) and the call returns HH_EINVAL naming it, after the
 * others are solved (hh_mpgmres does the same). */
int hh_mpgmres_x0(hh_problem* pb, int nrhs, const hh_c128* b, const hh_c128* x0, double tol,
                  int maxit, hh_c128* x, hh_stats* stats);

/* Releases the handle and all its device memory.  NULL is accepted. */
int hh_free(hh_problem* pb);

/* ---- device memory and streams from the caller ------------------------------
 * hh_set_allocator: every device buffer the library needs from now on
 * (operators, strip factors, Krylov bases, scratch) comes from alloc(bytes,
 * ctx) and goes back through free_fn(p, ctx), e.g. a framework's caching
 * allocator; both NULL restores the library's own cache over hipMalloc.  The
 * library frees a buffer only after the work that used it has completed on
 * its streams.  alloc must return device memory of the current device (NULL
 * on failure: the call that needed it returns HH_ENOMEM) and may be called
 * from the serving thread.  Only while the library holds no device memory
 * (every problem and server freed), else HH_EINVAL.  The static scratch of
 * hh_precond_apply_noalloc is not affected. */
int hh_set_allocator(void* (*alloc)(size_t bytes, void* ctx), void (*free_fn)(void* p, void* ctx),
                     void* ctx);

/* hh_set_streams: problems created from now on run their work on the
 * caller's HIP streams (hipStream_t handles, passed as void*): x carries
 * assembly, factorisation, sweeps (both directions share one launch) and the
 * MPGMRES iteration; y is kept as the problem's second stream.  One of them
 * may be NULL (the other is used for both); both NULL restores streams that
 * each problem creates and destroys.  The library does not destroy caller
 * streams, and calls stay synchronous with respect to the host. */
int hh_set_streams(void* x, void* y);

/* ---- autotuning of the sweep's segment plan ----------------------------------
 * A sweep launch runs its chains on one, two or sixteen workgroups each.  With
 * hh_autotune(1) (or HH_AUTOTUNE=1 in the environment) hh_mpgmres times every
 * plan that fits the first launch of each shape (precision, band, mesh, strip
 * count, chains rounded up to a power of two), keeps the fastest and reuses
 * it; without it, a stored choice is still used, else a fixed rule.  Off by
 * default: the plans sum in different orders, so a timed choice would let
 * the last bits of results vary between processes.  Choices persist in a JSON
 * file: hh_tune_save / hh_tune_load, or automatically when HH_TUNE_CACHE names
 * the file.  hh_tune_clear forgets them.  Errors: HH_EINVAL (unreadable or
 * unwritable file). */
int hh_autotune(int on);
int hh_tune_save(const char* path);
int hh_tune_load(const char* path);
int hh_tune_clear(void);

/* Releases the library's cached free device blocks and pooled timing events
 * (e.g. before the process exits).  Live handles are not affected. */
int hh_release_caches(void);

/* Message of the last failing call on this thread ("" if none). */
const char* hh_last_error(void);

/* ---- timing of the library's kernels ------------------------------------------
 * When enabled, every launch of the named kernel family is bracketed by HIP
 * events on the stream it runs on; hh_timing_get returns the number of
 * launches, their summed duration (ms) and the summed algorithmic bytes they
 * were charged (see the kernel's documentation) since the last reset.
 * Families: "sweep", "spmv", "factor", "orth", "assemble".
 * Timing adds an event query per launch; leave it off outside measurements. */
int hh_timing_enable(int on);
int hh_timing_reset(void);
int hh_timing_get(const char* family, long long* launches, double* total_ms, double* bytes);

/* ---- serving: continuous batching of solve requests ---------------------------
 * A server owns a scheduler thread that admits requests in arrival order
 * when their device footprint (operator, strip factors, Krylov workspace for
 * maxit iterations) fits the HBM budget, assembles and factors them, and
 * advances every admitted solve by one MPGMRES iteration per tick with
 * batched launches that mix requests of different sizes.  Results do not
 * depend on what else is in flight. */
typedef struct hh_server hh_server;

typedef struct {
  int n;                    /* nodes per side                                 */
  double omega;             /* angular frequency                              */
  int nlayers;              /* layer count                                    */
  const double* c_layers;   /* host pointer, copied at submit                 */
  int nsrc;                 /* right-hand sides in this request               */
  const hh_c128* f;         /* device pointer, nsrc x n*n nodal sources; read
                               until the request completes                   */
  hh_c128* x;               /* device pointer, nsrc x n*n solutions; written
                               before hh_poll reports completion             */
  int nstrips;              /* strips per direction                           */
  unsigned dirs;            /* HH_DIR_X | HH_DIR_Y                             */
  int precision;            /* HH_FP64 or HH_FP32                             */
  double tol;
  int maxit;
} hh_request;

typedef struct {
  int status;               /* HH_OK, HH_ENOCONV, or another error code       */
  int iterations_max;       /* largest iteration count over the request's RHS */
  double res_true_max;      /* largest FP64 relative residual over its RHS    */
  double t_submit;          /* seconds on the server clock                    */
  double t_admit;
  double t_done;
} hh_result;

/* hbm_budget: bytes of device memory the server may hold for requests;
 * max_active: cap on concurrently admitted requests (>= 1). */
int hh_server_create(size_t hbm_budget, int max_active, hh_server** out);
/* Thread-safe; never waits for the GPU.  HH_EBUDGET if the request alone
 * exceeds the budget, HH_EINVAL for invalid fields. */
int hh_submit(hh_server* srv, const hh_request* req, uint64_t* ticket);
/* HH_PENDING while the request is queued or running; otherwise fills res and
 * returns HH_OK (the ticket is then retired). */
int hh_poll(hh_server* srv, uint64_t ticket, hh_result* res);
/* Seconds on the server clock (the clock of hh_result's time stamps). */
double hh_server_clock(const hh_server* srv);
/* Waits for all requests, stops the scheduler, frees the server. */
int hh_server_destroy(hh_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* HH_H */
