/*
 * kgev.h -- C ABI of the MI355X (gfx950) k-point generalized Hermitian
 * eigensolver.
 *
 * The library solves, for every k-point of a batch, the dense complex
 * Hermitian-definite generalized eigenproblem H(k) C = S(k) C Lambda, the
 * diagonalisation at the heart of OpenMX's Band_DFT_Col (Parq, Sevre & Lee,
 * arXiv:1402.4247, Section III):
 *   Part 2  diagonalise S and rearrange it:  S = U diag(s) U^H,
 *           X = U diag(s)^(-1/2)  (canonical orthogonalisation);
 *   Part 3  form "S^H H S" = X^H H X  (matrix products);
 *   Part 4  diagonalise it with Eigen_HH and one matrix product C = X Y
 *           (evaluated as (X Q) Z, Q the Householder reflectors and Z the
 *           tridiagonal eigenvectors: the same C).
 * Eigen_HH (Section III) is: Householder tridiagonalisation (Procedures 1-6),
 * a tridiagonal eigensolve, back-transformation ("rearrangement of
 * eigenvectors") and normalisation.  Every step runs in HIP kernels on the
 * GPU; nothing falls back to the host.
 *
 * Conventions for every entry point:
 *   - Complex numbers are kgev_z = {double re, im}, layout-compatible with
 *     C99 double _Complex, std::complex<double> and torch.complex128.
 *   - Matrices are column-major: element (i, j) of a matrix with leading
 *     dimension ld is at offset i + j*ld.  A batch of nk matrices is stored
 *     back to back with stride ld*n elements.
 *   - Hermitian inputs are read from the LOWER triangle only (i >= j); the
 *     strict upper triangle is never read and the imaginary part of the
 *     diagonal is ignored.
 *   - Eigenvalues are returned ascending; column j of C is the eigenvector
 *     of eigenvalue j, normalised so that C^H S C = I.  Each column is
 *     unique only up to a unit-modulus phase (and within degenerate
 *     eigenspaces only the spanned space is unique).
 *   - Ownership: the caller owns every buffer it passes.  The library never
 *     frees caller memory and keeps no caller pointer after a host call
 *     returns, or after the stream work of a device call has completed.
 *   - Device entry points are asynchronous on the given stream (a
 *     hipStream_t passed as void*; NULL = the null stream).  Their results and
 *     the per-k status words are valid once that stream has completed.
 *   - A context is not thread-safe: use one per host thread.
 *
 * Status codes (LAPACK-style): 0 success; -i argument i is invalid;
 * positive values are numerical conditions reported per k-point; the
 * negative codes below -99 are resource/runtime errors.  A k-point that fails
 * leaves its output slice unspecified; the other k-points of the same call
 * are still solved.
 */
#ifndef KGEV_H
#define KGEV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } kgev_z;

typedef int32_t kgev_status;
#define KGEV_OK            0
#define KGEV_ENOTPD        1    /* S(k) not positive definite: s_min <= s_tol * s_max */
#define KGEV_ENOCONV       2    /* tridiagonal eigensolver did not converge */
#define KGEV_ENONFINITE    3    /* NaN or Inf in the lower triangle of H(k) or S(k) */
#define KGEV_ERANGE        4    /* kgev_fermi_device: nelec not inside (0, g n sum(wk)) */
#define KGEV_ENOMEM     (-100)  /* device or host allocation failed */
#define KGEV_EDEVICE    (-101)  /* a HIP runtime call failed */
#define KGEV_EUNSUPPORTED (-102)/* option combination not supported */

#define KGEV_PREC_FP64        0 /* every step in FP64 / complex128 */
#define KGEV_PREC_FP32_REFINE 1 /* Part 4 tridiagonalisation and back-transform in
                                   complex64, then FP64 eigenpair refinement */

typedef struct kgev_ctx kgev_ctx;

typedef struct {
    int32_t precision;    /* KGEV_PREC_FP64 (default) or KGEV_PREC_FP32_REFINE */
    int32_t want_vectors; /* 1 (default): eigenvalues and eigenvectors; 0: eigenvalues only */
    int32_t panel_nb;     /* Householder panel width; 0 = tuned default */
    int32_t refine_iters; /* mixed precision: refinement sweeps, 1..10; 0 = default (3) */
    double s_tol;         /* S(k) is rejected when s_min <= s_tol * s_max; 0 = default 1e-12 */
    int32_t use_graph;    /* 1: capture the whole batched solve as one HIP graph on the first call with
                             these sizes, buffers and stream, and replay it afterwards (the stream must
                             not be the null stream); 0 (default): launch kernel by kernel */
    int32_t streams;      /* k-point groups solved concurrently, each on its own stream forked from
                             (and joined back into) the caller's stream: 0 = default, 1..8 */
    int32_t s_method;     /* Part 2: KGEV_S_EIG (default, the paper's diagonalisation of S,
                             X = U s^-1/2, KGEV_ENOTPD when s_min <= s_tol s_max),
                             KGEV_S_CHOLESKY (S = L L^H, X = L^-H with its columns in reverse order:
                             the same eigenpairs with a cheaper
                             S side; a pivot <= s_tol * max_i S_ii gives KGEV_ENOTPD), or
                             KGEV_S_PRUNE (the paper's diagonalisation; the n - n' directions with
                             s_j <= s_tol s_max are dropped instead of failing: w[0:n'] are the
                             reduced pencil's eigenvalues ascending, w[n':n] = +inf and columns
                             n'..n-1 of C are zero) */
    int32_t hemv_slots;   /* Householder reduction: a column's Hermitian product takes one 64 x 64
                             tile per workgroup when four tiles per workgroup would launch fewer
                             than this many workgroups over all k-points of the call, else four;
                             0 = tuned (kgev_autotune) or the default 768 (three per CU);
                             1 = always four */
    int32_t gemm_slots;   /* complex products (Parts 3 and 4, back-transformations): 32 x 32 tiles
                             when 64 x 64 tiles would launch fewer than this many workgroups, else
                             64 x 64 (the results are the same bits either way); 0 = tuned or the
                             default 256 (one per CU); 1 = always 64 x 64 */
    int32_t reserved[3];  /* must be zero */
} kgev_opts;

#define KGEV_S_EIG      0
#define KGEV_S_CHOLESKY 1
#define KGEV_S_PRUNE    2

/* Fill *opts with the defaults listed above. */
void kgev_opts_default(kgev_opts* opts);

/* Static, human-readable text for a status code. */
const char* kgev_status_str(kgev_status st);

/*
 * Create a context bound to HIP device `device`.  The context owns an
 * internal device workspace (grown on demand when callers pass no
 * workspace), the tuned panel/tile table and a few small device buffers.
 * The first call for a device also looks up that device's address of the
 * static workspace of kgev_solve_k_device_noalloc.
 * Returns KGEV_OK, -1 (ctx NULL), -2 (no such device) or KGEV_EDEVICE.
 */
kgev_status kgev_create(kgev_ctx** ctx, int device);

/*
 * Autotuner of panel and tile sizes for pencils of order n.  Times, on
 * synthetic Hermitian matrices of order n (four at a time): the blocked
 * Householder reduction (Procedures 1-6 of Section III, the largest cost of
 * Eigen_HH) for the panel widths 16, 24, 32, 48 and 64; at the fastest
 * width, the reduction for the Hermitian-product tile grouping thresholds
 * (opts.hemv_slots) 1 (four tiles per workgroup throughout), 256, 768, 2048
 * and 2^30 (one tile per workgroup throughout); and the n x n x n complex
 * products of Parts 3 and 4 for the product tile thresholds (opts.gemm_slots)
 * 1 (64 x 64 tiles throughout), 64, 256, 1024 and 2^30 (32 x 32
 * throughout).  A threshold other than the default is taken only when it is
 * more than 2% faster.  The choices are recorded in the context for (n,
 * precision); later calls through this context leaving the corresponding
 * option 0 use them.  The tuned values depend only on n and precision, not
 * on the batch.
 * Results are bitwise reproducible for the same n, k-point count and
 * options; the tile grouping of a column follows the launch's workgroup
 * count, so the same k-point solved in calls of different k-point counts
 * agrees to rounding, not necessarily bitwise.  *best_nb (optional)
 * receives the panel width.  Synchronous; uses the context's internal
 * workspace.
 */
kgev_status kgev_autotune(kgev_ctx* ctx, int64_t n, int32_t precision, int32_t* best_nb);

/*
 * The panel width and the two tile thresholds that solves of order n and
 * this precision use through ctx when opts leave them 0: the tuned values
 * after kgev_autotune(ctx, n, precision, ...), else the defaults (32, 768,
 * 256).  *tuned (optional) is set to 1 when they come from the tuner.  Any
 * output pointer may be NULL.  Returns KGEV_OK, -1 (ctx NULL) or -3 (bad
 * precision).
 */
kgev_status kgev_tuned_params(kgev_ctx* ctx, int64_t n, int32_t precision, int32_t* panel_nb,
                              int32_t* hemv_slots, int32_t* gemm_slots, int32_t* tuned);

/* Release a context and everything it owns.  NULL is allowed. */
void kgev_destroy(kgev_ctx* ctx);

/*
 * Device workspace, in bytes, that kgev_solve_k_device needs for nk
 * problems of order n with the given options (NULL = defaults).  Returns 0
 * for invalid n or nk.
 */
size_t kgev_workspace_bytes(int64_t n, int64_t nk, const kgev_opts* opts);

/*
 * Host-pointer, synchronous solve of nk k-points (Band_DFT_Col Parts 2-4,
 * Section III).
 *   H, S : host, nk column-major n x n matrices (ld = n), lower triangles read.
 *   w    : host, nk*n doubles; eigenvalues of k-point q at w[q*n .. q*n+n-1].
 *   C    : host, nk*n*n kgev_z; may be NULL when opts->want_vectors == 0.
 *   bad_k: optional; receives the first failing k index (or -1).
 * Returns the first nonzero per-k status, or an argument/runtime error:
 *   -1 ctx, -2 H, -3 S, -4 n < 1, -5 nk < 1, -6 w, -7 C, -8 opts invalid.
 */
kgev_status kgev_solve_k(kgev_ctx* ctx, const kgev_z* H, const kgev_z* S, int64_t n, int64_t nk,
                         double* w, kgev_z* C, const kgev_opts* opts, int64_t* bad_k);

/*
 * Device-pointer, asynchronous solve of nk k-points on `stream`.
 *   dH, dS   : device, nk matrices n x n with leading dimension ld >= n and
 *              batch stride ld*n; lower triangles read; not modified.
 *   dw       : device, nk*n doubles (eigenvalues, ascending per k).
 *   dC       : device, nk matrices n x n, leading dimension ldc >= n, batch
 *              stride ldc*n; may be NULL for eigenvalues only.
 *   dwork    : device workspace of work_bytes >= kgev_workspace_bytes(n, nk,
 *              opts), or NULL to use the context's internal workspace (which
 *              the library may then allocate).
 *   d_status : device, nk int32 status words (KGEV_OK / KGEV_ENOTPD /
 *              KGEV_ENOCONV / KGEV_ENONFINITE), or NULL.
 * Returns an argument/runtime error immediately, else KGEV_OK once every
 * kernel is enqueued (-1 ctx, -2 dH, -3 dS, -4 n, -5 ld, -6 nk, -7 dw,
 * -8 dC/ldc, -9 work too small, -10 opts invalid).
 */
kgev_status kgev_solve_k_device(kgev_ctx* ctx, const kgev_z* dH, const kgev_z* dS, int64_t n,
                                int64_t ld, int64_t nk, double* dw, kgev_z* dC, int64_t ldc,
                                void* dwork, size_t work_bytes, int32_t* d_status,
                                const kgev_opts* opts, void* stream);

/*
 * kgev_solve_k_device for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It calls no hipMalloc, hipFree or other allocating routine; its
 * workspace is a static device array of KGEV_NOALLOC_SCRATCH_BYTES per GPU,
 * reserved when the library's device code is loaded on that GPU and held
 * until the process ends.  The caller still passes inputs and outputs, with
 * the meanings of kgev_solve_k_device; the results are bitwise those of
 * kgev_solve_k_device with the same options.
 *   Limit: kgev_workspace_bytes(n, nk, opts) <= KGEV_NOALLOC_SCRATCH_BYTES
 *   (for example n = 1024 with one k-point, n = 512 with four, n = 128 with up
 *   to 43); larger sizes return -9 and nothing is enqueued.
 *   opts.use_graph = 1 or opts.streams > 1 return KGEV_EUNSUPPORTED.
 *   Launches of this entry point are not timed by kgev_profile_begin.
 * Every call on a GPU uses that GPU's one array, which keeps the last call's
 * contents (the solve initialises everything it reads): two calls whose stream
 * work overlaps on one GPU race and give undefined results; serialise them
 * (one stream, or events between streams).
 * Returns -1 ctx, -2 dH, -3 dS, -4 n, -5 ld, -6 nk, -7 dw, -8 dC/ldc, -9 the
 * workspace exceeds the array, -10 opts invalid, KGEV_EUNSUPPORTED, else
 * KGEV_OK once every kernel is enqueued.
 */
#define KGEV_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
kgev_status kgev_solve_k_device_noalloc(kgev_ctx* ctx, const kgev_z* dH, const kgev_z* dS, int64_t n, int64_t ld,
                                        int64_t nk, double* dw, kgev_z* dC, int64_t ldc, int32_t* d_status,
                                        const kgev_opts* opts, void* stream);

/*
 * The per-k solve with the S-orthonormaliser X of Part 2 exported or reused.
 * Band_DFT_Col solves every k-point twice per step (eigenvalues, then
 * eigenvectors) and, spin-collinear, once per spin with the same S(k); Part 2
 * depends on S(k) only, so its X can be formed once and reused.
 *   dX     : device, nk matrices n x n (ld n, k-stride n*n)
 *   x_mode : KGEV_X_EXPORT - Part 2 from dS as in kgev_solve_k_device, and its
 *            X written to dX;  KGEV_X_REUSE - Part 2 skipped, X read from dX
 *            (as exported by an earlier call with the same S(k)); dS is not
 *            read (may be NULL) and no S-definiteness status is reported.
 * The other arguments, results and statuses are as for kgev_solve_k_device
 * (kernels are launched one by one; opts.use_graph and opts.streams are
 * ignored; KGEV_X_REUSE with KGEV_S_PRUNE is KGEV_EUNSUPPORTED).  The
 * workspace is kgev_workspace_bytes(n, nk, opts) with opts.streams = 1.
 * Returns -1 ctx, -2 dH, -3 dS (export), -4 n, -5 ld, -6 nk, -7 dw, -8 dC/ldc,
 * -10 dX, -11 x_mode, -13 work too small, -15 opts invalid.
 */
#define KGEV_X_EXPORT 0
#define KGEV_X_REUSE  1
kgev_status kgev_solve_k_x_device(kgev_ctx* ctx, const kgev_z* dH, const kgev_z* dS, int64_t n, int64_t ld,
                                  int64_t nk, double* dw, kgev_z* dC, int64_t ldc, kgev_z* dX, int32_t x_mode,
                                  void* dwork, size_t work_bytes, int32_t* d_status, const kgev_opts* opts,
                                  void* stream);

/*
 * A batch of systems of uneven order (the k-point loop of Band_DFT_Col,
 * Section III, over pencils of different sizes).  The problems are grouped
 * into size classes, largest order first: a problem joins the current class
 * when the class order N is at most 256 or at most 1.26 times its own order.
 * Every k-point of a class is embedded in a pencil of order N,
 * H' = [[H, 0], [0, 0]], S' = [[S, 0], [0, s I]] with s = max_i S_ii, and
 * the class is solved as one batched solve (each launch covers all of its
 * k-points); the pencil's eigenpairs are exactly the embedded ones that
 * vanish on the padded rows, and they are written to the problem's buffers
 * in ascending order.  A class of a single problem of the class order is
 * solved in place, bitwise as kgev_solve_k_device would solve it; others
 * agree with their own calls to rounding.  Classes run one after another on
 * `stream`, sharing one workspace.  With opts.use_graph and a non-null
 * stream, the whole batch is captured once as one HIP graph and replayed by
 * later calls with the same problems, buffers, workspace, options and
 * stream.
 *   probs  : host array of count problem descriptors (read during the call
 *            only); each field as the argument of kgev_solve_k_device of the
 *            same name (d_status may be NULL).
 *   dwork  : device workspace of work_bytes >= kgev_batch_workspace_bytes(
 *            probs, count, opts), or NULL for the context's workspace.
 * Returns -1 ctx, -2 probs, -3 count < 1, -4 work too small, -5 opts
 * invalid, -(1000 + q) for an invalid descriptor q (n < 1, ld < n, nk < 1,
 * a required pointer NULL, ldc < n with vectors), else KGEV_OK once every
 * kernel is enqueued; per-k statuses land in each problem's d_status.
 */
typedef struct kgev_problem {
    int64_t n, ld, nk;
    const kgev_z* dH;
    const kgev_z* dS;
    double* dw;
    kgev_z* dC;
    int64_t ldc;
    int32_t* d_status;
} kgev_problem;
/* the largest workspace of the batch's size classes: a class's solve
 * workspace plus, when it embeds, the embedded H', S' (and C' with vectors),
 * eigenvalues, statuses and column map (0 if a descriptor has n < 1 or nk < 1) */
size_t kgev_batch_workspace_bytes(const kgev_problem* probs, int64_t count, const kgev_opts* opts);
kgev_status kgev_solve_batch_device(kgev_ctx* ctx, const kgev_problem* probs, int64_t count, void* dwork,
                                    size_t work_bytes, const kgev_opts* opts, void* stream);

/*
 * Stage entry points.  Each runs one step of the path on nk problems and
 * exists so that every step can be checked on its own; all are device-pointer
 * and asynchronous on `stream`, with the argument conventions above.
 */

/*
 * Householder tridiagonalisation (Section III, Procedures 1-6; blocked).
 *   dA  : in/out, nk matrices n x n (ld lda); lower triangle read and
 *         destroyed.
 *   dd  : out, nk*n doubles (diagonal of T); de: out, nk*n doubles (entry
 *         q*n+i, i < n-1, is T(i+1, i)); dtau: out, nk*n kgev_z (tau_i at
 *         q*n+i, i < n-1).
 *   dV  : out, nk matrices n x n (ld n): column i holds v_i in rows i+1..n-1
 *         with v_i(i+1) = 1 and zeros elsewhere, H_i = I - tau_i v_i v_i^H,
 *         T = Q^H A Q, Q = H_0 H_1 ... H_{n-2}.
 */
kgev_status kgev_hetrd_device(kgev_ctx* ctx, kgev_z* dA, int64_t n, int64_t lda, int64_t nk,
                              double* dd, double* de, kgev_z* dtau, kgev_z* dV,
                              const kgev_opts* opts, void* stream);

/*
 * Real symmetric tridiagonal eigensolve (the tridiagonal step of Eigen_HH,
 * Section III; divide and conquer).
 *   dd, de : in, nk*n doubles each (layout as kgev_hetrd_device); not modified.
 *   dw     : out, nk*n eigenvalues ascending.
 *   dZ     : out, nk real matrices n x n (ld n), orthonormal eigenvectors;
 *            column j belongs to eigenvalue j.
 *   d_status: optional, nk int32 (KGEV_ENOCONV on failure).
 */
kgev_status kgev_stedc_device(kgev_ctx* ctx, const double* dd, const double* de, int64_t n,
                              int64_t nk, double* dw, double* dZ, int32_t* d_status, void* stream);

/*
 * Eigenvalues only of real symmetric tridiagonals (the tridiagonal step of
 * Eigen_HH, Section III, in the form Band_DFT_Col's eigenvalue pass needs), by
 * bisection on Sturm counts: the number of eigenvalues below x is the number
 * of negative pivots of T - x I.  The solve uses it whenever eigenvectors are
 * not requested (opts.want_vectors = 0, FP64).
 *   dd, de : in, nk*n doubles each (layout as kgev_hetrd_device); not modified.
 *   dw     : out, nk*n eigenvalues ascending (k-point q at dw + q*n).
 * Asynchronous on `stream`; uses the context's internal workspace.  Returns
 * -1 ctx, -2 dd, -3 de, -4 n, -5 nk, -6 dw, KGEV_ENOMEM / KGEV_EDEVICE, else
 * KGEV_OK.
 */
kgev_status kgev_stebz_device(kgev_ctx* ctx, const double* dd, const double* de, int64_t n, int64_t nk,
                              double* dw, void* stream);

/*
 * Back-transformation ("rearrangement of eigenvectors", Section III):
 * dU <- Q dU for nk problems, with Q = H_0 ... H_{n-2} given by dV, dtau as
 * produced by kgev_hetrd_device.  dU: in/out, nk matrices n x n (ld ldu).
 */
kgev_status kgev_unmtr_device(kgev_ctx* ctx, const kgev_z* dV, const kgev_z* dtau, int64_t n,
                              int64_t nk, kgev_z* dU, int64_t ldu, void* stream);

/*
 * Eigen_HH (Section III): eigenvalues (ascending, dw: nk*n) and unit-norm
 * eigenvectors (dY: nk matrices n x n, ld n; may be NULL for eigenvalues
 * only, then by bisection) of the Hermitian matrices whose lower triangles are
 * dA (ld lda; not modified).
 */
kgev_status kgev_eigh_device(kgev_ctx* ctx, const kgev_z* dA, int64_t n, int64_t lda, int64_t nk,
                             double* dw, kgev_z* dY, int32_t* d_status, const kgev_opts* opts,
                             void* stream);

/*
 * Batched complex matrix product (the ZGEMM of Parts 3 and 4, Section III):
 * C_q = alpha op(A_q) op(B_q) + beta C_q for q < batch, op in {'N', 'C'}
 * ('C' = conjugate transpose); C is m x n, inner dimension k; sA, sB, sC are
 * batch strides in elements.  lower != 0 computes and writes only the
 * entries with i >= j.  beta == 0 never reads C.
 */
kgev_status kgev_zgemm_device(kgev_ctx* ctx, char transa, char transb, int64_t m, int64_t n,
                              int64_t k, kgev_z alpha, const kgev_z* dA, int64_t lda, int64_t sA,
                              const kgev_z* dB, int64_t ldb, int64_t sB, kgev_z beta, kgev_z* dC,
                              int64_t ldc, int64_t sC, int64_t batch, int32_t lower, void* stream);

/*
 * Serving: a request loop that admits eigensolves of mixed order n and k-point
 * count as execution slots and device memory free up (continuous batching at
 * request granularity).  Each admitted request runs the batched per-k solve
 * (Band_DFT_Col Parts 2-4, Section III) on its own HIP stream, so requests
 * admitted while others run overlap with them on the device.  Admission is in
 * arrival order (optionally with bounded bypass, kgev_server_set_bypass); a
 * request is admitted when a slot is free and its workspace
 * footprint (kgev_workspace_bytes + status words) fits the remaining budget;
 * the caller's own dH, dS, dw and dC are not counted, since they are allocated
 * before the request is submitted.  Inputs and outputs stay device-resident: the caller keeps dH, dS, dw and dC
 * (as in kgev_solve_k_device) alive and untouched until kgev_server_wait
 * returns for the request.  The server owns only workspaces, streams and its
 * worker thread; all entry points are thread-safe.
 */
typedef struct kgev_server kgev_server;

typedef struct {
    int64_t n, nk, ld;          /* order, k-points, leading dimension of dH/dS (>= n) */
    const kgev_z* dH;           /* device, nk matrices, lower triangles read */
    const kgev_z* dS;
    double* dw;                 /* device, nk*n eigenvalues */
    kgev_z* dC;                 /* device, nk matrices (ld ldc), or NULL for eigenvalues only */
    int64_t ldc;
    int32_t precision;          /* KGEV_PREC_FP64 or KGEV_PREC_FP32_REFINE */
    int32_t reserved;           /* must be zero */
} kgev_request;

typedef struct {
    kgev_status status;         /* first nonzero per-k status, KGEV_ENOMEM if it can never fit, or 0 */
    int64_t bad_k;              /* k index of that status, or -1 */
    double t_submit, t_admit, t_done;   /* seconds on a monotonic clock */
    size_t footprint;           /* device bytes the request held while running */
} kgev_result;

/*
 * Start a server on HIP device `device` with `max_slots` (1..64) concurrent
 * requests and a device-memory budget in bytes (0 = free memory minus a 4 GiB
 * reserve).  Returns -1 (out NULL), -2 (device), -4 (slots) or KGEV_EDEVICE.
 */
kgev_status kgev_server_create(kgev_server** out, int device, size_t hbm_budget, int32_t max_slots);

/*
 * Bounded bypass of the arrival order: when the request at the head of the
 * queue does not fit the remaining budget, a later request that fits may
 * start first, at most max_bypass times for the same head (0, the default:
 * strict arrival order).  The head therefore waits at most for max_bypass
 * later requests beyond the running ones, and never starves.  Takes effect
 * at the server's next scheduling pass; results do not depend on it.
 * Returns -1 (srv NULL) or -2 (max_bypass < 0).
 */
kgev_status kgev_server_set_bypass(kgev_server* srv, int32_t max_bypass);

/* Queue a request; *ticket identifies it.  -2: invalid request fields. */
kgev_status kgev_server_submit(kgev_server* srv, const kgev_request* req, uint64_t* ticket);

/* *done = 1 once the request has completed (results valid), else 0. */
kgev_status kgev_server_poll(kgev_server* srv, uint64_t ticket, int32_t* done);

/* Block until the request completes, fill *result and forget the ticket. */
kgev_status kgev_server_wait(kgev_server* srv, uint64_t ticket, kgev_result* result);

/* Drain queued and running requests, then stop the worker and free the server. */
void kgev_server_destroy(kgev_server* srv);

/*
 * Kernel timing for measurement.  Between kgev_profile_begin and
 * kgev_profile_end, every stride-th launch (stride >= 1; the first launch is
 * always timed) of the chosen phase made through this context carries two
 * HIP events in its own dispatch (hipExtLaunchKernel: the runtime stamps
 * them when the kernel starts and when it ends, on the stream it is enqueued
 * on), and the phase's algorithmic work of the timed launches is tallied:
 *   KGEV_PHASE_HEMV : the Hermitian product A22 v of the tridiagonalisation
 *                     (Procedure 4); work = bytes of the lower triangle of the
 *                     trailing matrix, 16 m (m + 1) / 2 per k-point;
 *   KGEV_PHASE_GEMM : every complex matrix product on MFMA; work = real flops,
 *                     8 m n k per product (half for lower-only outputs).
 * kgev_profile_end waits for the recorded events, returns the number of
 * timed launches, the number of all launches of the phase, the summed
 * duration of the timed launches in milliseconds and their summed
 * algorithmic bytes and flops, and stops recording.  Timing adds no packet
 * to the stream; a stride above 1 keeps the host-side event work small.  Launches captured into a graph (opts.use_graph)
 * are not timed or counted, since the runtime does not time events recorded
 * by graph nodes; both calls drop the context's cached graphs.
 * Errors: -1 ctx, -2 phase, -3 stride < 1; kgev_profile_end without a
 * matching begin returns KGEV_EUNSUPPORTED, a failed event query
 * KGEV_EDEVICE.
 */
/*
 * Band_DFT_Col Part 5 (arXiv:1402.4247, the routine's outline in the
 * section applying the method to OpenMX: chemical potential and band energy),
 * on the device.  The paper names the step only; the occupation of state j
 * of k-point k is the Fermi-Dirac function at temperature kT,
 *   f_kj = 1 / (1 + exp((w_kj - mu) / kT)),
 * and mu is the root of  g sum_k wk[k] sum_j f_kj = nelec  (g = electrons
 * per state: 2 without spin, 1 per spin channel), found by bisection on a
 * bracket 50 kT beyond the extreme eigenvalues until the midpoint no longer
 * separates from its ends.  Then
 *   e_band = g sum_k wk[k] sum_j f_kj w_kj.
 *   dw      : device, nk x n eigenvalues, k-point k at dw + k * ldw (ldw >= n)
 *   d_wk    : device, nk k-point weights
 *   d_occ   : device, nk x n occupations f_kj written at d_occ + k * ldo
 *             (ldo >= n), or NULL
 *   d_result: device, 3 doubles {mu, e_band, electron count at mu}
 *   d_status: device, one int32: KGEV_OK, or KGEV_ERANGE when nelec is not
 *             inside (0, g n sum(wk)) (then nothing else is written)
 * One workgroup; asynchronous on `stream`.  Returns an argument error at once
 * (-1 ctx, -2 dw, -3 ldw, -4 n, -5 nk, -6 d_wk, -8 kT <= 0 or not finite,
 * -9 g <= 0, -11 ldo, -12 d_result, -13 d_status), else KGEV_OK.
 */
kgev_status kgev_fermi_device(kgev_ctx* ctx, const double* dw, int64_t ldw, int64_t n, int64_t nk,
                              const double* d_wk, double nelec, double kT, double g, double* d_occ, int64_t ldo,
                              double* d_result, int32_t* d_status, void* stream);

/*
 * Band_DFT_Col Part 6 (same outline: charge density matrix and energy density
 * matrix), on the device, over the first nocc eigenvectors of each k-point:
 *   rho = g sum_k wk[k] sum_{j < nocc} f_kj c_kj c_kj^H
 *   edm = g sum_k wk[k] sum_{j < nocc} f_kj w_kj c_kj c_kj^H
 * with c_kj column j of C_k (dC + k * ldc * n, column-major, ldc >= n: the
 * layout kgev_solve_k_device writes).  Only the lower triangles (i >= j) of
 * rho and edm are written (ld ldr >= n); edm may be NULL.  The products run
 * as batched MFMA products (one per k-point, lower half) into the workspace,
 * then a fixed-order sum over k.
 *   dwork : device workspace of at least kgev_density_workspace_bytes(n, nk,
 *           nocc) bytes, or NULL to use the context's internal workspace.
 * Asynchronous on `stream`.  Returns an argument error at once (-1 ctx, -2 dC,
 * -3 ldc, -4 n, -5 nk, -6 nocc not in [0, n], -7 dw, -8 ldw, -9 d_occ,
 * -10 ldo, -11 d_wk, -12 g <= 0, -13 d_rho, -15 ldr, -17 work_bytes too
 * small), KGEV_ENOMEM / KGEV_EDEVICE, else KGEV_OK.
 */
size_t kgev_density_workspace_bytes(int64_t n, int64_t nk, int64_t nocc);
kgev_status kgev_density_device(kgev_ctx* ctx, const kgev_z* dC, int64_t ldc, int64_t n, int64_t nk, int64_t nocc,
                                const double* dw, int64_t ldw, const double* d_occ, int64_t ldo, const double* d_wk,
                                double g, kgev_z* d_rho, kgev_z* d_edm, int64_t ldr, void* dwork, size_t work_bytes,
                                void* stream);

/*
 * Band_DFT_Col Part 1 (the routine's outline: giving S and H their k-point
 * dependence), on the device, as the Bloch sum of real-space blocks:
 *   out_k = sum over blocks q of exp(2 pi i kf_k . R_{rid[q]}) M_q
 * with M_q placed at rows off[bi[q]].., columns off[bj[q]].. (k and R in
 * fractional coordinates: reciprocal and direct lattice units).
 *   off     : host, natom+1 orbital offsets per atom, off[0] = 0, n = off[natom]
 *   bi, bj, rid, doff : host, nblocks entries, sorted by (bi, bj); block q's
 *             data is d_data + doff[q], (n_bi x n_bj) column-major
 *   d_data  : device, data_elems kgev_z
 *   R       : host, nR x 3 doubles;  kf : host, nk x 3 doubles
 *   d_out   : device, nk matrices n x n (ld n); entries no block covers are
 *             zero.  The solver reads lower triangles, so blocks with bi >= bj
 *             (diagonal blocks Hermitian) suffice for kgev_solve_k_device.
 * The metadata is validated on the host (indices, offsets against
 * data_elems, order) and copied to the device on `stream` before the call
 * returns; the sum itself is asynchronous.  Returns -1 ctx, -2 natom/off,
 * -3 off not a valid layout (or n > 65535), -4 nblocks or order, -5 bi/bj,
 * -7 rid, -8 doff, -10 data_elems, -11 nR/R, -13 nk/kf, -15 d_out,
 * KGEV_ENOMEM / KGEV_EDEVICE, else KGEV_OK.
 */
kgev_status kgev_bloch_device(kgev_ctx* ctx, int32_t natom, const int32_t* off, int64_t nblocks, const int32_t* bi,
                              const int32_t* bj, const int32_t* rid, const int64_t* doff, const kgev_z* d_data,
                              int64_t data_elems, int64_t nR, const double* R, int64_t nk, const double* kf,
                              kgev_z* d_out, void* stream);

#define KGEV_PHASE_HEMV 1
#define KGEV_PHASE_GEMM 2
kgev_status kgev_profile_begin(kgev_ctx* ctx, int32_t phase, int32_t stride);
kgev_status kgev_profile_end(kgev_ctx* ctx, int64_t* launches, int64_t* phase_launches, double* total_ms,
                             double* alg_bytes, double* alg_flops);

#ifdef __cplusplus
}
#endif

#endif /* KGEV_H */
