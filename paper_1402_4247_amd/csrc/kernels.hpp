// Internal launcher declarations and workspace descriptors of the HIP library.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace kgev {

// ---------------------------------------------------------------------------
// launch timing (profile.hip): while a phase is being profiled on this host
// thread, every stride-th launch of it carries a start and a stop event in
// its own dispatch (the runtime stamps them when the kernel starts and ends).
enum Phase { PH_NONE = 0, PH_HEMV = 1, PH_GEMM = 2 };
struct ProfLaunch {
    hipEvent_t start = nullptr, stop = nullptr;
};
// the events for this launch of the phase, or none if it is not timed
ProfLaunch prof_launch_begin(int phase, hipStream_t st);
// counts the launch; tallies its algorithmic work if it was timed
void prof_launch_end(int phase, hipStream_t st, const ProfLaunch& pl, double bytes, double flops);

template <typename F, typename... Args>
inline void launch_timed(const ProfLaunch& pl, F kernel, dim3 grid, dim3 block, hipStream_t st, Args... args)
{
    if (pl.start)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, pl.start, pl.stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

// ---------------------------------------------------------------------------
// matrix products (gemm.hip)
// Tile policy of the calling thread: products whose 64 x 64 grid has fewer
// workgroups than `slots` use 32 x 32 tiles; returns the previous value.
constexpr int GEMM_SMALL_SLOTS_DEFAULT = 256;
int gemm_small_tile_slots(int slots);
template <typename R>
hipError_t cgemm(hipStream_t st, char ta, char tb, int64_t m, int64_t n, int64_t k, cx<R> alpha,
                 const cx<R>* A, int64_t lda, int64_t sA, const cx<R>* B, int64_t ldb, int64_t sB,
                 cx<R> beta, cx<R>* C, int64_t ldc, int64_t sC, int64_t batch, bool lower);

// C = A B with A complex (m x k) and B real (k x n; ldb, sB in real elements)
template <typename R>
hipError_t cgemm_rb(hipStream_t st, int64_t m, int64_t n, int64_t k, const cx<R>* A, int64_t lda, int64_t sA,
                    const R* B, int64_t ldb, int64_t sB, cx<R>* C, int64_t ldc, int64_t sC, int64_t batch);

// C(lower) -= V W^H + W V^H   (m x m, inner dimension k)
// C_L = alpha op(A_L) op(B_L) + beta C_L for L = (l1, l2), l1 < batch,
// l2 < batch2, operands at base + l1 * s + l2 * s2
template <typename R>
hipError_t cgemm_batch2(hipStream_t st, char ta, char tb, int64_t m, int64_t n, int64_t k, cx<R> alpha,
                        const cx<R>* A, int64_t lda, int64_t sA, int64_t sA2, const cx<R>* B, int64_t ldb, int64_t sB,
                        int64_t sB2, cx<R> beta, cx<R>* C, int64_t ldc, int64_t sC, int64_t sC2, int64_t batch,
                        int64_t batch2);
template <typename R>
hipError_t cher2k_lower(hipStream_t st, int64_t m, int64_t k, const cx<R>* V, int64_t ldv, int64_t sV,
                        const cx<R>* W, int64_t ldw, int64_t sW, cx<R>* C, int64_t ldc, int64_t sC,
                        int64_t batch);

// ---------------------------------------------------------------------------
// blocked Householder tridiagonalisation (hetrd.hip)
template <typename R>
struct HetrdWs {
    int n, nb;
    int NBmax, CHmax;          // 64-row blocks of the largest trailing matrix; chunks per block column
    int zch;                   // tiles per chunk of the Hermitian product (set by hetrd: 4, or 1)
    int slots1;                // a column takes one-tile chunks when four-tile chunks would launch
                               // fewer workgroups than this over all problems (0: 768)
    cx<R>* A; int64_t lda, sA; // matrix (lower), reduced in place
    cx<R>* V; int64_t sV;      // reflectors, n x n, ld n (zero outside the reflector rows)
    cx<R>* W; int64_t sW;      // panel W, n x nb, ld n
    R* d; R* e; cx<R>* tau;    // stride n per problem
    // The per-column partials below come in two buffers selected by the
    // parity of the column they describe: the kernel that consumes column
    // i's partials writes column i+1's in the same launch.
    R* pnorm; int64_t s_pnorm; // partial squared norms, 2 x hetrd_pn(n)
    cx<R>* ypart; int64_t s_ypart;   // NBmax x NBmax x 64
    cx<R>* ypartT; int64_t s_ypartT; // NBmax x CHmax x 64
    // panel-dot partials W^H u and V^H u: per problem 2 x NBmax blocks of
    // [W part (nb), V part (nb)], so pvv = pvw + nb and the block stride is 2 nb
    cx<R>* pvw; cx<R>* pvv; int64_t s_pdot;
    R* qpart; int64_t s_qpart;       // NBmax x CHmax: per-chunk shares of Re(u^H A22 u)
};

inline int hetrd_nbmax(int64_t n) { return (int)((n - 1 + 63) / 64) > 0 ? (int)((n - 1 + 63) / 64) : 1; }
inline int hetrd_chmax(int64_t n) { return hetrd_nbmax(n); }   // room for one-tile chunks
int hetrd_pn(int64_t n);   // partial norms per column (one per 64-row block)

template <typename R>
hipError_t hetrd(hipStream_t st, const HetrdWs<R>& ws, int64_t nk);

// ---------------------------------------------------------------------------
// divide-and-conquer tridiagonal eigensolver (stedc.hip)
struct DcWs {
    int n;
    int64_t nk;
    const double* din; const double* ein; int64_t s_din;
    double* es;          // scaled off-diagonal, n per problem
    double* onrm;        // scale per problem
    double* D[2];        // n per problem
    double* Q[2]; int64_t sQ;  // n x n per problem; set by stedc()
    double* Vsec;        // n x n per problem
    int* kcnt; int* ndcnt; int* nrot; double* rho;   // per segment, stored at its first index
    int* perm; double* sd; double* sz;
    int* ndx; double* ndd; double* ndz;
    int* dfx; double* dfd;
    int* rota; int* rotb; double* rotc; double* rots;
    int* orgi; double* tauv; double* lam; double* zhat; int* cmap;
    int64_t s_w;         // stride of the eigenvalue output
    int* status;         // per problem (may be null)
};

hipError_t stedc(hipStream_t st, const DcWs& ws, double* w, double* Z, double* Qscratch, int64_t nk);

// eigenvalues only of nk tridiagonals (d, e with stride sde; e[i] couples
// rows i and i+1) by bisection on Sturm counts (bisect.hip); w: stride sw,
// ascending; work: stebz_work_bytes(nk) bytes
size_t stebz_work_bytes(int64_t nk);
hipError_t stebz(hipStream_t st, const double* d, const double* e, int64_t sde, int64_t n, int64_t nk, double* w,
                 int64_t sw, void* work);

// ---------------------------------------------------------------------------
// small kernels (util.hip)
hipError_t fill_zero(hipStream_t st, void* p, size_t bytes);
// dst(lower) = src(lower) for nk matrices; flags non-finite entries in status (code 3)
template <typename R>
hipError_t copy_lower_check(hipStream_t st, int64_t n, const double2* src, int64_t lds, int64_t ss,
                            cx<R>* dst, int64_t ldd, int64_t sd, int* status, int64_t nk);
// dst = full Hermitian matrix from the lower triangle of src (diagonal made real)
hipError_t hermitian_full(hipStream_t st, int64_t n, const double2* src, int64_t lds, int64_t ss, double2* dst,
                          int64_t ldd, int64_t sd, int64_t nk);
// dst (complex) = src (real), n x n, ld n
template <typename R>
hipError_t real_to_complex(hipStream_t st, int64_t n, const double* src, int64_t ss, cx<R>* dst, int64_t ldd,
                           int64_t sd, int64_t nk);
// columns to unit 2-norm, optionally divided by sqrt(s_j); with s given, also
// sets status 1 when s_0 <= s_tol * s_max
// (prune: a column with s_j <= s_tol s_max is zeroed instead, no status);
// s_max = s_{n-1}, or s_{nreal[k]-1} for problem k when nreal is given (an
// embedded problem whose padded directions sort last)
hipError_t normalize_cols(hipStream_t st, int64_t n, double2* U, int64_t ldu, int64_t su, const double* s,
                          int64_t ss, double s_tol, int* status, int64_t nk, int prune = 0,
                          const int* nreal = nullptr);
// pruned canonical orthogonalisation (util.hip): shift the dropped directions
// of A above its spectrum; afterwards set their eigenvalues to +inf and
// eigenvector columns to zero.  part: n doubles per k; ndrop: nk ints.
hipError_t prune_shift(hipStream_t st, int64_t n, double2* A, int64_t sA, double* part, const double* s, int64_t sst,
                       double s_tol, int* ndrop, int64_t nk, const int* nreal = nullptr);
hipError_t prune_finish(hipStream_t st, int64_t n, double* w, double2* C, int64_t ldc, const int* ndrop, int64_t nk);
hipError_t status_init(hipStream_t st, int* status, int64_t nk);
// nk synthetic matrices (entries in [-1, 1), real diagonal) for timing runs
template <typename R>
hipError_t fill_test_matrix(hipStream_t st, int64_t n, cx<R>* A, int64_t nk, uint64_t seed);
// Per-k status words are bit sets while the solve runs; status_finish turns
// them into the ABI codes, the input condition taking precedence:
// non-finite input > S not positive definite > no convergence.
constexpr int ST_NOTPD = 1, ST_NOCONV = 2, ST_NONFINITE = 4;
hipError_t status_finish(hipStream_t st, const int* bits, int32_t* codes, int64_t nk);

// mixed precision (refine.hip)
hipError_t float_to_double(hipStream_t st, const float* src, double* dst, int64_t count);
hipError_t c64_to_c128(hipStream_t st, const float2* src, double2* dst, int64_t count);
struct RefineWs {
    int64_t n;
    const double2* Af;        // full Hermitian FP64 matrix, n x n per problem
    double2* Y;               // in: eigenvector estimate; out: refined
    double2* Ynext;           // n x n scratch
    double2* G; double2* P; double2* S; double2* F;   // n x n scratch each
    double* pS; double* pR;   // n per problem
    double* delta;            // one per problem
    int* cid;                 // n per problem: cluster index of each eigenvalue
    int* status;              // per problem (ST_NOCONV when the last sweep was still far from converged)
};
// `iters` refinement sweeps; lam_out (n per problem) gets the refined eigenvalues
hipError_t refine(hipStream_t st, const RefineWs& ws, int64_t nk, int iters, double* lam_out);

// systems of uneven order embedded in one order N (batch.hip).  A chunk of
// at most BATCH_DESC problems travels by value in the kernel arguments;
// problem p of the chunk owns slots slot_base + slot0 .. + nk - 1 of the
// embedded batch.
struct BatchDesc {
    const double2* H;
    const double2* S;
    double* w;
    double2* C;
    int32_t* status;
    int64_t n, ld, ldc;
    int slot0;
};
constexpr int BATCH_DESC = 32;
struct BatchDescs {
    BatchDesc d[BATCH_DESC];
    int count;
    int64_t slot_base;
};
// per slot: the padding of S (mode 0: max_i S_ii; mode 1: 2 ||S||_F, above
// every eigenvalue of S, so the padded directions sort last) and the order
hipError_t batch_prep(hipStream_t st, const BatchDescs& ds, int64_t slots, int mode, double* spad, int* nreal);
hipError_t batch_embed(hipStream_t st, const BatchDescs& ds, int64_t slots, int64_t N, const double* spad, double2* Hp,
                       double2* Sp);
hipError_t batch_extract(hipStream_t st, const BatchDescs& ds, int64_t slots, int64_t N, const double2* Cp,
                         const double* wp, int* map, int* stp, bool with_vectors);

// back-transformation U <- Q U, or U <- U Q with right (util.hip); work: see
// unmtr_work_elems
template <typename R>
hipError_t unmtr(hipStream_t st, int64_t n, const cx<R>* V, int64_t sV, const cx<R>* tau, int64_t stau, cx<R>* U,
                 int64_t ldu, int64_t sU, cx<R>* work, int kb, int64_t nk, bool right = false);
// unit 2-norm columns of a real n x n matrix
hipError_t normalize_cols_real(hipStream_t st, int64_t n, double* Z, int64_t ldz, int64_t sz, int64_t nk);
int64_t unmtr_work_elems(int64_t n, int kb);   // complex elements per problem

// ---------------------------------------------------------------------------
// Band_DFT_Col Parts 5 and 6 (band.hip)
hipError_t fermi_level(hipStream_t st, const double* w, int64_t ldw, int n, int nk, const double* wk, double nelec,
                       double kT, double g, double* occ, int64_t ldo, double* out, int32_t* status);
size_t density_work_bytes(int64_t n, int64_t nk, int64_t nocc);
hipError_t density(hipStream_t st, const double2* C, int64_t ldc, int n, int nk, int nocc, const double* w,
                   int64_t ldw, const double* occ, int64_t ldo, const double* wk, double g, double2* rho,
                   double2* edm, int64_t ldr, void* work);

// ---------------------------------------------------------------------------
// Part 2 in Cholesky form (chol.hip): X = L^{-H} with S = L L^H.  A (the lower
// copy of S) is overwritten; L, Linv, X are n x n (ld n, stride n*n); work
// holds chol_work_elems(n) complex values per k; smax nk doubles.
int64_t chol_work_elems(int64_t n);
hipError_t cholesky_x(hipStream_t st, int64_t n, double2* A, int64_t lda, int64_t sA, double2* L, double2* Linv,
                      double2* X, double2* work, double* smax, double s_tol, int* status, int64_t nk);

// ---------------------------------------------------------------------------
// Band_DFT_Col Part 1 (bloch.hip): Bloch sum of real-space blocks grouped by
// atom pair (group g = blocks gptr[g] .. gptr[g+1]-1); all index arrays on
// the device and already validated; ph: nk x nR complex scratch.
hipError_t bloch_sum(hipStream_t st, int n, const int* off, int64_t ngroups, const int* gptr, const int* bi,
                     const int* bj, const int* rid, const int64_t* doff, const double2* data, int64_t nR,
                     const double* R, int64_t nk, const double* kf, double2* ph, double2* out);

}  // namespace kgev
