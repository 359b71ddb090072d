// Small bandwidth-bound kernels of the path: input copy with the non-finite
// check, full Hermitian matrix from the lower triangle, real -> complex,
// eigenvector normalisation (Eigen_HH's last step) fused with Part 2's
// rearrangement of S (x_j = u_j / sqrt(s_j)) and its definiteness check, and
// the triangular factor of a block of reflectors (compact WY).
#include <utility>

#include "common.hpp"
#include "lanes.hpp"
#include "kernels.hpp"

namespace kgev {

namespace {

__global__ __launch_bounds__(256) void k_fill_zero(uint32_t* p, int64_t words)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < words; q += stride) p[q] = 0u;
}

template <typename R>
__global__ __launch_bounds__(256) void k_copy_lower_check(int64_t n, const double2* __restrict__ src, int64_t lds,
                                                          int64_t ss, cx<R>* __restrict__ dst, int64_t ldd,
                                                          int64_t sd, int* status)
{
    const int64_t b = blockIdx.z;
    const int64_t j = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool bad = false;
    if (i < n && i >= j) {
        const double2 v = src[b * ss + i + j * lds];
        bad = !isfinite(v.x) || !isfinite(v.y);
        if (dst) dst[b * sd + i + j * ldd] = mk<R>((R)v.x, (R)((i == j) ? 0.0 : v.y));
    }
    if (__any(bad) && (threadIdx.x & 63) == 0 && status) atomicOr(status + b, ST_NONFINITE);
}

// 32x32 tiles through LDS; tiles on or below the diagonal only
__global__ __launch_bounds__(256) void k_hermitian_full(int64_t n, const double2* __restrict__ src, int64_t lds,
                                                        int64_t ss, double2* __restrict__ dst, int64_t ldd, int64_t sd)
{
    __shared__ double2 T[32][33];
    const int64_t b = blockIdx.z;
    const int bi = blockIdx.x, bj = blockIdx.y;
    if (bi < bj) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int64_t i0 = (int64_t)bi * 32, j0 = (int64_t)bj * 32;
    const double2* S = src + b * ss;
    double2* D = dst + b * sd;
    for (int c = ty; c < 32; c += 8) {
        const int64_t i = i0 + tx, j = j0 + c;
        T[c][tx] = (i < n && j < n) ? S[i + j * lds] : czero<double2>();
    }
    __syncthreads();
    for (int c = ty; c < 32; c += 8) {
        // direct: D(i0+tx, j0+c)
        const int64_t i = i0 + tx, j = j0 + c;
        if (i < n && j < n) {
            double2 v;
            if (i > j) v = T[c][tx];
            else if (i == j) v = mk<double>(T[c][tx].x, 0.0);
            else v = cconj(T[tx][c]);      // diagonal tile only: (i, j) with i < j
            D[i + j * ldd] = v;
        }
        // mirrored: D(j0+tx, i0+c) = conj(S(i0+c, j0+tx)) for the strict lower tile
        if (bi != bj) {
            const int64_t i2 = j0 + tx, j2 = i0 + c;
            if (i2 < n && j2 < n) D[i2 + j2 * ldd] = cconj(T[tx][c]);
        }
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_real_to_complex(int64_t n, const double* __restrict__ src, int64_t ss,
                                                         cx<R>* __restrict__ dst, int64_t ldd, int64_t sd)
{
    const int64_t b = blockIdx.z;
    const int64_t j = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[b * sd + i + j * ldd] = mk<R>((R)src[b * ss + i + j * n], (R)0);
}

// one workgroup per column
// s (when given): the ascending eigenvalues of S; the largest of the
// problem's own is s[nreal[b] - 1] when nreal is given (an embedded problem
// whose padded directions sort last), else s[n - 1]
__global__ __launch_bounds__(256) void k_normalize_cols(int64_t n, double2* U, int64_t ldu, int64_t su, const double* s,
                                                       int64_t sst, double s_tol, int* status, int prune,
                                                       const int* nreal)
{
    __shared__ double sh[4];
    const int64_t b = blockIdx.y;
    const int64_t j = blockIdx.x;
    double2* u = U + b * su + j * ldu;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double2 v = u[i];
        acc = fma(v.x, v.x, fma(v.y, v.y, acc));
    }
    acc = dpp_wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    const double ss = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    double f = 1.0 / sqrt(ss);
    if (s) {
        const double sj = s[b * sst + j];
        const double smax = s[b * sst + (nreal ? nreal[b] : n) - 1];
        f = f / sqrt(sj);
        if (prune) {
            // a pruned direction: its column of X is zero
            if (!(sj > s_tol * smax)) f = 0.0;
        } else if (j == 0 && threadIdx.x == 0 && status) {
            if (!(sj > s_tol * smax)) atomicOr(status + b, ST_NOTPD);
        }
    }
    for (int64_t i = threadIdx.x; i < n; i += 256) u[i] = cscale(u[i], f);
}

// unit 2-norm columns of a real matrix (n x n, ld ldz, batch stride sz)
__global__ __launch_bounds__(256) void k_normalize_cols_real(int64_t n, double* Z, int64_t ldz, int64_t sz)
{
    __shared__ double sh[4];
    double* z = Z + (int64_t)blockIdx.y * sz + (int64_t)blockIdx.x * ldz;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc = fma(z[i], z[i], acc);
    acc = dpp_wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    const double f = 1.0 / sqrt((sh[0] + sh[1]) + (sh[2] + sh[3]));
    for (int64_t i = threadIdx.x; i < n; i += 256) z[i] *= f;
}

// T (kk x kk, upper) for reflectors c0..c0+kk-1 (compact WY):
// T(j, j) = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j), G = V_b^H V_b.
constexpr int KBMAX = 64;
// Step q of the T recurrence below, for one lane of row r's quad: acc[m]
// holds the running sum of column part + 4m.  q is a template argument so
// that acc stays in registers (every index into it is a constant).
template <int Q, typename R>
__device__ inline void larft_step(cx<R> (&acc)[KBMAX / 4], const cx<R> (*gl)[KBMAX + 1], const cx<R>* tl, int r,
                                  int part, bool store, cx<R>* Tb, int kb)
{
    const cx<R> tq = tl[Q];
    // in the lane with part == Q % 4, acc[Q / 4] is column Q's full sum
    cx<R> t = csel(r < Q, cscale(cmul(tq, acc[Q >> 2]), (R)-1), csel(r == Q, tq, czero<cx<R>>()));
    t.x = quad_bcast<Q & 3>(t.x);
    t.y = quad_bcast<Q & 3>(t.y);
    if (store) Tb[r + (int64_t)Q * kb] = t;
    // the columns j > Q (a column j <= Q of a lane's set is finished and no
    // longer read, so the first group holding a j > Q is the bound)
#pragma unroll
    for (int m = (Q < 3 ? 0 : (Q - 3) / 4 + 1); m < KBMAX / 4; ++m)
        acc[m] = cfma(t, gl[part + 4 * m][Q], acc[m]);
}
template <typename R, int... Q>
__device__ inline void larft_steps(std::integer_sequence<int, Q...>, int kk, cx<R> (&acc)[KBMAX / 4],
                                   const cx<R> (*gl)[KBMAX + 1], const cx<R>* tl, int r, int part, bool store,
                                   cx<R>* Tb, int kb)
{
    ((Q < kk ? (larft_step<Q, R>(acc, gl, tl, r, part, store, Tb, kb), 0) : 0), ...);
}
// T factors of every reflector block at once, one workgroup per (block,
// k-point): T_b (kk x kk, ld kb) from G_b = V_b^H V_b (ld kb).  Row r of T
// (T(r, j) = -tau_j sum_{q<j} T(r, q) G(q, j), T(r, r) = tau_r, zero below
// the diagonal) depends on row r alone; it is taken by the quad of lanes
// 4r .. 4r+3, lane p of which keeps the running sums of the columns
// j = p + 4m in registers.  Step q finishes T(r, q) in the lane that owns
// column q, broadcasts it over the quad and adds its term to every later
// column's sum (right-looking), so the serial chain per step is one complex
// product, one broadcast and one fused multiply-add, and no step waits for
// memory written by another.
template <typename R>
__global__ __launch_bounds__(256) void k_larft_all(int kb, int nref, const cx<R>* G, int64_t sG,
                                                   const cx<R>* tau, int64_t stau, cx<R>* T, int64_t strT)
{
    __shared__ cx<R> gl[KBMAX][KBMAX + 1];   // gl[col][row] = G(row, col)
    __shared__ cx<R> tl[KBMAX];
    const int blk = blockIdx.x;
    const int64_t b = blockIdx.y;
    const int c0 = blk * kb;
    const int kk = nref - c0 < kb ? nref - c0 : kb;
    const int tid = threadIdx.x, r = tid >> 2, part = tid & 3;
    const cx<R>* g = G + b * sG + (int64_t)blk * kb * kb;
    for (int e = tid; e < kk * kk; e += 256) {
        const int rr = e % kk, cc = e / kk;
        gl[cc][rr] = g[rr + (int64_t)cc * kb];
    }
    if (tid < kk) tl[tid] = tau[b * stau + c0 + tid];
    __syncthreads();
    cx<R> acc[KBMAX / 4];
#pragma unroll
    for (int m = 0; m < KBMAX / 4; ++m) acc[m] = czero<cx<R>>();
    cx<R>* Tb = T + b * strT + (int64_t)blk * kb * kb;
    larft_steps<R>(std::make_integer_sequence<int, KBMAX>{}, kk, acc, gl, tl, r, part, part == 0 && r < kk, Tb, kb);
}

}  // namespace

hipError_t fill_zero(hipStream_t st, void* p, size_t bytes)
{
    if (bytes == 0) return hipSuccess;
    const int64_t words = (int64_t)(bytes / 4);
    int64_t blocks = (words + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t*)p, words);
    return hipGetLastError();
}

hipError_t status_init(hipStream_t st, int* status, int64_t nk) { return fill_zero(st, status, sizeof(int) * nk); }

namespace {
// deterministic pseudo-random value in [-1, 1) from an index (splitmix64 finaliser)
__device__ inline double hash_unit(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

template <typename R>
__global__ __launch_bounds__(256) void k_fill_test(int64_t n, cx<R>* A, uint64_t seed)
{
    const int64_t b = blockIdx.z, j = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint64_t key = ((seed * 1315423911ull + (uint64_t)b) * 2654435761ull + (uint64_t)j) * 40503ull + (uint64_t)i;
    const double re = hash_unit(2 * key), im = (i == j) ? 0.0 : hash_unit(2 * key + 1);
    A[b * n * n + i + j * n] = mk<R>((R)re, (R)im);
}
}  // namespace

template <typename R>
hipError_t fill_test_matrix(hipStream_t st, int64_t n, cx<R>* A, int64_t nk, uint64_t seed)
{
    dim3 g((unsigned)((n + 255) / 256), (unsigned)n, (unsigned)nk);
    hipLaunchKernelGGL(k_fill_test<R>, g, dim3(256), 0, st, n, A, seed);
    return hipGetLastError();
}
template hipError_t fill_test_matrix<double>(hipStream_t, int64_t, double2*, int64_t, uint64_t);
template hipError_t fill_test_matrix<float>(hipStream_t, int64_t, float2*, int64_t, uint64_t);

namespace {
__global__ __launch_bounds__(256) void k_status_finish(const int* bits, int32_t* codes, int64_t nk)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nk) return;
    const int b = bits[q];
    codes[q] = (b & ST_NONFINITE) ? 3 : (b & ST_NOTPD) ? 1 : (b & ST_NOCONV) ? 2 : 0;
}
}  // namespace

hipError_t status_finish(hipStream_t st, const int* bits, int32_t* codes, int64_t nk)
{
    hipLaunchKernelGGL(k_status_finish, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, st, bits, codes, nk);
    return hipGetLastError();
}

template <typename R>
hipError_t copy_lower_check(hipStream_t st, int64_t n, const double2* src, int64_t lds, int64_t ss, cx<R>* dst,
                            int64_t ldd, int64_t sd, int* status, int64_t nk)
{
    dim3 g((unsigned)((n + 255) / 256), (unsigned)n, (unsigned)nk);
    hipLaunchKernelGGL(k_copy_lower_check<R>, g, dim3(256), 0, st, n, src, lds, ss, dst, ldd, sd, status);
    return hipGetLastError();
}

hipError_t hermitian_full(hipStream_t st, int64_t n, const double2* src, int64_t lds, int64_t ss, double2* dst,
                          int64_t ldd, int64_t sd, int64_t nk)
{
    const unsigned t = (unsigned)((n + 31) / 32);
    hipLaunchKernelGGL(k_hermitian_full, dim3(t, t, (unsigned)nk), dim3(256), 0, st, n, src, lds, ss, dst, ldd, sd);
    return hipGetLastError();
}

template <typename R>
hipError_t real_to_complex(hipStream_t st, int64_t n, const double* src, int64_t ss, cx<R>* dst, int64_t ldd,
                           int64_t sd, int64_t nk)
{
    dim3 g((unsigned)((n + 255) / 256), (unsigned)n, (unsigned)nk);
    hipLaunchKernelGGL(k_real_to_complex<R>, g, dim3(256), 0, st, n, src, ss, dst, ldd, sd);
    return hipGetLastError();
}

hipError_t normalize_cols(hipStream_t st, int64_t n, double2* U, int64_t ldu, int64_t su, const double* s, int64_t ss,
                          double s_tol, int* status, int64_t nk, int prune, const int* nreal)
{
    hipLaunchKernelGGL(k_normalize_cols, dim3((unsigned)n, (unsigned)nk), dim3(256), 0, st, n, U, ldu, su, s, ss,
                       s_tol, status, prune, nreal);
    return hipGetLastError();
}

hipError_t normalize_cols_real(hipStream_t st, int64_t n, double* Z, int64_t ldz, int64_t sz, int64_t nk)
{
    hipLaunchKernelGGL(k_normalize_cols_real, dim3((unsigned)n, (unsigned)nk), dim3(256), 0, st, n, Z, ldz, sz);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pruned canonical orthogonalisation.  The s_j <= s_tol s_max directions are
// the first ndrop columns of X (s ascending) and are zero there, so rows and
// columns 0..ndrop-1 of A = X^H H X are zero; their diagonal is set to
// big = 2 ||A||_F + 1, above the spectrum of the kept block, which sorts
// their eigenvalues last and leaves them decoupled.  At the end those
// eigenvalues become +inf and their eigenvector columns zero.
namespace {
__global__ __launch_bounds__(256) void k_prune_colnorm(int64_t n, const double2* A, int64_t sA, double* part)
{
    __shared__ double sh[4];
    const int64_t b = blockIdx.y, j = blockIdx.x;
    const double2* a = A + b * sA + j * n;
    double acc = 0.0;
    for (int64_t i = j + threadIdx.x; i < n; i += 256) {
        const double2 v = a[i];
        acc = fma(i > j ? 2.0 : 1.0, fma(v.x, v.x, v.y * v.y), acc);
    }
    acc = dpp_wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[b * n + j] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(256) void k_prune_shift(int64_t n, double2* A, int64_t sA, const double* part,
                                                     const double* s, int64_t sst, double s_tol, int* ndrop,
                                                     const int* nreal)
{
    __shared__ double sh[4];
    __shared__ int sc[4];
    const int64_t b = blockIdx.x;
    const double smax = s[b * sst + (nreal ? nreal[b] : n) - 1];
    double acc = 0.0;
    int cnt = 0;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        acc += part[b * n + j];
        cnt += !(s[b * sst + j] > s_tol * smax);
    }
    acc = dpp_wave_sum(acc);
    cnt = dpp_wave_sum(cnt);
    if ((threadIdx.x & 63) == 0) {
        sh[threadIdx.x >> 6] = acc;
        sc[threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    const double big = 2.0 * sqrt((sh[0] + sh[1]) + (sh[2] + sh[3])) + 1.0;
    const int nd = (sc[0] + sc[1]) + (sc[2] + sc[3]);
    for (int64_t j = threadIdx.x; j < nd; j += 256) A[b * sA + j + j * n] = mk<double>(big, 0.0);
    if (threadIdx.x == 0) ndrop[b] = nd;
}

__global__ __launch_bounds__(256) void k_prune_finish(int64_t n, double* w, double2* C, int64_t ldc, const int* ndrop)
{
    const int64_t b = blockIdx.y, j = blockIdx.x;
    if (j < n - ndrop[b]) return;
    if (threadIdx.x == 0) w[b * n + j] = INFINITY;
    if (C)
        for (int64_t i = threadIdx.x; i < n; i += 256) C[b * ldc * n + j * ldc + i] = mk<double>(0.0, 0.0);
}
}  // namespace

hipError_t prune_shift(hipStream_t st, int64_t n, double2* A, int64_t sA, double* part, const double* s, int64_t sst,
                       double s_tol, int* ndrop, int64_t nk, const int* nreal)
{
    hipLaunchKernelGGL(k_prune_colnorm, dim3((unsigned)n, (unsigned)nk), dim3(256), 0, st, n, A, sA, part);
    hipLaunchKernelGGL(k_prune_shift, dim3((unsigned)nk), dim3(256), 0, st, n, A, sA, part, s, sst, s_tol, ndrop,
                       nreal);
    return hipGetLastError();
}

hipError_t prune_finish(hipStream_t st, int64_t n, double* w, double2* C, int64_t ldc, const int* ndrop, int64_t nk)
{
    hipLaunchKernelGGL(k_prune_finish, dim3((unsigned)n, (unsigned)nk), dim3(256), 0, st, n, w, C, ldc, ndrop);
    return hipGetLastError();
}


template hipError_t copy_lower_check<double>(hipStream_t, int64_t, const double2*, int64_t, int64_t, double2*,
                                             int64_t, int64_t, int*, int64_t);
template hipError_t copy_lower_check<float>(hipStream_t, int64_t, const double2*, int64_t, int64_t, float2*,
                                            int64_t, int64_t, int*, int64_t);
template hipError_t real_to_complex<double>(hipStream_t, int64_t, const double*, int64_t, double2*, int64_t,
                                            int64_t, int64_t);
template hipError_t real_to_complex<float>(hipStream_t, int64_t, const double*, int64_t, float2*, int64_t,
                                           int64_t, int64_t);

// ---------------------------------------------------------------------------
// Back-transformation U <- Q U, Q = H_0 ... H_{n-2}, in blocks of 2 kb
// reflectors applied last block first as (I - V_B T_B V_B^H).
//   * The Gram matrices G_b = V_b^H V_b of the kb-blocks and their T factors
//     are formed first, one launch each: V is zero above each reflector, so
//     every full block's G_b can be taken over rows 1..n-1, which gives all
//     of them one stride.
//   * Pairs of kb-blocks are joined into 2kb-blocks,
//     T_B = [[T_1, -T_1 (V_1^H V_2) T_2], [0, T_2]] (three batched products),
//     so the two products that apply a block have 2kb rows / a 2kb inner
//     dimension.
int64_t unmtr_work_elems(int64_t n, int kb)
{
    const int64_t nblk = (n - 1 + kb - 1) / kb, npair = (nblk + 1) / 2;
    const int64_t kb2 = (int64_t)kb * kb;
    return nblk * kb2                 // G of the kb-blocks
           + nblk * kb2               // T of the kb-blocks
           + npair * 4 * kb2          // T of the 2kb-blocks
           + 2 * npair * kb2          // V_1^H V_2 and (V_1^H V_2) T_2 per pair
           + 2 * 2 * (int64_t)kb * n; // W1, W2 (2kb x n)
}

namespace {
// T_B of every pair: diagonal blocks copied from the kb-block factors, the
// lower-left block zeroed (the upper-right block is written by products)
template <typename R>
__global__ __launch_bounds__(256) void k_pair_t(int kb, int nblk, const cx<R>* T, int64_t sT, cx<R>* TB, int64_t sTB)
{
    const int q = blockIdx.x;
    const int64_t b = blockIdx.y;
    const int b1 = 2 * q, b2 = 2 * q + 1;
    const int64_t kb2 = (int64_t)kb * kb, ld = 2 * kb;
    cx<R>* t = TB + b * sTB + (int64_t)q * 4 * kb2;
    const cx<R>* t1 = T + b * sT + (int64_t)b1 * kb2;
    const cx<R>* t2 = T + b * sT + (int64_t)b2 * kb2;
    for (int e = threadIdx.x; e < kb * kb; e += 256) {
        const int r = e % kb, c = e / kb;
        t[r + (int64_t)c * ld] = t1[r + (int64_t)c * kb];
        t[(kb + r) + (int64_t)c * ld] = czero<cx<R>>();
        if (b2 < nblk) t[(kb + r) + (int64_t)(kb + c) * ld] = t2[r + (int64_t)c * kb];
    }
}
}  // namespace

template <typename R>
hipError_t unmtr(hipStream_t st, int64_t n, const cx<R>* V, int64_t sV, const cx<R>* tau, int64_t stau, cx<R>* U,
                 int64_t ldu, int64_t sU, cx<R>* work, int kb, int64_t nk, bool right)
{
    const int64_t nref = n - 1;
    if (nref <= 0) return hipSuccess;
    if (kb > KBMAX || kb < 1) return hipErrorInvalidValue;
    const int64_t sw = unmtr_work_elems(n, kb);
    const int64_t nblk = (nref + kb - 1) / kb, nfull = nref / kb, npair = (nblk + 1) / 2;
    const int64_t kb2 = (int64_t)kb * kb, ld2 = 2 * kb;
    cx<R>* G = work;
    cx<R>* T = G + nblk * kb2;
    cx<R>* TB = T + nblk * kb2;
    cx<R>* G12 = TB + npair * 4 * kb2;
    cx<R>* X12 = G12 + npair * kb2;
    cx<R>* W1 = X12 + npair * kb2;
    cx<R>* W2 = W1 + 2 * (int64_t)kb * n;
    const cx<R> one = mk<R>(1, 0), zero = mk<R>(0, 0), mone = mk<R>(-1, 0);
    hipError_t e;
    // Gram matrices and T factors of the kb-blocks
    if (nfull > 0) {
        e = cgemm_batch2<R>(st, 'C', 'N', kb, kb, n - 1, one, V + 1, n, sV, kb * n, V + 1, n, sV, kb * n, zero, G, kb,
                            sw, kb2, nk, nfull);
        if (e != hipSuccess) return e;
    }
    if (nfull < nblk) {
        const int64_t c0 = nfull * kb;
        const int kk = (int)(nref - c0);
        const int64_t r0 = c0 + 1, m = n - r0;
        const cx<R>* Vb = V + r0 + c0 * n;
        e = cgemm<R>(st, 'C', 'N', kk, kk, m, one, Vb, n, sV, Vb, n, sV, zero, G + nfull * kb2, kb, sw, nk, false);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_larft_all<R>, dim3((unsigned)nblk, (unsigned)nk), dim3(256), 0, st, kb, (int)nref, G, sw,
                       tau, stau, T, sw);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // T of the 2kb-blocks: diagonal blocks, then T12 = -T_1 (V_1^H V_2) T_2
    hipLaunchKernelGGL(k_pair_t<R>, dim3((unsigned)npair, (unsigned)nk), dim3(256), 0, st, kb, (int)nblk, T, sw, TB,
                       sw);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nfp = nfull / 2;               // pairs of two full kb-blocks
    if (nfp > 0) {
        e = cgemm_batch2<R>(st, 'C', 'N', kb, kb, n - 1, one, V + 1, n, sV, 2 * kb * n, V + 1 + kb * n, n, sV,
                            2 * kb * n, zero, G12, kb, sw, kb2, nk, nfp);
        if (e != hipSuccess) return e;
        e = cgemm_batch2<R>(st, 'N', 'N', kb, kb, kb, one, G12, kb, sw, kb2, T + kb2, kb, sw, 2 * kb2, zero, X12, kb,
                            sw, kb2, nk, nfp);
        if (e != hipSuccess) return e;
        e = cgemm_batch2<R>(st, 'N', 'N', kb, kb, kb, mone, T, kb, sw, 2 * kb2, X12, kb, sw, kb2, zero, TB + kb * ld2,
                            ld2, sw, 4 * kb2, nk, nfp);
        if (e != hipSuccess) return e;
    }
    if (nfp < npair && 2 * nfp + 1 < nblk) {
        // last pair with a partial second block
        const int64_t q = nfp, c1 = 2 * q * kb, c2 = c1 + kb;
        const int kk2 = (int)(nref - c2);
        e = cgemm<R>(st, 'C', 'N', kb, kk2, n - 1, one, V + 1 + c1 * n, n, sV, V + 1 + c2 * n, n, sV, zero,
                     G12 + q * kb2, kb, sw, nk, false);
        if (e != hipSuccess) return e;
        e = cgemm<R>(st, 'N', 'N', kb, kk2, kk2, one, G12 + q * kb2, kb, sw, T + (2 * q + 1) * kb2, kb, sw, zero,
                     X12 + q * kb2, kb, sw, nk, false);
        if (e != hipSuccess) return e;
        e = cgemm<R>(st, 'N', 'N', kb, kk2, kb, mone, T + 2 * q * kb2, kb, sw, X12 + q * kb2, kb, sw, zero,
                     TB + q * 4 * kb2 + kb * ld2, ld2, sw, nk, false);
        if (e != hipSuccess) return e;
    }
    if (right) {
        // U <- U Q = U B_0 B_1 ..., B_q = I - V_q T_q V_q^H: first block first
        for (int64_t q = 0; q < npair; ++q) {
            const int64_t c0 = 2 * q * kb;
            const int kk = (int)((nref - c0) < 2 * kb ? (nref - c0) : 2 * kb);
            const int64_t r0 = c0 + 1, m = n - r0;
            const cx<R>* Vb = V + r0 + c0 * n;
            // W1 = U(:, r0:n) V_q (n x kk), W2 = W1 T_q, U(:, r0:n) -= W2 V_q^H
            e = cgemm<R>(st, 'N', 'N', n, kk, m, one, U + r0 * ldu, ldu, sU, Vb, n, sV, zero, W1, n, sw, nk, false);
            if (e != hipSuccess) return e;
            e = cgemm<R>(st, 'N', 'N', n, kk, kk, one, W1, n, sw, TB + q * 4 * kb2, ld2, sw, zero, W2, n, sw, nk,
                         false);
            if (e != hipSuccess) return e;
            e = cgemm<R>(st, 'N', 'C', n, m, kk, mone, W2, n, sw, Vb, n, sV, one, U + r0 * ldu, ldu, sU, nk, false);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    // apply the 2kb-blocks, last first
    for (int64_t q = npair - 1; q >= 0; --q) {
        const int64_t c0 = 2 * q * kb;
        const int kk = (int)((nref - c0) < 2 * kb ? (nref - c0) : 2 * kb);
        const int64_t r0 = c0 + 1, m = n - r0;
        const cx<R>* Vb = V + r0 + c0 * n;
        e = cgemm<R>(st, 'C', 'N', kk, n, m, one, Vb, n, sV, U + r0, ldu, sU, zero, W1, kk, sw, nk, false);
        if (e != hipSuccess) return e;
        e = cgemm<R>(st, 'N', 'N', kk, n, kk, one, TB + q * 4 * kb2, ld2, sw, W1, kk, sw, zero, W2, kk, sw, nk, false);
        if (e != hipSuccess) return e;
        e = cgemm<R>(st, 'N', 'N', m, n, kk, mone, Vb, n, sV, W2, kk, sw, one, U + r0, ldu, sU, nk, false);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t unmtr<double>(hipStream_t, int64_t, const double2*, int64_t, const double2*, int64_t, double2*,
                                  int64_t, int64_t, double2*, int, int64_t, bool);
template hipError_t unmtr<float>(hipStream_t, int64_t, const float2*, int64_t, const float2*, int64_t, float2*,
                                 int64_t, int64_t, float2*, int, int64_t, bool);

}  // namespace kgev
