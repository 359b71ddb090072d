// Batched complex matrix products on MFMA (the ZGEMMs of Parts 3 and 4 of
// Band_DFT_Col, the rank-2k trailing update of the blocked Householder
// reduction and the compact-WY back-transformation), plus the real product
// with column gathers/scatters used by the divide-and-conquer merges.
//
// Complex product: C = alpha * sum_s op(A_s) op(B_s) + beta * C with one or
// two terms s (two terms give the Hermitian rank-2k update V W^H + W V^H in
// one pass).  A complex tile product is four real MFMA products on planar
// (re, im) LDS tiles; op(A) = A^H is folded into the global->LDS copy.
#include "common.hpp"
#include "kernels.hpp"

namespace kgev {

namespace {

constexpr int GB_M = 64;   // workgroup tile rows
constexpr int GB_N = 64;   // workgroup tile cols
constexpr int GB_K = 16;   // K step per LDS stage
constexpr int G_THREADS = 256;

template <typename R>
struct CGemmArgs {
    int64_t m, n, k;
    int nseg;
    const cx<R>* A[2];
    const cx<R>* B[2];
    int64_t lda[2], ldb[2], sA[2], sB[2];
    int ta[2], tb[2];
    cx<R> alpha, beta;
    cx<R>* C;
    int64_t ldc, sC;
    int lower;
    int tiles_m;
    const int* dm;     // optional device-side sizes per batch entry (m, n, k) x batch; may be null
};

// global -> registers: this thread's 4 elements of the op(A) tile (GB_M x GB_K)
template <typename R>
__device__ inline void load_a(const cx<R>* __restrict__ A, int64_t lda, int ta, int64_t m, int64_t K,
                              int64_t i0, int64_t k0, int tid, cx<R> (&ra)[4])
{
    if (ta == 0) {
        const int r = tid & 63, kq = tid >> 6;
        const int64_t gi = i0 + r;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t gk = k0 + kq + 4 * q;
            ra[q] = (gi < m && gk < K) ? A[gi + gk * lda] : czero<cx<R>>();
        }
    } else {
        const int kk = tid & 15, rq = tid >> 4;
        const int64_t gk = k0 + kk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t gi = i0 + rq + 16 * q;
            ra[q] = (gi < m && gk < K) ? cconj(A[gk + gi * lda]) : czero<cx<R>>();
        }
    }
}

template <typename R>
__device__ inline void store_a(R (*sr)[GB_M + 1], R (*si)[GB_M + 1], int ta, int tid, const cx<R> (&ra)[4])
{
    if (ta == 0) {
        const int r = tid & 63, kq = tid >> 6;
#pragma unroll
        for (int q = 0; q < 4; ++q) { sr[kq + 4 * q][r] = ra[q].x; si[kq + 4 * q][r] = ra[q].y; }
    } else {
        const int kk = tid & 15, rq = tid >> 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) { sr[kk][rq + 16 * q] = ra[q].x; si[kk][rq + 16 * q] = ra[q].y; }
    }
}

// op(B) tile (GB_K x GB_N)
template <typename R>
__device__ inline void load_b(const cx<R>* __restrict__ B, int64_t ldb, int tb, int64_t n, int64_t K,
                              int64_t j0, int64_t k0, int tid, cx<R> (&rb)[4])
{
    if (tb == 0) {
        const int kk = tid & 15, jq = tid >> 4;
        const int64_t gk = k0 + kk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t gj = j0 + jq + 16 * q;
            rb[q] = (gj < n && gk < K) ? B[gk + gj * ldb] : czero<cx<R>>();
        }
    } else {
        const int j = tid & 63, kq = tid >> 6;
        const int64_t gj = j0 + j;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t gk = k0 + kq + 4 * q;
            rb[q] = (gj < n && gk < K) ? cconj(B[gj + gk * ldb]) : czero<cx<R>>();
        }
    }
}

template <typename R>
__device__ inline void store_b(R (*sr)[GB_N + 1], R (*si)[GB_N + 1], int tb, int tid, const cx<R> (&rb)[4])
{
    if (tb == 0) {
        const int kk = tid & 15, jq = tid >> 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) { sr[kk][jq + 16 * q] = rb[q].x; si[kk][jq + 16 * q] = rb[q].y; }
    } else {
        const int j = tid & 63, kq = tid >> 6;
#pragma unroll
        for (int q = 0; q < 4; ++q) { sr[kq + 4 * q][j] = rb[q].x; si[kq + 4 * q][j] = rb[q].y; }
    }
}

template <typename R>
__global__ __launch_bounds__(G_THREADS) void cgemm_kernel(CGemmArgs<R> p)
{
    using M = Mfma<R>;
    using acc_t = typename M::acc_t;
    __shared__ R sAr[2][GB_K][GB_M + 1], sAi[2][GB_K][GB_M + 1];
    __shared__ R sBr[2][GB_K][GB_N + 1], sBi[2][GB_K][GB_N + 1];

    const int64_t bz = blockIdx.z;
    const int64_t m = p.m, n = p.n, K = p.k;
    const int tm = blockIdx.x % p.tiles_m, tn = blockIdx.x / p.tiles_m;
    const int64_t i0 = (int64_t)tm * GB_M, j0 = (int64_t)tn * GB_N;
    if (i0 >= m || j0 >= n) return;
    if (p.lower && i0 + GB_M <= j0) return;   // tile entirely above the diagonal

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int li = lane & 15, lk = lane >> 4;

    acc_t accR[2][2], accI[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) { accR[a][b][r] = 0; accI[a][b][r] = 0; }

    const int nkt = (int)((K + GB_K - 1) / GB_K);
    const int total = nkt * p.nseg;
    cx<R> ra[4], rb[4];
    int cur = 0;
    if (total > 0) {
        load_a<R>(p.A[0] + bz * p.sA[0], p.lda[0], p.ta[0], m, K, i0, 0, tid, ra);
        load_b<R>(p.B[0] + bz * p.sB[0], p.ldb[0], p.tb[0], n, K, j0, 0, tid, rb);
        store_a<R>(sAr[0], sAi[0], p.ta[0], tid, ra);
        store_b<R>(sBr[0], sBi[0], p.tb[0], tid, rb);
    }
    __syncthreads();
    for (int it = 0; it < total; ++it) {
        const int nx = it + 1;
        const int sgn = nx / nkt, kt = nx % nkt;
        if (nx < total) {
            load_a<R>(p.A[sgn] + bz * p.sA[sgn], p.lda[sgn], p.ta[sgn], m, K, i0, (int64_t)kt * GB_K, tid, ra);
            load_b<R>(p.B[sgn] + bz * p.sB[sgn], p.ldb[sgn], p.tb[sgn], n, K, j0, (int64_t)kt * GB_K, tid, rb);
        }
#pragma unroll
        for (int ks = 0; ks < GB_K; ks += 4) {
            R ar[2], ai[2], br[2], bi[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                ar[t] = sAr[cur][ks + lk][wm * 32 + t * 16 + li];
                ai[t] = sAi[cur][ks + lk][wm * 32 + t * 16 + li];
                br[t] = sBr[cur][ks + lk][wn * 32 + t * 16 + li];
                bi[t] = sBi[cur][ks + lk][wn * 32 + t * 16 + li];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    accR[a][b] = M::mma(ar[a], br[b], accR[a][b]);
                    accR[a][b] = M::mma(-ai[a], bi[b], accR[a][b]);
                    accI[a][b] = M::mma(ar[a], bi[b], accI[a][b]);
                    accI[a][b] = M::mma(ai[a], br[b], accI[a][b]);
                }
        }
        if (nx < total) {
            store_a<R>(sAr[cur ^ 1], sAi[cur ^ 1], p.ta[sgn], tid, ra);
            store_b<R>(sBr[cur ^ 1], sBi[cur ^ 1], p.tb[sgn], tid, rb);
        }
        __syncthreads();
        cur ^= 1;
    }

    cx<R>* C = p.C + bz * p.sC;
    const bool rb0 = (p.beta.x != 0 || p.beta.y != 0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + wm * 32 + a * 16 + M::row(lk, r);
                const int64_t j = j0 + wn * 32 + b * 16 + li;
                if (i < m && j < n && (!p.lower || i >= j)) {
                    cx<R> v = mk<R>(accR[a][b][r], accI[a][b][r]);
                    cx<R> out = cmul(p.alpha, v);
                    if (rb0) out = cfma(p.beta, C[i + j * p.ldc], out);
                    C[i + j * p.ldc] = out;
                }
            }
}

template <typename R>
hipError_t launch_cgemm(const CGemmArgs<R>& a, int64_t batch, hipStream_t st)
{
    if (a.m <= 0 || a.n <= 0 || batch <= 0) return hipSuccess;
    CGemmArgs<R> p = a;
    p.tiles_m = (int)((a.m + GB_M - 1) / GB_M);
    const int64_t tiles_n = (a.n + GB_N - 1) / GB_N;
    dim3 grid((unsigned)(p.tiles_m * tiles_n), 1, (unsigned)batch);
    double flops = 8.0 * (double)a.m * (double)a.n * (double)a.k * (double)a.nseg * (double)batch;
    if (a.lower) flops *= 0.5;
    prof_before(PH_GEMM, st);
    hipLaunchKernelGGL(cgemm_kernel<R>, grid, dim3(G_THREADS), 0, st, p);
    prof_after(PH_GEMM, st, 0.0, flops);
    return hipGetLastError();
}

}  // namespace

template <typename R>
hipError_t cgemm(hipStream_t st, char ta, char tb, int64_t m, int64_t n, int64_t k, cx<R> alpha,
                 const cx<R>* A, int64_t lda, int64_t sA, const cx<R>* B, int64_t ldb, int64_t sB,
                 cx<R> beta, cx<R>* C, int64_t ldc, int64_t sC, int64_t batch, bool lower)
{
    CGemmArgs<R> a{};
    a.m = m; a.n = n; a.k = k; a.nseg = 1;
    a.A[0] = A; a.B[0] = B; a.lda[0] = lda; a.ldb[0] = ldb; a.sA[0] = sA; a.sB[0] = sB;
    a.ta[0] = (ta == 'C'); a.tb[0] = (tb == 'C');
    a.A[1] = A; a.B[1] = B; a.lda[1] = lda; a.ldb[1] = ldb; a.sA[1] = sA; a.sB[1] = sB;
    a.ta[1] = a.ta[0]; a.tb[1] = a.tb[0];
    a.alpha = alpha; a.beta = beta; a.C = C; a.ldc = ldc; a.sC = sC; a.lower = lower ? 1 : 0;
    return launch_cgemm<R>(a, batch, st);
}

template <typename R>
hipError_t cher2k_lower(hipStream_t st, int64_t m, int64_t k, const cx<R>* V, int64_t ldv, int64_t sV,
                        const cx<R>* W, int64_t ldw, int64_t sW, cx<R>* C, int64_t ldc, int64_t sC,
                        int64_t batch)
{
    // C(lower) -= V W^H + W V^H
    CGemmArgs<R> a{};
    a.m = m; a.n = m; a.k = k; a.nseg = 2;
    a.A[0] = V; a.lda[0] = ldv; a.sA[0] = sV; a.ta[0] = 0;
    a.B[0] = W; a.ldb[0] = ldw; a.sB[0] = sW; a.tb[0] = 1;
    a.A[1] = W; a.lda[1] = ldw; a.sA[1] = sW; a.ta[1] = 0;
    a.B[1] = V; a.ldb[1] = ldv; a.sB[1] = sV; a.tb[1] = 1;
    a.alpha = mk<R>(-1, 0); a.beta = mk<R>(1, 0);
    a.C = C; a.ldc = ldc; a.sC = sC; a.lower = 1;
    return launch_cgemm<R>(a, batch, st);
}

template hipError_t cgemm<double>(hipStream_t, char, char, int64_t, int64_t, int64_t, double2,
                                  const double2*, int64_t, int64_t, const double2*, int64_t, int64_t,
                                  double2, double2*, int64_t, int64_t, int64_t, bool);
template hipError_t cgemm<float>(hipStream_t, char, char, int64_t, int64_t, int64_t, float2,
                                 const float2*, int64_t, int64_t, const float2*, int64_t, int64_t,
                                 float2, float2*, int64_t, int64_t, int64_t, bool);
template hipError_t cher2k_lower<double>(hipStream_t, int64_t, int64_t, const double2*, int64_t, int64_t,
                                         const double2*, int64_t, int64_t, double2*, int64_t, int64_t,
                                         int64_t);
template hipError_t cher2k_lower<float>(hipStream_t, int64_t, int64_t, const float2*, int64_t, int64_t,
                                        const float2*, int64_t, int64_t, float2*, int64_t, int64_t,
                                        int64_t);

}  // namespace kgev
