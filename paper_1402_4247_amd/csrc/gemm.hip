// Batched complex matrix products on MFMA (the ZGEMMs of Parts 3 and 4 of
// Band_DFT_Col, the rank-2k trailing update of the blocked Householder
// reduction and the compact-WY back-transformation), plus the real product
// with column gathers/scatters used by the divide-and-conquer merges.
//
// Complex product: C = alpha * sum_s op(A_s) op(B_s) + beta * C with one or
// two terms s (two terms give the Hermitian rank-2k update V W^H + W V^H in
// one pass).  A complex tile product is formed from real MFMA products on
// planar (re, im) LDS tiles, either the four products of the definition or
// the three of the Gauss (3M) form, re = ar br - ai bi and
// im = (ar + ai)(br + bi) - ar br - ai bi, which saves a quarter of the MFMA
// work at a normwise (not componentwise) error bound of the same order;
// op(A) = A^H is folded into the global->LDS copy.
#include "common.hpp"
#include "kernels.hpp"

namespace kgev {

namespace {

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
    int tiles_m, tiles_n;
    int64_t batch;             // total products = batch1 * batch2
    int64_t batch2;            // inner batch: product L -> (L / batch2, L % batch2)
    int64_t sA2[2], sB2[2], sC2;   // strides of the inner batch index
    int remap;
    int tri;                   // enumerate only the tiles on or below the diagonal
};

// Work item of this workgroup.  Consecutive workgroups are dispatched round
// robin over the 8 XCDs, so the 1-D id is remapped to give each XCD a
// contiguous range of tiles (one L2 sees neighbouring tiles); inside a
// problem tiles go in groups of 4 tile-rows so the tiles running together
// share A row panels and B column panels.  A lower-triangle product of a
// square C (tri) launches only the tiles on or below the diagonal, taken
// row by row (row tm holds tiles 0..tm, starting at tm (tm + 1) / 2).
__device__ inline void tile_of(int64_t L, int64_t total, int tiles_m, int tiles_n, int remap, int tri, int64_t& b,
                               int& tm, int& tn)
{
    const int64_t logical = (remap && total % 8 == 0) ? (L % 8) * (total / 8) + L / 8 : L;
    if (tri) {
        const int64_t T = (int64_t)tiles_m * (tiles_m + 1) / 2;
        b = logical / T;
        const int64_t t = logical % T;
        int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while (r > 0 && (int64_t)r * (r + 1) / 2 > t) --r;
        while ((int64_t)(r + 1) * (r + 2) / 2 <= t) ++r;
        tm = r;
        tn = (int)(t - (int64_t)r * (r + 1) / 2);
        return;
    }
    const int64_t T = (int64_t)tiles_m * tiles_n;
    b = logical / T;
    const int t = (int)(logical % T);
    const int g = t / (4 * tiles_n);
    const int rows_g = min(4, tiles_m - 4 * g);
    const int local = t - 4 * g * tiles_n;
    tm = 4 * g + local % rows_g;
    tn = local / rows_g;
}

// global -> registers: this thread's elements of the op(A) tile (BM x GB_K).
// The loads come from clamped (in-bounds) addresses with no branch, so they
// stay in flight across the MFMA work of the current step; the bounds mask
// and the conjugation of op = ^H are applied when the registers are stored
// to LDS.
template <typename R, int BM, int TA>
__device__ inline void load_a(const cx<R>* __restrict__ A, int64_t lda, int64_t m, int64_t K, int64_t i0,
                              int64_t k0, int tid, cx<R> (&ra)[BM * GB_K / G_THREADS], unsigned& okmask)
{
    constexpr int NE = BM * GB_K / G_THREADS;
    okmask = 0;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int e = tid + G_THREADS * q;
        const int r = TA ? e / GB_K : e % BM;
        const int kk = TA ? e % GB_K : e / BM;
        const int64_t gi = i0 + r, gk = k0 + kk;
        const bool ok = gi < m && gk < K;
        const int64_t gic = gi < m ? gi : m - 1, gkc = gk < K ? gk : K - 1;
        ra[q] = TA ? A[gkc + gic * lda] : A[gic + gkc * lda];
        okmask |= (unsigned)ok << q;
    }
}

template <typename R, int BM, int TA>
__device__ inline void store_a(R (*sr)[BM + 1], R (*si)[BM + 1], int tid, const cx<R> (&ra)[BM * GB_K / G_THREADS],
                               unsigned okmask)
{
    constexpr int NE = BM * GB_K / G_THREADS;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int e = tid + G_THREADS * q;
        const int r = TA ? e / GB_K : e % BM;
        const int kk = TA ? e % GB_K : e / BM;
        const bool ok = (okmask >> q) & 1u;
        sr[kk][r] = ok ? ra[q].x : (R)0;
        si[kk][r] = ok ? (TA ? -ra[q].y : ra[q].y) : (R)0;
    }
}

// op(B) tile (GB_K x BN)
template <typename R, int BN, int TB>
__device__ inline void load_b(const cx<R>* __restrict__ B, int64_t ldb, int64_t n, int64_t K, int64_t j0,
                              int64_t k0, int tid, cx<R> (&rb)[BN * GB_K / G_THREADS], unsigned& okmask)
{
    constexpr int NE = BN * GB_K / G_THREADS;
    okmask = 0;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int e = tid + G_THREADS * q;
        const int c = TB == 1 ? e % BN : e / GB_K;
        const int kk = TB == 1 ? e / BN : e % GB_K;
        const int64_t gj = j0 + c, gk = k0 + kk;
        const bool ok = gj < n && gk < K;
        const int64_t gjc = gj < n ? gj : n - 1, gkc = gk < K ? gk : K - 1;
        if constexpr (TB == 2)
            rb[q] = mk<R>(reinterpret_cast<const R*>(B)[gkc + gjc * ldb], (R)0);
        else
            rb[q] = TB ? B[gjc + gkc * ldb] : B[gkc + gjc * ldb];
        okmask |= (unsigned)ok << q;
    }
}

template <typename R, int BN, int TB>
__device__ inline void store_b(R (*sr)[BN + 1], R (*si)[BN + 1], int tid, const cx<R> (&rb)[BN * GB_K / G_THREADS],
                               unsigned okmask)
{
    constexpr int NE = BN * GB_K / G_THREADS;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int e = tid + G_THREADS * q;
        const int c = TB == 1 ? e % BN : e / GB_K;
        const int kk = TB == 1 ? e / BN : e % GB_K;
        const bool ok = (okmask >> q) & 1u;
        sr[kk][c] = ok ? rb[q].x : (R)0;
        if constexpr (TB != 2) si[kk][c] = ok ? (TB ? -rb[q].y : rb[q].y) : (R)0;
    }
}

// BM x BN workgroup tile, four waves in a 2 x 2 arrangement, each owning a
// (BM/2) x (BN/2) block of 16 x 16 MFMA tiles.  While one K step is
// multiplied out of LDS, the next is fetched into registers; two LDS stages,
// the registers go to the other stage, one barrier per K step.
template <typename R, int BM, int BN, bool G3, int TA, int TB>
__global__ __launch_bounds__(G_THREADS, 2) void cgemm_kernel(CGemmArgs<R> p)
{
    using M = Mfma<R>;
    using acc_t = typename M::acc_t;
    constexpr int TM = BM / 32, TN = BN / 32;      // MFMA tiles per wave
    __shared__ R sAr[2][GB_K][BM + 1], sAi[2][GB_K][BM + 1];
    __shared__ R sBr[2][GB_K][BN + 1], sBi[2][GB_K][BN + 1];

    const int64_t total = (p.tri ? (int64_t)p.tiles_m * (p.tiles_m + 1) / 2 : (int64_t)p.tiles_m * p.tiles_n) * p.batch;
    int64_t bz;
    int tm, tn;
    tile_of(blockIdx.x, total, p.tiles_m, p.tiles_n, p.remap, p.tri, bz, tm, tn);
    const int64_t bo = bz / p.batch2, bi = bz - bo * p.batch2;
    const int64_t m = p.m, n = p.n, K = p.k;
    const int64_t i0 = (int64_t)tm * BM, j0 = (int64_t)tn * BN;
    if (p.lower && i0 + BM <= j0) return;   // tile entirely above the diagonal

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int li = lane & 15, lk = lane >> 4;

    // 4M: accR = re, accI = im.  3M: accR = sum ar br, accI = sum (ar+ai)(br+bi),
    // accT = sum ai bi.
    acc_t accR[TM][TN], accI[TM][TN], accT[G3 ? TM : 1][G3 ? TN : 1];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                accR[a][b][r] = 0;
                accI[a][b][r] = 0;
                if constexpr (G3) accT[a][b][r] = 0;
            }

    // operand B of term s (strides in real elements when B is real)
    auto bbase = [&](int sg) -> const cx<R>* {
        if constexpr (TB == 2)
            return reinterpret_cast<const cx<R>*>(reinterpret_cast<const R*>(p.B[sg]) + bo * p.sB[sg] +
                                                  bi * p.sB2[sg]);
        else
            return p.B[sg] + bo * p.sB[sg] + bi * p.sB2[sg];
    };
    const int nkt = (int)((K + GB_K - 1) / GB_K);
    const int total_k = nkt * p.nseg;
    cx<R> ra[BM * GB_K / G_THREADS], rb[BN * GB_K / G_THREADS];
    unsigned oka = 0, okb = 0;
    int cur = 0;
    if (total_k > 0) {
        load_a<R, BM, TA>(p.A[0] + bo * p.sA[0] + bi * p.sA2[0], p.lda[0], m, K, i0, 0, tid, ra, oka);
        load_b<R, BN, TB>(bbase(0), p.ldb[0], n, K, j0, 0, tid, rb, okb);
        store_a<R, BM, TA>(sAr[0], sAi[0], tid, ra, oka);
        store_b<R, BN, TB>(sBr[0], sBi[0], tid, rb, okb);
    }
    __syncthreads();
    for (int it = 0; it < total_k; ++it) {
        const int nx = it + 1;
        const int sn = nx / nkt, kt = nx % nkt;
        if (nx < total_k) {
            load_a<R, BM, TA>(p.A[sn] + bo * p.sA[sn] + bi * p.sA2[sn], p.lda[sn], m, K, i0, (int64_t)kt * GB_K, tid,
                              ra, oka);
            load_b<R, BN, TB>(bbase(sn), p.ldb[sn], n, K, j0, (int64_t)kt * GB_K, tid,
                              rb, okb);
        }
#pragma unroll
        for (int ks = 0; ks < GB_K; ks += 4) {
            R ar[TM], ai[TM], br[TN], bi[TN];
#pragma unroll
            for (int t = 0; t < TM; ++t) {
                ar[t] = sAr[cur][ks + lk][wm * (BM / 2) + t * 16 + li];
                ai[t] = sAi[cur][ks + lk][wm * (BM / 2) + t * 16 + li];
            }
#pragma unroll
            for (int t = 0; t < TN; ++t) {
                br[t] = sBr[cur][ks + lk][wn * (BN / 2) + t * 16 + li];
                bi[t] = TB == 2 ? (R)0 : sBi[cur][ks + lk][wn * (BN / 2) + t * 16 + li];
            }
            if constexpr (TB == 2) {
                // real B: two real products
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < TN; ++b) {
                        accR[a][b] = M::mma(ar[a], br[b], accR[a][b]);
                        accI[a][b] = M::mma(ai[a], br[b], accI[a][b]);
                    }
            } else if constexpr (G3) {
                R bs[TN];
#pragma unroll
                for (int t = 0; t < TN; ++t) bs[t] = br[t] + bi[t];
#pragma unroll
                for (int a = 0; a < TM; ++a) {
                    const R as = ar[a] + ai[a];
#pragma unroll
                    for (int b = 0; b < TN; ++b) {
                        accR[a][b] = M::mma(ar[a], br[b], accR[a][b]);
                        accI[a][b] = M::mma(as, bs[b], accI[a][b]);
                        accT[a][b] = M::mma(ai[a], bi[b], accT[a][b]);
                    }
                }
            } else {
#pragma unroll
                for (int a = 0; a < TM; ++a) {
                    const R nai = -ai[a];
#pragma unroll
                    for (int b = 0; b < TN; ++b) {
                        accR[a][b] = M::mma(ar[a], br[b], accR[a][b]);
                        accR[a][b] = M::mma(nai, bi[b], accR[a][b]);
                        accI[a][b] = M::mma(ar[a], bi[b], accI[a][b]);
                        accI[a][b] = M::mma(ai[a], br[b], accI[a][b]);
                    }
                }
            }
        }
        if (nx < total_k) {
            const int nxt = cur ^ 1;
            store_a<R, BM, TA>(sAr[nxt], sAi[nxt], tid, ra, oka);
            store_b<R, BN, TB>(sBr[nxt], sBi[nxt], tid, rb, okb);
        }
        __syncthreads();
        cur ^= 1;
    }

    cx<R>* C = p.C + bo * p.sC + bi * p.sC2;
    const bool rb0 = (p.beta.x != 0 || p.beta.y != 0);
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + wm * (BM / 2) + a * 16 + M::row(lk, r);
                const int64_t j = j0 + wn * (BN / 2) + b * 16 + li;
                if (i < m && j < n && (!p.lower || i >= j)) {
                    cx<R> v;
                    if constexpr (G3) {
                        const R pr = accR[a][b][r], qi = accT[a][b][r];
                        v = mk<R>(pr - qi, accI[a][b][r] - pr - qi);
                    } else {
                        v = mk<R>(accR[a][b][r], accI[a][b][r]);
                    }
                    cx<R> out = cmul(p.alpha, v);
                    if (rb0) out = cfma(p.beta, C[i + j * p.ldc], out);
                    C[i + j * p.ldc] = out;
                }
            }
}

template <typename R, int BM, int BN, bool G3, int TA, int TB>
hipError_t launch_tiles(CGemmArgs<R> p, hipStream_t st, const ProfLaunch& pl)
{
    p.tiles_m = (int)((p.m + BM - 1) / BM);
    p.tiles_n = (int)((p.n + BN - 1) / BN);
    p.tri = (p.lower && BM == BN && p.tiles_m == p.tiles_n) ? 1 : 0;
    const int64_t total = (p.tri ? (int64_t)p.tiles_m * (p.tiles_m + 1) / 2 : (int64_t)p.tiles_m * p.tiles_n) * p.batch;
    launch_timed(pl, cgemm_kernel<R, BM, BN, G3, TA, TB>, dim3((unsigned)total), dim3(G_THREADS), st, p);
    return hipGetLastError();
}

// the operand forms are compile-time so that the tile loads are straight-line
template <typename R, bool G3, int T>
hipError_t launch_forms(const CGemmArgs<R>& p, hipStream_t st, const ProfLaunch& pl)
{
    if (p.tb[0] == 2) return launch_tiles<R, T, T, false, 0, 2>(p, st, pl);
    const int f = p.ta[0] * 2 + p.tb[0];
    switch (f) {
    case 0: return launch_tiles<R, T, T, G3, 0, 0>(p, st, pl);
    case 1: return launch_tiles<R, T, T, G3, 0, 1>(p, st, pl);
    case 2: return launch_tiles<R, T, T, G3, 1, 0>(p, st, pl);
    default: return launch_tiles<R, T, T, G3, 1, 1>(p, st, pl);
    }
}

// Products whose 64 x 64 grid would launch fewer workgroups than this take
// 32 x 32 tiles (four times the workgroups, each a quarter of the work): set
// per calling thread by the solve entry points from their options.
thread_local int tl_small_tile_slots = GEMM_SMALL_SLOTS_DEFAULT;

template <typename R>
hipError_t launch_cgemm(const CGemmArgs<R>& a, int64_t batch, hipStream_t st)
{
    if (a.m <= 0 || a.n <= 0 || batch <= 0) return hipSuccess;
    CGemmArgs<R> p = a;
    if (p.batch2 < 1) p.batch2 = 1;
    p.batch = batch * p.batch2;
    double flops = 8.0 * (double)a.m * (double)a.n * (double)a.k * (double)a.nseg * (double)batch *
                   (double)(a.batch2 < 1 ? 1 : a.batch2);
    if (a.lower) flops *= 0.5;
    if (a.tb[0] == 2) flops *= 0.5;   // complex times real: 4 real flops per term
    // Tiles are remapped so each XCD sees a contiguous range; complex tile
    // products in the 3M form (1.22x the four-product form on gfx950 on the
    // path's products, with unchanged residuals).
    p.remap = 1;
    const int64_t tm = (p.m + 63) / 64, tn = (p.n + 63) / 64;
    const int64_t grid64 = (p.lower && tm == tn ? tm * (tm + 1) / 2 : tm * tn) * p.batch;
    const ProfLaunch pl = prof_launch_begin(PH_GEMM, st);
    const hipError_t e = grid64 < tl_small_tile_slots ? launch_forms<R, true, 32>(p, st, pl)
                                                      : launch_forms<R, true, 64>(p, st, pl);
    prof_launch_end(PH_GEMM, st, pl, 0.0, flops);
    return e;
}

}  // namespace

int gemm_small_tile_slots(int slots)
{
    const int old = tl_small_tile_slots;
    tl_small_tile_slots = slots;
    return old;
}

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
hipError_t cgemm_batch2(hipStream_t st, char ta, char tb, int64_t m, int64_t n, int64_t k, cx<R> alpha,
                        const cx<R>* A, int64_t lda, int64_t sA, int64_t sA2, const cx<R>* B, int64_t ldb, int64_t sB,
                        int64_t sB2, cx<R> beta, cx<R>* C, int64_t ldc, int64_t sC, int64_t sC2, int64_t batch,
                        int64_t batch2)
{
    CGemmArgs<R> a{};
    a.m = m; a.n = n; a.k = k; a.nseg = 1;
    a.A[0] = a.A[1] = A; a.B[0] = a.B[1] = B;
    a.lda[0] = a.lda[1] = lda; a.ldb[0] = a.ldb[1] = ldb;
    a.sA[0] = a.sA[1] = sA; a.sB[0] = a.sB[1] = sB;
    a.sA2[0] = a.sA2[1] = sA2; a.sB2[0] = a.sB2[1] = sB2;
    a.ta[0] = a.ta[1] = (ta == 'C'); a.tb[0] = a.tb[1] = (tb == 'C');
    a.alpha = alpha; a.beta = beta; a.C = C; a.ldc = ldc; a.sC = sC; a.sC2 = sC2; a.lower = 0;
    a.batch2 = batch2;
    return launch_cgemm<R>(a, batch, st);
}

template <typename R>
hipError_t cgemm_rb(hipStream_t st, int64_t m, int64_t n, int64_t k, const cx<R>* A, int64_t lda, int64_t sA,
                    const R* B, int64_t ldb, int64_t sB, cx<R>* C, int64_t ldc, int64_t sC, int64_t batch)
{
    // C = A B with B real (ldb, sB in real elements)
    CGemmArgs<R> a{};
    a.m = m; a.n = n; a.k = k; a.nseg = 1;
    a.A[0] = a.A[1] = A; a.lda[0] = a.lda[1] = lda; a.sA[0] = a.sA[1] = sA; a.ta[0] = a.ta[1] = 0;
    a.B[0] = a.B[1] = reinterpret_cast<const cx<R>*>(B);
    a.ldb[0] = a.ldb[1] = ldb; a.sB[0] = a.sB[1] = sB; a.tb[0] = a.tb[1] = 2;
    a.alpha = mk<R>(1, 0); a.beta = mk<R>(0, 0);
    a.C = C; a.ldc = ldc; a.sC = sC; a.lower = 0;
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
template hipError_t cgemm_batch2<double>(hipStream_t, char, char, int64_t, int64_t, int64_t, double2,
                                         const double2*, int64_t, int64_t, int64_t, const double2*, int64_t,
                                         int64_t, int64_t, double2, double2*, int64_t, int64_t, int64_t, int64_t,
                                         int64_t);
template hipError_t cgemm_batch2<float>(hipStream_t, char, char, int64_t, int64_t, int64_t, float2, const float2*,
                                        int64_t, int64_t, int64_t, const float2*, int64_t, int64_t, int64_t, float2,
                                        float2*, int64_t, int64_t, int64_t, int64_t, int64_t);
template hipError_t cgemm_rb<double>(hipStream_t, int64_t, int64_t, int64_t, const double2*, int64_t, int64_t,
                                     const double*, int64_t, int64_t, double2*, int64_t, int64_t, int64_t);
template hipError_t cher2k_lower<double>(hipStream_t, int64_t, int64_t, const double2*, int64_t, int64_t,
                                         const double2*, int64_t, int64_t, double2*, int64_t, int64_t,
                                         int64_t);
template hipError_t cher2k_lower<float>(hipStream_t, int64_t, int64_t, const float2*, int64_t, int64_t,
                                        const float2*, int64_t, int64_t, float2*, int64_t, int64_t,
                                        int64_t);

}  // namespace kgev
