// Blocked Householder tridiagonalisation of a batch of Hermitian matrices
// (lower storage): Section III, Procedures 1-6 of Eigen_HH, arXiv:1402.4247,
// reorganised in panels of nb columns.
//
// Per column i of a panel starting at p (j = i - p, o = i + 1), two kernels:
//   zhemv  : one chunk of the Hermitian product z = A22 u (Procedure 4) from
//       the lower triangle only, with u the column below the sub-diagonal as
//       it stands (u_o = 0, u_r = A(r, i)), plus the chunk's share of
//       q = Re(u^H z).  It needs nothing derived in this step, so the
//       workgroups only stream their tiles.
//   update : every workgroup derives the reflector (Procedure 2, stable sign,
//       real beta) from the partial norms, v = (1, scale * A(o+1:n, i)), and
//       forms for its rows y = tau (A22(:, o) + scale z - V (W^H v) - W (V^H v))
//       (A22 v = A22(:, o) + scale A22 u by linearity) and
//       w = y - (tau/2)(y^H v) v (Procedure 5).  y^H v needs no reduction over
//       y: with h = A22(:, o), v^H A22 v = h_o + 2 Re(scale z_o) + |scale|^2 q
//       and y^H v = conj(tau) (v^H A22 v - 2 Re((V^H v)^H (W^H v))), so
//       alpha2 = -(tau/2) y^H v = -|tau|^2 / 2 (...) is real and every
//       workgroup computes it, and row o of w, from the same partials.
//       Then the next column of the panel is brought up to date,
//       A(o:n, o) -= V(o:n, 0:j) conj(W(o, 0:j))^T + W(o:n, 0:j) conj(V(o, 0:j))^T,
//       and its squared norm below the sub-diagonal and its products with
//       the panel columns (the pieces of W^H v and V^H v for the next
//       reflector, taken on the unscaled column) are reduced in per-block
//       partials.
// After the panel the trailing matrix takes the rank-2nb update
// A22 -= V W^H + W V^H (Procedure 6, on MFMA).
// Once a panel's trailing matrix has at most 128 rows, the rest of the
// reduction runs in one launch, unblocked, with the matrix in LDS (tail).
// No atomics: every sum is taken in a fixed order, so results are bitwise
// reproducible run to run.
#include <type_traits>

#include "common.hpp"
#include "lanes.hpp"
#include "kernels.hpp"

namespace kgev {

// 32-bit raw buffer load (the 64- and 128-bit forms are in common.hpp)
__device__ int raw_buffer_load_i32(i4_t rsrc, int voffset, int soffset, int aux) __asm("llvm.amdgcn.raw.buffer.load.i32");

namespace {

constexpr int ZT = 64;          // ZHEMV tile edge
constexpr int ZCH = 4;          // tiles per ZHEMV chunk: one per wave of the workgroup
constexpr int RB = 64;          // rows per workgroup in the column kernels

// chunks of block column C in the four-tile form, and in the form a
// reduction uses (ws.zch: 4 tiles per chunk, or 1 for the one-tile form)
__device__ __host__ inline int nchunks(int NB, int C) { return (NB - C + ZCH - 1) / ZCH; }
__device__ __host__ inline int nchunks_z(int NB, int C, int zch) { return zch == 1 ? NB - C : (NB - C + 3) >> 2; }

// Procedure 2's reflector for the sub-column x = (alpha, x_2, ...) with
// sig2 = |x_2|^2 + ...: beta = -sign(Re alpha) ||x||, tau = (beta - alpha) /
// beta and the scale 1 / (alpha - beta) applied to x_2, ...; two reciprocals
// (the latency of a division chain dominates this single-lane step).
template <typename R>
__device__ inline void reflector_core(cx<R> alpha, R sig2, cx<R>& tau, cx<R>& scale, R& beta)
{
    if (sig2 == (R)0 && alpha.y == (R)0) {
        tau = czero<cx<R>>();
        scale = czero<cx<R>>();
        beta = alpha.x;
        return;
    }
    const R nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sig2);
    beta = (alpha.x >= (R)0) ? -nrm : nrm;
    const R ib = (R)1 / beta;
    tau = mk<R>((beta - alpha.x) * ib, -alpha.y * ib);
    const R dr = alpha.x - beta, di = alpha.y;
    const R iden = (R)1 / (dr * dr + di * di);
    scale = mk<R>(dr * iden, -di * iden);
}

// Partial norms of column i: lane q takes the per-block partials q, q + 64,
// ... (pn_first: the first of them, requested with the kernel's first batch
// of loads; pn_rest: the sum, in that order).
template <typename R>
__device__ inline const R* pnorm_base(const HetrdWs<R>& ws, int64_t b, int i)
{
    return ws.pnorm + b * ws.s_pnorm + (i & 1) * ((ws.n + RB - 1) / RB);
}
template <typename R>
__device__ inline R pn_first(const HetrdWs<R>& ws, int64_t b, int i, int lane)
{
    const int np = (ws.n - i + RB - 1) / RB;
    return pnorm_base(ws, b, i)[lane < np ? lane : 0];
}
template <typename R>
__device__ inline R pn_rest(const HetrdWs<R>& ws, int64_t b, int i, int lane, R first)
{
    const int np = (ws.n - i + RB - 1) / RB;
    const R* pn = pnorm_base(ws, b, i);
    R part = lane < np ? first : (R)0;
    for (int q = lane + 64; q < np; q += 64) part += pn[q];
    return part;
}

// LDS written by a wave and then read by other lanes of the same wave: a
// wave-scope fence and a scheduling barrier, no workgroup barrier
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One halving step of the transposing reduction: lanes with the MASK bit set
// keep values HALF..2HALF-1 (moved down to 0..HALF-1), the others keep
// 0..HALF-1; each adds its partner's copy of the values it keeps.  Across
// rows (MASK 16, 32) a permlane swap of the pair (t[q], t[q + HALF]) leaves
// both addends in place; within a row the sent value is selected and moved
// by DPP.
template <int MASK, int HALF, int NV, typename R>
__device__ __attribute__((always_inline)) inline void halve_step(cx<R> (&t)[NV], bool up)
{
#pragma unroll
    for (int q = 0; q < HALF; ++q) {
        if constexpr (MASK >= 16) {
            cx<R> a = t[q], c = t[q + HALF];
            swap_across<MASK>(a.x, c.x);
            swap_across<MASK>(a.y, c.y);
            t[q] = cadd(a, c);
        } else {
            const cx<R> send = csel(up, t[q], t[q + HALF]);
            const cx<R> keep = csel(up, t[q + HALF], t[q]);
            cx<R> rcv;
            rcv.x = lane_xor<MASK>(send.x);
            rcv.y = lane_xor<MASK>(send.y);
            t[q] = cadd(keep, rcv);
        }
    }
}

// r + r(lane ^ MASK), as vector-ALU lane exchanges
template <int MASK, typename R>
__device__ __attribute__((always_inline)) inline cx<R> xor_add_v(cx<R> r)
{
    r.x = xor_sum<MASK>(r.x);
    r.y = xor_sum<MASK>(r.y);
    return r;
}

// 8 complex values per lane -> lane l holds the sum over the wave of value
// (l >> 3) & 7 (three halving steps over lane bits 5..3, then plain xor sums
// over bits 2..0).
template <typename R>
__device__ __attribute__((always_inline)) inline cx<R> transpose_sum8(cx<R> (&t)[8], int lane)
{
    halve_step<32, 4, 8, R>(t, (lane & 32) != 0);
    halve_step<16, 2, 8, R>(t, (lane & 16) != 0);
    halve_step<8, 1, 8, R>(t, (lane & 8) != 0);
    cx<R> r = t[0];
    r = xor_add_v<4, R>(r);
    r = xor_add_v<2, R>(r);
    r = xor_add_v<1, R>(r);
    return r;
}

// ---------------------------------------------------------------------------
// First column of a panel: d_c and partial norms of rows c+2..n-1.
template <typename R>
__global__ __launch_bounds__(RB) void hetrd_colstart(HetrdWs<R> ws, int c)
{
    const int64_t b = blockIdx.y;
    const int64_t r = (int64_t)c + (int64_t)blockIdx.x * RB + threadIdx.x;
    R acc = 0;
    if (r < ws.n) {
        const cx<R> a = ws.A[b * ws.sA + r + (int64_t)c * ws.lda];
        if (r == c) ws.d[b * ws.n + c] = a.x;
        if (r >= c + 2) acc = a.x * a.x + a.y * a.y;
    }
    acc = dpp_wave_sum(acc);
    if (threadIdx.x == 0) ws.pnorm[b * ws.s_pnorm + (c & 1) * ((ws.n + RB - 1) / RB) + blockIdx.x] = acc;
}

// ---------------------------------------------------------------------------
// One chunk of z = A22 u.  A chunk is up to four 64x64 tiles (R0..R0+3, C) of
// one block column of the lower triangle; wave w owns tile R0 + w whole: the
// direct part z_R += A_RC u_C comes out complete per row, the transposed part
// z_C += A_RC^H u_R per column.  Each group of 8 columns is multiplied, its
// products go to the wave's LDS block, the next group is requested into the
// same registers, and the column sums are taken from LDS while it is in
// flight; the four waves' column sums are added once.  Three workgroups per
// CU.
template <typename R, bool BUF>
__global__ __launch_bounds__(256, 3) void hetrd_zhemv(HetrdWs<R> ws, int i, int rev)
{
    __shared__ cx<R> svC[ZCH][ZT];
    __shared__ cx<R> sT[ZCH][ZT];
    __shared__ cx<R> sP[ZCH][8][ZT + 1];      // per-wave staging of one group's products
    // rev: the workgroups take the chunks in reverse order (last k-point's
    // last chunk first), so that a launch after a forward one starts on the
    // tiles its predecessor read last
    const int64_t b = rev ? (int64_t)(gridDim.y - 1 - blockIdx.y) : (int64_t)blockIdx.y;
    const int lid = rev ? (int)(gridDim.x - 1 - blockIdx.x) : (int)blockIdx.x;
    const int n = ws.n;
    const int o = i + 1;
    const int m = n - o;
    const int NB = (m + ZT - 1) / ZT;

    // which (block column C, chunk ch) is ours
    int bid = lid, C = 0;
    for (; C < NB; ++C) {
        const int nc = nchunks(NB, C);
        if (bid < nc) break;
        bid -= nc;
    }
    if (C >= NB) return;
    const int ch = bid;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const cx<R>* A = ws.A + b * ws.sA;
    const cx<R>* Ai = A + (int64_t)i * ws.lda;
    const int64_t lda = ws.lda;
    const int Rb = C + ch * ZCH + w;
    const bool have_tile = Rb < NB;
    const int64_t gr = (int64_t)o + (int64_t)(have_tile ? Rb : C) * ZT + lane;
    const bool row_ok = gr < n;
    // Loads are unconditional from a clamped (in-bounds) address and the value
    // is masked afterwards, so no branch guards them.
    // Matrices under 2 GiB are read with buffer loads: one 32-bit row offset
    // per lane shared by every load of the tile, the column offset in a
    // scalar register (fewer vector registers and no 64-bit address
    // arithmetic); larger ones with plain global loads.
    const int rowc = row_ok ? (int)gr : n - 1;
    const int64_t gcb = (int64_t)o + (int64_t)C * ZT;
    const i4_t rsrc = buffer_rsrc(A, (uint32_t)(BUF ? (int64_t)sizeof(cx<R>) * lda * n : 0));
    auto load_one = [&](int g, int cc) -> cx<R> {
        const int64_t gc = gcb + g * 8 + cc;
        const int64_t gcc = gc < n ? gc : (int64_t)n - 1;
        if constexpr (BUF) {
            const int soff = (int)(gcc * lda * (int64_t)sizeof(cx<R>));
            if constexpr (sizeof(R) == 8)
                return __builtin_bit_cast(cx<R>, raw_buffer_load_v4i32(rsrc, rowc * (int)sizeof(cx<R>), soff, 0));
            else
                return __builtin_bit_cast(cx<R>, raw_buffer_load_v2i32(rsrc, rowc * (int)sizeof(cx<R>), soff, 0));
        } else {
            return A[gcc * lda + rowc];
        }
    };
    auto load_group = [&](int g, cx<R> (&a)[8]) {
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) a[cc] = load_one(g, cc);
    };
    // u first, then the first column group; each wave keeps its own copy of
    // u_C in LDS, so the waves do not wait for each other before the products
    const int64_t gcu = gcb + lane;
    const cx<R> uC = Ai[gcu < n ? gcu : (int64_t)n - 1];
    cx<R> uR = Ai[row_ok ? gr : (int64_t)n - 1];
    cx<R> a[8];
    load_group(0, a);
    svC[w][lane] = csel(gcu > o && gcu < n, uC, czero<cx<R>>());
    if (!(row_ok && gr > o)) uR = czero<cx<R>>();
    wave_sync();

    __shared__ R sq[ZCH];
    R qd = 0;
    if (have_tile) {
        const bool diag_tile = (Rb == C);
        cx<R> yd = czero<cx<R>>();
        // one group of 8 columns; NEXT: the next group's columns are requested
        // as this group's registers free up (the last group has none to fetch)
        auto group = [&](int g, auto next) {
            constexpr bool NEXT = decltype(next)::value;
            const int64_t gc0 = gcb + g * 8;
#pragma unroll
            for (int cc = 0; cc < 8; ++cc) {
                const int64_t gc = gc0 + cc;
                const bool ok = row_ok && gc < n && (!diag_tile || gr >= gc);
                const bool diag = diag_tile && (gr == gc);
                cx<R> x;
                x.x = ok ? a[cc].x : (R)0;
                x.y = (ok && !diag) ? a[cc].y : (R)0;
                yd = cfma(x, svC[w][g * 8 + cc], yd);
                // the diagonal entry is counted once (direct part only)
                sP[w][cc][lane] = csel(diag, czero<cx<R>>(), cmulc(x, uR));
                // the column's register is free: request the next group's
                // column at once, so that group streams in while this one is
                // still being multiplied out
                if constexpr (NEXT) a[cc] = load_one(g + 1, cc);
            }
            // the products are in this wave's LDS block; the column sums are
            // taken from LDS while the next group is in flight: lane l adds
            // rows 8 (l / 8) .. +7 of column l mod 8, then the eight lanes of
            // a column combine
            __builtin_amdgcn_wave_barrier();
            const int c = lane & 7, r0 = (lane >> 3) * 8;
            cx<R> cs = czero<cx<R>>();
#pragma unroll
            for (int r = 0; r < 8; ++r) cs = cadd(cs, sP[w][c][r0 + r]);
            cs = xor_add_v<8, R>(cs);
            cs = xor_add_v<16, R>(cs);
            cs = xor_add_v<32, R>(cs);
            if (lane < 8) sT[w][g * 8 + lane] = cs;
            __builtin_amdgcn_wave_barrier();
        };
#pragma unroll 1
        for (int g = 0; g < 7; ++g) group(g, std::true_type{});
        group(7, std::false_type{});
        ws.ypart[b * ws.s_ypart + ((int64_t)Rb * ws.NBmax + C) * ZT + lane] = yd;
        qd = uR.x * yd.x + uR.y * yd.y;
    } else {
        sT[w][lane] = czero<cx<R>>();
    }
    qd = dpp_wave_sum(qd);
    if (lane == 0) sq[w] = qd;
    __syncthreads();
    if (tid < ZT) {
        const cx<R> s = cadd(cadd(sT[0][tid], sT[1][tid]), cadd(sT[2][tid], sT[3][tid]));
        ws.ypartT[b * ws.s_ypartT + ((int64_t)C * ws.CHmax + ch) * ZT + tid] = s;
        R qt = svC[0][tid].x * s.x + svC[0][tid].y * s.y;
        qt = dpp_wave_sum(qt);
        if (tid == 0) ws.qpart[b * ws.s_qpart + lid] = ((sq[0] + sq[1]) + (sq[2] + sq[3])) + qt;
    }
}

// The same product in one-tile chunks, for launches where the four-tile form
// would give fewer workgroups than three per CU (few k-points): the four
// waves share one tile, wave w taking column groups 2w and 2w + 1; their
// direct parts are added in LDS, and each column's sum comes from the one
// wave that owns it.  Same partial-sum layout with one chunk per tile.
template <typename R, bool BUF>
__global__ __launch_bounds__(256, 3) void hetrd_zhemv_tile(HetrdWs<R> ws, int i, int rev)
{
    __shared__ cx<R> svC[ZCH][ZT];
    __shared__ cx<R> sT[ZCH][ZT];
    __shared__ cx<R> sP[ZCH][8][ZT + 1];
    const int64_t b = rev ? (int64_t)(gridDim.y - 1 - blockIdx.y) : (int64_t)blockIdx.y;
    const int lid = rev ? (int)(gridDim.x - 1 - blockIdx.x) : (int)blockIdx.x;
    const int n = ws.n;
    const int o = i + 1;
    const int m = n - o;
    const int NB = (m + ZT - 1) / ZT;
    // which tile (Rb, C) of the lower triangle is ours: tiles enumerated down
    // each block column
    int bid = lid, C = 0;
    for (; C < NB; ++C) {
        const int nc = NB - C;
        if (bid < nc) break;
        bid -= nc;
    }
    if (C >= NB) return;
    const int ch = bid;
    const int Rb = C + ch;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const cx<R>* A = ws.A + b * ws.sA;
    const cx<R>* Ai = A + (int64_t)i * ws.lda;
    const int64_t lda = ws.lda;
    const int64_t gr = (int64_t)o + (int64_t)Rb * ZT + lane;
    const bool row_ok = gr < n;
    const int rowc = row_ok ? (int)gr : n - 1;
    const int64_t gcb = (int64_t)o + (int64_t)C * ZT;
    const i4_t rsrc = buffer_rsrc(A, (uint32_t)(BUF ? (int64_t)sizeof(cx<R>) * lda * n : 0));
    auto load_one = [&](int g, int cc) -> cx<R> {
        const int64_t gc = gcb + g * 8 + cc;
        const int64_t gcc = gc < n ? gc : (int64_t)n - 1;
        if constexpr (BUF) {
            const int soff = (int)(gcc * lda * (int64_t)sizeof(cx<R>));
            if constexpr (sizeof(R) == 8)
                return __builtin_bit_cast(cx<R>, raw_buffer_load_v4i32(rsrc, rowc * (int)sizeof(cx<R>), soff, 0));
            else
                return __builtin_bit_cast(cx<R>, raw_buffer_load_v2i32(rsrc, rowc * (int)sizeof(cx<R>), soff, 0));
        } else {
            return A[gcc * lda + rowc];
        }
    };
    // u first, then the wave's first column group (the second group's columns
    // are requested as the first group's registers free up).  Each wave keeps
    // its own copy of u in LDS, so the waves do not wait for each other before
    // the products.
    const int64_t gcu = gcb + lane;
    const cx<R> uC = Ai[gcu < n ? gcu : (int64_t)n - 1];
    cx<R> uR = Ai[row_ok ? gr : (int64_t)n - 1];
    const int g0 = 2 * w;
    cx<R> a[8];
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) a[cc] = load_one(g0, cc);
    sT[w][lane] = czero<cx<R>>();      // the other waves' columns add zero
    // (every wave stores its own copy: a store in one wave only would let the
    // compiler move the load of u behind the tile's)
    svC[w][lane] = csel(gcu > o && gcu < n, uC, czero<cx<R>>());
    if (!(row_ok && gr > o)) uR = czero<cx<R>>();
    wave_sync();

    __shared__ R sq[ZCH];
    const bool diag_tile = (Rb == C);
    cx<R> yd = czero<cx<R>>();
    auto group = [&](int g, auto next) {
        constexpr bool NEXT = decltype(next)::value;
        const int64_t gc0 = gcb + g * 8;
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
            const int64_t gc = gc0 + cc;
            const bool ok = row_ok && gc < n && (!diag_tile || gr >= gc);
            const bool diag = diag_tile && (gr == gc);
            cx<R> x;
            x.x = ok ? a[cc].x : (R)0;
            x.y = (ok && !diag) ? a[cc].y : (R)0;
            yd = cfma(x, svC[w][g * 8 + cc], yd);
            sP[w][cc][lane] = csel(diag, czero<cx<R>>(), cmulc(x, uR));
            if constexpr (NEXT) a[cc] = load_one(g + 1, cc);
        }
        __builtin_amdgcn_wave_barrier();
        const int c = lane & 7, r0 = (lane >> 3) * 8;
        cx<R> cs = czero<cx<R>>();
#pragma unroll
        for (int r = 0; r < 8; ++r) cs = cadd(cs, sP[w][c][r0 + r]);
        cs = xor_add_v<8, R>(cs);
        cs = xor_add_v<16, R>(cs);
        cs = xor_add_v<32, R>(cs);
        if (lane < 8) sT[w][g * 8 + lane] = cs;
        __builtin_amdgcn_wave_barrier();
    };
    group(g0, std::true_type{});
    group(g0 + 1, std::false_type{});
    // the four waves' shares of the tile's direct part
    sP[w][0][lane] = yd;
    R qd = uR.x * yd.x + uR.y * yd.y;
    qd = dpp_wave_sum(qd);
    if (lane == 0) sq[w] = qd;
    __syncthreads();
    if (w == 0) {
        const cx<R> ys = cadd(cadd(sP[0][0][lane], sP[1][0][lane]), cadd(sP[2][0][lane], sP[3][0][lane]));
        ws.ypart[b * ws.s_ypart + ((int64_t)Rb * ws.NBmax + C) * ZT + lane] = ys;
        const cx<R> s = cadd(cadd(sT[0][lane], sT[1][lane]), cadd(sT[2][lane], sT[3][lane]));
        ws.ypartT[b * ws.s_ypartT + ((int64_t)C * ws.CHmax + ch) * ZT + lane] = s;
        R qt = svC[0][lane].x * s.x + svC[0][lane].y * s.y;
        qt = dpp_wave_sum(qt);
        if (lane == 0) ws.qpart[b * ws.s_qpart + lid] = ((sq[0] + sq[1]) + (sq[2] + sq[3])) + qt;
    }
}

// ---------------------------------------------------------------------------
// Partial sums read as buffer loads: an offset at or beyond the buffer's size
// returns 0, so a term that does not exist is read at OOB and added as 0, and
// every batch is loaded and added whole, without selects.
constexpr int OOB = 0x20000000;

// A descriptor built from workgroup-uniform values, pinned to scalar
// registers (64-bit offset arithmetic can leave it in vector registers, and a
// buffer load from those would loop over the lanes' distinct descriptors).
__device__ inline i4_t uniform_rsrc(const void* base, uint32_t bytes)
{
    i4_t r = buffer_rsrc(base, bytes);
    r.x = __builtin_amdgcn_readfirstlane(r.x);
    r.y = __builtin_amdgcn_readfirstlane(r.y);
    r.z = __builtin_amdgcn_readfirstlane(r.z);
    r.w = __builtin_amdgcn_readfirstlane(r.w);
    return r;
}

template <typename R>
__device__ inline R bload_r(i4_t rsrc, int voff)
{
    if constexpr (sizeof(R) == 8)
        return __builtin_bit_cast(R, raw_buffer_load_v2i32(rsrc, voff, 0, 0));
    else
        return __builtin_bit_cast(R, raw_buffer_load_i32(rsrc, voff, 0, 0));
}

template <typename R>
__device__ inline cx<R> bload(i4_t rsrc, int voff)
{
    if constexpr (sizeof(R) == 8)
        return __builtin_bit_cast(cx<R>, raw_buffer_load_v4i32(rsrc, voff, 0, 0));
    else
        return __builtin_bit_cast(cx<R>, raw_buffer_load_v2i32(rsrc, voff, 0, 0));
}

// z at one row: the partial sums over the block columns and chunks that
// touch it, split over the four waves (wave w takes the terms with index =
// w mod 4) and combined as (w0 + w1) + (w2 + w3).  A wave's terms are the
// block columns C = w, w + 4, ... <= Rb (per-block partials) and the chunks
// ch = w, w + 4, ... < nc (per-chunk partials); term t of each list goes to
// the first of two running sums if t is even, to the second if odd.  The
// first ZB terms of both lists are requested together (one memory round trip
// at n = 2000), longer lists load the rest as they are summed.
constexpr int ZB = 8;

template <typename R>
struct ZTerms {
    i4_t rp, rq;          // block row Rb's per-block and per-chunk partials
    int w, tp, tq, roff;  // wave (uniform), term counts, row offset in bytes
    __device__ ZTerms(const HetrdWs<R>& ws, int64_t b, int Rb, int NB, int r, int w_) : w(w_)
    {
        rp = uniform_rsrc(ws.ypart + b * ws.s_ypart + (int64_t)Rb * ws.NBmax * ZT,
                         (uint32_t)((int64_t)ws.NBmax * ZT * (int64_t)sizeof(cx<R>)));
        rq = uniform_rsrc(ws.ypartT + b * ws.s_ypartT + (int64_t)Rb * ws.CHmax * ZT,
                         (uint32_t)((int64_t)ws.CHmax * ZT * (int64_t)sizeof(cx<R>)));
        const int nc = nchunks_z(NB, Rb, ws.zch);
        tp = Rb >= w ? (Rb - w) / 4 + 1 : 0;
        tq = nc > w ? (nc - 1 - w) / 4 + 1 : 0;
        roff = r * (int)sizeof(cx<R>);
    }
    __device__ int off(int t, int tn) const
    {
        return (t < tn ? (w + 4 * t) * ZT * (int)sizeof(cx<R>) : OOB) + roff;
    }
    __device__ void load(int t0, cx<R> (&vp)[ZB], cx<R> (&vq)[ZB]) const
    {
#pragma unroll
        for (int t = 0; t < ZB; ++t) {
            vp[t] = bload<R>(rp, off(t0 + t, tp));
            vq[t] = bload<R>(rq, off(t0 + t, tq));
        }
    }
    // the whole sum, given the first batches (overwritten)
    __device__ cx<R> sum(cx<R> (&vp)[ZB], cx<R> (&vq)[ZB]) const
    {
        cx<R> y0 = czero<cx<R>>(), y1 = czero<cx<R>>();
#pragma unroll
        for (int t = 0; t < ZB; t += 2) {
            y0 = cadd(y0, vp[t]);
            y1 = cadd(y1, vp[t + 1]);
        }
        for (int t0 = ZB; t0 < tp; t0 += ZB) {
#pragma unroll
            for (int t = 0; t < ZB; ++t) vp[t] = bload<R>(rp, off(t0 + t, tp));
#pragma unroll
            for (int t = 0; t < ZB; t += 2) {
                y0 = cadd(y0, vp[t]);
                y1 = cadd(y1, vp[t + 1]);
            }
        }
#pragma unroll
        for (int t = 0; t < ZB; t += 2) {
            y0 = cadd(y0, vq[t]);
            y1 = cadd(y1, vq[t + 1]);
        }
        for (int t0 = ZB; t0 < tq; t0 += ZB) {
#pragma unroll
            for (int t = 0; t < ZB; ++t) vq[t] = bload<R>(rq, off(t0 + t, tq));
#pragma unroll
            for (int t = 0; t < ZB; t += 2) {
                y0 = cadd(y0, vq[t]);
                y1 = cadd(y1, vq[t + 1]);
            }
        }
        return cadd(y0, y1);
    }
};

// z at row o (row 0 of block 0), needed by every workgroup: the 1 + nc terms
// (block column 0, then the chunks of block row 0) spread over the lanes of
// one wave and summed by a fixed lane tree, so every workgroup holds the same
// bits.  z0_first is the lane's first term, requested with the kernel's first
// batch of loads; z0_rest adds the others (lane + 64, ...).
template <typename R>
__device__ inline cx<R> z0_first(const HetrdWs<R>& ws, int64_t b, int NB, int lane)
{
    const int T = 1 + nchunks_z(NB, 0, ws.zch);
    return lane == 0 ? ws.ypart[b * ws.s_ypart] : ws.ypartT[b * ws.s_ypartT + (int64_t)(lane < T ? lane - 1 : 0) * ZT];
}
template <typename R>
__device__ inline cx<R> z0_rest(const HetrdWs<R>& ws, int64_t b, int NB, int lane, cx<R> first)
{
    const cx<R>* yq = ws.ypartT + b * ws.s_ypartT;
    const int T = 1 + nchunks_z(NB, 0, ws.zch);
    cx<R> acc = csel(lane < T, first, czero<cx<R>>());
    for (int s = lane + 64; s < T; s += 64) acc = cadd(acc, yq[(int64_t)(s - 1) * ZT]);
    return acc;
}

template <typename C>
__device__ inline C sum4(const C (&s)[4][64], int l)
{
    return cadd(cadd(s[0][l], s[1][l]), cadd(s[2][l], s[3][l]));
}

// Column i: reflector, v and w for one 64-row block (rows o + 64 Rb ...),
// then (update_next) column o brought up to date for these rows with its
// partial norm and partial panel dots.  Every global value the block needs
// is requested in one first phase, including this thread's rows of the panel
// columns V(:, p + jj), W(:, jj) (the four waves take jj = w, w+4, ...; panels
// up to 32 wide are held in registers, wider ones reload the rest), which
// then serve the corrections, the column update and the panel dots.  Every
// wave forms the panel dots, the row-o scalars and v, w of the block itself,
// so the launch has three workgroup barriers: after the loads, after the
// corrections and after the column update.
template <typename R>
__global__ __launch_bounds__(256) void hetrd_update(HetrdWs<R> ws, int i, int p, int update_next, int nch)
{
    __shared__ cx<R> s1[4][64], s2[4][64], sy[4][64], sco[4][64];
    __shared__ cx<R> swv[4][64], svv[4][64];  // W^H v, V^H v (zero beyond j), one copy per wave
    __shared__ cx<R> sWo[64], sVo[64];        // row o of W(:, 0:j) and V(:, p:p+j) (zero beyond j)
    __shared__ R sqq[4];
    const int64_t b = blockIdx.y;
    const int n = ws.n, o = i + 1, m = n - o;
    const int NB = (m + ZT - 1) / ZT;
    const int Rb = blockIdx.x;
    const int j = i - p;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform (scalar) wave index
    const int64_t gr = (int64_t)o + (int64_t)Rb * ZT + lane;
    const int64_t grc = gr < n ? gr : (int64_t)n - 1;     // clamped row for unconditional loads
    const cx<R>* A = ws.A + b * ws.sA;
    cx<R>* V = ws.V + b * ws.sV;
    cx<R>* W = ws.W + b * ws.sW;
    const int npn = (n + RB - 1) / RB;
    const cx<R> zero = czero<cx<R>>();

    // ---- phase 1: every load that depends on nothing computed here, issued
    // whole before any of it is waited for (lists longer than their first
    // batch load the rest as they are summed)
    // V(gr, p + jj), W(gr, jj) for jj = w + 4q < j, else 0 (read past the
    // panel's buffers)
    const uint32_t panel_bytes = (uint32_t)((int64_t)n * ws.nb * (int64_t)sizeof(cx<R>));
    const i4_t rV = uniform_rsrc(V + (int64_t)p * n, panel_bytes), rW = uniform_rsrc(W, panel_bytes);
    const int roff = (int)grc * (int)sizeof(cx<R>);
    cx<R> pv[8], pw[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int jj = w + 4 * q;
        const int off = (jj < j ? jj * n * (int)sizeof(cx<R>) : OOB) + roff;
        pv[q] = bload<R>(rV, off);
        pw[q] = bload<R>(rW, off);
    }
    const cx<R> ai = A[grc + (int64_t)i * ws.lda];
    cx<R> h = A[grc + (int64_t)o * ws.lda];
    const cx<R> alpha = A[(int64_t)(i + 1) + (int64_t)i * ws.lda];
    const R hoo = A[(int64_t)o + (int64_t)o * ws.lda].x;
    const R npf = pn_first(ws, b, i, lane);
    const cx<R> z0f = z0_first(ws, b, NB, lane);
    // row o of the panel (stored to LDS by wave 1 once every load is issued)
    const int lc = lane < j ? lane : 0;
    const cx<R> wo_l = W[(int64_t)o + (int64_t)lc * n];
    const cx<R> vo_l = V[(int64_t)o + (int64_t)(p + lc) * n];
    // this row's z partials and the chunk shares of q = Re(u^H A22 u)
    const ZTerms<R> zt(ws, b, Rb, NB, lane, w);
    cx<R> zp[ZB], zq[ZB];
    zt.load(0, zp, zq);
    constexpr int QL = 4;
    const i4_t rq = uniform_rsrc(ws.qpart + b * ws.s_qpart, (uint32_t)((int64_t)nch * (int64_t)sizeof(R)));
    R qt[QL];
#pragma unroll
    for (int u = 0; u < QL; ++u) qt[u] = bload_r<R>(rq, (tid + 256 * u) * (int)sizeof(R));

    // the unscaled panel-dot partials of column i, blocks q = w, w + 4, ...
    // (added in that order); lanes 0-31 take the W parts of panel columns
    // 0-31, lanes 32-63 their V parts (columns 32 and up, for panels wider
    // than 32, in a second pass)
    constexpr int PL = 8;
    const int npd = (n - i + RB - 1) / RB;
    const int nb2 = 2 * ws.nb;
    const i4_t rpd = uniform_rsrc(ws.pvw + b * ws.s_pdot + (int64_t)(i & 1) * ws.NBmax * nb2,
                                 (uint32_t)((int64_t)ws.NBmax * nb2 * (int64_t)sizeof(cx<R>)));
    const int pd_half = lane >> 5, pd_c = lane & 31;
    auto pd_off = [&](int c0, int q) {
        const int loff = c0 + pd_c < j ? (pd_half * ws.nb + c0 + pd_c) * (int)sizeof(cx<R>) : OOB;
        return (q < npd ? q * nb2 * (int)sizeof(cx<R>) : OOB) + loff;
    };
    cx<R> pt[PL];
#pragma unroll
    for (int u = 0; u < PL; ++u) pt[u] = bload<R>(rpd, pd_off(0, w + 4 * u));

    // ---- sums of the partials (the remainders of long lists load here)
    if (w == 1) {
        sWo[lane] = csel(lane < j, wo_l, zero);
        sVo[lane] = csel(lane < j, vo_l, zero);
    }
    sy[w][lane] = zt.sum(zp, zq);
    {
        R qa = 0;
        for (int c0 = tid;; c0 += 256 * QL) {
#pragma unroll
            for (int u = 0; u < QL; ++u) qa += qt[u];
            if (c0 + 256 * QL >= nch) break;
#pragma unroll
            for (int u = 0; u < QL; ++u) qt[u] = bload_r<R>(rq, (c0 + 256 * QL + 256 * u) * (int)sizeof(R));
        }
        qa = dpp_wave_sum(qa);
        if (lane == 0) sqq[w] = qa;
    }
    cx<R> z0 = z0_rest(ws, b, NB, lane, z0f);
    // panel-dot sums (the first pass's loads were issued with the others)
    for (int c0 = 0; c0 < j; c0 += 32) {
        if (c0 > 0) {
#pragma unroll
            for (int u = 0; u < PL; ++u) pt[u] = bload<R>(rpd, pd_off(c0, w + 4 * u));
        }
        cx<R> a = zero;
        for (int q0 = w;; q0 += 4 * PL) {
#pragma unroll
            for (int u = 0; u < PL; ++u) a = cadd(a, pt[u]);
            if (q0 + 4 * PL >= npd) break;
#pragma unroll
            for (int u = 0; u < PL; ++u) pt[u] = bload<R>(rpd, pd_off(c0, q0 + 4 * PL + 4 * u));
        }
        if (pd_half == 0)
            s1[w][c0 + pd_c] = a;
        else
            s2[w][c0 + pd_c] = a;
    }
    cx<R> tau, scale;
    R beta;
    reflector_core(alpha, dpp_wave_sum(pn_rest(ws, b, i, lane, npf)), tau, scale, beta);
    if (gr == o) h.y = 0;
    __syncthreads();

    // ---- panel dots W^H v = conj(W(o, :)) + scale * partials (likewise V),
    // lane = panel column.  Every wave forms them (the same bits in each) and
    // keeps them in its own LDS row for the corrections, so no barrier is
    // needed before those.
    cx<R> wvl = zero, vvl = zero;
    if (lane < j) {
        wvl = cfma(scale, sum4(s1, lane), cconj(sWo[lane]));
        vvl = cfma(scale, sum4(s2, lane), cconj(sVo[lane]));
    }
    swv[w][lane] = wvl;
    svv[w][lane] = vvl;

    // ---- row o: y_o, alpha2 and w_o from fixed-order wave sums over the
    // panel columns, identical in every wave and every workgroup
    cx<R> co = cfma(sVo[lane], wvl, cmul(sWo[lane], vvl));
    R cross = vvl.x * wvl.x + vvl.y * wvl.y;   // Re(conj(V^H v) W^H v)
    co.x = dpp_wave_sum(co.x);
    co.y = dpp_wave_sum(co.y);
    cross = dpp_wave_sum(cross);
    z0.x = dpp_wave_sum(z0.x);
    z0.y = dpp_wave_sum(z0.y);
    const R qq = (sqq[0] + sqq[1]) + (sqq[2] + sqq[3]);
    const cx<R> sz = cmul(scale, z0);
    const R vav = hoo + (R)2 * sz.x + (scale.x * scale.x + scale.y * scale.y) * qq;
    const R a2 = (R)-0.5 * (tau.x * tau.x + tau.y * tau.y) * (vav - (R)2 * cross);
    const cx<R> wo = cadd(cmul(tau, csub(cadd(mk<R>(hoo, 0), sz), co)), mk<R>(a2, 0));
    wave_sync();

    // ---- this block's corrections V (W^H v) + W (V^H v), partial per wave
    cx<R> corr = zero;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int jj = w + 4 * q;
        corr = cfma(pv[q], swv[w][jj], corr);
        corr = cfma(pw[q], svv[w][jj], corr);
    }
    for (int jj = w + 32; jj < j; jj += 4) {
        corr = cfma(V[grc + (int64_t)(p + jj) * n], swv[w][jj], corr);
        corr = cfma(W[grc + (int64_t)jj * n], svv[w][jj], corr);
    }
    sco[w][lane] = corr;
    __syncthreads();

    // ---- v and w of this block's rows (every wave forms them, wave 0 stores)
    cx<R> myv = zero, myw = zero;
    if (gr < n) {
        myv = csel(gr == o, mk<R>(1, 0), cmul(ai, scale));
        if (gr == o) {
            myw = wo;
        } else {
            const cx<R> z = sum4(sy, lane);
            const cx<R> y = cmul(tau, csub(cfma(scale, z, h), sum4(sco, lane)));
            myw = cfma(mk<R>(a2, 0), myv, y);
        }
        if (w == 0) {
            V[gr + (int64_t)i * n] = myv;
            W[gr + (int64_t)j * n] = myw;
        }
    }
    if (w == 0 && Rb == 0 && lane == 0) {
        ws.e[b * n + i] = beta;
        ws.tau[b * n + i] = tau;
    }
    if (!update_next) return;

    // ---- column o -= V(:, 0:j) conj(W(o, 0:j))^T + W(:, 0:j) conj(V(o, 0:j))^T
    // (sWo, sVo hold row o of columns 0..j-1 and zero beyond; column j is
    // this block's v, w with row o = (1, w_o), added last by its wave)
    cx<R> acc = zero;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int jj = w + 4 * q;
        acc = cfma(pv[q], cconj(sWo[jj]), acc);
        acc = cfma(pw[q], cconj(sVo[jj]), acc);
    }
    if (j < 32 && ((j - w) & 3) == 0) {
        acc = cfma(myv, cconj(wo), acc);
        acc = cfma(myw, cconj(mk<R>(1, 0)), acc);
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (w + 4 * q == j) {
                pv[q] = myv;
                pw[q] = myw;
            }
    }
    for (int jj = w + 32; jj <= j; jj += 4) {
        const bool old = jj < j;
        const int jc = old ? jj : 0;
        const cx<R> vr = csel(old, V[grc + (int64_t)(p + jc) * n], myv);
        const cx<R> wr = csel(old, W[grc + (int64_t)jc * n], myw);
        acc = cfma(vr, cconj(csel(old, sWo[jj], wo)), acc);
        acc = cfma(wr, cconj(csel(old, sVo[jj], mk<R>(1, 0))), acc);
    }
    s2[w][lane] = acc;
    __syncthreads();
    // the updated column (every wave; wave 0 stores it, its diagonal and the
    // partial norm of rows o + 2 and below)
    cx<R> an = zero;
    {
        R nrm = 0;
        if (gr < n) {
            const cx<R> a = csub(h, sum4(s2, lane));
            if (w == 0) {
                if (gr == o) {
                    // the diagonal goes to d only: A(o, o) is read as it stood by
                    // every workgroup of this launch and is not needed afterwards
                    ws.d[b * n + o] = a.x;
                } else {
                    ws.A[b * ws.sA + gr + (int64_t)o * ws.lda] = a;
                }
            }
            if (gr >= o + 2) {
                nrm = a.x * a.x + a.y * a.y;
                an = a;
            }
        }
        if (w == 0) {
            nrm = dpp_wave_sum(nrm);
            if (lane == 0) ws.pnorm[b * ws.s_pnorm + (o & 1) * npn + Rb] = nrm;
        }
    }
    // products of the panel columns 0..j with the updated column below its
    // sub-diagonal: this block's share of the next reflector's panel dots,
    // eight columns per wave per transposing reduction
    const int64_t base = b * ws.s_pdot + ((int64_t)(o & 1) * ws.NBmax + Rb) * 2 * ws.nb;
    {
        cx<R> t1[8], t2[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            t1[q] = cmulc(pw[q], an);
            t2[q] = cmulc(pv[q], an);
        }
        const cx<R> r1 = transpose_sum8<R>(t1, lane);
        const cx<R> r2 = transpose_sum8<R>(t2, lane);
        const int jj = w + 4 * (lane >> 3);
        if ((lane & 7) == 0 && jj <= j) {
            ws.pvw[base + jj] = r1;
            ws.pvv[base + jj] = r2;
        }
    }
    if (j >= 32) {
        cx<R> t1[8], t2[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int jj = w + 32 + 4 * q;
            const bool old = jj < j;
            const int jc = old ? jj : 0;
            cx<R> vr = V[grc + (int64_t)(p + jc) * n];
            cx<R> wr = W[grc + (int64_t)jc * n];
            vr = csel(old, vr, csel(jj == j, myv, zero));
            wr = csel(old, wr, csel(jj == j, myw, zero));
            t1[q] = cmulc(wr, an);
            t2[q] = cmulc(vr, an);
        }
        const cx<R> r1 = transpose_sum8<R>(t1, lane);
        const cx<R> r2 = transpose_sum8<R>(t2, lane);
        const int jj = w + 32 + 4 * (lane >> 3);
        if ((lane & 7) == 0 && jj <= j) {
            ws.pvw[base + jj] = r1;
            ws.pvv[base + jj] = r2;
        }
    }
}

// ---------------------------------------------------------------------------
// The last columns, once the trailing matrix has at most TAIL_M rows: one
// workgroup per problem holds its lower triangle in LDS (packed by rows,
// element (r, s), r >= s, at tail_row(r) + s) and reduces it column by
// column, unblocked: Procedure 2's reflector from the column's norm,
// y = tau A22 v (Procedure 4), w = y - (tau / 2)(y^H v) v (Procedure 5) and
// A22 -= v w^H + w v^H (Procedure 6), with the same reflector convention as
// the blocked columns.  Sums are taken in a fixed order (bitwise
// reproducible).  It replaces two launches per column, whose fixed cost
// dominates at this size, by one launch for all of them.
//
// The kernel is bound by the latency of its dependent steps, so each column
// takes five barrier phases: (A) reflector, (B) v, (C) y with the partial
// sums of y^H v, (D) w, (E) the rank-2 update with the partial squared norms
// of the next column (rows two and more below its diagonal).  Eight threads
// share a row in (C) and (E) and take its entries in groups of four, so one
// LDS round trip serves four of them.
// over the lanes that agree in lane mod 8: the first three steps of
// dpp_wave_sum only, so where only the lanes 0 mod 8 hold nonzero values
// lane 0 ends with the wave's sum
template <typename T> __device__ inline T dpp_sum_mod8(T v)
{
    v = xor_sum<32>(v);
    v = xor_sum<16>(v);
    return xor_sum<8>(v);
}

constexpr int TAIL_M = 128;
constexpr int TAIL_T = 1024;
constexpr int TAIL_W = TAIL_T / 64;
static_assert(TAIL_T / 8 >= TAIL_M, "eight threads per row of the tail's trailing matrix");

// start of row r of the packed lower triangle
__host__ __device__ constexpr int tail_row(int r) { return r * (r + 1) / 2; }

template <typename R>
__global__ __launch_bounds__(TAIL_T) void hetrd_tail(HetrdWs<R> ws, int i0)
{
    __shared__ cx<R> P[tail_row(TAIL_M)];
    __shared__ cx<R> sv[TAIL_M], sy[TAIL_M], sw[TAIL_M];
    __shared__ R red[TAIL_W];
    __shared__ cx<R> sred[TAIL_W];
    __shared__ cx<R> sref[2];       // tau, scale
    const int64_t b = blockIdx.x;
    const int n = ws.n, M = n - i0, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r = tid >> 3, q = tid & 7;      // row share of phases C and E
    const cx<R>* A = ws.A + b * ws.sA;
    cx<R>* V = ws.V + b * ws.sV;
    const cx<R> zero = czero<cx<R>>();
    for (int e = tid; e < M * M; e += TAIL_T) {
        const int rr = e % M, c = e / M;
        if (rr >= c) P[tail_row(rr) + c] = A[(int64_t)(i0 + rr) + (int64_t)(i0 + c) * ws.lda];
    }
    __syncthreads();
    {
        // squared norm of rows 2.. of column 0
        R part = 0;
        if (tid >= 2 && tid < M) {
            const cx<R> x = P[tail_row(tid)];
            part = x.x * x.x + x.y * x.y;
        }
        part = dpp_wave_sum(part);
        if (lane == 0) red[wv] = part;
    }
    __syncthreads();
    for (int c = 0; c + 1 < M; ++c) {
        const int i = i0 + c, mm = M - c - 1;     // trailing order below column c
        // (A) Procedure 2 (wave 0: the sixteen partial norms summed across
        // lanes, then lane 0)
        if (wv == 0) {
            const R sig2 = dpp_sum<TAIL_W>(red[lane & (TAIL_W - 1)]);
            if (lane == 0) {
                const cx<R> alpha = P[tail_row(c + 1) + c];
                cx<R> tau, scale;
                R beta;
                reflector_core(alpha, sig2, tau, scale, beta);
                sref[0] = tau;
                sref[1] = scale;
                ws.d[b * n + i] = P[tail_row(c) + c].x;
                ws.e[b * n + i] = beta;
                ws.tau[b * n + i] = tau;
            }
        }
        __syncthreads();
        const cx<R> tau = sref[0];
        // (B) Procedure 3: v = (1, scale x_1, ...), stored for the back-transformation
        if (tid < mm) {
            const cx<R> v = tid == 0 ? mk<R>(1, 0) : cmul(sref[1], P[tail_row(c + 1 + tid) + c]);
            sv[tid] = v;
            V[(int64_t)(i + 1 + tid) + (int64_t)i * ws.n] = v;
        }
        __syncthreads();
        // (C) Procedure 4: y = tau A22 v, the row's stored part and then its
        // mirrored part read down column gr (the same terms in the same order
        // as one pass over s2 = q, q + 8, ...), combined over the eight
        // threads in a fixed order; and this wave's rows' share of y^H v
        {
            cx<R> acc = zero;
            if (r < mm) {
                const int gr = c + 1 + r;
                const cx<R>* Prow = P + tail_row(gr) + (c + 1);
                int s2 = q;
                for (; s2 + 24 <= r; s2 += 32) {
                    cx<R> a4[4], v4[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        a4[u] = Prow[s2 + 8 * u];
                        v4[u] = sv[s2 + 8 * u];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc = cfma(a4[u], v4[u], acc);
                }
                for (; s2 <= r; s2 += 8) acc = cfma(Prow[s2], sv[s2], acc);
                for (; s2 + 24 < mm; s2 += 32) {
                    cx<R> a4[4], v4[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int gs = c + 1 + s2 + 8 * u;
                        a4[u] = P[tail_row(gs) + gr];
                        v4[u] = sv[s2 + 8 * u];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc = cfma(cconj(a4[u]), v4[u], acc);
                }
                for (; s2 < mm; s2 += 8) {
                    const int gs = c + 1 + s2;
                    acc = cfma(cconj(P[tail_row(gs) + gr]), sv[s2], acc);
                }
            }
            acc.x = dpp_sum<8>(acc.x);
            acc.y = dpp_sum<8>(acc.y);
            cx<R> yv = zero;
            if (q == 0 && r < mm) {
                const cx<R> y = cmul(tau, acc);
                sy[r] = y;
                yv = cmulc(y, sv[r]);
            }
            // nonzero only in the lanes with q = 0 (0 mod 8)
            yv.x = dpp_sum_mod8(yv.x);
            yv.y = dpp_sum_mod8(yv.y);
            if (lane == 0) sred[wv] = yv;
        }
        __syncthreads();
        // (D) Procedure 5: w = y - (tau / 2) (y^H v) v
        cx<R> dot = sred[lane & (TAIL_W - 1)];
        dot.x = dpp_sum<TAIL_W>(dot.x);
        dot.y = dpp_sum<TAIL_W>(dot.y);
        if (tid < mm) {
            const cx<R> k = cscale(cmul(tau, dot), (R)0.5);
            sw[tid] = csub(sy[tid], cmul(k, sv[tid]));
        }
        __syncthreads();
        // (E) Procedure 6: A22 -= v w^H + w v^H (lower triangle), and the
        // partial squared norms of column c + 1 below its sub-diagonal
        {
            R part = 0;
            if (r < mm) {
                const int gr = c + 1 + r;
                const cx<R> vr = sv[r], wr = sw[r];
                cx<R>* Prow = P + tail_row(gr) + (c + 1);
                int s2 = q;
                for (; s2 + 24 <= r; s2 += 32) {
                    cx<R> a4[4], w4[4], v4[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        a4[u] = Prow[s2 + 8 * u];
                        w4[u] = sw[s2 + 8 * u];
                        v4[u] = sv[s2 + 8 * u];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) a4[u] = csub(a4[u], cadd(cmulc(w4[u], vr), cmulc(v4[u], wr)));
                    if (s2 == 0 && r >= 2) part = a4[0].x * a4[0].x + a4[0].y * a4[0].y;
#pragma unroll
                    for (int u = 0; u < 4; ++u) Prow[s2 + 8 * u] = a4[u];
                }
                for (; s2 <= r; s2 += 8) {
                    cx<R> a = Prow[s2];
                    a = csub(a, cadd(cmulc(sw[s2], vr), cmulc(sv[s2], wr)));
                    if (s2 == 0 && r >= 2) part = a.x * a.x + a.y * a.y;
                    Prow[s2] = a;
                }
            }
            part = dpp_sum_mod8(part);     // nonzero only where q = 0
            if (lane == 0) red[wv] = part;
        }
        __syncthreads();
    }
    if (tid == 0) ws.d[b * n + n - 1] = P[tail_row(M - 1) + (M - 1)].x;
}

}  // namespace

int hetrd_pn(int64_t n) { return (int)((n + RB - 1) / RB); }

template <typename R>
hipError_t hetrd(hipStream_t st, const HetrdWs<R>& ws0, int64_t nk)
{
    const int n = ws0.n, nb = ws0.nb;
    if (n < 1 || nk < 1) return hipSuccess;
    HetrdWs<R> ws = ws0;
    // Buffer offsets are 32-bit: a matrix (ld x n) of 2 GiB or more is read
    // with plain global loads instead.
    const bool buf = (double)sizeof(cx<R>) * (double)ws.lda * (double)n < 2147483648.0;
    for (int p = 0; p <= n - 1; p += nb) {
        if (n - p <= TAIL_M && p < n - 1) {
            hipLaunchKernelGGL(hetrd_tail<R>, dim3((unsigned)nk), dim3(TAIL_T), 0, st, ws, p);
            break;
        }
        dim3 g1((unsigned)((n - p + RB - 1) / RB), (unsigned)nk);
        hipLaunchKernelGGL(hetrd_colstart<R>, g1, dim3(RB), 0, st, ws, p);
        const int iend = min(p + nb, n - 1);
        for (int i = p; i < iend; ++i) {
            const int o = i + 1, m = n - o;
            const int NB = (m + ZT - 1) / ZT;
            // The one-tile form when the four-tile form would launch fewer
            // workgroups than ws.slots1 (default three per CU: its chains of
            // loads are a quarter as long); the product and the update of a column agree on the
            // chunk layout of the partial sums through ws.zch and ws.CHmax
            // (the buffers hold the one-tile form's NBmax chunks per column).
            int nch4 = 0;
            for (int C = 0; C < NB; ++C) nch4 += nchunks(NB, C);
            const int64_t slots1 = ws0.slots1 > 0 ? ws0.slots1 : 3 * 256;
            ws.zch = (int64_t)nch4 * nk < slots1 ? 1 : ZCH;
            ws.CHmax = ws.zch == 1 ? ws0.NBmax : (ws0.NBmax + ZCH - 1) / ZCH;
            const int nch = ws.zch == 1 ? NB * (NB + 1) / 2 : nch4;
            // Consecutive columns traverse their tiles in opposite orders (odd
            // columns from the last k-point's last chunk back), so each launch
            // starts on the tiles its predecessor read last, which the 256 MB
            // memory-side cache still holds once the lower triangles of all
            // k-points exceed it (n = 2000 x 16: 9% faster at m = 1500..1750).
            const int rev = i & 1;
            const ProfLaunch pl = prof_launch_begin(PH_HEMV, st);
            const dim3 gz((unsigned)nch, (unsigned)nk);
            if (ws.zch == 1) {
                if (buf)
                    launch_timed(pl, hetrd_zhemv_tile<R, true>, gz, dim3(256), st, ws, i, rev);
                else
                    launch_timed(pl, hetrd_zhemv_tile<R, false>, gz, dim3(256), st, ws, i, rev);
            } else {
                if (buf)
                    launch_timed(pl, hetrd_zhemv<R, true>, gz, dim3(256), st, ws, i, rev);
                else
                    launch_timed(pl, hetrd_zhemv<R, false>, gz, dim3(256), st, ws, i, rev);
            }
            prof_launch_end(PH_HEMV, st, pl,
                            (double)sizeof(cx<R>) * 0.5 * (double)m * (double)(m + 1) * (double)nk, 0.0);
            const int upd = (i + 1 < p + nb) && (o <= n - 1);
            hipLaunchKernelGGL(hetrd_update<R>, dim3((unsigned)NB, (unsigned)nk), dim3(256), 0, st, ws, i, p, upd, nch);
        }
        if (p + nb <= n - 1) {
            const int t0 = p + nb;
            const int64_t m2 = n - t0;
            hipError_t e = cher2k_lower<R>(st, m2, nb, ws.V + (int64_t)t0 + (int64_t)p * n, n, ws.sV,
                                           ws.W + t0, n, ws.sW, ws.A + (int64_t)t0 + (int64_t)t0 * ws.lda,
                                           ws.lda, ws.sA, nk);
            if (e != hipSuccess) return e;
        }
    }
    return hipGetLastError();
}

template hipError_t hetrd<double>(hipStream_t, const HetrdWs<double>&, int64_t);
template hipError_t hetrd<float>(hipStream_t, const HetrdWs<float>&, int64_t);

}  // namespace kgev
