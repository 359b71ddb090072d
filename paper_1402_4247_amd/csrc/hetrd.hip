// Blocked Householder tridiagonalisation of a batch of Hermitian matrices
// (lower storage): Section III, Procedures 1-6 of Eigen_HH, arXiv:1402.4247,
// reorganised in panels of nb columns.
//
// Per column i of a panel starting at p (j = i - p, o = i + 1):
//   zhemv    : one chunk of the Hermitian product z = A22 u (Procedure 4) from
//       the lower triangle only, with u the column below the sub-diagonal as
//       it stands (u_o = 0, u_r = A(r, i)): it needs nothing derived in this
//       step, so the workgroups only stream their tiles;
//   reduce   : derives the reflector (Procedure 2, stable sign, real beta)
//       from the partial norms, v = (1, scale * A(o+1:n, i)), stores v, and
//       forms y = tau (A22(:, o) + scale z - V (W^H v) - W (V^H v)), where
//       A22 v = A22(:, o) + scale A22 u by linearity;
//   finalize : w = y - (tau/2)(y^H v) v (Procedure 5), stored as column j of
//       W; then the next column of the panel is brought up to date,
//       A(o:n, o) -= V(o:n, 0:j) conj(W(o, 0:j))^T + W(o:n, 0:j) conj(V(o, 0:j))^T,
//       and its squared norm below the sub-diagonal and its products with
//       the panel columns (the pieces of W^H v and V^H v for the next
//       reflector) are reduced in per-block partials.
// After the panel the trailing matrix takes the rank-2nb update
// A22 -= V W^H + W V^H (Procedure 6, on MFMA).
// No atomics: every sum is taken in a fixed order, so results are bitwise
// reproducible run to run.
#include "common.hpp"
#include "kernels.hpp"

namespace kgev {

namespace {

constexpr int ZT = 64;          // ZHEMV tile edge
constexpr int ZCH = 4;          // tiles per ZHEMV chunk: one per wave of the workgroup
constexpr int RB = 64;          // rows per workgroup in the column kernels

__device__ __host__ inline int nchunks(int NB, int C) { return (NB - C + ZCH - 1) / ZCH; }

// Reflector from the partial norms: returns tau and the scale applied to x.
template <typename R>
__device__ inline void reflector(const HetrdWs<R>& ws, int64_t b, int i, cx<R>& tau, cx<R>& scale, R& beta)
{
    const int n = ws.n;
    const R* pn = ws.pnorm + b * ws.s_pnorm;
    const int np = (n - i + RB - 1) / RB;
    R sig2 = 0;
    for (int q = 0; q < np; ++q) sig2 += pn[q];
    const cx<R> alpha = ws.A[b * ws.sA + (int64_t)(i + 1) + (int64_t)i * ws.lda];
    if (sig2 == (R)0 && alpha.y == (R)0) {
        tau = czero<cx<R>>();
        scale = czero<cx<R>>();
        beta = alpha.x;
        return;
    }
    const R nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sig2);
    beta = (alpha.x >= (R)0) ? -nrm : nrm;
    tau = mk<R>((beta - alpha.x) / beta, -alpha.y / beta);
    // scale = 1 / (alpha - beta)
    const R dr = alpha.x - beta, di = alpha.y;
    const R den = dr * dr + di * di;
    scale = mk<R>(dr / den, -di / den);
}

// One halving step of the transposing reduction: lanes with the MASK bit set
// keep values HALF..2HALF-1 (moved down to 0..HALF-1), the others keep
// 0..HALF-1; each adds its partner's copy of the values it keeps.
template <int MASK, int HALF, int NV, typename R>
__device__ __attribute__((always_inline)) inline void halve_step(cx<R> (&t)[NV], bool up)
{
#pragma unroll
    for (int q = 0; q < HALF; ++q) {
        const cx<R> send = up ? t[q] : t[q + HALF];
        const cx<R> keep = up ? t[q + HALF] : t[q];
        cx<R> rcv;
        rcv.x = __shfl_xor(send.x, MASK, WAVE);
        rcv.y = __shfl_xor(send.y, MASK, WAVE);
        t[q] = cadd(keep, rcv);
    }
}

template <int MASK, typename R>
__device__ __attribute__((always_inline)) inline cx<R> xor_add(cx<R> r)
{
    r.x += __shfl_xor(r.x, MASK, WAVE);
    r.y += __shfl_xor(r.y, MASK, WAVE);
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
    r = xor_add<4, R>(r);
    r = xor_add<2, R>(r);
    r = xor_add<1, R>(r);
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
    acc = wave_sum(acc);
    if (threadIdx.x == 0) ws.pnorm[b * ws.s_pnorm + blockIdx.x] = acc;
}

// ---------------------------------------------------------------------------
// One chunk of z = A22 u.  A chunk is up to four 64x64 tiles (R0..R0+3, C) of
// one block column of the lower triangle; wave w owns tile R0 + w whole: the
// direct part z_R += A_RC u_C comes out complete per row, the transposed part
// z_C += A_RC^H u_R per column after a transposing wave reduction, and the
// four waves' column sums are added once.
template <typename R>
__global__ __launch_bounds__(256) void hetrd_zhemv(HetrdWs<R> ws, int i)
{
    __shared__ cx<R> svC[ZT];
    __shared__ cx<R> sT[ZCH][ZT];
    const int64_t b = blockIdx.y;
    const int n = ws.n;
    const int o = i + 1;
    const int m = n - o;
    const int NB = (m + ZT - 1) / ZT;

    // which (block column C, chunk ch) is ours
    int bid = blockIdx.x, C = 0;
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
    // is masked afterwards, so no branch guards them; each group of 8 columns
    // is requested one step ahead of its use.
    const cx<R>* Arow = A + (row_ok ? gr : (int64_t)n - 1);
    const int64_t gcb = (int64_t)o + (int64_t)C * ZT;
    auto load_group = [&](int g, cx<R> (&a)[8]) {
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
            const int64_t gc = gcb + g * 8 + cc;
            a[cc] = Arow[(gc < n ? gc : (int64_t)n - 1) * lda];
        }
    };
    cx<R> a[8], an[8];
    load_group(0, a);
    if (tid < ZT) {
        const int64_t gc = gcb + tid;
        const cx<R> u = Ai[gc < n ? gc : (int64_t)n - 1];
        svC[tid] = (gc > o && gc < n) ? u : czero<cx<R>>();
    }
    cx<R> uR = Ai[row_ok ? gr : (int64_t)n - 1];
    if (!(row_ok && gr > o)) uR = czero<cx<R>>();
    __syncthreads();

    if (have_tile) {
        const bool diag_tile = (Rb == C);
        cx<R> yd = czero<cx<R>>();
#pragma unroll 1
        for (int g = 0; g < 8; ++g) {
            if (g + 1 < 8) load_group(g + 1, an);
            const int64_t gc0 = gcb + g * 8;
#pragma unroll
            for (int cc = 0; cc < 8; ++cc) {
                const int64_t gc = gc0 + cc;
                const bool ok = row_ok && gc < n && (!diag_tile || gr >= gc);
                const bool diag = diag_tile && (gr == gc);
                cx<R> x;
                x.x = ok ? a[cc].x : (R)0;
                x.y = (ok && !diag) ? a[cc].y : (R)0;
                yd = cfma(x, svC[g * 8 + cc], yd);
                // the diagonal entry is counted once (direct part only)
                a[cc] = diag ? czero<cx<R>>() : cmulc(x, uR);
            }
            const cx<R> r = transpose_sum8<R>(a, lane);
            if ((lane & 7) == 0) sT[w][g * 8 + (lane >> 3)] = r;
#pragma unroll
            for (int cc = 0; cc < 8; ++cc) a[cc] = an[cc];
        }
        ws.ypart[b * ws.s_ypart + ((int64_t)Rb * ws.NBmax + C) * ZT + lane] = yd;
    } else {
        sT[w][lane] = czero<cx<R>>();
    }
    __syncthreads();
    if (tid < ZT) {
        const cx<R> s = cadd(cadd(sT[0][tid], sT[1][tid]), cadd(sT[2][tid], sT[3][tid]));
        ws.ypartT[b * ws.s_ypartT + ((int64_t)C * ws.CHmax + ch) * ZT + tid] = s;
    }
}

// ---------------------------------------------------------------------------
// Reflector of column i, v stored, and
// y = tau (A22(:, o) + scale z - V (W^H v) - W (V^H v)) for one 64-row block.
// The panel dots come as partials of the unscaled column, W^H v =
// conj(W(o, :)) + scale * sum_r conj(W(r, :)) A(r, i) over r > o (likewise
// V^H v).  The four waves split every sum (wave w takes the terms with
// index = w mod 4).
template <typename R>
__global__ __launch_bounds__(256) void hetrd_reduce(HetrdWs<R> ws, int i, int p)
{
    __shared__ cx<R> s1[4][64], s2[4][64], sy[4][64];
    __shared__ cx<R> swv[64], svv[64];
    const int64_t b = blockIdx.y;
    const int n = ws.n, o = i + 1, m = n - o;
    const int NB = (m + ZT - 1) / ZT;
    const int Rb = blockIdx.x;
    const int j = i - p;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t gr = (int64_t)o + (int64_t)Rb * ZT + lane;
    const cx<R>* A = ws.A + b * ws.sA;
    cx<R>* V = ws.V + b * ws.sV;
    const cx<R>* W = ws.W + b * ws.sW;
    // loads that do not depend on the reflector go first
    cx<R> ai = czero<cx<R>>(), h = czero<cx<R>>();
    if (w == 0 && gr < n) {
        ai = A[gr + (int64_t)i * ws.lda];
        h = A[gr + (int64_t)o * ws.lda];
        if (gr == o) h.y = 0;
    }
    // panel dot partials (lane = panel column)
    {
        cx<R> a1 = czero<cx<R>>(), a2 = czero<cx<R>>();
        if (lane < j) {
            const int np = (n - i + RB - 1) / RB;
            for (int q = w; q < np; q += 4) {
                a1 = cadd(a1, ws.pvw[b * ws.s_pdot + (int64_t)q * ws.nb + lane]);
                a2 = cadd(a2, ws.pvv[b * ws.s_pdot + (int64_t)q * ws.nb + lane]);
            }
        }
        s1[w][lane] = a1;
        s2[w][lane] = a2;
    }
    // partial sums of A22 u for these rows
    {
        cx<R> y = czero<cx<R>>();
        const cx<R>* yp = ws.ypart + b * ws.s_ypart + (int64_t)Rb * ws.NBmax * ZT + lane;
        for (int C = w; C <= Rb; C += 4) y = cadd(y, yp[(int64_t)C * ZT]);
        const int nc = nchunks(NB, Rb);
        const cx<R>* yq = ws.ypartT + b * ws.s_ypartT + (int64_t)Rb * ws.CHmax * ZT + lane;
        for (int ch = w; ch < nc; ch += 4) y = cadd(y, yq[(int64_t)ch * ZT]);
        sy[w][lane] = y;
    }
    cx<R> tau, scale;
    R beta;
    reflector(ws, b, i, tau, scale, beta);
    __syncthreads();
    if (tid < 64) {
        const cx<R> d1 = cadd(cadd(s1[0][tid], s1[1][tid]), cadd(s1[2][tid], s1[3][tid]));
        const cx<R> d2 = cadd(cadd(s2[0][tid], s2[1][tid]), cadd(s2[2][tid], s2[3][tid]));
        if (tid < j) {
            swv[tid] = cfma(scale, d1, cconj(W[(int64_t)o + (int64_t)tid * n]));
            svv[tid] = cfma(scale, d2, cconj(V[(int64_t)o + (int64_t)(p + tid) * n]));
        }
    }
    __syncthreads();
    cx<R> corr = czero<cx<R>>();
    if (gr < n) {
        for (int jj = w; jj < j; jj += 4) {
            corr = cfma(V[gr + (int64_t)(p + jj) * n], swv[jj], corr);
            corr = cfma(W[gr + (int64_t)jj * n], svv[jj], corr);
        }
    }
    s1[w][lane] = corr;     // s1 is free again (read before the last barrier)
    __syncthreads();
    if (w == 0) {
        cx<R> part = czero<cx<R>>();
        if (gr < n) {
            const cx<R> z = cadd(cadd(sy[0][lane], sy[1][lane]), cadd(sy[2][lane], sy[3][lane]));
            const cx<R> c = cadd(cadd(s1[0][lane], s1[1][lane]), cadd(s1[2][lane], s1[3][lane]));
            const cx<R> v = (gr == o) ? mk<R>(1, 0) : cmul(ai, scale);
            V[gr + (int64_t)i * n] = v;
            const cx<R> y = cmul(tau, csub(cfma(scale, z, h), c));
            ws.ybuf[b * n + gr] = y;
            part = cmulc(y, v);
        }
        part.x = wave_sum(part.x);
        part.y = wave_sum(part.y);
        if (lane == 0) ws.pyv[b * ws.NBmax + Rb] = part;
        if (Rb == 0 && lane == 0) {
            ws.e[b * n + i] = beta;
            ws.tau[b * n + i] = tau;
        }
    }
}

// ---------------------------------------------------------------------------
// w = y + alpha2 v (alpha2 = -(tau/2) y^H v), stored as W(:, j); then, when
// the panel continues, column i+1 is brought up to date (the four waves split
// the panel columns), and its partial norm and partial panel dots are reduced.
template <typename R>
__global__ __launch_bounds__(256) void hetrd_finalize(HetrdWs<R> ws, int i, int p, int update_next)
{
    __shared__ cx<R> sWr[64], sVr[64];
    __shared__ cx<R> sp[4][64];
    const int64_t b = blockIdx.y;
    const int n = ws.n, o = i + 1, m = n - o;
    const int NB = (m + ZT - 1) / ZT;
    const int j = i - p;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    cx<R> sum = czero<cx<R>>();
    for (int q = 0; q < NB; ++q) sum = cadd(sum, ws.pyv[b * ws.NBmax + q]);
    const cx<R> tau = ws.tau[b * n + i];
    const cx<R> a2 = cscale(cmul(tau, sum), (R)-0.5);

    const int64_t gr = (int64_t)o + (int64_t)blockIdx.x * RB + lane;
    cx<R>* V = ws.V + b * ws.sV;
    cx<R>* W = ws.W + b * ws.sW;
    cx<R> wv = czero<cx<R>>();
    if (gr < n) {
        wv = cfma(a2, V[gr + (int64_t)i * n], ws.ybuf[b * n + gr]);
        if (w == 0) W[gr + (int64_t)j * n] = wv;
    }
    if (!update_next) return;
    // row o of V and W for the update of column o
    if (tid <= j) {
        sVr[tid] = V[(int64_t)o + (int64_t)(p + tid) * n];
        sWr[tid] = (tid < j) ? W[(int64_t)o + (int64_t)tid * n] : cadd(ws.ybuf[b * n + o], a2);
    }
    __syncthreads();
    cx<R> acc = czero<cx<R>>();
    if (gr < n) {
        for (int jj = w; jj <= j; jj += 4) {
            const cx<R> wr = (jj < j) ? W[gr + (int64_t)jj * n] : wv;
            acc = cfma(V[gr + (int64_t)(p + jj) * n], cconj(sWr[jj]), acc);
            acc = cfma(wr, cconj(sVr[jj]), acc);
        }
    }
    sp[w][lane] = acc;
    __syncthreads();
    if (w == 0) {
        R nrm = 0;
        cx<R> an = czero<cx<R>>();
        if (gr < n) {
            cx<R>* A = ws.A + b * ws.sA;
            const cx<R> c = cadd(cadd(sp[0][lane], sp[1][lane]), cadd(sp[2][lane], sp[3][lane]));
            cx<R> a = csub(A[gr + (int64_t)o * ws.lda], c);
            if (gr == o) {
                a.y = 0;
                ws.d[b * n + o] = a.x;
            }
            A[gr + (int64_t)o * ws.lda] = a;
            if (gr >= o + 2) {
                nrm = a.x * a.x + a.y * a.y;
                an = a;
            }
        }
        nrm = wave_sum(nrm);
        if (lane == 0) ws.pnorm[b * ws.s_pnorm + blockIdx.x] = nrm;
        sp[0][lane] = an;
    }
    __syncthreads();
    // products of the panel columns 0..j with the updated column below its
    // sub-diagonal: this block's share of the next reflector's panel dots
    const cx<R> an = sp[0][lane];
    for (int jj = w; jj <= j; jj += 4) {
        cx<R> t1 = czero<cx<R>>(), t2 = czero<cx<R>>();
        if (gr < n) {
            const cx<R> wr = (jj < j) ? W[gr + (int64_t)jj * n] : wv;
            t1 = cmulc(wr, an);
            t2 = cmulc(V[gr + (int64_t)(p + jj) * n], an);
        }
        t1.x = wave_sum(t1.x); t1.y = wave_sum(t1.y);
        t2.x = wave_sum(t2.x); t2.y = wave_sum(t2.y);
        if (lane == 0) {
            ws.pvw[b * ws.s_pdot + (int64_t)blockIdx.x * ws.nb + jj] = t1;
            ws.pvv[b * ws.s_pdot + (int64_t)blockIdx.x * ws.nb + jj] = t2;
        }
    }
}

}  // namespace

int hetrd_pn(int64_t n) { return (int)((n + RB - 1) / RB); }

template <typename R>
hipError_t hetrd(hipStream_t st, const HetrdWs<R>& ws, int64_t nk)
{
    const int n = ws.n, nb = ws.nb;
    if (n < 1 || nk < 1) return hipSuccess;
    for (int p = 0; p <= n - 1; p += nb) {
        dim3 g1((unsigned)((n - p + RB - 1) / RB), (unsigned)nk);
        hipLaunchKernelGGL(hetrd_colstart<R>, g1, dim3(RB), 0, st, ws, p);
        const int iend = min(p + nb, n - 1);
        for (int i = p; i < iend; ++i) {
            const int o = i + 1, m = n - o;
            const int NB = (m + ZT - 1) / ZT;
            int nch = 0;
            for (int C = 0; C < NB; ++C) nch += nchunks(NB, C);
            prof_before(PH_HEMV, st);
            hipLaunchKernelGGL(hetrd_zhemv<R>, dim3((unsigned)nch, (unsigned)nk), dim3(256), 0, st, ws, i);
            prof_after(PH_HEMV, st, (double)sizeof(cx<R>) * 0.5 * (double)m * (double)(m + 1) * (double)nk, 0.0);
            hipLaunchKernelGGL(hetrd_reduce<R>, dim3((unsigned)NB, (unsigned)nk), dim3(256), 0, st, ws, i, p);
            const int upd = (i + 1 < p + nb) && (o <= n - 1);
            dim3 g4((unsigned)((n - o + RB - 1) / RB), (unsigned)nk);
            hipLaunchKernelGGL(hetrd_finalize<R>, g4, dim3(256), 0, st, ws, i, p, upd);
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
