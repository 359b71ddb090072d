// Blocked Householder tridiagonalisation of a batch of Hermitian matrices
// (lower storage): Section III, Procedures 1-6 of Eigen_HH, arXiv:1402.4247,
// reorganised in panels of nb columns.
//
// Per column i of a panel starting at p (j = i - p):
//   colstart / finalize : the column is brought up to date with the panel's
//       reflectors, A(i:n, i) -= V(i:n, 0:j) conj(W(i, 0:j))^T
//                                + W(i:n, 0:j) conj(V(i, 0:j))^T,
//       and its squared norm below the sub-diagonal is reduced in partials;
//   zhemv    : every workgroup derives the reflector (Procedure 2, stable
//       sign, real beta) from the partial norms, then forms one chunk of the
//       Hermitian product A22 v (Procedure 4) from the lower triangle only,
//       leaving deterministic partial sums;
//   reduce   : sums the partials per row and applies the panel corrections
//       y = tau (A22 v - V (W^H v) - W (V^H v));
//   finalize : w = y - (tau/2)(y^H v) v (Procedure 5), stored as column j of
//       W, then the next column of the panel is updated (above).
// After the panel the trailing matrix takes the rank-2nb update
// A22 -= V W^H + W V^H (Procedure 6, on MFMA).
// No atomics: every sum is taken in a fixed order, so results are bitwise
// reproducible run to run.
#include "common.hpp"
#include "kernels.hpp"

namespace kgev {

namespace {

constexpr int ZT = 64;          // ZHEMV tile edge
constexpr int ZCH = 4;          // tiles per ZHEMV chunk (one workgroup)
constexpr int RB = 256;         // rows per workgroup in the column kernels

__device__ __host__ inline int nchunks(int NB, int C) { return (NB - C + ZCH - 1) / ZCH; }

// block-wide sum of one real value per thread (blockDim.x == 256)
template <typename R>
__device__ inline R block_sum256(R v, R* sh)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    R s = sh[0] + sh[1] + sh[2] + sh[3];
    return s;
}

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

template <typename R>
__device__ inline cx<R> vval(const HetrdWs<R>& ws, int64_t b, int i, int64_t r, cx<R> scale)
{
    if (r == i + 1) return mk<R>(1, 0);
    if (r >= ws.n) return czero<cx<R>>();
    return cmul(ws.A[b * ws.sA + r + (int64_t)i * ws.lda], scale);
}

// ---------------------------------------------------------------------------
// First column of a panel: d_c and partial norms of rows c+2..n-1.
template <typename R>
__global__ __launch_bounds__(RB) void hetrd_colstart(HetrdWs<R> ws, int c)
{
    __shared__ R sh[4];
    const int64_t b = blockIdx.y;
    const int64_t r = (int64_t)c + (int64_t)blockIdx.x * RB + threadIdx.x;
    R acc = 0;
    if (r < ws.n) {
        const cx<R> a = ws.A[b * ws.sA + r + (int64_t)c * ws.lda];
        if (r == c) ws.d[b * ws.n + c] = a.x;
        if (r >= c + 2) acc = a.x * a.x + a.y * a.y;
    }
    const R s = block_sum256(acc, sh);
    if (threadIdx.x == 0) ws.pnorm[b * ws.s_pnorm + blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// Reflector + one chunk of the Hermitian product A22 v.
template <typename R>
__global__ __launch_bounds__(256) void hetrd_zhemv(HetrdWs<R> ws, int i, int p)
{
    __shared__ cx<R> svC[ZT];
    __shared__ cx<R> sy[4][ZT];
    const int64_t b = blockIdx.y;
    const int n = ws.n;
    const int o = i + 1;
    const int m = n - o;
    const int NB = (m + ZT - 1) / ZT;
    const int j = i - p;

    // which (block column C, chunk ch) is ours
    int bid = blockIdx.x, C = 0;
    for (; C < NB; ++C) {
        const int nc = nchunks(NB, C);
        if (bid < nc) break;
        bid -= nc;
    }
    if (C >= NB) return;
    const int ch = bid;

    cx<R> tau, scale;
    R beta;
    reflector(ws, b, i, tau, scale, beta);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid < ZT) svC[tid] = vval(ws, b, i, (int64_t)o + C * ZT + tid, scale);
    __syncthreads();

    const cx<R>* A = ws.A + b * ws.sA;
    const int64_t lda = ws.lda;
    cx<R> vC[16];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) vC[cc] = svC[w * 16 + cc];

    cx<R> yT = czero<cx<R>>();
    const int R0 = C + ch * ZCH;
    const int R1 = min(R0 + ZCH, NB);
    const int64_t gcol0 = (int64_t)o + (int64_t)C * ZT + w * 16;
    for (int Rb = R0; Rb < R1; ++Rb) {
        const int64_t gr = (int64_t)o + (int64_t)Rb * ZT + lane;
        const cx<R> vR = vval(ws, b, i, gr, scale);
        cx<R> a[16];
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
            const int64_t gc = gcol0 + cc;
            const bool ok = gr < n && gc < n && (Rb != C || gr >= gc);
            a[cc] = ok ? A[gr + gc * lda] : czero<cx<R>>();
        }
        // direct part: y_R += A_RC v_C (diagonal entries real)
        cx<R> yd = czero<cx<R>>();
        cx<R> t[16];
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
            const bool diag = (gr == gcol0 + cc);
            if (diag) a[cc].y = 0;
            yd = cfma(a[cc], vC[cc], yd);
            // transposed part: y_C += A_RC^H v_R (the diagonal counted once)
            t[cc] = diag ? czero<cx<R>>() : cmulc(a[cc], vR);
        }
        // butterfly: lane l ends with column (l >> 2) of this wave's 16
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int mask = 32 >> s, half = 8 >> s;
            const bool up = (lane & mask) != 0;
#pragma unroll
            for (int q = 0; q < half; ++q) {
                const cx<R> send = up ? t[q] : t[q + half];
                const cx<R> keep = up ? t[q + half] : t[q];
                cx<R> rcv;
                rcv.x = __shfl_xor(send.x, mask, WAVE);
                rcv.y = __shfl_xor(send.y, mask, WAVE);
                t[q] = cadd(keep, rcv);
            }
        }
        t[0].x += __shfl_xor(t[0].x, 2, WAVE);
        t[0].y += __shfl_xor(t[0].y, 2, WAVE);
        t[0].x += __shfl_xor(t[0].x, 1, WAVE);
        t[0].y += __shfl_xor(t[0].y, 1, WAVE);
        yT = cadd(yT, t[0]);
        sy[w][lane] = yd;
        __syncthreads();
        if (tid < ZT) {
            cx<R> s = cadd(cadd(sy[0][tid], sy[1][tid]), cadd(sy[2][tid], sy[3][tid]));
            ws.ypart[b * ws.s_ypart + ((int64_t)Rb * ws.NBmax + C) * ZT + tid] = s;
        }
        __syncthreads();
    }
    if ((lane & 3) == 0)
        ws.ypartT[b * ws.s_ypartT + ((int64_t)C * ws.CHmax + ch) * ZT + w * 16 + (lane >> 2)] = yT;

    if (ch == 0) {
        // this workgroup owns rows of block C: store v and the panel dots
        cx<R>* V = ws.V + b * ws.sV;
        const int64_t gr = (int64_t)o + (int64_t)C * ZT + lane;
        if (tid < ZT && gr < n) V[gr + (int64_t)i * n] = svC[tid];
        const cx<R> vl = svC[lane];
        const cx<R>* W = ws.W + b * ws.sW;
        for (int jj = w; jj < j; jj += 4) {
            cx<R> t1 = czero<cx<R>>(), t2 = czero<cx<R>>();
            if (gr < n) {
                t1 = cmulc(W[gr + (int64_t)jj * n], vl);
                t2 = cmulc(V[gr + (int64_t)(p + jj) * n], vl);
            }
            t1.x = wave_sum(t1.x); t1.y = wave_sum(t1.y);
            t2.x = wave_sum(t2.x); t2.y = wave_sum(t2.y);
            if (lane == 0) {
                ws.pvw[b * ws.s_pdot + (int64_t)C * ws.nb + jj] = t1;
                ws.pvv[b * ws.s_pdot + (int64_t)C * ws.nb + jj] = t2;
            }
        }
        if (C == 0 && tid == 0) {
            ws.e[b * n + i] = beta;
            ws.tau[b * n + i] = tau;
        }
    }
}

// ---------------------------------------------------------------------------
// y = tau (sum of partials - V (W^H v) - W (V^H v)) for one 64-row block.
template <typename R>
__global__ __launch_bounds__(64) void hetrd_reduce(HetrdWs<R> ws, int i, int p)
{
    __shared__ cx<R> swv[64], svv[64];
    const int64_t b = blockIdx.y;
    const int n = ws.n, o = i + 1, m = n - o;
    const int NB = (m + ZT - 1) / ZT;
    const int Rb = blockIdx.x;
    const int j = i - p;
    const int t = threadIdx.x;
    if (t < j) {
        cx<R> s1 = czero<cx<R>>(), s2 = czero<cx<R>>();
        for (int C = 0; C < NB; ++C) {
            s1 = cadd(s1, ws.pvw[b * ws.s_pdot + (int64_t)C * ws.nb + t]);
            s2 = cadd(s2, ws.pvv[b * ws.s_pdot + (int64_t)C * ws.nb + t]);
        }
        swv[t] = s1;
        svv[t] = s2;
    }
    __syncthreads();
    const int64_t gr = (int64_t)o + (int64_t)Rb * ZT + t;
    cx<R> y = czero<cx<R>>();
    for (int C = 0; C <= Rb; ++C) y = cadd(y, ws.ypart[b * ws.s_ypart + ((int64_t)Rb * ws.NBmax + C) * ZT + t]);
    const int nc = nchunks(NB, Rb);
    for (int ch = 0; ch < nc; ++ch) y = cadd(y, ws.ypartT[b * ws.s_ypartT + ((int64_t)Rb * ws.CHmax + ch) * ZT + t]);
    cx<R> part = czero<cx<R>>();
    if (gr < n) {
        const cx<R>* V = ws.V + b * ws.sV;
        const cx<R>* W = ws.W + b * ws.sW;
        for (int jj = 0; jj < j; ++jj) {
            y = csub(y, cmul(V[gr + (int64_t)(p + jj) * n], swv[jj]));
            y = csub(y, cmul(W[gr + (int64_t)jj * n], svv[jj]));
        }
        y = cmul(ws.tau[b * n + i], y);
        ws.ybuf[b * n + gr] = y;
        part = cmulc(y, V[gr + (int64_t)i * n]);
    }
    part.x = wave_sum(part.x);
    part.y = wave_sum(part.y);
    if (t == 0) ws.pyv[b * ws.NBmax + Rb] = part;
}

// ---------------------------------------------------------------------------
// w = y + alpha2 v (alpha2 = -(tau/2) y^H v), stored as W(:, j); then, when
// the panel continues, column i+1 is brought up to date and its partial norms
// are reduced.
template <typename R>
__global__ __launch_bounds__(RB) void hetrd_finalize(HetrdWs<R> ws, int i, int p, int update_next)
{
    __shared__ cx<R> sWr[64], sVr[64];
    __shared__ R sh[4];
    const int64_t b = blockIdx.y;
    const int n = ws.n, o = i + 1, m = n - o;
    const int NB = (m + ZT - 1) / ZT;
    const int j = i - p;
    const int t = threadIdx.x;
    cx<R> sum = czero<cx<R>>();
    for (int q = 0; q < NB; ++q) sum = cadd(sum, ws.pyv[b * ws.NBmax + q]);
    const cx<R> tau = ws.tau[b * n + i];
    const cx<R> a2 = cscale(cmul(tau, sum), (R)-0.5);

    const int64_t gr = (int64_t)o + (int64_t)blockIdx.x * RB + t;
    cx<R>* V = ws.V + b * ws.sV;
    cx<R>* W = ws.W + b * ws.sW;
    cx<R> wv = czero<cx<R>>();
    if (gr < n) {
        wv = cfma(a2, V[gr + (int64_t)i * n], ws.ybuf[b * n + gr]);
        W[gr + (int64_t)j * n] = wv;
    }
    if (!update_next) return;
    // row o of V and W for the update of column o
    if (t <= j) {
        sVr[t] = V[(int64_t)o + (int64_t)(p + t) * n];
        sWr[t] = (t < j) ? W[(int64_t)o + (int64_t)t * n] : cadd(ws.ybuf[b * n + o], a2);
    }
    __syncthreads();
    R acc = 0;
    if (gr < n) {
        cx<R>* A = ws.A + b * ws.sA;
        cx<R> a = A[gr + (int64_t)o * ws.lda];
        for (int jj = 0; jj <= j; ++jj) {
            const cx<R> wr = (jj < j) ? W[gr + (int64_t)jj * n] : wv;
            a = csub(a, cmul(V[gr + (int64_t)(p + jj) * n], cconj(sWr[jj])));
            a = csub(a, cmul(wr, cconj(sVr[jj])));
        }
        if (gr == o) {
            a.y = 0;
            ws.d[b * n + o] = a.x;
        }
        A[gr + (int64_t)o * ws.lda] = a;
        if (gr >= o + 2) acc = a.x * a.x + a.y * a.y;
    }
    const R s = block_sum256(acc, sh);
    if (t == 0) ws.pnorm[b * ws.s_pnorm + blockIdx.x] = s;
}

}  // namespace

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
            hipLaunchKernelGGL(hetrd_zhemv<R>, dim3((unsigned)nch, (unsigned)nk), dim3(256), 0, st, ws, i, p);
            prof_after(PH_HEMV, st, (double)sizeof(cx<R>) * 0.5 * (double)m * (double)(m + 1) * (double)nk, 0.0);
            hipLaunchKernelGGL(hetrd_reduce<R>, dim3((unsigned)NB, (unsigned)nk), dim3(64), 0, st, ws, i, p);
            const int upd = (i + 1 < p + nb) && (o <= n - 1);
            dim3 g4((unsigned)((n - o + RB - 1) / RB), (unsigned)nk);
            hipLaunchKernelGGL(hetrd_finalize<R>, g4, dim3(RB), 0, st, ws, i, p, upd);
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
