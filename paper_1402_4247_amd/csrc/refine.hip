// FP64 eigenpair refinement for the mixed-precision form of Part 4 (the
// complex-FP32 Eigen_HH result refined against the FP64 matrix), after
// Ogita & Aishima, "Iterative refinement for symmetric eigenvalue
// decomposition" (2018), restated for Hermitian matrices.  With Y the current
// eigenvector estimate (n x n), one sweep is
//   G = Y^H Y,  R = I - G,  S = Y^H A Y,
//   lambda_j = S_jj / G_jj,
//   delta = 2 (||S - diag(lambda)||_F + max|lambda| ||R||_F),
//   E_ij = (S_ij + lambda_j R_ij) / (lambda_j - lambda_i)   (|lambda_i - lambda_j| > delta)
//   E_ij = R_ij / 2                                          (otherwise, and i == j),
//   Y <- Y (I + E).
// Pairs closer than delta are only re-orthogonalised by that update, never
// rotated apart, and the mixing of near-degenerate vectors left by the FP32
// solve keeps S_ij (hence delta) above their gap, so they would never
// separate.  Each run of consecutive eigenvalues with gaps <= delta (a
// cluster) therefore also takes a Rayleigh-Ritz step inside its span: with
// lambda_c the cluster's mean, M = S_JJ + lambda_c R_JJ is the first-order
// form of the projected pencil (S_JJ, G_JJ), M = W diag(mu) W^H by Jacobi
// rotations in FP64, the cluster's columns of I + E are multiplied by W and
// its eigenvalues become mu (the same rotation inside the cluster's span as
// in Ogita & Aishima's treatment of clustered eigenvalues).
// After the last sweep the refined Y is checked once: a problem whose
// max |(Y^H Y - I)_ij| exceeds 1e-11 gets ST_NOCONV (refinement that has
// converged leaves Y orthonormal to rounding; a pair it failed to separate,
// or too few sweeps, leaves it visibly non-orthogonal).
// The products are the library's MFMA products; G and S are Hermitian, so
// only their lower triangles are formed (G_ij, S_ij for i < j are read as
// conj(G_ji), conj(S_ji)).  These kernels form lambda, the norms behind delta,
// the clusters and I + E.  Every sum is taken in a fixed order.
#include "common.hpp"
#include "lanes.hpp"
#include "kernels.hpp"

namespace kgev {

namespace {

// one workgroup per column j: lambda_j and the column's share of the squared
// Frobenius norms of S - diag(lambda) and R = I - G, from the lower
// triangles (each strictly-lower entry stands for itself and its mirror)
__global__ __launch_bounds__(256) void k_refine_stats(int64_t n, const double2* G, const double2* S, int64_t sNN,
                                                      double* lam, double* pS, double* pR)
{
    __shared__ double sh[8];
    const int64_t b = blockIdx.y, j = blockIdx.x;
    const double2* g = G + b * sNN + j * n;
    const double2* sc = S + b * sNN + j * n;
    const double lj = sc[j].x / g[j].x;
    double as = 0.0, ar = 0.0;
    for (int64_t i = j + threadIdx.x; i < n; i += 256) {
        double2 sv = sc[i], gv = g[i];
        double wgt = 2.0;
        if (i == j) {
            sv.x -= lj;
            sv.y = 0.0;
            gv.x -= 1.0;
            gv.y = 0.0;
            wgt = 1.0;
        }
        as = fma(wgt, fma(sv.x, sv.x, sv.y * sv.y), as);
        ar = fma(wgt, fma(gv.x, gv.x, gv.y * gv.y), ar);
    }
    as = dpp_wave_sum(as);
    ar = dpp_wave_sum(ar);
    if ((threadIdx.x & 63) == 0) { sh[threadIdx.x >> 6] = as; sh[4 + (threadIdx.x >> 6)] = ar; }
    __syncthreads();
    if (threadIdx.x == 0) {
        lam[b * n + j] = lj;
        pS[b * n + j] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        pR[b * n + j] = (sh[4] + sh[5]) + (sh[6] + sh[7]);
    }
}

// one workgroup per problem: delta
__global__ __launch_bounds__(256) void k_refine_delta(int64_t n, const double* lam, const double* pS, const double* pR,
                                                      double* delta)
{
    __shared__ double sh[12];
    const int64_t b = blockIdx.x;
    double s = 0.0, r = 0.0, lm = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        s += pS[b * n + j];
        r += pR[b * n + j];
        lm = fmax(lm, fabs(lam[b * n + j]));
    }
    s = dpp_wave_sum(s);
    r = dpp_wave_sum(r);
    lm = dpp_wave_max(lm);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sh[w] = s; sh[4 + w] = r; sh[8 + w] = lm; }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double ss = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        const double rr = (sh[4] + sh[5]) + (sh[6] + sh[7]);
        const double mx = fmax(fmax(sh[8], sh[9]), fmax(sh[10], sh[11]));
        delta[b] = 2.0 * (sqrt(ss) + mx * sqrt(rr));
    }
}

// Cluster index of every eigenvalue: a new cluster starts at j unless
// |lambda_j - lambda_(j-1)| <= delta (one workgroup per problem, each thread
// a contiguous chunk, the chunks' start counts scanned in LDS).
__global__ __launch_bounds__(256) void k_refine_clusters(int64_t n, const double* lam, const double* delta, int* cid)
{
    __shared__ int sc[256];
    const int64_t b = blockIdx.x;
    const double* l = lam + b * n;
    const double dl = delta[b];
    const int tid = threadIdx.x;
    const int64_t chunk = (n + 255) / 256;
    const int64_t j0 = (int64_t)tid * chunk, j1 = j0 + chunk < n ? j0 + chunk : n;
    int cnt = 0;
    for (int64_t j = j0; j < j1; ++j) cnt += (j == 0 || !(fabs(l[j] - l[j - 1]) <= dl)) ? 1 : 0;
    sc[tid] = cnt;
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int q = 0; q < 256; ++q) {
            const int t = sc[q];
            sc[q] = acc;
            acc += t;
        }
    }
    __syncthreads();
    int g = sc[tid] - 1;
    for (int64_t j = j0; j < j1; ++j) {
        if (j == 0 || !(fabs(l[j] - l[j - 1]) <= dl)) ++g;
        cid[b * n + j] = g;
    }
}

// F = I + E, column-major n x n per problem, one 32 x 32 tile per
// workgroup.  G and S hold lower triangles: a tile above the diagonal reads
// the mirrored lower tile through LDS (coalesced) and conjugates it.
constexpr int RT = 32;
__global__ __launch_bounds__(256) void k_refine_E(int64_t n, const double2* G, const double2* S, int64_t sNN,
                                                  const double* lam, const double* delta, const int* cid, double2* F)
{
    __shared__ double2 tg[RT][RT + 1], ts[RT][RT + 1];
    const int64_t b = blockIdx.z;
    const int64_t i0 = (int64_t)blockIdx.x * RT, j0 = (int64_t)blockIdx.y * RT;
    const bool upper = i0 < j0;        // tile strictly above the diagonal blocks
    const int tx = threadIdx.x & (RT - 1), ty = threadIdx.x / RT;   // 32 x 8
    const double2* g = G + b * sNN;
    const double2* sm = S + b * sNN;
    if (upper) {
        // stage the mirrored tile (rows j0.., columns i0..) as stored
        for (int c = ty; c < RT; c += 8) {
            const int64_t r = j0 + tx, col = i0 + c;
            double2 gv = mk<double>(0, 0), sv = mk<double>(0, 0);
            if (r < n && col < n) {
                gv = g[r + col * n];
                sv = sm[r + col * n];
            }
            tg[c][tx] = gv;
            ts[c][tx] = sv;
        }
        __syncthreads();
    }
    const double dl = delta[b];
    for (int c = ty; c < RT; c += 8) {
        const int64_t i = i0 + tx, j = j0 + c;
        if (i >= n || j >= n) continue;
        double2 gv, sv;
        if (upper) {
            // G_ij = conj(G_ji), G_ji staged at [i - i0][j - j0]
            gv = tg[tx][c];
            sv = ts[tx][c];
            gv.y = -gv.y;
            sv.y = -sv.y;
        } else if (i >= j) {
            gv = g[i + j * n];
            sv = sm[i + j * n];
        } else {
            // inside a diagonal tile, above the diagonal
            gv = g[j + i * n];
            sv = sm[j + i * n];
            gv.y = -gv.y;
            sv.y = -sv.y;
        }
        const double2 r = mk<double>((i == j ? 1.0 : 0.0) - gv.x, -gv.y);   // R = I - G
        const double li = lam[b * n + i], lj = lam[b * n + j];
        double2 e;
        const bool same = cid[b * n + i] == cid[b * n + j];
        if (i != j && !same && fabs(li - lj) > dl) {
            const double den = 1.0 / (lj - li);
            e = mk<double>((sv.x + lj * r.x) * den, (sv.y + lj * r.y) * den);
        } else {
            e = mk<double>(0.5 * r.x, 0.5 * r.y);
        }
        if (i == j) {
            e.x += 1.0;
            e.y = 0.0;
        }
        F[b * sNN + i + j * n] = e;
    }
}

// Rayleigh-Ritz inside one cluster of 2..RR_MAX consecutive eigenvalues (one
// wave per candidate first index j0; the wave that finds j0 opening a cluster
// does the work): M = S_JJ + lambda_c R_JJ in LDS, cyclic Jacobi with complex
// rotations until the off-diagonal part is at the rounding level of M, the
// eigenvalues sorted ascending with their vectors W, then F(:, J) <- F(:, J) W
// and lambda_J <- the sorted eigenvalues.  Larger clusters keep the
// re-orthogonalisation alone.
constexpr int RR_MAX = 32;
__global__ __launch_bounds__(64) void k_refine_rr(int64_t n, const double2* G, const double2* S, int64_t sNN,
                                                  const int* cid, double* lam, double2* F)
{
    __shared__ double2 sa[RR_MAX][RR_MAX + 1];     // sa[r][c] = M(r, c)
    __shared__ double2 sw[RR_MAX][RR_MAX + 1];     // accumulated rotations
    __shared__ int sord[RR_MAX];
    __shared__ double2 srow[RR_MAX][64];           // one row of F(:, J) per lane
    const int64_t b = blockIdx.y, j0 = blockIdx.x;
    const int lane = threadIdx.x;
    const int* cb = cid + b * n;
    const int g = cb[j0];
    if (j0 > 0 && cb[j0 - 1] == g) return;
    int k = 1;
    while (j0 + k < n && k <= RR_MAX && cb[j0 + k] == g) ++k;
    if (k < 2 || k > RR_MAX) return;
    const double2* Gb = G + b * sNN;
    const double2* Sb = S + b * sNN;
    double* lb = lam + b * n;
    double lc = 0.0;
    for (int r = 0; r < k; ++r) lc += lb[j0 + r];
    lc /= (double)k;
    for (int e = lane; e < k * k; e += 64) {
        const int r = e % k, c = e / k;
        const int64_t gi = j0 + r, gj = j0 + c;
        double2 sv, gv;
        if (gi >= gj) {
            sv = Sb[gi + gj * n];
            gv = Gb[gi + gj * n];
        } else {
            sv = cconj(Sb[gj + gi * n]);
            gv = cconj(Gb[gj + gi * n]);
        }
        // M = S + lambda_c (I - G)
        double2 m = mk<double>(fma(lc, (r == c ? 1.0 : 0.0) - gv.x, sv.x), fma(lc, -gv.y, sv.y));
        if (r == c) m.y = 0.0;
        sa[r][c] = m;
        sw[r][c] = mk<double>(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int e = lane; e < k * k; e += 64) {
            const int r = e % k, c = e / k;
            const double2 v = sa[r][c];
            const double a2 = v.x * v.x + v.y * v.y;
            if (r == c) dia += a2; else off += a2;
        }
        off = dpp_wave_sum(off);
        dia = dpp_wave_sum(dia);
        // ||off||_F <= k eps ||diag||_F: the rounding level of a rotation (or NaN)
        if (!(off > (double)(k * k) * 4.93e-32 * dia)) break;
        for (int p = 0; p + 1 < k; ++p)
            for (int q = p + 1; q < k; ++q) {
                const double2 apq = sa[p][q];
                const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
                if (!(mag > 0.0)) continue;                    // the same value in every lane
                const double app = sa[p][p].x, aqq = sa[q][q].x;
                const double tau = (aqq - app) / (2.0 * mag);
                const double t = fabs(tau) < 1e150 ? (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau))
                                                   : 0.5 / tau;
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
                const double2 u = mk<double>(apq.x / mag, apq.y / mag);   // M(p, q) = |M(p, q)| u
                __syncthreads();
                // columns p, q times W2 = [[cs, sn], [-conj(u) sn, conj(u) cs]]
                for (int r = lane; r < k; r += 64) {
                    const double2 x = sa[r][p], y = cmulc(u, sa[r][q]);
                    sa[r][p] = mk<double>(cs * x.x - sn * y.x, cs * x.y - sn * y.y);
                    sa[r][q] = mk<double>(sn * x.x + cs * y.x, sn * x.y + cs * y.y);
                    const double2 xw = sw[r][p], yw = cmulc(u, sw[r][q]);
                    sw[r][p] = mk<double>(cs * xw.x - sn * yw.x, cs * xw.y - sn * yw.y);
                    sw[r][q] = mk<double>(sn * xw.x + cs * yw.x, sn * xw.y + cs * yw.y);
                }
                __syncthreads();
                // rows p, q times W2^H = [[cs, -u sn], [sn, u cs]]
                for (int c = lane; c < k; c += 64) {
                    const double2 x = sa[p][c], y = cmul(u, sa[q][c]);
                    sa[p][c] = mk<double>(cs * x.x - sn * y.x, cs * x.y - sn * y.y);
                    sa[q][c] = mk<double>(sn * x.x + cs * y.x, sn * x.y + cs * y.y);
                }
                __syncthreads();
            }
    }
    if (lane == 0) {
        // ascending order of the diagonal (stable selection)
        bool used[RR_MAX];
        for (int r = 0; r < k; ++r) used[r] = false;
        for (int r = 0; r < k; ++r) {
            int best = -1;
            for (int q = 0; q < k; ++q)
                if (!used[q] && (best < 0 || sa[q][q].x < sa[best][best].x)) best = q;
            used[best] = true;
            sord[r] = best;
        }
    }
    __syncthreads();
    for (int r = lane; r < k; r += 64) lb[j0 + r] = sa[sord[r]][sord[r]].x;
    // F(:, J) <- F(:, J) W (columns of W in ascending order of their eigenvalue)
    // each lane stages its row of F(:, J) in LDS, then overwrites it
    double2* Fb = F + b * sNN;
    for (int64_t i = lane; i < n; i += 64) {
        for (int c = 0; c < k; ++c) srow[c][lane] = Fb[i + (j0 + c) * n];
        for (int c = 0; c < k; ++c) {
            const int src = sord[c];
            double2 acc = mk<double>(0.0, 0.0);
            for (int q = 0; q < k; ++q) acc = cfma(srow[q][lane], sw[q][src], acc);
            Fb[i + (j0 + c) * n] = acc;
        }
    }
}

// the final check: one workgroup per column j of every problem, the largest
// |G_ij - delta_ij| over the stored lower part i >= j
__global__ __launch_bounds__(256) void k_orth_colmax(int64_t n, const double2* G, int64_t sNN, double* pm)
{
    __shared__ double sh[4];
    const int64_t b = blockIdx.y, j = blockIdx.x;
    const double2* g = G + b * sNN + j * n;
    double m = 0.0;
    for (int64_t i = j + threadIdx.x; i < n; i += 256) {
        double2 v = g[i];
        if (i == j) v.x -= 1.0;
        const double a = fmax(fabs(v.x), fabs(v.y));
        m = (a > m || a != a) ? a : m;      // a NaN is kept
    }
    m = dpp_wave_max(m);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int q = 1; q < 4; ++q) t = (sh[q] > t || sh[q] != sh[q]) ? sh[q] : t;
        pm[b * n + j] = t;
    }
}

__global__ __launch_bounds__(256) void k_orth_flag(int64_t n, const double* pm, int* status, double tol)
{
    __shared__ int bad;
    const int64_t b = blockIdx.x;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int64_t j = threadIdx.x; j < n; j += 256)
        if (!(pm[b * n + j] <= tol)) bad = 1;
    __syncthreads();
    if (threadIdx.x == 0 && bad) atomicOr(status + b, ST_NOCONV);
}

__global__ __launch_bounds__(256) void k_f2d(const float* src, double* dst, int64_t count)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q < count) dst[q] = (double)src[q];
}

__global__ __launch_bounds__(256) void k_c64_to_c128(const float2* src, double2* dst, int64_t count)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q < count) dst[q] = mk<double>((double)src[q].x, (double)src[q].y);
}

}  // namespace

hipError_t float_to_double(hipStream_t st, const float* src, double* dst, int64_t count)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_f2d, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, src, dst, count);
    return hipGetLastError();
}

hipError_t c64_to_c128(hipStream_t st, const float2* src, double2* dst, int64_t count)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_c64_to_c128, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, src, dst, count);
    return hipGetLastError();
}

hipError_t refine(hipStream_t st, const RefineWs& ws, int64_t nk, int iters, double* lam_out)
{
    const int64_t n = ws.n, nn = n * n;
    const double2 one = mk<double>(1, 0), zero = mk<double>(0, 0);
    double2* Y = ws.Y;
    double2* Yn = ws.Ynext;
    for (int it = 0; it < iters; ++it) {
        hipError_t e;
        e = cgemm<double>(st, 'C', 'N', n, n, n, one, Y, n, nn, Y, n, nn, zero, ws.G, n, nn, nk, true);
        if (e != hipSuccess) return e;
        e = cgemm<double>(st, 'N', 'N', n, n, n, one, ws.Af, n, nn, Y, n, nn, zero, ws.P, n, nn, nk, false);
        if (e != hipSuccess) return e;
        e = cgemm<double>(st, 'C', 'N', n, n, n, one, Y, n, nn, ws.P, n, nn, zero, ws.S, n, nn, nk, true);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_refine_stats, dim3((unsigned)n, (unsigned)nk), dim3(256), 0, st, n, ws.G, ws.S, nn,
                           lam_out, ws.pS, ws.pR);
        hipLaunchKernelGGL(k_refine_delta, dim3((unsigned)nk), dim3(256), 0, st, n, lam_out, ws.pS, ws.pR, ws.delta);
        hipLaunchKernelGGL(k_refine_clusters, dim3((unsigned)nk), dim3(256), 0, st, n, lam_out, ws.delta, ws.cid);
        hipLaunchKernelGGL(k_refine_E, dim3((unsigned)((n + RT - 1) / RT), (unsigned)((n + RT - 1) / RT), (unsigned)nk),
                           dim3(256), 0, st, n, ws.G, ws.S, nn, lam_out, ws.delta, ws.cid, ws.F);
        hipLaunchKernelGGL(k_refine_rr, dim3((unsigned)n, (unsigned)nk), dim3(64), 0, st, n, ws.G, ws.S, nn, ws.cid,
                           lam_out, ws.F);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = cgemm<double>(st, 'N', 'N', n, n, n, one, Y, n, nn, ws.F, n, nn, zero, Yn, n, nn, nk, false);
        if (e != hipSuccess) return e;
        double2* t = Y;
        Y = Yn;
        Yn = t;
    }
    // the final check of orthonormality
    if (ws.status) {
        hipError_t e = cgemm<double>(st, 'C', 'N', n, n, n, one, Y, n, nn, Y, n, nn, zero, ws.G, n, nn, nk, true);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_orth_colmax, dim3((unsigned)n, (unsigned)nk), dim3(256), 0, st, n, ws.G, nn, ws.pR);
        hipLaunchKernelGGL(k_orth_flag, dim3((unsigned)nk), dim3(256), 0, st, n, ws.pR, ws.status, 1e-11);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // the refined vectors end in ws.Y
    if (Y != ws.Y) {
        hipError_t e = hipMemcpyAsync(ws.Y, Y, sizeof(double2) * (size_t)nn * nk, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace kgev
