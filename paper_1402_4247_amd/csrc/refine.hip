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
// The products are the library's MFMA products; G and S are Hermitian, so
// only their lower triangles are formed (G_ij, S_ij for i < j are read as
// conj(G_ji), conj(S_ji)).  These kernels form lambda, the norms behind delta
// and I + E.  Every sum is taken in a fixed order.
#include "common.hpp"
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
    as = wave_sum(as);
    ar = wave_sum(ar);
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
    s = wave_sum(s);
    r = wave_sum(r);
    lm = wave_max(lm);
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

// F = I + E, column-major n x n per problem, one 32 x 32 tile per
// workgroup.  G and S hold lower triangles: a tile above the diagonal reads
// the mirrored lower tile through LDS (coalesced) and conjugates it.
constexpr int RT = 32;
__global__ __launch_bounds__(256) void k_refine_E(int64_t n, const double2* G, const double2* S, int64_t sNN,
                                                  const double* lam, const double* delta, double2* F)
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
        if (i != j && fabs(li - lj) > dl) {
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
        hipLaunchKernelGGL(k_refine_E, dim3((unsigned)((n + RT - 1) / RT), (unsigned)((n + RT - 1) / RT), (unsigned)nk),
                           dim3(256), 0, st, n, ws.G, ws.S, nn, lam_out, ws.delta, ws.F);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = cgemm<double>(st, 'N', 'N', n, n, n, one, Y, n, nn, ws.F, n, nn, zero, Yn, n, nn, nk, false);
        if (e != hipSuccess) return e;
        double2* t = Y;
        Y = Yn;
        Yn = t;
    }
    // the refined vectors end in ws.Y
    if (Y != ws.Y) {
        hipError_t e = hipMemcpyAsync(ws.Y, Y, sizeof(double2) * (size_t)nn * nk, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace kgev
