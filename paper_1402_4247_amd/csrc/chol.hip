// Part 2 in Cholesky form (an option beside the paper's diagonalisation of S):
// S = L L^H, X = L^{-H} J, which satisfies X^H S X = I, so Parts 3 and 4 run
// unchanged with this X.  Blocked in 64-column steps, batched over k-points:
//   diagonal block : one workgroup per k factors it in LDS (right-looking,
//                    pivots checked against s_tol * max_i S_ii) and inverts
//                    the factor (forward substitution);
//   panel          : L21 = A21 L11^{-H}                 (MFMA product)
//   trailing       : A22 -= L21 L21^H, lower half        (MFMA product)
// then L^{-1} block row by block row,
//   L^{-1}(i, 0:i) = -L_ii^{-1} (L(i, 0:i) L^{-1}(0:i, 0:i)),
// and X = (L^{-1})^H J with J the reversal of the column order.  Any X with
// X^H S X = I serves Parts 3 and 4; the reversal matters for accuracy when S
// is ill-conditioned: the large entries of L^{-1} sit in its last rows (the
// small pivots come last), so A = X^H H X without J is large in its
// lower-right corner, which a Householder reduction starting from the first
// column spreads over every eigenvalue (about eps ||A|| each).  With J the
// large entries come first, where the reduction keeps them apart (graded
// from the top).  On an LCAO pencil with smallest overlap eigenvalue 1e-6 the
// unreversed form missed the first-order bound of a backward-stable solve by
// 11x in the oracle's own Householder reduction; reversed it is within 1%.
#include <algorithm>

#include "common.hpp"
#include "lanes.hpp"
#include "kernels.hpp"

namespace kgev {

namespace {

constexpr int CB = 64;

__global__ __launch_bounds__(256) void k_smax(int64_t n, const double2* A, int64_t lda, int64_t sA, double* smax)
{
    __shared__ double sh[4];
    const int64_t b = blockIdx.x;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, A[b * sA + i + i * lda].x);
    m = dpp_wave_max(m);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) smax[b] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// Factor and invert the diagonal block at j0 of every k-point.  Writes the
// factor into L (lower, ld n), its inverse into Linv (ld n) and into D
// (ld CB, one CB x CB block per k).  A failing pivot sets ST_NOTPD and is
// replaced by 1 so that the rest stays finite.
__global__ __launch_bounds__(256) void k_chol_diag(int n, int j0, const double2* A, int64_t lda, int64_t sA,
                                                   double2* L, double2* Linv, int64_t sN, double2* D, int64_t sD,
                                                   const double* smax, double s_tol, int* status)
{
    __shared__ double2 a[CB][CB + 1];   // a[col][row]
    __shared__ double2 v[CB][CB + 1];   // inverse, v[col][row]
    __shared__ int bad;
    const int64_t b = blockIdx.x;
    const int bs = n - j0 < CB ? n - j0 : CB;
    const int tid = threadIdx.x;
    const double2* Ab = A + b * sA + (int64_t)j0 + (int64_t)j0 * lda;
    for (int e = tid; e < CB * CB; e += 256) {
        const int r = e % CB, c = e / CB;
        double2 x = mk<double>(0, 0);
        if (r < bs && c <= r) x = Ab[r + (int64_t)c * lda];
        a[c][r] = x;
        v[c][r] = mk<double>(0, 0);
    }
    if (tid == 0) bad = 0;
    const double thr = s_tol * smax[b];
    __syncthreads();
    for (int c = 0; c < bs; ++c) {
        if (tid == 0) {
            double d = a[c][c].x;
            if (!(d > thr)) {
                bad = 1;
                d = 1.0;
            }
            a[c][c] = mk<double>(sqrt(d), 0.0);
        }
        __syncthreads();
        const double inv = 1.0 / a[c][c].x;
        for (int r = c + 1 + tid; r < bs; r += 256) a[c][r] = cscale(a[c][r], inv);
        __syncthreads();
        // trailing lower part: a[c2][r] -= a[c][r] conj(a[c][c2]), c < c2 <= r
        const int t = bs - c - 1;
        for (int e = tid; e < t * t; e += 256) {
            const int r = c + 1 + e % t, c2 = c + 1 + e / t;
            if (c2 <= r) a[c2][r] = csub(a[c2][r], cmulc(a[c][c2], a[c][r]));
        }
        __syncthreads();
    }
    // inverse by rows: v(r, cc) = (delta - sum_{k=cc}^{r-1} L(r, k) v(k, cc)) / L(r, r),
    // the four threads of a column splitting the sum
    const int cc = tid >> 2, part = tid & 3;
    for (int r = 0; r < bs; ++r) {
        double2 s = mk<double>(0, 0);
        if (cc <= r && cc < bs)
            for (int k = cc + part; k < r; k += 4) s = cfma(a[k][r], v[cc][k], s);
        s.x = dpp_sum<4>(s.x);
        s.y = dpp_sum<4>(s.y);
        if (part == 0 && cc <= r && cc < bs) {
            const double2 dl = mk<double>(r == cc ? 1.0 : 0.0, 0.0);
            v[cc][r] = cscale(csub(dl, s), 1.0 / a[r][r].x);
        }
        __syncthreads();
    }
    double2* Lb = L + b * sN + (int64_t)j0 + (int64_t)j0 * n;
    double2* Vb = Linv + b * sN + (int64_t)j0 + (int64_t)j0 * n;
    double2* Db = D + b * sD;
    for (int e = tid; e < CB * CB; e += 256) {
        const int r = e % CB, c = e / CB;
        if (r < bs && c < bs) {
            Lb[r + (int64_t)c * n] = a[c][r];
            Vb[r + (int64_t)c * n] = v[c][r];
        }
        Db[r + (int64_t)c * CB] = v[c][r];
    }
    if (tid == 0 && bad) atomicOr(status + b, ST_NOTPD);
}

// X = M^H J (n x n, ld n): X(r, n - 1 - c) = conj(M(c, r))
__global__ __launch_bounds__(256) void k_conj_transpose_rev(int64_t n, const double2* M, double2* X, int64_t sN)
{
    __shared__ double2 t[32][33];
    const int64_t b = blockIdx.z;
    const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int c = ty; c < 32; c += 8) {
        const int64_t r = i0 + tx, col = j0 + c;
        double2 x = mk<double>(0, 0);
        if (r < n && col < n) x = M[b * sN + r + col * n];
        t[c][tx] = x;
    }
    __syncthreads();
    for (int c = ty; c < 32; c += 8) {
        const int64_t r = j0 + tx, col = i0 + c;    // X(r, n - 1 - col) = conj(M(col, r))
        if (r < n && col < n) X[b * sN + r + (n - 1 - col) * n] = cconj(t[tx][c]);
    }
}

}  // namespace

// per k-point: the inverted diagonal blocks (nblk x CB x CB) and one CB x n
// block row of temporaries
int64_t chol_work_elems(int64_t n) { return ((n + CB - 1) / CB) * CB * CB + (int64_t)CB * n; }

hipError_t cholesky_x(hipStream_t st, int64_t n, double2* A, int64_t lda, int64_t sA, double2* L, double2* Linv,
                      double2* X, double2* work, double* smax, double s_tol, int* status, int64_t nk)
{
    const int64_t sN = n * n;
    const int64_t sW = chol_work_elems(n);
    double2* D = work;
    double2* Tw = work + ((n + CB - 1) / CB) * CB * CB;
    const double2 one = mk<double>(1, 0), zero = mk<double>(0, 0), mone = mk<double>(-1, 0);
    hipError_t e = fill_zero(st, L, sizeof(double2) * (size_t)sN * nk);
    if (e != hipSuccess) return e;
    e = fill_zero(st, Linv, sizeof(double2) * (size_t)sN * nk);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_smax, dim3((unsigned)nk), dim3(256), 0, st, n, A, lda, sA, smax);
    const int64_t nblk = (n + CB - 1) / CB;
    const int64_t sD = sW;
    for (int64_t q = 0; q < nblk; ++q) {
        const int64_t j0 = q * CB, bs = std::min<int64_t>(CB, n - j0), m = n - j0 - bs;
        double2* Dq = D + q * CB * CB;
        hipLaunchKernelGGL(k_chol_diag, dim3((unsigned)nk), dim3(256), 0, st, (int)n, (int)j0, A, lda, sA, L, Linv,
                           sN, Dq, sD, smax, s_tol, status);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (m <= 0) continue;
        // L21 = A21 L11^{-H}
        e = cgemm<double>(st, 'N', 'C', m, bs, bs, one, A + (j0 + bs) + j0 * lda, lda, sA, Dq, CB, sD, zero,
                          L + (j0 + bs) + j0 * n, n, sN, nk, false);
        if (e != hipSuccess) return e;
        // A22 -= L21 L21^H (lower)
        e = cgemm<double>(st, 'N', 'C', m, m, bs, mone, L + (j0 + bs) + j0 * n, n, sN, L + (j0 + bs) + j0 * n, n, sN,
                          one, A + (j0 + bs) + (j0 + bs) * lda, lda, sA, nk, true);
        if (e != hipSuccess) return e;
    }
    // L^{-1} below the diagonal blocks, block row by block row
    for (int64_t q = 1; q < nblk; ++q) {
        const int64_t i0 = q * CB, bi = std::min<int64_t>(CB, n - i0);
        e = cgemm<double>(st, 'N', 'N', bi, i0, i0, one, L + i0, n, sN, Linv, n, sN, zero, Tw, CB, sW, nk, false);
        if (e != hipSuccess) return e;
        e = cgemm<double>(st, 'N', 'N', bi, i0, bi, mone, D + q * CB * CB, CB, sD, Tw, CB, sW, zero, Linv + i0, n, sN,
                          nk, false);
        if (e != hipSuccess) return e;
    }
    const unsigned tb = (unsigned)((n + 31) / 32);
    hipLaunchKernelGGL(k_conj_transpose_rev, dim3(tb, tb, (unsigned)nk), dim3(256), 0, st, n, Linv, X, sN);
    return hipGetLastError();
}

}  // namespace kgev
