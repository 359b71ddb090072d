// Band_DFT_Col Parts 5 and 6 (the steps around the per-k solve in the
// routine's outline, arXiv:1402.4247, Section "Application to OpenMX"):
//   Part 5: chemical potential mu and band energy from the eigenvalues of
//           all k-points, with Fermi-Dirac occupations at temperature kT,
//           f_kj = 1 / (1 + exp((lambda_kj - mu) / kT)), mu the root of
//           g sum_k wk_k sum_j f_kj = nelec found by bisection;
//   Part 6: charge density matrix rho = g sum_k wk_k C_k diag(f_k) C_k^H and
//           energy density matrix with weights f_kj lambda_kj (lower
//           triangles), as one batched MFMA product per matrix plus a
//           fixed-order sum over k-points.
#include "common.hpp"
#include "lanes.hpp"
#include "kernels.hpp"
#include "../../include/kgev.h"

namespace kgev {

namespace {

constexpr int FT = 1024;          // threads of the Fermi-level workgroup
constexpr int FW = FT / WAVE;

__device__ inline double fermi_dirac(double x, double mu, double kT)
{
    const double t = (x - mu) / kT;
    if (t > 0.0) {
        const double e = exp(-t);
        return e / (1.0 + e);
    }
    return 1.0 / (1.0 + exp(t));
}

// fixed-order sum of one value per thread over the workgroup; every thread
// gets the result
__device__ inline double block_sum(double v, double* sh)
{
    v = dpp_wave_sum(v);
    const int w = threadIdx.x / WAVE;
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < FW; ++q) s += sh[q];
    return s;
}

__device__ inline double block_min(double v, double* sh)
{
    v = dpp_wave_min(v);
    const int w = threadIdx.x / WAVE;
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) sh[w] = v;
    __syncthreads();
    double s = sh[0];
#pragma unroll
    for (int q = 1; q < FW; ++q) s = fmin(s, sh[q]);
    return s;
}

// One workgroup: bracket, bisection (every thread takes the same decision
// from the same block sum), then occupations, band energy and final count.
// out = {mu, e_band, n_count}; status = 0, or KGEV_ERANGE when nelec is not
// inside (0, g n sum wk).
__global__ __launch_bounds__(FT) void k_fermi(const double* __restrict__ w, int64_t ldw, int n, int nk,
                                              const double* __restrict__ wk, double nelec, double kT, double g,
                                              double* occ, int64_t ldo, double* out, int32_t* status)
{
    __shared__ double sh[FW];
    double lo = INFINITY, hi = INFINITY, ws = 0.0;
    for (int k = 0; k < nk; ++k)
        for (int j = threadIdx.x; j < n; j += FT) {
            const double x = w[(int64_t)k * ldw + j];
            lo = fmin(lo, x);
            hi = fmin(hi, -x);
        }
    for (int k = threadIdx.x; k < nk; k += FT) ws += wk[k];
    lo = block_min(lo, sh);
    hi = -block_min(hi, sh);
    ws = block_sum(ws, sh);
    if (!(nelec > 0.0) || !(nelec < g * (double)n * ws)) {
        if (threadIdx.x == 0) *status = KGEV_ERANGE;
        return;
    }
    lo -= 50.0 * kT;
    hi += 50.0 * kT;
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        double s = 0.0;
        for (int k = 0; k < nk; ++k) {
            double t = 0.0;
            for (int j = threadIdx.x; j < n; j += FT) t += fermi_dirac(w[(int64_t)k * ldw + j], mid, kT);
            s = fma(wk[k], t, s);
        }
        const double cnt = g * block_sum(s, sh);
        if (cnt < nelec) lo = mid;
        else hi = mid;
    }
    const double mu = 0.5 * (lo + hi);
    double sc = 0.0, se = 0.0;
    for (int k = 0; k < nk; ++k) {
        double tc = 0.0, te = 0.0;
        for (int j = threadIdx.x; j < n; j += FT) {
            const double x = w[(int64_t)k * ldw + j];
            const double f = fermi_dirac(x, mu, kT);
            if (occ) occ[(int64_t)k * ldo + j] = f;
            tc += f;
            te = fma(f, x, te);
        }
        sc = fma(wk[k], tc, sc);
        se = fma(wk[k], te, se);
    }
    sc = block_sum(sc, sh);
    se = block_sum(se, sh);
    if (threadIdx.x == 0) {
        out[0] = mu;
        out[1] = g * se;
        out[2] = g * sc;
        *status = KGEV_OK;
    }
}

// Scaled copy for the density products: Cs_k(:, j) = g wk_k f_kj [lambda_kj] C_k(:, j)
// for j < nocc (column-major, ld n, k-stride n * nocc).
__global__ __launch_bounds__(256) void k_density_scale(const double2* __restrict__ C, int64_t ldc, int n, int nocc,
                                                       const double* __restrict__ w, int64_t ldw,
                                                       const double* __restrict__ occ, int64_t ldo,
                                                       const double* __restrict__ wk, double g, int energy,
                                                       double2* __restrict__ Cs)
{
    const int64_t k = blockIdx.z, j = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = g * wk[k] * occ[k * ldo + j];
    if (energy) s *= w[k * ldw + j];
    const double2 c = C[k * ldc * n + j * ldc + i];
    Cs[(k * nocc + j) * n + i] = mk<double>(s * c.x, s * c.y);
}

// out(lower) = sum over the nk partial products in k order
__global__ __launch_bounds__(256) void k_sum_partials(const double2* __restrict__ P, int n, int nk,
                                                      double2* __restrict__ out, int64_t ldr)
{
    const int64_t b = blockIdx.y;
    const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (a >= n || a < b) return;
    const int64_t nn = (int64_t)n * n;
    double2 s = P[a + b * n];
    for (int k = 1; k < nk; ++k) s = cadd(s, P[k * nn + a + b * n]);
    out[a + b * ldr] = s;
}

}  // namespace

hipError_t fermi_level(hipStream_t st, const double* w, int64_t ldw, int n, int nk, const double* wk, double nelec,
                       double kT, double g, double* occ, int64_t ldo, double* out, int32_t* status)
{
    hipLaunchKernelGGL(k_fermi, dim3(1), dim3(FT), 0, st, w, ldw, n, nk, wk, nelec, kT, g, occ, ldo, out, status);
    return hipGetLastError();
}

size_t density_work_bytes(int64_t n, int64_t nk, int64_t nocc)
{
    const size_t cs = sizeof(double2) * (size_t)n * (size_t)nocc * (size_t)nk;
    const size_t pr = sizeof(double2) * (size_t)n * (size_t)n * (size_t)nk;
    return ((cs + 255) & ~(size_t)255) + pr;
}

hipError_t density(hipStream_t st, const double2* C, int64_t ldc, int n, int nk, int nocc, const double* w,
                   int64_t ldw, const double* occ, int64_t ldo, const double* wk, double g, double2* rho,
                   double2* edm, int64_t ldr, void* work)
{
    double2* Cs = static_cast<double2*>(work);
    const size_t cs = sizeof(double2) * (size_t)n * (size_t)nocc * (size_t)nk;
    double2* P = reinterpret_cast<double2*>(static_cast<char*>(work) + ((cs + 255) & ~(size_t)255));
    const int64_t nn = (int64_t)n * n;
    const double2 one = mk<double>(1, 0), zero = mk<double>(0, 0);
    for (int pass = 0; pass < 2; ++pass) {
        double2* out = pass == 0 ? rho : edm;
        if (!out) continue;
        if (nocc > 0) {
            hipLaunchKernelGGL(k_density_scale, dim3((unsigned)((n + 255) / 256), (unsigned)nocc, (unsigned)nk),
                               dim3(256), 0, st, C, ldc, n, nocc, w, ldw, occ, ldo, wk, g, pass, Cs);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        // P_k = Cs_k C_k^H (lower), one batched product over the k-points
        hipError_t e = cgemm<double>(st, 'N', 'C', n, n, nocc, one, Cs, n, (int64_t)n * nocc, C, ldc, ldc * n,
                                     zero, P, n, nn, nk, true);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256), 0, st, P, n,
                           nk, out, ldr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace kgev
