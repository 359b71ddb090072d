// Band_DFT_Col Part 1 (k-point dependence of H and S, arXiv:1402.4247, the
// routine's outline in the section applying the method to OpenMX), as the
// Bloch sum of real-space blocks:
//   M(k)_{IJ} = sum over the blocks (I, J, R) of exp(2 pi i k.R) M_{IJ}(R),
// k and R in fractional coordinates.  The blocks come sorted by atom pair;
// one workgroup sums every block of its pair, in block order, for all
// k-points.  The phases are tabulated first (nk x nR values).
#include "common.hpp"
#include "kernels.hpp"

namespace kgev {

namespace {

__global__ __launch_bounds__(256) void k_phase_table(int64_t nk, int64_t nR, const double* kf, const double* R,
                                                     double2* ph)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= nk * nR) return;
    const int64_t k = q / nR, r = q % nR;
    const double t = 2.0 * M_PI * (kf[3 * k] * R[3 * r] + kf[3 * k + 1] * R[3 * r + 1] + kf[3 * k + 2] * R[3 * r + 2]);
    double s, c;
    sincos(t, &s, &c);
    ph[q] = mk<double>(c, s);
}

// group g: blocks gptr[g] .. gptr[g+1]-1, all of atom pair (bi, bj)
__global__ __launch_bounds__(256) void k_bloch(int n, const int* off, const int* gptr, const int* bi, const int* bj,
                                               const int* rid, const int64_t* doff, const double2* data, int64_t nR,
                                               const double2* ph, int64_t nk, double2* out)
{
    const int g = blockIdx.x;
    const int q0 = gptr[g], q1 = gptr[g + 1];
    if (q1 <= q0) return;
    const int I = bi[q0], J = bj[q0];
    const int I0 = off[I], ni = off[I + 1] - I0;
    const int J0 = off[J], nj = off[J + 1] - J0;
    const int64_t nn = (int64_t)n * n;
    for (int e = threadIdx.x; e < ni * nj; e += 256) {
        const int a = e % ni, c = e / ni;
        double2* o = out + (int64_t)(I0 + a) + (int64_t)(J0 + c) * n;
        for (int64_t k = 0; k < nk; ++k) {
            double2 acc = mk<double>(0, 0);
            for (int q = q0; q < q1; ++q) acc = cfma(ph[k * nR + rid[q]], data[doff[q] + e], acc);
            o[k * nn] = acc;
        }
    }
}

}  // namespace

hipError_t bloch_sum(hipStream_t st, int n, const int* off, int64_t ngroups, const int* gptr, const int* bi,
                     const int* bj, const int* rid, const int64_t* doff, const double2* data, int64_t nR,
                     const double* R, int64_t nk, const double* kf, double2* ph, double2* out)
{
    hipError_t e = fill_zero(st, out, sizeof(double2) * (size_t)n * n * nk);
    if (e != hipSuccess) return e;
    if (nR > 0) {
        hipLaunchKernelGGL(k_phase_table, dim3((unsigned)((nk * nR + 255) / 256)), dim3(256), 0, st, nk, nR, kf, R, ph);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (ngroups > 0)
        hipLaunchKernelGGL(k_bloch, dim3((unsigned)ngroups), dim3(256), 0, st, n, off, gptr, bi, bj, rid, doff, data, nR,
                           ph, nk, out);
    return hipGetLastError();
}

}  // namespace kgev
