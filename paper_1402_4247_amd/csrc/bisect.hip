// Eigenvalues only of real symmetric tridiagonal matrices, by bisection on
// Sturm counts: the values-only form of the tridiagonal step of Eigen_HH
// (Section III of arXiv:1402.4247; Band_DFT_Col's first pass over the
// k-points needs the eigenvalues only).
//
// By Sylvester's law of inertia the number of eigenvalues of T below x is the
// number of negative pivots of T - x I = L D L^T, whose pivots follow
//   q_0 = d_0 - x,   q_i = (d_i - x) - e_{i-1}^2 / q_{i-1},
// a pivot of magnitude below pivmin being replaced by -pivmin (so no division
// by zero; the count stays that of a matrix within rounding of T).  T is first
// scaled to max |entry| = 1, and every eigenvalue starts from the Gershgorin
// interval of the scaled T.  Four lanes share eigenvalue j: each round they
// count at the three quarter points of its interval [lo, hi] (count(lo) <= j <
// count(hi)) and keep the quarter that still brackets it, so the interval
// shrinks four-fold per round, until it holds no representable midpoint
// besides its ends, is within 2 eps of its magnitude, or is narrower than
// 2 eps in the scaled units (the absolute accuracy of any backward-stable
// solve, eps ||T||, which is all there is near zero); an eigenvalue that ends
// within 2 eps of zero is zero.  Every step is a fixed sequence of IEEE
// operations, so the results are reproducible bit for bit.
#include "common.hpp"
#include "lanes.hpp"
#include "kernels.hpp"

namespace kgev {

namespace {

constexpr double EPS = 2.220446049250313e-16;
constexpr double SAFMIN = 2.2250738585072014e-308;
constexpr int LANES = 4;        // lanes per eigenvalue
constexpr int MAX_ROUNDS = 40;  // 4^40 = 2^80 > the 2^64 steps between any two doubles

// per problem: scale, Gershgorin interval of the scaled T, pivmin
struct BzPrep {
    double scale, gl, gu, pivmin;
};

__global__ __launch_bounds__(256) void stebz_prep(const double* __restrict__ d, const double* __restrict__ e,
                                                  int64_t sde, int n, BzPrep* prep)
{
    __shared__ double sh[4][4];
    const int64_t b = blockIdx.x;
    const double* db = d + b * sde;
    const double* eb = e + b * sde;
    const int tid = threadIdx.x, w = tid >> 6;
    double mx = 0.0;
    for (int i = tid; i < n; i += 256) {
        mx = fmax(mx, fabs(db[i]));
        if (i + 1 < n) mx = fmax(mx, fabs(eb[i]));
    }
    mx = dpp_wave_max(mx);
    if ((tid & 63) == 0) sh[0][w] = mx;
    __syncthreads();
    double s = fmax(fmax(sh[0][0], sh[0][1]), fmax(sh[0][2], sh[0][3]));
    if (!(s > 0.0)) s = 1.0;
    const double inv = 1.0 / s;
    double lo = 1e300, hi = -1e300, e2 = 0.0;
    for (int i = tid; i < n; i += 256) {
        const double el = i > 0 ? fabs(eb[i - 1]) * inv : 0.0;
        const double er = i + 1 < n ? fabs(eb[i]) * inv : 0.0;
        const double di = db[i] * inv;
        lo = fmin(lo, di - el - er);
        hi = fmax(hi, di + el + er);
        e2 = fmax(e2, er * er);
    }
    lo = -dpp_wave_max(-lo);
    hi = dpp_wave_max(hi);
    e2 = dpp_wave_max(e2);
    __syncthreads();
    if ((tid & 63) == 0) {
        sh[1][w] = lo;
        sh[2][w] = hi;
        sh[3][w] = e2;
    }
    __syncthreads();
    if (tid == 0) {
        const double gl = fmin(fmin(sh[1][0], sh[1][1]), fmin(sh[1][2], sh[1][3]));
        const double gu = fmax(fmax(sh[2][0], sh[2][1]), fmax(sh[2][2], sh[2][3]));
        const double em = fmax(fmax(sh[3][0], sh[3][1]), fmax(sh[3][2], sh[3][3]));
        const double pivmin = SAFMIN * fmax(1.0, em);
        // widen by the rounding of the Gershgorin sums so count(gl) = 0 and
        // count(gu) = n hold for the computed counts too
        const double tn = fmax(fabs(gl), fabs(gu));
        const double pad = 2.0 * EPS * tn * (double)n + 2.0 * pivmin;
        BzPrep p;
        p.scale = s;
        p.gl = gl - pad;
        p.gu = gu + pad;
        p.pivmin = pivmin;
        prep[b] = p;
    }
}

// number of eigenvalues of the scaled T below x
__device__ inline int sturm_count(const double* __restrict__ d, const double* __restrict__ e, int n, double inv,
                                  double x, double pivmin)
{
    double q = d[0] * inv - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0 ? 1 : 0;
    for (int i = 1; i < n; ++i) {
        const double ei = e[i - 1] * inv;
        q = (d[i] * inv - x) - ei * ei / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0 ? 1 : 0;
    }
    return c;
}

// grid (ceil(n * LANES / 256), nk): lanes 4j..4j+3 of the grid row own
// eigenvalue j of problem blockIdx.y
__global__ __launch_bounds__(256) void stebz_bisect(const double* __restrict__ d, const double* __restrict__ e,
                                                    int64_t sde, int n, const BzPrep* __restrict__ prep,
                                                    double* __restrict__ w, int64_t sw)
{
    const int64_t b = blockIdx.y;
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int j = t / LANES, q = t % LANES;
    const bool live = j < n;
    const int jc = live ? j : n - 1;
    const double* db = d + b * sde;
    const double* eb = e + b * sde;
    const BzPrep p = prep[b];
    const double inv = 1.0 / p.scale;
    double lo = p.gl, hi = p.gu;
    for (int r = 0; r < MAX_ROUNDS; ++r) {
        const double width = hi - lo;
        const double mid = 0.5 * (lo + hi);
        // converged: within 2 eps of the magnitude (at least 2 eps absolute in
        // the scaled units), or no point strictly inside
        const bool done = width <= 2.0 * EPS * fmax(fmax(fabs(lo), fabs(hi)), 1.0) || mid <= lo || mid >= hi;
        // every lane of the group takes the same decision (same lo, hi)
        if (done) break;
        double x = lo + width * (double)(q + 1) * 0.25;
        if (q == 1) x = mid;                       // the midpoint exactly
        x = fmin(fmax(x, lo), hi);
        const int c = q < 3 ? sturm_count(db, eb, n, inv, x, p.pivmin) : 0;
        // gather the group's three points and counts (quad_perm broadcasts of
        // lanes 0, 1, 2 of the quad)
        const double xs[3] = {quad_bcast<0>(x), quad_bcast<1>(x), quad_bcast<2>(x)};
        const int cs[3] = {quad_bcast<0>(c), quad_bcast<1>(c), quad_bcast<2>(c)};
        double nlo = lo, nhi = hi;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (cs[k] <= jc) nlo = fmax(nlo, xs[k]);
        }
#pragma unroll
        for (int k = 2; k >= 0; --k) {
            if (cs[k] > jc) nhi = fmin(nhi, xs[k]);
        }
        if (nhi < nlo) nhi = nlo;                  // counts not monotone by rounding: keep a valid interval
        lo = nlo;
        hi = nhi;
    }
    // an eigenvalue within the absolute resolution of zero is zero
    double x = 0.5 * (lo + hi);
    if (fabs(x) <= 2.0 * EPS) x = 0.0;
    if (live && q == 0) w[b * sw + j] = x * p.scale;
}

}  // namespace

size_t stebz_work_bytes(int64_t nk) { return sizeof(BzPrep) * (size_t)nk; }

hipError_t stebz(hipStream_t st, const double* d, const double* e, int64_t sde, int64_t n, int64_t nk, double* w,
                 int64_t sw, void* work)
{
    if (n < 1 || nk < 1) return hipSuccess;
    BzPrep* prep = static_cast<BzPrep*>(work);
    hipLaunchKernelGGL(stebz_prep, dim3((unsigned)nk), dim3(256), 0, st, d, e, sde, (int)n, prep);
    const unsigned gx = (unsigned)((n * LANES + 255) / 256);
    hipLaunchKernelGGL(stebz_bisect, dim3(gx, (unsigned)nk), dim3(256), 0, st, d, e, sde, (int)n, prep, w, sw);
    return hipGetLastError();
}

}  // namespace kgev
