// Systems of uneven order in one batched solve: the k-points of several
// pencils of orders n_q <= N are embedded in pencils of one order N,
//   H' = [[H, 0], [0, 0]],   S' = [[S, 0], [0, s_pad I]],
// solved together (every launch of the solve covering all of them), and the
// pencil's own eigenpairs taken back out.
//
// Why the embedded eigenpairs are exact: every step of the solve keeps the
// two blocks apart in exact zeros, provided the padded directions stay
// contiguous.  In the paper's form (S diagonalised, eigenvalues ascending)
// s_pad = 2 ||S||_F exceeds every eigenvalue of S, so the padded directions
// of S come last and X' = diag(X, s_pad^-1/2 I); in the Cholesky form
// (no ordering; s_pad = max_i S_ii keeps the pivot threshold) L' = diag(L,
// s_pad^1/2 I) and the column reversal puts them first.  Either way A' is
// A bordered by an exact zero block: its Householder columns there are zero
// below the diagonal (tau = 0, e = 0), the reflectors of the pencil's columns
// are zero on the padded rows, the products only add exact zero terms, and
// the divide and conquer meets a zero off-diagonal at the boundary (its
// rank-one correction is zero, so every padded component is deflated and
// never rotated).  So the padded eigenvalues are exactly 0, their
// eigenvectors live on the padded rows only, and the pencil's eigenvectors
// are the columns that vanish there.  The definiteness test compares s_min
// with s_tol times the largest of the pencil's own eigenvalues of S.
//
// Descriptors travel by value in the kernel arguments (so a captured graph
// holds them), at most BATCH_DESC problems per launch.
#include "common.hpp"
#include "lanes.hpp"
#include "kernels.hpp"

namespace kgev {

namespace {

// per slot (one workgroup each): the padding of S and the pencil's order.
// mode 0: max_i Re S_ii; mode 1: 2 ||S||_F from the stored lower triangle
// (||S||_F >= ||S||_2, and the factor 2 keeps the computed eigenvalues of S
// below it as well)
__global__ __launch_bounds__(256) void k_batch_prep(BatchDescs ds, int mode, double* spad, int* nreal)
{
    __shared__ double sh[4];
    const int y = blockIdx.x;
    int p = 0;
    while (p + 1 < ds.count && ds.d[p + 1].slot0 <= y) ++p;
    const BatchDesc& d = ds.d[p];
    const int64_t k = y - d.slot0;
    const int64_t slot = ds.slot_base + y;
    const int64_t n = d.n, ld = d.ld;
    const double2* S = d.S + k * ld * n;
    double v = mode == 0 ? -1.0e308 : 0.0;
    if (mode == 0) {
        for (int64_t i = threadIdx.x; i < n; i += 256) v = fmax(v, S[i + i * ld].x);
        v = dpp_wave_max(v);
    } else {
        for (int64_t c = 0; c < n; ++c)
            for (int64_t r = c + threadIdx.x; r < n; r += 256) {
                const double2 x = S[r + c * ld];
                const double a = r == c ? x.x * x.x : 2.0 * (x.x * x.x + x.y * x.y);
                v += a;
            }
        v = dpp_wave_sum(v);
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        spad[slot] = mode == 0 ? fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]))
                               : 2.0 * sqrt((sh[0] + sh[1]) + (sh[2] + sh[3]));
        nreal[slot] = (int)n;
    }
}

// embed: grid (ceil(N*N / 256), slots of the chunk); block y is slot y of
// the chunk: problem p with slot0 <= y < slot0 + nk
__global__ __launch_bounds__(256) void k_batch_embed(BatchDescs ds, int64_t N, const double* spadv, double2* Hp,
                                                     double2* Sp)
{
    const int y = blockIdx.y;
    int p = 0;
    while (p + 1 < ds.count && ds.d[p + 1].slot0 <= y) ++p;
    const BatchDesc& d = ds.d[p];
    const int64_t k = y - d.slot0;
    const int64_t slot = ds.slot_base + y;
    const int64_t n = d.n, ld = d.ld;
    const double2* H = d.H + k * ld * n;
    const double2* S = d.S + k * ld * n;
    const double spad = spadv[slot];
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= N * N) return;
    const int64_t r = e % N, c = e / N;
    double2 h = mk<double>(0, 0), s = mk<double>(0, 0);
    if (r < n && c < n) {
        h = H[r + c * ld];
        s = S[r + c * ld];
    } else if (r == c) {
        s = mk<double>(spad, 0);
    }
    Hp[slot * N * N + e] = h;
    Sp[slot * N * N + e] = s;
}

// column map of one slot (one workgroup per slot): column j of the embedded
// result belongs to the pencil when it vanishes on the padded rows (with
// eigenvectors; a direction dropped by pruning is a zero column and still
// the pencil's), or when it is not one of the first N - n exact zeros
// (eigenvalues only); map[j] = its index among the pencil's columns, or -1
__global__ __launch_bounds__(256) void k_batch_map(BatchDescs ds, int64_t N, const double2* Cp, const double* wp,
                                                   int* map, int with_vectors, int* stp)
{
    __shared__ int sc[256];
    const int y = blockIdx.x;
    int p = 0;
    while (p + 1 < ds.count && ds.d[p + 1].slot0 <= y) ++p;
    const BatchDesc& d = ds.d[p];
    const int64_t slot = ds.slot_base + y;
    const int64_t n = d.n;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int* mp = map + slot * N;
    const double* wv = wp + slot * N;
    if (with_vectors) {
        // one wave per column, lanes over the padded rows
        const double2* C = Cp + slot * N * N;
        for (int64_t j = w; j < N; j += 4) {
            bool nz = false;
            for (int64_t r = n + lane; r < N; r += 64) {
                const double2 v = C[r + j * N];
                nz = nz || v.x != 0.0 || v.y != 0.0;
            }
            nz = __any(nz);
            if (lane == 0) mp[j] = nz ? 0 : 1;
        }
    } else {
        // the first N - n exact zeros in ascending order are the padded values
        const int64_t chunk = (N + 255) / 256;
        const int64_t j0 = tid * chunk, j1 = j0 + chunk < N ? j0 + chunk : N;
        int z = 0;
        for (int64_t j = j0; j < j1; ++j) z += wv[j] == 0.0 ? 1 : 0;
        sc[tid] = z;
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
        int zr = sc[tid];
        for (int64_t j = j0; j < j1; ++j) {
            const bool zero = wv[j] == 0.0;
            mp[j] = (zero && zr < N - n) ? 0 : 1;
            zr += zero ? 1 : 0;
        }
    }
    __syncthreads();
    // flags -> destination indices (chunked scan)
    const int64_t chunk = (N + 255) / 256;
    const int64_t j0 = tid * chunk, j1 = j0 + chunk < N ? j0 + chunk : N;
    int cnt = 0;
    for (int64_t j = j0; j < j1; ++j) cnt += mp[j];
    __syncthreads();
    sc[tid] = cnt;
    __syncthreads();
    __shared__ int total;
    if (tid == 0) {
        int acc = 0;
        for (int q = 0; q < 256; ++q) {
            const int t = sc[q];
            sc[q] = acc;
            acc += t;
        }
        total = acc;
    }
    __syncthreads();
    int pos = sc[tid];
    for (int64_t j = j0; j < j1; ++j) {
        const int f = mp[j];
        mp[j] = f ? pos : -1;
        pos += f;
    }
    // anything but n pencil columns in a slot whose solve succeeded means the
    // blocks did not stay apart
    if (tid == 0 && total != (int)n && stp[slot] == 0) stp[slot] = ST_NOCONV;
}

// extract: grid (N, slots of the chunk): block (j, y) moves column j of slot
// y to its place in the pencil's output (eigenvalue, and vector rows 0..n-1)
__global__ __launch_bounds__(64) void k_batch_extract(BatchDescs ds, int64_t N, const double2* Cp, const double* wp,
                                                      const int* map, const int* stp, int with_vectors)
{
    const int y = blockIdx.y;
    int p = 0;
    while (p + 1 < ds.count && ds.d[p + 1].slot0 <= y) ++p;
    const BatchDesc& d = ds.d[p];
    const int64_t k = y - d.slot0;
    const int64_t slot = ds.slot_base + y;
    const int64_t n = d.n, j = blockIdx.x;
    if (j == 0 && threadIdx.x == 0 && d.status) d.status[k] = stp[slot];
    const int dst = map[slot * N + j];
    if (dst < 0 || dst >= n) return;
    if (threadIdx.x == 0) d.w[k * n + dst] = wp[slot * N + j];
    if (!with_vectors) return;
    const double2* src = Cp + slot * N * N + j * N;
    double2* C = d.C + k * d.ldc * n + (int64_t)dst * d.ldc;
    for (int64_t r = threadIdx.x; r < n; r += 64) C[r] = src[r];
}

}  // namespace

hipError_t batch_prep(hipStream_t st, const BatchDescs& ds, int64_t slots, int mode, double* spad, int* nreal)
{
    hipLaunchKernelGGL(k_batch_prep, dim3((unsigned)slots), dim3(256), 0, st, ds, mode, spad, nreal);
    return hipGetLastError();
}

hipError_t batch_embed(hipStream_t st, const BatchDescs& ds, int64_t slots, int64_t N, const double* spad, double2* Hp,
                       double2* Sp)
{
    const unsigned gx = (unsigned)((N * N + 255) / 256);
    hipLaunchKernelGGL(k_batch_embed, dim3(gx, (unsigned)slots), dim3(256), 0, st, ds, N, spad, Hp, Sp);
    return hipGetLastError();
}

hipError_t batch_extract(hipStream_t st, const BatchDescs& ds, int64_t slots, int64_t N, const double2* Cp,
                         const double* wp, int* map, int* stp, bool with_vectors)
{
    hipLaunchKernelGGL(k_batch_map, dim3((unsigned)slots), dim3(256), 0, st, ds, N, Cp, wp, map,
                       with_vectors ? 1 : 0, stp);
    hipLaunchKernelGGL(k_batch_extract, dim3((unsigned)N, (unsigned)slots), dim3(64), 0, st, ds, N, Cp, wp, map,
                       stp, with_vectors ? 1 : 0);
    return hipGetLastError();
}

}  // namespace kgev
