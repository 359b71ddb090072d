// C ABI of the library (declared in include/kgev.h) and the host-side
// sequencing of the per-k solve, Band_DFT_Col Parts 2-4 (Section III of
// arXiv:1402.4247), batched over k-points:
//   Part 2: S -> tridiagonal (blocked Householder) -> divide and conquer ->
//           back-transformation -> X = U diag(s)^(-1/2) (+ definiteness check)
//   Part 3: G = H X, A = X^H G (lower half)
//   Part 4: A -> tridiagonal -> divide and conquer -> normalisation ->
//           C = X Y with Y = Q_A Z taken as (X Q_A) Z: the back-transformation
//           applied to a copy of X from the right, then the real Z
// Every step is a HIP kernel enqueued on the caller's stream; the host only
// sizes the workspace and issues launches.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "../../include/kgev.h"

using namespace kgev;

namespace kgev {
struct Profiler;
Profiler* prof_start(int phase, int stride, size_t reserve);
bool prof_stop(Profiler* p, int64_t* launches, int64_t* seen, double* ms, double* bytes, double* flops);
}  // namespace kgev

// Everything that identifies a captured solve: sizes, options, buffers, stream.
struct GraphKey {
    int64_t n, ld, nk, ldc;
    int32_t precision, want_vectors, panel_nb, refine_iters, streams, s_method;
    double s_tol;
    const void *H, *S, *w, *C, *work, *status, *stream;
    bool operator==(const GraphKey& o) const { return memcmp(this, &o, sizeof(GraphKey)) == 0; }
};

namespace kgev {
struct TunedParams {
    int nb, hemv_slots, gemm_slots;
};
}  // namespace kgev

struct kgev_ctx {
    int device;
    std::vector<hipStream_t> aux;      // streams of the concurrent k-point groups 1..
    std::vector<hipEvent_t> ev;        // ev[0]: fork, ev[q]: join of group q
    kgev::Profiler* prof;
    std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;   // most recent last
    std::vector<std::pair<std::vector<uintptr_t>, hipGraphExec_t>> batch_graphs;   // most recent last
    std::map<std::pair<int64_t, int>, kgev::TunedParams> tuned;   // (n, precision) -> tuned options
    void* work;
    size_t work_bytes;
    // host-pointer API staging buffers
    void* stage;
    size_t stage_bytes;
    hipStream_t stream;
};

namespace {

constexpr int DEFAULT_NB = 32;
constexpr int DEFAULT_SLOTS = 3 * 256;   // Hermitian-product workgroups below which one tile per workgroup
constexpr int DEFAULT_STREAMS = 1;
constexpr int UNMTR_KB = 64;

struct Layout {
    size_t total = 0;
    size_t add(size_t bytes)
    {
        const size_t off = total;
        total += (bytes + 255) & ~(size_t)255;
        return off;
    }
};

// Offsets of every workspace array for nk problems of order n.
struct SolvePlan {
    int64_t n, nk;
    int nb, kb;
    int slots1;                // Hermitian-product tile grouping threshold (HetrdWs::slots1)
    int NBmax, CHmax, PN;
    // complex128 arrays
    size_t Aw, Vs, X, G, Wp, tau, ypart, ypartT, pvw, qpart, uwork, cwork, ppart, ndrop;
    // real / int arrays
    size_t d, e, sS, wA, pnorm, Zr, Qs, Vsec;
    size_t dc_es, dc_onrm, dc_D0, dc_D1, dc_sd, dc_sz, dc_ndd, dc_ndz, dc_dfd, dc_rotc, dc_rots, dc_rho, dc_tauv,
        dc_lam, dc_zhat;
    size_t dc_kcnt, dc_ndcnt, dc_nrot, dc_perm, dc_ndx, dc_dfx, dc_rota, dc_rotb, dc_orgi, dc_cmap;
    size_t status, bz;
    // mixed precision: complex64 tridiagonalisation / back-transformation
    // buffers and the FP64 refinement scratch (size 0 in the FP64 form)
    bool mixed;
    size_t f_A, f_V, f_Y, f_W, f_tau, f_ypart, f_ypartT, f_pvw, f_qpart, f_uwork, f_d, f_e, f_pnorm;
    size_t r_Ynext, r_G, r_S, r_F, r_pS, r_pR, r_delta, r_cid;
    size_t total;
};

SolvePlan make_plan(int64_t n, int64_t nk, int nb, bool mixed = false, int slots1 = DEFAULT_SLOTS)
{
    SolvePlan p{};
    p.slots1 = slots1;
    p.mixed = mixed;
    p.n = n;
    p.nk = nk;
    p.nb = nb;
    p.kb = UNMTR_KB;
    p.NBmax = hetrd_nbmax(n);
    p.CHmax = hetrd_chmax(n);
    p.PN = hetrd_pn(n);
    Layout L;
    const size_t z = sizeof(double2), r = sizeof(double), i4 = sizeof(int);
    const size_t nn = (size_t)n * n;
    p.Aw = L.add(z * nn * nk);
    p.Vs = L.add(z * nn * nk);
    p.X = L.add(z * nn * nk);
    p.G = L.add(z * nn * nk);
    // nb-dependent arrays are sized for the widest panel (64), so a tuned
    // width never outgrows a workspace sized by kgev_workspace_bytes
    const size_t nbA = 64;
    p.Wp = L.add(z * n * nbA * nk);
    p.tau = L.add(z * n * nk);
    p.ypart = L.add(z * (size_t)p.NBmax * p.NBmax * 64 * nk);
    p.ypartT = L.add(z * (size_t)p.NBmax * p.CHmax * 64 * nk);
    p.pvw = L.add(z * 4 * (size_t)p.NBmax * nbA * nk);      // W and V parts interleaved by block
    p.qpart = L.add(r * (size_t)p.NBmax * p.CHmax * nk);
    p.uwork = L.add(z * (size_t)unmtr_work_elems(n, p.kb) * nk);
    p.cwork = L.add(z * (size_t)chol_work_elems(n) * nk);
    p.ppart = L.add(r * n * nk);
    p.ndrop = L.add(i4 * nk);
    p.d = L.add(r * n * nk);
    p.e = L.add(r * n * nk);
    p.sS = L.add(r * n * nk);
    p.wA = L.add(r * n * nk);
    p.pnorm = L.add(r * 2 * p.PN * nk);
    p.Zr = L.add(r * nn * nk);
    p.Qs = L.add(r * nn * nk);
    p.Vsec = L.add(r * nn * nk);
    size_t* dv[] = {&p.dc_es, &p.dc_D0, &p.dc_D1, &p.dc_sd, &p.dc_sz, &p.dc_ndd, &p.dc_ndz, &p.dc_dfd,
                    &p.dc_rotc, &p.dc_rots, &p.dc_rho, &p.dc_tauv, &p.dc_lam, &p.dc_zhat};
    for (size_t* q : dv) *q = L.add(r * n * nk);
    p.dc_onrm = L.add(r * nk);
    size_t* iv[] = {&p.dc_kcnt, &p.dc_ndcnt, &p.dc_nrot, &p.dc_perm, &p.dc_ndx, &p.dc_dfx, &p.dc_rota, &p.dc_rotb,
                    &p.dc_orgi, &p.dc_cmap};
    for (size_t* q : iv) *q = L.add(i4 * n * nk);
    p.status = L.add(i4 * nk);
    p.bz = L.add(stebz_work_bytes(nk));
    const size_t m = mixed ? 1 : 0;
    const size_t c = sizeof(float2), f = sizeof(float);
    p.f_A = L.add(m * c * nn * nk);
    p.f_V = L.add(m * c * nn * nk);
    p.f_Y = L.add(m * c * nn * nk);
    p.f_W = L.add(m * c * n * nbA * nk);
    p.f_tau = L.add(m * c * n * nk);
    p.f_ypart = L.add(m * c * (size_t)p.NBmax * p.NBmax * 64 * nk);
    p.f_ypartT = L.add(m * c * (size_t)p.NBmax * p.CHmax * 64 * nk);
    p.f_pvw = L.add(m * c * 4 * (size_t)p.NBmax * nbA * nk);
    p.f_qpart = L.add(m * f * (size_t)p.NBmax * p.CHmax * nk);
    p.f_uwork = L.add(m * c * (size_t)unmtr_work_elems(n, p.kb) * nk);
    p.f_d = L.add(m * f * n * nk);
    p.f_e = L.add(m * f * n * nk);
    p.f_pnorm = L.add(m * f * 2 * p.PN * nk);
    p.r_Ynext = L.add(m * z * nn * nk);
    p.r_G = L.add(m * z * nn * nk);
    p.r_S = L.add(m * z * nn * nk);
    p.r_F = L.add(m * z * nn * nk);
    p.r_pS = L.add(m * r * n * nk);
    p.r_pR = L.add(m * r * n * nk);
    p.r_delta = L.add(m * r * nk);
    p.r_cid = L.add(m * i4 * n * nk);
    p.total = L.total;
    return p;
}

HetrdWs<float> hetrd_ws32(const SolvePlan& p, void* w)
{
    HetrdWs<float> h{};
    h.n = (int)p.n;
    h.nb = p.nb;
    h.slots1 = p.slots1;
    h.NBmax = p.NBmax;
    h.CHmax = p.CHmax;
    h.A = reinterpret_cast<float2*>(static_cast<char*>(w) + p.f_A); h.lda = p.n; h.sA = p.n * p.n;
    h.V = reinterpret_cast<float2*>(static_cast<char*>(w) + p.f_V); h.sV = p.n * p.n;
    h.W = reinterpret_cast<float2*>(static_cast<char*>(w) + p.f_W); h.sW = p.n * p.nb;
    h.d = reinterpret_cast<float*>(static_cast<char*>(w) + p.f_d);
    h.e = reinterpret_cast<float*>(static_cast<char*>(w) + p.f_e);
    h.tau = reinterpret_cast<float2*>(static_cast<char*>(w) + p.f_tau);
    h.pnorm = reinterpret_cast<float*>(static_cast<char*>(w) + p.f_pnorm); h.s_pnorm = 2 * p.PN;
    h.ypart = reinterpret_cast<float2*>(static_cast<char*>(w) + p.f_ypart); h.s_ypart = (int64_t)p.NBmax * p.NBmax * 64;
    h.ypartT = reinterpret_cast<float2*>(static_cast<char*>(w) + p.f_ypartT); h.s_ypartT = (int64_t)p.NBmax * p.CHmax * 64;
    h.pvw = reinterpret_cast<float2*>(static_cast<char*>(w) + p.f_pvw);
    h.pvv = h.pvw + p.nb;
    h.s_pdot = 4 * (int64_t)p.NBmax * p.nb;
    h.qpart = reinterpret_cast<float*>(static_cast<char*>(w) + p.f_qpart); h.s_qpart = (int64_t)p.NBmax * p.CHmax;
    return h;
}

template <typename T> T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

HetrdWs<double> hetrd_ws(const SolvePlan& p, void* w, double2* A, int64_t lda, int64_t sA, double2* V, double* d,
                         double* e, double2* tau)
{
    HetrdWs<double> h{};
    h.n = (int)p.n;
    h.nb = p.nb;
    h.slots1 = p.slots1;
    h.NBmax = p.NBmax;
    h.CHmax = p.CHmax;
    h.A = A; h.lda = lda; h.sA = sA;
    h.V = V; h.sV = p.n * p.n;
    h.W = at<double2>(w, p.Wp); h.sW = p.n * p.nb;
    h.d = d; h.e = e; h.tau = tau;
    h.pnorm = at<double>(w, p.pnorm); h.s_pnorm = 2 * p.PN;
    h.ypart = at<double2>(w, p.ypart); h.s_ypart = (int64_t)p.NBmax * p.NBmax * 64;
    h.ypartT = at<double2>(w, p.ypartT); h.s_ypartT = (int64_t)p.NBmax * p.CHmax * 64;
    h.pvw = at<double2>(w, p.pvw); h.pvv = h.pvw + p.nb; h.s_pdot = 4 * (int64_t)p.NBmax * p.nb;
    h.qpart = at<double>(w, p.qpart); h.s_qpart = (int64_t)p.NBmax * p.CHmax;
    return h;
}

DcWs dc_ws(const SolvePlan& p, void* w, const double* d, const double* e, int* status)
{
    DcWs c{};
    c.n = (int)p.n;
    c.nk = p.nk;
    c.din = d; c.ein = e; c.s_din = p.n;
    c.es = at<double>(w, p.dc_es);
    c.onrm = at<double>(w, p.dc_onrm);
    c.D[0] = at<double>(w, p.dc_D0);
    c.D[1] = at<double>(w, p.dc_D1);
    c.sQ = p.n * p.n;
    c.Vsec = at<double>(w, p.Vsec);
    c.kcnt = at<int>(w, p.dc_kcnt); c.ndcnt = at<int>(w, p.dc_ndcnt); c.nrot = at<int>(w, p.dc_nrot);
    c.rho = at<double>(w, p.dc_rho);
    c.perm = at<int>(w, p.dc_perm); c.sd = at<double>(w, p.dc_sd); c.sz = at<double>(w, p.dc_sz);
    c.ndx = at<int>(w, p.dc_ndx); c.ndd = at<double>(w, p.dc_ndd); c.ndz = at<double>(w, p.dc_ndz);
    c.dfx = at<int>(w, p.dc_dfx); c.dfd = at<double>(w, p.dc_dfd);
    c.rota = at<int>(w, p.dc_rota); c.rotb = at<int>(w, p.dc_rotb);
    c.rotc = at<double>(w, p.dc_rotc); c.rots = at<double>(w, p.dc_rots);
    c.orgi = at<int>(w, p.dc_orgi); c.tauv = at<double>(w, p.dc_tauv); c.lam = at<double>(w, p.dc_lam);
    c.zhat = at<double>(w, p.dc_zhat); c.cmap = at<int>(w, p.dc_cmap);
    c.s_w = p.n;
    c.status = status;
    return c;
}

kgev_opts resolve_opts(const kgev_opts* o)
{
    kgev_opts r;
    kgev_opts_default(&r);
    if (o) r = *o;
    if (r.panel_nb == 0) r.panel_nb = DEFAULT_NB;
    if (r.hemv_slots == 0) r.hemv_slots = DEFAULT_SLOTS;
    if (r.gemm_slots == 0) r.gemm_slots = GEMM_SMALL_SLOTS_DEFAULT;
    if (r.s_tol == 0.0) r.s_tol = 1e-12;
    if (r.refine_iters == 0) r.refine_iters = 3;
    if (r.streams == 0) r.streams = DEFAULT_STREAMS;
    return r;
}

bool opts_valid(const kgev_opts& o)
{
    if (o.precision != KGEV_PREC_FP64 && o.precision != KGEV_PREC_FP32_REFINE) return false;
    if (o.refine_iters < 1 || o.refine_iters > 10) return false;
    if (o.want_vectors != 0 && o.want_vectors != 1) return false;
    if (o.panel_nb < 1 || o.panel_nb > 64) return false;
    if (o.hemv_slots < 1 || o.gemm_slots < 1) return false;
    if (!(o.s_tol > 0.0) || o.s_tol >= 1.0) return false;
    if (o.use_graph != 0 && o.use_graph != 1) return false;
    if (o.streams < 1 || o.streams > 8) return false;
    if (o.s_method != KGEV_S_EIG && o.s_method != KGEV_S_CHOLESKY && o.s_method != KGEV_S_PRUNE) return false;
    for (int q = 0; q < 3; ++q)
        if (o.reserved[q] != 0) return false;
    return true;
}

// The tuner's values for the fields the caller left 0 (user: the caller's
// options, null for all defaults).
void apply_tuned(const kgev_ctx* ctx, int64_t n, const kgev_opts* user, kgev_opts& o)
{
    auto it = ctx->tuned.find({n, o.precision});
    if (it == ctx->tuned.end()) return;
    if (!user || user->panel_nb == 0) o.panel_nb = it->second.nb;
    if (!user || user->hemv_slots == 0) o.hemv_slots = it->second.hemv_slots;
    if (!user || user->gemm_slots == 0) o.gemm_slots = it->second.gemm_slots;
}

// the product tile policy of one call, installed for the calling thread
struct TileScope {
    int old;
    explicit TileScope(int slots) : old(gemm_small_tile_slots(slots)) {}
    ~TileScope() { gemm_small_tile_slots(old); }
    TileScope(const TileScope&) = delete;
    TileScope& operator=(const TileScope&) = delete;
};

// With KGEV_DEBUG set in the environment, a failing HIP call is reported on
// stderr (call site and HIP error name) before KGEV_EDEVICE is returned.
bool debug_enabled()
{
    static const bool on = getenv("KGEV_DEBUG") != nullptr;
    return on;
}

#define KCHECK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            if (debug_enabled())                                                            \
                fprintf(stderr, "kgev: %s failed at %s:%d: %s\n", #expr, __FILE__, __LINE__, \
                        hipGetErrorName(e_));                                               \
            return KGEV_EDEVICE;                                                            \
        }                                                                                   \
    } while (0)

kgev_status ensure_work(kgev_ctx* ctx, size_t bytes)
{
    if (ctx->work_bytes >= bytes) return KGEV_OK;
    if (ctx->work) {
        if (hipDeviceSynchronize() != hipSuccess) return KGEV_EDEVICE;
        (void)hipFree(ctx->work);
        ctx->work = nullptr;
        ctx->work_bytes = 0;
    }
    if (hipMalloc(&ctx->work, bytes) != hipSuccess) {
        ctx->work = nullptr;
        return KGEV_ENOMEM;
    }
    ctx->work_bytes = bytes;
    return KGEV_OK;
}

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DevGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Eigen_HH on the batch whose working copies are in Aw (lower, ld n):
// eigenvalues -> wout (stride n); vectors (if Y) -> Y (ld n).  values_only:
// the tridiagonal step by bisection, eigenvalues only (no Z; Y must be null).
kgev_status eigen_hh(const SolvePlan& p, void* w, hipStream_t st, double* wout, double2* Y, int* status,
                     bool values_only = false)
{
    const int64_t n = p.n, nk = p.nk, nn = n * n;
    double2* Aw = at<double2>(w, p.Aw);
    double2* Vs = at<double2>(w, p.Vs);
    double* d = at<double>(w, p.d);
    double* e = at<double>(w, p.e);
    double2* tau = at<double2>(w, p.tau);
    KCHECK(fill_zero(st, Vs, sizeof(double2) * (size_t)nn * nk));
    KCHECK(hetrd<double>(st, hetrd_ws(p, w, Aw, n, nn, Vs, d, e, tau), nk));
    if (values_only) {
        KCHECK(stebz(st, d, e, n, n, nk, wout, n, at<void>(w, p.bz)));
        return KGEV_OK;
    }
    double* Zr = at<double>(w, p.Zr);
    KCHECK(stedc(st, dc_ws(p, w, d, e, status), wout, Zr, at<double>(w, p.Qs), nk));
    if (!Y) return KGEV_OK;
    KCHECK(real_to_complex<double>(st, n, Zr, nn, Y, n, nn, nk));
    KCHECK(unmtr<double>(st, n, Vs, nn, tau, n, Y, n, nn, at<double2>(w, p.uwork), p.kb, nk));
    return KGEV_OK;
}

// Part 4 in the mixed-precision form: A (FP64, lower, in Aw) is rounded to
// complex64, tridiagonalised and back-transformed on FP32 MFMA; the
// tridiagonal eigensolve runs in FP64 on the promoted d, e; the eigenpairs are
// then refined against the FP64 A (refine.hip).  Y (ld n) receives the
// refined vectors, wout the refined eigenvalues.
kgev_status eigen_hh_mixed(const SolvePlan& p, void* w, hipStream_t st, double* wout, double2* Y, int* status,
                           int iters)
{
    const int64_t n = p.n, nk = p.nk, nn = n * n;
    double2* Aw = at<double2>(w, p.Aw);
    HetrdWs<float> h = hetrd_ws32(p, w);
    KCHECK(copy_lower_check<float>(st, n, Aw, n, nn, h.A, n, nn, nullptr, nk));
    KCHECK(fill_zero(st, h.V, sizeof(float2) * (size_t)nn * nk));
    KCHECK(hetrd<float>(st, h, nk));
    double* d = at<double>(w, p.d);
    double* e = at<double>(w, p.e);
    KCHECK(float_to_double(st, h.d, d, n * nk));
    KCHECK(float_to_double(st, h.e, e, n * nk));
    double* Zr = at<double>(w, p.Zr);
    KCHECK(stedc(st, dc_ws(p, w, d, e, status), wout, Zr, at<double>(w, p.Qs), nk));
    float2* Y32 = at<float2>(w, p.f_Y);
    KCHECK(real_to_complex<float>(st, n, Zr, nn, Y32, n, nn, nk));
    KCHECK(unmtr<float>(st, n, h.V, nn, h.tau, n, Y32, n, nn, at<float2>(w, p.f_uwork), p.kb, nk));
    KCHECK(c64_to_c128(st, Y32, Y, nn * nk));
    double2* Af = at<double2>(w, p.Vs);
    KCHECK(hermitian_full(st, n, Aw, n, nn, Af, n, nn, nk));
    RefineWs rw{};
    rw.n = n;
    rw.Af = Af;
    rw.Y = Y;
    rw.Ynext = at<double2>(w, p.r_Ynext);
    rw.G = at<double2>(w, p.r_G);
    rw.P = Aw;                       // A itself is no longer needed
    rw.S = at<double2>(w, p.r_S);
    rw.F = at<double2>(w, p.r_F);
    rw.pS = at<double>(w, p.r_pS);
    rw.pR = at<double>(w, p.r_pR);
    rw.delta = at<double>(w, p.r_delta);
    rw.cid = at<int>(w, p.r_cid);
    rw.status = status;
    KCHECK(refine(st, rw, nk, iters, wout));
    return KGEV_OK;
}

// Xin: Part 2 skipped and this X (n x n per k, ld n) used; Xout: the X of
// Part 2 also written there.
// nreal: per problem, the order of an embedded pencil (its padded
// directions of S sort last), or nullptr
kgev_status solve_device(const SolvePlan& p, const kgev_opts& o, void* w, hipStream_t st, const double2* H,
                         const double2* S, int64_t ld, double* dw, double2* dC, int64_t ldc, int32_t* d_status,
                         const double2* Xin = nullptr, double2* Xout = nullptr, const int* nreal = nullptr)
{
    const TileScope tiles(o.gemm_slots);
    const int64_t n = p.n, nk = p.nk, nn = n * n;
    int* status = at<int>(w, p.status);
    double2* Aw = at<double2>(w, p.Aw);
    double2* Vs = at<double2>(w, p.Vs);
    double2* X = at<double2>(w, p.X);
    double2* G = at<double2>(w, p.G);
    double* sS = at<double>(w, p.sS);
    KCHECK(status_init(st, status, nk));
    // inputs: non-finite check on both, S copied into the working matrix
    KCHECK(copy_lower_check<double>(st, n, H, ld, ld * n, nullptr, 0, 0, status, nk));
    kgev_status r;
    if (Xin) {
        X = const_cast<double2*>(Xin);        // Part 2 done by an earlier call
    } else {
        KCHECK(copy_lower_check<double>(st, n, S, ld, ld * n, Aw, n, nn, status, nk));
        if (o.s_method == KGEV_S_CHOLESKY) {
            // Part 2 in Cholesky form: S = L L^H, X = L^(-H) J, J the column
            // reversal (L in Vs, L^(-1) in G)
            KCHECK(cholesky_x(st, n, Aw, n, nn, Vs, G, X, at<double2>(w, p.cwork), sS, o.s_tol, status, nk));
        } else {
            // Part 2: S = U diag(s) U^H, X = U diag(s)^(-1/2) (pruned: the
            // columns with s_j <= s_tol s_max are zero)
            r = eigen_hh(p, w, st, sS, X, status);
            if (r != KGEV_OK) return r;
            KCHECK(normalize_cols(st, n, X, n, nn, sS, n, o.s_tol, status, nk, o.s_method == KGEV_S_PRUNE, nreal));
        }
    }
    if (Xout) KCHECK(hipMemcpyAsync(Xout, X, sizeof(double2) * (size_t)nn * nk, hipMemcpyDeviceToDevice, st));
    // Part 3: A = X^H (H X), lower half
    KCHECK(hermitian_full(st, n, H, ld, ld * n, Vs, n, nn, nk));
    const double2 one = mk<double>(1, 0), zero = mk<double>(0, 0);
    KCHECK(cgemm<double>(st, 'N', 'N', n, n, n, one, Vs, n, nn, X, n, nn, zero, G, n, nn, nk, false));
    KCHECK(cgemm<double>(st, 'C', 'N', n, n, n, one, X, n, nn, G, n, nn, zero, Aw, n, nn, nk, true));
    if (o.s_method == KGEV_S_PRUNE)
        KCHECK(prune_shift(st, n, Aw, nn, at<double>(w, p.ppart), sS, n, o.s_tol, at<int>(w, p.ndrop), nk, nreal));
    // Part 4: A = Y diag(lambda) Y^H with Y = Q_A Z (Householder reflectors
    // Q_A, real tridiagonal eigenvectors Z), C = X Y
    if (o.precision == KGEV_PREC_FP32_REFINE) {
        r = eigen_hh_mixed(p, w, st, dw, G, status, o.refine_iters);
        if (r != KGEV_OK) return r;
        if (o.want_vectors) {
            KCHECK(normalize_cols(st, n, G, n, nn, nullptr, 0, 0.0, nullptr, nk));
            KCHECK(cgemm<double>(st, 'N', 'N', n, n, n, one, X, n, nn, G, n, nn, zero, dC, ldc, ldc * n, nk, false));
        }
    } else {
        // eigenvalues and Z; with vectors, C = (X Q_A) Z: the reflectors are
        // applied to a copy of X from the right, and the last product takes
        // the real Z as it is (two real products instead of three).  Without
        // vectors (Band_DFT_Col's eigenvalue pass) the tridiagonal step is
        // bisection for the eigenvalues alone.
        r = eigen_hh(p, w, st, dw, nullptr, status, !o.want_vectors);
        if (r != KGEV_OK) return r;
        if (o.want_vectors) {
            double* Zr = at<double>(w, p.Zr);
            KCHECK(normalize_cols_real(st, n, Zr, n, nn, nk));
            KCHECK(hipMemcpyAsync(G, X, sizeof(double2) * (size_t)nn * nk, hipMemcpyDeviceToDevice, st));
            KCHECK(unmtr<double>(st, n, Vs, nn, at<double2>(w, p.tau), n, G, n, nn, at<double2>(w, p.uwork), p.kb,
                                 nk, true));
            KCHECK(cgemm_rb<double>(st, n, n, n, G, n, nn, Zr, n, nn, dC, ldc, ldc * n, nk));
        }
    }
    if (o.s_method == KGEV_S_PRUNE)
        KCHECK(prune_finish(st, n, dw, o.want_vectors ? dC : nullptr, ldc, at<int>(w, p.ndrop), nk));
    if (d_status) KCHECK(status_finish(st, status, d_status, nk));
    return KGEV_OK;
}

// Concurrent k-point groups: G = min(streams, nk) groups of ceil(nk / G)
// k-points, each with its own workspace region; group 0 runs on the caller's
// stream, group q > 0 on a context stream forked from it and joined back, so
// the latency-bound phases of one group overlap the streaming and MFMA phases
// of the others.
struct Groups {
    int G;
    int64_t gsz;
    size_t region;
    SolvePlan p;
};

Groups make_groups(int64_t n, int64_t nk, const kgev_opts& o)
{
    Groups g;
    g.G = (int)std::min<int64_t>(o.streams, nk);
    g.gsz = (nk + g.G - 1) / g.G;
    g.G = (int)((nk + g.gsz - 1) / g.gsz);
    g.p = make_plan(n, g.gsz, o.panel_nb, o.precision == KGEV_PREC_FP32_REFINE, o.hemv_slots);
    g.region = (g.p.total + 255) & ~(size_t)255;
    return g;
}

kgev_status ensure_aux(kgev_ctx* ctx, int G)
{
    while ((int)ctx->aux.size() < G - 1) {
        hipStream_t s = nullptr;
        KCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        ctx->aux.push_back(s);
    }
    while ((int)ctx->ev.size() < G) {
        hipEvent_t e = nullptr;
        KCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->ev.push_back(e);
    }
    return KGEV_OK;
}

kgev_status solve_grouped(kgev_ctx* ctx, const Groups& g, const kgev_opts& o, void* w, hipStream_t st,
                          const double2* H, const double2* S, int64_t ld, int64_t nk, double* dw, double2* dC,
                          int64_t ldc, int32_t* d_status, const int* nreal = nullptr)
{
    const int64_t n = g.p.n;
    if (g.G == 1) return solve_device(g.p, o, w, st, H, S, ld, dw, dC, ldc, d_status, nullptr, nullptr, nreal);
    kgev_status r = ensure_aux(ctx, g.G);
    if (r != KGEV_OK) return r;
    KCHECK(hipEventRecord(ctx->ev[0], st));
    for (int q = 0; q < g.G; ++q) {
        const int64_t k0 = q * g.gsz, cnt = std::min<int64_t>(g.gsz, nk - k0);
        const SolvePlan pq = (cnt == g.gsz) ? g.p : make_plan(n, cnt, o.panel_nb, o.precision == KGEV_PREC_FP32_REFINE, o.hemv_slots);
        hipStream_t s = q == 0 ? st : ctx->aux[q - 1];
        if (q > 0) KCHECK(hipStreamWaitEvent(s, ctx->ev[0], 0));
        r = solve_device(pq, o, static_cast<char*>(w) + (size_t)q * g.region, s, H + k0 * ld * n, S + k0 * ld * n,
                         ld, dw + k0 * n, dC ? dC + k0 * ldc * n : nullptr, ldc, d_status ? d_status + k0 : nullptr,
                         nullptr, nullptr, nreal ? nreal + k0 : nullptr);
        if (r != KGEV_OK) return r;
        if (q > 0) KCHECK(hipEventRecord(ctx->ev[q], s));
    }
    for (int q = 1; q < g.G; ++q) KCHECK(hipStreamWaitEvent(st, ctx->ev[q], 0));
    return KGEV_OK;
}

// Destroy every cached graph of the context (after the device is idle).
void drop_graphs(kgev_ctx* ctx)
{
    if (ctx->graphs.empty() && ctx->batch_graphs.empty()) return;
    (void)hipDeviceSynchronize();
    for (auto& e : ctx->graphs) (void)hipGraphExecDestroy(e.second);
    ctx->graphs.clear();
    for (auto& e : ctx->batch_graphs) (void)hipGraphExecDestroy(e.second);
    ctx->batch_graphs.clear();
}

// Size classes of a batch of uneven order, largest order first: a problem
// joins the current class when the class order N is at most 256 (small
// pencils, where launches rather than arithmetic set the cost) or at most
// 1.26 n (at most twice its own arithmetic).
struct BatchClass {
    int64_t N = 0, K = 0;
    std::vector<int64_t> members;
};

std::vector<BatchClass> batch_classes(const kgev_problem* probs, int64_t count)
{
    std::vector<int64_t> idx((size_t)count);
    for (int64_t q = 0; q < count; ++q) idx[(size_t)q] = q;
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return probs[a].n > probs[b].n; });
    std::vector<BatchClass> cls;
    for (int64_t q : idx) {
        const int64_t n = probs[q].n;
        if (cls.empty() || !(cls.back().N <= 256 || (double)cls.back().N <= 1.26 * (double)n)) {
            cls.emplace_back();
            cls.back().N = n;
        }
        cls.back().members.push_back(q);
        cls.back().K += probs[q].nk;
    }
    return cls;
}

// A class of one problem of the class order is solved in place; any other
// is embedded (batch.hip): packed H', S', the embedded eigenvalues, vectors
// and statuses, the column map, then the solve's own workspace.
struct ClassLayout {
    bool direct;
    size_t Hp, Sp, wp, Cp, stp, map, spad, nreal, solve, total;
    Groups grp;
};

ClassLayout class_layout(const kgev_problem* probs, const BatchClass& c, const kgev_opts& o)
{
    ClassLayout L{};
    const int64_t N = c.N, K = c.K;
    L.direct = c.members.size() == 1 && probs[c.members[0]].n == N;
    L.grp = make_groups(N, K, o);
    Layout a;
    if (!L.direct) {
        const size_t nn = (size_t)N * N;
        L.Hp = a.add(sizeof(double2) * nn * K);
        L.Sp = a.add(sizeof(double2) * nn * K);
        L.wp = a.add(sizeof(double) * (size_t)N * K);
        L.Cp = a.add(o.want_vectors ? sizeof(double2) * nn * K : 0);
        L.stp = a.add(sizeof(int32_t) * (size_t)K);
        L.map = a.add(sizeof(int) * (size_t)N * K);
        L.spad = a.add(sizeof(double) * (size_t)K);
        L.nreal = a.add(sizeof(int) * (size_t)K);
    }
    L.solve = a.add(L.grp.region * (size_t)L.grp.G);
    L.total = a.total;
    return L;
}

kgev_status solve_class(kgev_ctx* ctx, const kgev_problem* probs, const BatchClass& c, const kgev_opts& o0,
                        void* w, hipStream_t st, const kgev_opts* user)
{
    kgev_opts o = o0;
    apply_tuned(ctx, c.N, user, o);
    const ClassLayout L = class_layout(probs, c, o);
    char* base = static_cast<char*>(w);
    if (L.direct) {
        const kgev_problem& pr = probs[c.members[0]];
        return solve_grouped(ctx, L.grp, o, base + L.solve, st, (const double2*)pr.dH, (const double2*)pr.dS, pr.ld,
                             pr.nk, pr.dw, o.want_vectors ? (double2*)pr.dC : nullptr, pr.ldc, pr.d_status);
    }
    const int64_t N = c.N;
    double2* Hp = reinterpret_cast<double2*>(base + L.Hp);
    double2* Sp = reinterpret_cast<double2*>(base + L.Sp);
    double* wp = reinterpret_cast<double*>(base + L.wp);
    double2* Cp = o.want_vectors ? reinterpret_cast<double2*>(base + L.Cp) : nullptr;
    int32_t* stp = reinterpret_cast<int32_t*>(base + L.stp);
    int* map = reinterpret_cast<int*>(base + L.map);
    double* spad = reinterpret_cast<double*>(base + L.spad);
    int* nreal = reinterpret_cast<int*>(base + L.nreal);
    // Cholesky form: no ordering by eigenvalue, the padding keeps the pivot
    // threshold (max_i S_ii); otherwise the padded directions must sort after
    // the pencil's own
    const int mode = o.s_method == KGEV_S_CHOLESKY ? 0 : 1;
    std::vector<std::pair<BatchDescs, int64_t>> chunks;
    int64_t slot = 0;
    for (size_t q0 = 0; q0 < c.members.size(); q0 += BATCH_DESC) {
        BatchDescs ds;
        memset(&ds, 0, sizeof(ds));
        ds.slot_base = slot;
        int rel = 0;
        for (size_t q = q0; q < c.members.size() && q < q0 + BATCH_DESC; ++q) {
            const kgev_problem& pr = probs[c.members[q]];
            BatchDesc& d = ds.d[ds.count++];
            d.H = (const double2*)pr.dH;
            d.S = (const double2*)pr.dS;
            d.w = pr.dw;
            d.C = (double2*)pr.dC;
            d.status = pr.d_status;
            d.n = pr.n;
            d.ld = pr.ld;
            d.ldc = pr.ldc;
            d.slot0 = rel;
            rel += (int)pr.nk;
        }
        KCHECK(batch_prep(st, ds, rel, mode, spad, nreal));
        KCHECK(batch_embed(st, ds, rel, N, spad, Hp, Sp));
        chunks.push_back({ds, rel});
        slot += rel;
    }
    const kgev_status r = solve_grouped(ctx, L.grp, o, base + L.solve, st, Hp, Sp, N, c.K, wp, Cp, N, stp,
                                        mode == 1 ? nreal : nullptr);
    if (r != KGEV_OK) return r;
    for (const auto& ch : chunks) KCHECK(batch_extract(st, ch.first, ch.second, N, Cp, wp, map, stp, o.want_vectors != 0));
    return KGEV_OK;
}

// Workspace of kgev_solve_k_device_noalloc: one static array per GPU, reserved
// when the library's device code is loaded on that GPU and held until the
// process ends.  Host code never uses the array's name as an address: its
// device address on each GPU comes from hipGetSymbolAddress (taken once per
// device, with that device current, in kgev_create) and is kept in
// g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[KGEV_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// the device address of this device's scratch array (the device is current)
kgev_status scratch_address(int device, void** out)
{
    if (device < 0 || device >= MAX_DEVICES) return KGEV_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        KCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return KGEV_EDEVICE;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return KGEV_OK;
}

}  // namespace

namespace kgev {
// suspends launch timing for the calling thread (profile.hip)
void* prof_suspend();
void prof_resume(void* saved);
}  // namespace kgev

extern "C" {

void kgev_opts_default(kgev_opts* o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->precision = KGEV_PREC_FP64;
    o->want_vectors = 1;
    o->panel_nb = 0;
    o->refine_iters = 0;
    o->s_tol = 0.0;
}

const char* kgev_status_str(kgev_status st)
{
    switch (st) {
    case KGEV_OK: return "ok";
    case KGEV_ENOTPD: return "S(k) is not positive definite";
    case KGEV_ENOCONV: return "tridiagonal eigensolver did not converge";
    case KGEV_ENONFINITE: return "non-finite value in H(k) or S(k)";
    case KGEV_ERANGE: return "electron count outside the range the states can hold";
    case KGEV_ENOMEM: return "out of memory";
    case KGEV_EDEVICE: return "HIP runtime error";
    case KGEV_EUNSUPPORTED: return "unsupported option";
    default: return st < 0 ? "invalid argument" : "unknown status";
    }
}

kgev_status kgev_create(kgev_ctx** ctx, int device)
{
    if (!ctx) return -1;
    *ctx = nullptr;
    int count = 0;
    KCHECK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return -2;
    DevGuard g(device);
    void* sp = nullptr;
    const kgev_status ss = scratch_address(device, &sp);
    if (ss != KGEV_OK) return ss;
    kgev_ctx* c = new kgev_ctx{};
    c->device = device;
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (debug_enabled()) fprintf(stderr, "kgev: hipStreamCreateWithFlags: %s\n", hipGetErrorName(e));
        delete c;
        return KGEV_EDEVICE;
    }
    *ctx = c;
    return KGEV_OK;
}

void kgev_destroy(kgev_ctx* ctx)
{
    if (!ctx) return;
    DevGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->prof) prof_stop(ctx->prof, nullptr, nullptr, nullptr, nullptr, nullptr);
    for (auto& e : ctx->graphs) (void)hipGraphExecDestroy(e.second);
    for (auto& e : ctx->batch_graphs) (void)hipGraphExecDestroy(e.second);
    if (ctx->work) (void)hipFree(ctx->work);
    if (ctx->stage) (void)hipFree(ctx->stage);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    for (hipStream_t x : ctx->aux) (void)hipStreamDestroy(x);
    for (hipEvent_t x : ctx->ev) (void)hipEventDestroy(x);
    delete ctx;
}

size_t kgev_workspace_bytes(int64_t n, int64_t nk, const kgev_opts* opts)
{
    if (n < 1 || nk < 1) return 0;
    kgev_opts o = resolve_opts(opts);
    const Groups g = make_groups(n, nk, o);
    return g.region * (size_t)g.G;
}

kgev_status kgev_solve_k_device(kgev_ctx* ctx, const kgev_z* dH, const kgev_z* dS, int64_t n, int64_t ld,
                                int64_t nk, double* dw, kgev_z* dC, int64_t ldc, void* dwork, size_t work_bytes,
                                int32_t* d_status, const kgev_opts* opts, void* stream)
{
    if (!ctx) return -1;
    if (!dH) return -2;
    if (!dS) return -3;
    if (n < 1) return -4;
    if (ld < n) return -5;
    if (nk < 1) return -6;
    if (!dw) return -7;
    if (!opts || opts->panel_nb == 0 || opts->hemv_slots == 0 || opts->gemm_slots == 0) {
        kgev_opts t = resolve_opts(opts);
        if (ctx->tuned.count({n, t.precision})) {
            apply_tuned(ctx, n, opts, t);     // every field now set: the call below does not come back here
            return kgev_solve_k_device(ctx, dH, dS, n, ld, nk, dw, dC, ldc, dwork, work_bytes, d_status, &t, stream);
        }
    }
    kgev_opts o = resolve_opts(opts);
    if (!opts_valid(o)) return -10;
    if (o.want_vectors && (!dC || ldc < n)) return -8;
    DevGuard g(ctx->device);
    const Groups grp = make_groups(n, nk, o);
    const size_t need = grp.region * (size_t)grp.G;
    void* w = dwork;
    if (w) {
        if (work_bytes < need) return -9;
    } else {
        kgev_status r = ensure_work(ctx, need);
        if (r != KGEV_OK) return r;
        w = ctx->work;
    }
    hipStream_t st = (hipStream_t)stream;
    double2* C2 = o.want_vectors ? (double2*)dC : nullptr;
    if (!o.use_graph || st == nullptr)
        return solve_grouped(ctx, grp, o, w, st, (const double2*)dH, (const double2*)dS, ld, nk, dw, C2, ldc,
                             d_status);

    GraphKey key;
    memset(&key, 0, sizeof(key));
    key.n = n; key.ld = ld; key.nk = nk; key.ldc = o.want_vectors ? ldc : 0;
    key.precision = o.precision; key.want_vectors = o.want_vectors; key.panel_nb = o.panel_nb;
    key.refine_iters = o.refine_iters; key.streams = o.streams; key.s_method = o.s_method; key.s_tol = o.s_tol;
    key.H = dH; key.S = dS; key.w = dw; key.C = o.want_vectors ? dC : nullptr; key.work = w; key.status = d_status;
    key.stream = stream;
    for (size_t q = 0; q < ctx->graphs.size(); ++q)
        if (ctx->graphs[q].first == key) {
            auto e = ctx->graphs[q];
            ctx->graphs.erase(ctx->graphs.begin() + q);
            ctx->graphs.push_back(e);
            KCHECK(hipGraphLaunch(e.second, st));
            return KGEV_OK;
        }
    KCHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    kgev_status r = solve_grouped(ctx, grp, o, w, st, (const double2*)dH, (const double2*)dS, ld, nk, dw, C2, ldc,
                                  d_status);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (r != KGEV_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
    }
    if (ec != hipSuccess) return KGEV_EDEVICE;
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return KGEV_EDEVICE;
    if (ctx->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(ctx->graphs.front().second);
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back({key, exec});
    KCHECK(hipGraphLaunch(exec, st));
    return KGEV_OK;
}

kgev_status kgev_solve_k_device_noalloc(kgev_ctx* ctx, const kgev_z* dH, const kgev_z* dS, int64_t n, int64_t ld,
                                        int64_t nk, double* dw, kgev_z* dC, int64_t ldc, int32_t* d_status,
                                        const kgev_opts* opts, void* stream)
{
    if (!ctx) return -1;
    if (!dH) return -2;
    if (!dS) return -3;
    if (n < 1) return -4;
    if (ld < n) return -5;
    if (nk < 1) return -6;
    if (!dw) return -7;
    kgev_opts o = resolve_opts(opts);
    apply_tuned(ctx, n, opts, o);
    if (!opts_valid(o)) return -10;
    if (o.want_vectors && (!dC || ldc < n)) return -8;
    if (o.use_graph || o.streams > 1) return KGEV_EUNSUPPORTED;
    const Groups grp = make_groups(n, nk, o);
    if (grp.region * (size_t)grp.G > KGEV_NOALLOC_SCRATCH_BYTES) return -9;
    DevGuard g(ctx->device);
    void* w = nullptr;
    const kgev_status rs = scratch_address(ctx->device, &w);
    if (rs != KGEV_OK) return rs;
    // no launch of this call is timed (timing may create events)
    void* saved = prof_suspend();
    const kgev_status r = solve_device(grp.p, o, w, (hipStream_t)stream, (const double2*)dH, (const double2*)dS, ld,
                                       dw, o.want_vectors ? (double2*)dC : nullptr, ldc, d_status);
    prof_resume(saved);
    return r;
}

size_t kgev_batch_workspace_bytes(const kgev_problem* probs, int64_t count, const kgev_opts* opts)
{
    if (!probs || count < 1) return 0;
    for (int64_t q = 0; q < count; ++q)
        if (probs[q].n < 1 || probs[q].nk < 1) return 0;
    const kgev_opts o = resolve_opts(opts);
    size_t mx = 0;
    for (const BatchClass& c : batch_classes(probs, count)) mx = std::max(mx, class_layout(probs, c, o).total);
    return mx;
}

kgev_status kgev_solve_batch_device(kgev_ctx* ctx, const kgev_problem* probs, int64_t count, void* dwork,
                                    size_t work_bytes, const kgev_opts* opts, void* stream)
{
    if (!ctx) return -1;
    if (!probs) return -2;
    if (count < 1) return -3;
    const kgev_opts o = resolve_opts(opts);
    if (!opts_valid(o)) return -5;
    for (int64_t q = 0; q < count; ++q) {
        const kgev_problem& pr = probs[q];
        const bool bad = pr.n < 1 || pr.ld < pr.n || pr.nk < 1 || !pr.dH || !pr.dS || !pr.dw ||
                         (o.want_vectors && (!pr.dC || pr.ldc < pr.n));
        if (bad) return (kgev_status)(-(1000 + q));
    }
    DevGuard g(ctx->device);
    const size_t need = kgev_batch_workspace_bytes(probs, count, opts);
    void* w = dwork;
    if (w) {
        if (work_bytes < need) return -4;
    } else {
        const kgev_status r = ensure_work(ctx, need);
        if (r != KGEV_OK) return r;
        w = ctx->work;
    }
    kgev_opts oe = o;     // the kernels are launched directly (a graph, if any, is taken around all of them)
    oe.use_graph = 0;
    const std::vector<BatchClass> classes = batch_classes(probs, count);
    auto run_all = [&](hipStream_t st) -> kgev_status {
        for (const BatchClass& c : classes) {
            const kgev_status r = solve_class(ctx, probs, c, oe, w, st, opts);
            if (r != KGEV_OK) return r;
        }
        return KGEV_OK;
    };
    hipStream_t st = (hipStream_t)stream;
    if (!o.use_graph || st == nullptr) return run_all(st);
    // the graph of this exact batch (problems, buffers, workspace, options, stream)
    std::vector<uintptr_t> key;
    key.reserve((size_t)count * 9 + 16);
    key.push_back((uintptr_t)count);
    key.push_back((uintptr_t)w);
    key.push_back((uintptr_t)stream);
    const unsigned char* ob = reinterpret_cast<const unsigned char*>(&o);
    for (size_t b = 0; b < sizeof(o); b += sizeof(uintptr_t)) {
        uintptr_t v = 0;
        memcpy(&v, ob + b, std::min(sizeof(uintptr_t), sizeof(o) - b));
        key.push_back(v);
    }
    for (int64_t q = 0; q < count; ++q) {
        const kgev_problem& pr = probs[q];
        key.push_back((uintptr_t)pr.n); key.push_back((uintptr_t)pr.ld); key.push_back((uintptr_t)pr.nk);
        key.push_back((uintptr_t)pr.dH); key.push_back((uintptr_t)pr.dS); key.push_back((uintptr_t)pr.dw);
        key.push_back((uintptr_t)(o.want_vectors ? pr.dC : nullptr));
        key.push_back((uintptr_t)(o.want_vectors ? pr.ldc : 0)); key.push_back((uintptr_t)pr.d_status);
    }
    for (size_t q = 0; q < ctx->batch_graphs.size(); ++q)
        if (ctx->batch_graphs[q].first == key) {
            auto e = ctx->batch_graphs[q];
            ctx->batch_graphs.erase(ctx->batch_graphs.begin() + q);
            ctx->batch_graphs.push_back(e);
            KCHECK(hipGraphLaunch(e.second, st));
            return KGEV_OK;
        }
    KCHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const kgev_status r = run_all(st);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (r != KGEV_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
    }
    if (ec != hipSuccess) return KGEV_EDEVICE;
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return KGEV_EDEVICE;
    if (ctx->batch_graphs.size() >= 4) {
        (void)hipStreamSynchronize(st);
        (void)hipGraphExecDestroy(ctx->batch_graphs.front().second);
        ctx->batch_graphs.erase(ctx->batch_graphs.begin());
    }
    ctx->batch_graphs.push_back({key, exec});
    KCHECK(hipGraphLaunch(exec, st));
    return KGEV_OK;
}

kgev_status kgev_solve_k_x_device(kgev_ctx* ctx, const kgev_z* dH, const kgev_z* dS, int64_t n, int64_t ld,
                                  int64_t nk, double* dw, kgev_z* dC, int64_t ldc, kgev_z* dX, int32_t x_mode,
                                  void* dwork, size_t work_bytes, int32_t* d_status, const kgev_opts* opts,
                                  void* stream)
{
    if (!ctx) return -1;
    if (!dH) return -2;
    if (x_mode != KGEV_X_EXPORT && x_mode != KGEV_X_REUSE) return -11;
    if (!dS && x_mode == KGEV_X_EXPORT) return -3;
    if (n < 1) return -4;
    if (ld < n) return -5;
    if (nk < 1) return -6;
    if (!dw) return -7;
    if (!dX) return -10;
    kgev_opts o = resolve_opts(opts);
    apply_tuned(ctx, n, opts, o);
    if (!opts_valid(o)) return -15;
    if (o.want_vectors && (!dC || ldc < n)) return -8;
    if (x_mode == KGEV_X_REUSE && o.s_method == KGEV_S_PRUNE) return KGEV_EUNSUPPORTED;
    DevGuard g(ctx->device);
    SolvePlan p = make_plan(n, nk, o.panel_nb, o.precision == KGEV_PREC_FP32_REFINE, o.hemv_slots);
    void* w = dwork;
    if (w) {
        if (work_bytes < p.total) return -13;
    } else {
        kgev_status r = ensure_work(ctx, p.total);
        if (r != KGEV_OK) return r;
        w = ctx->work;
    }
    return solve_device(p, o, w, (hipStream_t)stream, (const double2*)dH, (const double2*)dS, ld, dw,
                        o.want_vectors ? (double2*)dC : nullptr, ldc, d_status,
                        x_mode == KGEV_X_REUSE ? (const double2*)dX : nullptr,
                        x_mode == KGEV_X_EXPORT ? (double2*)dX : nullptr);
}

kgev_status kgev_solve_k(kgev_ctx* ctx, const kgev_z* H, const kgev_z* S, int64_t n, int64_t nk, double* w,
                         kgev_z* C, const kgev_opts* opts, int64_t* bad_k)
{
    if (bad_k) *bad_k = -1;
    if (!ctx) return -1;
    if (!H) return -2;
    if (!S) return -3;
    if (n < 1) return -4;
    if (nk < 1) return -5;
    if (!w) return -6;
    kgev_opts o = resolve_opts(opts);
    if (!opts_valid(o)) return -8;
    if (o.want_vectors && !C) return -7;
    DevGuard g(ctx->device);
    const size_t mb = sizeof(double2) * (size_t)n * n * nk;
    Layout L;
    const size_t oH = L.add(mb), oS = L.add(mb), oC = L.add(o.want_vectors ? mb : 0),
                 ow = L.add(sizeof(double) * n * nk), ost = L.add(sizeof(int) * nk);
    if (ctx->stage_bytes < L.total) {
        if (ctx->stage) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipFree(ctx->stage);
        }
        ctx->stage = nullptr;
        ctx->stage_bytes = 0;
        if (hipMalloc(&ctx->stage, L.total) != hipSuccess) return KGEV_ENOMEM;
        ctx->stage_bytes = L.total;
    }
    char* base = static_cast<char*>(ctx->stage);
    hipStream_t st = ctx->stream;
    KCHECK(hipMemcpyAsync(base + oH, H, mb, hipMemcpyHostToDevice, st));
    KCHECK(hipMemcpyAsync(base + oS, S, mb, hipMemcpyHostToDevice, st));
    kgev_status r = kgev_solve_k_device(ctx, (const kgev_z*)(base + oH), (const kgev_z*)(base + oS), n, n, nk,
                                        (double*)(base + ow), o.want_vectors ? (kgev_z*)(base + oC) : nullptr, n,
                                        nullptr, 0, (int32_t*)(base + ost), &o, st);
    if (r != KGEV_OK) return r;
    KCHECK(hipMemcpyAsync(w, base + ow, sizeof(double) * n * nk, hipMemcpyDeviceToHost, st));
    if (o.want_vectors) KCHECK(hipMemcpyAsync(C, base + oC, mb, hipMemcpyDeviceToHost, st));
    std::vector<int32_t> stv((size_t)nk);
    KCHECK(hipMemcpyAsync(stv.data(), base + ost, sizeof(int32_t) * nk, hipMemcpyDeviceToHost, st));
    KCHECK(hipStreamSynchronize(st));
    for (int64_t q = 0; q < nk; ++q)
        if (stv[q] != 0) {
            if (bad_k) *bad_k = q;
            return stv[q];
        }
    return KGEV_OK;
}

kgev_status kgev_hetrd_device(kgev_ctx* ctx, kgev_z* dA, int64_t n, int64_t lda, int64_t nk, double* dd, double* de,
                              kgev_z* dtau, kgev_z* dV, const kgev_opts* opts, void* stream)
{
    if (!ctx) return -1;
    if (!dA) return -2;
    if (n < 1) return -3;
    if (lda < n) return -4;
    if (nk < 1) return -5;
    if (!dd) return -6;
    if (!de) return -7;
    if (!dtau) return -8;
    if (!dV) return -9;
    kgev_opts o = resolve_opts(opts);
    if (o.panel_nb < 1 || o.panel_nb > 64 || o.hemv_slots < 1 || o.gemm_slots < 1) return -10;
    DevGuard g(ctx->device);
    const TileScope tiles(o.gemm_slots);
    SolvePlan p = make_plan(n, nk, o.panel_nb, false, o.hemv_slots);
    kgev_status r = ensure_work(ctx, p.total);
    if (r != KGEV_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    const int64_t nn = n * n;
    KCHECK(fill_zero(st, dV, sizeof(double2) * (size_t)nn * nk));
    KCHECK(hetrd<double>(st, hetrd_ws(p, ctx->work, (double2*)dA, lda, lda * n, (double2*)dV, dd, de, (double2*)dtau),
                         nk));
    return KGEV_OK;
}

kgev_status kgev_stedc_device(kgev_ctx* ctx, const double* dd, const double* de, int64_t n, int64_t nk, double* dw,
                              double* dZ, int32_t* d_status, void* stream)
{
    if (!ctx) return -1;
    if (!dd) return -2;
    if (!de) return -3;
    if (n < 1) return -4;
    if (nk < 1) return -5;
    if (!dw) return -6;
    if (!dZ) return -7;
    DevGuard g(ctx->device);
    SolvePlan p = make_plan(n, nk, DEFAULT_NB);
    kgev_status r = ensure_work(ctx, p.total);
    if (r != KGEV_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    int* status = at<int>(ctx->work, p.status);
    KCHECK(status_init(st, status, nk));
    KCHECK(stedc(st, dc_ws(p, ctx->work, dd, de, status), dw, dZ, at<double>(ctx->work, p.Qs), nk));
    if (d_status) KCHECK(status_finish(st, status, d_status, nk));
    return KGEV_OK;
}

kgev_status kgev_stebz_device(kgev_ctx* ctx, const double* dd, const double* de, int64_t n, int64_t nk, double* dw,
                              void* stream)
{
    if (!ctx) return -1;
    if (!dd) return -2;
    if (!de) return -3;
    if (n < 1) return -4;
    if (nk < 1) return -5;
    if (!dw) return -6;
    DevGuard g(ctx->device);
    const kgev_status r = ensure_work(ctx, stebz_work_bytes(nk));
    if (r != KGEV_OK) return r;
    KCHECK(stebz((hipStream_t)stream, dd, de, n, n, nk, dw, n, ctx->work));
    return KGEV_OK;
}

kgev_status kgev_unmtr_device(kgev_ctx* ctx, const kgev_z* dV, const kgev_z* dtau, int64_t n, int64_t nk, kgev_z* dU,
                              int64_t ldu, void* stream)
{
    if (!ctx) return -1;
    if (!dV) return -2;
    if (!dtau) return -3;
    if (n < 1) return -4;
    if (nk < 1) return -5;
    if (!dU) return -6;
    if (ldu < n) return -7;
    DevGuard g(ctx->device);
    SolvePlan p = make_plan(n, nk, DEFAULT_NB);
    kgev_status r = ensure_work(ctx, p.total);
    if (r != KGEV_OK) return r;
    const int64_t nn = n * n;
    KCHECK(unmtr<double>((hipStream_t)stream, n, (const double2*)dV, nn, (const double2*)dtau, n, (double2*)dU, ldu,
                         ldu * n, at<double2>(ctx->work, p.uwork), p.kb, nk));
    return KGEV_OK;
}

kgev_status kgev_eigh_device(kgev_ctx* ctx, const kgev_z* dA, int64_t n, int64_t lda, int64_t nk, double* dw,
                             kgev_z* dY, int32_t* d_status, const kgev_opts* opts, void* stream)
{
    if (!ctx) return -1;
    if (!dA) return -2;
    if (n < 1) return -3;
    if (lda < n) return -4;
    if (nk < 1) return -5;
    if (!dw) return -6;
    kgev_opts o = resolve_opts(opts);
    if (o.panel_nb < 1 || o.panel_nb > 64 || o.hemv_slots < 1 || o.gemm_slots < 1) return -9;
    DevGuard g(ctx->device);
    const TileScope tiles(o.gemm_slots);
    SolvePlan p = make_plan(n, nk, o.panel_nb, false, o.hemv_slots);
    kgev_status r = ensure_work(ctx, p.total);
    if (r != KGEV_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    void* w = ctx->work;
    int* status = at<int>(w, p.status);
    const int64_t nn = n * n;
    KCHECK(status_init(st, status, nk));
    KCHECK(copy_lower_check<double>(st, n, (const double2*)dA, lda, lda * n, at<double2>(w, p.Aw), n, nn, status, nk));
    r = eigen_hh(p, w, st, dw, (double2*)dY, status, dY == nullptr);
    if (r != KGEV_OK) return r;
    if (dY) KCHECK(normalize_cols(st, n, (double2*)dY, n, nn, nullptr, 0, 0.0, nullptr, nk));
    if (d_status) KCHECK(status_finish(st, status, d_status, nk));
    return KGEV_OK;
}

kgev_status kgev_zgemm_device(kgev_ctx* ctx, char transa, char transb, int64_t m, int64_t n, int64_t k, kgev_z alpha,
                              const kgev_z* dA, int64_t lda, int64_t sA, const kgev_z* dB, int64_t ldb, int64_t sB,
                              kgev_z beta, kgev_z* dC, int64_t ldc, int64_t sC, int64_t batch, int32_t lower,
                              void* stream)
{
    if (!ctx) return -1;
    if (transa != 'N' && transa != 'C') return -2;
    if (transb != 'N' && transb != 'C') return -3;
    if (m < 0) return -4;
    if (n < 0) return -5;
    if (k < 0) return -6;
    if (!dA && m > 0 && k > 0) return -8;
    if (lda < std::max<int64_t>(1, transa == 'N' ? m : k)) return -9;
    if (!dB && n > 0 && k > 0) return -11;
    if (ldb < std::max<int64_t>(1, transb == 'N' ? k : n)) return -12;
    if (!dC && m > 0 && n > 0) return -15;
    if (ldc < std::max<int64_t>(1, m)) return -16;
    if (batch < 0) return -18;
    if (lower && m != n) return -19;
    DevGuard g(ctx->device);
    KCHECK(cgemm<double>((hipStream_t)stream, transa, transb, m, n, k, mk<double>(alpha.re, alpha.im),
                         (const double2*)dA, lda, sA, (const double2*)dB, ldb, sB, mk<double>(beta.re, beta.im),
                         (double2*)dC, ldc, sC, batch, lower != 0));
    return KGEV_OK;
}

kgev_status kgev_fermi_device(kgev_ctx* ctx, const double* dw, int64_t ldw, int64_t n, int64_t nk,
                              const double* d_wk, double nelec, double kT, double g, double* d_occ, int64_t ldo,
                              double* d_result, int32_t* d_status, void* stream)
{
    if (!ctx) return -1;
    if (!dw) return -2;
    if (n < 1 || n > INT32_MAX) return -4;
    if (ldw < n) return -3;
    if (nk < 1 || nk > INT32_MAX) return -5;
    if (!d_wk) return -6;
    if (!(kT > 0.0) || !(kT < INFINITY)) return -8;
    if (!(g > 0.0) || !(g < INFINITY)) return -9;
    if (d_occ && ldo < n) return -11;
    if (!d_result) return -12;
    if (!d_status) return -13;
    DevGuard gd(ctx->device);
    KCHECK(fermi_level((hipStream_t)stream, dw, ldw, (int)n, (int)nk, d_wk, nelec, kT, g, d_occ, ldo, d_result,
                       d_status));
    return KGEV_OK;
}

size_t kgev_density_workspace_bytes(int64_t n, int64_t nk, int64_t nocc)
{
    if (n < 1 || nk < 1 || nocc < 0 || nocc > n) return 0;
    return density_work_bytes(n, nk, nocc);
}

kgev_status kgev_density_device(kgev_ctx* ctx, const kgev_z* dC, int64_t ldc, int64_t n, int64_t nk, int64_t nocc,
                                const double* dw, int64_t ldw, const double* d_occ, int64_t ldo, const double* d_wk,
                                double g, kgev_z* d_rho, kgev_z* d_edm, int64_t ldr, void* dwork, size_t work_bytes,
                                void* stream)
{
    if (!ctx) return -1;
    if (!dC) return -2;
    if (n < 1 || n > INT32_MAX) return -4;
    if (ldc < n) return -3;
    if (nk < 1 || nk > INT32_MAX) return -5;
    if (nocc < 0 || nocc > n) return -6;
    if (!dw) return -7;
    if (ldw < n) return -8;
    if (!d_occ) return -9;
    if (ldo < n) return -10;
    if (!d_wk) return -11;
    if (!(g > 0.0) || !(g < INFINITY)) return -12;
    if (!d_rho) return -13;
    if (ldr < n) return -15;
    if (n > 65535) return KGEV_EUNSUPPORTED;   // one grid row per column
    const size_t need = density_work_bytes(n, nk, nocc);
    DevGuard gd(ctx->device);
    void* w = dwork;
    if (!w) {
        const kgev_status s = ensure_work(ctx, need);
        if (s != KGEV_OK) return s;
        w = ctx->work;
    } else if (work_bytes < need) {
        return -17;
    }
    KCHECK(density((hipStream_t)stream, (const double2*)dC, ldc, (int)n, (int)nk, (int)nocc, dw, ldw, d_occ, ldo,
                   d_wk, g, (double2*)d_rho, (double2*)d_edm, ldr, w));
    return KGEV_OK;
}

kgev_status kgev_bloch_device(kgev_ctx* ctx, int32_t natom, const int32_t* off, int64_t nblocks, const int32_t* bi,
                              const int32_t* bj, const int32_t* rid, const int64_t* doff, const kgev_z* d_data,
                              int64_t data_elems, int64_t nR, const double* R, int64_t nk, const double* kf,
                              kgev_z* d_out, void* stream)
{
    if (!ctx) return -1;
    if (natom < 1 || !off) return -2;
    if (off[0] != 0) return -3;
    for (int32_t a = 0; a < natom; ++a)
        if (off[a + 1] < off[a]) return -3;
    const int64_t n = off[natom];
    if (n < 1 || n > 65535) return -3;
    if (nblocks < 0) return -4;
    if (nblocks > 0 && (!bi || !bj || !rid || !doff || !d_data)) return -5;
    if (data_elems < 0) return -10;
    if (nR < 0 || (nR > 0 && !R)) return -11;
    if (nk < 1 || !kf) return -13;
    if (!d_out) return -15;
    // validate every block and group consecutive blocks of one atom pair
    std::vector<int32_t> gptr;
    for (int64_t q = 0; q < nblocks; ++q) {
        if (bi[q] < 0 || bi[q] >= natom || bj[q] < 0 || bj[q] >= natom) return -5;
        if (rid[q] < 0 || rid[q] >= nR) return -7;
        const int64_t sz = (int64_t)(off[bi[q] + 1] - off[bi[q]]) * (off[bj[q] + 1] - off[bj[q]]);
        if (doff[q] < 0 || doff[q] + sz > data_elems) return -8;
        if (q > 0) {
            const bool same = bi[q] == bi[q - 1] && bj[q] == bj[q - 1];
            const bool after = bi[q] > bi[q - 1] || (bi[q] == bi[q - 1] && bj[q] > bj[q - 1]);
            if (!same && !after) return -4;      // blocks must be sorted by (I, J)
            if (!same) gptr.push_back((int32_t)q);
        } else {
            gptr.push_back(0);
        }
    }
    gptr.push_back((int32_t)nblocks);
    const int64_t ngroups = nblocks > 0 ? (int64_t)gptr.size() - 1 : 0;
    DevGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    // metadata: one stream-ordered allocation, freed after the kernels
    Layout L;
    const size_t o_off = L.add(sizeof(int32_t) * (natom + 1)), o_gp = L.add(sizeof(int32_t) * gptr.size()),
                 o_bi = L.add(sizeof(int32_t) * nblocks), o_bj = L.add(sizeof(int32_t) * nblocks),
                 o_rid = L.add(sizeof(int32_t) * nblocks), o_doff = L.add(sizeof(int64_t) * nblocks),
                 o_R = L.add(sizeof(double) * 3 * nR), o_k = L.add(sizeof(double) * 3 * nk),
                 o_ph = L.add(sizeof(double2) * nk * nR);
    std::vector<char> host(L.total);
    auto put = [&](size_t o, const void* src, size_t bytes) {
        if (bytes) memcpy(host.data() + o, src, bytes);
    };
    put(o_off, off, sizeof(int32_t) * (natom + 1));
    put(o_gp, gptr.data(), sizeof(int32_t) * gptr.size());
    put(o_bi, bi, sizeof(int32_t) * nblocks);
    put(o_bj, bj, sizeof(int32_t) * nblocks);
    put(o_rid, rid, sizeof(int32_t) * nblocks);
    put(o_doff, doff, sizeof(int64_t) * nblocks);
    put(o_R, R, sizeof(double) * 3 * nR);
    put(o_k, kf, sizeof(double) * 3 * nk);
    char* dm = nullptr;
    if (hipMallocAsync((void**)&dm, L.total, st) != hipSuccess) return KGEV_ENOMEM;
    KCHECK(hipMemcpyAsync(dm, host.data(), L.total, hipMemcpyHostToDevice, st));
    KCHECK(hipStreamSynchronize(st));          // the host staging may go out of scope
    const hipError_t e = bloch_sum(st, (int)n, (const int*)(dm + o_off), ngroups, (const int*)(dm + o_gp),
                                   (const int*)(dm + o_bi), (const int*)(dm + o_bj), (const int*)(dm + o_rid),
                                   (const int64_t*)(dm + o_doff), (const double2*)d_data, nR,
                                   (const double*)(dm + o_R), nk, (const double*)(dm + o_k), (double2*)(dm + o_ph),
                                   (double2*)d_out);
    (void)hipFreeAsync(dm, st);
    if (e != hipSuccess) return KGEV_EDEVICE;
    return KGEV_OK;
}

kgev_status kgev_profile_begin(kgev_ctx* ctx, int32_t phase, int32_t stride)
{
    if (!ctx) return -1;
    if (phase != KGEV_PHASE_HEMV && phase != KGEV_PHASE_GEMM) return -2;
    if (stride < 1) return -3;
    DevGuard g(ctx->device);
    drop_graphs(ctx);
    if (ctx->prof) prof_stop(ctx->prof, nullptr, nullptr, nullptr, nullptr, nullptr);
    ctx->prof = prof_start(phase, stride, 16384);
    return KGEV_OK;
}

kgev_status kgev_profile_end(kgev_ctx* ctx, int64_t* launches, int64_t* phase_launches, double* total_ms,
                             double* alg_bytes, double* alg_flops)
{
    if (!ctx) return -1;
    if (!ctx->prof) return KGEV_EUNSUPPORTED;
    DevGuard g(ctx->device);
    const bool ok = prof_stop(ctx->prof, launches, phase_launches, total_ms, alg_bytes, alg_flops);
    ctx->prof = nullptr;
    drop_graphs(ctx);
    return ok ? KGEV_OK : KGEV_EDEVICE;
}

kgev_status kgev_autotune(kgev_ctx* ctx, int64_t n, int32_t precision, int32_t* best_nb)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (precision != KGEV_PREC_FP64 && precision != KGEV_PREC_FP32_REFINE) return -3;
    DevGuard g(ctx->device);
    const int64_t nk = 4;
    const bool mixed = precision == KGEV_PREC_FP32_REFINE;
    SolvePlan base = make_plan(n, nk, 64, mixed);
    kgev_status r = ensure_work(ctx, base.total);
    if (r != KGEV_OK) return r;
    hipStream_t st = ctx->stream;
    hipEvent_t e0, e1;
    KCHECK(hipEventCreate(&e0));
    KCHECK(hipEventCreate(&e1));
    const int64_t nn = n * n;
    // one timed reduction of the nk synthetic matrices
    auto time_one = [&](int nb, int slots, float& ms) -> hipError_t {
        SolvePlan p = make_plan(n, nk, nb, mixed, slots);
        void* w = ctx->work;
        hipError_t e;
        if (mixed) {
            HetrdWs<float> h = hetrd_ws32(p, w);
            if ((e = fill_test_matrix<float>(st, n, h.A, nk, 17)) != hipSuccess) return e;
            if ((e = fill_zero(st, h.V, sizeof(float2) * (size_t)nn * nk)) != hipSuccess) return e;
            if ((e = hipEventRecord(e0, st)) != hipSuccess) return e;
            if ((e = hetrd<float>(st, h, nk)) != hipSuccess) return e;
        } else {
            double2* Aw = at<double2>(w, p.Aw);
            double2* Vs = at<double2>(w, p.Vs);
            if ((e = fill_test_matrix<double>(st, n, Aw, nk, 17)) != hipSuccess) return e;
            if ((e = fill_zero(st, Vs, sizeof(double2) * (size_t)nn * nk)) != hipSuccess) return e;
            if ((e = hipEventRecord(e0, st)) != hipSuccess) return e;
            if ((e = hetrd<double>(st, hetrd_ws(p, w, Aw, n, nn, Vs, at<double>(w, p.d), at<double>(w, p.e),
                                                at<double2>(w, p.tau)),
                                   nk)) != hipSuccess)
                return e;
        }
        if ((e = hipEventRecord(e1, st)) != hipSuccess) return e;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
        return hipEventElapsedTime(&ms, e0, e1);
    };
    // panel width (first pass warms up, second pass decides)
    const int cands[] = {16, 24, 32, 48, 64};
    int best = DEFAULT_NB;
    float best_ms = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
        for (int nb : cands) {
            float ms = 0;
            KCHECK(time_one(nb, DEFAULT_SLOTS, ms));
            if (rep == 1 && ms < best_ms) {
                best_ms = ms;
                best = nb;
            }
        }
    }
    // tile grouping of the Hermitian product at that width: the default
    // unless another threshold is faster by more than 2% (best of two runs)
    const int slots_c[] = {1, 256, DEFAULT_SLOTS, 2048, 1 << 30};
    float t_def = 1e30f;
    float t_c[5];
    for (int q = 0; q < 5; ++q) {
        t_c[q] = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
            float ms = 0;
            KCHECK(time_one(best, slots_c[q], ms));
            t_c[q] = std::min(t_c[q], ms);
        }
        if (slots_c[q] == DEFAULT_SLOTS) t_def = t_c[q];
    }
    int best_slots = DEFAULT_SLOTS;
    float best_t = t_def;
    for (int q = 0; q < 5; ++q)
        if (t_c[q] < 0.98f * t_def && t_c[q] < best_t) {
            best_t = t_c[q];
            best_slots = slots_c[q];
        }
    // product tiles: the n x n x n products of Parts 3 and 4 (G = H X, then
    // the lower half of X^H G) on the reduction's matrices
    const int gemm_c[] = {1, 64, GEMM_SMALL_SLOTS_DEFAULT, 1024, 1 << 30};
    float g_c[5], g_def = 1e30f;
    {
        SolvePlan p = make_plan(n, nk, best, false);
        double2* A = at<double2>(ctx->work, p.Aw);
        double2* B = at<double2>(ctx->work, p.Vs);
        double2* Cm = at<double2>(ctx->work, p.X);
        KCHECK(fill_test_matrix<double>(st, n, A, nk, 19));
        KCHECK(fill_test_matrix<double>(st, n, B, nk, 23));
        const double2 one = mk<double>(1, 0), zero = mk<double>(0, 0);
        for (int q = 0; q < 5; ++q) {
            g_c[q] = 1e30f;
            const TileScope tiles(gemm_c[q]);
            for (int rep = 0; rep < 2; ++rep) {
                KCHECK(hipEventRecord(e0, st));
                KCHECK(cgemm<double>(st, 'N', 'N', n, n, n, one, A, n, nn, B, n, nn, zero, Cm, n, nn, nk, false));
                KCHECK(cgemm<double>(st, 'C', 'N', n, n, n, one, B, n, nn, Cm, n, nn, zero, A, n, nn, nk, true));
                KCHECK(hipEventRecord(e1, st));
                KCHECK(hipEventSynchronize(e1));
                float ms = 0;
                KCHECK(hipEventElapsedTime(&ms, e0, e1));
                g_c[q] = std::min(g_c[q], ms);
            }
            if (gemm_c[q] == GEMM_SMALL_SLOTS_DEFAULT) g_def = g_c[q];
        }
    }
    int best_gemm = GEMM_SMALL_SLOTS_DEFAULT;
    float best_g = g_def;
    for (int q = 0; q < 5; ++q)
        if (g_c[q] < 0.98f * g_def && g_c[q] < best_g) {
            best_g = g_c[q];
            best_gemm = gemm_c[q];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->tuned[{n, precision}] = {best, best_slots, best_gemm};
    if (best_nb) *best_nb = best;
    return KGEV_OK;
}

kgev_status kgev_tuned_params(kgev_ctx* ctx, int64_t n, int32_t precision, int32_t* panel_nb, int32_t* hemv_slots,
                              int32_t* gemm_slots, int32_t* tuned)
{
    if (!ctx) return -1;
    if (precision != KGEV_PREC_FP64 && precision != KGEV_PREC_FP32_REFINE) return -3;
    auto it = ctx->tuned.find({n, precision});
    const bool t = it != ctx->tuned.end();
    if (panel_nb) *panel_nb = t ? it->second.nb : DEFAULT_NB;
    if (hemv_slots) *hemv_slots = t ? it->second.hemv_slots : DEFAULT_SLOTS;
    if (gemm_slots) *gemm_slots = t ? it->second.gemm_slots : GEMM_SMALL_SLOTS_DEFAULT;
    if (tuned) *tuned = t ? 1 : 0;
    return KGEV_OK;
}

}  // extern "C"
