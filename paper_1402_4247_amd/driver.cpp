// kgev_driver: a native command-line driver of the C ABI.  It solves nk
// Hermitian-definite pencils H C = S C Lambda of order n (Band_DFT_Col Parts
// 2-4, Section III of arXiv:1402.4247) with kgev_solve_k_device, inputs
// resident in device memory, and prints the time per call.  It needs no
// Python, so it can run under profilers that collect hardware counters.
//
// Inputs (seeded, synthetic): H with entries uniform in [-0.5, 0.5] (real
// diagonal), S = I + W with W Hermitian, zero diagonal and entries uniform
// in a disc of radius 0.5 / n, so every Gershgorin disc of S lies in
// [0.5, 1.5] and S is positive definite.  The cost of every step of the
// solve depends only on n and nk, not on the values.
//
// usage: kgev_driver [--n N] [--nk K] [--steps S] [--warmup W]
//        kgev_driver --copy-mib M   (three device-to-device copies of M MiB
//        and nothing else: the reference of known size for scaling a
//        profiler's HBM byte counters)
// exit status: 0 if every call returned KGEV_OK with every k-point's status
// 0, 1 otherwise.
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "kgev.h"

namespace {

// splitmix64: a seeded, portable stream of uniform doubles in [0, 1)
struct Rng {
    uint64_t s;
    double next()
    {
        uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    }
};

bool ok(hipError_t e, const char* what)
{
    if (e != hipSuccess) std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return e == hipSuccess;
}

}  // namespace

int main(int argc, char** argv)
{
    int64_t n = 2000, nk = 16, copy_mib = 0;
    int steps = 1, warmup = 1;
    for (int a = 1; a + 1 < argc; a += 2) {
        if (!std::strcmp(argv[a], "--n")) n = std::atoll(argv[a + 1]);
        else if (!std::strcmp(argv[a], "--nk")) nk = std::atoll(argv[a + 1]);
        else if (!std::strcmp(argv[a], "--steps")) steps = std::atoi(argv[a + 1]);
        else if (!std::strcmp(argv[a], "--warmup")) warmup = std::atoi(argv[a + 1]);
        else if (!std::strcmp(argv[a], "--copy-mib")) copy_mib = std::atoll(argv[a + 1]);
        else {
            std::fprintf(stderr, "usage: %s [--n N] [--nk K] [--steps S] [--warmup W]\n", argv[0]);
            return 1;
        }
    }
    if (n < 1 || nk < 1 || steps < 0 || warmup < 0 || copy_mib < 0) return 1;
    if (copy_mib > 0) {
        const size_t bytes = (size_t)copy_mib << 20;
        void *src = nullptr, *dst = nullptr;
        if (!ok(hipMalloc(&src, bytes), "hipMalloc") || !ok(hipMalloc(&dst, bytes), "hipMalloc") ||
            !ok(hipMemset(src, 1, bytes), "hipMemset"))
            return 1;
        for (int r = 0; r < 3; ++r)
            if (!ok(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToDevice), "hipMemcpy")) return 1;
        std::printf("[driver] copied %lld MiB three times\n", (long long)copy_mib);
        (void)hipFree(src);
        (void)hipFree(dst);
        return 0;
    }
    const size_t nn = (size_t)n * (size_t)n;
    std::vector<kgev_z> H(nn * nk), S(nn * nk);
    Rng rng{20260001};
    for (int64_t k = 0; k < nk; ++k) {
        kgev_z* h = H.data() + nn * k;
        kgev_z* s = S.data() + nn * k;
        for (int64_t c = 0; c < n; ++c)
            for (int64_t r = c; r < n; ++r) {
                kgev_z hv, sv;
                hv.re = rng.next() - 0.5;
                hv.im = r == c ? 0.0 : rng.next() - 0.5;
                if (r == c) {
                    sv.re = 1.0;
                    sv.im = 0.0;
                } else {
                    const double rad = 0.5 / (double)n * rng.next(), ang = 6.283185307179586 * rng.next();
                    sv.re = rad * __builtin_cos(ang);
                    sv.im = rad * __builtin_sin(ang);
                }
                h[r + c * n] = hv;
                s[r + c * n] = sv;
            }
    }
    kgev_z *dH = nullptr, *dS = nullptr, *dC = nullptr;
    double* dw = nullptr;
    int32_t* dst = nullptr;
    if (!ok(hipMalloc((void**)&dH, sizeof(kgev_z) * nn * nk), "hipMalloc") ||
        !ok(hipMalloc((void**)&dS, sizeof(kgev_z) * nn * nk), "hipMalloc") ||
        !ok(hipMalloc((void**)&dC, sizeof(kgev_z) * nn * nk), "hipMalloc") ||
        !ok(hipMalloc((void**)&dw, sizeof(double) * n * nk), "hipMalloc") ||
        !ok(hipMalloc((void**)&dst, sizeof(int32_t) * nk), "hipMalloc"))
        return 1;
    if (!ok(hipMemcpy(dH, H.data(), sizeof(kgev_z) * nn * nk, hipMemcpyHostToDevice), "hipMemcpy") ||
        !ok(hipMemcpy(dS, S.data(), sizeof(kgev_z) * nn * nk, hipMemcpyHostToDevice), "hipMemcpy"))
        return 1;
    kgev_ctx* ctx = nullptr;
    if (kgev_create(&ctx, 0) != KGEV_OK) {
        std::fprintf(stderr, "kgev_create failed\n");
        return 1;
    }
    hipStream_t st;
    if (!ok(hipStreamCreate(&st), "hipStreamCreate")) return 1;
    bool good = true;
    double total_ms = 0.0;
    for (int it = 0; it < warmup + steps; ++it) {
        const auto t0 = std::chrono::steady_clock::now();
        const kgev_status r = kgev_solve_k_device(ctx, dH, dS, n, n, nk, dw, dC, n, nullptr, 0, dst, nullptr, st);
        if (!ok(hipStreamSynchronize(st), "hipStreamSynchronize")) return 1;
        const auto t1 = std::chrono::steady_clock::now();
        std::vector<int32_t> stat(nk);
        if (!ok(hipMemcpy(stat.data(), dst, sizeof(int32_t) * nk, hipMemcpyDeviceToHost), "hipMemcpy")) return 1;
        bool all0 = r == KGEV_OK;
        for (int32_t v : stat) all0 = all0 && v == 0;
        good = good && all0;
        const double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        if (it >= warmup) total_ms += ms;
        std::printf("[driver] call %d: %.1f ms, %s\n", it, ms, all0 ? "ok" : "FAILED");
        std::fflush(stdout);
    }
    if (steps > 0)
        std::printf("[driver] n=%lld nk=%lld: %.1f ms per call, %.2f solves/s\n", (long long)n, (long long)nk,
                    total_ms / steps, 1e3 * (double)nk * steps / total_ms);
    (void)hipStreamDestroy(st);
    kgev_destroy(ctx);
    (void)hipFree(dH);
    (void)hipFree(dS);
    (void)hipFree(dC);
    (void)hipFree(dw);
    (void)hipFree(dst);
    return good ? 0 : 1;
}
