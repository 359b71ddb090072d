// Shared device helpers of the HIP library: complex arithmetic on interleaved
// (re, im) pairs, buffer loads and the MFMA wrappers (cross-lane reductions:
// lanes.hpp).  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kgev {

constexpr int WAVE = 64;

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef int i4_t __attribute__((ext_vector_type(4)));
typedef int i2_t __attribute__((ext_vector_type(2)));

// Raw buffer loads (MUBUF): address = base + voffset (per lane, 32-bit) +
// soffset (wave-uniform, 32-bit); an access at or beyond `bytes` returns 0.
// The descriptor's third word is the raw-buffer format of the gfx9 family.
__device__ i4_t raw_buffer_load_v4i32(i4_t rsrc, int voffset, int soffset, int aux) __asm("llvm.amdgcn.raw.buffer.load.v4i32");
__device__ i2_t raw_buffer_load_v2i32(i4_t rsrc, int voffset, int soffset, int aux) __asm("llvm.amdgcn.raw.buffer.load.v2i32");

__device__ inline i4_t buffer_rsrc(const void* base, uint32_t bytes)
{
    const uint64_t a = reinterpret_cast<uint64_t>(base);
    i4_t r;
    r.x = (int)(uint32_t)(a & 0xffffffffu);
    r.y = (int)(uint32_t)(a >> 32);
    r.z = (int)bytes;
    r.w = 0x00020000;
    return r;
}

// ---------------------------------------------------------------------------
// complex numbers: double2 / float2 with x = re, y = im
template <typename R> struct Cx;
template <> struct Cx<double> { using T = double2; };
template <> struct Cx<float> { using T = float2; };
template <typename R> using cx = typename Cx<R>::T;

template <typename R> __device__ __host__ inline cx<R> mk(R re, R im) { cx<R> z; z.x = re; z.y = im; return z; }
template <typename C> __device__ inline C cadd(C a, C b) { C z; z.x = a.x + b.x; z.y = a.y + b.y; return z; }
template <typename C> __device__ inline C csub(C a, C b) { C z; z.x = a.x - b.x; z.y = a.y - b.y; return z; }
template <typename C> __device__ inline C cmul(C a, C b)
{
    C z;
    z.x = a.x * b.x - a.y * b.y;
    z.y = a.x * b.y + a.y * b.x;
    return z;
}
// conj(a) * b
template <typename C> __device__ inline C cmulc(C a, C b)
{
    C z;
    z.x = a.x * b.x + a.y * b.y;
    z.y = a.x * b.y - a.y * b.x;
    return z;
}
// acc + a * b
template <typename C> __device__ inline C cfma(C a, C b, C acc)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a) * b
template <typename C> __device__ inline C cfmac(C a, C b, C acc)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
template <typename C> __device__ inline C cconj(C a) { a.y = -a.y; return a; }
template <typename C, typename R> __device__ inline C cscale(C a, R s) { a.x *= s; a.y *= s; return a; }
template <typename C> __device__ inline C czero() { C z; z.x = 0; z.y = 0; return z; }
// Component-wise select.  A conditional expression on the vector type itself
// can be lowered through scratch memory; selecting the components is not.
template <typename C> __device__ inline C csel(bool c, C a, C b)
{
    C r;
    r.x = c ? a.x : b.x;
    r.y = c ? a.y : b.y;
    return r;
}

// ---------------------------------------------------------------------------
// MFMA 16x16x4 (one block): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  Accumulator register r of lane l holds D[row][l % 16]
// with row = l / 16 + 4 r for the FP64 instruction and row = 4 (l / 16) + r
// for the FP32 one (both measured on gfx950 with an in-bounds probe).
template <typename R> struct Mfma;
template <> struct Mfma<double> {
    using acc_t = d4_t;
    static __device__ inline acc_t mma(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Mfma<float> {
    using acc_t = f4_t;
    static __device__ inline acc_t mma(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lk, int r) { return 4 * lk + r; }
};

}  // namespace kgev
