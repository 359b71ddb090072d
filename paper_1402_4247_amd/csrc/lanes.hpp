// Cross-lane exchanges and reductions as vector-ALU operations (DPP and the
// gfx950 permlane swaps).  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>

namespace kgev {

// Exchange with lane ^ M as a vector-ALU operation: DPP (a lane-permuting
// operand modifier) within rows of 16 lanes, the gfx950 permlane swaps across
// rows.  __shfl_xor goes through the LDS unit instead (ds_bpermute: one LDS
// round trip per butterfly step), and in latency-bound kernels those chains
// dominate.  DPP controls (GCN3+ encoding):
//   0xB1 quad_perm(1,0,3,2) = lane ^ 1,  0x4E quad_perm(2,3,0,1) = lane ^ 2,
//   0x141 row_half_mirror (i -> 7 - i in each 8) followed by
//   0x1B quad_perm(3,2,1,0) (i -> i ^ 3) = lane ^ 4,
//   0x128 row_ror:8 (rotation by 8 in each row of 16) = lane ^ 8.
// v_permlane16_swap / v_permlane32_swap of a register with itself return, in
// one of their two results, the values of the other row of a row pair / the
// other half of the wave.  All lanes taking part must be active.
// (every pattern used here reads a lane of the same row, so no lane keeps an
// old value and none needs initialising)
template <int CTRL> __device__ inline int dpp(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int M> __device__ inline int lane_xor(int v)
{
    static_assert(M == 1 || M == 2 || M == 4 || M == 8 || M == 16 || M == 32, "lane mask");
    if constexpr (M == 1) {
        return dpp<0xB1>(v);
    } else if constexpr (M == 2) {
        return dpp<0x4E>(v);
    } else if constexpr (M == 4) {
        return dpp<0x1B>(dpp<0x141>(v));
    } else if constexpr (M == 8) {
        return dpp<0x128>(v);
    } else if constexpr (M == 16) {
        const auto s = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
        return (int)((__lane_id() & 16) ? s[0] : s[1]);
    } else {
        const auto s = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
        return (int)((__lane_id() & 32) ? s[0] : s[1]);
    }
}
template <int M> __device__ inline float lane_xor(float v) { return __int_as_float(lane_xor<M>(__float_as_int(v))); }
template <int M> __device__ inline double lane_xor(double v)
{
    return __hiloint2double(lane_xor<M>(__double2hiint(v)), lane_xor<M>(__double2loint(v)));
}
// Transposing exchange of a pair (a, b) across lane bit M (16 or 32): lanes
// with the bit clear end with (own a, the partner's a), lanes with it set
// with (the partner's b, own b), so a + b is each lane's kept value (a below
// the bit, b above it) plus the partner's copy of it.  One permlane swap per
// 32-bit word and no selects.
template <int M> __device__ inline void swap_across(int& a, int& b)
{
    static_assert(M == 16 || M == 32, "row pair or wave half");
    if constexpr (M == 32) {
        const auto s = __builtin_amdgcn_permlane32_swap((unsigned)a, (unsigned)b, false, false);
        a = (int)s[0];
        b = (int)s[1];
    } else {
        const auto s = __builtin_amdgcn_permlane16_swap((unsigned)a, (unsigned)b, false, false);
        a = (int)s[0];
        b = (int)s[1];
    }
}
template <int M> __device__ inline void swap_across(double& a, double& b)
{
    int ah = __double2hiint(a), al = __double2loint(a), bh = __double2hiint(b), bl = __double2loint(b);
    swap_across<M>(ah, bh);
    swap_across<M>(al, bl);
    a = __hiloint2double(ah, al);
    b = __hiloint2double(bh, bl);
}
template <int M> __device__ inline void swap_across(float& a, float& b)
{
    int ai = __float_as_int(a), bi = __float_as_int(b);
    swap_across<M>(ai, bi);
    a = __int_as_float(ai);
    b = __int_as_float(bi);
}
// v + v(lane ^ M), the same bits in both lanes of a pair (the two addends
// are the same, and addition commutes); across rows by one permlane swap of
// v with a copy of itself, with no select
template <int M, typename T> __device__ inline T xor_sum(T v)
{
    if constexpr (M >= 16) {
        T a = v, b = v;
        swap_across<M>(a, b);
        return a + b;
    } else {
        return v + lane_xor<M>(v);
    }
}
// the value of lane l (wave-uniform l) in every lane
__device__ inline int lane_read(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline double lane_read(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}
// broadcast of lane Q of each quad
template <int Q, typename T> __device__ inline T quad_bcast(T v)
{
    static_assert(Q >= 0 && Q < 4, "lane of a quad");
    constexpr int C = Q | (Q << 2) | (Q << 4) | (Q << 6);
    if constexpr (sizeof(T) == 8) {
        const double d = v;
        return __hiloint2double(dpp<C>(__double2hiint(d)), dpp<C>(__double2loint(d)));
    } else if constexpr (sizeof(T) == 4 && __is_same(T, float)) {
        return __int_as_float(dpp<C>(__float_as_int(v)));
    } else {
        return dpp<C>(v);
    }
}

// sum (product) over aligned groups of G = 2..16 lanes, butterfly in
// ascending order: every lane of a group ends with the same bits
template <int G, typename T> __device__ inline T dpp_sum(T v)
{
    static_assert(G == 2 || G == 4 || G == 8 || G == 16, "group of 2 to 16 lanes");
    v += lane_xor<1>(v);
    if constexpr (G >= 4) v += lane_xor<2>(v);
    if constexpr (G >= 8) v += lane_xor<4>(v);
    if constexpr (G >= 16) v += lane_xor<8>(v);
    return v;
}
template <int G, typename T> __device__ inline T dpp_prod(T v)
{
    static_assert(G == 2 || G == 4 || G == 8 || G == 16, "group of 2 to 16 lanes");
    v *= lane_xor<1>(v);
    if constexpr (G >= 4) v *= lane_xor<2>(v);
    if constexpr (G >= 8) v *= lane_xor<4>(v);
    if constexpr (G >= 16) v *= lane_xor<8>(v);
    return v;
}
// over the wave, butterfly in descending order (32, 16, ..., 1): the same
// bits as a __shfl_xor butterfly in that order, in every lane
template <typename T> __device__ inline T dpp_wave_sum(T v)
{
    v = xor_sum<32>(v);
    v = xor_sum<16>(v);
    v = xor_sum<8>(v);
    v = xor_sum<4>(v);
    v = xor_sum<2>(v);
    v = xor_sum<1>(v);
    return v;
}
__device__ inline double dpp_wave_max(double v)
{
    v = fmax(v, lane_xor<32>(v));
    v = fmax(v, lane_xor<16>(v));
    v = fmax(v, lane_xor<8>(v));
    v = fmax(v, lane_xor<4>(v));
    v = fmax(v, lane_xor<2>(v));
    v = fmax(v, lane_xor<1>(v));
    return v;
}
__device__ inline double dpp_wave_min(double v)
{
    v = fmin(v, lane_xor<32>(v));
    v = fmin(v, lane_xor<16>(v));
    v = fmin(v, lane_xor<8>(v));
    v = fmin(v, lane_xor<4>(v));
    v = fmin(v, lane_xor<2>(v));
    v = fmin(v, lane_xor<1>(v));
    return v;
}

}  // namespace kgev
