// Device-side helpers shared by the HIP kernels: element types, conversions,
// run-time-constant division and index-group decoding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "internal.hpp"

namespace tlib {

// 16-bit storage types.  bf16 is kept as raw bits; f16 uses the native type.
struct bf16_t {
    uint16_t x;
};
using f16_t = _Float16;

template <typename T> struct AccOf { using type = float; };
template <> struct AccOf<double> { using type = double; };

__device__ __forceinline__ double to_acc(double v) { return v; }
__device__ __forceinline__ float to_acc(float v) { return v; }
__device__ __forceinline__ float to_acc(bf16_t v) { return __uint_as_float(uint32_t(v.x) << 16); }
__device__ __forceinline__ float to_acc(f16_t v) { return float(v); }

__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ double to_f64(float v) { return double(v); }
__device__ __forceinline__ double to_f64(bf16_t v) { return double(__uint_as_float(uint32_t(v.x) << 16)); }
__device__ __forceinline__ double to_f64(f16_t v) { return double(float(v)); }

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv& f) {
    uint32_t hi = __umulhi(x, f.m);
    return uint32_t((uint64_t(hi) + x) >> f.s);
}

// Offsets of index `idx` (< g.total) in a Grp for its two operands.
__device__ __forceinline__ void grp_decode(uint32_t idx, const Grp& g, int64_t& o0, int64_t& o1) {
    o0 = 0;
    o1 = 0;
    if (g.nd == 1) {
        o0 = int64_t(idx) * g.s0[0];
        o1 = int64_t(idx) * g.s1[0];
        return;
    }
#pragma unroll
    for (int d = 0; d < GMAXD; ++d) {
        if (d >= g.nd) break;
        uint32_t q = (d == g.nd - 1) ? 0u : fdiv(idx, g.fd[d]);
        uint32_t r = idx - q * uint32_t(g.n[d]);
        o0 += int64_t(r) * g.s0[d];
        o1 += int64_t(r) * g.s1[d];
        idx = q;
    }
}

// Offset of `idx` in a Grp for operand 0 only.
__device__ __forceinline__ int64_t grp_off0(uint32_t idx, const Grp& g) {
    if (g.nd == 1) return int64_t(idx) * g.s0[0];
    int64_t o = 0;
#pragma unroll
    for (int d = 0; d < GMAXD; ++d) {
        if (d >= g.nd) break;
        uint32_t q = (d == g.nd - 1) ? 0u : fdiv(idx, g.fd[d]);
        o += int64_t(idx - q * uint32_t(g.n[d])) * g.s0[d];
        idx = q;
    }
    return o;
}

__device__ __forceinline__ int64_t grp_off1(uint32_t idx, const Grp& g) {
    if (g.nd == 1) return int64_t(idx) * g.s1[0];
    int64_t o = 0;
#pragma unroll
    for (int d = 0; d < GMAXD; ++d) {
        if (d >= g.nd) break;
        uint32_t q = (d == g.nd - 1) ? 0u : fdiv(idx, g.fd[d]);
        o += int64_t(idx - q * uint32_t(g.n[d])) * g.s1[d];
        idx = q;
    }
    return o;
}

// Generic decode (64-bit division) of `lin` over GDims for up to three operands.
__device__ __forceinline__ void gd_decode(int64_t lin, const GDims& g, int nops, int64_t* off) {
    for (int o = 0; o < nops; ++o) off[o] = 0;
    for (int d = 0; d < g.nd; ++d) {
        int64_t q = (d == g.nd - 1) ? 0 : lin / g.n[d];
        int64_t r = lin - q * g.n[d];
        for (int o = 0; o < nops; ++o) off[o] += r * g.s[o][d];
        lin = q;
    }
}

template <typename T> __device__ __forceinline__ T warp_sum(T v, int width) {
    for (int o = width / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
    return v;
}

}  // namespace tlib
