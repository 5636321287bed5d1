// Multi-mode tensor-times-vector in one pass over A (Sec. 5.2,
// tensor_times_vectors, the product the higher-order power method needs):
//   c(i_r) = sum over all i_k, k != r, of A(i_1..i_p) * prod_{k != r} u_k(i_k).
//
// A is taken in storage order (modes sorted by stride).  Its innermost modes
// form the "positions" of a tile, at most TV_SLOTS of them; the remaining
// modes are the tile's "rows".  Every thread owns fixed positions, so their
// offset in A, their share of the weight (the vectors of the position modes)
// and, when r is a position mode, their target i_r are decoded once per
// block.  The rows are streamed: a row's offset and weight come from two small
// tables (outer lo modes and hi modes, filled by tv_prep_kernel), and every
// element is added to its slot's FP64 accumulator as A * w_row.
//
//   K1 (r among the position modes, few lo positions per value of i_r): a
//       block owns one chunk of positions and a range of rows; slots with the
//       same i_r are summed in LDS at the end.
//   K2 (r among the row modes): a block owns one value of i_r, one chunk of
//       positions and a range of the modes outside r; its slots all feed c(i_r).
//
// Each block writes FP64 partial sums; tv_finish_kernel adds them in a fixed
// order and rounds once to c's type, so the result does not depend on timing.
#include "device.hpp"

namespace tlib {

// Weight and offset of one index of a mode group (storage order, fastest
// first): w = prod u_d[digit_d] over the modes that carry a vector, off = sum
// digit_d * s_d.  64-bit division: used once per table entry.
template <typename TI>
__device__ void tv_decode64(int64_t idx, const TvModes& g, double& w, int64_t& off) {
    w = 1.0;
    off = 0;
    for (int d = 0; d < g.nd; ++d) {
        const int64_t q = idx / g.n[d];
        const int64_t digit = idx - q * g.n[d];
        idx = q;
        off += digit * g.s[d];
        if (g.u[d]) w *= to_f64(reinterpret_cast<const TI*>(g.u[d])[digit * g.us[d]]);
    }
}

// The same for a position index (< 2^31): run-time-constant division.
template <typename TI>
__device__ void tv_decode32(uint32_t idx, const TvModes& g, double& w, int64_t& off) {
    w = 1.0;
    off = 0;
    for (int d = 0; d < g.nd; ++d) {
        const uint32_t q = fdiv(idx, g.fd[d]);
        const uint32_t digit = idx - q * uint32_t(g.n[d]);
        idx = q;
        off += int64_t(digit) * g.s[d];
        if (g.u[d]) w *= to_f64(reinterpret_cast<const TI*>(g.u[d])[int64_t(digit) * g.us[d]]);
    }
}

// Source of the loads of rows past the end of a block's range.
__device__ __align__(16) double g_tv_zero[2] = {0.0, 0.0};

// Row tables.  General strides: entries [0, n_out) for the lo modes outside
// the positions and [n_out, n_out + n_hi) for the hi modes, weight and offset
// each.  Dense rows (lin): the weight of every row t = o + n_out * h, the
// offsets being arithmetic.
template <typename TI>
__global__ __launch_bounds__(256) void tv_prep_kernel(TvParams P, double* w, int64_t* off) {
    const int64_t total = P.lin ? P.n_out * P.n_hi : P.n_out + P.n_hi;
    for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < total; e += int64_t(gridDim.x) * 256) {
        double we;
        int64_t oe;
        if (P.lin) {
            // row counts stay below 2^26 here: run-time-constant division
            const uint32_t h = fdiv(uint32_t(e), P.fd_out);
            double wh;
            int64_t oh;
            tv_decode32<TI>(uint32_t(e) - h * uint32_t(P.n_out), P.out, we, oe);
            tv_decode32<TI>(h, P.hi, wh, oh);
            w[e] = we * wh;
        } else {
            if (e < P.n_out) tv_decode64<TI>(e, P.out, we, oe);
            else tv_decode64<TI>(e - P.n_out, P.hi, we, oe);
            w[e] = we;
            off[e] = oe;
        }
    }
}

template <typename TI> struct TvVec;
template <> struct TvVec<double> { typedef double v_t __attribute__((ext_vector_type(2))); };
template <> struct TvVec<float> { typedef float v_t __attribute__((ext_vector_type(4))); };
template <> struct TvVec<bf16_t> { typedef uint32_t v_t __attribute__((ext_vector_type(4))); };
template <> struct TvVec<f16_t> { typedef uint32_t v_t __attribute__((ext_vector_type(4))); };

// Element e of a 16-byte vector holding V elements of TI, as FP64.
template <typename TI>
__device__ __forceinline__ double tv_elem(const typename TvVec<TI>::v_t& v, int e) {
    if constexpr (std::is_same<TI, double>::value || std::is_same<TI, float>::value) return double(v[e]);
    else {
        const uint32_t wd = v[e >> 1];
        const uint16_t h = uint16_t((e & 1) ? (wd >> 16) : (wd & 0xffffu));
        if constexpr (std::is_same<TI, bf16_t>::value) return to_f64(bf16_t{h});
        else return to_f64(__builtin_bit_cast(f16_t, h));
    }
}

// V: elements per load (16 bytes / element size on the vector path, else 1).
// Slots of a thread: V consecutive positions per group, TV_SLOTS / (256 V)
// groups, group g at slot q = V * (tid + 256 g).
template <typename TI, int V, bool K2, bool LIN>
__global__ __launch_bounds__(256) void tv_main_kernel(TvParams P, const double* w, const int64_t* off) {
    constexpr int NG = TV_SLOTS / (256 * V);
    constexpr int NS = NG * V;
    static_assert(NG >= 1, "slot layout");
    using vec_t = typename TvVec<TI>::v_t;
    __shared__ double red[TV_SLOTS];
    __shared__ double wsum[4];

    const int tid = threadIdx.x;
    // block -> (i, position chunk fc, row range hc); rows t = o + n_out * h
    int64_t b = blockIdx.x;
    const int hc = int(b % P.HC);
    b /= P.HC;
    const int fc = int(b % P.nfc);
    const int64_t ib = K2 ? b / P.nfc : 0;  // K2: the block's i_r
    const int64_t t_begin = int64_t(hc) * P.hc_len;
    const int64_t cnt = min(P.hc_len, P.n_out * P.n_hi - t_begin);  // rows of this block
    const int64_t h_b = t_begin / P.n_out;
    const uint32_t o_b = uint32_t(t_begin - h_b * P.n_out);
    const int64_t f0 = int64_t(fc) * P.W;
    const int wlen = int(min(int64_t(P.W), P.npos - f0));  // positions of this chunk

    const TI* A = reinterpret_cast<const TI*>(P.A) + (K2 ? ib * P.s_r : 0);
    const double* w_out = w;
    const double* w_hi = w + P.n_out;
    const int64_t* off_out = off;
    const int64_t* off_hi = off + P.n_out;

    // fixed per-slot data: row within the tile, position offset and weight
    int rsub[NG];
    int64_t poff[NS];
    double pw[NS];
    double acc[NS];
    uint32_t live_mask = 0;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int q = V * (tid + 256 * g);
        rsub[g] = q / P.W;
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int fl = q + e - rsub[g] * P.W;
            const bool live = rsub[g] < P.G && fl < wlen && cnt > 0;
            double wd;
            int64_t o;
            tv_decode32<TI>(uint32_t(f0 + (live ? fl : 0)), P.pos, wd, o);
            poff[g * V + e] = o;
            pw[g * V + e] = wd;
            acc[g * V + e] = 0.0;
            live_mask |= live ? (1u << (g * V + e)) : 0u;
        }
    }

    const TI* zsrc = reinterpret_cast<const TI*>(g_tv_zero);
    auto row = [&](int64_t t0) {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const int64_t lt = t0 + rsub[g];
            const bool rok = lt < cnt;
            const uint32_t x = o_b + (rok ? uint32_t(lt) : 0u);
            const uint32_t hh = fdiv(x, P.fd_out);
            const uint32_t o = x - hh * uint32_t(P.n_out);
            // with dense row modes the offset is arithmetic, so the load of A
            // does not wait for a table entry
            const int64_t ro = LIN ? int64_t(o) * P.s_o + (h_b + hh) * P.s_h : off_out[o] + off_hi[h_b + hh];
            // rows past the range read zeros (their weight may meet Inf data)
            const TI* src = rok ? A + (ro + poff[g * V]) : zsrc;
            const double wr = LIN ? w[t_begin + (rok ? lt : 0)] : w_out[o] * w_hi[h_b + hh];
            if constexpr (V > 1) {
                // positions of the group are consecutive in A and 16-byte aligned
                const vec_t v = *reinterpret_cast<const vec_t*>(src);
#pragma unroll
                for (int e = 0; e < V; ++e) acc[g * V + e] += tv_elem<TI>(v, e) * wr;
            } else {
                acc[g] += to_f64(*src) * wr;
            }
        }
    };
    // four tile rows per iteration: more loads in flight
    int64_t t0 = 0;
    for (; t0 + 3 * int64_t(P.G) < cnt; t0 += 4 * int64_t(P.G)) {
        row(t0);
        row(t0 + P.G);
        row(t0 + 2 * int64_t(P.G));
        row(t0 + 3 * int64_t(P.G));
    }
    for (; t0 < cnt; t0 += P.G) row(t0);

    // slot value = accumulated rows times the slot's position weight; slots
    // outside the chunk contribute exactly zero
    double val[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) val[k] = ((live_mask >> k) & 1u) ? acc[k] * pw[k] : 0.0;

    const int lane = tid & 63, wave = tid >> 6;
    if constexpr (K2) {
        // every slot feeds c(ib): block sum in a fixed order
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) s += val[k];
        s = warp_sum(s, 64);
        if (lane == 0) wsum[wave] = s;
        __syncthreads();
        if (tid == 0)
            P.part[(ib * P.HC + hc) * P.nfc + fc] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    } else {
        // slot values to LDS (tile layout q = row * W + position), then every
        // local i_r summed by one wave over its rows and positions
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int e = 0; e < V; ++e) red[V * (tid + 256 * g) + e] = val[g * V + e];
        __syncthreads();
        const int64_t i_first = f0 / P.n_lo;
        const int64_t i_last = (f0 + wlen - 1) / P.n_lo;
        for (int64_t i = i_first + wave; i <= i_last; i += 4) {
            const int64_t p0 = max(i * P.n_lo, f0) - f0, p1 = min((i + 1) * P.n_lo, f0 + wlen) - f0;
            const int len = int(p1 - p0);
            const int cnt = len * P.G;
            double s = 0.0;
            for (int k = lane; k < cnt; k += 64) {
                const int rr = k / len;
                s += red[rr * P.W + int(p0) + (k - rr * len)];
            }
            s = warp_sum(s, 64);
            if (lane == 0) P.part[(int64_t(hc) * P.nfc + fc) * P.nloc + (i - i_first)] = s;
        }
    }
}

// c(i) = sum of the partials of i in a fixed order, rounded once: one wave
// per i, lane l adds partials l, l+64, ... and the wave sums the lanes with a
// fixed butterfly.
template <typename TA>
__global__ __launch_bounds__(64) void tv_finish_kernel(TvParams P, TA* c, int64_t cs, bool k2) {
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x;
    double s = 0.0;
    if (k2) {
        const double* p = P.part + i * P.HC * P.nfc;
        const int64_t cnt = int64_t(P.HC) * P.nfc;
        for (int64_t k = lane; k < cnt; k += 64) s += p[k];
    } else {
        const int64_t fa = (i * P.n_lo) / P.W, fb = ((i + 1) * P.n_lo - 1) / P.W;
        const int64_t nf = fb - fa + 1;
        const int64_t cnt = int64_t(P.HC) * nf;
        for (int64_t k = lane; k < cnt; k += 64) {
            const int64_t hc = k / nf, fc = fa + (k - hc * nf);
            s += P.part[(hc * P.nfc + fc) * P.nloc + (i - (fc * P.W) / P.n_lo)];
        }
    }
    s = warp_sum(s, 64);
    if (lane == 0) c[i * cs] = TA(s);
}

// ------------------------------------------------------------------ launch

template <typename TI>
static int tv_run(const TvParams& P, void* c, int64_t cs, bool vec, hipStream_t s) {
    using TA = typename AccOf<TI>::type;
    constexpr int VV = 16 / int(sizeof(TI));
    const int64_t ntab = P.lin ? P.n_out * P.n_hi : P.n_out + P.n_hi;
    double* w = P.tabw;
    int64_t* off = P.tabo;
    {
        const unsigned g = unsigned(std::min<int64_t>((ntab + 255) / 256, 4096));
        hipLaunchKernelGGL((tv_prep_kernel<TI>), dim3(g), dim3(256), 0, s, P, w, off);
    }
    const int64_t items = (P.k2 ? P.n_r : 1) * int64_t(P.nfc) * P.HC;
    const dim3 grid{static_cast<unsigned>(items)};
#define TLIB_TV_LAUNCH(VV_, K2_, LIN_) \
    hipLaunchKernelGGL((tv_main_kernel<TI, VV_, K2_, LIN_>), grid, dim3(256), 0, s, P, w, off)
    const bool lin = P.lin != 0;
    if (P.k2) {
        if (vec) { if (lin) TLIB_TV_LAUNCH(VV, true, true); else TLIB_TV_LAUNCH(VV, true, false); }
        else { if (lin) TLIB_TV_LAUNCH(1, true, true); else TLIB_TV_LAUNCH(1, true, false); }
    } else {
        if (vec) { if (lin) TLIB_TV_LAUNCH(VV, false, true); else TLIB_TV_LAUNCH(VV, false, false); }
        else { if (lin) TLIB_TV_LAUNCH(1, false, true); else TLIB_TV_LAUNCH(1, false, false); }
    }
#undef TLIB_TV_LAUNCH
    hipLaunchKernelGGL((tv_finish_kernel<TA>), dim3(unsigned(P.n_r)), dim3(64), 0, s, P, reinterpret_cast<TA*>(c),
                       cs, P.k2 != 0);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

int launch_tv(int dtype, const TvParams& P, void* c, int64_t cs, bool vec, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return tv_run<double>(P, c, cs, vec, s);
        case TLIB_F32: return tv_run<float>(P, c, cs, vec, s);
        case TLIB_BF16: return tv_run<bf16_t>(P, c, cs, vec, s);
        case TLIB_F16: return tv_run<f16_t>(P, c, cs, vec, s);
    }
    return TLIB_EDTYPE;
}

}  // namespace tlib
