// Streaming TTM (Sec. 5.2 Eq. ttm) for a short contraction (n_m <= 64):
//   C(.., j, ..) = sum_k B(j, k) A(.., k, ..)
// With a short k the cost is writing C (m/n_m times the size of A), so the
// kernel is built around keeping stores flowing:
//   * each persistent workgroup stages the whole matrix B (m x n_m, zero-padded
//     to the MFMA k-step) in LDS once;
//   * it then walks column tiles of A (the columns nu are A's modes other than
//     m, decoded through up to four (extent, stride) pairs); each wave loads
//     its A fragments straight from global memory into MFMA operand registers,
//     issuing the loads of its next tile before the MFMAs and stores of the
//     current one;
//   * the MFMA operand order is chosen so that the lanes of a store run along
//     C's unit-stride dimension.
// MFMAs: v_mfma_f64_16x16x4 (FP64), v_mfma_f32_16x16x4 (FP32) and
// v_mfma_f32_16x16x32_{bf16,f16} (16-bit inputs, FP32 accumulation).
#include <algorithm>

#include "device.hpp"

namespace tlib {

typedef double d4s_t __attribute__((ext_vector_type(4)));
typedef float f4s_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8s_t __attribute__((ext_vector_type(8)));
typedef _Float16 h8s_t __attribute__((ext_vector_type(8)));
typedef uint32_t u4s_t __attribute__((ext_vector_type(4)));

template <typename TI> struct SMfma {
    using acc_t = f4s_t;
    using frag_t = u4s_t;  // 8 x 16-bit
    static constexpr int KSTEP = 32;
};
template <> struct SMfma<double> {
    using acc_t = d4s_t;
    using frag_t = double;
    static constexpr int KSTEP = 4;
};
template <> struct SMfma<float> {
    using acc_t = f4s_t;
    using frag_t = float;
    static constexpr int KSTEP = 4;
};

template <typename TI>
__device__ __forceinline__ typename SMfma<TI>::acc_t smfma(typename SMfma<TI>::frag_t a, typename SMfma<TI>::frag_t b,
                                                          typename SMfma<TI>::acc_t c) {
    if constexpr (std::is_same<TI, double>::value) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else if constexpr (std::is_same<TI, float>::value) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    else if constexpr (std::is_same<TI, bf16_t>::value)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8s_t, a), __builtin_bit_cast(bf8s_t, b),
                                                       c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8s_t, a), __builtin_bit_cast(h8s_t, b), c,
                                                      0, 0, 0);
}

__device__ __forceinline__ uint32_t raw16(const bf16_t* p) { return *reinterpret_cast<const uint16_t*>(p); }
__device__ __forceinline__ uint32_t raw16(const f16_t* p) { return *reinterpret_cast<const uint16_t*>(p); }

// Per wave FM row blocks and FN column blocks of 16; WGM of the four waves
// split the rows (WGM * FM * 16 >= M), the others split the columns; KS
// k-steps.  TRANS: MFMA operands swapped so the lanes of the result run
// along M.
template <typename TI, int FM, int FN, int KS, bool TRANS, int WGM>
__global__ __launch_bounds__(256) void ttm_stream_kernel(TtmParams P) {
    using TA = typename AccOf<TI>::type;
    using acc_t = typename SMfma<TI>::acc_t;
    using frag_t = typename SMfma<TI>::frag_t;
    constexpr bool WIDE = sizeof(TI) == 2;
    constexpr int KSTEP = SMfma<TI>::KSTEP;
    constexpr int KP = KS * KSTEP;             // padded contraction length
    constexpr int M16 = WGM * FM * 16;
    constexpr int PB = WIDE ? (KP + 8) : (M16 + (sizeof(TI) == 8 ? 4 : 16));
    constexpr int RQ = std::is_same<TI, double>::value ? 1 : 4;  // result row of (kq, r): RQ*kq + RR*r
    constexpr int RR = std::is_same<TI, double>::value ? 4 : 1;
    constexpr int WGN = 4 / WGM;
    constexpr int COLS = WGN * FN * 16;        // columns per workgroup tile

    extern __shared__ __align__(16) unsigned char smem[];
    using RT = typename std::conditional<WIDE, uint16_t, TI>::type;
    RT* Bs = reinterpret_cast<RT*>(smem);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rl = lane & 15, kq = lane >> 4;
    const int wm = wave % WGM, wn = wave / WGM;
    const int row0 = wm * FM * 16;
    const TI* X = (const TI*)P.X;
    const TI* Y = (const TI*)P.Y;
    TA* C = (TA*)P.C;

    // stage B (M x K) zero-padded to M16 x KP
    for (int e = tid; e < M16 * KP; e += 256) {
        int m, k;
        if constexpr (WIDE) { m = e / KP; k = e % KP; }
        else { k = e / M16; m = e % M16; }
        RT v = RT(0);
        if (m < P.M && k < P.K) {
            const TI* src = X + int64_t(m) * P.sXm + int64_t(k) * P.sXk;
            if constexpr (WIDE) v = uint16_t(raw16(src));
            else v = *src;
        }
        if constexpr (WIDE) Bs[m * PB + k] = v;
        else Bs[k * PB + m] = v;
    }
    __syncthreads();

    const int T = (P.N + COLS - 1) / COLS;
    frag_t ycur[FN][KS], ynxt[FN][KS];

    // A fragments of tile t for this wave: block j holds columns
    // t*COLS + (wave*FN + j)*16 + rl; lane (rl, kq) supplies k = s*KSTEP + kq
    // (FP32/FP64) or k = s*32 + 8*kq + e (16-bit).
    auto load_y = [&](int t, frag_t (&y)[FN][KS]) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = t * COLS + (wn * FN + j) * 16 + rl;
            const bool cv = col < P.N;
            const int64_t yo = cv ? grp_off0(uint32_t(col), P.gn) : 0;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                if constexpr (WIDE) {
                    uint32_t w[4];
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        const int k0 = s * 32 + 8 * kq + 2 * h;
                        const uint32_t lo = (cv && k0 < P.K) ? raw16(Y + yo + int64_t(k0) * P.sYk) : 0u;
                        const uint32_t hi = (cv && k0 + 1 < P.K) ? raw16(Y + yo + int64_t(k0 + 1) * P.sYk) : 0u;
                        w[h] = lo | (hi << 16);
                    }
                    y[j][s] = u4s_t{w[0], w[1], w[2], w[3]};
                } else {
                    const int k = s * KSTEP + kq;
                    y[j][s] = (cv && k < P.K) ? Y[yo + int64_t(k) * P.sYk] : TI(0);
                }
            }
        }
    };

    int t = blockIdx.x;
    if (t < T) load_y(t, ycur);
    for (; t < T; t += gridDim.x) {
        const int tn = t + gridDim.x;
        if (tn < T) load_y(tn, ynxt);

        acc_t acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                frag_t b;
                if constexpr (WIDE) b = *reinterpret_cast<const u4s_t*>(&Bs[(row0 + i * 16 + rl) * PB + s * 32 + 8 * kq]);
                else b = Bs[(s * KSTEP + kq) * PB + row0 + i * 16 + rl];
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    if constexpr (TRANS) acc[i][j] = smfma<TI>(ycur[j][s], b, acc[i][j]);
                    else acc[i][j] = smfma<TI>(b, ycur[j][s], acc[i][j]);
                }
            }
        }

        // stores: block (i, j) covers rows (M) 16i.. and columns t*COLS + (wave*FN+j)*16 ..
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int cbase = t * COLS + (wn * FN + j) * 16;
            if constexpr (!TRANS) {
                // lane column = nu (rl), registers = rows of M
                // the row part of each address is uniform across the wave
                // except for kq: one lane base plus scalar offsets
                const int col = cbase + rl;
                if (col < P.N) {
                    TA* cp = C + grp_off1(uint32_t(col), P.gn) + int64_t(row0 + RQ * kq) * P.sCm;
                    const int rmax = P.M - row0 - RQ * kq;
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int dr = i * 16 + RR * r;
                            if (dr < rmax) cp[int64_t(dr) * P.sCm] = acc[i][j][r];
                        }
                }
            } else {
                // lane column = row of M (rl), registers = columns nu
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int col = cbase + RQ * kq + RR * r;
                    if (col < P.N) {
                        TA* cp = C + grp_off1(uint32_t(col), P.gn) + int64_t(row0 + rl) * P.sCm;
                        const int rmax = P.M - row0 - rl;
#pragma unroll
                        for (int i = 0; i < FM; ++i)
                            if (i * 16 < rmax) cp[int64_t(i * 16) * P.sCm] = acc[i][j][r];
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int s = 0; s < KS; ++s) ycur[j][s] = ynxt[j][s];
    }
}

// ------------------------------------------------------------------ launch

template <typename TI, int FM, int FN, int KS, bool TR, int WGM>
static int stream_launch(const TtmParams& p, int grid, hipStream_t s) {
    constexpr bool WIDE = sizeof(TI) == 2;
    constexpr int KP = KS * SMfma<TI>::KSTEP;
    constexpr int M16 = WGM * FM * 16;
    constexpr int PB = WIDE ? (KP + 8) : (M16 + (sizeof(TI) == 8 ? 4 : 16));
    const size_t lds = size_t(WIDE ? M16 * PB : KP * PB) * (WIDE ? 2 : sizeof(TI));
    hipLaunchKernelGGL((ttm_stream_kernel<TI, FM, FN, KS, TR, WGM>), dim3(grid), dim3(256), lds, s, p);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

// Dispatch over (FM, KS, TRANS); FN follows from the accumulator budget.
// KS (k-steps) is rounded up to one of the instantiated depths by the planner.
// fm: total row blocks (1, 4 or 16), all owned by each wave; FN column blocks
// per wave keep the accumulators at 64 values per lane.
template <typename TI, int FMT>
static int stream_fm(const TtmParams& p, int ks, bool tr, int grid, hipStream_t s) {
    // measured on MI355X: one wave owning all rows of a 16-column strip beats
    // splitting the rows over the waves, despite the lower occupancy
    constexpr int WGM = 1;
    constexpr int FM = FMT;
    constexpr int FN = FMT >= 16 ? 1 : FMT >= 4 ? 2 : 4;
#define TLIB_KS_CASE(K)                                                                                      \
    case K:                                                                                                  \
        return tr ? stream_launch<TI, FM, FN, K, true, WGM>(p, grid, s)                                      \
                  : stream_launch<TI, FM, FN, K, false, WGM>(p, grid, s);
    if constexpr (sizeof(TI) == 2) {
        switch (ks) {
            TLIB_KS_CASE(1)
            TLIB_KS_CASE(2)
        }
    } else {
        switch (ks) {
            TLIB_KS_CASE(1)
            TLIB_KS_CASE(2)
            TLIB_KS_CASE(3)
            TLIB_KS_CASE(4)
            TLIB_KS_CASE(5)
            TLIB_KS_CASE(6)
            TLIB_KS_CASE(8)
            TLIB_KS_CASE(10)
            TLIB_KS_CASE(12)
            TLIB_KS_CASE(16)
        }
    }
#undef TLIB_KS_CASE
    return TLIB_EINVAL;
}

int ttm_stream_ks(int dtype, int k) {
    if (dtype == TLIB_BF16 || dtype == TLIB_F16) return k <= 32 ? 1 : k <= 64 ? 2 : 0;
    const int ks = (k + 3) / 4;
    static const int depths[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};
    for (int d : depths)
        if (ks <= d) return d;
    return 0;
}

template <typename TI>
static int stream_dispatch(const TtmParams& p, int fm, int ks, bool tr, int grid, hipStream_t s) {
    switch (fm) {
        case 1: return stream_fm<TI, 1>(p, ks, tr, grid, s);
        case 4: return stream_fm<TI, 4>(p, ks, tr, grid, s);
        default: return stream_fm<TI, 16>(p, ks, tr, grid, s);
    }
}

int launch_ttm_stream(int dtype, const TtmParams& p, int fm, int ks, bool trans, int grid, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return stream_dispatch<double>(p, fm, ks, trans, grid, s);
        case TLIB_F32: return stream_dispatch<float>(p, fm, ks, trans, grid, s);
        case TLIB_BF16: return stream_dispatch<bf16_t>(p, fm, ks, trans, grid, s);
        case TLIB_F16: return stream_dispatch<f16_t>(p, fm, ks, trans, grid, s);
    }
    return TLIB_EDTYPE;
}

}  // namespace tlib
