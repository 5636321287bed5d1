// GEMM with every row in one tile, for a small M (<= 128):
//   C[m, n] = sum_k X[m, k] Y[k, n]
// with the same index groups as gemm_kernel (Sec. 5.2 Eq. ttt for TTT; Eq. ttm
// for a TTM with few matrix rows).  Such products (a TTT whose free B modes
// hold at most 128 indices, a TTM with m <= 128) are bound by streaming the
// large operand Y once; the small operand X is read by every column tile.
//
// A workgroup of four waves owns all M rows (padded to 16 FM) and 64 FN
// columns: wave w computes the 16 FN columns starting at 16 FN w.  K is walked
// in chunks of KC:
//   * X's chunk (M x KC) is staged in LDS by all threads with 16-byte (FP32:
//     8-byte) loads along k, stored row-major with k contiguous at a pitch
//     that keeps the MFMA fragment reads free of bank conflicts, double-
//     buffered so the next chunk's loads overlap this chunk's MFMAs;
//   * Y's fragments go from global memory straight into MFMA registers, one
//     chunk ahead: 16-bit operands as 16-byte groups of eight consecutive k
//     (Y's K dim has unit stride), FP32/FP64 one element per lane and k-step;
//   * the K offsets of a chunk are decoded once into LDS.
// Split-K writes FP32/FP64 partials summed by gemm_ksum_kernel, in the same
// order as the tiled GEMM's.
#include <algorithm>

#include "device.hpp"

namespace tlib {

namespace {

typedef double rd4_t __attribute__((ext_vector_type(4)));
typedef float rf4_t __attribute__((ext_vector_type(4)));
typedef __bf16 rbf8_t __attribute__((ext_vector_type(8)));
typedef _Float16 rh8_t __attribute__((ext_vector_type(8)));
typedef uint32_t ru4_t __attribute__((ext_vector_type(4)));
typedef uint32_t ru2_t __attribute__((ext_vector_type(2)));

__device__ __align__(16) double g_rows_zero[2] = {0.0, 0.0};

template <typename TI> struct RowsCfg;
template <> struct RowsCfg<double> {
    static constexpr int KSTEP = 4, KC = 16, G = 2;   // G: k per X load (16 bytes)
    using acc_t = rd4_t;
    using xg_t = ru4_t;
};
template <> struct RowsCfg<float> {
    static constexpr int KSTEP = 4, KC = 32, G = 2;   // 8-byte X loads
    using acc_t = rf4_t;
    using xg_t = ru2_t;
};
template <> struct RowsCfg<bf16_t> {
    static constexpr int KSTEP = 32, KC = 128, G = 8;
    using acc_t = rf4_t;
    using xg_t = ru4_t;
};
template <> struct RowsCfg<f16_t> {
    static constexpr int KSTEP = 32, KC = 128, G = 8;
    using acc_t = rf4_t;
    using xg_t = ru4_t;
};

__device__ __forceinline__ rd4_t rmfma(double a, double b, rd4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ rf4_t rmfma(float a, float b, rf4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename TI> __device__ __forceinline__ rf4_t rmfma16(ru4_t a, ru4_t b, rf4_t c) {
    if constexpr (std::is_same<TI, bf16_t>::value)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(rbf8_t, a), __builtin_bit_cast(rbf8_t, b),
                                                       c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(rh8_t, a), __builtin_bit_cast(rh8_t, b), c,
                                                      0, 0, 0);
}

}  // namespace

template <typename TI, int FM, int FN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_rows_kernel(GemmParams P) {
    using Cfg = RowsCfg<TI>;
    using TA = typename AccOf<TI>::type;
    using acc_t = typename Cfg::acc_t;
    using xg_t = typename Cfg::xg_t;
    constexpr bool WIDE = sizeof(TI) == 2;
    constexpr int KSTEP = Cfg::KSTEP, KC = Cfg::KC, G = Cfg::G;
    constexpr int NKS = KC / KSTEP;                   // k-steps per chunk
    constexpr int MR = 16 * FM;                       // rows (padded)
    constexpr int BN = 64 * FN;                       // columns per workgroup
    // row pitch: KC elements plus 16 bytes (144 bytes = 36 dwords for FP32 and
    // FP64 chunks, 272 = 68 for 16-bit ones), so the 16 rows of a fragment
    // start in 16 different groups of four banks
    constexpr int PX = KC + 16 / int(sizeof(TI));
    static_assert((PX * int(sizeof(TI))) % 16 == 0, "16-byte rows");
    constexpr int NG = MR * KC / G;                   // X groups per chunk
    constexpr int EG = (NG + 255) / 256;              // groups per thread
    using RT = typename std::conditional<WIDE, uint16_t, TI>::type;

    // X's two chunk buffers (dynamic: 70 KB for 128 rows of 16-bit chunks)
    extern __shared__ __align__(16) unsigned char rows_smem[];
    RT(*Xs)[MR * PX] = reinterpret_cast<RT(*)[MR * PX]>(rows_smem);
    __shared__ int64_t kx[2][KC], ky[2][KC];
    __shared__ int64_t xrow[MR], crow[MR];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rl = lane & 15, kq = lane >> 4;
    const int tn = blockIdx.x;
    const int64_t n0 = int64_t(tn) * BN + wave * 16 * FN;
    const int kz = blockIdx.y;
    const int kbeg = kz * P.kchunk;
    const int kend = min(P.K, kbeg + P.kchunk);
    const TI* X = (const TI*)P.X;
    const TI* Y = (const TI*)P.Y;
    const TI* zsrc = reinterpret_cast<const TI*>(g_rows_zero);

    for (int i = tid; i < MR; i += 256) {
        int64_t a = -1, c = -1;
        if (i < P.M) grp_decode(uint32_t(i), P.gm, a, c);
        xrow[i] = a;
        crow[i] = c;
    }
    // this lane's columns
    int64_t ycol[FN], ccol[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int64_t n = n0 + j * 16 + rl;
        int64_t a = -1, c = -1;
        if (n < P.N) grp_decode(uint32_t(n), P.gn, a, c);
        ycol[j] = a;
        ccol[j] = c;
    }
    auto ktable = [&](int k0, int b) {
        if (tid < KC) {
            int64_t a = -1, c = -1;
            if (k0 + tid < kend) grp_decode(uint32_t(k0 + tid), P.gk, a, c);
            kx[b][tid] = a;
            ky[b][tid] = c;
        }
    };
    // X chunk: group e = tid + 256 q is row e / (KC / G), k group e % (KC / G)
    xg_t xr[EG];
    auto fetch_x = [&](int b) {
#pragma unroll
        for (int q = 0; q < EG; ++q) {
            const int e = tid + 256 * q;
            const int row = min(e / (KC / G), MR - 1), g = e % (KC / G);
            const int64_t a = e < NG ? xrow[row] : -1, o = kx[b][g * G];
            xr[q] = *reinterpret_cast<const xg_t*>((a >= 0 && o >= 0) ? X + (a + o) : zsrc);
        }
    };
    auto store_x = [&](int b) {
#pragma unroll
        for (int q = 0; q < EG; ++q) {
            const int e = tid + 256 * q;
            if (e < NG) *reinterpret_cast<xg_t*>(&Xs[b][(e / (KC / G)) * PX + (e % (KC / G)) * G]) = xr[q];
        }
    };
    // Y fragments of a chunk: 16-bit: one 16-byte group (k = 8 kq .. 8 kq + 7 of
    // the k-step) per column block; FP32/FP64: element k = kq of the k-step
    using yf_t = typename std::conditional<WIDE, ru4_t, TI>::type;
    yf_t ya[NKS][FN], yb[NKS][FN];
    auto fetch_y = [&](int b, yf_t (&y)[NKS][FN]) {
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            const int kk = s * KSTEP + (WIDE ? 8 * kq : kq);
            const int64_t o = ky[b][kk];
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const bool ok = ycol[j] >= 0 && o >= 0;
                if constexpr (WIDE) y[s][j] = *reinterpret_cast<const ru4_t*>(ok ? Y + (ycol[j] + o) : zsrc);
                else y[s][j] = *(ok ? Y + (ycol[j] + o) : zsrc);
            }
        }
    };

    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{};

    int b = 0;
    if (kbeg < kend) {
        ktable(kbeg, 0);
        __syncthreads();
        fetch_x(0);
        fetch_y(0, ya);
        store_x(0);
    }
    __syncthreads();
    for (int k0 = kbeg; k0 < kend; k0 += KC) {
        const bool nxt = k0 + KC < kend;
        if (nxt) ktable(k0 + KC, b ^ 1);
        __syncthreads();
        if (nxt) {
            fetch_x(b ^ 1);
            fetch_y(b ^ 1, yb);
        }
#pragma unroll
        for (int s = 0; s < NKS; ++s) {
            if constexpr (WIDE) {
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const ru4_t a = *reinterpret_cast<const ru4_t*>(&Xs[b][(i * 16 + rl) * PX + s * KSTEP + 8 * kq]);
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = rmfma16<TI>(a, ya[s][j], acc[i][j]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const TI a = Xs[b][(i * 16 + rl) * PX + s * KSTEP + kq];
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = rmfma(a, ya[s][j], acc[i][j]);
                }
            }
        }
        if (nxt) store_x(b ^ 1);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < NKS; ++s)
#pragma unroll
            for (int j = 0; j < FN; ++j) ya[s][j] = yb[s][j];
        b ^= 1;
    }

    // result rows: 4 kq + r (FP32-accumulating MFMAs), kq + 4 r (FP64)
    constexpr int RQ = sizeof(TI) == 8 ? 1 : 4, RR = sizeof(TI) == 8 ? 4 : 1;
    if (P.ksplit > 1) {
        TA* part = (TA*)P.part + int64_t(kz) * P.M * P.N;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t col = n0 + j * 16 + rl;
            if (col >= P.N) continue;
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = i * 16 + RQ * kq + RR * r;
                    if (row < P.M) part[int64_t(row) * P.N + col] = acc[i][j][r];
                }
        }
        return;
    }
    TA* C = (TA*)P.C;
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        if (ccol[j] < 0) continue;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i * 16 + RQ * kq + RR * r;
                if (row < P.M) C[crow[row] + ccol[j]] = acc[i][j][r];
            }
    }
}

template <typename TI, int FM, int FN>
static int rows_launch(const GemmParams& p, hipStream_t s) {
    using RT = typename std::conditional<sizeof(TI) == 2, uint16_t, TI>::type;
    constexpr int KC = RowsCfg<TI>::KC;
    const size_t lds = size_t(2) * 16 * FM * (KC + 16 / sizeof(TI)) * sizeof(RT);
    if (lds > 65536 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_rows_kernel<TI, FM, FN>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) != hipSuccess)
        return TLIB_EHIP;
    const dim3 grid(unsigned((p.N + 64 * FN - 1) / (64 * FN)), unsigned(p.ksplit));
    hipLaunchKernelGGL((gemm_rows_kernel<TI, FM, FN>), grid, dim3(256), lds, s, p);
    if (hipGetLastError() != hipSuccess) return TLIB_EHIP;
    return TLIB_OK;
}

template <typename TI>
static int rows_dispatch(int fm, int fn, const GemmParams& p, hipStream_t s) {
#define TLIB_ROWS(FM_, FN_) \
    if (fm == FM_ && fn == FN_) return rows_launch<TI, FM_, FN_>(p, s);
    TLIB_ROWS(1, 1) TLIB_ROWS(2, 1) TLIB_ROWS(4, 1) TLIB_ROWS(8, 1)
    TLIB_ROWS(1, 2) TLIB_ROWS(2, 2) TLIB_ROWS(4, 2) TLIB_ROWS(8, 2)
#undef TLIB_ROWS
    return TLIB_EINVAL;
}

int launch_gemm_rows(int dtype, int fm, int fn, const GemmParams& p, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return rows_dispatch<double>(fm, fn, p, s);
        case TLIB_F32: return rows_dispatch<float>(fm, fn, p, s);
        case TLIB_BF16: return rows_dispatch<bf16_t>(fm, fn, p, s);
        case TLIB_F16: return rows_dispatch<f16_t>(fm, fn, p, s);
    }
    return TLIB_EDTYPE;
}

int gemm_rows_kchunk(int dtype) {
    switch (dtype) {
        case TLIB_F64: return RowsCfg<double>::KC;
        case TLIB_F32: return RowsCfg<float>::KC;
        default: return RowsCfg<bf16_t>::KC;
    }
}

}  // namespace tlib
