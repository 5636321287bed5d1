// TTM (Sec. 5.2 Eq. ttm) and TTT (Eq. ttt, ttt_indices) as one GEMM
//   C[m, n] = sum_k X[m, k] * Y[k, n]
// whose three index groups (M, N, K) each address their operands through up
// to four (extent, stride) pairs decoded on the fly; the tensors are read in
// place, never unfolded or transposed.  For TTM, X is the matrix B (M = its
// rows j), Y is A (N = the modes of A other than m) and K is mode m.  For TTT,
// X = A (M = free A modes in phi order), Y = B (N = free B modes in psi
// order) and K runs over the contracted pairs.
//
// Work decomposition: a 256-thread workgroup (four wave64s in a WGM x WGN
// grid) owns a BM x BN tile of C; K is walked in BK slices staged through LDS,
// with the next slice's global loads issued into registers before the MFMAs on
// the current slice.  Matrix cores: v_mfma_f64_16x16x4 (FP64),
// v_mfma_f32_16x16x4 (FP32) and v_mfma_f32_16x16x32_{bf16,f16} (16-bit inputs,
// FP32 accumulation).  Each operand's loads are coalesced along whichever of
// its two index groups has the unit stride.  Optional split-K writes FP32/FP64
// partials that a second kernel sums in a fixed order.
#include <algorithm>

#include "device.hpp"

namespace tlib {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));

template <typename TI> struct Mfma;

template <> struct Mfma<double> {
    using acc_t = d4_t;
    static constexpr int KSTEP = 4;
    static constexpr int BK = 16;
};
template <> struct Mfma<float> {
    using acc_t = f4_t;
    static constexpr int KSTEP = 4;
    static constexpr int BK = 16;
};
template <> struct Mfma<bf16_t> {
    using acc_t = f4_t;
    static constexpr int KSTEP = 32;
    static constexpr int BK = 32;
};
template <> struct Mfma<f16_t> {
    using acc_t = f4_t;
    static constexpr int KSTEP = 32;
    static constexpr int BK = 32;
};

__device__ __forceinline__ d4_t mfma_step(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_step(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_bf16(u4_t a, u4_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, a), __builtin_bit_cast(bf8_t, b), c,
                                                   0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_f16(u4_t a, u4_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8_t, a), __builtin_bit_cast(h8_t, b), c,
                                                  0, 0, 0);
}

// Raw element storage in LDS: 16-bit types as uint16_t.
template <typename TI> struct Raw { using type = TI; };
template <> struct Raw<bf16_t> { using type = uint16_t; };
template <> struct Raw<f16_t> { using type = uint16_t; };

template <typename TI> __device__ __forceinline__ typename Raw<TI>::type raw_load(const TI* p) {
    if constexpr (sizeof(TI) == 2) return *reinterpret_cast<const uint16_t*>(p);
    else return *p;
}

template <typename TI, int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(256) void gemm_kernel(GemmParams P) {
    using TA = typename AccOf<TI>::type;
    using RT = typename Raw<TI>::type;
    using acc_t = typename Mfma<TI>::acc_t;
    constexpr bool WIDE = sizeof(TI) == 2;
    constexpr int BK = Mfma<TI>::BK;
    constexpr int KSTEP = Mfma<TI>::KSTEP;
    constexpr int WM = BM / WGM, WN = BN / WGN;
    constexpr int FM = WM / 16, FN = WN / 16;
    // LDS row pitches (elements): k-major tiles for FP32/FP64 fragments,
    // m/n-major tiles (k contiguous) for the 16-bit fragments.
    constexpr int PX = WIDE ? (BK + 8) : (BM + 4);
    constexpr int PY = WIDE ? (BK + 8) : (BN + 4);
    constexpr int XS = WIDE ? BM * PX : BK * PX;
    constexpr int YS = WIDE ? BN * PY : BK * PY;
    constexpr int EX = BM * BK / 256;  // X elements per thread per K slice
    constexpr int EY = BN * BK / 256;
    static_assert(EX >= 1 && EY >= 1, "tile too small");

    __shared__ __align__(16) RT Xs[XS];
    __shared__ __align__(16) RT Ys[YS];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;

    const int bid = blockIdx.x;
    const int tm = bid % P.tiles_m, tn = bid / P.tiles_m;
    const int m0 = tm * BM, n0 = tn * BN;
    const int kz = blockIdx.y;
    const int kbeg = kz * P.kchunk;
    const int kend = min(P.K, kbeg + P.kchunk);

    const TI* X = (const TI*)P.X;
    const TI* Y = (const TI*)P.Y;

    // fixed per-thread element slots of the X and Y slices
    int xm[EX], xk[EX], yn[EY], yk[EY];
    int64_t xoff[EX], yoff[EY];
#pragma unroll
    for (int j = 0; j < EX; ++j) {
        const int e = tid + j * 256;
        if (P.x_kfast) { xk[j] = e % BK; xm[j] = e / BK; }
        else { xm[j] = e % BM; xk[j] = e / BM; }
        const int gm = m0 + xm[j];
        xoff[j] = gm < P.M ? grp_off0(uint32_t(gm), P.gm) : int64_t(-1);
    }
#pragma unroll
    for (int j = 0; j < EY; ++j) {
        const int e = tid + j * 256;
        if (P.y_kfast) { yk[j] = e % BK; yn[j] = e / BK; }
        else { yn[j] = e % BN; yk[j] = e / BN; }
        const int gn = n0 + yn[j];
        yoff[j] = gn < P.N ? grp_off0(uint32_t(gn), P.gn) : int64_t(-1);
    }

    RT xr[EX], yr[EY];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int j = 0; j < EX; ++j) {
            const int gk = k0 + xk[j];
            RT v = RT(0);
            if (xoff[j] >= 0 && gk < kend) v = raw_load(X + xoff[j] + grp_off0(uint32_t(gk), P.gk));
            xr[j] = v;
        }
#pragma unroll
        for (int j = 0; j < EY; ++j) {
            const int gk = k0 + yk[j];
            RT v = RT(0);
            if (yoff[j] >= 0 && gk < kend) v = raw_load(Y + yoff[j] + grp_off1(uint32_t(gk), P.gk));
            yr[j] = v;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int j = 0; j < EX; ++j) {
            if constexpr (WIDE) Xs[xm[j] * PX + xk[j]] = xr[j];
            else Xs[xk[j] * PX + xm[j]] = xr[j];
        }
#pragma unroll
        for (int j = 0; j < EY; ++j) {
            if constexpr (WIDE) Ys[yn[j] * PY + yk[j]] = yr[j];
            else Ys[yk[j] * PY + yn[j]] = yr[j];
        }
    };

    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{};

    const int rl = lane & 15, kq = lane >> 4;
    const int wm0 = wm * WM, wn0 = wn * WN;

    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        stash();
        __syncthreads();
        if (k0 + BK < kend) fetch(k0 + BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += KSTEP) {
            if constexpr (WIDE) {
                u4_t a[FM], b[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    a[i] = *reinterpret_cast<const u4_t*>(&Xs[(wm0 + i * 16 + rl) * PX + ks + 8 * kq]);
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    b[j] = *reinterpret_cast<const u4_t*>(&Ys[(wn0 + j * 16 + rl) * PY + ks + 8 * kq]);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) {
                        if constexpr (std::is_same<TI, bf16_t>::value) acc[i][j] = mfma_bf16(a[i], b[j], acc[i][j]);
                        else acc[i][j] = mfma_f16(a[i], b[j], acc[i][j]);
                    }
            } else {
                TI a[FM], b[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) a[i] = Xs[(ks + kq) * PX + wm0 + i * 16 + rl];
#pragma unroll
                for (int j = 0; j < FN; ++j) b[j] = Ys[(ks + kq) * PY + wn0 + j * 16 + rl];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = mfma_step(a[i], b[j], acc[i][j]);
            }
        }
        __syncthreads();
    }

    // epilogue: lane (rl, kq) holds column rl of each 16x16 block; register r is
    // row 4*kq + r for the FP32-accumulating MFMAs and row kq + 4*r for the FP64
    // one (lane layouts checked on gfx950).
    constexpr int RQ = std::is_same<TI, double>::value ? 1 : 4;
    constexpr int RR = std::is_same<TI, double>::value ? 4 : 1;
    if (P.ksplit > 1) {
        TA* part = (TA*)P.part + int64_t(kz) * P.M * P.N;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = n0 + wn0 + j * 16 + rl;
            if (col >= P.N) continue;
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = m0 + wm0 + i * 16 + RQ * kq + RR * r;
                    if (row < P.M) part[int64_t(row) * P.N + col] = acc[i][j][r];
                }
        }
        return;
    }
    TA* C = (TA*)P.C;
    int64_t rowoff[FM][4];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = m0 + wm0 + i * 16 + RQ * kq + RR * r;
            rowoff[i][r] = row < P.M ? grp_off1(uint32_t(row), P.gm) : int64_t(-1);
        }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int col = n0 + wn0 + j * 16 + rl;
        if (col >= P.N) continue;
        const int64_t coff = grp_off1(uint32_t(col), P.gn);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (rowoff[i][r] >= 0) C[rowoff[i][r] + coff] = acc[i][j][r];
    }
}

template <typename TA>
__global__ __launch_bounds__(256) void gemm_ksum_kernel(GemmParams P) {
    const int64_t MN = int64_t(P.M) * P.N;
    const TA* part = (const TA*)P.part;
    for (int64_t o = int64_t(blockIdx.x) * 256 + threadIdx.x; o < MN; o += int64_t(gridDim.x) * 256) {
        TA s = part[o];
        for (int z = 1; z < P.ksplit; ++z) s += part[int64_t(z) * MN + o];
        const int row = int(o / P.N), col = int(o % P.N);
        ((TA*)P.C)[grp_off1(uint32_t(row), P.gm) + grp_off1(uint32_t(col), P.gn)] = s;
    }
}

// Generic fallback: one thread per C element, 64-bit decoding of every group.
template <typename TI>
__global__ __launch_bounds__(256) void gemm_generic_kernel(const TI* X, const TI* Y, typename AccOf<TI>::type* C,
                                                           GDims gm, GDims gn, GDims gk) {
    using TA = typename AccOf<TI>::type;
    const int64_t total = gm.total * gn.total;
    for (int64_t o = int64_t(blockIdx.x) * 256 + threadIdx.x; o < total; o += int64_t(gridDim.x) * 256) {
        const int64_t mi = o % gm.total, ni = o / gm.total;
        int64_t om[2], on[2], ok[2];
        gd_decode(mi, gm, 2, om);
        gd_decode(ni, gn, 2, on);
        TA acc = TA(0);
        for (int64_t k = 0; k < gk.total; ++k) {
            gd_decode(k, gk, 2, ok);
            acc += to_acc(X[om[0] + ok[0]]) * to_acc(Y[on[0] + ok[1]]);
        }
        C[om[1] + on[1]] = acc;
    }
}

// ------------------------------------------------------------------ launchers

template <typename TI, int BM, int BN, int WGM, int WGN>
static int gemm_launch(const GemmParams& p, hipStream_t s) {
    using TA = typename AccOf<TI>::type;
    const unsigned tiles = unsigned(p.tiles_m) * unsigned(p.tiles_n);
    hipLaunchKernelGGL((gemm_kernel<TI, BM, BN, WGM, WGN>), dim3(tiles, unsigned(p.ksplit)), dim3(256), 0, s, p);
    if (hipGetLastError() != hipSuccess) return TLIB_EHIP;
    if (p.ksplit > 1) {
        const int64_t MN = int64_t(p.M) * p.N;
        const unsigned g = unsigned(std::min<int64_t>((MN + 255) / 256, 65536));
        hipLaunchKernelGGL((gemm_ksum_kernel<TA>), dim3(g), dim3(256), 0, s, p);
        if (hipGetLastError() != hipSuccess) return TLIB_EHIP;
    }
    return TLIB_OK;
}

template <typename TI>
static int gemm_dispatch(int tile, const GemmParams& p, hipStream_t s) {
    switch (tile) {
        case GT_16x256: return gemm_launch<TI, 16, 256, 1, 4>(p, s);
        case GT_64x128: return gemm_launch<TI, 64, 128, 2, 2>(p, s);
        case GT_128x128: return gemm_launch<TI, 128, 128, 2, 2>(p, s);
        case GT_256x64: return gemm_launch<TI, 256, 64, 4, 1>(p, s);
        case GT_64x64: return gemm_launch<TI, 64, 64, 2, 2>(p, s);
    }
    return TLIB_EINVAL;
}

int launch_gemm(int dtype, int tile, const GemmParams& p, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return gemm_dispatch<double>(tile, p, s);
        case TLIB_F32: return gemm_dispatch<float>(tile, p, s);
        case TLIB_BF16: return gemm_dispatch<bf16_t>(tile, p, s);
        case TLIB_F16: return gemm_dispatch<f16_t>(tile, p, s);
    }
    return TLIB_EDTYPE;
}

template <typename TI>
static int generic_launch(const void* X, const void* Y, void* C, const GDims& gm, const GDims& gn,
                          const GDims& gk, hipStream_t s) {
    using TA = typename AccOf<TI>::type;
    const int64_t total = gm.total * gn.total;
    const unsigned blocks = unsigned(std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536)));
    hipLaunchKernelGGL((gemm_generic_kernel<TI>), dim3(blocks), dim3(256), 0, s, (const TI*)X, (const TI*)Y,
                       (TA*)C, gm, gn, gk);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

int launch_gemm_generic(int dtype, const void* X, const void* Y, void* C, const GDims& m, const GDims& n,
                        const GDims& k, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return generic_launch<double>(X, Y, C, m, n, k, s);
        case TLIB_F32: return generic_launch<float>(X, Y, C, m, n, k, s);
        case TLIB_BF16: return generic_launch<bf16_t>(X, Y, C, m, n, k, s);
        case TLIB_F16: return generic_launch<f16_t>(X, Y, C, m, n, k, s);
    }
    return TLIB_EDTYPE;
}

}  // namespace tlib
