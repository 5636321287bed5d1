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
typedef uint32_t u2_t __attribute__((ext_vector_type(2)));

// Source of the loads that fall outside X or Y: selecting the address rather
// than the loaded value keeps the loads unconditional, without an exec branch
// around each one.
__device__ __align__(16) double g_gemm_zero[2] = {0.0, 0.0};

template <typename TI> struct Mfma;

// BK: depth of one K slice staged through LDS (several MFMA k-steps), chosen
// so that a slice moves at least 8 KB per workgroup in flight.
template <> struct Mfma<double> {
    using acc_t = d4_t;
    static constexpr int KSTEP = 4;
    static constexpr int BK = 16;
};
template <> struct Mfma<float> {
    using acc_t = f4_t;
    static constexpr int KSTEP = 4;
    static constexpr int BK = 32;
};
template <> struct Mfma<bf16_t> {
    using acc_t = f4_t;
    static constexpr int KSTEP = 32;
    static constexpr int BK = 128;
};
template <> struct Mfma<f16_t> {
    using acc_t = f4_t;
    static constexpr int KSTEP = 32;
    static constexpr int BK = 128;
};

// K slice depth of a tile: 16-bit slices hold four MFMA k-steps (two for
// tiles with BM + BN > 256, whose 128-deep slices would leave room for only
// one workgroup per CU) when both operands load 16-byte vectors (YW bit 0,
// and bit 1 or 2); an operand loaded element by element holds one register
// per element in flight, so its slices keep one k-step (deeper ones spill),
// or as many as one pass of Y's transposed vector stash covers.  The planner
// rounds K ranges to the deepest slice, a multiple of all of them.
template <typename TI, int BM, int BN, int YW = 7> struct SliceK {
    static constexpr bool VEC16 = (YW & 1) != 0 && (YW & 6) != 0;
    static constexpr int SHALLOW = (YW & 4) != 0 && 2048 / BN > 32 ? 2048 / BN : 32;
    static constexpr int value = sizeof(TI) != 2 ? Mfma<TI>::BK
                                 : !VEC16        ? SHALLOW
                                 : BM + BN > 256 ? 64
                                                 : Mfma<TI>::BK;
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

// amdgpu_waves_per_eu(2): at least two waves per SIMD.  With it the compiler
// keeps the accumulators in the unified VGPR file instead of splitting off
// AGPRs, which measured 12-17 % faster for the FP64 tiles on MI355X and
// neutral for the others.
// YW > 0: Y's slice loaded as vectors of YW elements along N (16 or 8
// bytes).  Each thread owns YW consecutive columns for the whole K walk (their offset is decoded once) and
// every RS-th row of each slice; a wave in which some thread's columns are not
// consecutive in memory (the end of a run of N's first dim, or past N) loads
// its columns one by one.
template <typename TI, int BM, int BN, int WGM, int WGN, int YW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_kernel(GemmParams P) {
    using TA = typename AccOf<TI>::type;
    using RT = typename Raw<TI>::type;
    using acc_t = typename Mfma<TI>::acc_t;
    constexpr bool WIDE = sizeof(TI) == 2;
    constexpr int BK = SliceK<TI, BM, BN, YW>::value;
    constexpr int KSTEP = Mfma<TI>::KSTEP;
    constexpr int WM = BM / WGM, WN = BN / WGN;
    constexpr int FM = WM / 16, FN = WN / 16;
    // LDS row pitches (elements): k-major tiles for FP32/FP64 fragments,
    // m/n-major tiles (k contiguous) for the 16-bit fragments.  The pads keep
    // the stores of k-pairs (lanes 2 k apart) and the fragment reads (16 rows
    // x 4 k) on distinct banks: FP32 X pitch = 18 mod 64 dwords, FP32 Y pitch
    // = 20 mod 64 (a multiple of 4, for its 16-byte row stores), FP64 pitches
    // = 2 mod 16 doubles (measured: FP32 GEMM 14-15 %, FP64 1-5 % faster than
    // pads of 16 / 4).
    constexpr int PADX = sizeof(TI) == 8 ? 2 : 18;
    constexpr int PADY = sizeof(TI) == 8 ? 2 : 20;
    constexpr int PX = WIDE ? (BK + 8) : (BM + PADX);
    constexpr int PY = WIDE ? (BK + 8) : (BN + PADY);
    constexpr int XS = WIDE ? BM * PX : BK * PX;
    constexpr int YS = WIDE ? BN * PY : BK * PY;
    constexpr int EX = BM * BK / 256;  // X elements per thread per K slice
    constexpr int EY = BN * BK / 256;
    static_assert(EX >= 1 && EY >= 1, "tile too small");
    // FP32/FP64: YW & 15 > 0 = Y as vectors of that many elements along N;
    // YW & 16 / YW & 32 = X / Y loaded as groups of 2 consecutive k.  16-bit:
    // YW bit 0 / bit 1 = X / Y loaded as 16-byte groups of 8 consecutive k
    // (see fetch).
    constexpr bool YV = WIDE ? (YW & 4) != 0 : (YW & 15) > 0;
    constexpr bool XKV = WIDE ? (YW & 1) != 0 : (YW & 16) != 0;
    constexpr bool YKV = WIDE ? (YW & 2) != 0 : (YW & 32) != 0;
    constexpr int GVX = WIDE ? 8 : 2;              // k per X / Y group
    constexpr int KGX = BK / GVX;                  // groups per slice row
    constexpr int KG = KGX;
    constexpr int NXV = BM * KGX, NYV = BN * KG;   // k groups per X / Y slice
    constexpr int EXV = (NXV + 255) / 256, EYK = (NYV + 255) / 256;
    using xg_t = typename std::conditional<(WIDE || sizeof(TI) == 8), u4_t, u2_t>::type;
    constexpr int VY = YV ? (WIDE ? 8 : (YW & 15)) : 1;
    constexpr int CG = BN / VY;                   // column groups of a Y slice
    constexpr int RS = YV ? 256 / CG : 1;         // rows of the slice per pass
    constexpr int EYV = YV ? BK / RS : 1;         // vectors per thread per slice
    static_assert(!YV || (256 % CG == 0 && BK % RS == 0 && EYV >= 1), "vector Y slice");
    using YE = typename std::conditional<(sizeof(TI) >= 4), TI, uint16_t>::type;
    typedef YE yv_t __attribute__((ext_vector_type(VY)));

    // The X/Y slices and, after the K loop, the epilogue's staging rows share
    // one LDS buffer.
    constexpr int SP = WN + (sizeof(TA) == 8 ? 2 : 4);  // staging pitch, 16-byte rows
    constexpr int XB = (XS * int(sizeof(RT)) + 15) / 16 * 16;
    constexpr int MAIN_B = XB + YS * int(sizeof(RT));
    constexpr int STAGE_B = 4 * 16 * SP * int(sizeof(TA));
    __shared__ __align__(16) unsigned char smem[MAIN_B > STAGE_B ? MAIN_B : STAGE_B];
    RT* Xs = reinterpret_cast<RT*>(smem);
    RT* Ys = reinterpret_cast<RT*>(smem + XB);
    // Offset tables: every row / column of the tile decoded once (-1 = outside),
    // the K offsets of a slice decoded once per slice (double-buffered).
    __shared__ int64_t xrow[BM], crow[BM], ycol[BN], ccol[BN];
    __shared__ int64_t kx[2][BK], ky[2][BK];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;

    // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs, so
    // renumber them such that consecutive logical tiles (the M tiles that share
    // one N tile of Y) run on the same XCD and meet in its L2.
    int bid = blockIdx.x;
    {
        const int T = P.tiles_m * P.tiles_n;
        const int xcd = bid & 7, idx = bid >> 3, per = T >> 3, rem = T & 7;
        bid = (xcd < rem) ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
    }
    const int tm = bid % P.tiles_m, tn = bid / P.tiles_m;
    const int m0 = tm * BM, n0 = tn * BN;
    const int kz = blockIdx.y;
    const int kbeg = kz * P.kchunk;
    const int kend = min(P.K, kbeg + P.kchunk);

    const TI* X = (const TI*)P.X;
    const TI* Y = (const TI*)P.Y;

    for (int i = tid; i < BM; i += 256) {
        int64_t a = -1, c = -1;
        if (m0 + i < P.M) grp_decode(uint32_t(m0 + i), P.gm, a, c);
        xrow[i] = a;
        crow[i] = c;
    }
    for (int i = tid; i < BN; i += 256) {
        int64_t a = -1, c = -1;
        if (n0 + i < P.N) grp_decode(uint32_t(n0 + i), P.gn, a, c);
        ycol[i] = a;
        ccol[i] = c;
    }
    auto ktable = [&](int k0, int slot) {
        if (tid < BK) {
            int64_t a = -1, b = -1;
            if (k0 + tid < kend) grp_decode(uint32_t(k0 + tid), P.gk, a, b);
            kx[slot][tid] = a;
            ky[slot][tid] = b;
        }
    };

    // Slot j of this thread in the X slice is element e = tid + 256 j, read
    // along k (x_kfast) or along m; the same for Y.
    auto xslot = [&](int j, int& mm, int& kk) {
        const int e = tid + j * 256;
        if (P.x_kfast) { kk = e % BK; mm = e / BK; }
        else { mm = e % BM; kk = e / BM; }
    };
    auto yslot = [&](int j, int& nn, int& kk) {
        const int e = tid + j * 256;
        if (P.y_kfast) { kk = e % BK; nn = e / BK; }
        else { nn = e % BN; kk = e / BN; }
    };

    RT xr[XKV ? 1 : EX], yr[(YV || YKV) ? 1 : EY];
    yv_t yvr[EYV];
    xg_t xg[XKV ? EXV : 1];
    xg_t yg[YKV ? EYK : 1];
    // YV: this thread's column group and first row, the group's offset and
    // whether every thread of the wave has VY consecutive, aligned columns
    const int ycg = tid % CG, yrow = tid / CG;
    int64_t ycv = 0;
    bool wvec = false;
    int k0n = 0;  // first k of the slice being fetched
    const TI* zsrc = reinterpret_cast<const TI*>(g_gemm_zero);
    // k groups: slot e = tid + 256 j is group e % KGX (X) or e % KG (16-bit
    // Y) of row / column e / KGX (e / KG).  The host enables them only where
    // K's first dim has unit stride in the operand and a multiple of the
    // group as extent and every other stride keeps the groups aligned, so
    // the group starting at a valid k is wholly inside the slice's K range
    // and contiguous in memory.
    auto fetch = [&](int slot) {
        if constexpr (XKV) {
#pragma unroll
            for (int j = 0; j < EXV; ++j) {
                const int e = tid + j * 256;
                const int mm = min(e / KGX, BM - 1), kv = e % KGX;
                const int64_t a = e < NXV ? xrow[mm] : -1, b = kx[slot][kv * GVX];
                xg[j] = *reinterpret_cast<const xg_t*>((a >= 0 && b >= 0) ? X + (a + b) : zsrc);
            }
        } else {
#pragma unroll
            for (int j = 0; j < EX; ++j) {
                int mm, kk;
                xslot(j, mm, kk);
                const int64_t a = xrow[mm], b = kx[slot][kk];
                xr[j] = raw_load((a >= 0 && b >= 0) ? X + (a + b) : zsrc);
            }
        }
        if constexpr (YKV) {
#pragma unroll
            for (int j = 0; j < EYK; ++j) {
                const int e = tid + j * 256;
                const int nn = min(e / KG, BN - 1), kv = e % KG;
                const int64_t a = e < NYV ? ycol[nn] : -1, b = ky[slot][kv * GVX];
                yg[j] = *reinterpret_cast<const xg_t*>((a >= 0 && b >= 0) ? Y + (a + b) : zsrc);
            }
        } else if constexpr (YV) {
            // the choice is per wave (wvec is uniform), so only one of the two
            // load sequences runs and no load waits for the other's registers
            if (wvec) {
                // all addresses first, then the loads back to back
                const yv_t* ap[EYV];
#pragma unroll
                for (int j = 0; j < EYV; ++j) {
                    const int k = k0n + yrow + RS * j;
                    ap[j] = reinterpret_cast<const yv_t*>(k < kend ? Y + (ycv + int64_t(k) * P.syk) : zsrc);
                }
#pragma unroll
                for (int j = 0; j < EYV; ++j) yvr[j] = *ap[j];
            } else {
#pragma unroll
                for (int j = 0; j < EYV; ++j) {
                    const int k = k0n + yrow + RS * j;
#pragma unroll
                    for (int e = 0; e < VY; ++e) {
                        const int64_t a = ycol[ycg * VY + e];
                        yvr[j][e] = raw_load((a >= 0 && k < kend) ? Y + (a + int64_t(k) * P.syk) : zsrc);
                    }
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < EY; ++j) {
                int nn, kk;
                yslot(j, nn, kk);
                const int64_t a = ycol[nn], b = ky[slot][kk];
                yr[j] = raw_load((a >= 0 && b >= 0) ? Y + (a + b) : zsrc);
            }
        }
    };
    auto stash = [&]() {
        if constexpr (XKV) {
#pragma unroll
            for (int j = 0; j < EXV; ++j) {
                const int e = tid + j * 256;
                if constexpr (WIDE) {
                    if (e < NXV) *reinterpret_cast<u4_t*>(&Xs[(e / KGX) * PX + (e % KGX) * GVX]) = xg[j];
                } else if (e < NXV) {
                    // k-major tile: the group's two k go to two rows
                    struct Pair {
                        TI v[2];
                    };
                    const Pair pv = __builtin_bit_cast(Pair, xg[j]);
                    const int mm = e / KGX, k2 = (e % KGX) * 2;
                    Xs[k2 * PX + mm] = pv.v[0];
                    Xs[(k2 + 1) * PX + mm] = pv.v[1];
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < EX; ++j) {
                int mm, kk;
                xslot(j, mm, kk);
                if constexpr (WIDE) Xs[mm * PX + kk] = xr[j];
                else Xs[kk * PX + mm] = xr[j];
            }
        }
        if constexpr (YKV) {
#pragma unroll
            for (int j = 0; j < EYK; ++j) {
                const int e = tid + j * 256;
                if constexpr (WIDE) {
                    if (e < NYV) *reinterpret_cast<u4_t*>(&Ys[(e / KG) * PY + (e % KG) * GVX]) = yg[j];
                } else if (e < NYV) {
                    struct Pair {
                        TI v[2];
                    };
                    const Pair pv = __builtin_bit_cast(Pair, yg[j]);
                    const int nn = e / KG, k2 = (e % KG) * 2;
                    Ys[k2 * PY + nn] = pv.v[0];
                    Ys[(k2 + 1) * PY + nn] = pv.v[1];
                }
            }
        } else if constexpr (YV) {
            if constexpr (WIDE) {
                // the slice is stored n-major (k contiguous per column, as the
                // 16-bit MFMA operands read it): each vector's eight columns
                // go to eight rows
#pragma unroll
                for (int j = 0; j < EYV; ++j)
#pragma unroll
                    for (int e = 0; e < VY; ++e) Ys[(ycg * VY + e) * PY + yrow + RS * j] = yvr[j][e];
            } else {
#pragma unroll
                for (int j = 0; j < EYV; ++j)
                    *reinterpret_cast<yv_t*>(&Ys[(yrow + RS * j) * PY + ycg * VY]) = yvr[j];
            }
        } else {
#pragma unroll
            for (int j = 0; j < EY; ++j) {
                int nn, kk;
                yslot(j, nn, kk);
                if constexpr (WIDE) Ys[nn * PY + kk] = yr[j];
                else Ys[kk * PY + nn] = yr[j];
            }
        }
    };

    acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{};

    const int rl = lane & 15, kq = lane >> 4;
    const int wm0 = wm * WM, wn0 = wn * WN;

    ktable(kbeg, 0);
    __syncthreads();
    if constexpr (YV) {
        ycv = ycol[ycg * VY];
        bool ok = ycv >= 0 && (ycv % VY) == 0;
#pragma unroll
        for (int e = 1; e < VY; ++e) ok = ok && ycol[ycg * VY + e] == ycv + e;
        wvec = __ballot(!ok) == 0;
    }
    k0n = kbeg;
    if (kbeg < kend) fetch(0);
    int slot = 0;
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        stash();
        if (k0 + BK < kend) ktable(k0 + BK, slot ^ 1);
        __syncthreads();
        k0n = k0 + BK;
        if (k0 + BK < kend) fetch(slot ^ 1);
        slot ^= 1;
        // the last slice of a K range stops at the first k-step that lies
        // wholly past its end (those rows of the slice are zero)
        const int klen = kend - k0;
#pragma unroll
        for (int ks = 0; ks < BK; ks += KSTEP) {
            if (ks >= klen) break;
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
    // Staged epilogue: each wave writes one 16-row block of its tile to LDS,
    // then stores whole rows with lanes running along C's columns (16-byte
    // vector stores when C's column strides allow it).  The staging rows are
    // the wave's own (the K loop's last barrier has already separated them
    // from the other waves' operand reads), so the waves go through their
    // blocks without waiting for each other.
    TA* C = (TA*)P.C;
    TA* stg = reinterpret_cast<TA*>(smem) + wave * 16 * SP;
    constexpr int V = 16 / int(sizeof(TA));
    constexpr int LPR = WN / V;   // lanes per staged row
    constexpr int RPI = 64 / LPR;  // rows per pass
    static_assert(WN % V == 0 && 64 % LPR == 0, "staging shape");
    typedef uint32_t v16_t __attribute__((ext_vector_type(4)));
    const int cl = (lane % LPR) * V;
    const int64_t cb = ccol[wn0 + cl];
    const bool vec = P.c_vec && cb >= 0;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) stg[(RQ * kq + RR * r) * SP + j * 16 + rl] = acc[i][j][r];
#pragma unroll
        for (int rr = lane / LPR; rr < 16; rr += RPI) {
            const int64_t ro = crow[wm0 + i * 16 + rr];
            if (ro < 0) continue;
            const TA* src = &stg[rr * SP + cl];
            if (vec) {
                *reinterpret_cast<v16_t*>(C + ro + cb) = *reinterpret_cast<const v16_t*>(src);
            } else {
#pragma unroll
                for (int t = 0; t < V; ++t) {
                    const int64_t co = ccol[wn0 + cl + t];
                    if (co >= 0) C[ro + co] = src[t];
                }
            }
        }
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
    const dim3 grid(tiles, unsigned(p.ksplit));
#define TLIB_GEMM(VM) hipLaunchKernelGGL((gemm_kernel<TI, BM, BN, WGM, WGN, VM>), grid, dim3(256), 0, s, p)
    const bool xg = (p.kvec & 1) != 0;
    if constexpr (sizeof(TI) == 8) {
        if (p.kvec & 2) {  // Y in k groups (then no vectors along N)
            if (xg) TLIB_GEMM(48);
            else TLIB_GEMM(32);
        } else if (p.y_vec == 2) {
            if (xg) TLIB_GEMM(18);
            else TLIB_GEMM(2);
        } else {
            if (xg) TLIB_GEMM(16);
            else TLIB_GEMM(0);
        }
    } else if constexpr (sizeof(TI) == 4) {
        if (p.kvec & 2) {
            if (xg) TLIB_GEMM(48);
            else TLIB_GEMM(32);
        } else if (p.y_vec == 4) {
            if (xg) TLIB_GEMM(20);
            else TLIB_GEMM(4);
        } else if (p.y_vec == 2) {
            if (xg) TLIB_GEMM(18);
            else TLIB_GEMM(2);
        } else {
            if (xg) TLIB_GEMM(16);
            else TLIB_GEMM(0);
        }
    } else {
        // bit 0 / 1: X / Y in k groups; bit 2: Y as 8-element vectors along N
        switch ((p.kvec & 3) | (p.y_vec ? 4 : 0)) {
            case 1: hipLaunchKernelGGL((gemm_kernel<TI, BM, BN, WGM, WGN, 1>), grid, dim3(256), 0, s, p); break;
            case 2: hipLaunchKernelGGL((gemm_kernel<TI, BM, BN, WGM, WGN, 2>), grid, dim3(256), 0, s, p); break;
            case 3: hipLaunchKernelGGL((gemm_kernel<TI, BM, BN, WGM, WGN, 3>), grid, dim3(256), 0, s, p); break;
            case 4: hipLaunchKernelGGL((gemm_kernel<TI, BM, BN, WGM, WGN, 4>), grid, dim3(256), 0, s, p); break;
            case 5: hipLaunchKernelGGL((gemm_kernel<TI, BM, BN, WGM, WGN, 5>), grid, dim3(256), 0, s, p); break;
            default: hipLaunchKernelGGL((gemm_kernel<TI, BM, BN, WGM, WGN, 0>), grid, dim3(256), 0, s, p);
        }
    }
#undef TLIB_GEMM
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
        case GT_128x64: return gemm_launch<TI, 128, 64, 2, 2>(p, s);
        case GT_256x32: return gemm_launch<TI, 256, 32, 4, 1>(p, s);
    }
    return TLIB_EINVAL;
}

int launch_gemm_ksum(int acc_dtype, const GemmParams& p, hipStream_t s) {
    const int64_t MN = int64_t(p.M) * p.N;
    const unsigned g = unsigned(std::min<int64_t>((MN + 255) / 256, 65536));
    if (acc_dtype == TLIB_F64) hipLaunchKernelGGL((gemm_ksum_kernel<double>), dim3(g), dim3(256), 0, s, p);
    else hipLaunchKernelGGL((gemm_ksum_kernel<float>), dim3(g), dim3(256), 0, s, p);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

template <typename TI>
static int slice_k(int tile) {
    switch (tile) {
        case GT_16x256: return SliceK<TI, 16, 256>::value;
        case GT_64x128: return SliceK<TI, 64, 128>::value;
        case GT_128x128: return SliceK<TI, 128, 128>::value;
        case GT_256x64: return SliceK<TI, 256, 64>::value;
        case GT_64x64: return SliceK<TI, 64, 64>::value;
        case GT_128x64: return SliceK<TI, 128, 64>::value;
        case GT_256x32: return SliceK<TI, 256, 32>::value;
    }
    return Mfma<TI>::BK;
}

int gemm_slice_k(int dtype, int tile) {
    switch (dtype) {
        case TLIB_F64: return slice_k<double>(tile);
        case TLIB_F32: return slice_k<float>(tile);
        case TLIB_BF16: return slice_k<bf16_t>(tile);
        default: return slice_k<f16_t>(tile);
    }
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
