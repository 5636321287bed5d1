// Two successive mode products in one pass over A (Sec. 5.2 Eq. ttm applied
// twice, the step pair of tensor_times_matrices / the Tucker chain):
//   C(.., j_g, .., j_f, ..) = sum_{i_g, i_f} Ug(j_g, i_g) Uf(j_f, i_f) A(.., i_g, .., i_f, ..)
// where f is the contracted mode with the smaller stride in A and g the other
// one.  The intermediate A x_f Uf is never written: a workgroup owns 16
// columns (the index tuples of the other modes) and walks i_g four values at
// a time.  Stage one: each wave forms T = Uf * A(i_g, :, columns) for its i_g
// on the matrix cores (Uf from LDS, A from LDS slabs or straight from
// memory) and stages T in LDS.  Stage two: the four i_g of the group are the k
// of one more MFMA step, C(j_g, (j_f, column)) += Ug(j_g, i_g) T(i_g, (j_f,
// column)), into the C tile (at most 32 x 32 x 16 values) held in the waves'
// accumulators.
#include "device.hpp"

namespace tlib {

typedef float t2f4_t __attribute__((ext_vector_type(4)));
typedef double t2d4_t __attribute__((ext_vector_type(4)));

template <typename TI> struct T2Mfma;
template <> struct T2Mfma<double> { using acc_t = t2d4_t; };
template <> struct T2Mfma<float> { using acc_t = t2f4_t; };

__device__ __forceinline__ t2d4_t t2_mfma(double a, double b, t2d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ t2f4_t t2_mfma(float a, float b, t2f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Source of the A fragment loads outside the operand.
__device__ __align__(16) double g_ttm2_zero[2] = {0.0, 0.0};

constexpr int T2_COLS = 16;  // columns per workgroup
constexpr int T2_KC = 8;     // k-steps of a fragment chunk

// FMB: 16-row blocks of Uf (n'_f <= 16 FMB).  LDS: Uf as [16 FMB][KFP + 1]
// (k fastest, odd pitch), Ug as [n_g][32] (j_g fastest), T as [4][32][16].
// VEC: the 16 columns of a tile are consecutive and 16-byte aligned in A, so
// each wave copies its slab A(i_g, :, columns) into LDS ([KFP][16], in place
// of Ug, whose columns are then read from memory) with 16-byte loads issued
// one group of i_g ahead into registers, and takes the MFMA fragments from
// there.
// NV: 16-byte loads per lane for one slab (VEC; 12 or 16 by the slab's rows)
template <typename TI, int FMB, bool VEC, int NV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void ttm2_kernel(Ttm2Params P) {
    using acc_t = typename T2Mfma<TI>::acc_t;
    extern __shared__ __align__(16) unsigned char smem[];
    const int KFP = (P.n_f + 3) & ~3;  // i_f padded to whole k-steps
    const int UPF = KFP + 1;
    TI* Ufs = reinterpret_cast<TI*>(smem);
    TI* Ts = Ufs + 16 * FMB * UPF;
    TI* As = Ts + 4 * 32 * T2_COLS;  // VEC: [4][KFP][16]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rl = lane & 15, kq = lane >> 4;
    const TI* A = reinterpret_cast<const TI*>(P.A);
    const TI* Uf = reinterpret_cast<const TI*>(P.Uf);
    const TI* Ug = reinterpret_cast<const TI*>(P.Ug);

    // factors to LDS, zero-padded
    for (int e = tid; e < 16 * FMB * UPF; e += 256) {
        const int r = e / UPF, k = e - r * UPF;
        Ufs[e] = (r < P.m_f && k < P.n_f) ? Uf[int64_t(r) * P.sUf0 + int64_t(k) * P.sUf1] : TI(0);
    }
    // this lane's column for the MFMA B operand (A fragments) and for the C
    // tile (stage two): column c0 + rl, offsets in A and C
    // tiles that share cache lines of A (neighbours) run on one XCD:
    // workgroups are dealt round-robin to the eight XCDs, so XCD x takes the
    // x-th contiguous range of tiles
    int64_t tile;
    {
        const int64_t nt = gridDim.x, b = blockIdx.x;
        const int64_t x = b & 7, idx = b >> 3, per = nt >> 3, rem = nt & 7;
        tile = x < rem ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
    }
    const int64_t c0 = tile * T2_COLS;
    const bool colok = c0 + rl < P.ncol;
    int64_t oa, oc;
    grp_decode(uint32_t(colok ? c0 + rl : 0), P.gc, oa, oc);
    int64_t oa0 = 0, oc0;
    if constexpr (VEC) grp_decode(uint32_t(c0), P.gc, oa0, oc0);
    const TI* zsrc = reinterpret_cast<const TI*>(g_ttm2_zero);

    // stage two on the matrix cores: C(j_g, (j_f, column)) += Ug(j_g, i_g)
    // T(i_g, (j_f, column)) with i_g as the k of a 16x16x4 MFMA; wave w owns
    // the j_f blocks 8w .. 8w+7 (16 columns each) for both 16-row j_g blocks
    acc_t cacc[2][8];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int b = 0; b < 8; ++b) cacc[mb][b] = acc_t{};
    __syncthreads();

    const int nks = KFP / 4;  // k-steps over i_f
    // VEC: lane l copies vectors v = l + 64 t of its wave's slab: row v / VPR,
    // columns VA (v % VPR) .. +VA-1 of the tile
    constexpr int VA = 16 / int(sizeof(TI));
    constexpr int VPR = T2_COLS / VA;
    typedef TI av_t __attribute__((ext_vector_type(VA)));
    av_t pre[VEC ? NV : 1];
    auto prefetch = [&](int ig) {
        if constexpr (VEC) {
            const bool gok = ig < P.n_g;
            const TI* base = A + (oa0 + int64_t(gok ? ig : 0) * P.s_g);
#pragma unroll
            for (int t = 0; t < NV; ++t) {
                const int v = lane + 64 * t;
                const int row = v / VPR, cq = v - row * VPR;
                const bool ok = gok && row < P.n_f;
                pre[t] = *reinterpret_cast<const av_t*>(ok ? base + (int64_t(row) * P.s_f + VA * cq) : zsrc);
            }
        }
    };
    if constexpr (VEC) prefetch(wave);
    for (int ig0 = 0; ig0 < P.n_g; ig0 += 4) {
        // stage one: wave w forms T for i_g = ig0 + w
        const int ig = ig0 + wave;
        const bool gok = ig < P.n_g;
        acc_t acc[FMB];
#pragma unroll
        for (int m = 0; m < FMB; ++m) acc[m] = acc_t{};
        if constexpr (VEC) {
            TI* aw = As + wave * KFP * T2_COLS;
#pragma unroll
            for (int t = 0; t < NV; ++t) {
                const int v = lane + 64 * t;
                if (v < KFP * VPR) *reinterpret_cast<av_t*>(&aw[v * VA]) = pre[t];
            }
            prefetch(ig + 4);
            __syncthreads();
            for (int s0 = 0; s0 < nks; ++s0) {
                const TI b = aw[(4 * s0 + kq) * T2_COLS + rl];
#pragma unroll
                for (int m = 0; m < FMB; ++m) acc[m] = t2_mfma(Ufs[(m * 16 + rl) * UPF + 4 * s0 + kq], b, acc[m]);
            }
        } else {
            const TI* arow = A + (oa + int64_t(gok ? ig : 0) * P.s_g);
            for (int s0 = 0; s0 < nks; s0 += T2_KC) {
                TI fr[T2_KC];
#pragma unroll
                for (int s = 0; s < T2_KC; ++s) {
                    const int k = 4 * (s0 + s) + kq;
                    fr[s] = *((gok && colok && k < P.n_f) ? arow + int64_t(k) * P.s_f : zsrc);
                }
#pragma unroll
                for (int s = 0; s < T2_KC; ++s) {
                    if (s0 + s >= nks) break;
#pragma unroll
                    for (int m = 0; m < FMB; ++m)
                        acc[m] = t2_mfma(Ufs[(m * 16 + rl) * UPF + 4 * (s0 + s) + kq], fr[s], acc[m]);
                }
            }
        }
        // T(j_f, column) to LDS: result register r of block m is row
        // 4 kq + r (FP32) or kq + 4 r (FP64) of the block, column rl
        TI* tw = Ts + wave * 32 * T2_COLS;
#pragma unroll
        for (int m = 0; m < FMB; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m * 16 + (sizeof(TI) == 8 ? kq + 4 * r : 4 * kq + r);
                if (row < 32) tw[row * T2_COLS + rl] = gok ? acc[m][r] : TI(0);
            }
        __syncthreads();
        // stage two: the four i_g of this group are the k of one MFMA step
        {
            const int igk = ig0 + kq;
            TI ua[2];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                const int jg = mb * 16 + rl;
                ua[mb] = *((jg < P.m_g && igk < P.n_g) ? Ug + (int64_t(jg) * P.sUg0 + int64_t(igk) * P.sUg1) : zsrc);
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int jf = 8 * wave + b;
                const TI tb = jf < 32 ? Ts[kq * 32 * T2_COLS + jf * T2_COLS + rl] : TI(0);
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) cacc[mb][b] = t2_mfma(ua[mb], tb, cacc[mb][b]);
            }
        }
        __syncthreads();
    }

    // write the C tile: lane (rl, kq) holds column c0 + rl of j_f = 8 w + b
    // and rows j_g = 16 mb + 4 kq + r (FP32) or 16 mb + kq + 4 r (FP64)
    if (colok) {
        TI* C = reinterpret_cast<TI*>(P.C) + oc;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int jf = 8 * wave + b;
            if (jf >= P.m_f) break;
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int jg = mb * 16 + (sizeof(TI) == 8 ? kq + 4 * r : 4 * kq + r);
                    if (jg < P.m_g) C[int64_t(jg) * P.sC_g + int64_t(jf) * P.sC_f] = cacc[mb][b][r];
                }
        }
    }
}

int ttm2_lds_bytes(int dtype, int m_f, int n_f, int n_g, bool vec) {
    const int fmb = (m_f + 15) / 16;
    const int kfp = (n_f + 3) & ~3;
    (void)n_g;
    return (16 * fmb * (kfp + 1) + (vec ? 4 * kfp * T2_COLS : 0) + 4 * 32 * T2_COLS) * esize(dtype);
}

int ttm2_vec_rows(int dtype) { return dtype == TLIB_F32 ? 64 * 16 / (T2_COLS / 4) : 0; }

template <typename TI>
static int ttm2_run(const Ttm2Params& P, bool vec, hipStream_t s) {
    const int lds = ttm2_lds_bytes(std::is_same<TI, double>::value ? TLIB_F64 : TLIB_F32, P.m_f, P.n_f, P.n_g, vec);
    const unsigned grid = unsigned((P.ncol + T2_COLS - 1) / T2_COLS);
    constexpr int VPR = T2_COLS / (16 / int(sizeof(TI)));
    const int kfp = (P.n_f + 3) & ~3;
#define TLIB_T2(FMB_, VEC_, NV_) hipLaunchKernelGGL((ttm2_kernel<TI, FMB_, VEC_, NV_>), dim3(grid), dim3(256), lds, s, P)
    bool launched = false;
    if constexpr (sizeof(TI) == 4) {  // FP64 slabs would spill registers
        if (vec) {
            const bool small = kfp * VPR <= 64 * 12;
            if (P.m_f <= 16) { if (small) TLIB_T2(1, true, 12); else TLIB_T2(1, true, 16); }
            else { if (small) TLIB_T2(2, true, 12); else TLIB_T2(2, true, 16); }
            launched = true;
        }
    }
    if (!launched) {
        if (P.m_f <= 16) TLIB_T2(1, false, 1);
        else TLIB_T2(2, false, 1);
    }
#undef TLIB_T2
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

int launch_ttm2(int dtype, const Ttm2Params& P, bool vec, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return ttm2_run<double>(P, vec, s);
        case TLIB_F32: return ttm2_run<float>(P, vec, s);
    }
    return TLIB_EDTYPE;
}

}  // namespace tlib
