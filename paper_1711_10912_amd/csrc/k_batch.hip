// Grouped launch for many small TTV / TTM / TTT requests (Sec. 5.2 Eq. ttv,
// ttm, ttt).
//
// The host plans a batch into a work table in device memory: a header and one
// item per request.  Every item is the contraction C[m, n] = sum_k X[m, k]
// Y[k, n] with its three index groups (M, N, K) addressed through up to four
// (extent, stride) pairs each, plus a prefix sum of work units.  One
// persistent kernel with fixed arguments walks the table, so the same launch
// can be captured once in a HIP graph and replayed for every batch after the
// table's contents change.
//
// Two kinds of unit.  TTV items (M = 1): 256 outputs, one per thread, each a
// dot product over K with lanes along the operand's fastest output dim.
// TTM and TTT items: a 16 x 64 tile of C on matrix cores -- each of the four
// waves owns a 16 x 16 block and feeds v_mfma_f64_16x16x4 /
// v_mfma_f32_16x16x4 / v_mfma_f32_16x16x32_{bf16,f16} straight from global
// memory (the operands of a small request sit in cache), with the K offsets
// of 64 k at a time decoded once into LDS.  A unit's arithmetic depends only
// on its item, so a request's result is the same in any batch.
#include <algorithm>

#include "device.hpp"

namespace tlib {

namespace {

typedef double bd4_t __attribute__((ext_vector_type(4)));
typedef float bf4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bbf8_t __attribute__((ext_vector_type(8)));
typedef _Float16 bh8_t __attribute__((ext_vector_type(8)));
typedef uint32_t bu4_t __attribute__((ext_vector_type(4)));

constexpr int BT_M = 16, BT_N = 64, BT_KC = 64;

// Loads outside an operand read this zero word (the address is selected, the
// load itself stays unconditional).
__device__ __align__(16) double g_batch_zero[2] = {0.0, 0.0};

struct BatchLds {
    int64_t xrow[BT_M], crow[BT_M], ycol[BT_N], ccol[BT_N];
    int64_t kx[BT_KC], ky[BT_KC];
};

__device__ __forceinline__ bd4_t bmfma(double a, double b, bd4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf4_t bmfma(float a, float b, bf4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename TI>
__device__ __forceinline__ void batch_scalar(const BatchItem& it, int64_t u) {
    using TA = typename AccOf<TI>::type;
    const int64_t o = u * 256 + threadIdx.x;
    if (o >= it.N) return;
    int64_t oy, oc;
    grp_decode(uint32_t(o), it.gn, oy, oc);
    const TI* X = (const TI*)it.X;
    const TI* Y = (const TI*)it.Y + oy;
    const int64_t sx = it.gk.nd ? it.gk.s0[0] : 0, sy = it.gk.nd ? it.gk.s1[0] : 0;
    TA acc = TA(0);
    for (int64_t k = 0; k < it.K; ++k) acc += to_acc(X[k * sx]) * to_acc(Y[k * sy]);
    ((TA*)it.C)[oc] = acc;
}

template <typename TI>
__device__ __forceinline__ void batch_tile(const BatchItem& it, int64_t u, BatchLds& L) {
    using TA = typename AccOf<TI>::type;
    constexpr bool WIDE = sizeof(TI) == 2;
    constexpr int KSTEP = WIDE ? 32 : 4;
    using acc_t = typename std::conditional<(sizeof(TI) == 8), bd4_t, bf4_t>::type;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rl = lane & 15, kq = lane >> 4;
    const int64_t tm = u / it.tiles_n, tn = u - tm * it.tiles_n;
    const int64_t m0 = tm * BT_M, n0 = tn * BT_N;
    if (tid < BT_M) {
        int64_t a = -1, c = -1;
        if (m0 + tid < it.M) grp_decode(uint32_t(m0 + tid), it.gm, a, c);
        L.xrow[tid] = a;
        L.crow[tid] = c;
    } else if (tid >= 64 && tid < 64 + BT_N) {
        const int t = tid - 64;
        int64_t a = -1, c = -1;
        if (n0 + t < it.N) grp_decode(uint32_t(n0 + t), it.gn, a, c);
        L.ycol[t] = a;
        L.ccol[t] = c;
    }
    const TI* X = (const TI*)it.X;
    const TI* Y = (const TI*)it.Y;
    const TI* zsrc = reinterpret_cast<const TI*>(g_batch_zero);
    acc_t acc = acc_t{};
    for (int64_t kc0 = 0; kc0 < it.K; kc0 += BT_KC) {
        __syncthreads();  // row/column tables written; the previous chunk's offsets read
        if (tid < BT_KC) {
            int64_t a = -1, b = -1;
            if (kc0 + tid < it.K) grp_decode(uint32_t(kc0 + tid), it.gk, a, b);
            L.kx[tid] = a;
            L.ky[tid] = b;
        }
        __syncthreads();
        const int64_t xr = L.xrow[rl], yc = L.ycol[wave * 16 + rl];
        const int klen = it.K - kc0 < BT_KC ? int(it.K - kc0) : BT_KC;
        for (int ks = 0; ks < klen; ks += KSTEP) {
            if constexpr (WIDE) {
                uint32_t av[4], bv[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k0 = ks + 8 * kq + 2 * t;
                    const int i0 = k0 < BT_KC ? k0 : BT_KC - 1, i1 = k0 + 1 < BT_KC ? k0 + 1 : BT_KC - 1;
                    const int64_t x0 = L.kx[i0], x1 = L.kx[i1], y0 = L.ky[i0], y1 = L.ky[i1];
                    const bool ok0 = k0 < klen, ok1 = k0 + 1 < klen;
                    const uint16_t a0 = *reinterpret_cast<const uint16_t*>((ok0 && xr >= 0 && x0 >= 0) ? X + (xr + x0) : zsrc);
                    const uint16_t a1 = *reinterpret_cast<const uint16_t*>((ok1 && xr >= 0 && x1 >= 0) ? X + (xr + x1) : zsrc);
                    const uint16_t b0 = *reinterpret_cast<const uint16_t*>((ok0 && yc >= 0 && y0 >= 0) ? Y + (yc + y0) : zsrc);
                    const uint16_t b1 = *reinterpret_cast<const uint16_t*>((ok1 && yc >= 0 && y1 >= 0) ? Y + (yc + y1) : zsrc);
                    av[t] = uint32_t(a0) | (uint32_t(a1) << 16);
                    bv[t] = uint32_t(b0) | (uint32_t(b1) << 16);
                }
                const bu4_t a4 = {av[0], av[1], av[2], av[3]}, b4 = {bv[0], bv[1], bv[2], bv[3]};
                if constexpr (std::is_same<TI, bf16_t>::value)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bbf8_t, a4),
                                                                  __builtin_bit_cast(bbf8_t, b4), acc, 0, 0, 0);
                else
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(bh8_t, a4),
                                                                 __builtin_bit_cast(bh8_t, b4), acc, 0, 0, 0);
            } else {
                const int k = ks + kq;
                const int kk = k < BT_KC ? k : BT_KC - 1;
                const int64_t xk = L.kx[kk], yk = L.ky[kk];
                const bool ok = k < klen;
                const TI a = *((ok && xr >= 0 && xk >= 0) ? X + (xr + xk) : zsrc);
                const TI b = *((ok && yc >= 0 && yk >= 0) ? Y + (yc + yk) : zsrc);
                acc = bmfma(a, b, acc);
            }
        }
    }
    // result rows: 4 kq + r for the FP32-accumulating MFMAs, kq + 4 r for FP64
    constexpr int RQ = sizeof(TI) == 8 ? 1 : 4, RR = sizeof(TI) == 8 ? 4 : 1;
    const int64_t cc = L.ccol[wave * 16 + rl];
    TA* C = (TA*)it.C;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t cr = L.crow[RQ * kq + RR * r];
        if (cr >= 0 && cc >= 0) C[cr + cc] = acc[r];
    }
    __syncthreads();  // the tables are rewritten by the next unit
}

}  // namespace

__global__ __launch_bounds__(256) void batch_kernel(const BatchHeader* hdr, const BatchItem* items) {
    __shared__ BatchLds L;
    __shared__ int s_item;
    const int n = hdr->n_items;
    const int64_t total = hdr->total_units;
    for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
        if (threadIdx.x == 0) {
            // last item whose first unit is <= u
            int lo = 0, hi = n - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (items[mid].unit_begin <= u) lo = mid;
                else hi = mid - 1;
            }
            s_item = lo;
        }
        __syncthreads();
        const BatchItem& it = items[s_item];
        const int64_t lu = u - it.unit_begin;
        if (it.kind == BATCH_TILE) {
            switch (it.dtype) {
                case TLIB_F64: batch_tile<double>(it, lu, L); break;
                case TLIB_F32: batch_tile<float>(it, lu, L); break;
                case TLIB_BF16: batch_tile<bf16_t>(it, lu, L); break;
                case TLIB_F16: batch_tile<f16_t>(it, lu, L); break;
            }
        } else {
            switch (it.dtype) {
                case TLIB_F64: batch_scalar<double>(it, lu); break;
                case TLIB_F32: batch_scalar<float>(it, lu); break;
                case TLIB_BF16: batch_scalar<bf16_t>(it, lu); break;
                case TLIB_F16: batch_scalar<f16_t>(it, lu); break;
            }
        }
        __syncthreads();
    }
}

int launch_batch(const void* table_dev, int grid, hipStream_t s) {
    const BatchHeader* hdr = (const BatchHeader*)table_dev;
    const BatchItem* items = (const BatchItem*)((const char*)table_dev + sizeof(BatchHeader));
    hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(256), 0, s, hdr, items);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

}  // namespace tlib
