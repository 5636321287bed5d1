// Tensor-times-vector kernels (Sec. 5.2 Eq. ttv) on the collapsed form
//   C(lo, hi) = sum_k A(lo, k, hi) * b(k),
// where lo gathers the output modes whose A-stride is below the contracted
// mode's and hi the ones above.  TTV streams A once and is HBM-bound, so the
// kernels are organised around coalesced reads of A:
//   col   (n_lo >= 64, or >= 32 without contiguous slabs): lanes run along lo (unit stride), the four waves of a
//         workgroup take interleaved k and are summed through LDS in a fixed
//         order; optional grid split over k with a second summing pass.  The
//         hi index is decoded over up to four dims, so views whose outer dims
//         do not merge (ranges, steps) stay on this kernel.
//         With a short k (and no grid split) each wave owns a whole
//         (lo tile, hi) unit instead and keeps all of its rows in flight.
//   slab  (n_lo < 64 and the (lo,k) slabs contiguous): a workgroup copies whole
//         contiguous slabs (and b, when short) into LDS with coalesced loads,
//         then groups of G lanes reduce each output's k-fiber out of LDS with a
//         shuffle tree.
//   fiber (n_lo < 32, slabs not contiguous: views; and n_lo = 1 with k of
//         unit stride and n_k >= 32, where every output is one contiguous
//         fiber): G lanes per output stream its k-fiber (coalesced when k has
//         unit stride) and reduce with a fixed shuffle tree; outputs decoded
//         over up to four dims.
//   generic: one thread per output, any strides.
// Accumulation is in FP64 for FP64 inputs and in FP32 otherwise.
#include <algorithm>

#include "device.hpp"

namespace tlib {

template <typename TI, int VEC>
__device__ __forceinline__ void load_vec(const TI* p, typename AccOf<TI>::type (&out)[VEC]) {
    if constexpr (VEC == 1) {
        out[0] = to_acc(p[0]);
    } else {
        struct alignas(sizeof(TI) * VEC) V {
            TI v[VEC];
        };
        V t = *reinterpret_cast<const V*>(p);
#pragma unroll
        for (int i = 0; i < VEC; ++i) out[i] = to_acc(t.v[i]);
    }
}

template <typename TI, int VEC>
__global__ __launch_bounds__(256) void ttv_col_kernel(TtvParams P, int64_t lo_tiles, int64_t kchunk,
                                                      typename AccOf<TI>::type* part) {
    using TA = typename AccOf<TI>::type;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t bid = blockIdx.x;
    const int64_t lt = bid % lo_tiles;
    bid /= lo_tiles;
    const int64_t hi = bid % P.n_hi;
    const int64_t ks = bid / P.n_hi;
    const int64_t lo0 = (lt * 64 + lane) * VEC;
    const int64_t kb = ks * kchunk;
    const int64_t ke = min(P.n_k, kb + kchunk);
    const bool active = lo0 < P.n_lo;
    int64_t hA, hC;
    grp_decode(uint32_t(hi), P.gh, hA, hC);

    TA acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = TA(0);
    if (active) {
        const TI* Ap = (const TI*)P.A + hA + lo0 * P.sA_lo;
        const TI* b = (const TI*)P.b;
        int64_t k = kb + wave;
        // four rows per wave per step; the next step's rows are loaded before
        // this step's are added, so eight are in flight
        auto load4 = [&](int64_t k0, TA (&x)[4][VEC], TA (&bk)[4]) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if constexpr (VEC > 1) load_vec<TI, VEC>(Ap + (k0 + 4 * r) * P.sA_k, x[r]);
                else x[r][0] = to_acc(Ap[(k0 + 4 * r) * P.sA_k]);
                bk[r] = to_acc(b[(k0 + 4 * r) * P.sb]);
            }
        };
        if (k + 12 < ke) {
            TA x[4][VEC], bx[4];
            load4(k, x, bx);
            for (; k + 28 < ke; k += 16) {
                TA y[4][VEC], by[4];
                load4(k + 16, y, by);
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) acc[v] += x[r][v] * bx[r];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    bx[r] = by[r];
#pragma unroll
                    for (int v = 0; v < VEC; ++v) x[r][v] = y[r][v];
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[v] += x[r][v] * bx[r];
            k += 16;
        }
        for (; k < ke; k += 4) {
            TA x0[VEC];
            if constexpr (VEC > 1) load_vec<TI, VEC>(Ap + k * P.sA_k, x0);
            else x0[0] = to_acc(Ap[k * P.sA_k]);
            const TA b0 = to_acc(b[k * P.sb]);
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] += x0[v] * b0;
        }
    }
    __shared__ TA red[4][64 * VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) red[wave][lane * VEC + v] = acc[v];
    __syncthreads();
    if (wave == 0 && active) {
        TA* C = (TA*)P.C;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int j = lane * VEC + v;
            const TA s = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
            const int64_t lo = lo0 + v;
            if (part) part[ks * (P.n_lo * P.n_hi) + hi * P.n_lo + lo] = s;
            else C[lo * P.sC_lo + hC] = s;
        }
    }
}

// Col kernel for a short contraction (n_k <= KR): each wave owns one
// (lo tile, hi) unit and keeps all of its k rows in flight at once (rows past
// n_k load from a zero word), so a unit costs one memory round trip and no
// workgroup barrier.  Each lane adds its rows in k order.
__device__ __align__(16) double g_ttv_zero[2] = {0.0, 0.0};

template <typename TI, int VEC, int KR>
__global__ __launch_bounds__(256) void ttv_colw_kernel(TtvParams P, int64_t lo_tiles, int64_t units) {
    using TA = typename AccOf<TI>::type;
    const int lane = threadIdx.x & 63;
    const int64_t u = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (u >= units) return;
    const int64_t hi = u / lo_tiles, lt = u - hi * lo_tiles;
    const int64_t lo0 = (lt * 64 + lane) * VEC;
    if (lo0 >= P.n_lo) return;
    int64_t hA, hC;
    grp_decode(uint32_t(hi), P.gh, hA, hC);
    const TI* Ap = (const TI*)P.A + hA + lo0 * P.sA_lo;
    const TI* b = (const TI*)P.b;
    const TI* zs = reinterpret_cast<const TI*>(g_ttv_zero);
    TA acc[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] = TA(0);
    for (int64_t k0 = 0; k0 < P.n_k; k0 += KR) {
        TA x[KR][VEC], bk[KR];
#pragma unroll
        for (int r = 0; r < KR; ++r) {
            const int64_t k = k0 + r;
            const bool in = k < P.n_k;
            load_vec<TI, VEC>(in ? Ap + k * P.sA_k : zs, x[r]);
            bk[r] = to_acc(*(in ? b + k * P.sb : zs));
        }
#pragma unroll
        for (int r = 0; r < KR; ++r)
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] += x[r][v] * bk[r];
    }
    TA* C = (TA*)P.C;
#pragma unroll
    for (int v = 0; v < VEC; ++v) C[(lo0 + v) * P.sC_lo + hC] = acc[v];
}

template <typename TA>
__global__ __launch_bounds__(256) void ttv_ksum_kernel(TtvParams P, int ksplit, const TA* part) {
    const int64_t outs = P.n_lo * P.n_hi;
    for (int64_t o = int64_t(blockIdx.x) * 256 + threadIdx.x; o < outs; o += int64_t(gridDim.x) * 256) {
        TA s = part[o];
        for (int k = 1; k < ksplit; ++k) s += part[int64_t(k) * outs + o];
        const int64_t lo = o % P.n_lo, hi = o / P.n_lo;
        ((TA*)P.C)[lo * P.sC_lo + grp_off1(uint32_t(hi), P.gh)] = s;
    }
}

// LDS holds `slabs` consecutive (lo,k)-slabs, restricted to k rows [k0, k0+kc).
// bl: whole slabs (kc >= n_k) and b staged in LDS behind them (16-byte
// aligned), so that the dot loops read both operands from LDS.
template <typename TI>
__global__ __launch_bounds__(256) void ttv_slab_kernel(TtvParams P, int slabs, int kc, int bl) {
    using TA = typename AccOf<TI>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    TI* L = reinterpret_cast<TI*>(smem_raw);
    const int tid = threadIdx.x;
    const int n_lo = int(P.n_lo);
    const int64_t n_k = P.n_k;
    const int64_t h0 = int64_t(blockIdx.x) * slabs;
    const int nS = int(min(int64_t(slabs), P.n_hi - h0));
    const int O = nS * n_lo;
    int G = 1;
    while (G < 64 && 2 * G * O <= 256) G *= 2;
    const TI* A = (const TI*)P.A;
    const TI* b = (const TI*)P.b;
    TA* C = (TA*)P.C;
    const int64_t slab = int64_t(n_lo) * n_k;

    if (kc >= n_k) {
        // whole slabs: one contiguous run of nS*slab elements, copied with
        // 16-byte loads (four in flight per thread) when the run is aligned
        const TI* src = A + h0 * slab;
        const int total = int(int64_t(nS) * slab);
        int i0 = 0;
        if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
            typedef uint32_t q4_t __attribute__((ext_vector_type(4)));
            constexpr int PER = 16 / int(sizeof(TI));
            const int nq = total / PER;
            const q4_t* sq = reinterpret_cast<const q4_t*>(src);
            q4_t* lq = reinterpret_cast<q4_t*>(L);
            int q = tid;
            for (; q + 768 < nq; q += 1024) {
                const q4_t v0 = sq[q], v1 = sq[q + 256], v2 = sq[q + 512], v3 = sq[q + 768];
                lq[q] = v0;
                lq[q + 256] = v1;
                lq[q + 512] = v2;
                lq[q + 768] = v3;
            }
            for (; q < nq; q += 256) lq[q] = sq[q];
            i0 = nq * PER;
        }
        int i = i0 + tid;
        for (; i + 768 < total; i += 1024) {
            TI v0 = src[i], v1 = src[i + 256], v2 = src[i + 512], v3 = src[i + 768];
            L[i] = v0;
            L[i + 256] = v1;
            L[i + 512] = v2;
            L[i + 768] = v3;
        }
        for (; i < total; i += 256) L[i] = src[i];
        TI* Lb = reinterpret_cast<TI*>(smem_raw + ((size_t(slabs) * size_t(slab) * sizeof(TI) + 15) & ~size_t(15)));
        if (bl)
            for (int e = tid; e < int(n_k); e += 256) Lb[e] = b[int64_t(e) * P.sb];
        __syncthreads();
        for (int base = 0; base < O * G; base += 256) {
            const int t = base + tid;
            const int o = t / G, g = t % G;
            TA acc = TA(0);
            if (o < O) {
                const int hl = o / n_lo, lo = o - hl * n_lo;
                const TI* Ls = L + int64_t(hl) * slab + lo;
                if (bl) {
                    const int nk = int(n_k);
#pragma unroll 4
                    for (int k = g; k < nk; k += G) acc += to_acc(Ls[k * n_lo]) * to_acc(Lb[k]);
                } else {
                    for (int64_t k = g; k < n_k; k += G) acc += to_acc(Ls[k * n_lo]) * to_acc(b[k * P.sb]);
                }
            }
            if (G > 1) acc = warp_sum(acc, G);
            if (o < O && g == 0) {
                const int hl = o / n_lo, lo = o - hl * n_lo;
                C[int64_t(lo) * P.sC_lo + (h0 + hl) * P.sC_hi] = acc;
            }
        }
    } else {
        // one slab (nS == 1) taken kc rows at a time; O = n_lo < 64 so O*G <= 256
        const int o = tid / G, g = tid % G;
        TA acc = TA(0);
        const TI* src0 = A + h0 * slab;
        for (int64_t k0 = 0; k0 < n_k; k0 += kc) {
            const int kn = int(min(int64_t(kc), n_k - k0));
            const int total = kn * n_lo;
            __syncthreads();
            for (int i = tid; i < total; i += 256) L[i] = src0[k0 * n_lo + i];
            __syncthreads();
            if (o < O)
                for (int k = g; k < kn; k += G) acc += to_acc(L[k * n_lo + o]) * to_acc(b[(k0 + k) * P.sb]);
        }
        if (G > 1) acc = warp_sum(acc, G);
        if (o < O && g == 0) C[int64_t(o) * P.sC_lo + h0 * P.sC_hi] = acc;
    }
}

__device__ uint64_t g_fiber_zero[2];

// G lanes per output fiber, J elements per lane per pass, RU outputs per group
// in flight (RU*J loads outstanding per lane).  Each lane sums its elements in
// k order; the group then reduces by shuffles.
template <typename TI, int J, int RU>
__global__ __launch_bounds__(256) void ttv_fiber_kernel(TtvParams P, Grp go, int G, int64_t outs) {
    using TA = typename AccOf<TI>::type;
    const TI* A = (const TI*)P.A;
    const TI* b = (const TI*)P.b;
    TA* C = (TA*)P.C;
    const TI* zs = reinterpret_cast<const TI*>(g_fiber_zero);
    const int g = threadIdx.x % G;
    const int64_t per = 256 / G * RU;
    // the outer loop runs the same rounds for every thread of the block
    // (outputs past the end take no elements), so every shuffle sees all
    // lanes of its group
    for (int64_t o0 = int64_t(blockIdx.x) * per; o0 < outs; o0 += int64_t(gridDim.x) * per) {
        const int64_t ob = o0 + int64_t(threadIdx.x / G) * RU;
        const TI* a[RU];
        int64_t oc[RU];
        bool ok[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            ok[u] = ob + u < outs;
            int64_t oa;
            grp_decode(uint32_t(ok[u] ? ob + u : 0), go, oa, oc[u]);
            a[u] = A + oa;
        }
        TA acc[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) acc[u] = TA(0);
        for (int64_t k = g; k < P.n_k; k += int64_t(J) * G) {
            TI xa[RU][J], xb[J];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int64_t kj = k + int64_t(j) * G;
                xb[j] = *(kj < P.n_k ? b + kj * P.sb : zs);
#pragma unroll
                for (int u = 0; u < RU; ++u) xa[u][j] = *(ok[u] && kj < P.n_k ? a[u] + kj * P.sA_k : zs);
            }
#pragma unroll
            for (int u = 0; u < RU; ++u)
#pragma unroll
                for (int j = 0; j < J; ++j) acc[u] += to_acc(xa[u][j]) * to_acc(xb[j]);
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const TA v = warp_sum(acc[u], G);
            if (ok[u] && g == 0) C[oc[u]] = v;
        }
    }
}

template <typename TI>
__global__ __launch_bounds__(256) void ttv_generic_kernel(TtvParams P, GDims g) {
    using TA = typename AccOf<TI>::type;
    const TI* A = (const TI*)P.A;
    const TI* b = (const TI*)P.b;
    TA* C = (TA*)P.C;
    for (int64_t o = int64_t(blockIdx.x) * 256 + threadIdx.x; o < g.total; o += int64_t(gridDim.x) * 256) {
        int64_t off[2];
        gd_decode(o, g, 2, off);
        TA acc = TA(0);
        for (int64_t k = 0; k < P.n_k; ++k) acc += to_acc(A[off[0] + k * P.sA_k]) * to_acc(b[k * P.sb]);
        C[off[1]] = acc;
    }
}

// ------------------------------------------------------------------ launchers

template <typename TI, int VEC>
static int col_launch(const TtvParams& p, int ksplit, void* ws, hipStream_t s) {
    using TA = typename AccOf<TI>::type;
    const int64_t lo_tiles = (p.n_lo + 64 * VEC - 1) / (64 * VEC);
    const int64_t kchunk = (p.n_k + ksplit - 1) / ksplit;
    const int64_t blocks = lo_tiles * p.n_hi * ksplit;
    TA* part = ksplit > 1 ? (TA*)ws : nullptr;
    hipLaunchKernelGGL((ttv_col_kernel<TI, VEC>), dim3(unsigned(blocks)), dim3(256), 0, s, p, lo_tiles,
                       kchunk, part);
    if (hipGetLastError() != hipSuccess) return TLIB_EHIP;
    if (ksplit > 1) {
        const int64_t outs = p.n_lo * p.n_hi;
        const unsigned g = unsigned(std::min<int64_t>((outs + 255) / 256, 65536));
        hipLaunchKernelGGL((ttv_ksum_kernel<TA>), dim3(g), dim3(256), 0, s, p, ksplit, part);
        if (hipGetLastError() != hipSuccess) return TLIB_EHIP;
    }
    return TLIB_OK;
}

template <typename TI, int VEC, int KR>
static int colw_launch(const TtvParams& p, hipStream_t s) {
    if constexpr (KR * VEC * int(sizeof(TI)) > 256) {
        return TLIB_EINVAL;
    } else {
        const int64_t lo_tiles = (p.n_lo + 64 * VEC - 1) / (64 * VEC);
        const int64_t units = lo_tiles * p.n_hi;
        const int64_t blocks = (units + 3) / 4;
        hipLaunchKernelGGL((ttv_colw_kernel<TI, VEC, KR>), dim3(unsigned(blocks)), dim3(256), 0, s, p, lo_tiles,
                           units);
        return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
    }
}

template <typename TI, int VEC>
static int colw_kr(const TtvParams& p, int kr, hipStream_t s) {
    switch (kr) {
        case 8: return colw_launch<TI, VEC, 8>(p, s);
        case 16: return colw_launch<TI, VEC, 16>(p, s);
        case 32: return colw_launch<TI, VEC, 32>(p, s);
        case 64: return colw_launch<TI, VEC, 64>(p, s);
    }
    return TLIB_EINVAL;
}

template <typename TI>
static int col_dispatch(const TtvParams& p, int vec, int ksplit, void* ws, hipStream_t s) {
    constexpr int MAXV = 16 / sizeof(TI);
    if (vec >= 8 && MAXV >= 8) return col_launch<TI, (MAXV >= 8 ? 8 : 1)>(p, ksplit, ws, s);
    if (vec >= 4 && MAXV >= 4) return col_launch<TI, (MAXV >= 4 ? 4 : 1)>(p, ksplit, ws, s);
    if (vec >= 2) return col_launch<TI, 2>(p, ksplit, ws, s);
    return col_launch<TI, 1>(p, ksplit, ws, s);
}

template <typename TI>
static int colw_dispatch(const TtvParams& p, int vec, int kr, hipStream_t s) {
    constexpr int MAXV = 16 / sizeof(TI);
    if (vec >= 8 && MAXV >= 8) return colw_kr<TI, (MAXV >= 8 ? 8 : 1)>(p, kr, s);
    if (vec >= 4 && MAXV >= 4) return colw_kr<TI, (MAXV >= 4 ? 4 : 1)>(p, kr, s);
    if (vec >= 2) return colw_kr<TI, 2>(p, kr, s);
    return colw_kr<TI, 1>(p, kr, s);
}

int launch_ttv_colw(int dtype, const TtvParams& p, int vec, int kr, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return colw_dispatch<double>(p, vec, kr, s);
        case TLIB_F32: return colw_dispatch<float>(p, vec, kr, s);
        case TLIB_BF16: return colw_dispatch<bf16_t>(p, vec, kr, s);
        case TLIB_F16: return colw_dispatch<f16_t>(p, vec, kr, s);
    }
    return TLIB_EDTYPE;
}

int launch_ttv_col(int dtype, const TtvParams& p, int vec, int ksplit, void* ws, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return col_dispatch<double>(p, vec, ksplit, ws, s);
        case TLIB_F32: return col_dispatch<float>(p, vec, ksplit, ws, s);
        case TLIB_BF16: return col_dispatch<bf16_t>(p, vec, ksplit, ws, s);
        case TLIB_F16: return col_dispatch<f16_t>(p, vec, ksplit, ws, s);
    }
    return TLIB_EDTYPE;
}

template <typename TI>
static int slab_launch(const TtvParams& p, int slabs, int kc, hipStream_t s) {
    const int64_t blocks = (p.n_hi + slabs - 1) / slabs;
    const int64_t rows = kc >= p.n_k ? p.n_k : kc;
    size_t lds = size_t(slabs) * size_t(rows) * size_t(p.n_lo) * sizeof(TI);
    // b joins the slabs in LDS when they are whole and it is small
    const int bl = kc >= p.n_k && p.n_k * int64_t(sizeof(TI)) <= 4096 ? 1 : 0;
    if (bl) lds = ((lds + 15) & ~size_t(15)) + size_t(p.n_k) * sizeof(TI);
    hipLaunchKernelGGL((ttv_slab_kernel<TI>), dim3(unsigned(blocks)), dim3(256), lds, s, p, slabs, kc, bl);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

int launch_ttv_slab(int dtype, const TtvParams& p, int slabs, int kc, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return slab_launch<double>(p, slabs, kc, s);
        case TLIB_F32: return slab_launch<float>(p, slabs, kc, s);
        case TLIB_BF16: return slab_launch<bf16_t>(p, slabs, kc, s);
        case TLIB_F16: return slab_launch<f16_t>(p, slabs, kc, s);
    }
    return TLIB_EDTYPE;
}

template <typename TI>
static int fiber_launch(const TtvParams& p, const Grp& go, int G, hipStream_t s) {
    const int64_t outs = go.total;
    const int64_t J = std::min<int64_t>(4, (p.n_k + G - 1) / G);
    const int RU = J <= 2 ? 8 : 4;
    const int64_t per = 256 / G * RU;
    const unsigned blocks = unsigned(std::max<int64_t>(1, std::min<int64_t>((outs + per - 1) / per, 8192)));
    if (J == 1)
        hipLaunchKernelGGL((ttv_fiber_kernel<TI, 1, 8>), dim3(blocks), dim3(256), 0, s, p, go, G, outs);
    else if (J == 2)
        hipLaunchKernelGGL((ttv_fiber_kernel<TI, 2, 8>), dim3(blocks), dim3(256), 0, s, p, go, G, outs);
    else if (J == 3)
        hipLaunchKernelGGL((ttv_fiber_kernel<TI, 3, 4>), dim3(blocks), dim3(256), 0, s, p, go, G, outs);
    else
        hipLaunchKernelGGL((ttv_fiber_kernel<TI, 4, 4>), dim3(blocks), dim3(256), 0, s, p, go, G, outs);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

int launch_ttv_fiber(int dtype, const TtvParams& p, const Grp& go, int G, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return fiber_launch<double>(p, go, G, s);
        case TLIB_F32: return fiber_launch<float>(p, go, G, s);
        case TLIB_BF16: return fiber_launch<bf16_t>(p, go, G, s);
        case TLIB_F16: return fiber_launch<f16_t>(p, go, G, s);
    }
    return TLIB_EDTYPE;
}

template <typename TI>
static int generic_launch(const TtvParams& p, const GDims& g, hipStream_t s) {
    const unsigned blocks = unsigned(std::max<int64_t>(1, std::min<int64_t>((g.total + 255) / 256, 65536)));
    hipLaunchKernelGGL((ttv_generic_kernel<TI>), dim3(blocks), dim3(256), 0, s, p, g);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

int launch_ttv_generic(int dtype, const TtvParams& p, const GDims& g, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return generic_launch<double>(p, g, s);
        case TLIB_F32: return generic_launch<float>(p, g, s);
        case TLIB_BF16: return generic_launch<bf16_t>(p, g, s);
        case TLIB_F16: return generic_launch<f16_t>(p, g, s);
    }
    return TLIB_EDTYPE;
}

}  // namespace tlib
