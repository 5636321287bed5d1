// Streaming kernels: inner product / Frobenius norm (Sec. 5.2 Table 3) and
// entrywise C = alpha A + beta B (Sec. 5.1 Eq. scaling, Eq. transform), which
// also serves relayout and transposition (a permuted stride tuple for A).
//
// inner/norm: two passes with a fixed partition (a block per contiguous range
// of the collapsed iteration space, or per range of rows of the innermost dim
// when the dims of a view do not merge, a fixed shuffle/LDS tree inside the
// block, then one block summing the partials in index order), so the FP64
// result only depends on the shapes and strides, never on scheduling.
#include <algorithm>

#include "device.hpp"

namespace tlib {

constexpr int DOT_BLOCK = 256;

int dot_partials(int64_t total) {
    int64_t np = (total + 65535) / 65536;
    if (np < 1) np = 1;
    if (np > 2048) np = 2048;
    return int(np);
}

// Views whose dims do not merge go by rows (below); they take at least one
// workgroup per 256 rows, up to 2048, so that a short row's load latency is
// spread over enough waves (f64 sliced / trimmed 90^4 views 8-11 % faster
// than with the flat count).
static bool dot_by_rows(const GDims& g) { return g.nd >= 2 && g.total / g.n[0] < (int64_t(1) << 31); }
int dot_partials_g(const GDims& g) {
    int64_t np = dot_partials(g.total);
    if (dot_by_rows(g)) np = std::max<int64_t>(np, std::min<int64_t>(2048, (g.total / g.n[0] + 255) / 256));
    return int(np);
}

// CT = 1 (norm) / 2 (inner): one dim of unit stride in every operand, read
// with unit-stride addresses and 32 bytes per lane in flight; same summation
// order as the strided flat walk.
template <typename TI, int CT>
__global__ __launch_bounds__(DOT_BLOCK) void dot_pass1(const TI* A, const TI* B, GDims g, int64_t chunk,
                                                       double* part) {
    const int tid = threadIdx.x;
    const int64_t beg = int64_t(blockIdx.x) * chunk;
    const int64_t end = min(g.total, beg + chunk);
    // one dim (any strides): a strided flat walk
    const bool flat = g.nd <= 1;
    const int64_t sa = g.nd == 1 ? g.s[0][0] : 0, sb = g.nd == 1 ? g.s[1][0] : 0;
    double acc = 0.0;
    if constexpr (CT > 0) {
        constexpr int U = sizeof(TI) >= 8 ? 4 : sizeof(TI) == 4 ? 8 : 16;
        int64_t i = beg + tid;
        for (; i + (U - 1) * DOT_BLOCK < end; i += U * DOT_BLOCK) {
            TI xa[U], xb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                xa[u] = A[i + u * DOT_BLOCK];
                if constexpr (CT == 2) xb[u] = B[i + u * DOT_BLOCK];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double x = to_f64(xa[u]);
                acc += x * (CT == 2 ? to_f64(xb[u]) : x);
            }
        }
        for (; i < end; i += DOT_BLOCK) {
            const double x = to_f64(A[i]);
            acc += x * (CT == 2 ? to_f64(B[i]) : x);
        }
    } else if (flat) {
        int64_t i = beg + tid;
        for (; i + 3 * DOT_BLOCK < end; i += 4 * DOT_BLOCK) {
            const double a0 = to_f64(A[i * sa]), a1 = to_f64(A[(i + DOT_BLOCK) * sa]);
            const double a2 = to_f64(A[(i + 2 * DOT_BLOCK) * sa]), a3 = to_f64(A[(i + 3 * DOT_BLOCK) * sa]);
            if (B) {
                acc += a0 * to_f64(B[i * sb]);
                acc += a1 * to_f64(B[(i + DOT_BLOCK) * sb]);
                acc += a2 * to_f64(B[(i + 2 * DOT_BLOCK) * sb]);
                acc += a3 * to_f64(B[(i + 3 * DOT_BLOCK) * sb]);
            } else {
                acc += a0 * a0;
                acc += a1 * a1;
                acc += a2 * a2;
                acc += a3 * a3;
            }
        }
        for (; i < end; i += DOT_BLOCK) {
            const double a = to_f64(A[i * sa]);
            acc += a * (B ? to_f64(B[i * sb]) : a);
        }
    } else {
        for (int64_t i = beg + tid; i < end; i += DOT_BLOCK) {
            int64_t off[2];
            gd_decode(i, g, 2, off);
            const double a = to_f64(A[off[0]]);
            acc += a * (B ? to_f64(B[off[1]]) : a);
        }
    }
    acc = warp_sum(acc, 64);
    __shared__ double red[DOT_BLOCK / 64];
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Views whose dims do not merge: rows along the innermost dim (n0 elements,
// stride sa / sb), each row's offsets decoded (32-bit fast divide) over the
// other dims.  G lanes per row take J elements each per pass; a group keeps RU
// rows in flight, so that a lane has RU*J loads outstanding.  Workgroup b owns
// rows [b rpb, (b+1) rpb).  The partition and every summation order are fixed.
struct DotRowDec {
    int nr = 0;
    uint32_t n[MAXP] = {};
    FastDiv fd[MAXP];
    int64_t s0[MAXP] = {}, s1[MAXP] = {};
};

__device__ uint64_t g_dot_zero[2];

template <typename TI, int J, int RU>
__global__ __launch_bounds__(DOT_BLOCK) void dot_rows(const TI* A, const TI* B, int64_t n0, int64_t sa, int64_t sb,
                                                      DotRowDec R, uint32_t rows, uint32_t rpb, int G,
                                                      double* part) {
    const int tid = threadIdx.x;
    const int gi = tid / G, l = tid % G, per = DOT_BLOCK / G;
    const uint32_t r0 = blockIdx.x * rpb, r1 = min(rows, r0 + rpb);
    const TI* zs = reinterpret_cast<const TI*>(g_dot_zero);
    double acc = 0.0;
    for (uint32_t r = r0 + uint32_t(gi) * RU; r < r1; r += uint32_t(per) * RU) {
        const TI* a[RU];
        const TI* b[RU];
        bool lv[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            lv[u] = r + u < r1;
            uint32_t lin = lv[u] ? r + u : r;
            int64_t oa = 0, ob = 0;
#pragma unroll
            for (int d = 0; d < MAXP; ++d) {
                if (d >= R.nr) break;
                const uint32_t q = d == R.nr - 1 ? 0u : fdiv(lin, R.fd[d]);
                const int64_t i = int64_t(lin - q * R.n[d]);
                oa += i * R.s0[d];
                ob += i * R.s1[d];
                lin = q;
            }
            a[u] = A + oa;
            b[u] = B ? B + ob : zs;
        }
        for (int64_t c = l; c < n0; c += int64_t(J) * G) {
            TI xa[RU][J], xb[RU][J];
#pragma unroll
            for (int u = 0; u < RU; ++u)
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    const int64_t cj = c + int64_t(j) * G;
                    const bool in = lv[u] && cj < n0;
                    xa[u][j] = *(in ? a[u] + cj * sa : zs);
                    if (B) xb[u][j] = *(in ? b[u] + cj * sb : zs);
                }
#pragma unroll
            for (int u = 0; u < RU; ++u)
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    const double x = to_f64(xa[u][j]);
                    acc += x * (B ? to_f64(xb[u][j]) : x);
                }
        }
    }
    acc = warp_sum(acc, 64);
    __shared__ double red[DOT_BLOCK / 64];
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(DOT_BLOCK) void dot_pass2(const double* part, int np, double* out, int do_sqrt) {
    const int tid = threadIdx.x;
    double acc = 0.0;
    for (int i = tid; i < np; i += DOT_BLOCK) acc += part[i];
    acc = warp_sum(acc, 64);
    __shared__ double red[DOT_BLOCK / 64];
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        const double s = ((red[0] + red[1]) + red[2]) + red[3];
        out[0] = do_sqrt ? sqrt(s) : s;
    }
}

template <typename TI>
static int dot_launch(const void* A, const void* B, const GDims& g, double* out, bool sq, void* ws,
                      hipStream_t s) {
    int np = dot_partials_g(g);
    if (dot_by_rows(g)) {
        const int64_t rows = g.total / g.n[0];
        const int G = g.n[0] >= 256 ? 64 : g.n[0] >= 64 ? 32 : g.n[0] >= 16 ? 16 : 8;
        const int64_t rpb = (rows + np - 1) / np;
        np = int((rows + rpb - 1) / rpb);
        DotRowDec R;
        R.nr = g.nd - 1;
        for (int d = 1; d < g.nd; ++d) {
            R.n[d - 1] = uint32_t(g.n[d]);
            R.fd[d - 1] = make_fastdiv(uint32_t(g.n[d]));
            R.s0[d - 1] = g.s[0][d];
            R.s1[d - 1] = g.s[1][d];
        }
        const int64_t J = std::min<int64_t>(4, (g.n[0] + G - 1) / G);
#define TLIB_DOT_ROWS(JJ, RR)                                                                                   \
    hipLaunchKernelGGL((dot_rows<TI, JJ, RR>), dim3(np), dim3(DOT_BLOCK), 0, s, (const TI*)A, (const TI*)B, g.n[0], \
                       g.s[0][0], g.s[1][0], R, uint32_t(rows), uint32_t(rpb), G, (double*)ws)
        if (J == 1) TLIB_DOT_ROWS(1, 8);
        else if (J == 2) TLIB_DOT_ROWS(2, 8);
        else if (J == 3) TLIB_DOT_ROWS(3, 4);
        else TLIB_DOT_ROWS(4, 4);
#undef TLIB_DOT_ROWS
    } else {
        const int64_t chunk = (g.total + np - 1) / np;
        const bool unit = g.nd == 1 && g.s[0][0] == 1 && (!B || g.s[1][0] == 1);
        if (unit && B)
            hipLaunchKernelGGL((dot_pass1<TI, 2>), dim3(np), dim3(DOT_BLOCK), 0, s, (const TI*)A, (const TI*)B, g,
                               chunk, (double*)ws);
        else if (unit)
            hipLaunchKernelGGL((dot_pass1<TI, 1>), dim3(np), dim3(DOT_BLOCK), 0, s, (const TI*)A, (const TI*)B, g,
                               chunk, (double*)ws);
        else
            hipLaunchKernelGGL((dot_pass1<TI, 0>), dim3(np), dim3(DOT_BLOCK), 0, s, (const TI*)A, (const TI*)B, g,
                               chunk, (double*)ws);
    }
    if (hipGetLastError() != hipSuccess) return TLIB_EHIP;
    hipLaunchKernelGGL(dot_pass2, dim3(1), dim3(DOT_BLOCK), 0, s, (const double*)ws, np, out, sq ? 1 : 0);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

int launch_dot(int dtype, const void* A, const void* B, const GDims& d, double* out, bool sqrt_out, void* ws,
               size_t ws_bytes, hipStream_t s) {
    if (ws_bytes < size_t(dot_partials_g(d)) * sizeof(double)) return TLIB_ENOMEM;
    switch (dtype) {
        case TLIB_F64: return dot_launch<double>(A, B, d, out, sqrt_out, ws, s);
        case TLIB_F32: return dot_launch<float>(A, B, d, out, sqrt_out, ws, s);
        case TLIB_BF16: return dot_launch<bf16_t>(A, B, d, out, sqrt_out, ws, s);
        case TLIB_F16: return dot_launch<f16_t>(A, B, d, out, sqrt_out, ws, s);
    }
    return TLIB_EDTYPE;
}

// ------------------------------------------------------------------ entrywise

// Correct rounding of a double to a narrower type: round to odd into FP32
// first (keeps a sticky bit), then round to nearest even into the target.
__device__ __forceinline__ float to_f32_odd(double v) {
    float f = float(v);
    if (double(f) != v && f == f) {
        uint32_t u = __float_as_uint(f);
        if (fabs(double(f)) > fabs(v)) u -= 1;  // truncate toward zero
        u |= 1u;
        f = __uint_as_float(u);
    }
    return f;
}

template <typename TI> __device__ __forceinline__ TI round_out(double v);
template <> __device__ __forceinline__ double round_out<double>(double v) { return v; }
template <> __device__ __forceinline__ float round_out<float>(double v) { return float(v); }
template <> __device__ __forceinline__ f16_t round_out<f16_t>(double v) { return f16_t(to_f32_odd(v)); }
template <> __device__ __forceinline__ bf16_t round_out<bf16_t>(double v) {
    const float f = to_f32_odd(v);
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return bf16_t{uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u))};
    u += 0x7fffu + ((u >> 16) & 1u);
    return bf16_t{uint16_t(u >> 16)};
}

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void axpby_kernel(double alpha, const TI* A, double beta, const TI* B, TO* C,
                                                    GDims g) {
#pragma clang fp contract(off)
    const bool flat = g.nd <= 1 && g.s[0][0] == 1 && g.s[2][0] == 1 && (!B || g.s[1][0] == 1);
    const int64_t stride = int64_t(gridDim.x) * 256;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < g.total; i += stride) {
        int64_t off[3];
        if (flat) {
            off[0] = off[1] = off[2] = i;
        } else {
            gd_decode(i, g, 3, off);
        }
        double v = alpha * to_f64(A[off[0]]);
        if (B) v = v + beta * to_f64(B[off[1]]);
        C[off[2]] = round_out<TO>(v);
    }
}

// The same op on one unit-stride run with 16-byte aligned operands: V
// consecutive elements per thread and pass (16-byte accesses for the wider of
// the two types), the same arithmetic per element.
template <typename TI, typename TO, int V>
__global__ __launch_bounds__(256) void axpby_flat_kernel(double alpha, const TI* A, double beta, const TI* B, TO* C,
                                                         int64_t total) {
#pragma clang fp contract(off)
    struct alignas(sizeof(TI) * V) VI {
        TI v[V];
    };
    struct alignas(sizeof(TO) * V) VO {
        TO v[V];
    };
    const int64_t nv = total / V;
    const int64_t stride = int64_t(gridDim.x) * 256;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < nv; i += stride) {
        const VI a = reinterpret_cast<const VI*>(A)[i];
        VI b;
        if (B) b = reinterpret_cast<const VI*>(B)[i];
        VO c;
#pragma unroll
        for (int e = 0; e < V; ++e) {
            double v = alpha * to_f64(a.v[e]);
            if (B) v = v + beta * to_f64(b.v[e]);
            c.v[e] = round_out<TO>(v);
        }
        reinterpret_cast<VO*>(C)[i] = c;
    }
    // the tail (fewer than V elements) one by one
    const int64_t t = nv * V + int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (t < total) {
        double v = alpha * to_f64(A[t]);
        if (B) v = v + beta * to_f64(B[t]);
        C[t] = round_out<TO>(v);
    }
}

template <typename TI, typename TO>
static int axpby_launch(double alpha, const void* A, double beta, const void* B, void* C, const GDims& g,
                        hipStream_t s) {
    constexpr int V = 16 / int(sizeof(TI) > sizeof(TO) ? sizeof(TI) : sizeof(TO));
    const bool flat = g.nd <= 1 && g.s[0][0] == 1 && g.s[2][0] == 1 && (!B || g.s[1][0] == 1);
    const bool aligned = (uintptr_t(A) % (sizeof(TI) * V)) == 0 && (!B || (uintptr_t(B) % (sizeof(TI) * V)) == 0) &&
                         (uintptr_t(C) % (sizeof(TO) * V)) == 0;
    if (flat && aligned && g.total >= 256 * V) {
        const unsigned blocks = unsigned(std::max<int64_t>(1, std::min<int64_t>((g.total / V + 255) / 256, 8192)));
        hipLaunchKernelGGL((axpby_flat_kernel<TI, TO, V>), dim3(blocks), dim3(256), 0, s, alpha, (const TI*)A, beta,
                           (const TI*)B, (TO*)C, g.total);
        return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
    }
    const unsigned blocks = unsigned(std::max<int64_t>(1, std::min<int64_t>((g.total + 255) / 256, 8192)));
    hipLaunchKernelGGL((axpby_kernel<TI, TO>), dim3(blocks), dim3(256), 0, s, alpha, (const TI*)A, beta,
                       (const TI*)B, (TO*)C, g);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

template <typename TI>
static int axpby_out(int out_dtype, double alpha, const void* A, double beta, const void* B, void* C,
                     const GDims& d, hipStream_t s) {
    switch (out_dtype) {
        case TLIB_F64: return axpby_launch<TI, double>(alpha, A, beta, B, C, d, s);
        case TLIB_F32: return axpby_launch<TI, float>(alpha, A, beta, B, C, d, s);
        case TLIB_BF16: return axpby_launch<TI, bf16_t>(alpha, A, beta, B, C, d, s);
        case TLIB_F16: return axpby_launch<TI, f16_t>(alpha, A, beta, B, C, d, s);
    }
    return TLIB_EDTYPE;
}

int launch_axpby(int in_dtype, int out_dtype, double alpha, const void* A, double beta, const void* B, void* C,
                 const GDims& d, hipStream_t s) {
    switch (in_dtype) {
        case TLIB_F64: return axpby_out<double>(out_dtype, alpha, A, beta, B, C, d, s);
        case TLIB_F32: return axpby_out<float>(out_dtype, alpha, A, beta, B, C, d, s);
        case TLIB_BF16: return axpby_out<bf16_t>(out_dtype, alpha, A, beta, B, C, d, s);
        case TLIB_F16: return axpby_out<f16_t>(out_dtype, alpha, A, beta, B, C, d, s);
    }
    return TLIB_EDTYPE;
}

// C = A / den[0] with den in device memory (the normalisation step of the
// higher-order power method after the norm kernel wrote den): the quotient
// is formed in FP64 and rounded once to C's type.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void div_kernel(const double* den, const TI* A, TO* C, GDims g) {
    const double d = den[0];
    const bool flat = g.nd <= 1 && g.s[0][0] == 1 && g.s[2][0] == 1;
    const int64_t stride = int64_t(gridDim.x) * 256;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < g.total; i += stride) {
        int64_t off[3];
        if (flat) off[0] = off[1] = off[2] = i;
        else gd_decode(i, g, 3, off);
        C[off[2]] = round_out<TO>(to_f64(A[off[0]]) / d);
    }
}

template <typename TI, typename TO>
static int div_launch(const double* den, const void* A, void* C, const GDims& g, hipStream_t s) {
    const unsigned blocks = unsigned(std::max<int64_t>(1, std::min<int64_t>((g.total + 255) / 256, 8192)));
    hipLaunchKernelGGL((div_kernel<TI, TO>), dim3(blocks), dim3(256), 0, s, den, (const TI*)A, (TO*)C, g);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

template <typename TI>
static int div_out(int out_dtype, const double* den, const void* A, void* C, const GDims& g, hipStream_t s) {
    switch (out_dtype) {
        case TLIB_F64: return div_launch<TI, double>(den, A, C, g, s);
        case TLIB_F32: return div_launch<TI, float>(den, A, C, g, s);
        case TLIB_BF16: return div_launch<TI, bf16_t>(den, A, C, g, s);
        case TLIB_F16: return div_launch<TI, f16_t>(den, A, C, g, s);
    }
    return TLIB_EDTYPE;
}

int launch_div(int in_dtype, int out_dtype, const double* den, const void* A, void* C, const GDims& g,
               hipStream_t s) {
    switch (in_dtype) {
        case TLIB_F64: return div_out<double>(out_dtype, den, A, C, g, s);
        case TLIB_F32: return div_out<float>(out_dtype, den, A, C, g, s);
        case TLIB_BF16: return div_out<bf16_t>(out_dtype, den, A, C, g, s);
        case TLIB_F16: return div_out<f16_t>(out_dtype, den, A, C, g, s);
    }
    return TLIB_EDTYPE;
}

// ------------------------------------------------------------------ tiled relayout
// The same entrywise op when C's fastest dimension x is not A's fastest y
// (a transpose, or add/scale into another layout).  A block owns a 32 x 32
// tile of (x, y) for EW_RZ slices of the remaining dims: it reads A (and B
// when B is laid out like A) with consecutive lanes along y, parks the values
// in LDS, and writes C (reading B there when B is laid out like C) with
// consecutive lanes along x, so both HBM streams move whole 128-B lines.
// Arithmetic is axpby_kernel's, element for element.
__device__ uint64_t g_ew_zero[2];

__device__ __forceinline__ void ew_rest(uint32_t r, const EwTile& P, int64_t* o) {
    o[0] = o[1] = o[2] = 0;
#pragma unroll
    for (int d = 0; d < MAXP; ++d) {
        if (d >= P.nr) break;
        const uint32_t q = (d == P.nr - 1) ? 0u : fdiv(r, P.rfd[d]);
        const int64_t i = int64_t(r - q * P.rn[d]);
        o[0] += i * P.rs[0][d];
        o[1] += i * P.rs[1][d];
        o[2] += i * P.rs[2][d];
        r = q;
    }
}

template <typename TI, typename TO, int BM>
__global__ __launch_bounds__(256) void axpby_tile_kernel(double alpha, const TI* A, double beta, const TI* B,
                                                         TO* C, EwTile P) {
#pragma clang fp contract(off)
    constexpr int TS = EW_RZ * EW_T * (EW_T + 1);
    __shared__ __align__(8) unsigned char smem[(BM == 2 ? 2 : 1) * TS * sizeof(TI)];
    TI* ta = reinterpret_cast<TI*>(smem);
    TI* tb = ta + TS;
    const TI* zs = reinterpret_cast<const TI*>(g_ew_zero);
    const int lx = threadIdx.x & (EW_T - 1), ly = threadIdx.x / EW_T;  // 32 x 8
    for (uint32_t t = blockIdx.x; t < P.ntiles; t += gridDim.x) {
        const uint32_t q = fdiv(t, P.ftx);
        const int64_t x0 = int64_t(t - q * P.tx) * EW_T;
        const uint32_t rb = fdiv(q, P.fty);
        const int64_t y0 = int64_t(q - rb * P.ty) * EW_T;
        int64_t ro[EW_RZ][3];
        bool rv[EW_RZ];
#pragma unroll
        for (int z = 0; z < EW_RZ; ++z) {
            const uint32_t r = rb * EW_RZ + z;
            rv[z] = r < P.nrest;
            ew_rest(rv[z] ? r : 0u, P, ro[z]);
        }
        // read phase: lanes along y
        TI va[EW_RZ][EW_T / 8], vb[EW_RZ][EW_T / 8];
        const int64_t yr = y0 + lx;
#pragma unroll
        for (int z = 0; z < EW_RZ; ++z)
#pragma unroll
            for (int j = 0; j < EW_T / 8; ++j) {
                const int64_t xr = x0 + ly + 8 * j;
                const bool ok = rv[z] && xr < P.nx && yr < P.ny;
                va[z][j] = *(ok ? A + (ro[z][0] + xr * P.sx[0] + yr * P.sy[0]) : zs);
                if (BM == 2) vb[z][j] = *(ok ? B + (ro[z][1] + xr * P.sx[1] + yr * P.sy[1]) : zs);
            }
        __syncthreads();
#pragma unroll
        for (int z = 0; z < EW_RZ; ++z)
#pragma unroll
            for (int j = 0; j < EW_T / 8; ++j) {
                const int e = (z * EW_T + ly + 8 * j) * (EW_T + 1) + lx;
                ta[e] = va[z][j];
                if (BM == 2) tb[e] = vb[z][j];
            }
        __syncthreads();
        // write phase: lanes along x
        const int64_t xw = x0 + lx;
#pragma unroll
        for (int z = 0; z < EW_RZ; ++z)
#pragma unroll
            for (int j = 0; j < EW_T / 8; ++j) {
                const int64_t yw = y0 + ly + 8 * j;
                const bool ok = rv[z] && xw < P.nx && yw < P.ny;
                const int e = (z * EW_T + lx) * (EW_T + 1) + ly + 8 * j;
                double v = alpha * to_f64(ta[e]);
                if (BM == 1) v = v + beta * to_f64(*(ok ? B + (ro[z][1] + xw * P.sx[1] + yw * P.sy[1]) : zs));
                if (BM == 2) v = v + beta * to_f64(tb[e]);
                if (ok) C[ro[z][2] + xw * P.sx[2] + yw * P.sy[2]] = round_out<TO>(v);
            }
    }
}

template <typename TI, typename TO>
static int axpby_tile_launch(double alpha, const void* A, double beta, const void* B, void* C, const EwTile& t,
                             int bm, hipStream_t s) {
    const unsigned blocks = unsigned(std::max<uint32_t>(1, std::min<uint32_t>(t.ntiles, 1u << 20)));
    if (bm == 0)
        hipLaunchKernelGGL((axpby_tile_kernel<TI, TO, 0>), dim3(blocks), dim3(256), 0, s, alpha, (const TI*)A,
                           beta, (const TI*)B, (TO*)C, t);
    else if (bm == 1)
        hipLaunchKernelGGL((axpby_tile_kernel<TI, TO, 1>), dim3(blocks), dim3(256), 0, s, alpha, (const TI*)A,
                           beta, (const TI*)B, (TO*)C, t);
    else
        hipLaunchKernelGGL((axpby_tile_kernel<TI, TO, 2>), dim3(blocks), dim3(256), 0, s, alpha, (const TI*)A,
                           beta, (const TI*)B, (TO*)C, t);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

template <typename TI>
static int axpby_tile_out(int out_dtype, double alpha, const void* A, double beta, const void* B, void* C,
                          const EwTile& t, int bm, hipStream_t s) {
    switch (out_dtype) {
        case TLIB_F64: return axpby_tile_launch<TI, double>(alpha, A, beta, B, C, t, bm, s);
        case TLIB_F32: return axpby_tile_launch<TI, float>(alpha, A, beta, B, C, t, bm, s);
        case TLIB_BF16: return axpby_tile_launch<TI, bf16_t>(alpha, A, beta, B, C, t, bm, s);
        case TLIB_F16: return axpby_tile_launch<TI, f16_t>(alpha, A, beta, B, C, t, bm, s);
    }
    return TLIB_EDTYPE;
}

int launch_axpby_tile(int in_dtype, int out_dtype, double alpha, const void* A, double beta, const void* B,
                      void* C, const EwTile& t, int b_mode, hipStream_t s) {
    if (b_mode < 0 || b_mode > 2) return TLIB_EINVAL;
    switch (in_dtype) {
        case TLIB_F64: return axpby_tile_out<double>(out_dtype, alpha, A, beta, B, C, t, b_mode, s);
        case TLIB_F32: return axpby_tile_out<float>(out_dtype, alpha, A, beta, B, C, t, b_mode, s);
        case TLIB_BF16: return axpby_tile_out<bf16_t>(out_dtype, alpha, A, beta, B, C, t, b_mode, s);
        case TLIB_F16: return axpby_tile_out<f16_t>(out_dtype, alpha, A, beta, B, C, t, b_mode, s);
    }
    return TLIB_EDTYPE;
}

}  // namespace tlib
