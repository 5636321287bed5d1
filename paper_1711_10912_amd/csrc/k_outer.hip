// Outer product (Sec. 5.2 Table 3 outer_product, the q = 0 case of Eq. ttt
// and ttt_indices): every element of C is one product
//   C[m, n] = X[m] * Y[n],
// m running over the free modes of one operand and n over those of the other,
// each group addressed through up to four (extent, stride) pairs.  N is the
// group that holds C's unit-stride mode, so lanes run along C's memory.
//
// The kernel is a write stream: C holds |X| |Y| elements and is written
// once, the inputs are read from cache.  A workgroup owns a chunk of CW
// column vectors (V consecutive columns each: 16-byte stores when C's rows
// allow them) and R = 256 / CW rows at a time; a thread loads its V values of
// Y and decodes its column offset in C once, then walks rows, one product
// per element.  The product is formed in the output type (FP32 for FP32 and
// 16-bit inputs, FP64 for FP64), so each element is rounded once.
#include <algorithm>

#include "device.hpp"

namespace tlib {

template <typename TI, int V>
__global__ __launch_bounds__(256) void outer_kernel(OuterParams P) {
    using TA = typename AccOf<TI>::type;
    const TI* X = (const TI*)P.X;
    const TI* Y = (const TI*)P.Y;
    TA* C = (TA*)P.C;
    const int tid = threadIdx.x;
    const int c = tid & (P.cw - 1), r = tid >> P.cw_log2;
    const int64_t nvi = int64_t(blockIdx.x) * P.cw + c;  // column vector of this lane
    if (nvi >= P.nv) return;
    const uint32_t n0 = uint32_t(nvi * V);
    TA y[V];
    int64_t cc[V];
#pragma unroll
    for (int t = 0; t < V; ++t) {
        int64_t oy, oc;
        grp_decode(n0 + t, P.gn, oy, oc);
        y[t] = to_acc(Y[oy]);
        cc[t] = oc;
    }
    const int rows = P.rows_per_wg;  // 256 / cw
    for (int64_t m = int64_t(blockIdx.y) * rows + r; m < P.M; m += int64_t(gridDim.y) * rows) {
        int64_t ox, ocm;
        grp_decode(uint32_t(m), P.gm, ox, ocm);
        const TA x = to_acc(X[ox]);
        if constexpr (V > 1) {
            typedef TA vt __attribute__((ext_vector_type(V)));
            vt v;
#pragma unroll
            for (int t = 0; t < V; ++t) v[t] = x * y[t];
            *reinterpret_cast<vt*>(C + (ocm + cc[0])) = v;
        } else {
            C[ocm + cc[0]] = x * y[0];
        }
    }
}

template <typename TI>
static int outer_launch(const OuterParams& p, hipStream_t s) {
    using TA = typename AccOf<TI>::type;
    constexpr int VV = 16 / int(sizeof(TA));
    const int64_t rows = p.rows_per_wg;
    const unsigned gx = unsigned((p.nv + p.cw - 1) / p.cw);
    // about four rows per thread, at most 65535 row blocks
    int64_t gy = (p.M + rows * 4 - 1) / (rows * 4);
    gy = std::max<int64_t>(1, std::min<int64_t>(gy, 65535));
    const dim3 grid(gx, unsigned(gy));
    if (p.vec > 1) hipLaunchKernelGGL((outer_kernel<TI, VV>), grid, dim3(256), 0, s, p);
    else hipLaunchKernelGGL((outer_kernel<TI, 1>), grid, dim3(256), 0, s, p);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

int launch_outer(int dtype, const OuterParams& p, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return outer_launch<double>(p, s);
        case TLIB_F32: return outer_launch<float>(p, s);
        case TLIB_BF16: return outer_launch<bf16_t>(p, s);
        case TLIB_F16: return outer_launch<f16_t>(p, s);
    }
    return TLIB_EDTYPE;
}

}  // namespace tlib
