// Grouped launch for many small TTV / TTM requests (Sec. 5.2 Eq. ttv, ttm).
//
// The host plans a batch into a work table in device memory: a header and one
// item per request, each in the collapsed (lo, k, hi) form, with a prefix sum
// of work units (256 outputs each).  One persistent kernel with fixed
// arguments walks the table, so the same launch can be captured once in a HIP
// graph and replayed for every batch after the table's contents change.
// Within a unit one thread computes one output: consecutive threads take
// consecutive lo, so reads of A at fixed k are coalesced.
#include <algorithm>

#include "device.hpp"

namespace tlib {

template <typename TI>
__device__ __forceinline__ void batch_unit(const BatchItem& it, int64_t u) {
    using TA = typename AccOf<TI>::type;
    const int64_t o = u * 256 + threadIdx.x;
    const int64_t outs = it.n_lo * it.m * it.n_hi;
    if (o >= outs) return;
    // output order: lo fastest, then j, then hi
    const int64_t lo = o % it.n_lo;
    const int64_t r = o / it.n_lo;
    const int64_t j = r % it.m;
    const int64_t hi = r / it.m;
    const TI* A = (const TI*)it.A + lo * it.sA_lo + hi * it.sA_hi;
    const TI* B = (const TI*)it.B + j * it.sB_j;
    TA acc = TA(0);
    for (int64_t k = 0; k < it.n_k; ++k) acc += to_acc(A[k * it.sA_k]) * to_acc(B[k * it.sB_k]);
    ((TA*)it.C)[lo * it.sC_lo + j * it.sC_j + hi * it.sC_hi] = acc;
}

__global__ __launch_bounds__(256) void batch_kernel(const BatchHeader* hdr, const BatchItem* items) {
    const int n = hdr->n_items;
    const int64_t total = hdr->total_units;
    __shared__ int s_item;
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
        switch (it.dtype) {
            case TLIB_F64: batch_unit<double>(it, lu); break;
            case TLIB_F32: batch_unit<float>(it, lu); break;
            case TLIB_BF16: batch_unit<bf16_t>(it, lu); break;
            case TLIB_F16: batch_unit<f16_t>(it, lu); break;
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
