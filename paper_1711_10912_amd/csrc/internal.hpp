// Internal declarations shared by the host planner (plan.cpp, abi.cpp) and the
// HIP kernels (k_*.hip).  Not part of the public ABI (see include/tlib.h).
#pragma once

#include <cstdint>
#include <hip/hip_runtime_api.h>

#include "tlib.h"

namespace tlib {

constexpr int MAXP = TLIB_MAX_ORDER;

// ------------------------------------------------------------------ descriptors

// A validated tensor: data pointer, dtype, order, extents and element strides.
struct Ten {
    void* data = nullptr;
    int dtype = 0;
    int p = 0;
    int64_t n[MAXP] = {};
    int64_t w[MAXP] = {};
    int64_t numel() const {
        int64_t s = 1;
        for (int r = 0; r < p; ++r) s *= n[r];
        return s;
    }
};

inline int esize(int dtype) { return dtype == TLIB_F64 ? 8 : dtype == TLIB_F32 ? 4 : 2; }
// Output dtype of a contraction: FP64 for FP64 input, FP32 otherwise.
inline int acc_dtype(int dtype) { return dtype == TLIB_F64 ? TLIB_F64 : TLIB_F32; }

// Unsigned 32-bit division by a run-time constant: q = (umulhi(x, m) + x) >> s
// (round-up multiplier method, valid for every 32-bit x and divisor >= 1).
struct FastDiv {
    uint32_t d = 1, m = 1, s = 0;
};
FastDiv make_fastdiv(uint32_t d);

// A dimension after coalescing, with the strides of up to three operands.
struct Dim {
    int64_t n;
    int64_t s[3];
};

// Remove extent-1 dims, sort by the strides of operand `key` (ascending), and
// merge neighbours i, i+1 whose strides chain for every operand
// (s_op[i+1] == s_op[i] * n[i]).  Returns the new number of dims.
int coalesce(Dim* d, int nd, int nops, int key);

// Up to GMAXD dims of one index group (M, N or K of a GEMM, or the output
// index of a streaming kernel) with the strides of two operands.
constexpr int GMAXD = 4;
struct Grp {
    int nd = 0;
    int64_t total = 1;
    int64_t n[GMAXD] = {1, 1, 1, 1};
    int64_t s0[GMAXD] = {};
    int64_t s1[GMAXD] = {};
    FastDiv fd[GMAXD];
};

// Up to MAXP dims for the generic (per-element decode) kernels; 64-bit divide.
struct GDims {
    int nd = 0;
    int64_t total = 1;
    int64_t n[MAXP] = {};
    int64_t s[3][MAXP] = {};
};

// Entrywise op whose output's fastest dimension (x) is not the input's (y):
// 32x32 tiles over (x, y) times slices of the other dims; 32-bit fast-divide
// decode.  Strides: operand 0 = A, 1 = B, 2 = C.
constexpr int EW_T = 32;   // tile edge
constexpr int EW_RZ = 2;   // slices of the other dims per tile
struct EwTile {
    int64_t nx = 1, ny = 1;
    int64_t sx[3] = {}, sy[3] = {};
    uint32_t tx = 1, ty = 1, nrest = 1, ntiles = 1;
    FastDiv ftx, fty;
    int nr = 0;
    uint32_t rn[MAXP] = {};
    FastDiv rfd[MAXP];
    int64_t rs[3][MAXP] = {};
};

// ------------------------------------------------------------------ kernel parameters

// TTV on the collapsed (lo, k, hi) form: A(lo,k,hi) at lo*sA_lo + k*sA_k + hi*sA_hi.
struct TtvParams {
    const void* A;
    const void* b;
    void* C;
    int64_t n_lo, n_k, n_hi;
    int64_t sA_lo, sA_k, sA_hi, sb, sC_lo, sC_hi;
    // col kernel: the hi index decoded over up to GMAXD dims (s0 = A stride,
    // s1 = C stride), so views whose outer dims do not merge keep the kernel
    Grp gh;
};

struct GemmParams {
    const void* X;  // M x K operand
    const void* Y;  // K x N operand
    void* C;        // M x N result (or split-K partials)
    int32_t M, N, K;
    Grp gm;  // s0 = X stride, s1 = C stride
    Grp gn;  // s0 = Y stride, s1 = C stride
    Grp gk;  // s0 = X stride, s1 = Y stride
    int32_t x_kfast, y_kfast;
    int32_t c_vec;  // C rows can take 16-byte vector stores along N
    int32_t tiles_m, tiles_n;
    int32_t ksplit, kchunk;  // split-K: each z-slice handles kchunk of K
    void* part;              // split-K partials [ksplit][M][N] (accumulator type)
    int32_t y_vec;           // > 0: Y loaded as vectors of y_vec elements along N (K one dim, stride syk)
    int64_t syk;
    int32_t kvec;            // bit 0 / bit 1: X / Y loaded as groups of consecutive k (8 for 16-bit, 2 for FP32/FP64)
};

// Multi-mode TTV (one pass over A).  A group of modes in storage order,
// fastest first: extents, A strides, and the vector of each mode (nullptr for
// the excluded mode r).
struct TvModes {
    int nd = 0;
    int64_t n[MAXP] = {};
    FastDiv fd[MAXP];
    int64_t s[MAXP] = {};
    const void* u[MAXP] = {};
    int64_t us[MAXP] = {};
};

constexpr int TV_SLOTS = 2048;  // positions per tile (8 per thread)

// pos: the tile's position modes (K1: ending with r); out: the lo modes
// between the positions and r (K2 only); hi: the modes after r.  A block
// (ib, fc, hc) streams rows t = o + n_out * (h - h0), o < n_out, h in
// [h0, h0 + hc_len), G rows of W positions per tile.
struct TvParams {
    const void* A = nullptr;
    TvModes pos, out, hi;
    int64_t npos = 1;    // positions (product of pos extents), < 2^31
    int64_t n_lo = 1;    // K1: positions per value of i_r
    int64_t n_r = 1;
    int32_t W = 1;       // positions per tile row
    int32_t G = 1;       // rows per tile (G * W <= TV_SLOTS)
    int32_t nfc = 1;     // position chunks
    int32_t nloc = 1;    // K1: partial slots per chunk
    int32_t HC = 1;      // row chunks
    int32_t k2 = 0;
    int64_t n_out = 1, n_hi = 1;
    FastDiv fd_out;
    int64_t hc_len = 1;  // slabs per row chunk (n_out * hc_len < 2^31)
    int64_t s_r = 0;     // K2: A stride of mode r
    int32_t lin = 0;     // row offset = o * s_o + h * s_h (no offset table), and
                         // one weight per row t in tabw (n_out * n_hi entries)
    int64_t s_o = 0, s_h = 0;
    double* tabw = nullptr;   // lin: row weights [n_out * n_hi]; else weights [n_out + n_hi]
    int64_t* tabo = nullptr;  // row offsets [n_out + n_hi] (not lin)
    double* part = nullptr;   // partial sums
};

// Two mode products in one pass: C = (A x_f Uf) x_g Ug, f the contracted
// mode with the smaller stride in A.  Columns are the index tuples of the
// other modes (gc: s0 = A stride, s1 = C stride).
struct Ttm2Params {
    const void* A = nullptr;
    const void* Uf = nullptr;
    const void* Ug = nullptr;
    void* C = nullptr;
    int32_t n_f = 1, n_g = 1, m_f = 1, m_g = 1;  // contracted extents, factor rows (<= 32)
    int64_t s_f = 0, s_g = 0;                    // A strides of the contracted modes
    int64_t sUf0 = 0, sUf1 = 0, sUg0 = 0, sUg1 = 0;
    int64_t sC_f = 0, sC_g = 0;                  // C strides of j_f, j_g
    int64_t ncol = 1;
    Grp gc;
};

// Streaming TTM with a short contraction: X = B (M x K, strides sXm, sXk),
// Y = A (columns nu over gn, stride sYk along k), C(j, nu) at j*sCm + gn.s1.
struct TtmParams {
    const void* X;
    const void* Y;
    void* C;
    int32_t M, N, K;
    int64_t sXm, sXk, sYk, sCm;
    Grp gn;  // s0 = Y stride, s1 = C stride
};

// Streaming TTM with C strided along j (the row index of B): the columns nu
// split into runs of n_lo along C's innermost column dim (strides sYlo in A,
// sClo in C) and the remaining column dims gh (s0 = A stride, s1 = C stride).
// Work units are (run h, chunk t) pairs; mode selects how rows are written:
//   TTM_ROWS_PLAIN   64-column windows starting at 64 t
//   TTM_ROWS_ALIGNED 64-column windows shifted per row to start on a 128-byte
//                    line of C (needs sClo == 1; computes 128 bytes more)
//   TTM_ROWS_BAND    whole runs, with rows j contiguous in C (sClo == 1,
//                    sCm == n_lo): written as one linear range per row group
//                    (two column blocks, n_lo <= 32; BAND1: one, n_lo <= 16;
//                    BANDW: eleven, 128 < n_lo <= 176, FP32/FP64, k <= 16)
enum { TTM_ROWS_PLAIN = 0, TTM_ROWS_ALIGNED = 1, TTM_ROWS_BAND = 2, TTM_ROWS_BAND1 = 3, TTM_ROWS_BANDW = 4 };
struct TtmRowParams {
    const void* X;
    const void* Y;
    void* C;
    int32_t M, K;
    int64_t sXm, sXk, sYk, sCm;
    int32_t n_lo;
    int32_t Tc;  // chunks per run
    int64_t sYlo, sClo;
    int64_t units;  // runs * Tc
    FastDiv fd_tc, fd_lo;
    Grp gh;
    int32_t mr;   // rows of B served by one workgroup (multiple of 16)
    int32_t nrg;  // row groups, ceil(M / mr); the grid is a multiple of 8 * nrg when nrg > 1
};

// Outer product (k_outer.hip): C[m, n] = X[m] * Y[n]; gm: s0 = X stride, s1 =
// C stride; gn: s0 = Y stride, s1 = C stride (N holds C's unit-stride mode).
// Columns go in vectors of `vec` (16-byte stores) or singly; a workgroup
// chunk holds cw (a power of two <= 256) column vectors and takes
// rows_per_wg = 256 / cw rows at a time.
struct OuterParams {
    const void* X;
    const void* Y;
    void* C;
    int64_t M, N, nv;
    Grp gm, gn;
    int32_t vec, cw, cw_log2, rows_per_wg;
};
int launch_outer(int dtype, const OuterParams& p, hipStream_t s);

// Work table of a grouped launch (k_batch.hip): a header followed by items.
struct BatchHeader {
    int32_t n_items;
    int32_t pad0;
    int64_t total_units;  // units of 256 outputs over all items
    int64_t pad1[2];
};
// Item kinds: BATCH_SCALAR = one thread per output (M = 1, K one dim),
// BATCH_TILE = 16 x 64 tiles of C on matrix cores.
enum { BATCH_SCALAR = 0, BATCH_TILE = 1 };
// One request as C[m, n] = sum_k X[m, k] Y[k, n]; gm: s0 = X, s1 = C;
// gn: s0 = Y, s1 = C; gk: s0 = X, s1 = Y.
struct BatchItem {
    int32_t dtype;  // input dtype; C is FP64 for FP64 input, FP32 otherwise
    int32_t kind;
    int64_t unit_begin;  // first unit of this item (prefix sum)
    const void* X;
    const void* Y;
    void* C;
    int64_t M, N, K;
    int64_t tiles_n;  // BATCH_TILE: ceil(N / 64)
    Grp gm, gn, gk;
};
int launch_batch(const void* table_dev, int grid, hipStream_t s);

enum GemmTile {
    GT_16x256 = 0, GT_64x128 = 1, GT_128x128 = 2, GT_256x64 = 3, GT_64x64 = 4, GT_128x64 = 5, GT_256x32 = 6,
    GT_COUNT
};
struct TileShape {
    int bm, bn;
};
TileShape tile_shape(int t);

// ------------------------------------------------------------------ launchers (k_*.hip)
// Each returns TLIB_OK or TLIB_EHIP.
// Col kernel with one wave per (lo tile, hi) unit and kr >= n_k rows in flight
// (kr in {8, 16, 32, 64}, kr * vec * element size <= 256 bytes).
int launch_ttv_colw(int dtype, const TtvParams& p, int vec, int kr, hipStream_t s);
int launch_ttv_col(int dtype, const TtvParams& p, int vec, int ksplit, void* ws, hipStream_t s);
int launch_ttv_slab(int dtype, const TtvParams& p, int slabs, int kc, hipStream_t s);
int launch_ttv_generic(int dtype, const TtvParams& p, const GDims& out, hipStream_t s);
// G lanes per output stream its k-fiber; outputs decoded over go (s0 = A, s1 = C)
int launch_ttv_fiber(int dtype, const TtvParams& p, const Grp& go, int G, hipStream_t s);

int launch_gemm(int dtype, int tile, const GemmParams& p, hipStream_t s);
int gemm_slice_k(int dtype, int tile);  // K depth of one LDS slice of the tile
// All-rows GEMM (k_gemm_rows.hip) for M <= 16 fm: fm in {1, 2, 4, 8}, 64 fn
// columns per workgroup, fn in {1, 2}.  Needs X's K groups contiguous (16
// bytes, FP32 8) and, for 16-bit inputs, Y's as well (kvec bits 0 and 1).
int launch_gemm_rows(int dtype, int fm, int fn, const GemmParams& p, hipStream_t s);
int gemm_rows_kchunk(int dtype);  // K per chunk (the split granularity)
// Sum of split-K partials [ksplit][M][N] into C (acc_dtype = FP32 or FP64).
int launch_gemm_ksum(int acc_dtype, const GemmParams& p, hipStream_t s);
// prep + main + finish kernels of the one-pass multi-mode TTV; vec: 16-byte loads
int launch_tv(int dtype, const TvParams& P, void* c, int64_t cs, bool vec, hipStream_t s);
int launch_ttm2(int dtype, const Ttm2Params& P, bool vec, hipStream_t s);
int ttm2_lds_bytes(int dtype, int m_f, int n_f, int n_g, bool vec);
int ttm2_vec_rows(int dtype);  // largest n_f of the slab-copy path
// fm: row blocks (1, 4 or 16); ks: k-steps from ttm_stream_ks (0 = unsupported)
int launch_ttm_stream(int dtype, const TtmParams& p, int fm, int ks, bool trans, int grid, hipStream_t s);
int ttm_stream_ks(int dtype, int k);
// Row-streaming TTM (TtmRowParams); ks from ttm_rows_ks, lds from ttm_rows_lds
// (m = rows per workgroup, p.mr).
int launch_ttm_rows(int dtype, const TtmRowParams& p, int mode, int ks, int grid, hipStream_t s);
int ttm_rows_ks(int dtype, int mode, int k);
int64_t ttm_rows_lds(int dtype, int mode, int m, int ks);
int launch_gemm_generic(int dtype, const void* X, const void* Y, void* C, const GDims& m,
                        const GDims& n, const GDims& k, hipStream_t s);

// Two-pass deterministic FP64 dot product over a GDims iteration space with
// strides s[0] (A) and s[1] (B); B == nullptr means A . A.  `sqrt_out` takes
// the square root of the final sum (norm).
int launch_dot(int dtype, const void* A, const void* B, const GDims& d, double* out, bool sqrt_out,
               void* ws, size_t ws_bytes, hipStream_t s);
int dot_partials(int64_t total);  // number of first-pass partials for a given size
int dot_partials_g(const GDims& g);  // first-pass partials of a coalesced iteration space

// C = A / den[0] (den in device memory) over GDims (strides s[0] = A, s[2] = C).
int launch_div(int in_dtype, int out_dtype, const double* den, const void* A, void* C, const GDims& g,
               hipStream_t s);
// C = alpha*A + beta*B over GDims (strides s[0]=A, s[1]=B, s[2]=C); B may be null.
// A and B have in_dtype; C has out_dtype (correctly rounded from FP64).
int launch_axpby(int in_dtype, int out_dtype, double alpha, const void* A, double beta, const void* B,
                 void* C, const GDims& d, hipStream_t s);
// The same op through LDS tiles (EwTile); b_mode 0 = no B, 1 = B read along x
// (laid out like C), 2 = B read along y (laid out like A).
int launch_axpby_tile(int in_dtype, int out_dtype, double alpha, const void* A, double beta, const void* B,
                      void* C, const EwTile& t, int b_mode, hipStream_t s);

// ------------------------------------------------------------------ workspace (abi.cpp)
// Scratch of one call: the stream's workspace (acquired on the first take),
// or a fixed buffer the caller brings (`fixed`).  take() hands out 256-byte
// aligned pieces from the start and returns nullptr when the buffer cannot
// hold them (or cannot be allocated); it never frees or waits.
struct WsCtx {
    hipStream_t s = nullptr;
    char* base = nullptr;
    size_t size = 0, used = 0;
    size_t hint = 0;   // bytes the whole call will take (first allocation size)
    size_t peak = 0;   // largest used + need() seen (plan-only probes)
    bool fixed = false;
    void* take(size_t bytes);
    void need(size_t bytes);
    size_t avail() const { return size > used ? size - used : 0; }
};

}  // namespace tlib
