// Streaming TTM (Sec. 5.2 Eq. ttm) for a short contraction (n_m <= 64):
//   C(.., j, ..) = sum_k B(j, k) A(.., k, ..)
// With a short k the cost is writing C (m/n_m times the size of A), so both
// kernels here are built around the stores:
//   * each persistent workgroup stages the whole matrix B (m x n_m, zero-padded
//     to the MFMA k-step) in LDS once and then walks a contiguous range of
//     units of A's columns nu (the modes other than m), loading A fragments
//     straight into MFMA operand registers one unit ahead;
//   * ttm_stream_kernel serves C contiguous along j: MFMA operands are swapped
//     so the lanes of a result register run along j;
//   * ttm_rows_kernel serves C strided along j: results go through a small
//     per-wave LDS stage and leave as row windows that start on 128-byte lines
//     (or as one linear range when rows of a run are adjacent in C), because
//     stores that split lines between instructions cost up to half the
//     write bandwidth on MI355X.
// MFMAs: v_mfma_f64_16x16x4 (FP64), v_mfma_f32_16x16x4 (FP32) and
// v_mfma_f32_16x16x32_{bf16,f16} (16-bit inputs, FP32 accumulation).
#include <algorithm>

#include "device.hpp"

namespace tlib {

typedef double d4s_t __attribute__((ext_vector_type(4)));
typedef float f4s_t __attribute__((ext_vector_type(4)));

// Element p of the result holds element p ^ g of a (g in 0..3).
__device__ __forceinline__ f4s_t swz4(f4s_t a, int g) {
    return g == 0 ? a : g == 1 ? a.yxwz : g == 2 ? a.zwxy : a.wzyx;
}

// Buffer resource of a wave-uniform range.  The address and size are taken
// from the first lane so that the descriptor lives in scalar registers: the
// compiler cannot always prove them uniform and would otherwise wrap every
// store in a loop over the distinct descriptors of the wave.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t wave_rsrc(const void* p, uint32_t nbytes) {
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(a));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(a >> 32));
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>((uint64_t(hi) << 32) | lo), 0,
                                             int(__builtin_amdgcn_readfirstlane(nbytes)), 0x00020000);
}
typedef __bf16 bf8s_t __attribute__((ext_vector_type(8)));
typedef _Float16 h8s_t __attribute__((ext_vector_type(8)));
typedef uint32_t u4s_t __attribute__((ext_vector_type(4)));
typedef uint32_t u2s_t __attribute__((ext_vector_type(2)));

template <typename TI> struct SMfma {
    using acc_t = f4s_t;
    using frag_t = u4s_t;  // 8 x 16-bit
    static constexpr int KSTEP = 32;
};
template <> struct SMfma<double> {
    using acc_t = d4s_t;
    using frag_t = double;
    static constexpr int KSTEP = 4;
};
template <> struct SMfma<float> {
    using acc_t = f4s_t;
    using frag_t = float;
    static constexpr int KSTEP = 4;
};

template <typename TI>
__device__ __forceinline__ typename SMfma<TI>::acc_t smfma(typename SMfma<TI>::frag_t a, typename SMfma<TI>::frag_t b,
                                                          typename SMfma<TI>::acc_t c) {
    if constexpr (std::is_same<TI, double>::value) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else if constexpr (std::is_same<TI, float>::value) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    else if constexpr (std::is_same<TI, bf16_t>::value)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8s_t, a), __builtin_bit_cast(bf8s_t, b),
                                                       c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8s_t, a), __builtin_bit_cast(h8s_t, b), c,
                                                      0, 0, 0);
}

__device__ __forceinline__ uint32_t raw16(const bf16_t* p) { return *reinterpret_cast<const uint16_t*>(p); }
__device__ __forceinline__ uint32_t raw16(const f16_t* p) { return *reinterpret_cast<const uint16_t*>(p); }

// Source of the fragment loads that fall outside the operand.
__device__ __align__(16) double g_ttm_zero[2] = {0.0, 0.0};

// The MFMA A-operand fragments of one column (base y) for KS k-steps: lane
// (rl, kq) supplies k = s*KSTEP + kq (FP32/FP64) or k = s*32 + 8*kq + e, e < 8
// (16-bit, packed in pairs).  Entries outside the operand (column not valid,
// k >= K) load from a zero word instead: selecting the address rather than
// the loaded value keeps every load unconditional, where a select after the
// load lets the compiler sink the load into a branch and wait for it there
// (and a wait on loads is also a wait on all of the wave's earlier stores).
template <typename TI, int KS>
__device__ __forceinline__ void load_frags(const TI* y, int64_t sk, int K, bool cv,
                                           int kq, typename SMfma<TI>::frag_t (&f)[KS]) {
    constexpr int KSTEP = SMfma<TI>::KSTEP;
    const TI* zsrc = reinterpret_cast<const TI*>(g_ttm_zero);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        if constexpr (sizeof(TI) == 2) {
            uint32_t w[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int k0 = s * 32 + 8 * kq + 2 * h;
                const uint32_t lo = raw16(cv && k0 < K ? y + int64_t(k0) * sk : zsrc);
                const uint32_t hi = raw16(cv && k0 + 1 < K ? y + int64_t(k0 + 1) * sk : zsrc);
                w[h] = lo | (hi << 16);
            }
            f[s] = u4s_t{w[0], w[1], w[2], w[3]};
        } else {
            const int k = s * KSTEP + kq;
            f[s] = *(cv && k < K ? y + int64_t(k) * sk : zsrc);
        }
    }
}

// Persistent work walk shared by the streaming TTM kernels.  Workgroups are
// dealt round-robin to the eight XCDs, so the grid is split into min(8, G)
// groups by blockIdx % 8 and each group walks its own contiguous range of
// units: neighbouring units, which share cache lines of C at their edges, are
// written through the same L2.  `workers` units are in flight per workgroup.
struct Walk {
    int64_t u, end, step;
};
__device__ __forceinline__ Walk xcd_walk(int64_t units, int workers, int worker, int blk, int G) {
    const int ng = G < 8 ? G : 8, xg = blk % ng, ix = blk / ng;
    const int nx = (G - xg + ng - 1) / ng;
    Walk w;
    w.end = int64_t(xg + 1) * units / ng;
    w.u = int64_t(xg) * units / ng + int64_t(ix) * workers + worker;
    w.step = int64_t(nx) * workers;
    return w;
}

// C contiguous along j (TRANS): each wave owns FM row blocks (all rows) of a
// 16*FN-column strip; the MFMA operands are swapped so that the lanes of a
// result register run along j, and every store instruction writes four
// columns' 16-row segments.
template <typename TI, int FM, int FN, int KS>
__global__ __launch_bounds__(256) void ttm_stream_kernel(TtmParams P) {
    using TA = typename AccOf<TI>::type;
    using acc_t = typename SMfma<TI>::acc_t;
    using frag_t = typename SMfma<TI>::frag_t;
    constexpr bool WIDE = sizeof(TI) == 2;
    constexpr int KSTEP = SMfma<TI>::KSTEP;
    constexpr int KP = KS * KSTEP;             // padded contraction length
    constexpr int M16 = FM * 16;
    constexpr int PB = WIDE ? (KP + 8) : (M16 + (sizeof(TI) == 8 ? 4 : 16));
    constexpr int RQ = std::is_same<TI, double>::value ? 1 : 4;  // result row of (kq, r): RQ*kq + RR*r
    constexpr int RR = std::is_same<TI, double>::value ? 4 : 1;
    constexpr int COLS = 4 * FN * 16;          // columns per workgroup tile

    extern __shared__ __align__(16) unsigned char smem[];
    using RT = typename std::conditional<WIDE, uint16_t, TI>::type;
    RT* Bs = reinterpret_cast<RT*>(smem);

    // wave index through readfirstlane, so that everything derived from it
    // (unit, run, chunk, block activity) is known to be wave-uniform
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rl = lane & 15, kq = lane >> 4;
    const TI* X = (const TI*)P.X;
    const TI* Y = (const TI*)P.Y;
    TA* C = (TA*)P.C;

    // stage B (M x K) zero-padded to M16 x KP
    for (int e = tid; e < M16 * KP; e += 256) {
        int m, k;
        if constexpr (WIDE) { m = e / KP; k = e % KP; }
        else { k = e / M16; m = e % M16; }
        RT v = RT(0);
        if (m < P.M && k < P.K) {
            const TI* src = X + int64_t(m) * P.sXm + int64_t(k) * P.sXk;
            if constexpr (WIDE) v = uint16_t(raw16(src));
            else v = *src;
        }
        if constexpr (WIDE) Bs[m * PB + k] = v;
        else Bs[k * PB + m] = v;
    }
    __syncthreads();

    const int64_t T = (int64_t(P.N) + COLS - 1) / COLS;
    frag_t ycur[FN][KS], ynxt[FN][KS];

    // A fragments of tile t for this wave: block j holds columns
    // t*COLS + (wave*FN + j)*16 + rl; lane (rl, kq) supplies k = s*KSTEP + kq
    // (FP32/FP64) or k = s*32 + 8*kq + e (16-bit).
    auto load_y = [&](int64_t t, frag_t (&y)[FN][KS]) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = int(t * COLS) + (wave * FN + j) * 16 + rl;
            const bool cv = col < P.N;
            const int64_t yo = grp_off0(uint32_t(cv ? col : P.N - 1), P.gn);
            load_frags<TI, KS>(Y + yo, P.sYk, P.K, cv, kq, y[j]);
        }
    };

    Walk wk = xcd_walk(T, 1, 0, blockIdx.x, gridDim.x);
    if (wk.u < wk.end) load_y(wk.u, ycur);
    for (; wk.u < wk.end; wk.u += wk.step) {
        const int64_t tn = wk.u + wk.step;
        if (tn < wk.end) load_y(tn, ynxt);

        acc_t acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                frag_t b;
                if constexpr (WIDE) b = *reinterpret_cast<const u4s_t*>(&Bs[(i * 16 + rl) * PB + s * 32 + 8 * kq]);
                else b = Bs[(s * KSTEP + kq) * PB + i * 16 + rl];
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = smfma<TI>(ycur[j][s], b, acc[i][j]);
            }
        }

        // lane column = row of M (rl), registers = columns nu.  A tile with
        // every row and column inside C (all but the last, when M fills the
        // row blocks) stores without per-lane tests, so its stores carry no
        // exec branches.
        if (P.M == M16 && (wk.u + 1) * COLS <= int64_t(P.N)) {
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int cbase = int(wk.u * COLS) + (wave * FN + j) * 16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int col = cbase + RQ * kq + RR * r;
                    TA* cp = C + grp_off1(uint32_t(col), P.gn) + int64_t(rl) * P.sCm;
#pragma unroll
                    for (int i = 0; i < FM; ++i) cp[int64_t(i * 16) * P.sCm] = acc[i][j][r];
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int cbase = int(wk.u * COLS) + (wave * FN + j) * 16;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int col = cbase + RQ * kq + RR * r;
                    if (col < P.N) {
                        TA* cp = C + grp_off1(uint32_t(col), P.gn) + int64_t(rl) * P.sCm;
                        const int rmax = P.M - rl;
#pragma unroll
                        for (int i = 0; i < FM; ++i)
                            if (i * 16 < rmax) cp[int64_t(i * 16) * P.sCm] = acc[i][j][r];
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int s = 0; s < KS; ++s) ycur[j][s] = ynxt[j][s];
    }
}

// Row-streaming TTM for C strided along j (see TtmRowParams).  B (M x K,
// zero-padded to 16-row blocks and the MFMA k-step) is staged in LDS once per
// workgroup; each of the four waves then walks its own (run, chunk) units: it
// loads the chunk's A fragments (16*FN columns, all k) into registers and, for
// every 16-row block of C, runs the MFMAs, stages the block in its own LDS rows
// and writes them back as whole 64-column windows (or, in band mode, as one
// linear range).  Stores are raw buffer stores whose lanes outside the run or
// past the last row get an out-of-range offset, which the buffer's range
// check drops: the store sequence has no branches.  (Software-pipelining the
// MFMAs of the next row block into the stores of this one, with or without
// scheduling barriers, measured no faster on MI355X.)
template <typename TI, int FN, int KS, int MODE>
__global__ __launch_bounds__(256) void ttm_rows_kernel(TtmRowParams P) {
    using TA = typename AccOf<TI>::type;
    using acc_t = typename SMfma<TI>::acc_t;
    using frag_t = typename SMfma<TI>::frag_t;
    constexpr bool WIDE = sizeof(TI) == 2;
    constexpr bool F64 = std::is_same<TI, double>::value;
    constexpr int KSTEP = SMfma<TI>::KSTEP;
    constexpr int KP = KS * KSTEP;
    constexpr int RQ = F64 ? 1 : 4;  // result row of (kq, r): RQ*kq + RR*r
    constexpr int RR = F64 ? 4 : 1;
    constexpr int W = 64;                       // written columns per row window
    constexpr int L = 128 / int(sizeof(TA));    // elements of C per 128-byte line
    constexpr int SR = F64 ? 4 : 16;            // rows staged per pass (one result register for FP64)
    constexpr int SP = FN * 16 + 2;              // FP64 staging: row pitch
    constexpr int SPC = 20;                      // FP32 staging: column pitch (16-byte aligned)
    constexpr int STG = F64 ? SR * SP : FN * 16 * SPC;  // staged elements per wave
    constexpr bool BAND = MODE == TTM_ROWS_BAND || MODE == TTM_ROWS_BAND1 || MODE == TTM_ROWS_BANDW;
    constexpr uint32_t OOB = 0x80000000u;       // buffer offset past every range: store dropped
    using RT = typename std::conditional<WIDE, uint16_t, TI>::type;
    static_assert(MODE != TTM_ROWS_ALIGNED || FN * 16 >= W + L, "aligned windows need W + L staged columns");
    static_assert(MODE != TTM_ROWS_PLAIN || FN * 16 >= W, "plain windows need W staged columns");

    extern __shared__ __align__(16) unsigned char smem[];
    // wave index through readfirstlane, so that everything derived from it
    // (unit, run, chunk) is known to be wave-uniform
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rl = lane & 15, kq = lane >> 4;
    // Row groups: with P.nrg > 1 each workgroup serves the P.mr rows
    // [rg*mr, rg*mr + mr) of B and C, so that B's slice fits in LDS.  The
    // grid is a multiple of 8*nrg; the nrg workgroups that share a block
    // index for the walk sit on one XCD and read the same A chunks through
    // its L2.
    const int rg = P.nrg > 1 ? int(blockIdx.x / 8) % P.nrg : 0;
    const int wblk = P.nrg > 1 ? int(blockIdx.x / (8 * P.nrg)) * 8 + int(blockIdx.x % 8) : int(blockIdx.x);
    const int wgrid = P.nrg > 1 ? int(gridDim.x) / P.nrg : int(gridDim.x);
    const int row0 = rg * P.mr;                          // first row of B / C served here
    const int M16 = (min(P.M - row0, P.mr) + 15) & ~15;  // rows staged, padded to 16
    const int PB = WIDE ? (KP + 8) : (M16 + (F64 ? 4 : 16));
    RT* Bs = reinterpret_cast<RT*>(smem);
    const int bbytes = ((WIDE ? M16 * PB : KP * PB) * int(sizeof(RT)) + 15) & ~15;
    TA* stg = reinterpret_cast<TA*>(smem + bbytes) + wave * STG;
    // FP32 staging in the plain and band-wide modes puts row r of column c at
    // position r ^ ((c >> 4) & 3) of the column: the four columns c, c+16,
    // c+32, c+48 whose pitch-20 starts share a bank quad then hold a given
    // row on four different banks, so a read of one row across 64
    // consecutive columns is free of conflicts.  (In the aligned and narrow
    // band modes the extra address arithmetic measured slower than the
    // conflicts it removes.)
    constexpr bool SWZ = !F64 && (MODE == TTM_ROWS_PLAIN || MODE == TTM_ROWS_BANDW);
    auto stage_at = [&](int row, int col) -> TA {
        return F64 ? stg[row * SP + col] : stg[col * SPC + (SWZ ? row ^ ((col >> 4) & 3) : row)];
    };
    const TI* X = (const TI*)P.X;
    const TI* Y = (const TI*)P.Y;
    TA* C = (TA*)P.C;

    for (int e = tid; e < M16 * KP; e += 256) {
        int m, k;
        if constexpr (WIDE) { m = e / KP; k = e - m * KP; }
        else { k = e / M16; m = e - k * M16; }
        RT v = RT(0);
        if (row0 + m < P.M && k < P.K) {
            const TI* src = X + int64_t(row0 + m) * P.sXm + int64_t(k) * P.sXk;
            if constexpr (WIDE) v = uint16_t(raw16(src));
            else v = *src;
        }
        if constexpr (WIDE) Bs[m * PB + k] = v;
        else Bs[k * PB + m] = v;
    }
    __syncthreads();

    // unit u -> run h (A and C offsets of its first element), chunk t and the
    // first staged column c0
    auto unit_pos = [&](int64_t u, int64_t& ya, int64_t& yc, int& t, int& c0) {
        const uint32_t uu = uint32_t(u);
        const uint32_t h = fdiv(uu, P.fd_tc);
        t = int(uu - h * uint32_t(P.Tc));
        grp_decode(h, P.gh, ya, yc);
        c0 = MODE == TTM_ROWS_ALIGNED ? W * t - L : MODE == TTM_ROWS_PLAIN ? W * t : 0;
    };
    frag_t ycur[FN][KS];
    auto load_y = [&](int64_t u, frag_t (&y)[FN][KS]) {
        int64_t ya, yc;
        int t, c0;
        unit_pos(u, ya, yc, t, c0);
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = c0 + j * 16 + rl;
            const bool cv = col >= 0 && col < P.n_lo;
            const int64_t yo = ya + int64_t(min(max(col, 0), P.n_lo - 1)) * P.sYlo;
            load_frags<TI, KS>(Y + yo, P.sYk, P.K, cv, kq, y[j]);
        }
    };
    // MFMAs of one 16-row block, one k-step at a time.  Every column block
    // runs (blocks outside the run hold zero fragments: a conditional MFMA
    // costs more in register copies of the accumulators than the MFMA
    // itself).
    auto mfma_step = [&](int i, int s, acc_t (&acc)[FN]) {
        const int ib = i;
        if (s == 0) {
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[j] = acc_t{};
        }
        frag_t b;
        if constexpr (WIDE) b = *reinterpret_cast<const u4s_t*>(&Bs[(ib * 16 + rl) * PB + s * 32 + 8 * kq]);
        else b = Bs[(s * KSTEP + kq) * PB + ib * 16 + rl];
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[j] = smfma<TI>(b, ycur[j][s], acc[j]);
    };
    // Stage and store one 16-row block in four pieces of four rows.  The
    // buffer range of the block covers its rows below M and the run's
    // columns; every other lane's offset is out of range.
    constexpr int NPC = 4;
    auto store_piece = [&](int i, int pc, const acc_t (&acc)[FN], int64_t yc, int t, int c0) {
        const int j0 = row0 + i * 16;
        const int nrows = max(0, min(16, P.M - j0));
        TA* base = C + yc + int64_t(j0) * P.sCm;
        // Every lane also checks its row against nrows: with m = 1 the stride
        // of j is arbitrary, so rows past the last one can land inside the
        // range.  The range then only backs up the lane predicates.
        const uint32_t live = nrows > 0 ? 0xffffffffu : 0u;
        const uint32_t nbytes =
            live & (BAND ? uint32_t(nrows * P.n_lo) * uint32_t(sizeof(TA))
                         : uint32_t((int64_t(nrows - 1) * P.sCm + int64_t(P.n_lo - 1) * P.sClo + 1) *
                                    int64_t(sizeof(TA))));
        const __amdgpu_buffer_rsrc_t rs = wave_rsrc(base, nbytes);
        // Stage layout: FP64 row-major, the four rows kq of result register
        // pc; FP32 column-major with the four rows 4kq..4kq+3 of a result
        // register written as one 16-byte vector (permuted as stage_at reads
        // it: column j*16+rl has (c >> 4) & 3 == j & 3), all sixteen rows at
        // piece 0.
        // (Row-major FP32 staging with scalar stores was miscompiled by hipcc
        // for gfx950: two stores merged into a ds_write2_b32 with a wrong
        // first offset.)
        if (F64 || pc == 0) {
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                if constexpr (F64) stg[kq * SP + j * 16 + rl] = acc[j][pc];
                else *reinterpret_cast<f4s_t*>(&stg[(j * 16 + rl) * SPC + 4 * kq]) = swz4(acc[j], SWZ ? j & 3 : 0);
            }
        }
        const int r0 = F64 ? 0 : 4 * pc;  // first staged row of this piece
        auto put = [&](TA v, bool ok, uint32_t byte_off) {
            const uint32_t off = ok ? byte_off : OOB;
            if constexpr (F64)
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2s_t, v), rs, int(off), 0, 0);
            else
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, int(off), 0, 0);
        };
        if constexpr (BAND) {
            // rows 4pc .. 4pc+3 of the block are one linear range
            const int e0 = 4 * pc * P.n_lo;
#pragma unroll
            for (int it = 0; it < (4 * 16 * FN + 63) / 64; ++it) {
                const int e = it * 64 + lane;
                const int rr = int(fdiv(uint32_t(e), P.fd_lo));
                const bool ok = e < 4 * P.n_lo && 4 * pc + rr < nrows;
                const TA v = stage_at(ok ? r0 + rr : 0, ok ? e - rr * P.n_lo : 0);
                put(v, ok, uint32_t(e0 + e) * uint32_t(sizeof(TA)));
            }
        } else {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int jr = 4 * pc + rr;  // row within the block
                int ws = W * t;
                if constexpr (MODE == TTM_ROWS_ALIGNED)
                    ws -= int((reinterpret_cast<uintptr_t>(base + int64_t(jr) * P.sCm) & 127) / sizeof(TA));
                const int col = ws + lane;
                const bool ok = col >= 0 && col < P.n_lo && jr < nrows;
                const TA v = stage_at(r0 + rr, ok ? col - c0 : 0);
                put(v, ok, uint32_t((int64_t(jr) * P.sCm + int64_t(col) * P.sClo) * int64_t(sizeof(TA))));
            }
        }
    };
    // FP32 results of the aligned and band modes: a whole 16-row block is
    // staged once and written with 16-byte stores (each lane four
    // consecutive elements of a row window or of the block's linear range),
    // a quarter of the store instructions of the piece-wise path.  It takes
    // blocks of 16 rows whose windows lie inside the run (aligned: not the
    // first or last chunk; each window starts on a 128-byte line by design)
    // or whose linear range starts 16-byte aligned (band); other blocks go
    // the piece-wise way.
    constexpr bool VBLK = !F64 && MODE != TTM_ROWS_PLAIN;
    auto store_block_vec = [&](int i, const acc_t (&acc)[FN], int64_t yc, int t, int c0) -> bool {
      if constexpr (!VBLK) {
        return false;
      } else {
        const int j0 = row0 + i * 16;
        const int nrows = max(0, min(16, P.M - j0));
        TA* base = C + yc + int64_t(j0) * P.sCm;
        // whole blocks only: 16 rows, and (band) a 16-byte aligned range or
        // (aligned windows) every row's window inside the run
        if (nrows < 16) return false;
        if (BAND && (reinterpret_cast<uintptr_t>(base) & 15) != 0) return false;
        if (!BAND && (t == 0 || W * t + W > P.n_lo)) return false;
        const uint32_t live = nrows > 0 ? 0xffffffffu : 0u;
        const uint32_t nbytes =
            live & (BAND ? uint32_t(nrows * P.n_lo) * uint32_t(sizeof(TA))
                         : uint32_t((int64_t(nrows - 1) * P.sCm + int64_t(P.n_lo - 1) * P.sClo + 1) *
                                    int64_t(sizeof(TA))));
        const __amdgpu_buffer_rsrc_t rs = wave_rsrc(base, nbytes);
#pragma unroll
        for (int j = 0; j < FN; ++j)
            *reinterpret_cast<f4s_t*>(&stg[(j * 16 + rl) * SPC + 4 * kq]) = swz4(acc[j], SWZ ? j & 3 : 0);
        // four elements at byte offset off, all inside or all outside the
        // range (lanes past its end get an out-of-range offset)
        auto put4 = [&](const f4s_t& v, bool ok, uint32_t off) {
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4s_t, v), rs, int(ok ? off : OOB), 0, 0);
        };
        if constexpr (BAND) {
            constexpr int MAXLEN = 16 * (MODE == TTM_ROWS_BAND1 ? 16 : MODE == TTM_ROWS_BAND ? 32 : 176);
            const int len = nrows * P.n_lo;
#pragma unroll
            for (int it = 0; it < (MAXLEN + 255) / 256; ++it) {
                // len = 16 n_lo is a multiple of 4: a lane's four are all in or all out
                const int e = it * 256 + 4 * lane;
                const bool ok = e < len;
                int r = int(fdiv(uint32_t(ok ? e : 0), P.fd_lo));
                int c = (ok ? e : 0) - r * P.n_lo;
                f4s_t v;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    v[u] = stage_at(r, c);
                    if (++c == P.n_lo) {
                        c = 0;
                        ++r;
                    }
                }
                put4(v, ok, uint32_t(e) * uint32_t(sizeof(TA)));
            }
        } else {
            // 16 lanes per row window, four rows per pass
            const int rq = lane >> 4, qq = lane & 15;
#pragma unroll
            for (int pc = 0; pc < 4; ++pc) {
                const int jr = 4 * pc + rq;
                const int ws = W * t - int((reinterpret_cast<uintptr_t>(base + int64_t(jr) * P.sCm) & 127) / sizeof(TA));
                const int col = ws + 4 * qq;  // inside the run: checked above
                f4s_t v;
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = stage_at(jr, col + u - c0);
                put4(v, true, uint32_t((int64_t(jr) * P.sCm + col) * int64_t(sizeof(TA))));
            }
        }
        return true;
      }
    };
    Walk wk = xcd_walk(P.units, 4, wave, wblk, wgrid);
    const int nb = M16 / 16;
    for (; wk.u < wk.end; wk.u += wk.step) {
        load_y(wk.u, ycur);
        int64_t ya, yc;
        int t, c0;
        unit_pos(wk.u, ya, yc, t, c0);
        acc_t acc[FN];
        for (int i = 0; i < nb; ++i) {
#pragma unroll
            for (int q = 0; q < KS; ++q) mfma_step(i, q, acc);
            bool done = false;
            if constexpr (VBLK) done = store_block_vec(i, acc, yc, t, c0);
            if (!done) {
#pragma unroll
                for (int q = 0; q < NPC; ++q) store_piece(i, q, acc, yc, t, c0);
            }
        }
    }
}

// ------------------------------------------------------------------ launch

template <typename TI, int FM, int FN, int KS>
static int stream_launch(const TtmParams& p, int grid, hipStream_t s) {
    constexpr bool WIDE = sizeof(TI) == 2;
    constexpr int KP = KS * SMfma<TI>::KSTEP;
    constexpr int M16 = FM * 16;
    constexpr int PB = WIDE ? (KP + 8) : (M16 + (sizeof(TI) == 8 ? 4 : 16));
    const size_t lds = size_t(WIDE ? M16 * PB : KP * PB) * (WIDE ? 2 : sizeof(TI));
    // gfx950 gives a workgroup up to 160 KB of LDS; above 64 KB the kernel
    // has to ask for it
    if (lds > 65536 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&ttm_stream_kernel<TI, FM, FN, KS>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)) != hipSuccess)
        return TLIB_EHIP;
    hipLaunchKernelGGL((ttm_stream_kernel<TI, FM, FN, KS>), dim3(grid), dim3(256), lds, s, p);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

// Dispatch over (FM, KS).  KS (k-steps) is rounded up to one of the
// instantiated depths by the planner.  fm: total row blocks (1, 4 or 16), all
// owned by each wave; FN column blocks per wave keep the accumulators at 64
// values per lane.
template <typename TI, int FM>
static int stream_fm(const TtmParams& p, int ks, int grid, hipStream_t s) {
    constexpr int FN = FM >= 16 ? 1 : FM >= 4 ? 2 : 4;
#define TLIB_KS_CASE(K) \
    case K: return stream_launch<TI, FM, FN, K>(p, grid, s);
    if constexpr (sizeof(TI) == 2) {
        switch (ks) {
            TLIB_KS_CASE(1)
            TLIB_KS_CASE(2)
        }
    } else {
        switch (ks) {
            TLIB_KS_CASE(1)
            TLIB_KS_CASE(2)
            TLIB_KS_CASE(3)
            TLIB_KS_CASE(4)
            TLIB_KS_CASE(5)
            TLIB_KS_CASE(6)
            TLIB_KS_CASE(8)
            TLIB_KS_CASE(10)
            TLIB_KS_CASE(12)
            TLIB_KS_CASE(16)
        }
    }
#undef TLIB_KS_CASE
    return TLIB_EINVAL;
}

int ttm_stream_ks(int dtype, int k) {
    if (dtype == TLIB_BF16 || dtype == TLIB_F16) return k <= 32 ? 1 : k <= 64 ? 2 : 0;
    const int ks = (k + 3) / 4;
    static const int depths[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};
    for (int d : depths)
        if (ks <= d) return d;
    return 0;
}

template <typename TI>
static int stream_dispatch(const TtmParams& p, int fm, int ks, int grid, hipStream_t s) {
    switch (fm) {
        case 1: return stream_fm<TI, 1>(p, ks, grid, s);
        case 4: return stream_fm<TI, 4>(p, ks, grid, s);
        default: return stream_fm<TI, 16>(p, ks, grid, s);
    }
}

int launch_ttm_stream(int dtype, const TtmParams& p, int fm, int ks, bool trans, int grid, hipStream_t s) {
    if (!trans) return TLIB_EINVAL;  // C strided along j: launch_ttm_rows
    switch (dtype) {
        case TLIB_F64: return stream_dispatch<double>(p, fm, ks, grid, s);
        case TLIB_F32: return stream_dispatch<float>(p, fm, ks, grid, s);
        case TLIB_BF16: return stream_dispatch<bf16_t>(p, fm, ks, grid, s);
        case TLIB_F16: return stream_dispatch<f16_t>(p, fm, ks, grid, s);
    }
    return TLIB_EDTYPE;
}

// Row-streaming kernel: staged column blocks per mode.
template <typename TI> constexpr int rows_fn(int mode) {
    return mode == TTM_ROWS_ALIGNED ? (64 + 128 / int(sizeof(typename AccOf<TI>::type))) / 16
           : mode == TTM_ROWS_PLAIN ? 4
           : mode == TTM_ROWS_BAND  ? 2
           : mode == TTM_ROWS_BANDW ? 11
                                    : 1;
}

template <typename TI>
static int64_t rows_lds(int mode, int m, int ks) {
    using TA = typename AccOf<TI>::type;
    constexpr bool WIDE = sizeof(TI) == 2;
    constexpr bool F64 = std::is_same<TI, double>::value;
    const int kp = ks * SMfma<TI>::KSTEP;
    const int m16 = (m + 15) & ~15;
    const int pb = WIDE ? (kp + 8) : (m16 + (F64 ? 4 : 16));
    const int64_t bbytes = (int64_t(WIDE ? m16 * pb : kp * pb) * (WIDE ? 2 : int(sizeof(TI))) + 15) & ~int64_t(15);
    const int fn = rows_fn<TI>(mode);
    const int stg = F64 ? 4 * (fn * 16 + 2) : fn * 16 * 20;  // per wave, as in ttm_rows_kernel
    return bbytes + int64_t(4) * stg * int64_t(sizeof(TA));
}

int64_t ttm_rows_lds(int dtype, int mode, int m, int ks) {
    switch (dtype) {
        case TLIB_F64: return rows_lds<double>(mode, m, ks);
        case TLIB_F32: return rows_lds<float>(mode, m, ks);
        default: return rows_lds<bf16_t>(mode, m, ks);
    }
}

// k-step depths instantiated for the row kernel: aligned windows keep
// FN * KS <= 36 fragments in registers.
int ttm_rows_ks(int dtype, int mode, int k) {
    if (dtype == TLIB_BF16 || dtype == TLIB_F16) {
        if (mode == TTM_ROWS_BANDW) return 0;
        return k <= 32 ? 1 : k <= 64 ? 2 : 0;
    }
    const int ks = (k + 3) / 4;
    static const int depths[] = {1, 2, 3, 4, 5, 6, 8, 10};
    const int cap = mode == TTM_ROWS_ALIGNED ? 6 : mode == TTM_ROWS_BANDW ? 4 : 10;
    for (int d : depths)
        if (ks <= d) return d <= cap ? d : 0;
    return 0;
}

template <typename TI, int MODE, int KS>
static int rows_launch(const TtmRowParams& p, int grid, hipStream_t s) {
    constexpr int FN = rows_fn<TI>(MODE);
    const size_t lds = size_t(rows_lds<TI>(MODE, p.mr, KS));
    hipLaunchKernelGGL((ttm_rows_kernel<TI, FN, KS, MODE>), dim3(grid), dim3(256), lds, s, p);
    return hipGetLastError() == hipSuccess ? TLIB_OK : TLIB_EHIP;
}

template <typename TI, int MODE>
static int rows_ks(const TtmRowParams& p, int ks, int grid, hipStream_t s) {
#define TLIB_KS_CASE(K) \
    case K: return rows_launch<TI, MODE, K>(p, grid, s);
    if constexpr (sizeof(TI) == 2) {
        if constexpr (MODE != TTM_ROWS_BANDW) {
            switch (ks) {
                TLIB_KS_CASE(1)
                TLIB_KS_CASE(2)
            }
        }
    } else if constexpr (MODE == TTM_ROWS_BANDW) {
        switch (ks) {
            TLIB_KS_CASE(1)
            TLIB_KS_CASE(2)
            TLIB_KS_CASE(3)
            TLIB_KS_CASE(4)
        }
    } else if constexpr (MODE == TTM_ROWS_ALIGNED) {
        switch (ks) {
            TLIB_KS_CASE(1)
            TLIB_KS_CASE(2)
            TLIB_KS_CASE(3)
            TLIB_KS_CASE(4)
            TLIB_KS_CASE(5)
            TLIB_KS_CASE(6)
        }
    } else {
        switch (ks) {
            TLIB_KS_CASE(1)
            TLIB_KS_CASE(2)
            TLIB_KS_CASE(3)
            TLIB_KS_CASE(4)
            TLIB_KS_CASE(5)
            TLIB_KS_CASE(6)
            TLIB_KS_CASE(8)
            TLIB_KS_CASE(10)
        }
    }
#undef TLIB_KS_CASE
    return TLIB_EINVAL;
}

template <typename TI>
static int rows_mode(const TtmRowParams& p, int mode, int ks, int grid, hipStream_t s) {
    switch (mode) {
        case TTM_ROWS_PLAIN: return rows_ks<TI, TTM_ROWS_PLAIN>(p, ks, grid, s);
        case TTM_ROWS_ALIGNED: return rows_ks<TI, TTM_ROWS_ALIGNED>(p, ks, grid, s);
        case TTM_ROWS_BAND: return rows_ks<TI, TTM_ROWS_BAND>(p, ks, grid, s);
        case TTM_ROWS_BAND1: return rows_ks<TI, TTM_ROWS_BAND1>(p, ks, grid, s);
        case TTM_ROWS_BANDW: return rows_ks<TI, TTM_ROWS_BANDW>(p, ks, grid, s);
    }
    return TLIB_EINVAL;
}

int launch_ttm_rows(int dtype, const TtmRowParams& p, int mode, int ks, int grid, hipStream_t s) {
    switch (dtype) {
        case TLIB_F64: return rows_mode<double>(p, mode, ks, grid, s);
        case TLIB_F32: return rows_mode<float>(p, mode, ks, grid, s);
        case TLIB_BF16: return rows_mode<bf16_t>(p, mode, ks, grid, s);
        case TLIB_F16: return rows_mode<f16_t>(p, mode, ks, grid, s);
    }
    return TLIB_EDTYPE;
}

}  // namespace tlib
