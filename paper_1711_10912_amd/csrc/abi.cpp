// C-ABI entry points and host planner.
//
// Every entry point validates its descriptors, derives strides from layouts
// (Sec. 3.1 Eq. stride.tuple.permutation), checks shapes against the defining
// equation, then collapses the problem: dims of extent 1 are dropped and
// neighbouring dims whose strides chain for every operand are merged, which
// turns any dense layout into at most a few (extent, stride) pairs.  The
// collapsed problem picks the kernel: TTV by its (lo, k, hi) regime, TTM/TTT
// as one GEMM whose operands are addressed through per-group strides (no
// unfolding, no transposed copy), inner/norm and add/scale/transpose as
// streaming passes.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <string>
#include <utility>
#include <vector>

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace tlib {

// ------------------------------------------------------------------ thread-local state

static thread_local std::string g_err;
static thread_local std::string g_plan;
static thread_local bool g_plan_only = false;

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

static void plan_note(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_plan = buf;
}

static const char* dname(int dt) {
    switch (dt) {
        case TLIB_F64: return "f64";
        case TLIB_F32: return "f32";
        case TLIB_BF16: return "bf16";
        case TLIB_F16: return "f16";
    }
    return "?";
}

// ------------------------------------------------------------------ helpers

FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d ? d : 1;
    uint32_t s = 0;
    while ((uint64_t(1) << s) < f.d) ++s;
    f.s = s;
    f.m = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << s) - f.d)) / f.d + 1);
    return f;
}

int coalesce(Dim* d, int nd, int nops, int key) {
    int k = 0;
    for (int i = 0; i < nd; ++i)
        if (d[i].n != 1) d[k++] = d[i];
    nd = k;
    std::stable_sort(d, d + nd, [key, nops](const Dim& a, const Dim& b) {
        if (a.s[key] != b.s[key]) return a.s[key] < b.s[key];
        for (int o = 0; o < nops; ++o)
            if (a.s[o] != b.s[o]) return a.s[o] < b.s[o];
        return false;
    });
    int out = 0;
    for (int i = 0; i < nd; ++i) {
        if (out > 0) {
            Dim& prev = d[out - 1];
            bool chain = true;
            for (int o = 0; o < nops; ++o)
                if (d[i].s[o] != prev.s[o] * prev.n) chain = false;
            if (chain) {
                prev.n *= d[i].n;
                continue;
            }
        }
        d[out++] = d[i];
    }
    return out;
}

TileShape tile_shape(int t) {
    switch (t) {
        case GT_16x256: return {16, 256};
        case GT_64x128: return {64, 128};
        case GT_128x128: return {128, 128};
        case GT_256x64: return {256, 64};
        case GT_128x64: return {128, 64};
        case GT_256x32: return {256, 32};
        default: return {64, 64};
    }
}

static bool fill_grp(Grp& g, const Dim* d, int nd, int o0, int o1) {
    if (nd > GMAXD) return false;
    g = Grp();
    g.nd = nd;
    g.total = 1;
    for (int i = 0; i < nd; ++i) {
        g.n[i] = d[i].n;
        g.s0[i] = d[i].s[o0];
        g.s1[i] = d[i].s[o1];
        g.fd[i] = make_fastdiv(uint32_t(d[i].n));
        g.total *= d[i].n;
    }
    return g.total < (int64_t(1) << 31);
}

static void fill_gdims(GDims& g, const Dim* d, int nd, int nops) {
    g = GDims();
    g.nd = nd;
    g.total = 1;
    for (int i = 0; i < nd; ++i) {
        g.n[i] = d[i].n;
        for (int o = 0; o < nops; ++o) g.s[o][i] = d[i].s[o];
        g.total *= d[i].n;
    }
}

static int normalize(const tlib_tensor* t, Ten& o, const char* name) {
    if (!t) return fail(TLIB_EINVAL, "%s is NULL", name);
    if (t->order < 0 || t->order > MAXP)
        return fail(TLIB_EINVAL, "%s: order %d out of range 0..%d", name, t->order, MAXP);
    if (t->dtype < TLIB_F64 || t->dtype > TLIB_F16)
        return fail(TLIB_EDTYPE, "%s: unknown dtype %d", name, t->dtype);
    if (!t->data) return fail(TLIB_EINVAL, "%s: data pointer is NULL", name);
    if (t->order > 0 && !t->extents) return fail(TLIB_EINVAL, "%s: extents is NULL", name);
    o.data = t->data;
    o.dtype = t->dtype;
    o.p = t->order;
    for (int r = 0; r < o.p; ++r) {
        if (t->extents[r] < 1) return fail(TLIB_EINVAL, "%s: extent n_%d = %lld < 1", name, r + 1,
                                           (long long)t->extents[r]);
        o.n[r] = t->extents[r];
    }
    if (t->strides) {
        for (int r = 0; r < o.p; ++r) {
            if (t->strides[r] < 0)
                return fail(TLIB_EINVAL, "%s: stride w_%d < 0", name, r + 1);
            o.w[r] = t->strides[r];
        }
    } else {
        int32_t pi[MAXP];
        for (int r = 0; r < o.p; ++r) pi[r] = t->layout ? t->layout[r] : r + 1;
        bool seen[MAXP] = {};
        for (int r = 0; r < o.p; ++r) {
            if (pi[r] < 1 || pi[r] > o.p || seen[pi[r] - 1])
                return fail(TLIB_EMODE, "%s: layout is not a permutation of 1..%d", name, o.p);
            seen[pi[r] - 1] = true;
        }
        // Eq. stride.tuple.permutation: w_{pi_1} = 1, w_{pi_r} = prod_{q<r} n_{pi_q}
        int64_t acc = 1;
        for (int r = 0; r < o.p; ++r) {
            o.w[pi[r] - 1] = acc;
            acc *= o.n[pi[r] - 1];
        }
    }
    // the largest element offset must fit comfortably in 62 bits
    long double span = 0;
    for (int r = 0; r < o.p; ++r) span += (long double)(o.n[r] - 1) * (long double)o.w[r];
    if (span > 4.0e18L) return fail(TLIB_EINVAL, "%s: address range too large", name);
    return TLIB_OK;
}

// Sufficient condition for distinct addresses: sorted by stride, every
// stride is at least the previous stride times its extent.
static bool injective(const Ten& t) {
    Dim d[MAXP];
    int nd = 0;
    for (int r = 0; r < t.p; ++r)
        if (t.n[r] > 1) d[nd++] = {t.n[r], {t.w[r], 0, 0}};
    std::sort(d, d + nd, [](const Dim& a, const Dim& b) { return a.s[0] < b.s[0]; });
    int64_t need = 1;
    for (int i = 0; i < nd; ++i) {
        if (d[i].s[0] < need) return false;
        need = d[i].s[0] * d[i].n;
    }
    return true;
}

static void span(const Ten& t, uintptr_t& lo, uintptr_t& hi) {
    int64_t last = 0;
    for (int r = 0; r < t.p; ++r) last += (t.n[r] - 1) * t.w[r];
    lo = uintptr_t(t.data);
    hi = lo + uintptr_t((last + 1) * esize(t.dtype));
}

static bool overlaps(const Ten& a, const Ten& b) {
    uintptr_t a0, a1, b0, b1;
    span(a, a0, a1);
    span(b, b0, b1);
    return a0 < b1 && b0 < a1;
}

static bool same_view(const Ten& a, const Ten& b) {
    if (a.data != b.data || a.p != b.p || a.dtype != b.dtype) return false;
    for (int r = 0; r < a.p; ++r)
        if (a.n[r] != b.n[r] || (a.n[r] > 1 && a.w[r] != b.w[r])) return false;
    return true;
}

static int check_output(const Ten& c, const char* name) {
    if (!injective(c))
        return fail(TLIB_ESTRIDE, "%s: strides may map two multi-indices to one address", name);
    return TLIB_OK;
}

// ------------------------------------------------------------------ workspace
//
// One device buffer per (device, stream) holds reduction and split-K
// partials and the intermediate of a two-TTM chain.  Calls on one stream run
// in stream order, so every call may use the whole buffer from its start.
// The buffer is allocated by tlib_workspace_reserve, or by the first call on
// the stream that needs scratch while the stream is not capturing (then to
// max(need, TLIB_WORKSPACE_DEFAULT_BYTES)).  Entry points never free, grow or
// wait on it: a call that needs more than the buffer holds fails with
// TLIB_ENOMEM before launching anything.  A buffer replaced by a larger
// reserve is kept until tlib_workspace_release, so graphs captured with it
// stay valid.

namespace {
struct WsBuf {
    char* ptr = nullptr;
    size_t bytes = 0;
    std::vector<void*> retired;  // replaced buffers, freed by tlib_workspace_release
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, WsBuf> g_ws;

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}
}  // namespace

static constexpr size_t WS_ALIGN = 256;
static size_t ws_round(size_t b) { return (b + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }

static void* ws_alloc(size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void* WsCtx::take(size_t bytes) {
    bytes = ws_round(bytes);
    if (bytes == 0) return base ? base + used : nullptr;
    if (!base) {
        if (fixed) return nullptr;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return nullptr;
        std::lock_guard<std::mutex> lk(g_ws_mu);
        WsBuf& e = g_ws[{dev, s}];
        if (!e.ptr) {
            if (capturing(s)) return nullptr;  // no allocation while a graph is captured
            const size_t want = std::max({ws_round(hint), used + bytes, size_t(TLIB_WORKSPACE_DEFAULT_BYTES)});
            void* p = ws_alloc(want);
            if (!p) return nullptr;
            e.ptr = static_cast<char*>(p);
            e.bytes = want;
        }
        base = e.ptr;
        size = e.bytes;
    }
    if (used + bytes > size) return nullptr;
    void* p = base + used;
    used += bytes;
    return p;
}

// Record the scratch a planned launch takes (plan-only probes read it).
void WsCtx::need(size_t bytes) { peak = std::max(peak, used + ws_round(bytes)); }

static int ws_fail(const WsCtx& ws, size_t bytes, const char* op) {
    if (ws.fixed)
        return fail(TLIB_ENOMEM, "%s: needs %zu bytes of scratch beyond the %zu of the static buffer", op, bytes,
                    ws.size - ws.used);
    return fail(TLIB_ENOMEM,
                "%s: needs %zu bytes of workspace at offset %zu; the stream's workspace holds %zu bytes (reserve "
                "more with tlib_workspace_reserve before the call, outside graph capture)",
                op, bytes, ws.used, ws.size);
}

// ------------------------------------------------------------------ launch records
//
// Planning a TTV / TTM / TTT call ends in a Launch: the kernel, its parameter
// block and launch shape, the scratch it takes and the plan text, with the
// operand pointers left to be filled in.  exec_launch fills them in and
// launches.  Records are cached per call shape (plan cache below), so a
// repeated shape skips planning.

enum LaunchKind {
    LK_NONE = 0, LK_TTV_COLW, LK_TTV_COL, LK_TTV_SLAB, LK_TTV_FIBER, LK_TTV_GENERIC,
    LK_GEMM, LK_GEMM_GENERIC, LK_TTM_STREAM, LK_TTM_ROWS, LK_OUTER, LK_GEMM_ROWS
};

struct Launch {
    int kind = LK_NONE;
    int dtype = 0;
    int i0 = 0, i1 = 0, i2 = 0;  // kernel-specific: vec/ks/kr, slabs/kc, G, tile, fm/mode, ks, grid
    int xsrc = 0;                // GEMM: X is operand 0 (A) or 1 (B / b) of the call
    size_t wsb = 0;              // scratch bytes taken from the call's workspace
    size_t xwsb = 0;             // GEMM: bytes of X packed into the workspace (gd[0]: the copy), or 0
    const char* op = "";
    TtvParams ttv{};
    Grp go{};
    GDims gd[3]{};
    GemmParams gemm{};
    TtmParams tstr{};
    TtmRowParams trow{};
    OuterParams outer{};
    std::string note;
};

// in0 = A, in1 = b / B, out = C
static int exec_launch(const Launch& L, const void* in0, const void* in1, void* out, WsCtx& ws, hipStream_t s) {
    ws.need(L.xwsb ? ws_round(L.wsb) + L.xwsb : L.wsb);
    if (g_plan_only) return TLIB_OK;
    void* w = nullptr;
    if (L.wsb) {
        w = ws.take(L.wsb);
        if (!w) return ws_fail(ws, L.wsb, L.op);
    }
    // GEMM with a packed X: copy X (gd[0]: its strides, the packed ones) into
    // the workspace first
    const void* xpk = nullptr;
    if (L.xwsb) {
        void* xp = ws.take(L.xwsb);
        if (!xp) return ws_fail(ws, ws_round(L.wsb) + L.xwsb, L.op);
        const int prc = launch_axpby(L.dtype, L.dtype, 1.0, L.xsrc ? in1 : in0, 0.0, nullptr, xp, L.gd[0], s);
        if (prc) return fail(prc, "%s: packing X failed", L.op);
        xpk = xp;
    }
    int rc = TLIB_EHIP;
    if (L.kind >= LK_TTV_COLW && L.kind <= LK_TTV_GENERIC) {
        TtvParams P = L.ttv;
        P.A = in0;
        P.b = in1;
        P.C = out;
        switch (L.kind) {
            case LK_TTV_COLW: rc = launch_ttv_colw(L.dtype, P, L.i0, L.i1, s); break;
            case LK_TTV_COL: rc = launch_ttv_col(L.dtype, P, L.i0, L.i1, w, s); break;
            case LK_TTV_SLAB: rc = launch_ttv_slab(L.dtype, P, L.i0, L.i1, s); break;
            case LK_TTV_FIBER: rc = launch_ttv_fiber(L.dtype, P, L.go, L.i0, s); break;
            default: rc = launch_ttv_generic(L.dtype, P, L.gd[0], s); break;
        }
    } else if (L.kind == LK_GEMM) {
        GemmParams P = L.gemm;
        P.X = xpk ? xpk : L.xsrc ? in1 : in0;
        P.Y = L.xsrc ? in0 : in1;
        P.C = out;
        P.part = w;
        rc = launch_gemm(L.dtype, L.i0, P, s);
    } else if (L.kind == LK_GEMM_ROWS) {
        GemmParams P = L.gemm;
        P.X = xpk ? xpk : L.xsrc ? in1 : in0;
        P.Y = L.xsrc ? in0 : in1;
        P.C = out;
        P.part = w;
        rc = launch_gemm_rows(L.dtype, L.i0, L.i1, P, s);
        if (rc == TLIB_OK && P.ksplit > 1) rc = launch_gemm_ksum(acc_dtype(L.dtype), P, s);
    } else if (L.kind == LK_GEMM_GENERIC) {
        rc = launch_gemm_generic(L.dtype, L.xsrc ? in1 : in0, L.xsrc ? in0 : in1, out, L.gd[0], L.gd[1], L.gd[2], s);
    } else if (L.kind == LK_TTM_STREAM) {
        TtmParams T = L.tstr;
        T.X = in1;
        T.Y = in0;
        T.C = out;
        rc = launch_ttm_stream(L.dtype, T, L.i0, L.i1, true, L.i2, s);
    } else if (L.kind == LK_OUTER) {
        OuterParams O = L.outer;
        O.X = L.xsrc ? in1 : in0;
        O.Y = L.xsrc ? in0 : in1;
        O.C = out;
        rc = launch_outer(L.dtype, O, s);
    } else if (L.kind == LK_TTM_ROWS) {
        TtmRowParams R = L.trow;
        R.X = in1;
        R.Y = in0;
        R.C = out;
        rc = launch_ttm_rows(L.dtype, R, L.i0, L.i1, L.i2, s);
    }
    return rc ? fail(rc, "%s: launch failed", L.op) : TLIB_OK;
}

// ------------------------------------------------------------------ plan cache
//
// Launch records keyed by the call shape: operation, modes, and per operand
// its dtype, order, extents, strides and address modulo 16 (the planner's
// vector-width decisions read nothing finer).  Guarded by a lock; emptied when
// full and whenever the autotune table or mode changes (the key does not hold
// the kernel choice).

namespace {
std::mutex g_pc_mu;
std::unordered_map<std::string, std::shared_ptr<const Launch>> g_pc;
std::atomic<int64_t> g_pc_hits{0}, g_pc_misses{0};
constexpr size_t PC_MAX = 8192;
enum { PCK_TTV = 1, PCK_TTM = 2, PCK_TTT = 3, PCK_TTT_NOALLOC = 4 };
}  // namespace

static void pk(std::string& k, int64_t v) { k.append(reinterpret_cast<const char*>(&v), sizeof(v)); }

static void pk_ten(std::string& k, const Ten& t) {
    pk(k, int64_t(t.dtype) | (int64_t(t.p) << 8) | (int64_t(uintptr_t(t.data) & 15) << 16));
    for (int r = 0; r < t.p; ++r) {
        pk(k, t.n[r]);
        pk(k, t.w[r]);
    }
}

static std::shared_ptr<const Launch> pc_get(const std::string& k) {
    std::lock_guard<std::mutex> lk(g_pc_mu);
    auto it = g_pc.find(k);
    if (it == g_pc.end()) {
        ++g_pc_misses;
        return nullptr;
    }
    ++g_pc_hits;
    return it->second;
}

static void pc_put(const std::string& k, const Launch& L) {
    auto v = std::make_shared<const Launch>(L);
    std::lock_guard<std::mutex> lk(g_pc_mu);
    if (g_pc.size() >= PC_MAX) g_pc.clear();
    g_pc[k] = std::move(v);
}

static void pc_clear() {
    std::lock_guard<std::mutex> lk(g_pc_mu);
    g_pc.clear();
}

// ------------------------------------------------------------------ TTV planning

static int plan_ttv(const Ten& a, const Ten& b, int mi, const Ten& c, Launch& L) {
    L.op = "ttv";
    L.dtype = a.dtype;
    Dim d[MAXP];
    int nd = 0;
    for (int r = 0, k = 0; r < a.p; ++r) {
        if (r == mi) continue;
        d[nd++] = {a.n[r], {a.w[r], c.w[k], 0}};
        ++k;
    }
    nd = coalesce(d, nd, 2, 0);

    TtvParams P{};
    P.A = a.data;
    P.b = b.data;
    P.C = c.data;
    P.n_k = a.n[mi];
    P.sA_k = a.w[mi];
    P.sb = b.w[0];
    P.n_lo = P.n_hi = 1;
    P.sA_lo = P.sA_hi = P.sC_lo = P.sC_hi = 0;
    int nlo = 0, nhi = 0;
    for (int i = 0; i < nd; ++i) {
        if (d[i].s[0] < P.sA_k || P.n_k == 1) {
            if (nlo == 0 && nhi == 0) {
                P.n_lo = d[i].n;
                P.sA_lo = d[i].s[0];
                P.sC_lo = d[i].s[1];
            }
            ++nlo;
        } else {
            if (nhi == 0) {
                P.n_hi = d[i].n;
                P.sA_hi = d[i].s[0];
                P.sC_hi = d[i].s[1];
            }
            ++nhi;
        }
    }
    // n_k == 1 puts every dim in "lo"; re-split so that at most one is lo
    if (P.n_k == 1 && nlo == 2 && nhi == 0) {
        P.n_hi = d[1].n;
        P.sA_hi = d[1].s[0];
        P.sC_hi = d[1].s[1];
        nlo = 1;
        nhi = 1;
    }
    const int64_t outs = P.n_lo * P.n_hi;
    const bool fast = nlo <= 1 && nhi <= 1 && outs < (int64_t(1) << 31) && P.n_k < (int64_t(1) << 31);
    const int es = esize(a.dtype);
    int64_t nout = 1;
    for (int i = 0; i < nd; ++i) nout *= d[i].n;
    P.gh = Grp{};
    if (fast) {
        if (P.n_hi > 1) {
            Dim h = {P.n_hi, {P.sA_hi, P.sC_hi, 0}};
            fill_grp(P.gh, &h, 1, 0, 1);
        }
    }
    // views whose dims do not merge: lo = the dim of smallest A stride when it
    // is below k's and holds >= 32 outputs, hi = every other output dim
    bool colview = false;
    if (!fast && nd >= 1 && d[0].s[0] < P.sA_k && d[0].n >= 32 && nd - 1 <= GMAXD && nout < (int64_t(1) << 31) &&
        P.n_k < (int64_t(1) << 31)) {
        P.n_lo = d[0].n;
        P.sA_lo = d[0].s[0];
        P.sC_lo = d[0].s[1];
        colview = fill_grp(P.gh, d + 1, nd - 1, 0, 1);
        P.n_hi = P.gh.total;
        P.sA_hi = P.sC_hi = 0;
    }

    // dense operand: its (lo,k) slabs are contiguous.  For n_lo of 32..63
    // the slab kernel (b staged in LDS beside the slabs) beats lanes along lo
    // when whole slabs fit its 32 KB and there are enough of them to fill the
    // chip; otherwise the col kernel (with its k splits) keeps those shapes.
    const bool slabs_dense = fast && (P.n_lo == 1 || P.sA_lo == 1) && (P.n_k == 1 || P.sA_k == P.n_lo) &&
                             (P.n_hi == 1 || P.sA_hi == P.n_lo * P.n_k);
    const bool mid_slabs = slabs_dense && P.n_lo * P.n_k * esize(a.dtype) <= 32768 && P.n_hi >= 2048;
    if ((fast && (P.n_lo >= 64 || (P.n_lo >= 32 && !mid_slabs))) || colview) {
        const int maxvec = 16 / es;
        auto vec_ok = [&](int v) {
            if (v == 1) return true;
            if (P.sA_lo != 1 || P.n_lo % v) return false;
            if (P.n_k > 1 && P.sA_k % v) return false;
            for (int j = 0; j < P.gh.nd; ++j)
                if (P.gh.n[j] > 1 && P.gh.s0[j] % v) return false;
            return (uintptr_t(P.A) % (uintptr_t)(v * es)) == 0;
        };
        auto blocks = [&](int v) { return ((P.n_lo + 64 * v - 1) / (64 * v)) * P.n_hi; };
        // the widest vector the strides allow, narrowed only while it would
        // leave fewer than 1024 workgroups (406^3 FP64 TTVs with 16-byte
        // loads over 1624 workgroups: 16-20 % faster than 8-byte loads over
        // 2842)
        int vec = maxvec;
        while (vec > 1 && !vec_ok(vec)) vec /= 2;
        while (vec > 1 && blocks(vec) < 1024) vec /= 2;
        int64_t nb = blocks(vec);
        int ks = 1;
        if (nb < 2048) {
            int64_t want = (2048 + nb - 1) / nb;
            int64_t maxk = std::max<int64_t>(1, P.n_k / 32);
            ks = int(std::min<int64_t>(std::min<int64_t>(want, maxk), 64));
        }
        // short k and enough units: one wave per (lo tile, hi) unit with all
        // rows in flight (at most 256 bytes of rows per lane)
        int kr = 0;
        if (ks == 1 && nb >= 4096)
            for (int c : {8, 16, 32, 64})
                if (P.n_k <= c && int64_t(c) * vec * es <= 256) {
                    kr = c;
                    break;
                }
        size_t wsb = ks > 1 ? size_t(ks) * size_t(outs) * size_t(esize(acc_dtype(a.dtype))) : 0;
        plan_note("ttv col dtype=%s n_lo=%lld n_k=%lld n_hi=%lld sA=(%lld,%lld,%lld) sC=(%lld,%lld) "
                  "hidims=%d vec=%d ksplit=%d kr=%d blocks=%lld",
                  dname(a.dtype), (long long)P.n_lo, (long long)P.n_k, (long long)P.n_hi,
                  (long long)P.sA_lo, (long long)P.sA_k, (long long)P.sA_hi, (long long)P.sC_lo,
                  (long long)P.sC_hi, P.gh.nd, vec, ks, kr, (long long)(kr ? (nb + 3) / 4 : nb * ks));
        L.ttv = P;
        L.i0 = vec;
        if (kr) {
            L.kind = LK_TTV_COLW;
            L.i1 = kr;
        } else {
            L.kind = LK_TTV_COL;
            L.i1 = ks;
            L.wsb = wsb;
        }
        return TLIB_OK;
    }
    // n_lo == 1 with k of unit stride and n_k >= 32: every output is one
    // contiguous fiber, which the fiber kernel streams without staging
    // (below); shorter fibers fill its lane groups poorly and stay on slabs
    const bool row_fibers = fast && P.n_lo == 1 && P.sA_k == 1 && P.n_k >= 32;
    const bool slab_ok = slabs_dense && !row_fibers;
    if (slab_ok) {
        const int64_t cap = 32768 / es;
        const int64_t slab = P.n_lo * P.n_k;
        int64_t S, kc;
        if (slab <= cap) {
            S = cap / slab;
            kc = P.n_k;
            // keep at least ~2048 blocks when the problem allows it
            int64_t want_blocks = std::min<int64_t>(2048, P.n_hi);
            int64_t smax = std::max<int64_t>(1, P.n_hi / want_blocks);
            S = std::max<int64_t>(1, std::min(S, smax));
            // a multiple of slabs that spans whole 16-byte units, so that every
            // workgroup's run starts aligned and is copied with 16-byte loads
            const int64_t sb = slab * es;
            const int64_t unit = 16 / (sb % 16 == 0 ? 16 : sb % 8 == 0 ? 8 : sb % 4 == 0 ? 4 : sb % 2 == 0 ? 2 : 1);
            if (S >= unit) S -= S % unit;
        } else {
            S = 1;
            kc = std::max<int64_t>(1, cap / P.n_lo);
        }
        plan_note("ttv slab dtype=%s n_lo=%lld n_k=%lld n_hi=%lld sC=(%lld,%lld) slabs=%lld kc=%lld "
                  "blocks=%lld",
                  dname(a.dtype), (long long)P.n_lo, (long long)P.n_k, (long long)P.n_hi,
                  (long long)P.sC_lo, (long long)P.sC_hi, (long long)S, (long long)kc,
                  (long long)((P.n_hi + S - 1) / S));
        L.kind = LK_TTV_SLAB;
        L.ttv = P;
        L.i0 = int(S);
        L.i1 = int(kc);
        return TLIB_OK;
    }
    // views with slabs that are not contiguous: G lanes per output fiber
    {
        Grp go;
        if (nd <= GMAXD && nout < (int64_t(1) << 31) && P.n_k < (int64_t(1) << 31) && fill_grp(go, d, nd, 0, 1)) {
            const int G = P.n_k >= 256 ? 64 : P.n_k >= 64 ? 32 : P.n_k >= 16 ? 16 : 8;
            plan_note("ttv fiber dtype=%s dims=%d outputs=%lld n_k=%lld sA_k=%lld G=%d", dname(a.dtype), nd,
                      (long long)nout, (long long)P.n_k, (long long)P.sA_k, G);
            L.kind = LK_TTV_FIBER;
            L.ttv = P;
            L.go = go;
            L.i0 = G;
            return TLIB_OK;
        }
    }
    GDims g;
    fill_gdims(g, d, nd, 2);
    plan_note("ttv generic dtype=%s dims=%d outputs=%lld n_k=%lld", dname(a.dtype), nd,
              (long long)g.total, (long long)P.n_k);
    L.kind = LK_TTV_GENERIC;
    L.ttv = P;
    L.gd[0] = g;
    return TLIB_OK;
}

// ------------------------------------------------------------------ autotuning
//
// Per-key choice among the launch candidates of one call shape (op, modes,
// extents, strides and dtypes; data pointers are not part of the key).  With
// autotuning on, the first call of a new key runs every applicable candidate
// once to warm up, then times them round-robin under HIP events on the
// caller's stream (three rounds; that call synchronises the stream), keeps
// the fastest, and finishes with one more launch of it, which produces the
// result.  Later calls of the key go
// straight to the stored pick.  Calls made while the stream is capturing a
// graph, and calls in plan-only mode, never tune.

constexpr int PICK_NA = -1000;  // the candidate does not apply to this call

static std::atomic<int> g_autotune{0};  // TLIB_AUTOTUNE_OFF / _ON / _FROZEN
static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune;

static void key_int(std::string& k, long long v) {
    char buf[32];
    snprintf(buf, sizeof(buf), "|%lld", v);
    k += buf;
}

static void key_ten(std::string& k, const Ten& t) {
    char buf[64];
    snprintf(buf, sizeof(buf), "|%d:%d", t.dtype, t.p);
    k += buf;
    for (int r = 0; r < t.p; ++r) {
        snprintf(buf, sizeof(buf), ",%lld/%lld", (long long)t.n[r], (long long)t.w[r]);
        k += buf;
    }
}

// Shape class of a call: the features the kernel choice follows, so that a
// choice tuned on one shape serves the other shapes of its class (a served
// stream rarely repeats an exact shape).  Extents enter as base-4 log buckets.
static int lg4(int64_t x) {
    int b = 0;
    while (x >= 4) {
        x >>= 2;
        ++b;
    }
    return b;
}

static int64_t min_stride(const Ten& t, const int* modes, int nm) {
    int64_t m = INT64_MAX;
    for (int i = 0; i < nm; ++i)
        if (t.n[modes[i]] > 1) m = std::min(m, t.w[modes[i]]);
    return m;
}

// TTM: dtype; whether mode m has A's smallest stride (contiguous k-fibers)
// and C's smallest stride (C contiguous along j); buckets of n_m, of B's rows,
// of the columns N / n_m and of n_lo (the extent below mode m in A's memory).
static std::string ttm_class_key(const Ten& a, const Ten& bm, const Ten& c, int mi) {
    int64_t n_lo = 1, cols = 1;
    bool jmin = true;
    for (int r = 0; r < a.p; ++r) {
        if (r == mi) continue;
        cols *= a.n[r];
        if (a.n[r] > 1 && a.w[r] < a.w[mi]) n_lo *= a.n[r];
        if (c.n[r] > 1 && c.w[r] < c.w[mi]) jmin = false;
    }
    std::string k = "class:ttm";
    key_int(k, a.dtype);
    key_int(k, n_lo == 1);
    key_int(k, jmin);
    key_int(k, lg4(a.n[mi]));
    key_int(k, lg4(bm.n[0]));
    key_int(k, lg4(cols));
    key_int(k, lg4(n_lo));
    return k;
}

// TTT: dtype; whether the contracted modes hold the smallest stride of A and
// of B, whether C's smallest stride is among the free modes of A; buckets of
// M, N and K.
static std::string ttt_class_key(const Ten& a, const Ten& b, const Ten& c, int q, const int32_t* phi,
                                 const int32_t* psi) {
    const int r = a.p - q, s = b.p - q;
    int fa[MAXP], ka[MAXP], fb[MAXP], kb[MAXP], ca[MAXP], cb[MAXP];
    int64_t M = 1, N = 1, K = 1;
    for (int i = 0; i < r; ++i) {
        fa[i] = phi[i] - 1;
        M *= a.n[fa[i]];
        ca[i] = i;
    }
    for (int i = 0; i < q; ++i) {
        ka[i] = phi[r + i] - 1;
        kb[i] = psi[s + i] - 1;
        K *= a.n[ka[i]];
    }
    for (int i = 0; i < s; ++i) {
        fb[i] = psi[i] - 1;
        N *= b.n[fb[i]];
        cb[i] = r + i;
    }
    std::string k = "class:ttt";
    key_int(k, a.dtype);
    key_int(k, min_stride(a, ka, q) < min_stride(a, fa, r));
    key_int(k, min_stride(b, kb, q) < min_stride(b, fb, s));
    key_int(k, min_stride(c, ca, r) < min_stride(c, cb, s));
    key_int(k, lg4(M));
    key_int(k, lg4(N));
    key_int(k, lg4(K));
    return k;
}

// *settled: the launch the call ended with is the key's lasting choice (the
// planner's rule with autotuning off or frozen, a stored pick, or a pick just
// tuned), so a plan cache may keep it; false when tuning was due but could
// not run (plan-only mode, a capturing stream).
// A shape without its own entry takes the entry of its class (ckey) when the
// table has one and the mode is frozen; in ON mode it is tuned.  Tuning a new
// shape stores its pick under both keys (the class entry only if the class has
// none yet).
template <class F>
static int tuned(const std::string& key, const std::string& ckey, const int* cands, int nc, hipStream_t s, F&& run,
                 bool* settled) {
    *settled = true;
    const int mode = g_autotune.load();
    if (mode == TLIB_AUTOTUNE_OFF) return run(-1);
    int pick = PICK_NA;
    bool by_class = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            pick = it->second;
        } else if ((it = g_tune.find(ckey)) != g_tune.end()) {
            pick = it->second;
            by_class = true;
        }
    }
    // in ON mode a shape with only a class entry is tuned for itself
    if (pick != PICK_NA && !(by_class && mode == TLIB_AUTOTUNE_ON)) {
        const int rc = run(pick);
        if (rc != PICK_NA) {
            g_plan += by_class ? " autotuned(class)" : " autotuned";
            return rc;
        }
        return run(-1);
    }
    if (mode != TLIB_AUTOTUNE_ON) return run(-1);
    *settled = false;
    if (g_plan_only) return run(-1);
    if (capturing(s)) return run(-1);
    static thread_local hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!e0 && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
        e0 = e1 = nullptr;
        return run(-1);
    }
    // warm every applicable candidate once, then time them round-robin
    // (three rounds, best of three per candidate) so that drift in clocks or
    // memory state during tuning hits every candidate alike
    constexpr int MAXC = 32, ROUNDS = 3;
    int live[MAXC];
    float tmin[MAXC];
    int nl = 0;
    for (int i = 0; i < nc && nl < MAXC; ++i) {
        const int rc = run(cands[i]);
        if (rc == PICK_NA || rc == TLIB_ENOMEM) continue;  // not applicable, or more scratch than the stream holds
        if (rc != TLIB_OK) return rc;
        live[nl] = cands[i];
        tmin[nl++] = 0.f;
    }
    for (int round = 0; round < ROUNDS; ++round)
        for (int i = 0; i < nl; ++i) {
            if (hipEventRecord(e0, s) != hipSuccess) return fail(TLIB_EHIP, "autotune: event record failed");
            const int rc = run(live[i]);
            if (rc != TLIB_OK) return rc;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return fail(TLIB_EHIP, "autotune: event wait failed");
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return fail(TLIB_EHIP, "autotune: event time failed");
            if (round == 0 || ms < tmin[i]) tmin[i] = ms;
        }
    int bp = PICK_NA;
    float best = 0.f;
    for (int i = 0; i < nl; ++i)
        if (bp == PICK_NA || tmin[i] < best) {
            best = tmin[i];
            bp = live[i];
        }
    if (bp == PICK_NA) return run(-1);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = bp;
        g_tune.emplace(ckey, bp);
    }
    const int rc = run(bp);
    if (rc == TLIB_OK) g_plan += " autotuned(new)";
    *settled = true;
    return rc;
}

// ------------------------------------------------------------------ GEMM planning

// dm: M-group dims with strides (X, C); dn: N-group (Y, C); dk: K-group (X, Y).
// x_is: X is operand 0 or 1 of the call.  ws_cap: scratch available when the
// call brings a fixed buffer (SIZE_MAX: the stream's workspace).
// tile_force >= 0 replaces the tile heuristic (autotuning candidates):
// tile_force % GT_COUNT is the tile, tile_force / GT_COUNT the split target
// (0: about 1024 workgroups, 1: 512, 2: 256 -- fewer, deeper K slices and
// fewer partials for products that would otherwise split K many ways).
static int plan_gemm(int dtype, int x_is, const void* X, const void* Y, void* C, Dim* dm, int ndm, Dim* dn,
                     int ndn, Dim* dk, int ndk, const char* op, size_t ws_cap, Launch& L, int tile_force = -1) {
    L.op = op;
    L.dtype = dtype;
    L.xsrc = x_is;
    // Dims are stored with strides in slots 0/1 as documented above.
    int64_t M = 1, N = 1, K = 1;
    for (int i = 0; i < ndm; ++i) M *= dm[i].n;
    for (int i = 0; i < ndn; ++i) N *= dn[i].n;
    for (int i = 0; i < ndk; ++i) K *= dk[i].n;
    // Roles: the MFMA result puts consecutive columns of C in consecutive
    // lanes, so the group holding C's unit-stride dim becomes N.
    auto minstride = [](const Dim* d, int nd, int o) {
        int64_t m = INT64_MAX;
        for (int i = 0; i < nd; ++i)
            if (d[i].n > 1) m = std::min(m, d[i].s[o]);
        return m;
    };
    if (minstride(dm, ndm, 1) < minstride(dn, ndn, 1)) {
        L.xsrc = 1 - L.xsrc;
        std::swap(X, Y);
        std::swap(M, N);
        Dim tmp[MAXP];
        for (int i = 0; i < ndm; ++i) tmp[i] = dm[i];
        for (int i = 0; i < ndn; ++i) dm[i] = dn[i];
        for (int i = 0; i < ndm; ++i) dn[i] = tmp[i];
        std::swap(ndm, ndn);
        for (int i = 0; i < ndk; ++i) std::swap(dk[i].s[0], dk[i].s[1]);
    }
    ndm = coalesce(dm, ndm, 2, 1);
    ndn = coalesce(dn, ndn, 2, 1);
    // K is walked in the order of the larger operand's strides so that its
    // loads run along memory.
    ndk = coalesce(dk, ndk, 2, M > N ? 0 : 1);

    // Packed X: a small X (at most 4M elements and a sixteenth of Y's
    // elements, Y at least 4 MB) whose first K dim does not have unit stride
    // is copied into the workspace as an M x K matrix with k fastest, in the
    // K order chosen above (Y's), so that the GEMM loads groups of
    // consecutive k of X (16-bit MFMA operands take eight, FP32/FP64 loads
    // two), and K's dims merge wherever Y's do (one K dim lets Y load vectors
    // along N).  The copy's dims are K's then M's, with X's strides and the
    // packed ones.
    GDims xpack{};
    size_t xwsb = 0;
    Dim dm0[MAXP], dk0[MAXP];
    const void* X0 = X;
    for (int i = 0; i < ndm; ++i) dm0[i] = dm[i];
    for (int i = 0; i < ndk; ++i) dk0[i] = dk[i];
    {
        const int gv = (dtype == TLIB_BF16 || dtype == TLIB_F16) ? 8 : 2;
        if (ws_cap == SIZE_MAX && ndk >= 1 && ndk + ndm <= MAXP && dk[0].s[0] != 1 && dk[0].n % gv == 0 &&
            M * K <= (int64_t(1) << 22) && 16 * M <= N && K >= 64 &&
            N * K * int64_t(esize(dtype)) >= (int64_t(4) << 20)) {
            int64_t st = 1;
            for (int i = 0; i < ndk; ++i) {
                xpack.n[xpack.nd] = dk[i].n;
                xpack.s[0][xpack.nd] = dk[i].s[0];
                xpack.s[2][xpack.nd++] = st;
                dk[i].s[0] = st;
                st *= dk[i].n;
            }
            for (int i = 0; i < ndm; ++i) {
                xpack.n[xpack.nd] = dm[i].n;
                xpack.s[0][xpack.nd] = dm[i].s[0];
                xpack.s[2][xpack.nd++] = st;
                dm[i].s[0] = st;
                st *= dm[i].n;
            }
            xpack.total = st;
            xwsb = size_t(st) * size_t(esize(dtype));
            X = reinterpret_cast<const void*>(uintptr_t(WS_ALIGN));  // workspace pieces are 256-byte aligned
            ndk = coalesce(dk, ndk, 2, 1);
        }
    }

    GemmParams P{};
    bool fast = fill_grp(P.gm, dm, ndm, 0, 1) && fill_grp(P.gn, dn, ndn, 0, 1) &&
                fill_grp(P.gk, dk, ndk, 0, 1);
    if (fast) {
        P.X = X;
        P.Y = Y;
        P.C = C;
        P.M = int32_t(M);
        P.N = int32_t(N);
        P.K = int32_t(K);
        {
            // 16-byte stores along N: unit stride on N's first dim, runs of whole
            // vectors in every dim, and a 16-byte aligned base.
            const int v = 16 / esize(acc_dtype(dtype));
            bool ok = ndn >= 1 && dn[0].s[1] == 1 && dn[0].n % v == 0 && (uintptr_t(C) % 16) == 0;
            for (int i = 1; i < ndn; ++i) ok = ok && dn[i].s[1] % v == 0;
            for (int i = 0; i < ndm; ++i) ok = ok && dm[i].s[1] % v == 0;
            P.c_vec = ok ? 1 : 0;
        }
        P.x_kfast = ndk > 0 && (ndm == 0 || minstride(dk, ndk, 0) < minstride(dm, ndm, 0));
        P.y_kfast = ndk > 0 && (ndn == 0 || minstride(dk, ndk, 1) < minstride(dn, ndn, 0));
        {
            // Y as vectors along N: FP32/FP64, N's first dim of unit stride in
            // Y, K one dim; 16-byte vectors when K's stride keeps them
            // aligned, else 8-byte ones (FP32) when it keeps those aligned.
            // 16-bit: eight elements, stored transposed into the slice with
            // one 2-byte LDS write each and 128-deep slices, which pays only
            // on long contractions (TTT, K = 3072: 42 against 43 us) and
            // costs on short ones (the BF16 Tucker chain's TTMs, K = 160:
            // 1.67 against 0.94 ms), so it needs K >= 1024.
            P.syk = ndk == 1 ? dk[0].s[1] : 0;
            P.y_vec = 0;
            if (!P.y_kfast && ndk == 1 && ndn >= 1 && dn[0].s[0] == 1) {
                const int v16 = 16 / esize(dtype);
                if (P.syk % v16 == 0 && (uintptr_t(Y) % 16) == 0 && (esize(dtype) > 2 || K >= 1024))
                    P.y_vec = v16;
                else if (dtype == TLIB_F32 && P.syk % 2 == 0 && (uintptr_t(Y) % 8) == 0) P.y_vec = 2;
            }
        }
        {
            // Operands whose K has a first dim of unit stride load groups of
            // consecutive k (16-bit: 8 k; FP32/FP64: 2 k), where
            // that dim's extent is a multiple of the group and every other
            // stride and the base keep the groups aligned.
            P.kvec = 0;
            const bool wide = dtype == TLIB_BF16 || dtype == TLIB_F16;
            const int gv = wide ? 8 : 2;  // k per group: 16 bytes (16-bit, FP64) or 8 bytes (FP32)
            const int gb = gv * esize(dtype);
            auto groups_ok = [&](int o, const void* base, const Dim* d, int nd) {
                if (ndk < 1 || dk[0].n % gv != 0 || dk[0].s[o] != 1 || (uintptr_t(base) % gb) != 0) return false;
                for (int i = 1; i < ndk; ++i)
                    if (dk[i].s[o] % gv != 0) return false;
                for (int i = 0; i < nd; ++i)
                    if (d[i].s[0] % gv != 0) return false;
                return true;
            };
            if (groups_ok(0, X, dm, ndm)) P.kvec |= 1;
            if (P.y_vec == 0 && groups_ok(1, Y, dn, ndn)) P.kvec |= 2;
        }
        // The all-rows kernel (M <= 128 in one tile, Y streamed straight into
        // the MFMAs): X's K groups must be contiguous (16 bytes; FP32 8), and
        // for 16-bit inputs Y's as well.  Chosen only by the autotuner (picks
        // from 3 GT_COUNT on: 64 fn columns per workgroup, fn = 1 + r % 2,
        // split target 1024 >> (r / 2)).
        {
            const bool wide = dtype == TLIB_BF16 || dtype == TLIB_F16;
            const int gx = wide ? 8 : 2;
            auto k_groups = [&](int o, const void* base, const Dim* d, int nd, int gv) {
                if (ndk < 1 || dk[0].n % gv != 0 || dk[0].s[o] != 1 ||
                    (uintptr_t(base) % (size_t(gv) * esize(dtype))) != 0)
                    return false;
                for (int i = 1; i < ndk; ++i)
                    if (dk[i].s[o] % gv != 0) return false;
                for (int i = 0; i < nd; ++i)
                    if (d[i].s[0] % gv != 0) return false;
                return true;
            };
            const bool rows_ok = M <= 128 && k_groups(0, X, dm, ndm, gx) && (!wide || k_groups(1, Y, dn, ndn, 8));
            const bool forced = tile_force >= 3 * GT_COUNT && tile_force < 3 * GT_COUNT + 6;
            if (forced && !rows_ok) return PICK_NA;
            if (rows_ok && forced) {
                const int r = forced ? tile_force - 3 * GT_COUNT : 0;
                const int fn = 1 + r % 2, target = 1024 >> (r / 2);
                int fm = 1;
                while (16 * fm < M) fm *= 2;
                const int64_t tiles = (N + 64 * fn - 1) / (64 * fn);
                const int kc = gemm_rows_kchunk(dtype);
                int ks = 1;
                if (tiles < target) {
                    const int64_t want = (target + tiles - 1) / tiles;
                    const int64_t maxk = std::max<int64_t>(1, K / (4 * kc));
                    ks = int(std::min<int64_t>(std::min<int64_t>(want, maxk), 32));
                }
                P.kchunk = int32_t(((K + ks - 1) / ks + kc - 1) / kc * kc);
                P.ksplit = int((K + P.kchunk - 1) / P.kchunk);
                if (ws_cap != SIZE_MAX && P.ksplit > 1) {
                    const size_t per = size_t(M) * size_t(N) * size_t(esize(acc_dtype(dtype)));
                    const int cap = int(std::max<int64_t>(1, std::min<int64_t>(P.ksplit, int64_t(ws_cap / per))));
                    if (cap < P.ksplit) {
                        P.kchunk = int32_t(((K + cap - 1) / cap + kc - 1) / kc * kc);
                        P.ksplit = int((K + P.kchunk - 1) / P.kchunk);
                    }
                }
                P.tiles_m = 1;
                P.tiles_n = int32_t(tiles);
                plan_note("%s gemm-rows dtype=%s M=%lld N=%lld K=%lld dims=(%d,%d,%d) fm=%d fn=%d ksplit=%d tiles=%lld",
                          op, dname(dtype), (long long)M, (long long)N, (long long)K, ndm, ndn, ndk, fm, fn,
                          P.ksplit, (long long)tiles);
                if (xwsb) g_plan += " xpack";
                L.kind = LK_GEMM_ROWS;
                P.X = P.Y = nullptr;
                P.C = nullptr;
                L.gemm = P;
                L.i0 = fm;
                L.i1 = fn;
                L.gd[0] = xpack;
                L.xwsb = xwsb;
                L.wsb = P.ksplit > 1 ? size_t(P.ksplit) * size_t(M) * size_t(N) * size_t(esize(acc_dtype(dtype))) : 0;
                return TLIB_OK;
            }
        }
        // FP64 accumulators are twice as wide: keep a wave's tile at 64x32 so
        // that two waves fit per SIMD.
        const bool wide_acc = dtype == TLIB_F64;
        auto ntiles = [&](int t) {
            TileShape ts = tile_shape(t);
            return ((M + ts.bm - 1) / ts.bm) * ((N + ts.bn - 1) / ts.bn);
        };
        int tile;
        if (M <= 16) tile = GT_16x256;
        else if (N <= 32) tile = GT_256x32;
        else if (N <= 64) tile = wide_acc ? GT_256x32 : GT_256x64;
        else if (M <= 64) tile = GT_64x128;
        else if (M <= 128) tile = wide_acc ? GT_128x64 : GT_128x128;
        else if (N <= 128) tile = wide_acc ? GT_128x64 : GT_128x128;
        else tile = wide_acc ? GT_128x64 : GT_128x128;
        if (ntiles(tile) < 1024 && tile != GT_16x256 && ntiles(GT_64x64) > ntiles(tile)) tile = GT_64x64;
        int split_target = 1024;
        if (tile_force >= 0 && tile_force < 3 * GT_COUNT) {
            tile = tile_force % GT_COUNT;
            split_target = 1024 >> (tile_force / GT_COUNT);
        }
        TileShape ts = tile_shape(tile);
        P.tiles_m = int32_t((M + ts.bm - 1) / ts.bm);
        P.tiles_n = int32_t((N + ts.bn - 1) / ts.bn);
        int64_t nt = int64_t(P.tiles_m) * P.tiles_n;
        const int bk = gemm_slice_k(dtype, tile);
        int ks = 1;
        if (nt < split_target) {
            int64_t want = (split_target + nt - 1) / nt;
            int64_t maxk = std::max<int64_t>(1, K / (4 * bk));
            ks = int(std::min<int64_t>(std::min<int64_t>(want, maxk), 32));
        }
        if (ws_cap != SIZE_MAX && ks > 1) {
            // a fixed scratch buffer bounds the split: fewer slices (the same
            // sums in another order), none when one slice does not fit
            const size_t per = size_t(M) * size_t(N) * size_t(esize(acc_dtype(dtype)));
            ks = int(std::max<int64_t>(1, std::min<int64_t>(ks, int64_t(ws_cap / per))));
        }
        P.ksplit = ks;
        P.kchunk = int32_t(((K + ks - 1) / ks + bk - 1) / bk * bk);
        if (ks > 1) P.ksplit = int((K + P.kchunk - 1) / P.kchunk);
        size_t wsb = P.ksplit > 1 ? size_t(P.ksplit) * size_t(M) * size_t(N) *
                                        size_t(esize(acc_dtype(dtype)))
                                  : 0;
        plan_note("%s gemm dtype=%s M=%lld N=%lld K=%lld dims=(%d,%d,%d) tile=%dx%d kfast=(%d,%d) "
                  "cvec=%d yvec=%d kvec=%d ksplit=%d tiles=%lld",
                  op, dname(dtype), (long long)M, (long long)N, (long long)K, ndm, ndn, ndk, ts.bm,
                  ts.bn, P.x_kfast, P.y_kfast, P.c_vec, P.y_vec, P.kvec, P.ksplit, (long long)nt);
        if (xwsb) g_plan += " xpack";
        L.kind = LK_GEMM;
        P.X = P.Y = nullptr;
        P.C = nullptr;
        L.gemm = P;
        L.i0 = tile;
        L.wsb = P.ksplit > 1 ? wsb : 0;
        L.gd[0] = xpack;
        L.xwsb = xwsb;
        return TLIB_OK;
    }
    if (xwsb) {
        // the generic kernel reads X where it lies
        for (int i = 0; i < ndm; ++i) dm[i] = dm0[i];
        for (int i = 0; i < ndk; ++i) dk[i] = dk0[i];
        X = X0;
        xwsb = 0;
    }
    GDims gm, gn, gk;
    fill_gdims(gm, dm, ndm, 2);
    fill_gdims(gn, dn, ndn, 2);
    fill_gdims(gk, dk, ndk, 2);
    plan_note("%s generic dtype=%s M=%lld N=%lld K=%lld dims=(%d,%d,%d)", op, dname(dtype),
              (long long)M, (long long)N, (long long)K, ndm, ndn, ndk);
    L.kind = LK_GEMM_GENERIC;
    L.gd[0] = gm;
    L.gd[1] = gn;
    L.gd[2] = gk;
    return TLIB_OK;
}

static int check_ttv(const tlib_tensor* A, const tlib_tensor* b, int32_t m, const tlib_tensor* C, Ten& a,
                     Ten& v, Ten& c) {
    int rc;
    if ((rc = normalize(A, a, "A")) || (rc = normalize(b, v, "b")) || (rc = normalize(C, c, "C")))
        return rc;
    if (a.p < 2) return fail(TLIB_EINVAL, "ttv: order of A must be >= 2 (got %d)", a.p);
    if (m < 1 || m > a.p) return fail(TLIB_EMODE, "ttv: mode %d out of 1..%d", m, a.p);
    const int mi = m - 1;
    if (v.p != 1 || v.n[0] != a.n[mi])
        return fail(TLIB_ESHAPE, "ttv: b must be a vector of length n_%d = %lld", m, (long long)a.n[mi]);
    if (c.p != a.p - 1) return fail(TLIB_ESHAPE, "ttv: C must have order %d", a.p - 1);
    for (int r = 0, k = 0; r < a.p; ++r) {
        if (r == mi) continue;
        if (c.n[k] != a.n[r]) return fail(TLIB_ESHAPE, "ttv: extent %d of C must be %lld", k + 1,
                                          (long long)a.n[r]);
        ++k;
    }
    if (v.dtype != a.dtype) return fail(TLIB_EDTYPE, "ttv: b must have A's dtype");
    if (c.dtype != acc_dtype(a.dtype)) return fail(TLIB_EDTYPE, "ttv: C must be %s", dname(acc_dtype(a.dtype)));
    if ((rc = check_output(c, "C"))) return rc;
    if (overlaps(c, a) || overlaps(c, v)) return fail(TLIB_EALIAS, "ttv: C overlaps an input");
    return TLIB_OK;
}

static int check_ttm(const tlib_tensor* A, const tlib_tensor* B, int32_t m, const tlib_tensor* C, Ten& a,
                     Ten& bm, Ten& c) {
    int rc;
    if ((rc = normalize(A, a, "A")) || (rc = normalize(B, bm, "B")) || (rc = normalize(C, c, "C")))
        return rc;
    if (a.p < 2) return fail(TLIB_EINVAL, "ttm: order of A must be >= 2 (got %d)", a.p);
    if (m < 1 || m > a.p) return fail(TLIB_EMODE, "ttm: mode %d out of 1..%d", m, a.p);
    const int mi = m - 1;
    if (bm.p != 2 || bm.n[1] != a.n[mi])
        return fail(TLIB_ESHAPE, "ttm: B must have shape (n', n_%d = %lld)", m, (long long)a.n[mi]);
    if (c.p != a.p) return fail(TLIB_ESHAPE, "ttm: C must have order %d", a.p);
    for (int r = 0; r < a.p; ++r) {
        int64_t want = r == mi ? bm.n[0] : a.n[r];
        if (c.n[r] != want)
            return fail(TLIB_ESHAPE, "ttm: extent %d of C must be %lld", r + 1, (long long)want);
    }
    if (bm.dtype != a.dtype) return fail(TLIB_EDTYPE, "ttm: B must have A's dtype");
    if (c.dtype != acc_dtype(a.dtype)) return fail(TLIB_EDTYPE, "ttm: C must be %s", dname(acc_dtype(a.dtype)));
    if ((rc = check_output(c, "C"))) return rc;
    if (overlaps(c, a) || overlaps(c, bm)) return fail(TLIB_EALIAS, "ttm: C overlaps an input");
    return TLIB_OK;
}

// One grouped request as C[m, n] = sum_k X[m, k] Y[k, n] (a BatchItem).
// TTV: X = b, Y = A, M = 1; TTM: X = B, Y = A; TTT: X = A, Y = B, the pairs
// (phi_{r+k}, psi_{s+k}) forming K.  Returns false when a group does not
// collapse to GMAXD dims and 2^31 indices.
static int64_t min_c_stride(const Dim* d, int nd) {
    int64_t m = INT64_MAX;
    for (int i = 0; i < nd; ++i)
        if (d[i].n > 1) m = std::min(m, d[i].s[1]);
    return m;
}

static bool batch_item(int op, const Ten& a, const Ten& b, const Ten& c, int mi, int q, const int32_t* phi,
                       const int32_t* psi, BatchItem& it) {
    Dim dm[MAXP], dn[MAXP], dk[MAXP];
    int ndm = 0, ndn = 0, ndk = 0;
    const void* X = nullptr;
    const void* Y = nullptr;
    if (op == 0) {
        for (int r = 0, k = 0; r < a.p; ++r) {
            if (r == mi) continue;
            dn[ndn++] = {a.n[r], {a.w[r], c.w[k++], 0}};
        }
        dk[ndk++] = {a.n[mi], {b.w[0], a.w[mi], 0}};
        X = b.data;
        Y = a.data;
    } else if (op == 1) {
        dm[ndm++] = {b.n[0], {b.w[0], c.w[mi], 0}};
        for (int r = 0; r < a.p; ++r)
            if (r != mi) dn[ndn++] = {a.n[r], {a.w[r], c.w[r], 0}};
        dk[ndk++] = {a.n[mi], {b.w[1], a.w[mi], 0}};
        X = b.data;
        Y = a.data;
    } else {
        const int r = a.p - q, s = b.p - q;
        for (int k = 0; k < r; ++k) dm[ndm++] = {a.n[phi[k] - 1], {a.w[phi[k] - 1], c.w[k], 0}};
        for (int k = 0; k < s; ++k) dn[ndn++] = {b.n[psi[k] - 1], {b.w[psi[k] - 1], c.w[r + k], 0}};
        for (int k = 0; k < q; ++k) dk[ndk++] = {a.n[phi[r + k] - 1], {a.w[phi[r + k] - 1], b.w[psi[s + k] - 1], 0}};
        X = a.data;
        Y = b.data;
    }
    it = BatchItem{};
    it.dtype = a.dtype;
    it.C = c.data;
    if (op == 0) {
        it.kind = BATCH_SCALAR;
        ndn = coalesce(dn, ndn, 2, 0);  // lanes along A's fastest output dim
        ndk = coalesce(dk, ndk, 2, 1);
    } else {
        it.kind = BATCH_TILE;
        if (min_c_stride(dm, ndm) < min_c_stride(dn, ndn)) {
            // lanes run along N: N takes the group holding C's smallest stride
            Dim t[MAXP];
            for (int i = 0; i < ndm; ++i) t[i] = dm[i];
            for (int i = 0; i < ndn; ++i) dm[i] = dn[i];
            for (int i = 0; i < ndm; ++i) dn[i] = t[i];
            std::swap(ndm, ndn);
            std::swap(X, Y);
            for (int i = 0; i < ndk; ++i) std::swap(dk[i].s[0], dk[i].s[1]);
        }
        ndm = coalesce(dm, ndm, 2, 1);
        ndn = coalesce(dn, ndn, 2, 1);
        ndk = coalesce(dk, ndk, 2, 0);
    }
    if (!fill_grp(it.gm, dm, ndm, 0, 1) || !fill_grp(it.gn, dn, ndn, 0, 1) || !fill_grp(it.gk, dk, ndk, 0, 1))
        return false;
    if (it.kind == BATCH_SCALAR && ndk > 1) return false;
    it.X = X;
    it.Y = Y;
    it.M = it.gm.total;
    it.N = it.gn.total;
    it.K = it.gk.total;
    it.tiles_n = (it.N + 63) / 64;
    return true;
}

static int64_t batch_units(const BatchItem& it) {
    if (it.kind == BATCH_SCALAR) return (it.N + 255) / 256;
    return (it.M + 15) / 16 * it.tiles_n;
}


static bool is_perm(int p, const int32_t* v) {
    if (!v && p > 0) return false;
    bool seen[MAXP] = {};
    for (int r = 0; r < p; ++r) {
        if (v[r] < 1 || v[r] > p || seen[v[r] - 1]) return false;
        seen[v[r] - 1] = true;
    }
    return true;
}

static void begin_call() {
    g_err.clear();
    g_plan.clear();
}

}  // namespace tlib

using namespace tlib;

// ------------------------------------------------------------------ static scratch (no-allocation TTT)
//
// Split-K partials of tlib_ttt_noalloc live in this file-scope device array:
// one copy per GPU, loaded with the library's code object and held until the
// process ends.  On the host the array's name is only a stand-in, never a
// device address: host code uses the address that hipGetSymbolAddress
// returns, looked up once per device (with that device current) on the first
// call there and kept in g_scratch_dev.
static __device__ __align__(256) unsigned char scratch[TLIB_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[SCRATCH_MAX_DEVICES] = {};
}  // namespace

static int scratch_address(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(TLIB_EHIP, "ttt_noalloc: no current device");
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return fail(TLIB_EINVAL, "ttt_noalloc: device %d beyond the %d supported", dev, SCRATCH_MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(TLIB_EHIP, "ttt_noalloc: hipGetSymbolAddress of the scratch array failed (%s)",
                        hipGetErrorString(e));
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return TLIB_OK;
}

extern "C" {

int tlib_ttv(const tlib_tensor* A, const tlib_tensor* b, int32_t m, const tlib_tensor* C,
             void* stream) {
    begin_call();
    Ten a, v, c;
    int rc = check_ttv(A, b, m, C, a, v, c);
    if (rc) return rc;
    std::string key;
    key.reserve(32 * (a.p + v.p + c.p) + 48);
    pk(key, PCK_TTV);
    pk(key, m);
    pk_ten(key, a);
    pk_ten(key, v);
    pk_ten(key, c);
    WsCtx ws;
    ws.s = hipStream_t(stream);
    auto L = pc_get(key);
    if (L) {
        g_plan = L->note;
        return exec_launch(*L, a.data, v.data, c.data, ws, hipStream_t(stream));
    }
    Launch N;
    if ((rc = plan_ttv(a, v, m - 1, c, N))) return rc;
    N.note = g_plan;
    pc_put(key, N);
    return exec_launch(N, a.data, v.data, c.data, ws, hipStream_t(stream));
}

// One TTM launch.  pick: TTM_PICK_HEUR (planner's rule), TTM_PICK_STREAM
// (streaming kernel for this layout), TTM_PICK_ROWS_PLAIN (row kernel with
// unshifted windows), TTM_PICK_GEMM + tile (tiled GEMM; tile GT_COUNT = the
// GEMM's own tile rule).  Returns PICK_NA when the pick does not apply.
enum { TTM_PICK_HEUR = -1, TTM_PICK_STREAM = 0, TTM_PICK_ROWS_PLAIN = 1, TTM_PICK_GEMM = 2 };

static int plan_ttm(const Ten& a, const Ten& bm, int mi, const Ten& c, int pick, Launch& L) {
    L.op = "ttm";
    L.dtype = a.dtype;
    // Short contraction: the streaming kernels (B resident in LDS, A streamed).
    {
        const int64_t Mr = bm.n[0], Kr = a.n[mi];
        Dim dn[MAXP];
        int ndn = 0;
        for (int r = 0; r < a.p; ++r)
            if (r != mi) dn[ndn++] = {a.n[r], {a.w[r], c.w[r], 0}};
        ndn = coalesce(dn, ndn, 2, 1);  // C's innermost column dim first
        int64_t cmin = INT64_MAX, ncols = 1;
        for (int i = 0; i < ndn; ++i) {
            cmin = std::min(cmin, dn[i].s[1]);
            ncols *= dn[i].n;
        }
        const bool trans = Mr > 1 && c.w[mi] < cmin;
        const bool wide = a.dtype == TLIB_BF16 || a.dtype == TLIB_F16;
        if (trans && pick <= 0) {
            // C contiguous along j
            const int ks = ttm_stream_ks(a.dtype, int(std::min<int64_t>(Kr, 1 << 20)));
            const int fm = Mr <= 16 ? 1 : Mr <= 64 ? 4 : Mr <= 256 ? 16 : 0;
            TtmParams T{};
            const int kstep = wide ? 32 : 4;
            const int64_t m16 = int64_t(fm) * 16, kp = int64_t(ks) * kstep;
            const int64_t lds =
                wide ? m16 * (kp + 8) * 2 : kp * (m16 + (a.dtype == TLIB_F64 ? 4 : 16)) * esize(a.dtype);
            if (ks > 0 && fm > 0 && Kr <= 64 && lds <= 163840 && fill_grp(T.gn, dn, ndn, 0, 1)) {
                T.X = bm.data;
                T.Y = a.data;
                T.C = c.data;
                T.M = int32_t(Mr);
                T.N = int32_t(T.gn.total);
                T.K = int32_t(Kr);
                T.sXm = bm.w[0];
                T.sXk = bm.w[1];
                T.sYk = a.w[mi];
                T.sCm = c.w[mi];
                const int fn = fm >= 16 ? 1 : fm >= 4 ? 2 : 4;
                const int64_t cols = 64 * fn;  // columns per workgroup tile
                const int64_t tiles = (T.N + cols - 1) / cols;
                const int per_cu = lds <= 20480 ? 4 : lds <= 40960 ? 3 : lds <= 65536 ? 2 : 1;
                const int grid = int(std::max<int64_t>(1, std::min<int64_t>(tiles, 256 * per_cu)));
                plan_note("ttm stream dtype=%s M=%lld N=%d K=%lld dims=%d fm=%d cols=%lld ks=%d lds=%lld grid=%d "
                          "tiles=%lld",
                          dname(a.dtype), (long long)Mr, T.N, (long long)Kr, ndn, fm, (long long)cols, ks,
                          (long long)lds, grid, (long long)tiles);
                L.kind = LK_TTM_STREAM;
                L.tstr = T;
                L.i0 = fm;
                L.i1 = ks;
                L.i2 = grid;
                return TLIB_OK;
            }
        } else if (!trans && pick <= 1 && Mr <= 256 && ndn >= 1 && ndn <= GMAXD + 1 && ncols < (int64_t(1) << 31)) {
            // C strided along j: runs along C's innermost column dim
            TtmRowParams R{};
            const int64_t n_lo = dn[0].n, sclo = dn[0].s[1];
            const int lpc = 128 / esize(acc_dtype(a.dtype));  // C elements per 128-byte line
            int mode = TTM_ROWS_PLAIN;
            if (sclo == 1 && c.w[mi] == n_lo && n_lo <= 32) mode = n_lo <= 16 ? TTM_ROWS_BAND1 : TTM_ROWS_BAND;
            else if (sclo == 1 && c.w[mi] == n_lo && n_lo > 128 && n_lo <= 176 &&
                     ttm_rows_ks(a.dtype, TTM_ROWS_BANDW, int(std::min<int64_t>(Kr, 1 << 20))) > 0)
                mode = TTM_ROWS_BANDW;
            else if (sclo == 1 && ttm_rows_ks(a.dtype, TTM_ROWS_ALIGNED, int(std::min<int64_t>(Kr, 1 << 20))) > 0)
                mode = TTM_ROWS_ALIGNED;
            if (pick == TTM_PICK_ROWS_PLAIN) {
                if (mode == TTM_ROWS_PLAIN) return PICK_NA;  // same launch as the streaming pick
                mode = TTM_ROWS_PLAIN;
            }
            const int ks = ttm_rows_ks(a.dtype, mode, int(std::min<int64_t>(Kr, 1 << 20)));
            // rows of B per workgroup: all of them if B's slice fits in LDS,
            // else halve into row groups
            int mr = int((Mr + 15) / 16 * 16);
            int64_t lds = ks > 0 ? ttm_rows_lds(a.dtype, mode, mr, ks) : INT64_MAX;
            while (ks > 0 && lds > 65536 && mr > 16) {
                mr = (mr / 2 + 15) / 16 * 16;
                lds = ttm_rows_lds(a.dtype, mode, mr, ks);
            }
            const int nrg = int((Mr + mr - 1) / mr);
            const int64_t tc = mode == TTM_ROWS_ALIGNED ? (n_lo + lpc - 1 + 63) / 64
                               : mode == TTM_ROWS_PLAIN ? (n_lo + 63) / 64
                                                        : 1;
            const int64_t units = ncols / n_lo * tc;
            // a 16-row block of C is addressed with 32-bit buffer offsets
            const int64_t blk_bytes = (16 * c.w[mi] + n_lo * sclo) * int64_t(esize(acc_dtype(a.dtype)));
            if (ks > 0 && lds <= 65536 && units < (int64_t(1) << 31) && blk_bytes < (int64_t(1) << 31) &&
                fill_grp(R.gh, dn + 1, ndn - 1, 0, 1)) {
                R.X = bm.data;
                R.Y = a.data;
                R.C = c.data;
                R.M = int32_t(Mr);
                R.K = int32_t(Kr);
                R.sXm = bm.w[0];
                R.sXk = bm.w[1];
                R.sYk = a.w[mi];
                R.sCm = c.w[mi];
                R.n_lo = int32_t(n_lo);
                R.Tc = int32_t(tc);
                R.sYlo = dn[0].s[0];
                R.sClo = sclo;
                R.units = units;
                R.fd_tc = make_fastdiv(uint32_t(tc));
                R.fd_lo = make_fastdiv(uint32_t(n_lo));
                R.mr = mr;
                R.nrg = nrg;
                const int per_cu = int(std::max<int64_t>(1, std::min<int64_t>(4, 160 * 1024 / lds)));
                int64_t g0 = std::max<int64_t>(1, std::min<int64_t>((units + 3) / 4, 256 * per_cu / nrg));
                if (nrg > 1) g0 = (g0 + 7) / 8 * 8;  // the row-group mapping needs whole XCD rounds
                const int grid = int(g0 * nrg);
                plan_note("ttm rows dtype=%s mode=%s M=%lld K=%lld n_lo=%lld runs=%lld chunks=%lld ks=%d lds=%lld "
                          "rowgroups=%dx%d grid=%d",
                          dname(a.dtype),
                          mode == TTM_ROWS_BAND ? "band" : mode == TTM_ROWS_BAND1 ? "band1"
                                                 : mode == TTM_ROWS_BANDW ? "bandw"
                                                 : mode == TTM_ROWS_ALIGNED ? "aligned" : "plain",
                          (long long)Mr, (long long)Kr, (long long)n_lo, (long long)(ncols / n_lo), (long long)tc, ks,
                          (long long)lds, nrg, mr, grid);
                L.kind = LK_TTM_ROWS;
                L.trow = R;
                L.i0 = mode;
                L.i1 = ks;
                L.i2 = grid;
                return TLIB_OK;
            }
        }
    }
    if (pick == TTM_PICK_STREAM || pick == TTM_PICK_ROWS_PLAIN) return PICK_NA;
    // GEMM roles: X = B (M = j), Y = A (N = the modes of A other than m), K = mode m.
    Dim dm[1] = {{bm.n[0], {bm.w[0], c.w[mi], 0}}};
    Dim dn[MAXP];
    int ndn = 0;
    for (int r = 0; r < a.p; ++r)
        if (r != mi) dn[ndn++] = {a.n[r], {a.w[r], c.w[r], 0}};
    Dim dk[1] = {{a.n[mi], {bm.w[1], a.w[mi], 0}}};
    // TTM_PICK_GEMM + t: t < GT_COUNT a tile, GT_COUNT the GEMM's own rule,
    // GT_COUNT + 1 + r the all-rows kernel variant r (0..5)
    const int t = pick >= TTM_PICK_GEMM ? pick - TTM_PICK_GEMM : -1;
    int force = -1;
    if (t >= 0 && t < GT_COUNT) force = t;
    else if (t > GT_COUNT && t <= GT_COUNT + 6) force = 3 * GT_COUNT + (t - GT_COUNT - 1);
    return plan_gemm(a.dtype, 1, bm.data, a.data, c.data, dm, 1, dn, ndn, dk, 1, "ttm", SIZE_MAX, L, force);
}

// Plan and launch one TTM (no plan cache): the pieces of a ttm2 chain.
static int ttm_dispatch(const Ten& a, const Ten& bm, int mi, const Ten& c, int pick, void* stream, WsCtx& wsc) {
    Launch L;
    const int rc = plan_ttm(a, bm, mi, c, pick, L);
    if (rc != TLIB_OK) return rc;
    return exec_launch(L, a.data, bm.data, c.data, wsc, hipStream_t(stream));
}

int tlib_set_autotune(int mode) {
    if (mode != TLIB_AUTOTUNE_OFF && mode != TLIB_AUTOTUNE_ON && mode != TLIB_AUTOTUNE_FROZEN) return -1;
    const int prev = g_autotune.exchange(mode);
    if (prev != mode) pc_clear();
    return prev;
}

int64_t tlib_autotune_entries(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return int64_t(g_tune.size());
}

void tlib_autotune_clear(void) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune.clear();
    }
    pc_clear();
}

int tlib_autotune_save(const char* path) {
    begin_call();
    if (!path) return fail(TLIB_EINVAL, "autotune_save: null path");
    FILE* f = fopen(path, "w");
    if (!f) return fail(TLIB_EINVAL, "autotune_save: cannot write %s", path);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto& kv : g_tune) fprintf(f, "%d %s\n", kv.second, kv.first.c_str());
    }
    const bool ok = fclose(f) == 0;
    return ok ? TLIB_OK : fail(TLIB_EINVAL, "autotune_save: write to %s failed", path);
}

int tlib_autotune_load(const char* path) {
    begin_call();
    if (!path) return fail(TLIB_EINVAL, "autotune_load: null path");
    FILE* f = fopen(path, "r");
    if (!f) return fail(TLIB_EINVAL, "autotune_load: cannot read %s", path);
    char line[4096];
    int rc = TLIB_OK, lineno = 0;
    while (fgets(line, sizeof(line), f)) {
        ++lineno;
        size_t n = strlen(line);
        while (n > 0 && (line[n - 1] == '\n' || line[n - 1] == '\r')) line[--n] = 0;
        if (n == 0) continue;
        int pick = 0, used = 0;
        if (sscanf(line, "%d %n", &pick, &used) != 1 || used <= 0 || line[used] == 0 || n == sizeof(line) - 1) {
            rc = fail(TLIB_EINVAL, "autotune_load: %s line %d is malformed", path, lineno);
            break;
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[std::string(line + used)] = pick;
    }
    fclose(f);
    pc_clear();
    return rc;
}

int tlib_ttm(const tlib_tensor* A, const tlib_tensor* B, int32_t m, const tlib_tensor* C,
             void* stream) {
    begin_call();
    Ten a, bm, c;
    int rc = check_ttm(A, B, m, C, a, bm, c);
    if (rc) return rc;
    const int mi = m - 1;
    const hipStream_t s = hipStream_t(stream);
    std::string pkey;
    pkey.reserve(32 * (a.p + bm.p + c.p) + 48);
    pk(pkey, PCK_TTM);
    pk(pkey, m);
    pk_ten(pkey, a);
    pk_ten(pkey, bm);
    pk_ten(pkey, c);
    WsCtx ws;
    ws.s = s;
    auto L = pc_get(pkey);
    if (L) {
        g_plan = L->note;
        return exec_launch(*L, a.data, bm.data, c.data, ws, s);
    }
    static const int cands[] = {TTM_PICK_STREAM,          TTM_PICK_ROWS_PLAIN,        TTM_PICK_GEMM + GT_COUNT,
                                TTM_PICK_GEMM + GT_128x64, TTM_PICK_GEMM + GT_128x128, TTM_PICK_GEMM + GT_64x128,
                                TTM_PICK_GEMM + GT_256x64, TTM_PICK_GEMM + GT_64x64,   TTM_PICK_GEMM + GT_COUNT + 1,
                                TTM_PICK_GEMM + GT_COUNT + 2};
    std::string key = "ttm";
    key_int(key, m);
    key_ten(key, a);
    key_ten(key, bm);
    key_ten(key, c);
    Launch last;
    bool settled = false;
    rc = tuned(key, ttm_class_key(a, bm, c, mi), cands, int(sizeof(cands) / sizeof(cands[0])), s, [&](int pick) {
        Launch N;
        int r = plan_ttm(a, bm, mi, c, pick, N);
        if (r != TLIB_OK) return r;
        ws.used = 0;
        r = exec_launch(N, a.data, bm.data, c.data, ws, s);
        if (r == TLIB_OK) last = std::move(N);
        return r;
    }, &settled);
    if (rc == TLIB_OK && settled && last.kind != LK_NONE) {
        last.note = g_plan;
        pc_put(pkey, last);
    }
    return rc;
}

// Two mode products C = (A x_a Ua) x_b Ub in one pass (Sec. 5.2 Eq. ttm
// twice; a step pair of tensor_times_matrices).  The fused kernel serves
// FP32/FP64 with factor rows <= 32, contracted extents <= 256 and columns that
// collapse to a few (extent, stride) pairs; otherwise the two products run as
// TTMs through an intermediate in the stream's second workspace.
int tlib_ttm2(const tlib_tensor* A, const tlib_tensor* Ua, int32_t ma, const tlib_tensor* Ub, int32_t mb,
              const tlib_tensor* C, void* stream) {
    begin_call();
    Ten a, ua, ub, c;
    int rc;
    if ((rc = normalize(A, a, "A")) || (rc = normalize(Ua, ua, "Ua")) || (rc = normalize(Ub, ub, "Ub")) ||
        (rc = normalize(C, c, "C")))
        return rc;
    if (a.p < 2) return fail(TLIB_EINVAL, "ttm2: order of A must be >= 2 (got %d)", a.p);
    if (ma < 1 || ma > a.p || mb < 1 || mb > a.p || ma == mb)
        return fail(TLIB_EMODE, "ttm2: modes %d, %d must be distinct and in 1..%d", ma, mb, a.p);
    const int ia = ma - 1, ib = mb - 1;
    if (ua.p != 2 || ua.n[1] != a.n[ia])
        return fail(TLIB_ESHAPE, "ttm2: Ua must have shape (n', n_%d = %lld)", ma, (long long)a.n[ia]);
    if (ub.p != 2 || ub.n[1] != a.n[ib])
        return fail(TLIB_ESHAPE, "ttm2: Ub must have shape (n', n_%d = %lld)", mb, (long long)a.n[ib]);
    if (c.p != a.p) return fail(TLIB_ESHAPE, "ttm2: C must have order %d", a.p);
    for (int r = 0; r < a.p; ++r) {
        const int64_t want = r == ia ? ua.n[0] : r == ib ? ub.n[0] : a.n[r];
        if (c.n[r] != want) return fail(TLIB_ESHAPE, "ttm2: extent %d of C must be %lld", r + 1, (long long)want);
    }
    if (a.dtype != TLIB_F64 && a.dtype != TLIB_F32)
        return fail(TLIB_EDTYPE, "ttm2: A must be FP64 or FP32 (16-bit inputs: two tlib_ttm calls)");
    if (ua.dtype != a.dtype || ub.dtype != a.dtype || c.dtype != a.dtype)
        return fail(TLIB_EDTYPE, "ttm2: Ua, Ub and C must have A's dtype");
    if ((rc = check_output(c, "C"))) return rc;
    if (overlaps(c, a) || overlaps(c, ua) || overlaps(c, ub)) return fail(TLIB_EALIAS, "ttm2: C overlaps an input");
    hipStream_t s = hipStream_t(stream);

    // f: the contracted mode with the smaller stride in A
    const bool a_fast = a.w[ia] <= a.w[ib];
    const int fi = a_fast ? ia : ib, gi = a_fast ? ib : ia;
    const Ten& uf = a_fast ? ua : ub;
    const Ten& ug = a_fast ? ub : ua;
    Ttm2Params P{};
    P.A = a.data;
    P.Uf = uf.data;
    P.Ug = ug.data;
    P.C = c.data;
    P.n_f = int32_t(std::min<int64_t>(a.n[fi], 1 << 30));
    P.n_g = int32_t(std::min<int64_t>(a.n[gi], 1 << 30));
    P.m_f = int32_t(std::min<int64_t>(uf.n[0], 1 << 30));
    P.m_g = int32_t(std::min<int64_t>(ug.n[0], 1 << 30));
    P.s_f = a.w[fi];
    P.s_g = a.w[gi];
    P.sUf0 = uf.w[0];
    P.sUf1 = uf.w[1];
    P.sUg0 = ug.w[0];
    P.sUg1 = ug.w[1];
    P.sC_f = c.w[fi];
    P.sC_g = c.w[gi];
    Dim dc[MAXP];
    int ndc = 0;
    int64_t ncol = 1;
    for (int r = 0; r < a.p; ++r)
        if (r != fi && r != gi) {
            dc[ndc++] = {a.n[r], {a.w[r], c.w[r], 0}};
            ncol *= a.n[r];
        }
    ndc = coalesce(dc, ndc, 2, 0);
    P.ncol = ncol;
    // slab copy with 16-byte loads: the columns' first dim has unit stride
    // in A and whole tiles of 16, and every A offset of a tile start is a
    // multiple of the vector
    const int va = 16 / esize(a.dtype);
    bool vec = ndc >= 1 && dc[0].s[0] == 1 && dc[0].n % 16 == 0 && (uintptr_t(a.data) % 16) == 0 &&
               P.s_f % va == 0 && P.s_g % va == 0 && a.n[fi] <= ttm2_vec_rows(a.dtype);
    for (int i = 1; i < ndc; ++i) vec = vec && dc[i].s[0] % va == 0;
    int lds = ttm2_lds_bytes(a.dtype, P.m_f, P.n_f, P.n_g, vec);
    if (vec && lds > 73728) {
        vec = false;
        lds = ttm2_lds_bytes(a.dtype, P.m_f, P.n_f, P.n_g, false);
    }
    // a grid of fewer than 256 column tiles leaves most of the chip idle: a
    // large tensor with few columns takes the two TTMs
    const bool fused = uf.n[0] <= 32 && ug.n[0] <= 32 && a.n[fi] <= 256 && a.n[gi] <= 256 &&
                       lds <= (vec ? 73728 : 65536) && ncol < (int64_t(1) << 31) &&
                       (ncol >= 256 * 16 || a.numel() <= (int64_t(1) << 22)) && fill_grp(P.gc, dc, ndc, 0, 1);
    if (fused) {
        plan_note("ttm2 fused dtype=%s f=%d g=%d n=(%d,%d) m=(%d,%d) columns=%lld dims=%d vec=%d lds=%d grid=%lld",
                  dname(a.dtype), fi + 1, gi + 1, P.n_f, P.n_g, P.m_f, P.m_g, (long long)ncol, ndc, vec ? 1 : 0, lds,
                  (long long)((ncol + 15) / 16));
        if (g_plan_only) return TLIB_OK;
        rc = launch_ttm2(a.dtype, P, vec, s);
        return rc ? fail(rc, "ttm2: launch failed") : TLIB_OK;
    }
    // two TTMs: T = A x_a Ua in A's storage order, then C = T x_b Ub
    Ten t = a;
    t.n[ia] = ua.n[0];
    {
        int ord[MAXP];
        for (int r = 0; r < a.p; ++r) ord[r] = r;
        std::stable_sort(ord, ord + a.p, [&](int x, int y) { return a.w[x] < a.w[y]; });
        int64_t acc = 1;
        for (int k = 0; k < a.p; ++k) {
            t.w[ord[k]] = acc;
            acc *= t.n[ord[k]];
        }
    }
    const size_t tb = size_t(t.numel()) * size_t(esize(a.dtype));
    // scratch of the two TTMs (split-K partials), probed by planning them
    // with a placeholder intermediate; the intermediate comes first
    size_t part = 0;
    {
        const bool po = g_plan_only;
        g_plan_only = true;
        t.data = a.data;
        WsCtx probe;
        if ((rc = ttm_dispatch(a, ua, ia, t, TTM_PICK_HEUR, stream, probe)) == TLIB_OK)
            rc = ttm_dispatch(t, ub, ib, c, TTM_PICK_HEUR, stream, probe);
        g_plan_only = po;
        if (rc) return rc;
        part = probe.peak;
    }
    plan_note("ttm2 chain dtype=%s a=%d b=%d intermediate=%zu bytes", dname(a.dtype), ma, mb, tb);
    if (g_plan_only) return TLIB_OK;
    WsCtx ws;
    ws.s = s;
    ws.hint = ws_round(tb) + part;
    t.data = ws.take(tb);
    if (!t.data || ws.avail() < part) return ws_fail(ws, ws_round(tb) + part, "ttm2");
    const size_t mark = ws.used;
    if ((rc = ttm_dispatch(a, ua, ia, t, TTM_PICK_HEUR, stream, ws))) return rc;
    ws.used = mark;  // the first product's partials are consumed before the second runs
    return ttm_dispatch(t, ub, ib, c, TTM_PICK_HEUR, stream, ws);
}

static int check_ttt(const tlib_tensor* A, const tlib_tensor* B, int32_t q, const int32_t* phi, const int32_t* psi,
                     const tlib_tensor* C, Ten& a, Ten& b, Ten& c) {
    int rc;
    if ((rc = normalize(A, a, "A")) || (rc = normalize(B, b, "B")) || (rc = normalize(C, c, "C")))
        return rc;
    const int r = a.p - q, s = b.p - q;
    if (q < 0 || r < 0 || s < 0) return fail(TLIB_EINVAL, "ttt: q=%d exceeds an operand order", q);
    if (a.p == 0 || b.p == 0) return fail(TLIB_EINVAL, "ttt: q+r and q+s must be > 0");
    if (!is_perm(a.p, phi)) return fail(TLIB_EMODE, "ttt: phi is not a permutation of 1..%d", a.p);
    if (!is_perm(b.p, psi)) return fail(TLIB_EMODE, "ttt: psi is not a permutation of 1..%d", b.p);
    if (c.p != r + s) return fail(TLIB_ESHAPE, "ttt: C must have order %d", r + s);
    for (int k = 0; k < r; ++k)
        if (c.n[k] != a.n[phi[k] - 1]) return fail(TLIB_ESHAPE, "ttt: extent %d of C mismatch", k + 1);
    for (int k = 0; k < s; ++k)
        if (c.n[r + k] != b.n[psi[k] - 1])
            return fail(TLIB_ESHAPE, "ttt: extent %d of C mismatch", r + k + 1);
    for (int k = 0; k < q; ++k)
        if (a.n[phi[r + k] - 1] != b.n[psi[s + k] - 1])
            return fail(TLIB_ESHAPE, "ttt: contracted pair %d has extents %lld and %lld", k + 1,
                        (long long)a.n[phi[r + k] - 1], (long long)b.n[psi[s + k] - 1]);
    if (b.dtype != a.dtype) return fail(TLIB_EDTYPE, "ttt: B must have A's dtype");
    if (c.dtype != acc_dtype(a.dtype)) return fail(TLIB_EDTYPE, "ttt: C must be %s", dname(acc_dtype(a.dtype)));
    if ((rc = check_output(c, "C"))) return rc;
    if (overlaps(c, a) || overlaps(c, b)) return fail(TLIB_EALIAS, "ttt: C overlaps an input");
    return TLIB_OK;
}

// GEMM roles: X = A (M = free A modes), Y = B (N = free B modes), K = pairs.
static int plan_ttt(const Ten& a, const Ten& b, int q, const int32_t* phi, const int32_t* psi, const Ten& c,
                    size_t ws_cap, Launch& L, int tile) {
    const int r = a.p - q, s = b.p - q;
    Dim dm[MAXP], dn[MAXP], dk[MAXP];
    for (int k = 0; k < r; ++k) dm[k] = {a.n[phi[k] - 1], {a.w[phi[k] - 1], c.w[k], 0}};
    for (int k = 0; k < s; ++k) dn[k] = {b.n[psi[k] - 1], {b.w[psi[k] - 1], c.w[r + k], 0}};
    for (int k = 0; k < q; ++k) dk[k] = {a.n[phi[r + k] - 1], {a.w[phi[r + k] - 1], b.w[psi[s + k] - 1], 0}};
    return plan_gemm(a.dtype, 0, a.data, b.data, c.data, dm, r, dn, s, dk, q, "ttt", ws_cap, L, tile);
}

// Outer product (q = 0): C(free A modes in phi order, free B modes in psi
// order) = A(.) B(.), one product per element, written as a stream along C's
// unit-stride mode.  Returns PICK_NA when a group does not collapse to at most
// GMAXD dims or 2^31 indices (the GEMM path then takes it).
static int plan_outer(const Ten& a, const Ten& b, const int32_t* phi, const int32_t* psi, const Ten& c,
                      Launch& L) {
    const int r = a.p, s = b.p;
    Dim dm[MAXP], dn[MAXP];
    for (int k = 0; k < r; ++k) dm[k] = {a.n[phi[k] - 1], {a.w[phi[k] - 1], c.w[k], 0}};
    for (int k = 0; k < s; ++k) dn[k] = {b.n[psi[k] - 1], {b.w[psi[k] - 1], c.w[r + k], 0}};
    int ndm = coalesce(dm, r, 2, 1), ndn = coalesce(dn, s, 2, 1);
    int xsrc = 0;
    auto minc = [](const Dim* d, int nd) {
        int64_t m = INT64_MAX;
        for (int i = 0; i < nd; ++i) m = std::min(m, d[i].s[1]);
        return m;
    };
    if (minc(dm, ndm) < minc(dn, ndn)) {  // the group with C's unit stride runs along lanes
        Dim t[MAXP];
        for (int i = 0; i < ndm; ++i) t[i] = dm[i];
        for (int i = 0; i < ndn; ++i) dm[i] = dn[i];
        for (int i = 0; i < ndm; ++i) dn[i] = t[i];
        std::swap(ndm, ndn);
        xsrc = 1;
    }
    OuterParams O{};
    if (!fill_grp(O.gm, dm, ndm, 0, 1) || !fill_grp(O.gn, dn, ndn, 0, 1)) return PICK_NA;
    O.M = O.gm.total;
    O.N = O.gn.total;
    const int v = 16 / esize(acc_dtype(a.dtype));
    bool vec = ndn >= 1 && dn[0].s[1] == 1 && dn[0].n % v == 0 && (uintptr_t(c.data) % 16) == 0;
    for (int i = 1; i < ndn; ++i) vec = vec && dn[i].s[1] % v == 0;
    for (int i = 0; i < ndm; ++i) vec = vec && dm[i].s[1] % v == 0;
    O.vec = vec ? v : 1;
    O.nv = O.N / O.vec;
    int cw = 1, lg = 0;
    while (cw < 256 && cw < O.nv) {
        cw *= 2;
        ++lg;
    }
    O.cw = cw;
    O.cw_log2 = lg;
    O.rows_per_wg = 256 / cw;
    plan_note("ttt outer dtype=%s M=%lld N=%lld dims=(%d,%d) vec=%d cw=%d", dname(a.dtype), (long long)O.M,
              (long long)O.N, ndm, ndn, O.vec, cw);
    L = Launch();
    L.kind = LK_OUTER;
    L.op = "ttt";
    L.dtype = a.dtype;
    L.xsrc = xsrc;
    L.outer = O;
    return TLIB_OK;
}

static std::string ttt_pkey(int kind, const Ten& a, const Ten& b, const Ten& c, int q, const int32_t* phi,
                            const int32_t* psi) {
    std::string key;
    key.reserve(32 * (a.p + b.p + c.p) + 64);
    pk(key, kind);
    pk(key, q);
    for (int k = 0; k < a.p; ++k) pk(key, phi[k]);
    for (int k = 0; k < b.p; ++k) pk(key, psi[k]);
    pk_ten(key, a);
    pk_ten(key, b);
    pk_ten(key, c);
    return key;
}

static std::string ttt_key(const Ten& a, const Ten& b, const Ten& c, int q, const int32_t* phi, const int32_t* psi) {
    std::string key = "ttt";
    key_int(key, q);
    for (int k = 0; k < a.p; ++k) key_int(key, phi[k]);
    for (int k = 0; k < b.p; ++k) key_int(key, psi[k]);
    key_ten(key, a);
    key_ten(key, b);
    key_ten(key, c);
    return key;
}

int tlib_ttt(const tlib_tensor* A, const tlib_tensor* B, int32_t q, const int32_t* phi,
             const int32_t* psi, const tlib_tensor* C, void* stream) {
    begin_call();
    Ten a, b, c;
    int rc = check_ttt(A, B, q, phi, psi, C, a, b, c);
    if (rc) return rc;
    const hipStream_t st = hipStream_t(stream);
    const std::string pkey = ttt_pkey(PCK_TTT, a, b, c, q, phi, psi);
    WsCtx ws;
    ws.s = st;
    auto L = pc_get(pkey);
    if (L) {
        g_plan = L->note;
        return exec_launch(*L, a.data, b.data, c.data, ws, st);
    }
    if (q == 0) {
        Launch O;
        if (plan_outer(a, b, phi, psi, c, O) == TLIB_OK) {
            rc = exec_launch(O, a.data, b.data, c.data, ws, st);
            if (rc == TLIB_OK) {
                O.note = g_plan;
                pc_put(pkey, O);
            }
            return rc;
        }
    }
    Launch last;
    bool settled = false;
    auto run = [&](int tile) {
        Launch N;
        int r = plan_ttt(a, b, q, phi, psi, c, SIZE_MAX, N, tile);
        if (r != TLIB_OK) return r;
        ws.used = 0;
        r = exec_launch(N, a.data, b.data, c.data, ws, st);
        if (r == TLIB_OK) last = std::move(N);
        return r;
    };
    // every tile with three split targets (about 1024, 512 and 256
    // workgroups), then the all-rows kernel (64 or 128 columns per workgroup)
    // with the same three targets
    static const int cands[] = {3 * GT_COUNT + 0, 3 * GT_COUNT + 1, 3 * GT_COUNT + 2, 3 * GT_COUNT + 3,
                                3 * GT_COUNT + 4, 3 * GT_COUNT + 5, GT_16x256, GT_64x128, GT_128x128, GT_256x64, GT_64x64, GT_128x64, GT_256x32,
                                GT_COUNT + GT_16x256, GT_COUNT + GT_64x128, GT_COUNT + GT_128x128,
                                GT_COUNT + GT_256x64, GT_COUNT + GT_64x64, GT_COUNT + GT_128x64,
                                GT_COUNT + GT_256x32, 2 * GT_COUNT + GT_16x256, 2 * GT_COUNT + GT_64x128,
                                2 * GT_COUNT + GT_128x128, 2 * GT_COUNT + GT_256x64, 2 * GT_COUNT + GT_64x64,
                                2 * GT_COUNT + GT_128x64, 2 * GT_COUNT + GT_256x32};
    rc = tuned(ttt_key(a, b, c, q, phi, psi), ttt_class_key(a, b, c, q, phi, psi), cands,
               int(sizeof(cands) / sizeof(cands[0])), st, run, &settled);
    if (rc == TLIB_OK && settled && last.kind != LK_NONE) {
        last.note = g_plan;
        pc_put(pkey, last);
    }
    return rc;
}

// TTT whose scratch is the static array above: the split-K slices are bounded
// by its size (fewer slices, the same sums in another order; none when one
// slice does not fit), the tile is the planner's rule (no autotuning, which
// would synchronise), and nothing is allocated.  Partials are written in full
// by every call before they are summed, so the array needs no clearing.
int tlib_ttt_noalloc(const tlib_tensor* A, const tlib_tensor* B, int32_t q, const int32_t* phi,
                     const int32_t* psi, const tlib_tensor* C, void* stream) {
    begin_call();
    Ten a, b, c;
    int rc = check_ttt(A, B, q, phi, psi, C, a, b, c);
    if (rc) return rc;
    const hipStream_t st = hipStream_t(stream);
    WsCtx ws;
    ws.s = st;
    ws.fixed = true;
    ws.size = TLIB_NOALLOC_SCRATCH_BYTES;
    if (!g_plan_only) {
        void* p = nullptr;
        if ((rc = scratch_address(&p))) return rc;
        ws.base = static_cast<char*>(p);
    }
    const std::string pkey = ttt_pkey(PCK_TTT_NOALLOC, a, b, c, q, phi, psi);
    if (auto L = pc_get(pkey)) {
        g_plan = L->note;
        return exec_launch(*L, a.data, b.data, c.data, ws, st);
    }
    Launch N;
    if (q != 0 || plan_outer(a, b, phi, psi, c, N) != TLIB_OK) {
        rc = plan_ttt(a, b, q, phi, psi, c, TLIB_NOALLOC_SCRATCH_BYTES, N, -1);
        if (rc) return rc;
    }
    rc = exec_launch(N, a.data, b.data, c.data, ws, st);
    if (rc == TLIB_OK) {
        N.note = g_plan;
        pc_put(pkey, N);
    }
    return rc;
}

static int run_dot(const Ten& a, const Ten* b, double* out, bool sq, hipStream_t s, const char* op) {
    WsCtx wsc;
    wsc.s = s;
    Dim d[MAXP];
    for (int r = 0; r < a.p; ++r) d[r] = {a.n[r], {a.w[r], b ? b->w[r] : a.w[r], 0}};
    int nd = coalesce(d, a.p, 2, 0);
    GDims g;
    fill_gdims(g, d, nd, 2);
    int np = dot_partials_g(g);
    size_t wsb = size_t(np) * sizeof(double);
    plan_note("%s dot dtype=%s dims=%d total=%lld partials=%d", op, dname(a.dtype), nd,
              (long long)g.total, np);
    wsc.need(wsb);
    if (g_plan_only) return TLIB_OK;
    void* ws = wsc.take(wsb);
    if (!ws) return ws_fail(wsc, wsb, op);
    int rc = launch_dot(a.dtype, a.data, b ? b->data : nullptr, g, out, sq, ws, wsb, s);
    return rc ? fail(rc, "%s: launch failed", op) : TLIB_OK;
}

int tlib_inner(const tlib_tensor* A, const tlib_tensor* B, double* out_dev, void* stream) {
    begin_call();
    Ten a, b;
    int rc;
    if ((rc = normalize(A, a, "A")) || (rc = normalize(B, b, "B"))) return rc;
    if (!out_dev) return fail(TLIB_EINVAL, "inner: out_dev is NULL");
    if (a.p != b.p) return fail(TLIB_ESHAPE, "inner: orders differ");
    for (int r = 0; r < a.p; ++r)
        if (a.n[r] != b.n[r]) return fail(TLIB_ESHAPE, "inner: extent %d differs", r + 1);
    if (a.dtype != b.dtype) return fail(TLIB_EDTYPE, "inner: dtypes differ");
    return run_dot(a, &b, out_dev, false, hipStream_t(stream), "inner");
}

int tlib_norm(const tlib_tensor* A, double* out_dev, void* stream) {
    begin_call();
    Ten a;
    int rc;
    if ((rc = normalize(A, a, "A"))) return rc;
    if (!out_dev) return fail(TLIB_EINVAL, "norm: out_dev is NULL");
    return run_dot(a, nullptr, out_dev, true, hipStream_t(stream), "norm");
}

// u = v / ||v|| with the norm written to norm_dev (Sec. 5.2, the normalisation
// step of the higher-order power method): the norm kernel, then a division
// that reads the norm from device memory, so nothing returns to the host.
int tlib_normalize(const tlib_tensor* A, double* norm_dev, const tlib_tensor* C, void* stream) {
    begin_call();
    Ten a, c;
    int rc;
    if ((rc = normalize(A, a, "A")) || (rc = normalize(C, c, "C"))) return rc;
    if (!norm_dev) return fail(TLIB_EINVAL, "normalize: norm_dev is NULL");
    if (a.p != c.p) return fail(TLIB_ESHAPE, "normalize: orders differ");
    for (int r = 0; r < a.p; ++r)
        if (a.n[r] != c.n[r]) return fail(TLIB_ESHAPE, "normalize: extent %d differs", r + 1);
    if ((rc = check_output(c, "C"))) return rc;
    const bool in_place = same_view(a, c) && a.dtype == c.dtype;
    if (!in_place && overlaps(c, a)) return fail(TLIB_EALIAS, "normalize: C overlaps A (only C = A is allowed)");
    const hipStream_t s = hipStream_t(stream);
    if ((rc = run_dot(a, nullptr, norm_dev, true, s, "normalize"))) return rc;
    Dim d[MAXP];
    for (int r = 0; r < a.p; ++r) d[r] = {a.n[r], {a.w[r], a.w[r], c.w[r]}};
    const int nd = coalesce(d, a.p, 3, 2);
    GDims g;
    fill_gdims(g, d, nd, 3);
    const std::string dot_plan = g_plan;
    plan_note("; div dtype=%s->%s total=%lld", dname(a.dtype), dname(c.dtype), (long long)g.total);
    g_plan = dot_plan + g_plan;
    if (g_plan_only) return TLIB_OK;
    rc = launch_div(a.dtype, c.dtype, norm_dev, a.data, c.data, g, s);
    return rc ? fail(rc, "normalize: launch failed") : TLIB_OK;
}

static int run_axpby(double alpha, const Ten& a, double beta, const Ten* b, const Ten& c,
                     const int64_t* wA_by_c, hipStream_t s, const char* op) {
    Dim d[MAXP];
    // slot 1 holds B's strides; without B it repeats C's so that it never blocks a merge
    for (int r = 0; r < c.p; ++r) d[r] = {c.n[r], {wA_by_c[r], b ? b->w[r] : c.w[r], c.w[r]}};
    int nd = coalesce(d, c.p, 3, 2);
    // C's fastest dim is d[0]; when A's fastest is another dim y, go through
    // LDS tiles so that A is read along y and C written along x.
    int y = -1;
    for (int i = 1; i < nd; ++i)
        if (y < 0 || d[i].s[0] < d[y].s[0]) y = i;
    if (y > 0 && d[0].s[2] == 1 && d[y].s[0] >= 1 && d[y].s[0] <= 2 && d[0].s[0] > 8 * d[y].s[0] &&
        d[0].n >= 16 && d[y].n >= 16) {
        EwTile t;
        t.nx = d[0].n;
        t.ny = d[y].n;
        for (int o = 0; o < 3; ++o) {
            t.sx[o] = d[0].s[o];
            t.sy[o] = d[y].s[o];
        }
        int64_t nrest = 1;
        for (int i = 1; i < nd; ++i) {
            if (i == y) continue;
            t.rn[t.nr] = uint32_t(d[i].n);
            t.rfd[t.nr] = make_fastdiv(uint32_t(d[i].n));
            for (int o = 0; o < 3; ++o) t.rs[o][t.nr] = d[i].s[o];
            ++t.nr;
            nrest *= d[i].n;
        }
        const int64_t tx = (t.nx + EW_T - 1) / EW_T, ty = (t.ny + EW_T - 1) / EW_T;
        const int64_t ntiles = tx * ty * ((nrest + EW_RZ - 1) / EW_RZ);
        if (ntiles < (int64_t(1) << 31) && nrest < (int64_t(1) << 31)) {
            t.tx = uint32_t(tx);
            t.ty = uint32_t(ty);
            t.ftx = make_fastdiv(t.tx);
            t.fty = make_fastdiv(t.ty);
            t.nrest = uint32_t(nrest);
            t.ntiles = uint32_t(ntiles);
            const int bm = !b ? 0 : (d[y].s[1] < d[0].s[1] ? 2 : 1);
            plan_note("%s ewise tile dtype=%s->%s x=%lld y=%lld rest=%lld b=%d tiles=%lld", op, dname(a.dtype),
                      dname(c.dtype), (long long)t.nx, (long long)t.ny, (long long)nrest, bm, (long long)ntiles);
            if (g_plan_only) return TLIB_OK;
            int rc = launch_axpby_tile(a.dtype, c.dtype, alpha, a.data, beta, b ? b->data : nullptr, c.data, t, bm, s);
            return rc ? fail(rc, "%s: launch failed", op) : TLIB_OK;
        }
    }
    GDims g;
    fill_gdims(g, d, nd, 3);
    plan_note("%s ewise dtype=%s->%s dims=%d total=%lld%s", op, dname(a.dtype), dname(c.dtype), nd, (long long)g.total,
              (nd == 1 && g.s[0][0] == 1 && g.s[2][0] == 1 && (!b || g.s[1][0] == 1)) ? " flat" : "");
    if (g_plan_only) return TLIB_OK;
    int rc = launch_axpby(a.dtype, c.dtype, alpha, a.data, beta, b ? b->data : nullptr, c.data, g, s);
    return rc ? fail(rc, "%s: launch failed", op) : TLIB_OK;
}

int tlib_add(double alpha, const tlib_tensor* A, double beta, const tlib_tensor* B,
             const tlib_tensor* C, void* stream) {
    begin_call();
    Ten a, b, c;
    int rc;
    if ((rc = normalize(A, a, "A")) || (rc = normalize(B, b, "B")) || (rc = normalize(C, c, "C")))
        return rc;
    if (a.p != b.p || a.p != c.p) return fail(TLIB_ESHAPE, "add: orders differ");
    for (int r = 0; r < a.p; ++r)
        if (a.n[r] != b.n[r] || a.n[r] != c.n[r]) return fail(TLIB_ESHAPE, "add: extent %d differs", r + 1);
    if (a.dtype != b.dtype || a.dtype != c.dtype) return fail(TLIB_EDTYPE, "add: dtypes differ");
    if ((rc = check_output(c, "C"))) return rc;
    if ((overlaps(c, a) && !same_view(c, a)) || (overlaps(c, b) && !same_view(c, b)))
        return fail(TLIB_EALIAS, "add: C overlaps an input without being that input");
    return run_axpby(alpha, a, beta, &b, c, a.w, hipStream_t(stream), "add");
}

int tlib_scale(double alpha, const tlib_tensor* A, const tlib_tensor* C, void* stream) {
    begin_call();
    Ten a, c;
    int rc;
    if ((rc = normalize(A, a, "A")) || (rc = normalize(C, c, "C"))) return rc;
    if (a.p != c.p) return fail(TLIB_ESHAPE, "scale: orders differ");
    for (int r = 0; r < a.p; ++r)
        if (a.n[r] != c.n[r]) return fail(TLIB_ESHAPE, "scale: extent %d differs", r + 1);
    if ((rc = check_output(c, "C"))) return rc;
    if (overlaps(c, a) && !(same_view(c, a) && a.dtype == c.dtype))
        return fail(TLIB_EALIAS, "scale: C overlaps A without being A");
    return run_axpby(alpha, a, 0.0, nullptr, c, a.w, hipStream_t(stream), "scale");
}

// Multi-mode TTV in one pass (Sec. 5.2 tensor_times_vectors).  A's modes in
// storage order: the position modes of a tile are the innermost ones (K1:
// every mode up to and including r when few lo positions share an i_r; K2:
// the longest prefix of the lo modes that fits a tile), the rest are rows.
// Modes of extent 1 other than r only contribute u_k(0) to the weight and
// join the hi group.
int tlib_times_vectors(const tlib_tensor* A, const tlib_tensor* const* us, int32_t r, const tlib_tensor* C,
                       void* stream) {
    begin_call();
    Ten a, c;
    Ten u[MAXP];
    int rc;
    if ((rc = normalize(A, a, "A")) || (rc = normalize(C, c, "c"))) return rc;
    if (a.p < 2) return fail(TLIB_EINVAL, "times_vectors: order of A must be >= 2 (got %d)", a.p);
    if (r < 1 || r > a.p) return fail(TLIB_EMODE, "times_vectors: mode %d out of 1..%d", r, a.p);
    if (!us) return fail(TLIB_EINVAL, "times_vectors: us is NULL");
    const int ri = r - 1;
    for (int k = 0; k < a.p; ++k) {
        if (k == ri) continue;
        char nm[16];
        snprintf(nm, sizeof(nm), "u_%d", k + 1);
        if ((rc = normalize(us[k], u[k], nm))) return rc;
        if (u[k].p != 1 || u[k].n[0] != a.n[k])
            return fail(TLIB_ESHAPE, "times_vectors: u_%d must be a vector of length %lld", k + 1,
                        (long long)a.n[k]);
        if (u[k].dtype != a.dtype) return fail(TLIB_EDTYPE, "times_vectors: u_%d must have A's dtype", k + 1);
    }
    if (c.p != 1 || c.n[0] != a.n[ri])
        return fail(TLIB_ESHAPE, "times_vectors: c must be a vector of length n_%d = %lld", r, (long long)a.n[ri]);
    if (c.dtype != acc_dtype(a.dtype))
        return fail(TLIB_EDTYPE, "times_vectors: c must be %s", dname(acc_dtype(a.dtype)));
    if (overlaps(c, a)) return fail(TLIB_EALIAS, "times_vectors: c overlaps A");
    for (int k = 0; k < a.p; ++k)
        if (k != ri && overlaps(c, u[k])) return fail(TLIB_EALIAS, "times_vectors: c overlaps u_%d", k + 1);

    // storage order of the modes of extent > 1 and r
    int ord[MAXP], no = 0, ones[MAXP], n1 = 0;
    for (int k = 0; k < a.p; ++k) {
        if (a.n[k] > 1 || k == ri) ord[no++] = k;
        else ones[n1++] = k;
    }
    std::stable_sort(ord, ord + no, [&](int x, int y) { return a.w[x] < a.w[y]; });
    int rho = 0;
    while (ord[rho] != ri) ++rho;
    int64_t n_lo = 1;
    for (int j = 0; j < rho; ++j) n_lo *= a.n[ord[j]];

    TvParams P{};
    P.A = a.data;
    P.n_r = a.n[ri];
    auto add_mode = [&](TvModes& g, int k) {
        g.n[g.nd] = a.n[k];
        g.fd[g.nd] = make_fastdiv(uint32_t(std::min<int64_t>(a.n[k], 0x7fffffff)));
        g.s[g.nd] = a.w[k];
        g.u[g.nd] = k == ri ? nullptr : u[k].data;
        g.us[g.nd] = k == ri ? 0 : u[k].w[0];
        ++g.nd;
    };
    const bool k2 = n_lo >= 64;
    int a_end;  // position modes are ord[0 .. a_end)
    if (!k2) {
        a_end = rho + 1;
    } else {
        a_end = 1;
        int64_t pp = a.n[ord[0]];
        while (a_end < rho && pp * a.n[ord[a_end]] <= TV_SLOTS) pp *= a.n[ord[a_end++]];
    }
    int64_t npos = 1;
    for (int j = 0; j < a_end; ++j) {
        add_mode(P.pos, ord[j]);
        npos *= a.n[ord[j]];
    }
    int64_t n_out = 1, n_hi = 1;
    if (k2)
        for (int j = a_end; j < rho; ++j) {
            add_mode(P.out, ord[j]);
            n_out *= a.n[ord[j]];
        }
    for (int j = rho + 1; j < no; ++j) {
        add_mode(P.hi, ord[j]);
        n_hi *= a.n[ord[j]];
    }
    for (int j = 0; j < n1; ++j) add_mode(P.hi, ones[j]);
    if (npos >= (int64_t(1) << 31) || n_out >= (int64_t(1) << 30) || a.n[ri] >= (int64_t(1) << 31))
        return fail(TLIB_EINVAL, "times_vectors: A too large for one pass (%lld positions, %lld rows per i)",
                    (long long)npos, (long long)n_out);
    P.k2 = k2 ? 1 : 0;
    P.npos = npos;
    P.n_lo = k2 ? 1 : n_lo;
    P.W = int32_t(std::min<int64_t>(npos, TV_SLOTS));
    P.G = npos <= TV_SLOTS ? int32_t(TV_SLOTS / npos) : 1;
    P.nfc = int32_t((npos + P.W - 1) / P.W);
    P.nloc = k2 ? 1 : int32_t(P.W / n_lo + 2);
    P.n_out = n_out;
    P.n_hi = n_hi;
    P.fd_out = make_fastdiv(uint32_t(n_out));
    P.s_r = a.w[ri];
    // dense row groups: the offset of row (o, h) is o * s_o + h * s_h
    {
        auto linear = [](const TvModes& g, int64_t& s0) {
            s0 = 0;
            int64_t want = -1;
            for (int j = 0; j < g.nd; ++j) {
                if (g.n[j] == 1) continue;
                if (want < 0) s0 = g.s[j];
                else if (g.s[j] != want) return false;
                want = g.s[j] * g.n[j];
            }
            return true;
        };
        // (one weight per row when the row count stays modest, <= 2^26)
        P.lin = (linear(P.out, P.s_o) && linear(P.hi, P.s_h) && n_out * n_hi <= (int64_t(1) << 26)) ? 1 : 0;
    }
    // rows per i_r: n_out * n_hi, split into HC ranges so that the grid holds
    // about 2048 workgroups; a range is at most 2^30 rows
    const int64_t rows = n_out * n_hi;
    const int64_t items = (k2 ? P.n_r : 1) * int64_t(P.nfc);
    int64_t hc = std::max<int64_t>(1, std::min<int64_t>((2048 + items - 1) / items, (rows + P.G - 1) / P.G));
    int64_t tlen = (rows + hc - 1) / hc;
    tlen = std::min<int64_t>(tlen, int64_t(1) << 30);
    hc = (rows + tlen - 1) / tlen;
    if (items * hc >= (int64_t(1) << 31)) return fail(TLIB_EINVAL, "times_vectors: grid too large");
    P.HC = int32_t(hc);
    P.hc_len = tlen;
    // 16-byte loads: dense positions (offset = index), a multiple of the
    // vector in every row offset and in the tile width, aligned base
    const int esz = esize(a.dtype), vlen = 16 / esz;
    bool vec = (uintptr_t(a.data) % 16) == 0 && npos % vlen == 0;
    {
        int64_t want = 1;
        for (int j = 0; j < P.pos.nd; ++j) {
            vec = vec && P.pos.s[j] == want;
            want *= P.pos.n[j];
        }
        for (int j = 0; j < P.out.nd; ++j) vec = vec && (P.out.n[j] == 1 || P.out.s[j] % vlen == 0);
        for (int j = 0; j < P.hi.nd; ++j) vec = vec && (P.hi.n[j] == 1 || P.hi.s[j] % vlen == 0);
        if (k2) vec = vec && (P.n_r == 1 || P.s_r % vlen == 0);
    }
    const int64_t ntab = P.lin ? n_out * n_hi : n_out + n_hi;
    const int64_t nparts = k2 ? P.n_r * P.HC * P.nfc : int64_t(P.HC) * P.nfc * P.nloc;
    const size_t wsb = size_t(ntab) * 16 + size_t(nparts) * 8;
    plan_note("times_vectors %s dtype=%s mode=%d positions=%lld W=%d G=%d chunks=%d rows=%lld (out %lld x hi %lld) "
              "HC=%d vec=%d lin=%d grid=%lld",
              k2 ? "k2" : "k1", dname(a.dtype), r, (long long)npos, P.W, P.G, P.nfc, (long long)rows,
              (long long)n_out, (long long)n_hi, P.HC, vec ? 1 : 0, P.lin, (long long)(items * hc));
    if (g_plan_only) return TLIB_OK;
    hipStream_t s = hipStream_t(stream);
    WsCtx wsc;
    wsc.s = s;
    char* ws = static_cast<char*>(wsc.take(wsb));
    if (!ws) return ws_fail(wsc, wsb, "times_vectors");
    P.tabw = reinterpret_cast<double*>(ws);
    P.tabo = reinterpret_cast<int64_t*>(ws + ntab * 8);
    P.part = reinterpret_cast<double*>(ws + ntab * 16);
    rc = launch_tv(a.dtype, P, c.data, c.w[0], vec, s);
    return rc ? fail(rc, "times_vectors: launch failed") : TLIB_OK;
}

int tlib_transpose(const tlib_tensor* A, const int32_t* tau, const tlib_tensor* C, void* stream) {
    begin_call();
    Ten a, c;
    int rc;
    if ((rc = normalize(A, a, "A")) || (rc = normalize(C, c, "C"))) return rc;
    if (!is_perm(a.p, tau)) return fail(TLIB_EMODE, "transpose: tau is not a permutation of 1..%d", a.p);
    if (c.p != a.p) return fail(TLIB_ESHAPE, "transpose: orders differ");
    int64_t wa[MAXP];
    for (int r = 0; r < a.p; ++r) {
        if (c.n[r] != a.n[tau[r] - 1])
            return fail(TLIB_ESHAPE, "transpose: extent %d of C must be n_%d of A", r + 1, tau[r]);
        wa[r] = a.w[tau[r] - 1];  // C(i^c) = A(i^a), i^c_r = i^a_{tau_r}
    }
    if (a.dtype != c.dtype) return fail(TLIB_EDTYPE, "transpose: dtypes differ");
    if ((rc = check_output(c, "C"))) return rc;
    if (overlaps(c, a)) return fail(TLIB_EALIAS, "transpose: C overlaps A");
    return run_axpby(1.0, a, 0.0, nullptr, c, wa, hipStream_t(stream), "transpose");
}

int tlib_request_check(int32_t op, const tlib_tensor* A, const tlib_tensor* B, int32_t mode, int32_t q,
                       const int32_t* phi, const int32_t* psi, const tlib_tensor* C) {
    begin_call();
    if (op < 0 || op > 2) return fail(TLIB_EINVAL, "request: unknown op %d", op);
    if (!A || !B || !C) return fail(TLIB_EINVAL, "request: NULL descriptor");
    if (op == 2 && (!phi || !psi)) return fail(TLIB_EINVAL, "request: TTT needs phi and psi");
    // a result the server places later is checked at a stand-in address far
    // below any device allocation
    tlib_tensor c = *C;
    if (!c.data) c.data = reinterpret_cast<void*>(uintptr_t(4096));
    const bool po = g_plan_only;
    const std::string plan = g_plan;
    g_plan_only = true;
    int rc;
    if (op == 0) rc = tlib_ttv(A, B, mode, &c, nullptr);
    else if (op == 1) rc = tlib_ttm(A, B, mode, &c, nullptr);
    else rc = tlib_ttt(A, B, q, phi, psi, &c, nullptr);
    g_plan_only = po;
    g_plan = plan;
    return rc;
}

size_t tlib_batch_table_bytes(int32_t n) {
    return sizeof(BatchHeader) + size_t(n < 0 ? 0 : n) * sizeof(BatchItem);
}

// Validate one grouped request and collapse it (rc TLIB_ESTRIDE: valid, but
// not for the grouped kernel).
static int batch_request(const tlib_request& r, BatchItem& it) {
    Ten a, b, c;
    int rc;
    if (r.op == 0) rc = check_ttv(r.A, r.B, r.mode, r.C, a, b, c);
    else if (r.op == 1) rc = check_ttm(r.A, r.B, r.mode, r.C, a, b, c);
    else if (r.op == 2) rc = check_ttt(r.A, r.B, r.q, r.phi, r.psi, r.C, a, b, c);
    else return fail(TLIB_EINVAL, "batch: unknown op %d", r.op);
    if (rc) return rc;
    if (!batch_item(r.op, a, b, c, r.mode - 1, r.q, r.phi, r.psi, it))
        return fail(TLIB_ESTRIDE, "batch: a request does not collapse to the grouped kernel's index groups");
    // one grouped thread or tile carries the whole contraction in one FP32
    // (or FP64) accumulator chain; longer ones go to the single entry points,
    // whose split-K keeps the chains short
    if (it.K > TLIB_BATCH_MAX_K)
        return fail(TLIB_EINVAL, "batch: contraction of %lld exceeds the grouped kernel's %d", (long long)it.K,
                    TLIB_BATCH_MAX_K);
    return TLIB_OK;
}

int tlib_batch_plan(const tlib_request* reqs, int32_t n, void* table_host, size_t table_bytes,
                    int64_t* units, int32_t* bad) {
    begin_call();
    if (bad) *bad = -1;
    if (n < 0 || (n > 0 && !reqs) || !table_host) return fail(TLIB_EINVAL, "batch: NULL argument");
    if (table_bytes < tlib_batch_table_bytes(n)) return fail(TLIB_EINVAL, "batch: table too small");
    BatchHeader* hdr = (BatchHeader*)table_host;
    BatchItem* items = (BatchItem*)((char*)table_host + sizeof(BatchHeader));
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        const int rc = batch_request(reqs[i], items[i]);
        if (rc) {
            if (bad) *bad = i;
            return rc;
        }
        items[i].unit_begin = total;
        total += batch_units(items[i]);
    }
    hdr->n_items = n;
    hdr->total_units = total;
    if (units) *units = total;
    plan_note("batch items=%d units=%lld", n, (long long)total);
    return TLIB_OK;
}

int tlib_request_groupable(const tlib_request* r) {
    begin_call();
    if (!r || !r->C) return 0;
    // a result the server places later is checked at a stand-in address
    tlib_tensor c = *r->C;
    if (!c.data) c.data = reinterpret_cast<void*>(uintptr_t(4096));
    tlib_request q = *r;
    q.C = &c;
    BatchItem it;
    return batch_request(q, it) == TLIB_OK ? 1 : 0;
}

int tlib_batch_run(const void* table_dev, int32_t grid, void* stream) {
    begin_call();
    if (!table_dev) return fail(TLIB_EINVAL, "batch: table is NULL");
    if (grid < 0) return fail(TLIB_EINVAL, "batch: grid < 0");
    if (g_plan_only) {
        plan_note("batch run grid=%d", grid ? grid : 1024);
        return TLIB_OK;
    }
    int rc = launch_batch(table_dev, grid ? grid : 1024, hipStream_t(stream));
    return rc ? fail(rc, "batch: launch failed") : TLIB_OK;
}

int tlib_strides_from_layout(int32_t order, const int64_t* extents, const int32_t* layout,
                             int64_t* strides_out) {
    begin_call();
    if (order < 0 || order > MAXP) return fail(TLIB_EINVAL, "order out of range");
    if ((order > 0 && !extents) || !strides_out) return fail(TLIB_EINVAL, "NULL argument");
    int64_t dummy = 0;
    tlib_tensor t{&dummy, TLIB_F64, order, extents, nullptr, layout};
    Ten o;
    int rc = normalize(&t, o, "tensor");
    if (rc) return rc;
    for (int r = 0; r < order; ++r) strides_out[r] = o.w[r];
    return TLIB_OK;
}

int tlib_workspace_reserve(void* stream, size_t bytes) {
    begin_call();
    hipStream_t s = hipStream_t(stream);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(TLIB_EHIP, "workspace_reserve: no device");
    if (capturing(s)) return fail(TLIB_EINVAL, "workspace_reserve: the stream is capturing a graph");
    bytes = ws_round(std::max<size_t>(bytes, 1));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    WsBuf& e = g_ws[{dev, s}];
    if (e.ptr && e.bytes >= bytes) return TLIB_OK;
    void* p = ws_alloc(bytes);
    if (!p) return fail(TLIB_ENOMEM, "workspace_reserve: hipMalloc of %zu bytes failed", bytes);
    if (e.ptr) e.retired.push_back(e.ptr);  // graphs captured earlier may still use it
    e.ptr = static_cast<char*>(p);
    e.bytes = bytes;
    return TLIB_OK;
}

size_t tlib_workspace_size(void* stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({dev, hipStream_t(stream)});
    return it == g_ws.end() ? 0 : it->second.bytes;
}

int tlib_workspace_release(void* stream) {
    begin_call();
    hipStream_t s = hipStream_t(stream);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(TLIB_EHIP, "workspace_release: no device");
    if (capturing(s)) return fail(TLIB_EINVAL, "workspace_release: the stream is capturing a graph");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find({dev, s});
    if (it == g_ws.end()) return TLIB_OK;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(TLIB_EHIP, "workspace_release: stream wait failed");
    for (void* p : it->second.retired) (void)hipFree(p);
    if (it->second.ptr) (void)hipFree(it->second.ptr);
    g_ws.erase(it);
    return TLIB_OK;
}

void tlib_plan_cache_stats(int64_t* entries, int64_t* hits, int64_t* misses) {
    std::lock_guard<std::mutex> lk(g_pc_mu);
    if (entries) *entries = int64_t(g_pc.size());
    if (hits) *hits = g_pc_hits.load();
    if (misses) *misses = g_pc_misses.load();
}

void tlib_plan_cache_clear(void) { pc_clear(); }

const char* tlib_last_error(void) { return g_err.c_str(); }

const char* tlib_strerror(int code) {
    switch (code) {
        case TLIB_OK: return "ok";
        case TLIB_EINVAL: return "invalid argument";
        case TLIB_ESHAPE: return "shape mismatch";
        case TLIB_EMODE: return "invalid mode or permutation";
        case TLIB_EDTYPE: return "unsupported or mismatched dtype";
        case TLIB_EALIAS: return "output overlaps an input";
        case TLIB_ESTRIDE: return "output strides overlap";
        case TLIB_ENOMEM: return "not enough workspace";
        case TLIB_EHIP: return "HIP launch failed";
    }
    return "unknown error";
}

void tlib_set_plan_only(int enable) { g_plan_only = enable != 0; }
const char* tlib_last_plan(void) { return g_plan.c_str(); }
const char* tlib_version(void) { return "tlib-mi355x 0.1 (gfx950)"; }

}  // extern "C"
