/*
 * tlib -- MI355X (gfx950) tensor-contraction library, C ABI.
 *
 * Operations of Bassoy, "TLib: A Flexible C++ Tensor Framework for Numerical
 * Tensor Calculus" (arXiv 1711.10912), Sec. 5: tensor-times-vector (Eq. ttv),
 * tensor-times-matrix (Eq. ttm), tensor-times-tensor (Eq. ttt, ttt_indices),
 * inner product and Frobenius norm (Table 3), entrywise scaling and sums
 * (Sec. 5.1 Eq. scaling, Eq. transform) and transposition (Table 3).
 *
 * Tensors.  A tensor is described by a tlib_tensor: a device pointer to its
 * element with multi-index (0,...,0), its order p, its shape tuple n and its
 * stride tuple w in elements (Sec. 3.1).  The element with zero-based
 * multi-index i lives at data[ sum_r w_r i_r ] (layout function, Sec. 3.2
 * Eq. f with zero index offsets).  Either the strides are given explicitly, or
 * they are derived from a 1-based layout tuple pi by Sec. 3.1
 * Eq. stride.tuple.permutation (pi = NULL means first-order, Eq.
 * layout.tuple.first.order).  A view (Sec. 3.3) is passed as its parent's
 * pointer plus gamma (Eq. view_gamma) with strides w_r * t_r.  Strides must
 * be >= 0; the strides of an output must map distinct multi-indices to
 * distinct addresses (checked conservatively: sorted by stride, each stride
 * must be at least the previous stride times its extent).
 *
 * Modes (m, phi, psi, tau) are 1-based as in the paper's equations.
 *
 * Data types.  A, B and b share one dtype.  Contractions write C in FP64 for
 * FP64 inputs and in FP32 for FP32, BF16 and FP16 inputs (accumulation in
 * FP64 resp. FP32).  add / transpose keep the input dtype, scale may convert.  inner and
 * norm accumulate and return FP64 for every input dtype.
 *
 * Ownership.  The caller owns every buffer.  The library never allocates or
 * frees caller-visible memory.  It keeps one workspace per (device, stream)
 * for reduction and split-K partials and for the intermediate of a two-TTM
 * chain (see tlib_workspace_reserve); host arrays (extents, strides, layout,
 * phi, psi, tau) are read during the call only.
 *
 * Synchronisation.  Arguments are validated on the host before anything is
 * launched.  Kernels are enqueued on `stream` (a hipStream_t; NULL is the
 * default stream) and the call returns without waiting for them: no entry
 * point synchronises, frees memory or grows the workspace (the one exception
 * is the first call of a new call shape with autotuning on, see
 * tlib_set_autotune).  Every call can therefore be captured in a HIP graph
 * once the stream's workspace exists and is large enough.  C is
 * overwritten, never accumulated into.  Calls on one stream run in order;
 * calls on different streams may overlap.
 *
 * Errors.  Every entry point returns 0 (TLIB_OK) or one of the codes below;
 * nothing is thrown across the ABI.  On an error nothing has been launched
 * and C is untouched (TLIB_EHIP: a launch failed; C is unspecified).
 * tlib_last_error() returns a message for the calling thread's last error.
 */
#ifndef TLIB_H
#define TLIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TLIB_MAX_ORDER 16

typedef enum { TLIB_F64 = 0, TLIB_F32 = 1, TLIB_BF16 = 2, TLIB_F16 = 3 } tlib_dtype;

enum {
    TLIB_OK = 0,
    TLIB_EINVAL = 1,  /* null pointer, order out of range, extent < 1, stride < 0, p < 2 for TTV/TTM */
    TLIB_ESHAPE = 2,  /* extents do not match the operation's shape rules */
    TLIB_EMODE = 3,   /* a mode out of 1..p, or phi/psi/tau/layout not a permutation */
    TLIB_EDTYPE = 4,  /* unsupported dtype, or operands / output of the wrong dtype */
    TLIB_EALIAS = 5,  /* the output overlaps an input (add/scale may run in place, see there) */
    TLIB_ESTRIDE = 6, /* the output's strides may map two multi-indices to one address */
    TLIB_ENOMEM = 7,  /* the stream's workspace is too small (or could not be allocated) */
    TLIB_EHIP = 8     /* a HIP call or kernel launch failed */
};

typedef struct {
    void* data;              /* device pointer to element (0,...,0) */
    int32_t dtype;           /* tlib_dtype */
    int32_t order;           /* p, 0 <= p <= TLIB_MAX_ORDER */
    const int64_t* extents;  /* n[0..p-1], each >= 1 (host memory) */
    const int64_t* strides;  /* w[0..p-1] in elements, or NULL (host memory) */
    const int32_t* layout;   /* pi[0..p-1], 1-based, used when strides == NULL; NULL = first-order */
} tlib_tensor;

/* Mode-m tensor-times-vector, Sec. 5.2 Eq. ttv:
 *   C(i_1..i_{m-1}, i_{m+1}..i_p) = sum_{i_m} A(i_1..i_p) * b(i_m).
 * A: order p >= 2.  b: order 1, extent n_m, any stride.  C: order p-1 with the
 * extents of A without n_m, in the mode order of A.  1 <= m <= p. */
int tlib_ttv(const tlib_tensor* A, const tlib_tensor* b, int32_t m,
             const tlib_tensor* C, void* stream);

/* Mode-m tensor-times-matrix, Sec. 5.2 Eq. ttm:
 *   C(i_1..i_{m-1}, j, i_{m+1}..i_p) = sum_{i_m} A(i_1..i_p) * B(j, i_m).
 * A: order p >= 2.  B: order 2 with shape (n', n_m), any strides.
 * C: order p, extents of A with n_m replaced by n'. */
int tlib_ttm(const tlib_tensor* A, const tlib_tensor* B, int32_t m,
             const tlib_tensor* C, void* stream);

/* Two mode products in one pass, C = (A x_a Ua) x_b Ub (Sec. 5.2 Eq. ttm in
 * modes a and b, a != b; one step pair of tensor_times_matrices, as in the
 * Tucker chain):
 *   C(.., j_a, .., j_b, ..) = sum_{i_a, i_b} Ua(j_a, i_a) Ub(j_b, i_b) A(.., i_a, .., i_b, ..).
 * A: order p >= 2, FP64 or FP32, any strides.  Ua: shape (n'_a, n_a), Ub:
 * shape (n'_b, n_b), A's dtype, any strides.  C: extents of A with n_a, n_b
 * replaced by n'_a, n'_b, A's dtype, any injective strides, no overlap with
 * an input.  Without writing A x_a Ua when n'_a, n'_b <= 32 and n_a, n_b <=
 * 256 (the result is the same product summed in another order); otherwise
 * two TTMs through an intermediate held in the stream's workspace
 * (TLIB_ENOMEM if it is too small).  16-bit inputs:
 * TLIB_EDTYPE (use two tlib_ttm calls). */
int tlib_ttm2(const tlib_tensor* A, const tlib_tensor* Ua, int32_t a, const tlib_tensor* Ub,
              int32_t b, const tlib_tensor* C, void* stream);

/* (q, phi, psi)-mode tensor-times-tensor, Sec. 5.2 Eq. ttt and ttt_indices.
 * A has order q+r, B order q+s (r, s, q >= 0, q+r > 0, q+s > 0); phi (length
 * q+r) and psi (length q+s) are 1-based permutations.  C has order r+s with
 * n^c_k = n^a_{phi_k} (k <= r), n^c_{r+k} = n^b_{psi_k} (k <= s); the pairs
 * (phi_{r+k}, psi_{s+k}), k = 1..q, are contracted and must have equal
 * extents.  q = 0 is the outer product; r = s = 0 gives an order-0 C (one
 * element) holding the inner product. */
int tlib_ttt(const tlib_tensor* A, const tlib_tensor* B, int32_t q,
             const int32_t* phi, const int32_t* psi,
             const tlib_tensor* C, void* stream);

/* tlib_ttt for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same operation, arguments and errors as tlib_ttt, but no workspace.  Its
 * split-K partials live in a static device array of
 * TLIB_NOALLOC_SCRATCH_BYTES per GPU, part of the library's code object and
 * held until the process ends; the split is bounded by that size (a product
 * whose single slice would not fit runs unsplit, so no size is refused; a
 * plan that needed more would return TLIB_ENOMEM before launching).  The tile
 * is the planner's rule (no autotuning).  The call allocates nothing and never
 * synchronises.  Every call on one GPU shares that GPU's array, which keeps
 * the last call's partials: calls that may overlap on one GPU (different
 * streams, or graphs replayed concurrently) race on it and must be ordered by
 * the caller.  Results equal tlib_ttt's within the summation-order rounding. */
#define TLIB_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
int tlib_ttt_noalloc(const tlib_tensor* A, const tlib_tensor* B, int32_t q,
                     const int32_t* phi, const int32_t* psi,
                     const tlib_tensor* C, void* stream);

/* Inner product <A, B> = sum_i A(i) B(i) (Sec. 5.2 Table 3) over equal shapes
 * with independent layouts.  Accumulates in FP64 in a fixed order that only
 * depends on the shapes and strides; writes one double to out_dev (device). */
int tlib_inner(const tlib_tensor* A, const tlib_tensor* B, double* out_dev, void* stream);

/* Frobenius norm sqrt(<A, A>) (Sec. 5.2 Table 3); one double to out_dev (device). */
int tlib_norm(const tlib_tensor* A, double* out_dev, void* stream);

/* Normalisation step of the higher-order power method (Sec. 5.2):
 * *norm_dev = ||A||_F (FP64, as tlib_norm) and C = A / ||A||_F, the quotient
 * formed in FP64 and rounded once to C's dtype.  norm_dev is device memory
 * and the division reads it there, so the pair runs without a host round
 * trip.  C has A's shape, any dtype and injective strides; C may be A itself
 * (same pointer, strides and dtype), any other overlap is TLIB_EALIAS.  Uses
 * the stream's workspace for the norm's partial sums. */
int tlib_normalize(const tlib_tensor* A, double* norm_dev, const tlib_tensor* C, void* stream);

/* C = alpha A + beta B (Sec. 5.1 Eq. transform with a scaled sum).  A, B, C
 * have equal shapes and independent layouts and share one dtype.  C may be
 * the same tensor as A or B (same data pointer and same strides); any other
 * overlap is TLIB_EALIAS. */
int tlib_add(double alpha, const tlib_tensor* A, double beta, const tlib_tensor* B,
             const tlib_tensor* C, void* stream);

/* C = alpha A (Sec. 5.1 Eq. scaling).  Equal shapes, independent layouts: with
 * a different layout for C this is a relayout.  C may have another dtype than
 * A (a conversion, rounded once to nearest-even from the FP64 value alpha*A).
 * C may be A itself (same pointer, strides and dtype). */
int tlib_scale(double alpha, const tlib_tensor* A, const tlib_tensor* C, void* stream);

/* Transposition C = A^tau (Sec. 5.2 Table 3): C(i^c) = A(i^a) with
 * i^c_r = i^a_{tau_r} and n^c_r = n^a_{tau_r}; tau is a 1-based permutation.
 * Same dtype in and out; C must not overlap A. */
int tlib_transpose(const tlib_tensor* A, const int32_t* tau, const tlib_tensor* C, void* stream);

/* Multi-mode tensor-times-vector (Sec. 5.2 tensor_times_vectors, the product
 * of the higher-order power method), in one pass over A:
 *   c(i_r) = sum over all i_k, k != r, of A(i_1..i_p) * prod_{k != r} u_k(i_k).
 * A: order p >= 2, any strides.  us: array of p descriptor pointers (host
 * memory); us[r-1] is not read and may be NULL, every other us[k-1] is a
 * vector of length n_k with A's dtype, any stride.  c: order 1, length n_r,
 * FP64 for FP64 A and FP32 otherwise; it must not overlap A or a vector.
 * Accumulates in FP64 in a fixed order (bitwise reproducible) and rounds once
 * to c's dtype.  Uses the stream's workspace (16 bytes per index of the
 * modes outside the tile positions plus the partial sums; TLIB_ENOMEM if it
 * is too small); TLIB_EINVAL if A has more than 2^31 tile positions or 2^30
 * row entries outside r. */
int tlib_times_vectors(const tlib_tensor* A, const tlib_tensor* const* us, int32_t r,
                       const tlib_tensor* c, void* stream);

/* ---- Grouped launch of many small TTV / TTM / TTT requests -------------------
 * A request is a TTV (op 0, B = the vector b, mode = m), a TTM (op 1, B = the
 * matrix, mode = m) or a TTT (op 2, q, phi, psi) with the same argument rules
 * as tlib_ttv / tlib_ttm / tlib_ttt.  tlib_batch_plan validates n requests and
 * writes a work table into caller-provided host memory of
 * tlib_batch_table_bytes(n) bytes; the caller copies the table to device
 * memory and runs it with tlib_batch_run, which enqueues one kernel whose
 * arguments depend only on the table's device address and the grid: the
 * launch can be captured in a HIP graph once and replayed after the table's
 * contents change.  TTV requests run one thread per output; TTM and TTT
 * requests run as 16 x 64 tiles of C on matrix cores.  Each request's result
 * depends only on the request, never on the rest of the batch.  Requests must
 * not alias each other's outputs.  A request whose index groups do not
 * collapse to at most four (extent, stride) pairs each (and 2^31 indices) is
 * rejected with TLIB_ESTRIDE and its index in *bad (run it with the single
 * entry points instead; tlib_request_groupable tells in advance).  A request
 * whose contraction (n_m for TTV / TTM, the product of the contracted extents
 * for TTT) exceeds TLIB_BATCH_MAX_K is rejected the same way with
 * TLIB_EINVAL: a grouped thread or tile accumulates the whole contraction in
 * one chain, and the single entry points split long ones, which keeps FP32
 * results within their error bound.  *units receives the number of work
 * units. */
#define TLIB_BATCH_MAX_K 8192
typedef struct {
    int32_t op;              /* 0 = TTV, 1 = TTM, 2 = TTT */
    int32_t mode;            /* TTV / TTM: m, 1-based */
    const tlib_tensor* A;
    const tlib_tensor* B;
    const tlib_tensor* C;
    int32_t q;               /* TTT: number of contracted pairs */
    int32_t reserved;
    const int32_t* phi;      /* TTT: length order(A), 1-based (host memory) */
    const int32_t* psi;      /* TTT: length order(B), 1-based (host memory) */
} tlib_request;

size_t tlib_batch_table_bytes(int32_t n);
int tlib_batch_plan(const tlib_request* reqs, int32_t n, void* table_host, size_t table_bytes,
                    int64_t* units, int32_t* bad);
/* table_dev: device copy of a planned table; grid: persistent workgroups (0 = 1024). */
int tlib_batch_run(const void* table_dev, int32_t grid, void* stream);
/* 1 if the request is valid and fits the grouped kernel, 0 otherwise (host only). */
int tlib_request_groupable(const tlib_request* r);

/* ---- Request server (continuous batching on one GPU) ------------------------
 * tlib_server_create starts a scheduler thread with `slots` HIP streams and an
 * output arena of `output_budget` bytes of device memory (the HBM budget for
 * results in flight; 0 = outputs always supplied by the caller).  Requests are
 * admitted in arrival order while a slot is free and the output fits; requests
 * that arrive while others run start as soon as a slot and memory free up.
 * Consecutive TTV/TTM/TTT requests of at most `group_macs` multiply-adds that
 * fit the grouped kernel (tlib_request_groupable) are fused (up to
 * `group_max`) into one grouped launch replayed from a per-slot HIP graph.  A request's kernel depends only on the request, so its result is the
 * same alone and in any mix.
 * tlib_server_submit: op 0 = TTV (B = b), 1 = TTM (B = matrix), 2 = TTT (q,
 * phi, psi as tlib_ttt); A and B are caller-owned device tensors that must be
 * fully written before submission (the slots do not wait on other streams)
 * and stay valid until the request completes.  C gives the result's shape and
 * strides or layout; with C->data == NULL the server places the result in its
 * arena (released at completion unless keep_results), otherwise it writes to
 * C->data.  Arguments are validated at submission by tlib_request_check (an
 * invalid request returns its error code and is not queued); a request whose
 * launch fails is counted in the statistics' `errors`.  Returns TLIB_ENOMEM
 * if the result can never fit the arena.  *rid receives the request id.
 * Each slot's stream gets a workspace of TLIB_WORKSPACE_DEFAULT_BYTES at
 * creation; a request that needs more fails with TLIB_ENOMEM.
 * tlib_server_result: the output descriptor and error code of a completed
 * request (keep_results servers only; pointers valid until destroy).
 * tlib_server_drain waits until nothing is pending or running.
 * Statistics cover requests completed since creation or the last reset:
 * latency = completion (GPU event, on the host clock) - submission. */
typedef struct tlib_server tlib_server;
typedef struct {
    int64_t completed, grouped, errors;
    double p50_s, p99_s, mean_s, req_per_s;
} tlib_server_stats_t;

tlib_server* tlib_server_create(int32_t device, size_t output_budget, int32_t slots, int32_t group_max,
                                int64_t group_macs, int32_t keep_results);
/* Validate one request without running it (the checks of tlib_ttv, tlib_ttm
 * or tlib_ttt, every descriptor read only after its order and pointers are
 * checked); C->data may be NULL (a result the server places).  Host only. */
int tlib_request_check(int32_t op, const tlib_tensor* A, const tlib_tensor* B, int32_t mode, int32_t q,
                       const int32_t* phi, const int32_t* psi, const tlib_tensor* C);
int tlib_server_submit(tlib_server* s, int32_t op, const tlib_tensor* A, const tlib_tensor* B, int32_t mode,
                       int32_t q, const int32_t* phi, const int32_t* psi, const tlib_tensor* C, int64_t* rid);
int tlib_server_drain(tlib_server* s, double timeout_s);
int tlib_server_stats(tlib_server* s, tlib_server_stats_t* out);
int tlib_server_result(tlib_server* s, int64_t rid, tlib_tensor* out, int32_t* err);
void tlib_server_reset_stats(tlib_server* s);
void tlib_server_destroy(tlib_server* s);

/* ---- Workspace -------------------------------------------------------------
 * Scratch that some calls need (reduction partials of inner/norm, split-K
 * partials of TTM/TTT, k-split partials of TTV, tables and partials of
 * times_vectors, the intermediate of a ttm2 chain) comes from one device
 * buffer per (device, stream); a call uses it from its start, so calls on the
 * same stream share it in stream order.  The buffer is created by
 * tlib_workspace_reserve, or else by the first call on the stream that needs
 * scratch while the stream is not capturing a graph, with
 * max(that call's need, TLIB_WORKSPACE_DEFAULT_BYTES) bytes.  A call that needs
 * more than the buffer holds, or that needs scratch on a capturing stream
 * without one, returns TLIB_ENOMEM before launching anything.
 * tlib_workspace_reserve(stream, bytes): make the stream's buffer at least
 *   `bytes` (current device; not on a capturing stream: TLIB_EINVAL).  A
 *   smaller buffer it replaces is kept until tlib_workspace_release, so graphs
 *   captured with it stay valid.  Does not wait for the stream.
 * tlib_workspace_size(stream): bytes of the stream's buffer (0 if none).
 * tlib_workspace_release(stream): wait for the stream, then free its buffers.
 *   Graphs captured from calls on the stream must not be replayed afterwards. */
#define TLIB_WORKSPACE_DEFAULT_BYTES ((size_t)256 << 20)
int tlib_workspace_reserve(void* stream, size_t bytes);
size_t tlib_workspace_size(void* stream);
int tlib_workspace_release(void* stream);

/* Stride tuple from shape and 1-based layout (Sec. 3.1 Eq. stride.tuple.permutation),
 * layout NULL = first-order.  Host only; writes order values to strides_out. */
int tlib_strides_from_layout(int32_t order, const int64_t* extents, const int32_t* layout,
                             int64_t* strides_out);

/* Message for the calling thread's last error ("" if none); the pointer stays
 * valid until the thread's next tlib call. */
const char* tlib_last_error(void);

/* Static text for an error code. */
const char* tlib_strerror(int code);

/* Plan-only mode for the calling thread: when enabled, the entry points above
 * validate and plan but launch nothing and touch no device; tlib_last_plan()
 * then describes the kernel and the collapsed problem that would have run.
 * Used to test the host logic without a GPU. */
void tlib_set_plan_only(int enable);
const char* tlib_last_plan(void);

/* Autotuning of the kernel choice for tlib_ttm and tlib_ttt.  The extents,
 * layouts and modes of a call decide which kernel and tile shape run fastest
 * on MI355X; with autotuning the choice is measured instead of taken from the
 * planner's rules.  Process-wide mode:
 *   TLIB_AUTOTUNE_OFF     the planner's fixed rules (default);
 *   TLIB_AUTOTUNE_ON      the first call of each new call shape (op, modes,
 *                         extents, strides, dtypes) times every applicable
 *                         candidate on the caller's stream, which makes that
 *                         one call synchronous, and keeps the fastest; later
 *                         calls of the shape use the stored choice;
 *   TLIB_AUTOTUNE_FROZEN  stored choices are used, new shapes get the rules.
 * Each tuned choice is stored twice: for the exact call shape and for its
 * shape class (op, dtype, which operands hold their smallest stride in a
 * contracted mode, where C holds its smallest stride, and the base-4
 * logarithms of the problem's extents), the first tuned shape of a class
 * giving the class its choice.  A call shape
 * with no exact entry takes its class's choice in FROZEN mode and is tuned
 * in ON mode.  Calls on a stream that is capturing a graph never tune.  The table is
 * shared by all threads and guarded by a lock.  tlib_autotune_entries
 * returns the number of stored choices; tlib_autotune_clear empties the
 * table.  Candidates differ only in summation order inside the MFMAs, so
 * results are reproducible for a fixed table. */
#define TLIB_AUTOTUNE_OFF 0
#define TLIB_AUTOTUNE_ON 1
#define TLIB_AUTOTUNE_FROZEN 2
int tlib_set_autotune(int mode);  /* returns the previous mode, or -1 (and changes nothing) for an unknown mode */
int64_t tlib_autotune_entries(void);
void tlib_autotune_clear(void);
/* The table as text, one "<choice> <call shape>" line per entry: save writes
 * it to `path` (TLIB_EINVAL if the file cannot be written); load adds the
 * entries of such a file to the table (TLIB_EINVAL if it cannot be read or a
 * line is malformed; entries before the bad line are kept).  A saved table
 * lets another process (a profiler run, a server restart) reuse the choices
 * without tuning again. */
int tlib_autotune_save(const char* path);
int tlib_autotune_load(const char* path);

/* Plan cache.  tlib_ttv, tlib_ttm and tlib_ttt keep the plan of each call
 * shape (operation, modes, and per operand its dtype, order, extents,
 * strides and address modulo 16): a repeated shape skips the
 * planner and only fills in the data pointers.  Thread-safe; emptied when it
 * holds 8192 plans and whenever the autotune mode or table changes.  Stats
 * count the lookups of validated calls since the library was loaded. */
void tlib_plan_cache_stats(int64_t* entries, int64_t* hits, int64_t* misses);
void tlib_plan_cache_clear(void);

/* Library version string. */
const char* tlib_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TLIB_H */
