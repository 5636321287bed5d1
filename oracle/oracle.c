/*
 * Plain FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Each function is the defining equation of the paper written out as loops:
 * one output element at a time, its multi-index decoded from a first-order
 * counter, the contracted indices visited in ascending (odometer, first index
 * fastest) order, accumulation in double.  The only parallelism is OpenMP over
 * independent output elements, which does not change any result.
 */
#include "oracle.h"
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORA_MAXP 32

/* Decode a first-order (first index fastest) linear counter into a multi-index. */
static void decode_first_order(int64_t lin, int p, const int64_t* n, int64_t* idx)
{
    for (int r = 0; r < p; ++r) {
        idx[r] = lin % n[r];
        lin /= n[r];
    }
}

/* Layout function with zero offsets (Sec. 3.2 Eq. f): sum_r w_r * i_r. */
static int64_t layout_fn(int p, const int64_t* w, const int64_t* idx)
{
    int64_t a = 0;
    for (int r = 0; r < p; ++r) a += w[r] * idx[r];
    return a;
}

static int64_t prod(int p, const int64_t* n)
{
    int64_t s = 1;
    for (int r = 0; r < p; ++r) s *= n[r];
    return s;
}

/* 1-based permutation check. */
static int is_perm(int p, const int32_t* v)
{
    int seen[ORA_MAXP];
    if (p < 0 || p > ORA_MAXP) return 0;
    memset(seen, 0, sizeof(seen));
    for (int r = 0; r < p; ++r) {
        if (v[r] < 1 || v[r] > p || seen[v[r] - 1]) return 0;
        seen[v[r] - 1] = 1;
    }
    return 1;
}

int ora_strides(int p, const int64_t* n, const int32_t* pi, int64_t* w)
{
    if (!is_perm(p, pi)) return -1;
    /* w_{pi_1} = 1; w_{pi_r} = prod_{q=1}^{r-1} n_{pi_q} */
    int64_t acc = 1;
    for (int r = 0; r < p; ++r) {
        w[pi[r] - 1] = acc;
        acc *= n[pi[r] - 1];
    }
    return 0;
}

int ora_ttv(int p, const int64_t* n, const double* A, const int64_t* wA,
            const double* b, int64_t wb, int m, double* C, const int64_t* wC)
{
    if (p < 2 || p > ORA_MAXP || m < 1 || m > p) return -1;
    const int mi = m - 1;
    int64_t nc[ORA_MAXP];
    for (int r = 0, k = 0; r < p; ++r)
        if (r != mi) nc[k++] = n[r];
    const int64_t total = prod(p - 1, nc);
    const int64_t nm = n[mi];
#pragma omp parallel for schedule(static)
    for (int64_t lin = 0; lin < total; ++lin) {
        int64_t c[ORA_MAXP], i[ORA_MAXP];
        decode_first_order(lin, p - 1, nc, c);
        /* i_r = c_r for r < m, i_r = c_{r-1} for r > m (Eq. ttv, shape of C) */
        for (int r = 0, k = 0; r < p; ++r)
            i[r] = (r == mi) ? 0 : c[k++];
        double acc = 0.0;
        for (int64_t im = 0; im < nm; ++im) {
            i[mi] = im;
            acc += A[layout_fn(p, wA, i)] * b[im * wb];
        }
        C[layout_fn(p - 1, wC, c)] = acc;
    }
    return 0;
}

int ora_ttm(int p, const int64_t* n, const double* A, const int64_t* wA,
            int64_t nb0, const double* B, const int64_t* wB, int m,
            double* C, const int64_t* wC)
{
    if (p < 2 || p > ORA_MAXP || m < 1 || m > p || nb0 < 1) return -1;
    const int mi = m - 1;
    int64_t nc[ORA_MAXP];
    for (int r = 0; r < p; ++r) nc[r] = n[r];
    nc[mi] = nb0;
    const int64_t total = prod(p, nc);
    const int64_t nm = n[mi];
#pragma omp parallel for schedule(static)
    for (int64_t lin = 0; lin < total; ++lin) {
        int64_t c[ORA_MAXP], i[ORA_MAXP];
        decode_first_order(lin, p, nc, c);
        const int64_t j = c[mi];
        for (int r = 0; r < p; ++r) i[r] = c[r];
        double acc = 0.0;
        for (int64_t im = 0; im < nm; ++im) {
            i[mi] = im;
            acc += A[layout_fn(p, wA, i)] * B[j * wB[0] + im * wB[1]];
        }
        C[layout_fn(p, wC, c)] = acc;
    }
    return 0;
}

int ora_ttt(int pa, const int64_t* na, const double* A, const int64_t* wA,
            int pb, const int64_t* nb, const double* B, const int64_t* wB,
            int q, const int32_t* phi, const int32_t* psi,
            double* C, const int64_t* wC)
{
    const int r = pa - q, s = pb - q;
    if (q < 0 || r < 0 || s < 0 || pa > ORA_MAXP || pb > ORA_MAXP) return -1;
    if (pa == 0 || pb == 0) return -1; /* r+q > 0 and s+q > 0 */
    if (!is_perm(pa, phi) || !is_perm(pb, psi)) return -1;
    /* Eq. ttt_indices: shape of C and of the contracted index space. */
    int64_t nc[ORA_MAXP], nq[ORA_MAXP];
    for (int k = 0; k < r; ++k) nc[k] = na[phi[k] - 1];
    for (int k = 0; k < s; ++k) nc[r + k] = nb[psi[k] - 1];
    for (int k = 0; k < q; ++k) {
        nq[k] = na[phi[r + k] - 1];
        if (nq[k] != nb[psi[s + k] - 1]) return -2;
    }
    const int64_t total = prod(r + s, nc);
    const int64_t kq = prod(q, nq);
#pragma omp parallel for schedule(static)
    for (int64_t lin = 0; lin < total; ++lin) {
        int64_t c[ORA_MAXP], ia[ORA_MAXP], ib[ORA_MAXP], j[ORA_MAXP];
        decode_first_order(lin, r + s, nc, c);
        for (int k = 0; k < r; ++k) ia[phi[k] - 1] = c[k];
        for (int k = 0; k < s; ++k) ib[psi[k] - 1] = c[r + k];
        double acc = 0.0;
        for (int64_t jl = 0; jl < kq; ++jl) {
            decode_first_order(jl, q, nq, j); /* j_1 fastest */
            for (int k = 0; k < q; ++k) {
                ia[phi[r + k] - 1] = j[k];
                ib[psi[s + k] - 1] = j[k];
            }
            acc += A[layout_fn(pa, wA, ia)] * B[layout_fn(pb, wB, ib)];
        }
        C[layout_fn(r + s, wC, c)] = acc;
    }
    return 0;
}

double ora_inner(int p, const int64_t* n, const double* A, const int64_t* wA,
                 const double* B, const int64_t* wB)
{
    /* Neumaier's improved Kahan summation, in first-order index order. */
    const int64_t total = prod(p, n);
    double sum = 0.0, comp = 0.0;
    int64_t i[ORA_MAXP];
    for (int64_t lin = 0; lin < total; ++lin) {
        decode_first_order(lin, p, n, i);
        const double x = A[layout_fn(p, wA, i)] * B[layout_fn(p, wB, i)];
        const double t = sum + x;
        if (fabs(sum) >= fabs(x)) comp += (sum - t) + x;
        else                      comp += (x - t) + sum;
        sum = t;
    }
    return sum + comp;
}

int ora_axpby(int p, const int64_t* n, double alpha, const double* A, const int64_t* wA,
              double beta, const double* B, const int64_t* wB,
              double* C, const int64_t* wC)
{
    if (p < 0 || p > ORA_MAXP) return -1;
    const int64_t total = prod(p, n);
#pragma omp parallel for schedule(static)
    for (int64_t lin = 0; lin < total; ++lin) {
        int64_t i[ORA_MAXP];
        decode_first_order(lin, p, n, i);
        double v = alpha * A[layout_fn(p, wA, i)];
        if (B) v += beta * B[layout_fn(p, wB, i)];
        C[layout_fn(p, wC, i)] = v;
    }
    return 0;
}

int ora_transpose(int p, const int64_t* n, const double* A, const int64_t* wA,
                  const int32_t* tau, double* C, const int64_t* wC)
{
    if (p < 1 || p > ORA_MAXP || !is_perm(p, tau)) return -1;
    int64_t nc[ORA_MAXP];
    for (int r = 0; r < p; ++r) nc[r] = n[tau[r] - 1];
    const int64_t total = prod(p, nc);
#pragma omp parallel for schedule(static)
    for (int64_t lin = 0; lin < total; ++lin) {
        int64_t ic[ORA_MAXP], ia[ORA_MAXP];
        decode_first_order(lin, p, nc, ic);
        for (int r = 0; r < p; ++r) ia[tau[r] - 1] = ic[r]; /* i^c_r = i^a_{tau_r} */
        C[layout_fn(p, wC, ic)] = A[layout_fn(p, wA, ia)];
    }
    return 0;
}
