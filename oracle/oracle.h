/*
 * Plain FP64 CPU oracle for the tensor-contraction hot path of
 * Bassoy, "TLib: A Flexible C++ Tensor Framework for Numerical Tensor
 * Calculus" (arXiv 1711.10912).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * includes this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark call it.  It shares no code with the HIP path.
 *
 * Every tensor is given as (base pointer, order p, extents n[p], strides w[p])
 * with element strides.  The element with zero-based multi-index i lives at
 * base[ sum_r w_r * i_r ]  (layout function, Sec. 3.2 Eq. f with zero index
 * offsets; for a view the base already includes gamma and w = parent stride
 * times step, Sec. 3.3 Eq. view_gamma / lambda_view, Sec. 5.1 Eq. final_address).
 *
 * Modes are 1-based as in the paper's equations (Sec. 5.2).
 * All functions return 0 on success and a negative value on a shape/mode error.
 */
#ifndef TLIB_ORACLE_H
#define TLIB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sec. 3.1 Eq. stride.tuple.permutation: w[pi_1] = 1, w[pi_r] = prod_{q<r} n[pi_q].
 * pi is 1-based.  Returns -1 if pi is not a permutation of 1..p. */
int ora_strides(int p, const int64_t* n, const int32_t* pi, int64_t* w);

/* Sec. 5.2 Eq. ttv: C(i without i_m) = sum_{i_m} A(i) * b(i_m).  C has order p-1. */
int ora_ttv(int p, const int64_t* n, const double* A, const int64_t* wA,
            const double* b, int64_t wb, int m,
            double* C, const int64_t* wC);

/* Sec. 5.2 Eq. ttm: C(i_1..j..i_p) = sum_{i_m} A(i) * B(j, i_m); B has shape (nb0, n_m). */
int ora_ttm(int p, const int64_t* n, const double* A, const int64_t* wA,
            int64_t nb0, const double* B, const int64_t* wB, int m,
            double* C, const int64_t* wC);

/* Sec. 5.2 Eq. ttt + ttt_indices: A has order q+r, B order q+s, C order r+s.
 * phi (length q+r) and psi (length q+s) are 1-based permutations. */
int ora_ttt(int pa, const int64_t* na, const double* A, const int64_t* wA,
            int pb, const int64_t* nb, const double* B, const int64_t* wB,
            int q, const int32_t* phi, const int32_t* psi,
            double* C, const int64_t* wC);

/* Sec. 5.2 Table 3 inner_product: sum_i A(i) B(i) over the common multi-index
 * set, visited in first-order index order, Neumaier-compensated. */
double ora_inner(int p, const int64_t* n, const double* A, const int64_t* wA,
                 const double* B, const int64_t* wB);

/* Sec. 5.1 Eq. transform / Eq. scaling: C(i) = alpha A(i) + beta B(i).
 * B may be NULL (then beta is ignored and C = alpha A). */
int ora_axpby(int p, const int64_t* n, double alpha, const double* A, const int64_t* wA,
              double beta, const double* B, const int64_t* wB,
              double* C, const int64_t* wC);

/* Sec. 5.2 Table 3 transpose: C(i^c) = A(i^a) with i^c_r = i^a_{tau_r}, n^c_r = n^a_{tau_r}.
 * tau is 1-based; n and wA describe A, wC the strides of C (indexed by C's modes). */
int ora_transpose(int p, const int64_t* n, const double* A, const int64_t* wA,
                  const int32_t* tau, double* C, const int64_t* wC);

#ifdef __cplusplus
}
#endif
#endif
