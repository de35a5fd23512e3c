/*
 * Reference (oracle) implementation of sparse MTTKRP and of the sparse CP
 * least-squares loss, in plain sequential C with FP64 arithmetic.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code with the HIP path.
 *
 * Every loop below is the plain definition, one nonzero at a time, in input
 * order, with no blocking, sorting or reordering:
 *
 *   MTTKRP, mode d   (Eq. 1 of Sec. 2.1 written element-wise, accumulated as
 *                     in the elementwise computation "EC" of Sec. 3):
 *       Y[i, r] = sum over nonzeros k with i_d(k) = i of
 *                 val(k) * prod_{w != d} A_w[i_w(k), r]
 *       The output starts at zero and every row is written, so rows that no
 *       nonzero touches are 0.
 *
 *   CP model value at a nonzero (the rank-R CP model of Sec. 2.1):
 *       xhat(k) = sum_r prod_{w} A_w[i_w(k), r]
 *
 *   Sparse CP loss:  L = sum_k (val(k) - xhat(k))^2
 *
 * All inputs arrive as float64 (the callers upcast their float32 / bfloat16
 * data exactly).  Indices are int32 in the [order][nnz] layout.
 */
#include <stdint.h>
#include <string.h>

/* MTTKRP along `mode`; out is dims[mode] x R, row-major, overwritten. */
void oracle_mttkrp(int order, const int64_t *dims, int64_t nnz,
                   const int32_t *idx, const double *val, int mode, int R,
                   const double *const *A, double *out)
{
    memset(out, 0, (size_t)dims[mode] * (size_t)R * sizeof(double));
    for (int64_t k = 0; k < nnz; ++k) {
        const int64_t i = idx[(int64_t)mode * nnz + k];
        for (int r = 0; r < R; ++r) {
            double prod = val[k];
            for (int w = 0; w < order; ++w) {
                if (w == mode) continue;
                const int64_t iw = idx[(int64_t)w * nnz + k];
                prod *= A[w][iw * R + r];
            }
            out[i * R + r] += prod;
        }
    }
}

/* CP model value xhat(k) at every nonzero. */
void oracle_cp_model(int order, int64_t nnz, const int32_t *idx, int R,
                     const double *const *A, double *xhat)
{
    for (int64_t k = 0; k < nnz; ++k) {
        double s = 0.0;
        for (int r = 0; r < R; ++r) {
            double prod = 1.0;
            for (int w = 0; w < order; ++w) {
                const int64_t iw = idx[(int64_t)w * nnz + k];
                prod *= A[w][iw * R + r];
            }
            s += prod;
        }
        xhat[k] = s;
    }
}

/* L = sum_k (val(k) - xhat(k))^2, also returning the residuals e(k). */
double oracle_cp_loss(int order, int64_t nnz, const int32_t *idx,
                      const double *val, int R, const double *const *A,
                      double *resid)
{
    double loss = 0.0;
    oracle_cp_model(order, nnz, idx, R, A, resid);
    for (int64_t k = 0; k < nnz; ++k) {
        const double e = val[k] - resid[k];
        resid[k] = e;
        loss += e * e;
    }
    return loss;
}
