// Vector and transfer kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

namespace stmg {

template <typename T> hipError_t vec_axpby(long long n, T a, const T *x, T b, T *y, hipStream_t s);
template <typename T> hipError_t vec_fill(long long n, T v, T *y, hipStream_t s);
template <typename S, typename D> hipError_t vec_cast(long long n, const S *x, D *y, hipStream_t s);

// out[k] (+)= u . V_k for k < nk (V_k at V + k*ldv); partial: scratch of
// multidot_partial_words(nk) doubles
hipError_t vec_multidot(long long n, int nk, const double *u, const double *V, long long ldv, double *out,
                        double *partial, int accumulate, hipStream_t s);
size_t multidot_partial_words(int nk);
// w -= sum_k h[k] V_k
hipError_t vec_subtract_combination(long long n, int nk, const double *h, const double *V, long long ldv, double *w,
                                    hipStream_t s);
// x = sum_k y[k] Z_k
hipError_t vec_combination(long long n, int nk, const double *y, const double *Z, long long ldz, double *x,
                           hipStream_t s);

// y[ot][c][row] = sum_it Tm[ot][it] (CSR x[it][c][.])[row] + beta * y
template <typename T> struct KronCsrArgs {
    const int *rowptr;
    const int *col;
    const T *val;
    int nrows;
    int nt_out, nt_in, ncomp;
    const T *Tm;              // device, nt_out x nt_in
    long long in_t_stride, in_c_stride, out_t_stride, out_c_stride;
    const T *x;
    T *y;
    T beta;
};
template <typename T> hipError_t kron_csr_apply(const KronCsrArgs<T> &a, hipStream_t s);

} // namespace stmg
