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

// FGMRES least-squares bookkeeping in FP64 on the device (Givens form of the
// Hessenberg system).  H: (maxit+1) x maxit column-major; cs, sn: maxit;
// g: maxit+1.  Column j of H is h1[i] + h2[i] (the two Gram-Schmidt passes,
// i <= j) with sqrt(max(hn, 0)) below the diagonal; the previous rotations
// are applied to it, the rotation eliminating its subdiagonal entry is
// formed and applied to g.  report[0] = |g[j+1]| (the residual estimate),
// report[1] = the subdiagonal entry before rotation.
hipError_t krylov_givens_column(int j, int maxit, const double *h1, const double *h2, const double *hn, double *H,
                                double *cs, double *sn, double *g, double *report, hipStream_t s);
// y = H(0:its, 0:its)^{-1} g(0:its) (upper triangular, column-major ld maxit+1)
hipError_t krylov_upper_solve(int its, int maxit, const double *H, const double *g, double *y, hipStream_t s);

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
    int lpr;                  // lanes per row (1, 4, 16 or 64; 0 = 1), see kron_lanes
};
// lanes per CSR row for a matrix with nnz entries in nrows rows: long rows
// (restrictions gather hundreds of fine values) are read by a group of
// lanes, consecutive entries by consecutive lanes
inline int kron_lanes(long long nnz, long long nrows)
{
    const long long avg = nrows > 0 ? nnz / nrows : 0;
    return avg < 6 ? 1 : avg < 24 ? 4 : avg < 96 ? 16 : 64;
}
template <typename T> hipError_t kron_csr_apply(const KronCsrArgs<T> &a, hipStream_t s);

} // namespace stmg
