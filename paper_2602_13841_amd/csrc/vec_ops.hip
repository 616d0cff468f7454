// Streaming vector kernels of the Krylov and multigrid layers (HBM bound).
//
// Reductions are deterministic: a fixed grid of blocks writes partial sums,
// one block sums them in a fixed order; results stay on the device.
#include "vec_ops.h"

namespace stmg {

namespace {

constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 512;

template <typename T> __global__ void axpby_kernel(long long n, T a, const T *__restrict__ x, T b, T *__restrict__ y)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) y[i] = a * x[i] + (b == T(0) ? T(0) : b * y[i]);
}

template <typename S, typename D> __global__ void cast_kernel(long long n, const S *__restrict__ x, D *__restrict__ y)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) y[i] = (D)x[i];
}

template <typename T> __global__ void fill_kernel(long long n, T v, T *__restrict__ y)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) y[i] = v;
}

// partial[k * RED_BLOCKS + block] = sum over this block's slice of u * V_k
__global__ void __launch_bounds__(RED_THREADS)
    multidot_partial(long long n, int nk, const double *__restrict__ u, const double *__restrict__ V,
                     long long ldv, double *__restrict__ partial)
{
    __shared__ double red[RED_THREADS];
    const int k = blockIdx.y;
    const double *v = V + (long long)k * ldv;
    double s = 0;
    for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < n; i += (long long)RED_BLOCKS * RED_THREADS)
        s += u[i] * v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[k * RED_BLOCKS + blockIdx.x] = red[0];
    (void)nk;
}

// out[k] = (accumulate ? out[k] : 0) + sum_b partial[k][b]
__global__ void __launch_bounds__(RED_THREADS)
    multidot_final(int nk, const double *__restrict__ partial, double *__restrict__ out, int accumulate)
{
    __shared__ double red[RED_THREADS];
    for (int k = 0; k < nk; ++k) {
        double s = 0;
        for (int b = threadIdx.x; b < RED_BLOCKS; b += RED_THREADS) s += partial[k * RED_BLOCKS + b];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = (accumulate ? out[k] : 0.0) + red[0];
        __syncthreads();
    }
}

// w -= sum_k h[k] V_k  and (if MV) u -= sum_k h[k] MV_k ; h on the device
__global__ void subtract_combination(long long n, int nk, const double *__restrict__ h, const double *__restrict__ V,
                                     long long ldv, double *__restrict__ w)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        double s = w[i];
        for (int k = 0; k < nk; ++k) s -= h[k] * V[(long long)k * ldv + i];
        w[i] = s;
    }
}

// x = sum_k y[k] Z_k (y on the device)
__global__ void combination(long long n, int nk, const double *__restrict__ y, const double *__restrict__ Z, long long ldz,
                            double *__restrict__ x)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        double s = 0;
        for (int k = 0; k < nk; ++k) s += y[k] * Z[(long long)k * ldz + i];
        x[i] = s;
    }
}

// y[ot][c][row] (+)= sum_it Tm[ot][it] sum_{k in row} val[k] x[it][c][col[k]]:
// LPR lanes per row read the row's entries once for every component and input
// time node (at most 3 and 4), lane j the entries k0 + j, k0 + j + LPR, ...;
// per output the lane sums run over their k in order and are added by a fixed
// xor tree, then the time coefficients in order, skipping zero ones
template <typename T, int LPR>
__global__ void __launch_bounds__(256) kron_csr_kernel(KronCsrArgs<T> A)
{
    constexpr int MC = 3, MT = 4;
    static_assert(LPR >= 1 && LPR <= 64 && (LPR & (LPR - 1)) == 0, "lanes per row: a power of two up to 64");
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int row = (int)(g / LPR), sub = (int)(g % LPR);
    if (row >= A.nrows) return;   // whole groups of LPR lanes
    const int k0 = A.rowptr[row], k1 = A.rowptr[row + 1];
    const int nti = A.nt_in, nc = A.ncomp;
    T sum[MC][MT];
#pragma unroll
    for (int c = 0; c < MC; ++c)
#pragma unroll
        for (int it = 0; it < MT; ++it) sum[c][it] = T(0);
    for (int k = k0 + sub; k < k1; k += LPR) {
        const T v = A.val[k];
        const long long cl = A.col[k];
#pragma unroll
        for (int c = 0; c < MC; ++c)
#pragma unroll
            for (int it = 0; it < MT; ++it)
                if (c < nc && it < nti) sum[c][it] += v * A.x[it * A.in_t_stride + c * A.in_c_stride + cl];
    }
    if constexpr (LPR > 1) {
#pragma unroll
        for (int off = LPR / 2; off > 0; off >>= 1)
#pragma unroll
            for (int c = 0; c < MC; ++c)
#pragma unroll
                for (int it = 0; it < MT; ++it) sum[c][it] += __shfl_xor(sum[c][it], off, 64);
        if (sub != 0) return;
    }
#pragma unroll
    for (int ot = 0; ot < MT; ++ot)
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            if (ot >= A.nt_out || c >= nc) continue;
            T acc = 0;
#pragma unroll
            for (int it = 0; it < MT; ++it) {
                if (it >= nti) continue;
                const T tm = A.Tm[ot * nti + it];
                if (tm == T(0)) continue;
                acc += tm * sum[c][it];
            }
            T *yp = A.y + ot * A.out_t_stride + c * A.out_c_stride + row;
            *yp = A.beta == T(0) ? acc : acc + A.beta * *yp;
        }
}

// one thread: the rotations of a column depend on each other in order, and a
// column has at most maxit + 1 entries
__global__ void givens_column_kernel(int j, int maxit, const double *__restrict__ h1, const double *__restrict__ h2,
                                     const double *__restrict__ hn, double *__restrict__ H, double *__restrict__ cs,
                                     double *__restrict__ sn, double *__restrict__ g, double *__restrict__ report)
{
    if (threadIdx.x != 0) return;
    double *col = H + (long long)j * (maxit + 1);
    for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
    const double sub = sqrt(fmax(hn[0], 0.0));
    col[j + 1] = sub;
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double den = hypot(a, b);
    const double c = den > 0.0 ? a / den : 1.0, sv = den > 0.0 ? b / den : 0.0;
    cs[j] = c;
    sn[j] = sv;
    col[j] = c * a + sv * b;
    col[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sv * gj;
    g[j] = c * gj;
    report[0] = fabs(g[j + 1]);
    report[1] = sub;
}

__global__ void upper_solve_kernel(int its, int maxit, const double *__restrict__ H, const double *__restrict__ g,
                                   double *__restrict__ y)
{
    if (threadIdx.x != 0) return;
    const long long ld = maxit + 1;
    for (int i = its - 1; i >= 0; --i) {
        double t = g[i];
        for (int k = i + 1; k < its; ++k) t -= H[k * ld + i] * y[k];
        y[i] = t / H[i * ld + i];
    }
}

inline int grid_for(long long n, int th = 256)
{
    long long b = (n + th - 1) / th;
    if (b > 65535LL * 16) b = 65535LL * 16;
    return (int)(b < 1 ? 1 : b);
}

} // namespace

template <typename T> hipError_t vec_axpby(long long n, T a, const T *x, T b, T *y, hipStream_t s)
{
    hipLaunchKernelGGL(axpby_kernel<T>, dim3(grid_for(n)), dim3(256), 0, s, n, a, x, b, y);
    return hipGetLastError();
}

template <typename T> hipError_t vec_fill(long long n, T v, T *y, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel<T>, dim3(grid_for(n)), dim3(256), 0, s, n, v, y);
    return hipGetLastError();
}

template <typename S, typename D> hipError_t vec_cast(long long n, const S *x, D *y, hipStream_t s)
{
    hipLaunchKernelGGL((cast_kernel<S, D>), dim3(grid_for(n)), dim3(256), 0, s, n, x, y);
    return hipGetLastError();
}

hipError_t vec_multidot(long long n, int nk, const double *u, const double *V, long long ldv, double *out,
                        double *partial, int accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(multidot_partial, dim3(RED_BLOCKS, nk), dim3(RED_THREADS), 0, s, n, nk, u, V, ldv, partial);
    hipLaunchKernelGGL(multidot_final, dim3(1), dim3(RED_THREADS), 0, s, nk, partial, out, accumulate);
    return hipGetLastError();
}

size_t multidot_partial_words(int nk) { return (size_t)nk * RED_BLOCKS; }

hipError_t vec_subtract_combination(long long n, int nk, const double *h, const double *V, long long ldv, double *w,
                                    hipStream_t s)
{
    hipLaunchKernelGGL(subtract_combination, dim3(grid_for(n)), dim3(256), 0, s, n, nk, h, V, ldv, w);
    return hipGetLastError();
}

hipError_t vec_combination(long long n, int nk, const double *y, const double *Z, long long ldz, double *x,
                           hipStream_t s)
{
    hipLaunchKernelGGL(combination, dim3(grid_for(n)), dim3(256), 0, s, n, nk, y, Z, ldz, x);
    return hipGetLastError();
}

hipError_t krylov_givens_column(int j, int maxit, const double *h1, const double *h2, const double *hn, double *H,
                                double *cs, double *sn, double *g, double *report, hipStream_t s)
{
    hipLaunchKernelGGL(givens_column_kernel, dim3(1), dim3(64), 0, s, j, maxit, h1, h2, hn, H, cs, sn, g, report);
    return hipGetLastError();
}

hipError_t krylov_upper_solve(int its, int maxit, const double *H, const double *g, double *y, hipStream_t s)
{
    hipLaunchKernelGGL(upper_solve_kernel, dim3(1), dim3(64), 0, s, its, maxit, H, g, y);
    return hipGetLastError();
}

template <typename T> hipError_t kron_csr_apply(const KronCsrArgs<T> &a, hipStream_t s)
{
    if (a.ncomp < 1 || a.ncomp > 3 || a.nt_in < 1 || a.nt_in > 4 || a.nt_out < 1 || a.nt_out > 4 || a.nrows < 0)
        return hipErrorInvalidValue;
    if (a.nrows == 0) return hipSuccess;
    const int th = 256;
    const long long n1 = a.nrows;
    switch (a.lpr) {
    case 0:
    case 1: hipLaunchKernelGGL((kron_csr_kernel<T, 1>), dim3((unsigned)((n1 + th - 1) / th)), dim3(th), 0, s, a); break;
    case 4: hipLaunchKernelGGL((kron_csr_kernel<T, 4>), dim3((unsigned)((4 * n1 + th - 1) / th)), dim3(th), 0, s, a); break;
    case 16: hipLaunchKernelGGL((kron_csr_kernel<T, 16>), dim3((unsigned)((16 * n1 + th - 1) / th)), dim3(th), 0, s, a); break;
    case 64: hipLaunchKernelGGL((kron_csr_kernel<T, 64>), dim3((unsigned)((64 * n1 + th - 1) / th)), dim3(th), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t vec_axpby<double>(long long, double, const double *, double, double *, hipStream_t);
template hipError_t vec_axpby<float>(long long, float, const float *, float, float *, hipStream_t);
template hipError_t vec_fill<double>(long long, double, double *, hipStream_t);
template hipError_t vec_fill<float>(long long, float, float *, hipStream_t);
template hipError_t vec_cast<double, float>(long long, const double *, float *, hipStream_t);
template hipError_t vec_cast<float, double>(long long, const float *, double *, hipStream_t);
template hipError_t vec_cast<double, double>(long long, const double *, double *, hipStream_t);
template hipError_t kron_csr_apply<double>(const KronCsrArgs<double> &, hipStream_t);
template hipError_t kron_csr_apply<float>(const KronCsrArgs<float> &, hipStream_t);

} // namespace stmg
