// Matrix-free cell kernels of one space-time slab on gfx950.
//
// One workgroup handles one spatial cell and all k+1 time nodes of the slab
// (the Kronecker evaluation of Sec. "Matrix-free operator evaluation": the
// spatial operator once per temporal node, then the small dense time
// mixing).  Per cell and time node:
//
//   1. coalesced gather of the nodal values (velocity, pressure modes, state)
//      into LDS,
//   2. sum-factorized 1D sweeps to the Gauss points (values), collocation
//      derivatives at the Gauss points for gradients,
//   3. the quadrature-point physics (register staged, in place in LDS),
//   4. transposed collocation + transposed sweeps back to the nodes,
//   5. for cells on the domain boundary: the Nitsche / convective boundary
//      terms of eq. def-a-gam-tp and eq. def-b-gam, with face sweeps,
//   6. velocity results go to a cell-local buffer E (no atomics); a second
//      kernel sums E over the cells sharing each node in a fixed order, so
//      results are bitwise reproducible.
//
// Modes:
//   Jac  : y = J_n(U) x  (eq. JacobianLocal; convective part eq. Defcp)
//   Res  : y = R_n(U; V_{n-1}) (eq. InAlgNS), rhs and V_{n-1} optional
//   Mass : y = blockdiag(M^tau (x) M_h, M^tau (x) M_h^p) x (weight of the
//          M-norm of eq. inexact)
#include "stmg_internal.h"

#include <cstdlib>
#include <mutex>
#include <type_traits>

namespace stmg {

namespace {

template <int DIM, int R> struct Sizes {
    static constexpr int N1 = R + 2;
    static constexpr int NL = DIM == 2 ? N1 * N1 : N1 * N1 * N1;
    static constexpr int RP1 = R + 1;
    static constexpr int NPF = DIM == 2 ? RP1 * RP1 : RP1 * RP1 * RP1;   // full tensor of modes
    static constexpr int NPM = DIM == 2 ? (R + 1) * (R + 2) / 2 : (R + 1) * (R + 2) * (R + 3) / 6;
};

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// ---------------------------------------------------------------------------
// Tensor sweep: out[f][o2][o1][o0] (+)= sum A2[o2][i2] A1[o1][i1] A0[o0][i0]
// in[f][i2][i1][i0], NF fields, input/output field strides is/os.  Matrices
// are row-major O x I.  All threads of the block cooperate; ends with a
// barrier.  In 2D the third axis is absent.
// ---------------------------------------------------------------------------
template <int DIM, int NF, int I0, int I1, int I2, int O0, int O1, int O2, bool ACC, typename T>
__device__ __forceinline__ void sweep(const T *__restrict__ in, int is, T *__restrict__ out, int os,
                                      T *__restrict__ t1, T *__restrict__ t2, const T *A0,
                                      const T *A1, const T *A2)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    if constexpr (DIM == 2) {
        constexpr int n1 = I1 * O0;
        for (int e = tid; e < NF * n1; e += nth) {
            int f = e / n1, rr = e - f * n1, o0 = rr % O0, i1 = rr / O0;
            const T *src = in + f * is + i1 * I0;
            const T *a = A0 + o0 * I0;
            T s = 0;
#pragma unroll
            for (int i = 0; i < I0; ++i) s += a[i] * src[i];
            t1[e] = s;
        }
        __syncthreads();
        constexpr int n2 = O1 * O0;
        for (int e = tid; e < NF * n2; e += nth) {
            int f = e / n2, rr = e - f * n2, o0 = rr % O0, o1 = rr / O0;
            const T *src = t1 + f * n1 + o0;
            const T *a = A1 + o1 * I1;
            T s = 0;
#pragma unroll
            for (int i = 0; i < I1; ++i) s += a[i] * src[i * O0];
            if constexpr (ACC) out[f * os + rr] += s;
            else out[f * os + rr] = s;
        }
        __syncthreads();
    } else {
        constexpr int n1 = I2 * I1 * O0;
        for (int e = tid; e < NF * n1; e += nth) {
            int f = e / n1, rr = e - f * n1, o0 = rr % O0, i21 = rr / O0;
            const T *src = in + f * is + i21 * I0;
            const T *a = A0 + o0 * I0;
            T s = 0;
#pragma unroll
            for (int i = 0; i < I0; ++i) s += a[i] * src[i];
            t1[e] = s;
        }
        __syncthreads();
        constexpr int n2 = I2 * O1 * O0;
        for (int e = tid; e < NF * n2; e += nth) {
            int f = e / n2, rr = e - f * n2, o0 = rr % O0, o1 = (rr / O0) % O1, i2 = rr / (O0 * O1);
            const T *src = t1 + f * n1 + i2 * I1 * O0 + o0;
            const T *a = A1 + o1 * I1;
            T s = 0;
#pragma unroll
            for (int i = 0; i < I1; ++i) s += a[i] * src[i * O0];
            t2[e] = s;
        }
        __syncthreads();
        constexpr int n3 = O2 * O1 * O0;
        for (int e = tid; e < NF * n3; e += nth) {
            int f = e / n3, rr = e - f * n3, o01 = rr % (O0 * O1), o2 = rr / (O0 * O1);
            const T *src = t2 + f * n2 + o01;
            const T *a = A2 + o2 * I2;
            T s = 0;
#pragma unroll
            for (int i = 0; i < I2; ++i) s += a[i] * src[i * O0 * O1];
            if constexpr (ACC) out[f * os + rr] += s;
            else out[f * os + rr] = s;
        }
        __syncthreads();
    }
}

// multilinear map: Jacobian J[a][b] = dx_a/dxi_b at xi; vertices X[v*3+a]
template <int DIM, typename T>
__device__ __forceinline__ void map_jac(const T *X, const T xi[3], T J[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) J[a][b] = 0;
#pragma unroll
    for (int v = 0; v < (1 << DIM); ++v) {
        T f[3], df[3];
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            int o = (v >> b) & 1;
            f[b] = o ? xi[b] : T(1) - xi[b];
            df[b] = o ? T(1) : T(-1);
        }
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            T g = df[b];
#pragma unroll
            for (int e = 0; e < DIM; ++e)
                if (e != b) g *= f[e];
#pragma unroll
            for (int a = 0; a < DIM; ++a) J[a][b] += X[v * 3 + a] * g;
        }
    }
}

// det J and Jit = J^{-T}
template <int DIM, typename T>
__device__ __forceinline__ T inv_t(const T J[3][3], T Jit[3][3])
{
    if constexpr (DIM == 2) {
        T det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        T id = T(1) / det;
        Jit[0][0] = J[1][1] * id;
        Jit[0][1] = -J[1][0] * id;
        Jit[1][0] = -J[0][1] * id;
        Jit[1][1] = J[0][0] * id;
        return det;
    } else {
        T c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        T c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        T c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        T det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        T id = T(1) / det;
        Jit[0][0] = c00 * id;
        Jit[0][1] = c01 * id;
        Jit[0][2] = c02 * id;
        Jit[1][0] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
        Jit[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
        Jit[1][2] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
        Jit[2][0] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
        Jit[2][1] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
        Jit[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
        return det;
    }
}

template <typename T> __device__ __forceinline__ T ominus(T y) { return T(0.5) * (fabs(y) - y); }
template <typename T> __device__ __forceinline__ T dominus(T y)
{
    return y > T(0) ? T(0) : (y < T(0) ? T(-1) : T(-0.5));
}

// ---------------------------------------------------------------------------
// Register-pencil tensor contractions of the volume pass.  A stage treats all
// fields of two groups at once (group A: NFA fields, nodal extent IA, 1D
// matrices of group A; group B: NFB fields, IB); a work item is one pencil
// along the contracted axis: its I inputs go to registers and its NQ outputs
// are written back (I + NQ LDS accesses per item).  Layouts are x fastest;
// every stage ends with a barrier.  Matrices are NQ x I row-major.
// ---------------------------------------------------------------------------
template <int DIM, int NQ, int NFA, int IA, int NFB, int IB> struct PencilSizes {
    // rows along x of the buffer feeding the x contraction are padded to an
    // odd length (conflict-free strided row reads)
    static constexpr int RA = IA | 1, RB = IB | 1;
    static constexpr int B1A = DIM == 3 ? NQ * IA * IA : NQ * RA;    // after the first contraction
    static constexpr int B1B = DIM == 3 ? NQ * IB * IB : NQ * RB;
    static constexpr int B2A = DIM == 3 ? NQ * NQ * RA : 0;          // after the second (3D)
    static constexpr int B2B = DIM == 3 ? NQ * NQ * RB : 0;
    static constexpr int BUF1 = NFA * B1A + NFB * B1B;
    static constexpr int BUF2 = (NFA * B2A + NFB * B2B) > 1 ? NFA * B2A + NFB * B2B : 1;
};

// contract one pencil: out[o * os] = sum_i M[o * I + i] in[i * is], o < NQ
template <int I, int NQ, typename T, typename MP>
__device__ __forceinline__ void pencil_apply(const T *__restrict__ in, int is, T *__restrict__ out, int os, MP M)
{
    T u[I];
#pragma unroll
    for (int i = 0; i < I; ++i) u[i] = in[i * is];
#pragma unroll
    for (int o = 0; o < NQ; ++o) {
        T s = 0;
#pragma unroll
        for (int i = 0; i < I; ++i) s += M[o * I + i] * u[i];
        out[o * os] = s;
    }
}

// transposed: out[i * os] = sum_o M[o * I + i] in[o * is], i < I
template <int I, int NQ, typename T, typename MP>
__device__ __forceinline__ void pencil_apply_t(const T *__restrict__ in, int is, T *__restrict__ out, int os, MP M)
{
    T u[NQ];
#pragma unroll
    for (int o = 0; o < NQ; ++o) u[o] = in[o * is];
#pragma unroll
    for (int i = 0; i < I; ++i) {
        T s = 0;
#pragma unroll
        for (int o = 0; o < NQ; ++o) s += M[o * I + i] * u[o];
        out[i * os] = s;
    }
}

// nodes -> Gauss points.  inA [NFA][IA^DIM], inB [NFB][IB^DIM]; field f of
// group A to QA + f * NQ^DIM, of group B to QB + f * NQ^DIM.  For the first
// NGRAD fields of group A also the reference derivative along x (nodal
// derivative table DA, NQ x IA) to GX + f * DIM * NQ^DIM.
template <int DIM, int NQ, int NFA, int IA, int NFB, int IB, int NGRAD, int NTH, typename T, typename MP>
__device__ __forceinline__ void pencil_fwd(const T *__restrict__ inA, const T *__restrict__ inB, T *__restrict__ QA,
                                           T *__restrict__ QB, T *__restrict__ GX, T *__restrict__ buf1,
                                           T *__restrict__ buf2, MP MA, MP DA, MP MB)
{
    using PS = PencilSizes<DIM, NQ, NFA, IA, NFB, IB>;
    constexpr int NQV = DIM == 3 ? NQ * NQ * NQ : NQ * NQ;
    const int tid = threadIdx.x;
    if constexpr (DIM == 3) {
        // z: item (f, j, i)
        constexpr int NA = NFA * IA * IA, NB = NFB * IB * IB;
        for (int w = tid; w < NA + NB; w += NTH) {
            if (w < NA) {
                const int f = w / (IA * IA), ji = w - f * IA * IA;
                pencil_apply<IA, NQ>(inA + f * IA * IA * IA + ji, IA * IA, buf1 + f * PS::B1A + ji, IA * IA, MA);
            } else {
                const int ww = w - NA, f = ww / (IB * IB), ji = ww - f * IB * IB;
                pencil_apply<IB, NQ>(inB + f * IB * IB * IB + ji, IB * IB, buf1 + NFA * PS::B1A + f * PS::B1B + ji,
                                     IB * IB, MB);
            }
        }
        __syncthreads();
        // y: item (f, qz, i)
        constexpr int NA2 = NFA * NQ * IA, NB2 = NFB * NQ * IB;
        for (int w = tid; w < NA2 + NB2; w += NTH) {
            if (w < NA2) {
                const int f = w / (NQ * IA), rr = w - f * NQ * IA, qz = rr / IA, i = rr - qz * IA;
                pencil_apply<IA, NQ>(buf1 + f * PS::B1A + qz * IA * IA + i, IA,
                                     buf2 + f * PS::B2A + qz * NQ * PS::RA + i, PS::RA, MA);
            } else {
                const int ww = w - NA2, f = ww / (NQ * IB), rr = ww - f * NQ * IB, qz = rr / IB, i = rr - qz * IB;
                pencil_apply<IB, NQ>(buf1 + NFA * PS::B1A + f * PS::B1B + qz * IB * IB + i, IB,
                                     buf2 + NFA * PS::B2A + f * PS::B2B + qz * NQ * PS::RB + i, PS::RB, MB);
            }
        }
        __syncthreads();
        // x: item (f, qz, qy)
        constexpr int NA3 = NFA * NQ * NQ, NB3 = NFB * NQ * NQ;
        for (int w = tid; w < NA3 + NB3; w += NTH) {
            if (w < NA3) {
                const int f = w / (NQ * NQ), rr = w - f * NQ * NQ;
                const T *src = buf2 + f * PS::B2A + rr * PS::RA;
                pencil_apply<IA, NQ>(src, 1, QA + f * NQV + rr * NQ, 1, MA);
                if (f < NGRAD) pencil_apply<IA, NQ>(src, 1, GX + f * DIM * NQV + rr * NQ, 1, DA);
            } else {
                const int ww = w - NA3, f = ww / (NQ * NQ), rr = ww - f * NQ * NQ;
                pencil_apply<IB, NQ>(buf2 + NFA * PS::B2A + f * PS::B2B + rr * PS::RB, 1, QB + f * NQV + rr * NQ, 1,
                                     MB);
            }
        }
        __syncthreads();
    } else {
        // y: item (f, i)
        constexpr int NA = NFA * IA, NB = NFB * IB;
        for (int w = tid; w < NA + NB; w += NTH) {
            if (w < NA) {
                const int f = w / IA, i = w - f * IA;
                pencil_apply<IA, NQ>(inA + f * IA * IA + i, IA, buf1 + f * PS::B1A + i, PS::RA, MA);
            } else {
                const int ww = w - NA, f = ww / IB, i = ww - f * IB;
                pencil_apply<IB, NQ>(inB + f * IB * IB + i, IB, buf1 + NFA * PS::B1A + f * PS::B1B + i, PS::RB, MB);
            }
        }
        __syncthreads();
        // x: item (f, qy)
        constexpr int NA2 = NFA * NQ, NB2 = NFB * NQ;
        for (int w = tid; w < NA2 + NB2; w += NTH) {
            if (w < NA2) {
                const int f = w / NQ, qy = w - f * NQ;
                const T *src = buf1 + f * PS::B1A + qy * PS::RA;
                pencil_apply<IA, NQ>(src, 1, QA + f * NQV + qy * NQ, 1, MA);
                if (f < NGRAD) pencil_apply<IA, NQ>(src, 1, GX + f * DIM * NQV + qy * NQ, 1, DA);
            } else {
                const int ww = w - NA2, f = ww / NQ, qy = ww - f * NQ;
                pencil_apply<IB, NQ>(buf1 + NFA * PS::B1A + f * PS::B1B + qy * PS::RB, 1, QB + f * NQV + qy * NQ, 1,
                                     MB);
            }
        }
        __syncthreads();
    }
}

// reference derivatives along y (and z) of NF fields at the Gauss points by
// collocation (Dq, NQ x NQ): field f at U + f * NQ^DIM, derivative along axis
// d (1 <= d < DIM) to G + (f * DIM + d) * NQ^DIM
template <int DIM, int NQ, int NF, int NTH, typename T, typename MP>
__device__ __forceinline__ void colloc_fwd(const T *__restrict__ U, T *__restrict__ G, MP Dq)
{
    constexpr int NQV = DIM == 3 ? NQ * NQ * NQ : NQ * NQ;
    constexpr int NP = DIM == 3 ? NQ * NQ : NQ;      // pencils per field and axis
    const int tid = threadIdx.x;
    for (int w = tid; w < NF * (DIM - 1) * NP; w += NTH) {
        const int f = w / ((DIM - 1) * NP), rr = w - f * (DIM - 1) * NP, d = 1 + rr / NP, p = rr - (d - 1) * NP;
        int base, st;
        if (d == 1) {                 // pencil along y through (qz, qx), p = qz * NQ + qx
            const int qz = DIM == 3 ? p / NQ : 0, qxx = DIM == 3 ? p - qz * NQ : p;
            base = qz * NQ * NQ + qxx;
            st = NQ;
        } else {                      // pencil along z through (qy, qx), p = qy * NQ + qx
            base = p;
            st = NQ * NQ;
        }
        pencil_apply<NQ, NQ>(U + f * NQV + base, st, G + (f * DIM + d) * NQV + base, st, Dq);
    }
    __syncthreads();
}

// transposed collocation of the test-function gradients along z and y, in
// place: Y_c += Dq_d^T F[c][d] for d = DIM-1 .. 1 (F at F0 + (c * DIM + d) *
// NQ^DIM, Y_c at Y0 + c * NQ^DIM); the x part is applied by pencil_bwd with
// the nodal derivative table
template <int DIM, int NQ, int NTH, typename T, typename MP>
__device__ __forceinline__ void colloc_bwd(const T *__restrict__ F0, T *__restrict__ Y0, MP Dq)
{
    constexpr int NQV = DIM == 3 ? NQ * NQ * NQ : NQ * NQ;
    constexpr int NP = DIM == 3 ? NQ * NQ : NQ;
    const int tid = threadIdx.x;
#pragma unroll 1
    for (int d = DIM - 1; d >= 1; --d) {
        for (int w = tid; w < DIM * NP; w += NTH) {
            const int c = w / NP, p = w - c * NP;
            int base, st;
            if (d == 1) {
                const int qz = DIM == 3 ? p / NQ : 0, qxx = DIM == 3 ? p - qz * NQ : p;
                base = qz * NQ * NQ + qxx;
                st = NQ;
            } else {
                base = p;
                st = NQ * NQ;
            }
            const T *f = F0 + (c * DIM + d) * NQV + base;
            T *y = Y0 + c * NQV + base;
            T u[NQ];
#pragma unroll
            for (int m = 0; m < NQ; ++m) u[m] = f[m * st];
#pragma unroll
            for (int o = 0; o < NQ; ++o) {
                T s = y[o * st];
#pragma unroll
                for (int m = 0; m < NQ; ++m) s += Dq[m * NQ + o] * u[m];
                y[o * st] = s;
            }
        }
        __syncthreads();
    }
}

// Gauss points -> nodes (transposed interpolation) of group A (NFA fields at
// QA + f * NQ^DIM, with the x part of the test gradient: FX + f * NQ^DIM
// contracted with the transposed nodal derivative table DA when NXG > 0) and
// group B; results to outA [NFA][IA^DIM], outB [NFB][IB^DIM]
template <int DIM, int NQ, int NFA, int IA, int NFB, int IB, bool XGRAD, int NTH, typename T, typename MP>
__device__ __forceinline__ void pencil_bwd(const T *__restrict__ QA, const T *__restrict__ FX, int fx_stride,
                                           const T *__restrict__ QB, T *__restrict__ outA, T *__restrict__ outB,
                                           T *__restrict__ buf1, T *__restrict__ buf2, MP MA, MP DA, MP MB)
{
    using PS = PencilSizes<DIM, NQ, NFA, IA, NFB, IB>;
    constexpr int NQV = DIM == 3 ? NQ * NQ * NQ : NQ * NQ;
    const int tid = threadIdx.x;
    // x: item (f, row) with the row over qx; rows = NQ^(DIM-1)
    constexpr int NR = DIM == 3 ? NQ * NQ : NQ;
    constexpr int NA = NFA * NR, NB = NFB * NR;
    T *dstA = DIM == 3 ? buf2 : buf1;
    constexpr int SA = DIM == 3 ? PS::B2A : PS::B1A, SB = DIM == 3 ? PS::B2B : PS::B1B;
    for (int w = tid; w < NA + NB; w += NTH) {
        if (w < NA) {
            const int f = w / NR, rr = w - f * NR;
            const T *y = QA + f * NQV + rr * NQ;
            T u[NQ], g[NQ];
#pragma unroll
            for (int o = 0; o < NQ; ++o) u[o] = y[o];
            if constexpr (XGRAD) {
                const T *fx = FX + f * fx_stride + rr * NQ;
#pragma unroll
                for (int o = 0; o < NQ; ++o) g[o] = fx[o];
            }
            T *out = dstA + f * SA + rr * PS::RA;
#pragma unroll
            for (int i = 0; i < IA; ++i) {
                T s = 0;
#pragma unroll
                for (int o = 0; o < NQ; ++o) {
                    s += MA[o * IA + i] * u[o];
                    if constexpr (XGRAD) s += DA[o * IA + i] * g[o];
                }
                out[i] = s;
            }
        } else {
            const int ww = w - NA, f = ww / NR, rr = ww - f * NR;
            pencil_apply_t<IB, NQ>(QB + f * NQV + rr * NQ, 1, dstA + NFA * SA + f * SB + rr * PS::RB, 1, MB);
        }
    }
    __syncthreads();
    if constexpr (DIM == 3) {
        // y: item (f, qz, i), buf2 [f][qz][qy][i] -> buf1 [f][qz][j][i]
        constexpr int NA2 = NFA * NQ * IA, NB2 = NFB * NQ * IB;
        for (int w = tid; w < NA2 + NB2; w += NTH) {
            if (w < NA2) {
                const int f = w / (NQ * IA), rr = w - f * NQ * IA, qz = rr / IA, i = rr - qz * IA;
                pencil_apply_t<IA, NQ>(buf2 + f * PS::B2A + qz * NQ * PS::RA + i, PS::RA,
                                       buf1 + f * PS::B1A + qz * IA * IA + i, IA, MA);
            } else {
                const int ww = w - NA2, f = ww / (NQ * IB), rr = ww - f * NQ * IB, qz = rr / IB, i = rr - qz * IB;
                pencil_apply_t<IB, NQ>(buf2 + NFA * PS::B2A + f * PS::B2B + qz * NQ * PS::RB + i, PS::RB,
                                       buf1 + NFA * PS::B1A + f * PS::B1B + qz * IB * IB + i, IB, MB);
            }
        }
        __syncthreads();
        // z: item (f, j, i), buf1 [f][qz][j][i] -> out [f][k][j][i]
        constexpr int NA3 = NFA * IA * IA, NB3 = NFB * IB * IB;
        for (int w = tid; w < NA3 + NB3; w += NTH) {
            if (w < NA3) {
                const int f = w / (IA * IA), ji = w - f * IA * IA;
                pencil_apply_t<IA, NQ>(buf1 + f * PS::B1A + ji, IA * IA, outA + f * IA * IA * IA + ji, IA * IA, MA);
            } else {
                const int ww = w - NA3, f = ww / (IB * IB), ji = ww - f * IB * IB;
                pencil_apply_t<IB, NQ>(buf1 + NFA * PS::B1A + f * PS::B1B + ji, IB * IB, outB + f * IB * IB * IB + ji,
                                       IB * IB, MB);
            }
        }
        __syncthreads();
    } else {
        // y: item (f, i), buf1 [f][qy][i] -> out [f][j][i]
        constexpr int NA2 = NFA * IA, NB2 = NFB * IB;
        for (int w = tid; w < NA2 + NB2; w += NTH) {
            if (w < NA2) {
                const int f = w / IA, i = w - f * IA;
                pencil_apply_t<IA, NQ>(buf1 + f * PS::B1A + i, PS::RA, outA + f * IA * IA + i, IA, MA);
            } else {
                const int ww = w - NA2, f = ww / IB, i = ww - f * IB;
                pencil_apply_t<IB, NQ>(buf1 + NFA * PS::B1A + f * PS::B1B + i, PS::RB, outB + f * IB * IB + i, IB, MB);
            }
        }
        __syncthreads();
    }
}

// LDS layout (in units of T) of the cell kernel
template <int DIM, int R, int NQ, typename T, Mode MODE> struct Lds {
    using Z = Sizes<DIM, R>;
    static constexpr int NQV = ipow(NQ, DIM);
    // nodal input fields of the volume pass: xhat, state (Jac), mixed field (not Mass)
    static constexpr int NFA = MODE == Mode::Jac ? 3 * DIM : (MODE == Mode::Res ? 2 * DIM : DIM);
    // quadrature-point record: NFA velocity-type fields, pressure, reference
    // gradients of xhat [c][d]; the physics overwrites them at its own point
    // (F into the gradients, value coefficients into xhat, the pressure
    // coefficient into the pressure)
    static constexpr int DQ0 = NFA + 1;                       // reference gradients of xhat
    static constexpr int Q_SIZE = (NFA + 1 + (MODE == Mode::Mass ? 0 : DIM * DIM)) * NQV;
    // temporaries of the pencil stages
    using PS = PencilSizes<DIM, NQ, NFA, Z::N1, 1, Z::RP1>;
    static constexpr int TMP1 = PS::BUF1;
    static constexpr int TMP2 = PS::BUF2 > 1 ? PS::BUF2 : 1;
    // 3D: the first pencil buffer is live only while the quadrature record is
    // dead (forward z/y stages, backward y/z stages), so it shares its words
    static constexpr bool T1_IN_Q = DIM == 3 && TMP1 <= Q_SIZE;
    // only the quadrature weights and abscissae are read from LDS
    static constexpr int QTAB = (2 * NQ + 1) & ~1;
};

} // namespace

// ---------------------------------------------------------------------------
// Helpers shared by the volume and face passes
// ---------------------------------------------------------------------------
// full-tensor index of the m-th admissible pressure multi-index (first index
// fastest, total degree <= R)
template <int DIM, int R>
__device__ __forceinline__ int pmode_full(int m)
{
    constexpr int RP1 = R + 1;
    int cnt = 0;
    for (int a2 = 0; a2 <= (DIM == 3 ? R : 0); ++a2)
        for (int a1 = 0; a1 <= R; ++a1)
            for (int a0 = 0; a0 <= R; ++a0) {
                if (a0 + a1 + a2 > R) continue;
                if (cnt == m) return a0 + RP1 * (a1 + RP1 * a2);
                ++cnt;
            }
    return 0;
}

// geometry at a reference point: J^{-T} and det J (Cartesian cells: diagonal)
template <int DIM, typename T>
__device__ __forceinline__ T geometry(bool mapped, const T *X, const T xi[3], const T h[3], T Jit[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Jit[a][b] = 0;
    if (mapped) {
        T J[3][3];
        map_jac<DIM>(X, xi, J);
        return inv_t<DIM>(J, Jit);
    }
    T det = 1;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        Jit[d][d] = T(1) / h[d];
        det *= h[d];
    }
    return det;
}

// LDS words of the cell kernel for nt time nodes
template <int DIM, int R, int NQ, typename T, Mode MODE>
__host__ __device__ constexpr int lds_words(int nt, int tabwords)
{
    using Z = Sizes<DIM, R>;
    using LY = Lds<DIM, R, NQ, T, MODE>;
    (void)tabwords;
    return LY::QTAB + nt * DIM * Z::NL + nt * Z::NPF + LY::NFA * Z::NL + Z::NPF + LY::Q_SIZE +
           (LY::T1_IN_Q ? 0 : LY::TMP1) + LY::TMP2 + 32;
}

// ---------------------------------------------------------------------------
// The cell kernel
// ---------------------------------------------------------------------------
// MAPPED: vertex-perturbed (multilinear) cells with J^{-T} and det J per
// point; else affine axis-aligned cells, whose J^{-T} = diag(1/h) is applied
// as a diagonal (a third of the point arithmetic of the general 3 x 3 form)
template <int DIM, int R, int NQ, int NTH, typename T, Mode MODE, bool MAPPED>
__global__ void __launch_bounds__(NTH) cell_kernel(CellArgs<T> A)
{
    using Z = Sizes<DIM, R>;
    using LY = Lds<DIM, R, NQ, T, MODE>;
    constexpr int N1 = Z::N1, NL = Z::NL, RP1 = Z::RP1, NPF = Z::NPF, NPM = Z::NPM;
    constexpr int NQV = LY::NQV;
    constexpr int QPT = (NQV + NTH - 1) / NTH;   // quadrature points per thread

    extern __shared__ unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);

    const int tid = threadIdx.x;
    const int cell = xcd_cell(blockIdx.x, gridDim.x);
    const int vec = blockIdx.y;
    const int nt = A.nt;
    const T *__restrict__ x = A.x + vec * A.xstride;
    T *__restrict__ y = A.y + vec * A.ystride;
    T *__restrict__ E = A.E + (long long)vec * A.ncell * nt * DIM * NL;

    // ---- LDS carve-up -------------------------------------------------------
    TableLayout lay;
    lay.init(R, NQ);
    T *qtab = sm;                                  // [NQ] weights, [NQ] abscissae
    T *xs = qtab + LY::QTAB;                       // [nt][DIM][NL] nodal x
    T *xpf = xs + nt * DIM * NL;                   // [nt][NPF] full-tensor pressure modes
    constexpr int NFA = LY::NFA;
    T *cur = xpf + nt * NPF;                       // [NFA][NL] nodal xhat^a, state^a (Jac), mixed field
    T *ns = cur + DIM * NL;                        // state (Jac)
    T *ys = cur;                                   // [DIM][NL] nodal output (inputs are dead by then)
    T *ypf = cur + NFA * NL;                       // [NPF] pressure output (full tensor)
    T *Q = ypf + NPF;                              // quadrature record
    T *t1 = LY::T1_IN_Q ? Q : Q + LY::Q_SIZE;
    T *t2 = Q + LY::Q_SIZE + (LY::T1_IN_Q ? 0 : LY::TMP1);
    T *geo = t2 + LY::TMP2;                        // [8][3] vertices

    static_assert([] {
        TableLayout t;
        t.init(R, NQ);
        return t.qx == t.qw + NQ;
    }(), "quadrature weights and abscissae are adjacent in the table block");
    for (int i = tid; i < 2 * NQ; i += NTH) qtab[i] = A.tab[lay.qw + i];

    // 1D matrices of the sweeps: uniform across the workgroup, read through the
    // scalar (read-only) path from global memory; point tables from LDS
    using CP = const __attribute__((address_space(4))) T *;   // constant for the whole kernel
    const CP S = (CP)(A.tab + lay.S), D = (CP)(A.tab + lay.D), Dq = (CP)(A.tab + lay.Dq), Lp = (CP)(A.tab + lay.L);
    const T *qw = qtab, *qx = qtab + NQ;

    // ---- cell coordinates and nodal gather ------------------------------------
    const int c0 = cell % A.n0;
    const int c1 = (cell / A.n0) % A.n1;
    const int c2 = DIM == 3 ? cell / (A.n0 * A.n1) : 0;
    const long long N0 = (long long)(R + 1) * A.n0 + 1;
    const long long N1g = (long long)(R + 1) * A.n1 + 1;
    auto gnode = [&](int l) -> long long {
        int i0 = l % N1, i1 = (l / N1) % N1, i2 = DIM == 3 ? l / (N1 * N1) : 0;
        long long g0 = (long long)(R + 1) * c0 + i0, g1 = (long long)(R + 1) * c1 + i1;
        long long g2 = (long long)(R + 1) * c2 + i2;
        return g0 + N0 * (g1 + N1g * g2);
    };

    // state velocity of the next time node, prefetched into registers so its
    // global latency overlaps the current node's work
    constexpr int PF = (DIM * NL + NTH - 1) / NTH;
    T spre[PF];
    const T *st = MODE == Mode::Jac ? A.state + vec * A.sstride : nullptr;
    auto load_state = [&](int a) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int e = tid + j * NTH;
            if (e < DIM * NL) {
                const int l = e % NL, c = e / NL;
                spre[j] = st[a * A.Nv1 + c * A.Nn + gnode(l)];
            }
        }
    };
    if constexpr (MODE == Mode::Jac) load_state(0);

    const long long pbase = (long long)nt * A.Nv1;
    for (int e = tid; e < nt * DIM * NL; e += NTH) {
        int l = e % NL, c = (e / NL) % DIM, a = e / (NL * DIM);
        xs[e] = x[a * A.Nv1 + c * A.Nn + gnode(l)];
    }
    // pressure modes of all time nodes into registers (same batch of loads),
    // scattered into the zeroed full-tensor array after the barrier
    constexpr int PP = (MAX_NT * NPM + NTH - 1) / NTH;
    T ppre[PP];
#pragma unroll
    for (int j = 0; j < PP; ++j) {
        const int e = tid + j * NTH;
        if (e < nt * NPM) ppre[j] = x[pbase + (e / NPM) * A.Np1 + (long long)cell * NPM + e % NPM];
    }
    for (int e = tid; e < nt * NPF; e += NTH) xpf[e] = 0;
    const T hcar[3] = {T(1) / A.n0, T(1) / A.n1, DIM == 3 ? T(1) / A.n2 : T(1)};
    // Cartesian cells: J^{-T} = diag(1/h) and det J, the same for every point
    // (formed once here instead of per point and time node)
    const T hinv[3] = {T(1) / hcar[0], T(1) / hcar[1], T(1) / hcar[2]};
    T det_c = 1;
#pragma unroll
    for (int d = 0; d < DIM; ++d) det_c *= hcar[d];
    constexpr bool mapped = MAPPED;
    if (mapped && tid < (1 << DIM)) {
        int v = tid;
        int o0 = v & 1, o1 = (v >> 1) & 1, o2 = (v >> 2) & 1;
        long long vi = (c0 + o0) + (long long)(A.n0 + 1) * ((c1 + o1) + (long long)(A.n1 + 1) * (c2 + o2));
        for (int a = 0; a < 3; ++a) geo[v * 3 + a] = a < DIM ? T(A.vert[vi * DIM + a]) : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PP; ++j) {
        const int e = tid + j * NTH;
        if (e < nt * NPM) xpf[(e / NPM) * NPF + pmode_full<DIM, R>(e % NPM)] = ppre[j];
    }

    __syncthreads();

    for (int a = 0; a < nt; ++a) {
        // ---- nodal inputs: xhat^a, state^a (Jac), mixed field sum_b K_ab x^b (- phi0_a vprev)
        constexpr int MIXF = MODE == Mode::Jac ? 2 * DIM : DIM;
        if constexpr (MODE == Mode::Jac) {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                const int e = tid + j * NTH;
                if (e < DIM * NL) {
                    const int l = e % NL, c = e / NL;
                    cur[e] = xs[(a * DIM + c) * NL + l];
                    ns[e] = spre[j];
                    T m = 0;
                    for (int b = 0; b < nt; ++b) m += A.K[a * nt + b] * xs[(b * DIM + c) * NL + l];
                    cur[MIXF * NL + e] = m;
                }
            }
            if (a + 1 < nt) load_state(a + 1);
        } else {
            for (int e = tid; e < DIM * NL; e += NTH) {
                const int l = e % NL, c = e / NL;
                cur[e] = xs[(a * DIM + c) * NL + l];
                if constexpr (MODE == Mode::Res) {
                    T m = 0;
                    for (int b = 0; b < nt; ++b) m += A.K[a * nt + b] * xs[(b * DIM + c) * NL + l];
                    if (A.vprev) m -= A.phi0[a] * A.vprev[c * A.Nn + gnode(l)];
                    cur[MIXF * NL + e] = m;
                }
            }
        }
        __syncthreads();

        // ---- nodes -> Gauss points: Q fields [0, NFA) velocity-type, NFA pressure
        constexpr int NG = MODE == Mode::Mass ? 0 : DIM;
        T *G = Q + LY::DQ0 * NQV;
        pencil_fwd<DIM, NQ, NFA, N1, 1, RP1, NG, NTH, T>(cur, xpf + a * NPF, Q, Q + NFA * NQV, G, t1, t2, S, D, Lp);
        if constexpr (MODE != Mode::Mass) colloc_fwd<DIM, NQ, DIM, NTH, T>(Q, G, Dq);

        // ---- quadrature-point physics, in place at each point ----------------------
        const T wa = A.w[a];
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const int q = tid + j * NTH;
            if (q < NQV) {
                const int qi[3] = {q % NQ, (q / NQ) % NQ, DIM == 3 ? q / (NQ * NQ) : 0};
                T xi[3] = {0, 0, 0}, Jit[3][3];
#pragma unroll
                for (int d = 0; d < DIM; ++d) xi[d] = qx[qi[d]];
                T det;
                if constexpr (MAPPED) {
                    det = geometry<DIM>(true, geo, xi, hcar, Jit);
                } else {
                    det = det_c;
                }
                T jxw = det;
#pragma unroll
                for (int d = 0; d < DIM; ++d) jxw *= qw[qi[d]];
                const T sc = wa * jxw;
                T xh[3] = {0, 0, 0}, v[3] = {0, 0, 0};
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    xh[c] = Q[c * NQV + q];
                    if constexpr (MODE == Mode::Jac) v[c] = Q[(DIM + c) * NQV + q];
                    else v[c] = xh[c];
                }
                const T ph = Q[NFA * NQV + q];
                if constexpr (MODE == Mode::Mass) {
#pragma unroll
                    for (int c = 0; c < DIM; ++c) Q[c * NQV + q] = sc * xh[c];
                    Q[NFA * NQV + q] = sc * ph;
                } else {
                    T divx = 0;
#pragma unroll
                    for (int c = 0; c < DIM; ++c) {
                        T gref[3];
#pragma unroll
                        for (int jd = 0; jd < DIM; ++jd) gref[jd] = G[(c * DIM + jd) * NQV + q];
                        T Fc[3];
#pragma unroll
                        for (int d = 0; d < DIM; ++d) {
                            T g = 0;
                            if constexpr (MAPPED) {
#pragma unroll
                                for (int jd = 0; jd < DIM; ++jd) g += Jit[d][jd] * gref[jd];
                            } else {
                                g = hinv[d] * gref[d];
                            }
                            if (d == c) divx += g;
                            // nu grad x - x (x) v - v (x) x - p I (Jacobian); Res: v = x, one convective term
                            Fc[d] = A.nu * g - xh[c] * v[d] - (MODE == Mode::Jac ? v[c] * xh[d] : T(0));
                            if (d == c) Fc[d] -= ph;
                        }
#pragma unroll
                        for (int jd = 0; jd < DIM; ++jd) {
                            T s = 0;
                            if constexpr (MAPPED) {
#pragma unroll
                                for (int d = 0; d < DIM; ++d) s += Fc[d] * Jit[d][jd];
                            } else {
                                s = Fc[jd] * hinv[jd];
                            }
                            G[(c * DIM + jd) * NQV + q] = s * sc;
                        }
                    }
                    T xm[3];
#pragma unroll
                    for (int c = 0; c < DIM; ++c) xm[c] = Q[(MIXF + c) * NQV + q];
#pragma unroll
                    for (int c = 0; c < DIM; ++c) Q[c * NQV + q] = jxw * xm[c];
                    Q[NFA * NQV + q] = -sc * divx;
                }
            }
        }
        __syncthreads();

        // ---- transposed collocation along y, z (into the value fields), then Gauss
        //      points -> nodes with the x part of the test gradient
        if constexpr (MODE != Mode::Mass) colloc_bwd<DIM, NQ, NTH, T>(G, Q, Dq);
        pencil_bwd<DIM, NQ, DIM, N1, 1, RP1, MODE != Mode::Mass, NTH, T>(Q, G, DIM * NQV, Q + NFA * NQV, ys, ypf, t1,
                                                                        t2, S, D, Lp);

        // ---- write results ---------------------------------------------------------
        T *Ec = E + ((long long)cell * nt + a) * DIM * NL;
        for (int e = tid; e < DIM * NL; e += NTH) Ec[e] = ys[e];
        for (int e = tid; e < NPM; e += NTH) {
            const long long gi = pbase + a * A.Np1 + (long long)cell * NPM + e;
            T val = ypf[pmode_full<DIM, R>(e)];
            if constexpr (MODE == Mode::Res) {
                if (A.rhs) val -= A.rhs[gi];
            }
            y[gi] = val;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 3D Jacobian volume kernel (eq. JacobianLocal, convective part eq. Defcp).
//
// Same cell / time-node decomposition as cell_kernel, different contraction
// order: the reference gradient of the direction field is obtained by
// contracting with the nodal derivative table D along the axis in question
// (z and y during the first two sweeps, x in the last), not by collocation at
// the Gauss points.  The last forward contraction then needs only rows that
// the earlier sweeps left in LDS, so one thread per quadrature point finishes
// the interpolation, evaluates the point physics and writes its 13
// coefficients; three sweeps take them back to the nodes and the last one
// writes E and the pressure rows from registers.  Per time node that is six
// barrier-separated stages (z, y, x + physics, x^T, y^T, z^T).  The
// time-mixed field sum_b K_ab x^b is formed while loading the z columns.
// Every item type of a stage starts on a wavefront boundary so that no
// wavefront executes two item types.
// ---------------------------------------------------------------------------
constexpr int al64(int v) { return (v + 63) & ~63; }
constexpr int al4(int v) { return (v + 3) & ~3; }

template <int R, int NQ> struct JacLds {
    static constexpr int N1 = R + 2, RP1 = R + 1, NL = N1 * N1 * N1, NQV = NQ * NQ * NQ;
    static constexpr int QN2 = NQ * N1 * N1;     // one field after the z sweep [qz][j][i]
    static constexpr int QQN = NQ * NQ * N1;     // one field after the y sweep [qz][qy][i]
    // 1D tables (rows per quadrature point for the thread-per-point stage)
    static constexpr int TS = 0, TD = TS + NQ * N1, TL = TD + NQ * N1, QW = TL + NQ * RP1, QX = QW + NQ;
    static constexpr int GEO = al4(QX + NQ);     // [8][3] vertices (mapped cells)
    // region P: z-sweep results (xhat along z by S and by D, state, mixed field,
    // pressure), then the point record [13][NQV], then the y^T results; the
    // nodal state of the next time node sits behind the z-sweep results
    static constexpr int ZXS = 0, ZXD = 3 * QN2, ZS = 6 * QN2, ZM = 9 * QN2, ZP = 12 * QN2;
    static constexpr int NSO = al4(ZP + NQ * RP1 * RP1);
    static constexpr int WA = 0, WC = 3 * QN2, WP = 6 * QN2;
    static constexpr int RPW = al4(NSO + 3 * NL > 13 * NQV ? NSO + 3 * NL : 13 * NQV);
    // region Y: y-sweep results (xhat: S_y S_z, D_y S_z, S_y D_z; state; mixed;
    // pressure), then the x^T results (value + x-gradient, y-gradient,
    // z-gradient coefficients; pressure)
    static constexpr int YSS = 0, YDS = 3 * QQN, YSD = 6 * QQN, YS = 9 * QQN, YM = 12 * QQN, YP = 15 * QQN;
    static constexpr int BA = 0, BB = 3 * QQN, BC = 6 * QQN, BP = 9 * QQN;
    static constexpr int RYW = al4(15 * QQN + NQ * NQ * RP1);
    static constexpr int RP = GEO + 24, RY = RP + RPW;
    // then [nt][NPF] pressure modes and [nt][3][NL] nodal x of all time nodes
    static constexpr int XP0 = RY + RYW;
    static_assert(WP + NQ * RP1 * RP1 <= NSO, "y^T results stay clear of the nodal state");
};

template <int R, int NQ, typename T>
__host__ __device__ constexpr int jac_lds_words(int nt)
{
    using LY = JacLds<R, NQ>;
    return LY::XP0 + nt * ((R + 1) * (R + 1) * (R + 1) + 3 * LY::NL);
}

// position of the pressure multi-index (i0, i1, i2) in the admissible
// ordering of pmode_full (first index fastest), or -1 if its degree exceeds R
template <int R>
__device__ __forceinline__ int pmode_compact(int i0, int i1, int i2)
{
    if (i0 + i1 + i2 > R) return -1;
    int cnt = 0;
    for (int a2 = 0; a2 < i2; ++a2) cnt += (R - a2 + 1) * (R - a2 + 2) / 2;
    for (int a1 = 0; a1 < i1; ++a1) cnt += R - i2 - a1 + 1;
    return cnt + i0;
}

// FUSED: the boundary-face items run in the same launch and add onto this
// cell's E entries and pressure rows; for cells on the domain boundary the
// volume result is then added atomically too (onto entries zeroed before the
// launch)
template <int R, int NQ, int NTH, typename T, bool MAPPED, bool FUSED>
__device__ __forceinline__ void jac_cell_body(const CellArgs<T> &A, const int cell, const int vec, T *sm,
                                              const int tid)
{
    using LY = JacLds<R, NQ>;
    constexpr int N1 = R + 2, RP1 = R + 1, NL = LY::NL, NPF = RP1 * RP1 * RP1, NPM = Sizes<3, R>::NPM;
    constexpr int NQV = LY::NQV, QN2 = LY::QN2, QQN = LY::QQN, N2 = N1 * N1, RP2 = RP1 * RP1;

    T *tS = sm + LY::TS, *tD = sm + LY::TD, *tL = sm + LY::TL, *qw = sm + LY::QW, *qxs = sm + LY::QX;
    T *geo = sm + LY::GEO;
    T *P = sm + LY::RP, *Y = sm + LY::RY;
    T *NS = P + LY::NSO;
    const int nt = A.nt;
    T *XP = sm + LY::XP0;                 // [nt][NPF]
    T *XS = XP + nt * NPF;                // [nt][3][NL]

    const T *__restrict__ x = A.x + vec * A.xstride;
    T *__restrict__ y = A.y + vec * A.ystride;
    T *__restrict__ E = A.E + (long long)vec * A.ncell * nt * 3 * NL;

    TableLayout lay;
    lay.init(R, NQ);
    // matrices indexed by compile-time row/column in the sweeps: scalar path
    using CP = const __attribute__((address_space(4))) T *;
    const CP S = (CP)(A.tab + lay.S), D = (CP)(A.tab + lay.D), L = (CP)(A.tab + lay.L);
    // rows selected by the point's own x index: from LDS
    for (int i = tid; i < NQ * N1; i += NTH) {
        tS[i] = A.tab[lay.S + i];
        tD[i] = A.tab[lay.D + i];
    }
    for (int i = tid; i < NQ * RP1; i += NTH) tL[i] = A.tab[lay.L + i];
    for (int i = tid; i < NQ; i += NTH) {
        qw[i] = A.tab[lay.qw + i];
        qxs[i] = A.tab[lay.qx + i];
    }

    const int c0 = cell % A.n0;
    const int c1 = (cell / A.n0) % A.n1;
    const int c2 = cell / (A.n0 * A.n1);
    const bool atomic_out =
        FUSED && (c0 == 0 || c0 == A.n0 - 1 || c1 == 0 || c1 == A.n1 - 1 || c2 == 0 || c2 == A.n2 - 1);
    const long long N0 = (long long)(R + 1) * A.n0 + 1;
    const long long N1g = (long long)(R + 1) * A.n1 + 1;
    auto gnode = [&](int l) -> long long {
        int i0 = l % N1, i1 = (l / N1) % N1, i2 = l / N2;
        long long g0 = (long long)(R + 1) * c0 + i0, g1 = (long long)(R + 1) * c1 + i1;
        long long g2 = (long long)(R + 1) * c2 + i2;
        return g0 + N0 * (g1 + N1g * g2);
    };

    // state of a time node into registers (element e = tid + j * NTH)
    constexpr int PF = (3 * NL + NTH - 1) / NTH;
    T spre[PF];
    const T *st = A.state + vec * A.sstride;
    auto load_state = [&](int a) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int e = tid + j * NTH;
            if (e < 3 * NL) {
                const int l = e % NL, c = e / NL;
                spre[j] = st[a * A.Nv1 + c * A.Nn + gnode(l)];
            }
        }
    };
    auto store_state = [&]() {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int e = tid + j * NTH;
            if (e < 3 * NL) NS[e] = spre[j];
        }
    };
    load_state(0);
    for (int e = tid; e < nt * 3 * NL; e += NTH) {
        const int l = e % NL, c = (e / NL) % 3, a = e / (3 * NL);
        XS[e] = x[a * A.Nv1 + c * A.Nn + gnode(l)];
    }
    const long long pbase = (long long)nt * A.Nv1;
    constexpr int PP = (MAX_NT * NPM + NTH - 1) / NTH;
    T ppre[PP];
#pragma unroll
    for (int j = 0; j < PP; ++j) {
        const int e = tid + j * NTH;
        if (e < nt * NPM) ppre[j] = x[pbase + (e / NPM) * A.Np1 + (long long)cell * NPM + e % NPM];
    }
    for (int e = tid; e < nt * NPF; e += NTH) XP[e] = 0;
    const T hcar[3] = {T(1) / A.n0, T(1) / A.n1, T(1) / A.n2};
    const T hinv[3] = {T(1) / hcar[0], T(1) / hcar[1], T(1) / hcar[2]};
    const T det_c = hcar[0] * hcar[1] * hcar[2];
    if (MAPPED && tid < 8) {
        const int v = tid, o0 = v & 1, o1 = (v >> 1) & 1, o2 = (v >> 2) & 1;
        const long long vi = (c0 + o0) + (long long)(A.n0 + 1) * ((c1 + o1) + (long long)(A.n1 + 1) * (c2 + o2));
        for (int k = 0; k < 3; ++k) geo[v * 3 + k] = T(A.vert[vi * 3 + k]);
    }
    store_state();
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PP; ++j) {
        const int e = tid + j * NTH;
        if (e < nt * NPM) XP[(e / NPM) * NPF + pmode_full<3, R>(e % NPM)] = ppre[j];
    }
    if (nt > 1) load_state(1);
    __syncthreads();

    for (int a = 0; a < nt; ++a) {
        // ---- z sweep: xhat by S and D, state and mixed field by S, pressure by L
        {
            constexpr int NX = 3 * N2, O1 = al64(NX), O2 = O1 + al64(3 * N2), TOT = O2 + RP2;
            for (int w = tid; w < TOT; w += NTH) {
                if (w < NX) {
                    const int c = w / N2, ji = w - c * N2;
                    const T *src = XS + (a * 3 + c) * NL + ji;
                    T u[N1];
#pragma unroll
                    for (int k = 0; k < N1; ++k) u[k] = src[k * N2];
                    T *oS = P + LY::ZXS + c * QN2 + ji, *oD = P + LY::ZXD + c * QN2 + ji;
#pragma unroll
                    for (int qz = 0; qz < NQ; ++qz) {
                        T s = 0, d = 0;
#pragma unroll
                        for (int k = 0; k < N1; ++k) {
                            s += S[qz * N1 + k] * u[k];
                            d += D[qz * N1 + k] * u[k];
                        }
                        oS[qz * N2] = s;
                        oD[qz * N2] = d;
                    }
                } else if (w >= O1 && w < O1 + 3 * N2) {
                    const int ww = w - O1, c = ww / N2, ji = ww - c * N2;
                    T u[N1], m[N1];
#pragma unroll
                    for (int k = 0; k < N1; ++k) {
                        u[k] = NS[c * NL + k * N2 + ji];
                        m[k] = 0;
                    }
                    for (int b = 0; b < nt; ++b) {
                        const T kab = A.K[a * nt + b];
                        const T *src = XS + (b * 3 + c) * NL + ji;
#pragma unroll
                        for (int k = 0; k < N1; ++k) m[k] += kab * src[k * N2];
                    }
                    T *os = P + LY::ZS + c * QN2 + ji, *om = P + LY::ZM + c * QN2 + ji;
#pragma unroll
                    for (int qz = 0; qz < NQ; ++qz) {
                        T s = 0, mm = 0;
#pragma unroll
                        for (int k = 0; k < N1; ++k) {
                            s += S[qz * N1 + k] * u[k];
                            mm += S[qz * N1 + k] * m[k];
                        }
                        os[qz * N2] = s;
                        om[qz * N2] = mm;
                    }
                } else if (w >= O2) {
                    const int ji = w - O2;
                    const T *src = XP + a * NPF + ji;
                    T u[RP1];
#pragma unroll
                    for (int k = 0; k < RP1; ++k) u[k] = src[k * RP2];
                    T *op = P + LY::ZP + ji;
#pragma unroll
                    for (int qz = 0; qz < NQ; ++qz) {
                        T s = 0;
#pragma unroll
                        for (int k = 0; k < RP1; ++k) s += L[qz * RP1 + k] * u[k];
                        op[qz * RP2] = s;
                    }
                }
            }
            __syncthreads();
        }
        // ---- y sweep: xhat -> S_y S_z, D_y S_z, S_y D_z; state, mixed -> S_y; pressure -> L
        {
            constexpr int NX = 3 * NQ * N1, O1 = al64(NX), O2 = O1 + al64(3 * NQ * N1), TOT = O2 + NQ * RP1;
            for (int w = tid; w < TOT; w += NTH) {
                if (w < NX) {
                    const int c = w / (NQ * N1), rr = w - c * NQ * N1, qz = rr / N1, i = rr - qz * N1;
                    const T *sS = P + LY::ZXS + c * QN2 + qz * N2 + i, *sD = P + LY::ZXD + c * QN2 + qz * N2 + i;
                    T u[N1], v[N1];
#pragma unroll
                    for (int j = 0; j < N1; ++j) {
                        u[j] = sS[j * N1];
                        v[j] = sD[j * N1];
                    }
                    const int ob = c * QQN + qz * NQ * N1 + i;
#pragma unroll
                    for (int qy = 0; qy < NQ; ++qy) {
                        T ss = 0, ds = 0, sd = 0;
#pragma unroll
                        for (int j = 0; j < N1; ++j) {
                            ss += S[qy * N1 + j] * u[j];
                            ds += D[qy * N1 + j] * u[j];
                            sd += S[qy * N1 + j] * v[j];
                        }
                        Y[LY::YSS + ob + qy * N1] = ss;
                        Y[LY::YDS + ob + qy * N1] = ds;
                        Y[LY::YSD + ob + qy * N1] = sd;
                    }
                } else if (w >= O1 && w < O1 + 3 * NQ * N1) {
                    const int ww = w - O1, c = ww / (NQ * N1), rr = ww - c * NQ * N1, qz = rr / N1, i = rr - qz * N1;
                    const T *sS = P + LY::ZS + c * QN2 + qz * N2 + i, *sM = P + LY::ZM + c * QN2 + qz * N2 + i;
                    T u[N1], m[N1];
#pragma unroll
                    for (int j = 0; j < N1; ++j) {
                        u[j] = sS[j * N1];
                        m[j] = sM[j * N1];
                    }
                    const int ob = c * QQN + qz * NQ * N1 + i;
#pragma unroll
                    for (int qy = 0; qy < NQ; ++qy) {
                        T s = 0, mm = 0;
#pragma unroll
                        for (int j = 0; j < N1; ++j) {
                            s += S[qy * N1 + j] * u[j];
                            mm += S[qy * N1 + j] * m[j];
                        }
                        Y[LY::YS + ob + qy * N1] = s;
                        Y[LY::YM + ob + qy * N1] = mm;
                    }
                } else if (w >= O2) {
                    const int ww = w - O2, qz = ww / RP1, ip = ww - qz * RP1;
                    const T *src = P + LY::ZP + qz * RP2 + ip;
                    T u[RP1];
#pragma unroll
                    for (int j = 0; j < RP1; ++j) u[j] = src[j * RP1];
                    T *op = Y + LY::YP + qz * NQ * RP1 + ip;
#pragma unroll
                    for (int qy = 0; qy < NQ; ++qy) {
                        T s = 0;
#pragma unroll
                        for (int j = 0; j < RP1; ++j) s += L[qy * RP1 + j] * u[j];
                        op[qy * RP1] = s;
                    }
                }
            }
            __syncthreads();
        }
        // ---- x sweep and point physics: one thread per quadrature point ---------------
        {
            const T wa = A.w[a];
            for (int q = tid; q < NQV; q += NTH) {
                const int qx = q % NQ, qy = (q / NQ) % NQ, qz = q / (NQ * NQ);
                const int row = qz * NQ + qy;
                T sx[N1], dx[N1], lx[RP1];
#pragma unroll
                for (int i = 0; i < N1; ++i) {
                    sx[i] = tS[qx * N1 + i];
                    dx[i] = tD[qx * N1 + i];
                }
#pragma unroll
                for (int i = 0; i < RP1; ++i) lx[i] = tL[qx * RP1 + i];
                T xh[3], gref[3][3], v[3], xm[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int rb = c * QQN + row * N1;
                    T a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
#pragma unroll
                    for (int i = 0; i < N1; ++i) {
                        const T u = Y[LY::YSS + rb + i];
                        a0 += sx[i] * u;
                        a1 += dx[i] * u;
                        a2 += sx[i] * Y[LY::YDS + rb + i];
                        a3 += sx[i] * Y[LY::YSD + rb + i];
                        a4 += sx[i] * Y[LY::YS + rb + i];
                        a5 += sx[i] * Y[LY::YM + rb + i];
                    }
                    xh[c] = a0;
                    gref[c][0] = a1;
                    gref[c][1] = a2;
                    gref[c][2] = a3;
                    v[c] = a4;
                    xm[c] = a5;
                }
                T ph = 0;
#pragma unroll
                for (int i = 0; i < RP1; ++i) ph += lx[i] * Y[LY::YP + row * RP1 + i];
                T det, Jit[3][3];
                if constexpr (MAPPED) {
                    const T xi[3] = {qxs[qx], qxs[qy], qxs[qz]};
                    det = geometry<3>(true, geo, xi, hcar, Jit);
                } else {
                    det = det_c;
                }
                const T jxw = det * qw[qx] * qw[qy] * qw[qz];
                const T sc = wa * jxw;
                T divx = 0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    T Fc[3];
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        T g = 0;
                        if constexpr (MAPPED) {
#pragma unroll
                            for (int jd = 0; jd < 3; ++jd) g += Jit[d][jd] * gref[c][jd];
                        } else {
                            g = hinv[d] * gref[c][d];
                        }
                        if (d == c) divx += g;
                        // nu grad x - x (x) v - v (x) x - p I
                        Fc[d] = A.nu * g - xh[c] * v[d] - v[c] * xh[d];
                        if (d == c) Fc[d] -= ph;
                    }
#pragma unroll
                    for (int jd = 0; jd < 3; ++jd) {
                        T s = 0;
                        if constexpr (MAPPED) {
#pragma unroll
                            for (int d = 0; d < 3; ++d) s += Fc[d] * Jit[d][jd];
                        } else {
                            s = Fc[jd] * hinv[jd];
                        }
                        P[(3 + c * 3 + jd) * NQV + q] = s * sc;
                    }
                    P[c * NQV + q] = jxw * xm[c];
                }
                P[12 * NQV + q] = -sc * divx;
            }
            __syncthreads();
        }
        // ---- x^T: per (component, qz, qy) pencil, value + x-gradient (S, D), y- and
        //      z-gradient coefficients (S); pressure by L
        {
            constexpr int NI = 3 * NQ * NQ, O1 = al64(NI), TOT = O1 + NQ * NQ;
            for (int w = tid; w < TOT; w += NTH) {
                if (w < NI) {
                    const int c = w / (NQ * NQ), row = w - c * NQ * NQ;
                    const T *pv = P + c * NQV + row * NQ, *pg = P + (3 + c * 3) * NQV + row * NQ;
                    T u[NQ], g0[NQ], g1[NQ], g2[NQ];
#pragma unroll
                    for (int o = 0; o < NQ; ++o) {
                        u[o] = pv[o];
                        g0[o] = pg[o];
                        g1[o] = pg[NQV + o];
                        g2[o] = pg[2 * NQV + o];
                    }
                    const int ob = c * QQN + row * N1;
#pragma unroll
                    for (int i = 0; i < N1; ++i) {
                        T sa = 0, sb = 0, scc = 0;
#pragma unroll
                        for (int o = 0; o < NQ; ++o) {
                            sa += S[o * N1 + i] * u[o];
                            sa += D[o * N1 + i] * g0[o];
                            sb += S[o * N1 + i] * g1[o];
                            scc += S[o * N1 + i] * g2[o];
                        }
                        Y[LY::BA + ob + i] = sa;
                        Y[LY::BB + ob + i] = sb;
                        Y[LY::BC + ob + i] = scc;
                    }
                } else if (w >= O1) {
                    const int row = w - O1;
                    const T *pp = P + 12 * NQV + row * NQ;
                    T u[NQ];
#pragma unroll
                    for (int o = 0; o < NQ; ++o) u[o] = pp[o];
#pragma unroll
                    for (int i = 0; i < RP1; ++i) {
                        T s = 0;
#pragma unroll
                        for (int o = 0; o < NQ; ++o) s += L[o * RP1 + i] * u[o];
                        Y[LY::BP + row * RP1 + i] = s;
                    }
                }
            }
            __syncthreads();
        }
        // ---- y^T: per (component, qz, i) pencil; pressure by L
        {
            constexpr int NI = 3 * NQ * N1, O1 = al64(NI), TOT = O1 + NQ * RP1;
            for (int w = tid; w < TOT; w += NTH) {
                if (w < NI) {
                    const int c = w / (NQ * N1), rr = w - c * NQ * N1, qz = rr / N1, i = rr - qz * N1;
                    const int sb = c * QQN + qz * NQ * N1 + i;
                    T ua[NQ], ub[NQ], uc[NQ];
#pragma unroll
                    for (int o = 0; o < NQ; ++o) {
                        ua[o] = Y[LY::BA + sb + o * N1];
                        ub[o] = Y[LY::BB + sb + o * N1];
                        uc[o] = Y[LY::BC + sb + o * N1];
                    }
                    const int ob = c * QN2 + qz * N2 + i;
#pragma unroll
                    for (int j = 0; j < N1; ++j) {
                        T sa = 0, scc = 0;
#pragma unroll
                        for (int o = 0; o < NQ; ++o) {
                            sa += S[o * N1 + j] * ua[o];
                            sa += D[o * N1 + j] * ub[o];
                            scc += S[o * N1 + j] * uc[o];
                        }
                        P[LY::WA + ob + j * N1] = sa;
                        P[LY::WC + ob + j * N1] = scc;
                    }
                } else if (w >= O1) {
                    const int ww = w - O1, qz = ww / RP1, ip = ww - qz * RP1;
                    T u[NQ];
#pragma unroll
                    for (int o = 0; o < NQ; ++o) u[o] = Y[LY::BP + qz * NQ * RP1 + o * RP1 + ip];
#pragma unroll
                    for (int j = 0; j < RP1; ++j) {
                        T s = 0;
#pragma unroll
                        for (int o = 0; o < NQ; ++o) s += L[o * RP1 + j] * u[o];
                        P[LY::WP + qz * RP2 + j * RP1 + ip] = s;
                    }
                }
            }
            __syncthreads();
        }
        // ---- z^T: per (component, j, i) column, straight to E; pressure rows; the
        //      next time node's state into LDS (clear of the y^T results)
        {
            constexpr int NI = 3 * N2, O1 = al64(NI), TOT = O1 + RP2;
            T *Ec = E + ((long long)cell * nt + a) * 3 * NL;
            for (int w = tid; w < TOT; w += NTH) {
                if (w < NI) {
                    const int c = w / N2, ji = w - c * N2;
                    T ua[NQ], uc[NQ];
#pragma unroll
                    for (int o = 0; o < NQ; ++o) {
                        ua[o] = P[LY::WA + c * QN2 + o * N2 + ji];
                        uc[o] = P[LY::WC + c * QN2 + o * N2 + ji];
                    }
#pragma unroll
                    for (int k = 0; k < N1; ++k) {
                        T s = 0;
#pragma unroll
                        for (int o = 0; o < NQ; ++o) {
                            s += S[o * N1 + k] * ua[o];
                            s += D[o * N1 + k] * uc[o];
                        }
                        if (atomic_out) unsafeAtomicAdd(Ec + c * NL + k * N2 + ji, s);
                        else Ec[c * NL + k * N2 + ji] = s;
                    }
                } else if (w >= O1) {
                    const int ji = w - O1, jp = ji / RP1, ip = ji - jp * RP1;
                    T u[NQ];
#pragma unroll
                    for (int o = 0; o < NQ; ++o) u[o] = P[LY::WP + o * RP2 + ji];
#pragma unroll
                    for (int kp = 0; kp < RP1; ++kp) {
                        const int e = pmode_compact<R>(ip, jp, kp);
                        if (e >= 0) {
                            T s = 0;
#pragma unroll
                            for (int o = 0; o < NQ; ++o) s += L[o * RP1 + kp] * u[o];
                            if (atomic_out) unsafeAtomicAdd(y + pbase + a * A.Np1 + (long long)cell * NPM + e, s);
                            else y[pbase + a * A.Np1 + (long long)cell * NPM + e] = s;
                        }
                    }
                }
            }
            if (a + 1 < nt) {
                store_state();
                if (a + 2 < nt) load_state(a + 2);
            }
            __syncthreads();
        }
    }
}

template <int R, int NQ, int NTH, typename T, bool MAPPED>
__global__ void __launch_bounds__(NTH) jac_cell_kernel(CellArgs<T> A)
{
    extern __shared__ unsigned char smem_raw[];
    jac_cell_body<R, NQ, NTH, T, MAPPED, false>(A, xcd_cell(blockIdx.x, gridDim.x), blockIdx.y,
                                                reinterpret_cast<T *>(smem_raw), threadIdx.x);
}

// ---------------------------------------------------------------------------
// Boundary-face kernel: the Nitsche and convective boundary terms (eq.
// def-a-gam-tp, eq. def-b-gam) of the cells on the domain boundary, one
// workgroup per boundary cell and time node.  Runs after the volume
// kernel on the same stream and adds to its results (cell buffer E, pressure
// rows), so the summation order is fixed.
// ---------------------------------------------------------------------------
template <int DIM, int R, int NQ, typename T> struct FaceLds {
    using Z = Sizes<DIM, R>;
    static constexpr int NQV = ipow(NQ, DIM);
    static constexpr int NQF = ipow(NQ, DIM - 1);
    static constexpr int NF_F = DIM + DIM * DIM + DIM + 1;    // xhat, grad xhat, v, p
    // the point terms overwrite their inputs with the (fewer) output fields
    static_assert(DIM + DIM * DIM + 1 <= NF_F, "face outputs fit over the inputs");
    static constexpr int Q_SIZE = NF_F * NQF;
    // normal-reduced layers and the tangential pencil buffer (also used by the
    // h_F reductions: one word per thread, NQF face points)
    static constexpr int LN = DIM == 3 ? Z::N1 * Z::N1 : Z::N1;
    static constexpr int LP = DIM == 3 ? Z::RP1 * Z::RP1 : Z::RP1;
    static constexpr int L1 = 3 * DIM * LN + LP;
    static constexpr int L2 = DIM == 3 ? 4 * DIM * Z::N1 * NQ + Z::RP1 * NQ : 1;
    // one word per thread of the (64-thread) volume reduction in TMP1
    static constexpr int TMP1 = L1 > 64 ? L1 : 64;
    static constexpr int TMP2 = L2 > NQF ? L2 : NQF;
    // 3D: the layer buffer is live only while the face record is dead (the
    // normal reduction and the first tangential stage; the last tangential
    // stage and the normal expansion), so it shares its words
    static constexpr bool T1_IN_Q = DIM == 3;
    static constexpr int SCR1 = T1_IN_Q ? (Q_SIZE > TMP1 ? Q_SIZE : TMP1) : Q_SIZE + TMP1;
    // face rows of the 1D tables (Se, De, Le) and the Gauss weights/abscissae
    static constexpr int FTAB = (4 * Z::N1 + 2 * Z::RP1 + 2 * NQ + 1) & ~1;
};

template <int DIM, int R, int NQ, typename T>
__host__ __device__ constexpr int face_lds_words(int tabwords)
{
    using Z = Sizes<DIM, R>;
    using LY = FaceLds<DIM, R, NQ, T>;
    (void)tabwords;
    return LY::FTAB + 2 * DIM * Z::NL + 2 * Z::NPF + LY::SCR1 + LY::TMP2 + 32;
}

// barrier of one face item: the workgroup, or (FUSED: several items per
// workgroup, one per wavefront, each with its own LDS slice) the wavefront,
// whose LDS accesses complete in issue order
template <bool WAVE> __device__ __forceinline__ void face_sync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// One (boundary cell, time node) item, bsl = index into the boundary cells x
// time nodes, by NTH = 64 threads.  Not FUSED: added to the volume result
// already in E and in the pressure rows.  FUSED: the volume pass runs in the
// same launch and adds its result atomically as well, onto entries zeroed
// before the launch; with exactly two contributions per entry the sum does not
// depend on their order, so results stay bitwise reproducible.
template <int DIM, int R, int NQ, int NTH, typename T, Mode MODE, bool FUSED>
__device__ __forceinline__ void face_item(const CellArgs<T> &A, const int bsl, const int vec, T *sm, const int tid)
{
    using Z = Sizes<DIM, R>;
    using LY = FaceLds<DIM, R, NQ, T>;
    constexpr int N1 = Z::N1, NL = Z::NL, RP1 = Z::RP1, NPF = Z::NPF, NPM = Z::NPM;
    constexpr int NQV = LY::NQV, NQF = LY::NQF;
    constexpr int NQ2 = DIM == 2 ? 1 : NQ;
    constexpr int N12 = DIM == 2 ? 1 : N1;
    constexpr int RP12 = DIM == 2 ? 1 : RP1;

    static_assert(NTH == 64, "one wavefront per face item");
    const int cell = A.bcells[bsl / A.nt];
    const int a = bsl % A.nt;                     // one time node per item
    const int nt = A.nt;
    const T *__restrict__ x = A.x + vec * A.xstride;
    T *__restrict__ y = A.y + vec * A.ystride;
    T *__restrict__ E = A.E + (long long)vec * A.ncell * nt * DIM * NL;

    TableLayout lay;
    lay.init(R, NQ);
    T *ftab = sm;                                  // Se, De, Le, qw, qx
    T *xs = ftab + LY::FTAB;                       // [DIM][NL] nodal x of the time node
    T *ns = xs + DIM * NL;                         // [DIM][NL] nodal state
    T *xpf = ns + DIM * NL;                        // [NPF] pressure modes (full tensor)
    T *ypf = xpf + NPF;                            // [NPF] pressure output
    T *Q = ypf + NPF;                              // face record
    T *t1 = LY::T1_IN_Q ? Q : Q + LY::Q_SIZE;
    T *t2 = Q + LY::SCR1;
    T *geo = t2 + LY::TMP2;                        // [8][3] vertices, [6] h_F, [1] volume

    static_assert([] {
        TableLayout t;
        t.init(R, NQ);
        return t.De == t.Se + 2 * (R + 2) && t.qw == t.Le + 2 * (R + 1) && t.qx == t.qw + NQ;
    }(), "face rows and point tables are adjacent in the table block");
    using CP = const __attribute__((address_space(4))) T *;   // constant for the whole kernel
    const CP S = (CP)(A.tab + lay.S), D = (CP)(A.tab + lay.D), Lp = (CP)(A.tab + lay.L);
    const T *Se = ftab, *De = ftab + 2 * N1, *Lpe = ftab + 4 * N1, *qw = Lpe + 2 * RP1;
    const T *qx = qw + NQ;

    const int c0 = cell % A.n0;
    const int c1 = (cell / A.n0) % A.n1;
    const int c2 = DIM == 3 ? cell / (A.n0 * A.n1) : 0;
    const long long N0 = (long long)(R + 1) * A.n0 + 1;
    const long long N1g = (long long)(R + 1) * A.n1 + 1;
    auto gnode = [&](int l) -> long long {
        int i0 = l % N1, i1 = (l / N1) % N1, i2 = DIM == 3 ? l / (N1 * N1) : 0;
        long long g0 = (long long)(R + 1) * c0 + i0, g1 = (long long)(R + 1) * c1 + i1;
        long long g2 = (long long)(R + 1) * c2 + i2;
        return g0 + N0 * (g1 + N1g * g2);
    };
    const long long pbase = (long long)nt * A.Nv1;
    const T hcar[3] = {T(1) / A.n0, T(1) / A.n1, DIM == 3 ? T(1) / A.n2 : T(1)};
    const bool mapped = A.mapped != 0;

    // ---- one batch of global loads: tables, vertices, x and state of the time
    //      node, the volume result of the cell (accumulated into), pressure
    //      modes and pressure rows (registers, scattered after the barrier) ----
    for (int i = tid; i < 4 * N1; i += NTH) ftab[i] = A.tab[lay.Se + i];
    for (int i = tid; i < 2 * RP1 + 2 * NQ; i += NTH) ftab[4 * N1 + i] = A.tab[lay.Le + i];
    if (mapped && tid < (1 << DIM)) {
        int v = tid;
        int o0 = v & 1, o1 = (v >> 1) & 1, o2 = (v >> 2) & 1;
        long long vi = (c0 + o0) + (long long)(A.n0 + 1) * ((c1 + o1) + (long long)(A.n1 + 1) * (c2 + o2));
        for (int k = 0; k < 3; ++k) geo[v * 3 + k] = k < DIM ? T(A.vert[vi * DIM + k]) : T(0);
    }
    // nodal velocity output, starting at the volume result: element
    // e = tid + j * NTH lives in yr[j] of its thread (registers, not LDS, so
    // that 16 of these workgroups fit a CU in FP64)
    T *Ec = E + ((long long)cell * nt + a) * DIM * NL;
    constexpr int YR = (DIM * NL + NTH - 1) / NTH;
    T yr[YR];
#pragma unroll
    for (int j = 0; j < YR; ++j) {
        const int e = tid + j * NTH;
        if (e < DIM * NL) {
            const int l = e % NL, c = e / NL;
            const long long g = a * A.Nv1 + c * A.Nn + gnode(l);
            xs[e] = x[g];
            if constexpr (MODE == Mode::Jac) {
                const T *st = A.state + vec * A.sstride;
                ns[e] = st[g];
            }
            yr[j] = FUSED ? T(0) : Ec[e];
        }
    }
    constexpr int PP = (NPM + NTH - 1) / NTH;
    T px[PP], py[PP];
#pragma unroll
    for (int j = 0; j < PP; ++j) {
        const int e = tid + j * NTH;
        if (e < NPM) {
            const long long gi = pbase + a * A.Np1 + (long long)cell * NPM + e;
            px[j] = x[gi];
            py[j] = FUSED ? T(0) : y[gi];
        }
    }
    for (int e = tid; e < NPF; e += NTH) {
        xpf[e] = 0;
        ypf[e] = 0;
    }
    face_sync<FUSED>();
#pragma unroll
    for (int j = 0; j < PP; ++j) {
        const int e = tid + j * NTH;
        if (e < NPM) {
            const int f = pmode_full<DIM, R>(e);
            xpf[f] = px[j];
            ypf[f] = py[j];
        }
    }
    T *hF = geo + 24;   // |K| / |F| per face id

    // ---- h_F of the boundary faces (reading: |K|/|F| by the cell's quadrature) ----
    {
        if (!mapped) {
            if (tid < 2 * DIM) hF[tid] = hcar[tid / 2];
        } else {
            // volume: fixed-order reduction of det J w over the volume Gauss points
            T part = 0;
            for (int q = tid; q < NQV; q += NTH) {
                int qi[3] = {q % NQ, (q / NQ) % NQ, DIM == 3 ? q / (NQ * NQ) : 0};
                T xi[3] = {0, 0, 0}, Jit[3][3];
                for (int d = 0; d < DIM; ++d) xi[d] = qx[qi[d]];
                T det = geometry<DIM>(true, geo, xi, hcar, Jit);
                T w = det;
                for (int d = 0; d < DIM; ++d) w *= qw[qi[d]];
                part += w;
            }
            t1[tid] = part;
            face_sync<FUSED>();
            if (tid == 0) {
                T vol = 0;
                for (int i = 0; i < NTH; ++i) vol += t1[i];
                geo[30] = vol;
            }
            face_sync<FUSED>();
            // face areas: one face at a time, fixed order
            for (int fid = 0; fid < 2 * DIM; ++fid) {
                int ax = fid / 2, side = fid % 2;
                for (int q = tid; q < NQF; q += NTH) {
                    int tq[2] = {q % NQ, DIM == 3 ? q / NQ : 0};
                    T xi[3] = {0, 0, 0}, Jit[3][3], wt = 1;
                    int t = 0;
                    for (int d = 0; d < DIM; ++d) {
                        if (d == ax) xi[d] = T(side);
                        else { xi[d] = qx[tq[t]]; wt *= qw[tq[t]]; ++t; }
                    }
                    T det = geometry<DIM>(true, geo, xi, hcar, Jit);
                    T len = 0;
                    for (int d = 0; d < DIM; ++d) len += Jit[d][ax] * Jit[d][ax];
                    t2[q] = fabs(det) * sqrt(len) * wt;
                }
                face_sync<FUSED>();
                if (tid == 0) {
                    T area = 0;
                    for (int q = 0; q < NQF; ++q) area += t2[q];
                    hF[fid] = geo[30] / area;
                }
                face_sync<FUSED>();
            }
        }
    }
    face_sync<FUSED>();


    {
        const T wa = A.w[a];
        // ---- boundary faces ----------------------------------------------------------
        {
            {
                // one face; its normal axis and side are compile-time constants
                // so that the strides and index selections of the stages fold
                auto face_one = [&](auto axc, auto sidec) {
                        constexpr int ax = decltype(axc)::value;
                        constexpr int side = decltype(sidec)::value;
                        const int cc = ax == 0 ? c0 : (ax == 1 ? c1 : c2);
                        const int nn = ax == 0 ? A.n0 : (ax == 1 ? A.n1 : A.n2);
                        if (!(side == 0 ? cc == 0 : cc == nn - 1)) return;
                        const int fid = 2 * ax + side;
                        const bool isD = (A.dmask >> fid) & 1u;
                        // face record (each field NQF long):
                        //   inputs : [0,D) xhat, [D, D+D^2) ref grad (c*D+j), [D+D^2, 2D+D^2) v, p
                        //   outputs: value coef (D), ref-grad test coef (D^2), pressure test coef
                        // penalty length: |K|/|F| over the squared velocity degree
                        const T hf = hF[fid] / T((R + 1) * (R + 1));
                        // tangential axes (ta0 < ta1) and strides of the nodal / modal tensors
                        constexpr int ta0 = DIM == 2 ? 1 - ax : (ax == 0 ? 1 : 0);
                        constexpr int ta1 = DIM == 2 ? 0 : (ax == 2 ? 1 : 2);
                        constexpr int sN[3] = {1, N1, N1 * N1}, sP[3] = {1, RP1, RP1 * RP1};
                        const T *Srow = Se + side * N1, *Drow = De + side * N1, *Lrow = Lpe + side * RP1;
                        constexpr int LN = DIM == 3 ? N1 * N1 : N1;      // nodes of a layer
                        constexpr int LP = DIM == 3 ? RP1 * RP1 : RP1;   // modes of a layer
                        T *lay = t1;                                     // [3D fields][LN] + [LP]
                        T *play = lay + 3 * DIM * LN;
                        T *abuf = t2;                                    // 3D: [pipe][j1][q0]
                        T *FQ = Q;
                        constexpr int FV = 0, FG = DIM, FS = DIM + DIM * DIM, FP = 2 * DIM + DIM * DIM;
                        constexpr int FO = 0;   // outputs over the inputs, point by point
                        // 1. reduce along the normal: value layers of xhat and v, normal-derivative
                        //    layers of xhat, value layer of the pressure modes
                        for (int w = tid; w < 3 * DIM * LN + LP; w += NTH) {
                            if (w < 3 * DIM * LN) {
                                const int f = w / LN, it = w - f * LN;
                                const int j0 = DIM == 3 ? it % N1 : it, j1 = DIM == 3 ? it / N1 : 0;
                                const int base = j0 * sN[ta0] + (DIM == 3 ? j1 * sN[ta1] : 0);
                                const int grp = f / DIM, c = f - grp * DIM;
                                const T *src = (grp == 2 && MODE == Mode::Jac ? ns : xs) + c * NL + base;
                                const T *wr = grp == 1 ? Drow : Srow;
                                T s = 0;
#pragma unroll
                                for (int i = 0; i < N1; ++i) s += wr[i] * src[i * sN[ax]];
                                lay[w] = s;
                            } else {
                                const int it = w - 3 * DIM * LN;
                                const int j0 = DIM == 3 ? it % RP1 : it, j1 = DIM == 3 ? it / RP1 : 0;
                                const T *src = xpf + j0 * sP[ta0] + (DIM == 3 ? j1 * sP[ta1] : 0);
                                T s = 0;
#pragma unroll
                                for (int i = 0; i < RP1; ++i) s += Lrow[i] * src[i * sP[ax]];
                                play[it] = s;
                            }
                        }
                        face_sync<FUSED>();
                        // 2. tangential interpolation to the face points q = q0 + NQ q1
                        if constexpr (DIM == 3) {
                            // contract t0: pipes xS (DIM), xD (DIM), nS (DIM), vS (DIM), p; item (pipe, j1)
                            constexpr int NPV = 4 * DIM;
                            for (int w = tid; w < NPV * N1 + RP1; w += NTH) {
                                if (w < NPV * N1) {
                                    const int pipe = w / N1, j1 = w - pipe * N1;
                                    const int grp = pipe / DIM, c = pipe - grp * DIM;
                                    const int lf = grp == 0 || grp == 1 ? c : (grp == 2 ? DIM + c : 2 * DIM + c);
                                    // uniform table pointer per branch (scalar-path loads)
                                    if (grp == 1)
                                        pencil_apply<N1, NQ>(lay + lf * LN + j1 * N1, 1, abuf + pipe * N1 * NQ + j1 * NQ,
                                                             1, D);
                                    else
                                        pencil_apply<N1, NQ>(lay + lf * LN + j1 * N1, 1, abuf + pipe * N1 * NQ + j1 * NQ,
                                                             1, S);
                                } else {
                                    const int j1 = w - NPV * N1;
                                    pencil_apply<RP1, NQ>(play + j1 * RP1, 1, abuf + NPV * N1 * NQ + j1 * NQ, 1, Lp);
                                }
                            }
                            face_sync<FUSED>();
                            // contract t1: item (output field, q0); outputs x (S), g_t1 (D), g_t0, g_ax, v, p
                            constexpr int NOF = 5 * DIM + 1;
                            for (int w = tid; w < NOF * NQ; w += NTH) {
                                const int of = w / NQ, q0 = w - of * NQ;
                                const int grp = of / DIM, c = of - grp * DIM;
                                if (of < 5 * DIM) {
                                    int pipe, dst;
                                    if (grp == 0) { pipe = c; dst = FV + c; }
                                    else if (grp == 1) { pipe = c; dst = FG + c * DIM + ta1; }
                                    else if (grp == 2) { pipe = DIM + c; dst = FG + c * DIM + ta0; }
                                    else if (grp == 3) { pipe = 2 * DIM + c; dst = FG + c * DIM + ax; }
                                    else { pipe = 3 * DIM + c; dst = FS + c; }
                                    if (grp == 1)
                                        pencil_apply<N1, NQ>(abuf + pipe * N1 * NQ + q0, NQ, FQ + dst * NQF + q0, NQ, D);
                                    else
                                        pencil_apply<N1, NQ>(abuf + pipe * N1 * NQ + q0, NQ, FQ + dst * NQF + q0, NQ, S);
                                } else {
                                    pencil_apply<RP1, NQ>(abuf + NPV * N1 * NQ + q0, NQ, FQ + FP * NQF + q0, NQ, Lp);
                                }
                            }
                            face_sync<FUSED>();
                        } else {
                            // one tangential axis: item = output field
                            for (int w = tid; w < 4 * DIM + 1; w += NTH) {
                                const int grp = w / DIM, c = w - grp * DIM;
                                if (w < 4 * DIM) {
                                    int lf, dst;
                                    if (grp == 0) { lf = c; dst = FV + c; }
                                    else if (grp == 1) { lf = c; dst = FG + c * DIM + ta0; }
                                    else if (grp == 2) { lf = DIM + c; dst = FG + c * DIM + ax; }
                                    else { lf = 2 * DIM + c; dst = FS + c; }
                                    if (grp == 1) pencil_apply<N1, NQ>(lay + lf * LN, 1, FQ + dst * NQF, 1, D);
                                    else pencil_apply<N1, NQ>(lay + lf * LN, 1, FQ + dst * NQF, 1, S);
                                } else {
                                    pencil_apply<RP1, NQ>(play, 1, FQ + FP * NQF, 1, Lp);
                                }
                            }
                            face_sync<FUSED>();
                        }
                        // 3. point terms
                        for (int q = tid; q < NQF; q += NTH) {
                            const int tq[2] = {q % NQ, DIM == 3 ? q / NQ : 0};
                            T xi[3] = {0, 0, 0}, Jit[3][3], wt = 1;
                            {
                                int t = 0;
                                for (int d = 0; d < DIM; ++d) {
                                    if (d == ax) xi[d] = T(side);
                                    else { xi[d] = qx[tq[t]]; wt *= qw[tq[t]]; ++t; }
                                }
                            }
                            const T det = geometry<DIM>(mapped, geo, xi, hcar, Jit);
                            const T sg = side ? T(1) : T(-1);
                            T nv[3] = {0, 0, 0}, len = 0;
                            for (int d = 0; d < DIM; ++d) {
                                nv[d] = sg * Jit[d][ax];
                                len += nv[d] * nv[d];
                            }
                            len = sqrt(len);
                            wt *= fabs(det) * len;
                            for (int d = 0; d < DIM; ++d) nv[d] /= len;
                            T xh[3] = {0, 0, 0}, v[3] = {0, 0, 0}, G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                            for (int c = 0; c < DIM; ++c) {
                                xh[c] = FQ[(FV + c) * NQF + q];
                                if constexpr (MODE == Mode::Jac) v[c] = FQ[(FS + c) * NQF + q];
                                else v[c] = xh[c];
                                for (int d = 0; d < DIM; ++d) {
                                    T s = 0;
                                    for (int jd = 0; jd < DIM; ++jd) s += Jit[d][jd] * FQ[(FG + c * DIM + jd) * NQF + q];
                                    G[c][d] = s;
                                }
                            }
                            const T ph = FQ[FP * NQF + q];
                            T vn = 0, xn = 0;
                            for (int d = 0; d < DIM; ++d) {
                                vn += v[d] * nv[d];
                                xn += xh[d] * nv[d];
                            }
                            T val[3] = {0, 0, 0}, gco[3] = {0, 0, 0}, pco = 0;
                            if constexpr (MODE == Mode::Jac) {
                                // <(xv.n) v + (v.n) xv, z>_Gamma
                                for (int c = 0; c < DIM; ++c) val[c] = xn * v[c] + vn * xh[c];
                                if (isD) {
                                    const T om = ominus(vn), dom = dominus(vn);
                                    const T pen1 = A.nu * A.g1 / hf, pen2 = A.g2 / hf;
                                    for (int c = 0; c < DIM; ++c) {
                                        T gn = 0;
                                        for (int d = 0; d < DIM; ++d) gn += G[c][d] * nv[d];
                                        val[c] += -A.nu * gn + ph * nv[c] - dom * xn * v[c] - om * xh[c] +
                                                  pen1 * xh[c] + pen2 * xn * nv[c];
                                        gco[c] = -A.nu * xh[c];
                                    }
                                    pco = xn;
                                }
                            } else {
                                for (int c = 0; c < DIM; ++c) val[c] = vn * v[c];
                                if (isD) {
                                    const T om = ominus(vn);
                                    const T pen1 = A.nu * A.g1 / hf, pen2 = A.g2 / hf;
                                    for (int c = 0; c < DIM; ++c) {
                                        T gn = 0;
                                        for (int d = 0; d < DIM; ++d) gn += G[c][d] * nv[d];
                                        val[c] += -A.nu * gn + ph * nv[c] - om * v[c] + pen1 * v[c] + pen2 * vn * nv[c];
                                        gco[c] = -A.nu * v[c];
                                    }
                                    pco = vn;
                                }
                            }
                            const T sc = wa * wt;
                            for (int c = 0; c < DIM; ++c) FQ[(FO + c) * NQF + q] = sc * val[c];
                            for (int c = 0; c < DIM; ++c)
                                for (int jd = 0; jd < DIM; ++jd) {
                                    T jn = 0;
                                    for (int d = 0; d < DIM; ++d) jn += nv[d] * Jit[d][jd];
                                    FQ[(FO + DIM + c * DIM + jd) * NQF + q] = sc * gco[c] * jn;
                                }
                            FQ[(FO + DIM + DIM * DIM) * NQF + q] = sc * pco;
                        }
                        face_sync<FUSED>();
                        // 4. transposed tangential passes into value / normal-derivative layers
                        //    A_c (value layer: val, tangential gradient coefficients), B_c (normal
                        //    derivative layer: normal gradient coefficient), P (pressure)
                        T *Alay = lay, *Blay = lay + DIM * LN, *Play = lay + 2 * DIM * LN;
                        if constexpr (DIM == 3) {
                            // contract q1: pipes (val S + g_t1 D) (DIM), g_t0 S (DIM), g_ax S (DIM), p Lp;
                            // item (pipe, q0), rows j1
                            constexpr int NPB = 3 * DIM;
                            for (int w = tid; w < (NPB + 1) * NQ; w += NTH) {
                                const int pipe = w / NQ, q0 = w - pipe * NQ;
                                const int grp = pipe / DIM, c = pipe - grp * DIM;
                                T *out = abuf + pipe * N1 * NQ + q0;
                                if (pipe < NPB) {
                                    T u[NQ], g[NQ];
                                    const int fa = grp == 0 ? FO + c : (grp == 1 ? FO + DIM + c * DIM + ta0 : FO + DIM + c * DIM + ax);
#pragma unroll
                                    for (int q1 = 0; q1 < NQ; ++q1) u[q1] = FQ[fa * NQF + q0 + NQ * q1];
                                    if (grp == 0)
#pragma unroll
                                        for (int q1 = 0; q1 < NQ; ++q1) g[q1] = FQ[(FO + DIM + c * DIM + ta1) * NQF + q0 + NQ * q1];
#pragma unroll
                                    for (int j1 = 0; j1 < N1; ++j1) {
                                        T s = 0;
#pragma unroll
                                        for (int q1 = 0; q1 < NQ; ++q1) {
                                            s += S[q1 * N1 + j1] * u[q1];
                                            if (grp == 0) s += D[q1 * N1 + j1] * g[q1];
                                        }
                                        out[j1 * NQ] = s;
                                    }
                                } else {
                                    pencil_apply_t<RP1, NQ>(FQ + (FO + DIM + DIM * DIM) * NQF + q0, NQ, out, NQ, Lp);
                                }
                            }
                            face_sync<FUSED>();
                            // contract q0: item (layer, j1); A_c = S^T(pipe c) + D^T(pipe DIM+c), B_c = S^T(pipe 2DIM+c)
                            for (int w = tid; w < 2 * DIM * N1 + RP1; w += NTH) {
                                if (w < 2 * DIM * N1) {
                                    const int lf = w / N1, j1 = w - lf * N1;
                                    const int grp = lf / DIM, c = lf - grp * DIM;
                                    T *out = (grp == 0 ? Alay : Blay) + c * LN + j1 * N1;
                                    const T *u0 = abuf + (grp == 0 ? c : 2 * DIM + c) * N1 * NQ + j1 * NQ;
                                    const T *u1 = abuf + (DIM + c) * N1 * NQ + j1 * NQ;
                                    T u[NQ], g[NQ];
#pragma unroll
                                    for (int q0 = 0; q0 < NQ; ++q0) {
                                        u[q0] = u0[q0];
                                        g[q0] = grp == 0 ? u1[q0] : T(0);
                                    }
#pragma unroll
                                    for (int j0 = 0; j0 < N1; ++j0) {
                                        T s = 0;
#pragma unroll
                                        for (int q0 = 0; q0 < NQ; ++q0) s += S[q0 * N1 + j0] * u[q0] + D[q0 * N1 + j0] * g[q0];
                                        out[j0] = s;
                                    }
                                } else {
                                    const int j1 = w - 2 * DIM * N1;
                                    pencil_apply_t<RP1, NQ>(abuf + 3 * DIM * N1 * NQ + j1 * NQ, 1, Play + j1 * RP1, 1, Lp);
                                }
                            }
                            face_sync<FUSED>();
                        } else {
                            for (int w = tid; w < 2 * DIM + 1; w += NTH) {
                                const int grp = w / DIM, c = w - grp * DIM;
                                if (w < 2 * DIM) {
                                    T *out = (grp == 0 ? Alay : Blay) + c * LN;
                                    T u[NQ], g[NQ];
                                    const int fa = grp == 0 ? FO + c : FO + DIM + c * DIM + ax;
#pragma unroll
                                    for (int q0 = 0; q0 < NQ; ++q0) {
                                        u[q0] = FQ[fa * NQF + q0];
                                        g[q0] = grp == 0 ? FQ[(FO + DIM + c * DIM + ta0) * NQF + q0] : T(0);
                                    }
#pragma unroll
                                    for (int j0 = 0; j0 < N1; ++j0) {
                                        T s = 0;
#pragma unroll
                                        for (int q0 = 0; q0 < NQ; ++q0) s += S[q0 * N1 + j0] * u[q0] + D[q0 * N1 + j0] * g[q0];
                                        out[j0] = s;
                                    }
                                } else {
                                    pencil_apply_t<RP1, NQ>(FQ + (FO + DIM + DIM * DIM) * NQF, 1, Play, 1, Lp);
                                }
                            }
                            face_sync<FUSED>();
                        }
                        // 5. expansion along the normal into the nodal (registers) and
                        //    modal outputs
#pragma unroll
                        for (int j = 0; j < YR; ++j) {
                            const int w = tid + j * NTH;
                            if (w < DIM * NL) {
                                const int c = w / NL, l = w - c * NL;
                                const int li[3] = {l % N1, (l / N1) % N1, DIM == 3 ? l / (N1 * N1) : 0};
                                const int it = li[ta0] + (DIM == 3 ? N1 * li[ta1] : 0);
                                yr[j] += Srow[li[ax]] * Alay[c * LN + it] + Drow[li[ax]] * Blay[c * LN + it];
                            }
                        }
                        for (int m = tid; m < NPF; m += NTH) {
                            const int mi[3] = {m % RP1, (m / RP1) % RP1, DIM == 3 ? m / (RP1 * RP1) : 0};
                            const int it = mi[ta0] + (DIM == 3 ? RP1 * mi[ta1] : 0);
                            ypf[m] += Lrow[mi[ax]] * Play[it];
                        }
                        face_sync<FUSED>();
                };
                // faces in the fixed order x-, x+, y-, y+, z-, z+
                using I0 = std::integral_constant<int, 0>;
                using I1 = std::integral_constant<int, 1>;
                using I2 = std::integral_constant<int, 2>;
                face_one(I0{}, I0{});
                face_one(I0{}, I1{});
                face_one(I1{}, I0{});
                face_one(I1{}, I1{});
                if constexpr (DIM == 3) {
                    face_one(I2{}, I0{});
                    face_one(I2{}, I1{});
                }
            }
        }

        // ---- volume + boundary results back --------------------------------------------
#pragma unroll
        for (int j = 0; j < YR; ++j) {
            const int e = tid + j * NTH;
            if (e < DIM * NL) {
                if constexpr (FUSED) unsafeAtomicAdd(Ec + e, yr[j]);
                else Ec[e] = yr[j];
            }
        }
        for (int e = tid; e < NPM; e += NTH) {
            const long long gi = pbase + a * A.Np1 + (long long)cell * NPM + e;
            if constexpr (FUSED) unsafeAtomicAdd(y + gi, ypf[pmode_full<DIM, R>(e)]);
            else y[gi] = ypf[pmode_full<DIM, R>(e)];
        }
    }
}

template <int DIM, int R, int NQ, int NTH, typename T, Mode MODE>
__global__ void __launch_bounds__(NTH) face_kernel(CellArgs<T> A)
{
    extern __shared__ unsigned char smem_raw[];
    face_item<DIM, R, NQ, NTH, T, MODE, false>(A, xcd_cell(blockIdx.x, gridDim.x), blockIdx.y,
                                              reinterpret_cast<T *>(smem_raw), threadIdx.x);
}

// ---------------------------------------------------------------------------
// 3D Jacobian, volume and boundary faces in one launch.  Workgroups come in
// groups of eight consecutive blocks (one per XCD); after every `period`
// volume groups comes one face group, whose workgroups give each of their
// NTH / 64 wavefronts one (boundary cell, time node) item with its own LDS
// slice, so face work runs beside the volume work instead of after it.
// Volume groups keep the XCD-contiguous cell order of xcd_cell.  The E
// entries and pressure rows of boundary cells are zeroed before the launch
// (zero_boundary_kernel); both passes add onto them atomically.
// ---------------------------------------------------------------------------
struct FusedGrid {
    int nvg;      // volume groups: ceil(ncell / 8)
    int nfg;      // face groups
    int period;   // volume groups per face group
};

template <int R, int NQ, int NTH, typename T, bool MAPPED>
__global__ void __launch_bounds__(NTH) jac_fused_kernel(CellArgs<T> A, FusedGrid F)
{
    extern __shared__ unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    const int b = blockIdx.x, x = b & 7, g = b >> 3;
    const int p1 = F.period + 1, per = g / p1, pos = g - per * p1;
    if (pos == F.period && per < F.nfg) {
        constexpr int W = NTH / 64;
        const int w = threadIdx.x >> 6;
        const int item = (per * 8 + x) * W + w;
        if (item >= A.nbcell * A.nt) return;   // whole wavefront; face items synchronize per wavefront
        face_item<3, R, NQ, 64, T, Mode::Jac, true>(A, item, blockIdx.y, sm + w * face_lds_words<3, R, NQ, T>(0),
                                                    threadIdx.x & 63);
        return;
    }
    const int vg = g - min(per, F.nfg);
    const int q = A.ncell >> 3, rem = A.ncell & 7;
    if (vg >= q + (x < rem ? 1 : 0)) return;   // whole workgroup
    jac_cell_body<R, NQ, NTH, T, MAPPED, true>(A, x * q + min(x, rem) + vg, blockIdx.y, sm, threadIdx.x);
}

// E entries (3 (r+2)^3 per time node) and pressure rows of the boundary cells,
// all time nodes and vectors, set to zero
template <typename T>
__global__ void __launch_bounds__(256) zero_boundary_kernel(CellArgs<T> A, int nl, int npm)
{
    const int per = 3 * nl + npm;
    const long long n = (long long)A.nbcell * A.nt * per;
    const int vec = blockIdx.y;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const int e = (int)(i % per);
        const long long bsl = i / per;
        const int cell = A.bcells[bsl / A.nt], a = (int)(bsl % A.nt);
        if (e < 3 * nl)
            A.E[(long long)vec * A.ncell * A.nt * 3 * nl + ((long long)cell * A.nt + a) * 3 * nl + e] = T(0);
        else
            A.y[vec * A.ystride + (long long)A.nt * A.Nv1 + a * A.Np1 + (long long)cell * npm + (e - 3 * nl)] = T(0);
    }
}

// ---------------------------------------------------------------------------
// Gather of the cell-local velocity results: y[a][c][node] = sum over the (up
// to 2^d) cells holding the node, in a fixed order; minus rhs if given.
// ---------------------------------------------------------------------------
template <typename T, int DIM, int R>
__global__ void __launch_bounds__(256) gather_kernel(GatherArgs<T> G)
{
    constexpr int R1 = R + 1, NL1 = R + 2, NLOC = DIM == 3 ? NL1 * NL1 * NL1 : NL1 * NL1;
    // node blocks: a contiguous node range per XCD (its L2 holds the cells
    // around those nodes); y = (time node, component), z = right-hand side
    const unsigned nblk = gridDim.x;
    const unsigned node = (unsigned)xcd_cell((int)blockIdx.x, (int)nblk) * blockDim.x + threadIdx.x;
    const unsigned Nn = (unsigned)G.Nn;
    if (node >= Nn) return;
    const int ac = blockIdx.y;                  // a * DIM + c
    const int vec = blockIdx.z;
    const unsigned N0 = (unsigned)(R1 * G.n0 + 1), N1 = (unsigned)(R1 * G.n1 + 1);
    const unsigned t = node / N0;
    const unsigned gg[3] = {node - t * N0, DIM == 3 ? t % N1 : t, DIM == 3 ? t / N1 : 0u};
    const int ncells[3] = {G.n0, G.n1, G.n2};
    // along each axis the node lies in cell c_lo (local index l_lo) and, on an
    // interface between two cells, also in cell c_lo + 1 (local index 0)
    int clo[3], llo[3];
    bool two[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        clo[d] = 0;
        llo[d] = 0;
        two[d] = false;
        if (d < DIM) {
            const int cc = (int)(gg[d] / R1), l = (int)(gg[d] - (unsigned)cc * R1);
            const bool iface = l == 0 && cc > 0;
            clo[d] = iface ? cc - 1 : cc;
            llo[d] = iface ? R1 : l;
            two[d] = iface && cc < ncells[d];
        }
    }
    const long long ncell = (long long)G.n0 * G.n1 * (DIM == 3 ? G.n2 : 1);
    // E[cell][a][c][l]: the (a, c) block of a cell starts at (cell * nt * DIM + ac) * NLOC
    const T *Ev = G.E + (long long)vec * ncell * G.nt * DIM * NLOC + (long long)ac * NLOC;
    const long long cstride = (long long)G.nt * DIM * NLOC;
    // all (up to 2^DIM) loads in flight at once; summed in a fixed order
    // (z outer, x inner; lower cell first), absent cells contributing zero
    constexpr int NC = 1 << DIM;
    T v[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const int j0 = k & 1, j1 = (k >> 1) & 1, j2 = DIM == 3 ? (k >> 2) & 1 : 0;
        const bool ok = (!j0 || two[0]) && (!j1 || two[1]) && (!j2 || two[2]);
        const long long cell = (clo[0] + j0) + (long long)G.n0 * ((clo[1] + j1) + (long long)G.n1 * (clo[2] + j2));
        const int l = (j0 ? 0 : llo[0]) + NL1 * ((j1 ? 0 : llo[1]) + NL1 * (j2 ? 0 : llo[2]));
        v[k] = ok ? Ev[cell * cstride + l] : T(0);
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < NC; ++k) s += v[k];
    const int mult = (two[0] ? 2 : 1) * (two[1] ? 2 : 1) * (two[2] ? 2 : 1);
    const long long idx = (long long)ac * G.Nn + node;
    T *y = G.y + vec * G.ystride;
    if (G.inv_mult) s /= T(mult);
    s *= G.alpha;
    if (G.rhs) s -= G.rhs[idx];
    if (G.accumulate) s += y[idx];
    y[idx] = s;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int DIM, int R, int NQ, typename T, Mode MODE>
static hipError_t launch_face(const CellArgs<T> &a, int nvec, hipStream_t s)
{
    constexpr int NTH = 64;   // one wavefront per (boundary cell, time node)
    if (a.nbcell <= 0) return hipSuccess;
    TableLayout lay;
    lay.init(R, NQ);
    size_t bytes = (size_t)face_lds_words<DIM, R, NQ, T>(lay.total) * sizeof(T);
    auto kern = face_kernel<DIM, R, NQ, NTH, T, MODE>;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    static size_t attr_bytes = 0;
    if (bytes > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        attr_bytes = bytes;
    }
    dim3 grid(a.nbcell * a.nt, nvec);
    hipLaunchKernelGGL(kern, grid, dim3(NTH), bytes, s, a);
    return hipGetLastError();
}

// workgroup size of jac_cell_kernel, measured at 16^3 cells on one MI355X
// (time per launch, 128 vs 256 threads): r = 1, n_q = 4: FP64 28 vs 44 us,
// FP32 19 vs 26; r = 2, n_q = 5: FP64 78 vs 73, FP32 42 vs 46; r = 2,
// n_q = 4: FP64 58 vs 64, FP32 34 vs 40; r = 3, n_q = 7 (k = 1): FP64 231
// vs 150, FP32 106 vs 88.  192 threads: FP64 r = 2, n_q = 5 72 us (at 121
// VGPRs a CU holds five 3-wavefront groups against four of 4 wavefronts, and
// five groups' LDS, 31.6 KB each, still fit in 160 KB); FP32 r = 3 87 us
// against 93 at 256 (130 VGPRs: four groups against three).  FP64 r = 3
// (178 VGPRs, two wavefronts per SIMD) gains nothing from it: 185 us.
template <int R, int NQ, typename T> constexpr int jac_threads()
{
    if (R == 3) return sizeof(T) == 8 ? 256 : 192;
    if (R == 2 && NQ == 5 && sizeof(T) == 8) return 192;
    return 128;
}

template <int R, int NQ, typename T>
static hipError_t launch_jac(const CellArgs<T> &a, int nvec, hipStream_t s)
{
    constexpr int NTH = jac_threads<R, NQ, T>();
    size_t bytes = (size_t)jac_lds_words<R, NQ, T>(a.nt) * sizeof(T);
    auto kern = a.mapped ? jac_cell_kernel<R, NQ, NTH, T, true> : jac_cell_kernel<R, NQ, NTH, T, false>;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    static size_t attr_bytes[2] = {0, 0};   // per kernel (affine, mapped)
    size_t &have = attr_bytes[a.mapped ? 1 : 0];
    static int max_lds = -1;
    if (max_lds < 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            max_lds = 65536;
    }
    if (bytes > (size_t)max_lds) return hipErrorInvalidConfiguration;
    if (bytes > have) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        have = bytes;
    }
    dim3 grid(a.ncell, nvec);
    hipLaunchKernelGGL(kern, grid, dim3(NTH), bytes, s, a);
    return hipGetLastError();
}

// 3D Jacobian with its boundary faces in one launch (after zeroing what both
// passes add to)
template <int R, int NQ, typename T>
static hipError_t launch_jac_fused(const CellArgs<T> &a, int nvec, hipStream_t s)
{
    constexpr int NTH = jac_threads<R, NQ, T>();
    constexpr int W = NTH / 64;
    constexpr int nl = (R + 2) * (R + 2) * (R + 2), npm = Sizes<3, R>::NPM;
    if (a.nbcell > 0) {
        const long long n = (long long)a.nbcell * a.nt * (3 * nl + npm);
        const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
        hipLaunchKernelGGL(zero_boundary_kernel<T>, dim3(blocks, nvec), dim3(256), 0, s, a, nl, npm);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    FusedGrid F;
    F.nvg = (a.ncell + 7) / 8;
    const int fwg = (a.nbcell * a.nt + W - 1) / W;
    F.nfg = (fwg + 7) / 8;
    F.period = F.nfg > 0 ? F.nvg / F.nfg : F.nvg;
    const size_t words = std::max<size_t>(jac_lds_words<R, NQ, T>(a.nt), (size_t)W * face_lds_words<3, R, NQ, T>(0));
    const size_t bytes = words * sizeof(T);
    auto kern = a.mapped ? jac_fused_kernel<R, NQ, NTH, T, true> : jac_fused_kernel<R, NQ, NTH, T, false>;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    static size_t attr_bytes[2] = {0, 0};   // per kernel (affine, mapped)
    size_t &have = attr_bytes[a.mapped ? 1 : 0];
    static int max_lds = -1;
    if (max_lds < 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            max_lds = 65536;
    }
    if (bytes > (size_t)max_lds) return hipErrorInvalidConfiguration;
    if (bytes > have) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        have = bytes;
    }
    dim3 grid(8 * (F.nvg + F.nfg), nvec);
    hipLaunchKernelGGL(kern, grid, dim3(NTH), bytes, s, a, F);
    return hipGetLastError();
}

template <int R, typename T>
static hipError_t dispatch_fused_nq(int nq, const CellArgs<T> &a, int nvec, hipStream_t s)
{
    constexpr int NQD = (3 * R + 5) / 2;
    if (nq == NQD) return launch_jac_fused<R, NQD, T>(a, nvec, s);
    if constexpr (R + 2 != NQD) {
        if (nq == R + 2) return launch_jac_fused<R, R + 2, T>(a, nvec, s);
    }
    return hipErrorInvalidValue;
}

template <int DIM, int R, int NQ, typename T, Mode MODE>
static hipError_t launch_one(const CellArgs<T> &a, int nvec, hipStream_t s)
{
    if constexpr (DIM == 3 && MODE == Mode::Jac) return launch_jac<R, NQ, T>(a, nvec, s);
    constexpr int NTH = DIM == 2 ? 64 : 256;
    TableLayout lay;
    lay.init(R, NQ);
    size_t bytes = (size_t)lds_words<DIM, R, NQ, T, MODE>(a.nt, lay.total) * sizeof(T);
    auto kern = a.mapped ? cell_kernel<DIM, R, NQ, NTH, T, MODE, true> : cell_kernel<DIM, R, NQ, NTH, T, MODE, false>;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    static size_t attr_bytes[2] = {0, 0};   // per kernel (affine, mapped)
    size_t &have = attr_bytes[a.mapped ? 1 : 0];
    static int max_lds = -1;
    if (max_lds < 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            max_lds = 65536;
    }
    if (bytes > (size_t)max_lds) return hipErrorInvalidConfiguration;
    if (bytes > have) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        have = bytes;
    }
    dim3 grid(a.ncell, nvec);
    hipLaunchKernelGGL(kern, grid, dim3(NTH), bytes, s, a);
    return hipGetLastError();
}

template <int DIM, int R, typename T, Mode MODE>
static hipError_t dispatch_nq(int nq, const CellArgs<T> &a, int nvec, hipStream_t s)
{
    constexpr int NQD = (3 * R + 5) / 2;
    if (nq == NQD) return launch_one<DIM, R, NQD, T, MODE>(a, nvec, s);
    if constexpr (R + 2 != NQD) {
        if (nq == R + 2) return launch_one<DIM, R, R + 2, T, MODE>(a, nvec, s);
    }
    return hipErrorInvalidValue;
}

template <int DIM, typename T, Mode MODE>
static hipError_t dispatch_r(int r, int nq, const CellArgs<T> &a, int nvec, hipStream_t s)
{
    switch (r) {
    case 1: return dispatch_nq<DIM, 1, T, MODE>(nq, a, nvec, s);
    case 2: return dispatch_nq<DIM, 2, T, MODE>(nq, a, nvec, s);
    case 3: return dispatch_nq<DIM, 3, T, MODE>(nq, a, nvec, s);
    default: return hipErrorInvalidValue;
    }
}

template <int DIM, typename T, Mode MODE>
static hipError_t dispatch_face(int r, int nq, const CellArgs<T> &a, int nvec, hipStream_t s)
{
    switch (r) {
    case 1:
        if (nq == 4) return launch_face<DIM, 1, 4, T, MODE>(a, nvec, s);
        if (nq == 3) return launch_face<DIM, 1, 3, T, MODE>(a, nvec, s);
        break;
    case 2:
        if (nq == 5) return launch_face<DIM, 2, 5, T, MODE>(a, nvec, s);
        if (nq == 4) return launch_face<DIM, 2, 4, T, MODE>(a, nvec, s);
        break;
    case 3:
        if (nq == 7) return launch_face<DIM, 3, 7, T, MODE>(a, nvec, s);
        if (nq == 5) return launch_face<DIM, 3, 5, T, MODE>(a, nvec, s);
        break;
    default: break;
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_face_op(Mode mode, int dim, int r, int nq, const CellArgs<T> &a, int nvec, hipStream_t s)
{
    if (mode == Mode::Mass) return hipSuccess;
    if (dim == 2) {
        if (mode == Mode::Jac) return dispatch_face<2, T, Mode::Jac>(r, nq, a, nvec, s);
        if constexpr (std::is_same<T, double>::value) return dispatch_face<2, T, Mode::Res>(r, nq, a, nvec, s);
    } else {
        if (mode == Mode::Jac) return dispatch_face<3, T, Mode::Jac>(r, nq, a, nvec, s);
        if constexpr (std::is_same<T, double>::value) return dispatch_face<3, T, Mode::Res>(r, nq, a, nvec, s);
    }
    return hipErrorInvalidValue;
}

// whether the 3D Jacobian runs its boundary faces in the volume launch: in
// FP32 only.  Measured on one MI355X, one Jacobian application at 16^3 cells
// (separate launches vs one launch): r = 2, n_q = 5: FP64 117 vs 138 us (the
// union of both passes needs 133 VGPRs, a workgroup per CU less than the
// volume pass alone), FP32 79 vs 74; n_q = 4: FP64 97 vs 98, FP32 67 vs 62;
// the 32^3 r = 3 slab solve 2.18 s either way.  STMG_JAC_FUSED=0/1 overrides
// the choice (for measurement).
bool jac_fuse_faces(int r, int nq, bool f64)
{
    static const int env = [] {
        const char *e = std::getenv("STMG_JAC_FUSED");
        return e ? std::atoi(e) : -1;
    }();
    if (env == 0 || env == 1) return env == 1;
    (void)r;
    (void)nq;
    return !f64;
}

template <typename T>
hipError_t launch_jac_fused_op(int r, int nq, const CellArgs<T> &a, int nvec, hipStream_t s)
{
    switch (r) {
    case 1: return dispatch_fused_nq<1, T>(nq, a, nvec, s);
    case 2: return dispatch_fused_nq<2, T>(nq, a, nvec, s);
    case 3: return dispatch_fused_nq<3, T>(nq, a, nvec, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_cell_op(Mode mode, int dim, int r, int nq, const CellArgs<T> &a, int nvec, hipStream_t s)
{
    if (dim == 2) {
        if (mode == Mode::Jac) return dispatch_r<2, T, Mode::Jac>(r, nq, a, nvec, s);
        if (mode == Mode::Mass) return dispatch_r<2, T, Mode::Mass>(r, nq, a, nvec, s);
        if constexpr (std::is_same<T, double>::value) return dispatch_r<2, T, Mode::Res>(r, nq, a, nvec, s);
    } else {
        if (mode == Mode::Jac) return dispatch_r<3, T, Mode::Jac>(r, nq, a, nvec, s);
        if (mode == Mode::Mass) return dispatch_r<3, T, Mode::Mass>(r, nq, a, nvec, s);
        if constexpr (std::is_same<T, double>::value) return dispatch_r<3, T, Mode::Res>(r, nq, a, nvec, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, int DIM, int R>
static hipError_t launch_gather_t(const GatherArgs<T> &g, int nvec, hipStream_t s)
{
    const int threads = 256;
    dim3 grid((unsigned)((g.Nn + threads - 1) / threads), (unsigned)(g.nt * DIM), (unsigned)nvec);
    hipLaunchKernelGGL((gather_kernel<T, DIM, R>), grid, dim3(threads), 0, s, g);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const GatherArgs<T> &g, int nvec, hipStream_t s)
{
    // 32-bit node indices inside the kernel
    if (g.Nn <= 0 || g.Nn >= (1LL << 31) || nvec < 1 || nvec > 65535) return hipErrorInvalidValue;
    if (g.nl != (g.dim == 3 ? (g.r + 2) * (g.r + 2) * (g.r + 2) : (g.r + 2) * (g.r + 2))) return hipErrorInvalidValue;
    if (g.dim == 2) {
        switch (g.r) {
        case 1: return launch_gather_t<T, 2, 1>(g, nvec, s);
        case 2: return launch_gather_t<T, 2, 2>(g, nvec, s);
        case 3: return launch_gather_t<T, 2, 3>(g, nvec, s);
        default: break;
        }
    } else if (g.dim == 3) {
        switch (g.r) {
        case 1: return launch_gather_t<T, 3, 1>(g, nvec, s);
        case 2: return launch_gather_t<T, 3, 2>(g, nvec, s);
        case 3: return launch_gather_t<T, 3, 3>(g, nvec, s);
        default: break;
        }
    }
    return hipErrorInvalidValue;
}

template hipError_t launch_face_op<double>(Mode, int, int, int, const CellArgs<double> &, int, hipStream_t);
template hipError_t launch_face_op<float>(Mode, int, int, int, const CellArgs<float> &, int, hipStream_t);
template hipError_t launch_jac_fused_op<double>(int, int, const CellArgs<double> &, int, hipStream_t);
template hipError_t launch_jac_fused_op<float>(int, int, const CellArgs<float> &, int, hipStream_t);
template hipError_t launch_cell_op<double>(Mode, int, int, int, const CellArgs<double> &, int, hipStream_t);
template hipError_t launch_cell_op<float>(Mode, int, int, int, const CellArgs<float> &, int, hipStream_t);
template hipError_t launch_gather<double>(const GatherArgs<double> &, int, hipStream_t);
template hipError_t launch_gather<float>(const GatherArgs<float> &, int, hipStream_t);

} // namespace stmg
