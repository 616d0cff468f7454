// Inexact space-time Vanka smoother on gfx950 (Sec. "Inexact space-time
// Vanka smoother", eq. LVS, eq. DefTildeHn, eq. DefVnAst, eq. vanka0).
//
// Rebuild, once per smoother update:
//   1. elem_kernel      one workgroup per cell: the spatial element matrices
//                       at the midpoint state V* (velocity block of the
//                       linearized A^tp_gamma incl. boundary faces, velocity
//                       mass, velocity-pressure coupling).  The pair (i, j)
//                       x point-chunk loop is a small dense contraction held
//                       in registers (2x2 pairs per thread).
//   2. patch_kernel     one workgroup per cell K: the principal submatrix of
//                       the surrogate on all unknowns of K at all time nodes,
//                       summing the element matrices of every cell that
//                       holds both nodes of an entry, expanded with the time
//                       matrices: K_ab M_S + delta_ab w_a L_S (velocity),
//                       delta_ab w_a B_S^(T) (pressure).  Row-major.
//   3. lu_kernel        one workgroup per patch: blocked right-looking LU
//                       with partial pivoting (row-major, so row interchanges
//                       move contiguous rows); the panel lives in LDS and is
//                       factored with three barriers per column; the trailing
//                       update streams the patch once per panel, on MFMA
//                       (FP32) or register tiles (FP64).
// Apply, per smoothing step:
//   4. solve_kernel     one workgroup per patch: gather the defect, apply the
//                       pivots, blocked forward/backward substitution (64-wide
//                       diagonal blocks inside one wavefront), velocity result
//                       to a cell-local buffer, pressure result added in place
//                       (pressure unknowns belong to a single patch).
//   5. the deterministic node gather of cell_ops adds omega * sum over the
//      patches sharing each velocity node.
#include "stmg_internal.h"
#include "vanka.h"

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <type_traits>
#include <unordered_map>

namespace stmg {

namespace {

constexpr int ipow_(int b, int e) { return e == 0 ? 1 : b * ipow_(b, e - 1); }

typedef float floatx4_t __attribute__((ext_vector_type(4)));
typedef _Float16 halfx4_t __attribute__((ext_vector_type(4)));
typedef short shortx4_t __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (finite inputs; overflow -> inf)
__device__ __forceinline__ short bf16_rne(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// load one stored factor entry as T (unsigned short: BF16 bits, exact widening)
template <typename T, typename TF> __device__ __forceinline__ T ld_factor(const TF *p)
{
    if constexpr (std::is_same<TF, unsigned short>::value) return (T)__uint_as_float((unsigned)(*p) << 16);
    else return (T)(*p);
}
typedef double doublex4_t __attribute__((ext_vector_type(4)));

// 16 x 16 x 4 matrix FMA per precision (v_mfma_f32_16x16x4f32 /
// v_mfma_f64_16x16x4f64).  Operands: A lane l -> (row l%16, k l/16), B lane
// l -> (k l/16, col l%16) in both.  The accumulator differs (measured): lane l
// register i holds (row 4(l/16)+i, col l%16) in FP32 but (row l/16+4i, col
// l%16) in FP64; row(g, i) gives the row for lane group g = l/16.
template <typename T> struct Mfma;
template <> struct Mfma<float> {
    using acc = floatx4_t;
    static __device__ __forceinline__ acc fma(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ constexpr int row(int g, int i) { return 4 * g + i; }
};
template <> struct Mfma<double> {
    using acc = doublex4_t;
    static __device__ __forceinline__ acc fma(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ constexpr int row(int g, int i) { return g + 4 * i; }
};

template <int DIM, int R> struct VS {
    static constexpr int N1 = R + 2;
    static constexpr int NL = ipow_(N1, DIM);
    static constexpr int RP1 = R + 1;
    static constexpr int NPM = DIM == 2 ? (R + 1) * (R + 2) / 2 : (R + 1) * (R + 2) * (R + 3) / 6;
};

template <int DIM, int R> __device__ __forceinline__ void pmode(int m, int al[3])
{
    int cnt = 0;
    for (int a2 = 0; a2 <= (DIM == 3 ? R : 0); ++a2)
        for (int a1 = 0; a1 <= R; ++a1)
            for (int a0 = 0; a0 <= R; ++a0) {
                if (a0 + a1 + a2 > R) continue;
                if (cnt == m) {
                    al[0] = a0;
                    al[1] = a1;
                    al[2] = a2;
                    return;
                }
                ++cnt;
            }
}

template <int DIM, typename T> __device__ __forceinline__ void map_jac_v(const T *X, const T xi[3], T J[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) J[a][b] = 0;
    for (int v = 0; v < (1 << DIM); ++v) {
        T f[3], df[3];
        for (int b = 0; b < DIM; ++b) {
            int o = (v >> b) & 1;
            f[b] = o ? xi[b] : T(1) - xi[b];
            df[b] = o ? T(1) : T(-1);
        }
        for (int b = 0; b < DIM; ++b) {
            T g = df[b];
            for (int e = 0; e < DIM; ++e)
                if (e != b) g *= f[e];
            for (int a = 0; a < DIM; ++a) J[a][b] += X[v * 3 + a] * g;
        }
    }
}

template <int DIM, typename T> __device__ __forceinline__ T inv_t_v(const T J[3][3], T Jit[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Jit[a][b] = 0;
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

template <typename T> __device__ __forceinline__ T om_(T y) { return T(0.5) * (fabs(y) - y); }
template <typename T> __device__ __forceinline__ T dom_(T y) { return y > T(0) ? T(0) : (y < T(0) ? T(-1) : T(-0.5)); }

// ---------------------------------------------------------------------------
// element matrices at the midpoint state
// ---------------------------------------------------------------------------
constexpr int EL_THREADS = 256;
constexpr int PCH = 8;        // points per chunk
constexpr int TILE = 32;      // pair tile (TILE x TILE), 2x2 pairs per thread
constexpr int PREC = 24;      // words of a point record

// point record fields
enum : int {
    P_W = 0, P_V = 1, P_N = 4, P_JIT = 7, P_FACE = 16, P_ISD = 17, P_VN = 18, P_OM = 19, P_DOM = 20, P_PEN1 = 21,
    P_PEN2 = 22
};

// FACE_ONLY: boundary cells only (A.bcells), boundary-face points only, results
// added to the records written by the volume kernel
template <int DIM, int R, int NQ, typename T, bool FACE_ONLY = false>
__global__ void __launch_bounds__(EL_THREADS) elem_kernel(ElemArgs<T> A)
{
    using Z = VS<DIM, R>;
    constexpr int N1 = Z::N1, NL = Z::NL, RP1 = Z::RP1, NPM = Z::NPM;
    constexpr int NQV = ipow_(NQ, DIM), NQF = ipow_(NQ, DIM - 1);
    constexpr int NT = EL_THREADS;
    __shared__ T tabS[NQ * N1], tabD[NQ * N1], tabSe[2 * N1], tabDe[2 * N1], tabL[NQ * RP1], tabLe[2 * RP1];
    __shared__ T qw[NQ], qx[NQ];
    __shared__ T vloc[DIM * NL];
    __shared__ T geo[32];
    // point records: all of them, built once, where they fit (the boundary-face
    // points of a 3D cell in FP32: at most 6 NQF), else one chunk at a time
    constexpr int NPTS_MAX = (FACE_ONLY ? 0 : NQV) + 2 * DIM * NQF;
    constexpr int NPCH_MAX = (NPTS_MAX + PCH - 1) / PCH * PCH;
    constexpr bool PRE = (size_t)NPCH_MAX * (PREC * sizeof(T) + 3 * sizeof(int)) <= 32768;
    constexpr int NREC = PRE ? NPCH_MAX : PCH;
    __shared__ T prec[NREC * PREC];
    __shared__ int pidx[NREC * 3];                // per-axis 1D index (>=0 Gauss, -1 s=0, -2 s=1)
    __shared__ T Bi[PCH * TILE * 4], Bj[PCH * TILE * 4];
    __shared__ T red[NT];
    __shared__ int faces[6];
    __shared__ int nfaces;

    const int tid = threadIdx.x;
    const int cell = FACE_ONLY ? A.bcells[xcd_cell(blockIdx.x, gridDim.x)] : xcd_cell(blockIdx.x, gridDim.x);
    TableLayout lay;
    lay.init(R, NQ);
    for (int i = tid; i < NQ * N1; i += NT) {
        tabS[i] = A.tab[lay.S + i];
        tabD[i] = A.tab[lay.D + i];
    }
    for (int i = tid; i < 2 * N1; i += NT) {
        tabSe[i] = A.tab[lay.Se + i];
        tabDe[i] = A.tab[lay.De + i];
    }
    for (int i = tid; i < NQ * RP1; i += NT) tabL[i] = A.tab[lay.L + i];
    for (int i = tid; i < 2 * RP1; i += NT) tabLe[i] = A.tab[lay.Le + i];
    for (int i = tid; i < NQ; i += NT) {
        qw[i] = A.tab[lay.qw + i];
        qx[i] = A.tab[lay.qx + i];
    }
    const int c0 = cell % A.n0, c1 = (cell / A.n0) % A.n1, c2 = DIM == 3 ? cell / (A.n0 * A.n1) : 0;
    const long long N0 = (long long)(R + 1) * A.n0 + 1, N1g = (long long)(R + 1) * A.n1 + 1;
    for (int e = tid; e < DIM * NL; e += NT) {
        int l = e % NL, c = e / NL;
        int i0 = l % N1, i1 = (l / N1) % N1, i2 = DIM == 3 ? l / (N1 * N1) : 0;
        long long g = ((long long)(R + 1) * c0 + i0) + N0 * (((long long)(R + 1) * c1 + i1) + N1g * ((long long)(R + 1) * c2 + i2));
        vloc[e] = A.vstar[c * A.Nn + g];
    }
    const bool mapped = A.mapped != 0;
    if (mapped && tid < (1 << DIM)) {
        int v = tid, o0 = v & 1, o1 = (v >> 1) & 1, o2 = (v >> 2) & 1;
        long long vi = (c0 + o0) + (long long)(A.n0 + 1) * ((c1 + o1) + (long long)(A.n1 + 1) * (c2 + o2));
        for (int a = 0; a < 3; ++a) geo[v * 3 + a] = a < DIM ? T(A.vert[vi * DIM + a]) : T(0);
    }
    if (tid == 0) {
        int nf = 0;
        int cc[3] = {c0, c1, c2}, nn[3] = {A.n0, A.n1, A.n2};
        for (int ax = 0; ax < DIM; ++ax) {
            if (cc[ax] == 0) faces[nf++] = 2 * ax;
            if (cc[ax] == nn[ax] - 1) faces[nf++] = 2 * ax + 1;
        }
        nfaces = nf;
    }
    __syncthreads();
    const T hcar[3] = {T(1) / A.n0, T(1) / A.n1, DIM == 3 ? T(1) / A.n2 : T(1)};
    T *hF = geo + 24;
    // |K| / |F| (mapped cells by quadrature, fixed-order sums)
    if (nfaces > 0) {
        if (!mapped) {
            if (tid < 2 * DIM) hF[tid] = hcar[tid / 2];
        } else {
            T part = 0;
            for (int q = tid; q < NQV; q += NT) {
                int qi[3] = {q % NQ, (q / NQ) % NQ, DIM == 3 ? q / (NQ * NQ) : 0};
                T xi[3] = {0, 0, 0}, J[3][3], Jit[3][3];
                for (int d = 0; d < DIM; ++d) xi[d] = qx[qi[d]];
                map_jac_v<DIM>(geo, xi, J);
                T w = inv_t_v<DIM>(J, Jit);
                for (int d = 0; d < DIM; ++d) w *= qw[qi[d]];
                part += w;
            }
            red[tid] = part;
            __syncthreads();
            if (tid == 0) {
                T vol = 0;
                for (int i = 0; i < NT; ++i) vol += red[i];
                geo[31] = vol;
            }
            __syncthreads();
            for (int fid = 0; fid < 2 * DIM; ++fid) {
                int ax = fid / 2, side = fid % 2;
                T part2 = 0;
                if (tid < NQF) {
                    int q = tid, tq[2] = {q % NQ, DIM == 3 ? q / NQ : 0}, t = 0;
                    T xi[3] = {0, 0, 0}, J[3][3], Jit[3][3], wt = 1;
                    for (int d = 0; d < DIM; ++d) {
                        if (d == ax) xi[d] = T(side);
                        else { xi[d] = qx[tq[t]]; wt *= qw[tq[t]]; ++t; }
                    }
                    map_jac_v<DIM>(geo, xi, J);
                    T det = inv_t_v<DIM>(J, Jit), len = 0;
                    for (int d = 0; d < DIM; ++d) len += Jit[d][ax] * Jit[d][ax];
                    part2 = fabs(det) * sqrt(len) * wt;
                }
                red[tid] = part2;
                __syncthreads();
                if (tid == 0) {
                    T area = 0;
                    for (int q = 0; q < NQF; ++q) area += red[q];
                    hF[fid] = geo[31] / area;
                }
                __syncthreads();
            }
        }
    }
    __syncthreads();
    const int npts = (FACE_ONLY ? 0 : NQV) + nfaces * NQF;
    const int nchunks = (npts + PCH - 1) / PCH;

    // 1D value / derivative of basis index i on axis value index idx
    auto sv = [&](int idx, int i) -> T { return idx >= 0 ? tabS[idx * N1 + i] : tabSe[(idx == -1 ? 0 : 1) * N1 + i]; };
    auto dv = [&](int idx, int i) -> T { return idx >= 0 ? tabD[idx * N1 + i] : tabDe[(idx == -1 ? 0 : 1) * N1 + i]; };
    auto lv = [&](int idx, int i) -> T { return idx >= 0 ? tabL[idx * RP1 + i] : tabLe[(idx == -1 ? 0 : 1) * RP1 + i]; };

    // point record of point p0 -> P / ix
    auto build_point = [&](int p0, T *P, int *ix) {
        {
            const int p = FACE_ONLY ? p0 + NQV : p0;
            if (p0 >= npts) {
                P[P_W] = 0;
                P[P_FACE] = T(-2);
                ix[0] = ix[1] = ix[2] = 0;
            } else {
                int fid = -1, ax = -1, side = 0;
                if (p < NQV) {
                    ix[0] = p % NQ;
                    ix[1] = DIM > 1 ? (p / NQ) % NQ : 0;
                    ix[2] = DIM == 3 ? p / (NQ * NQ) : 0;
                } else {
                    int f = (p - NQV) / NQF, q = (p - NQV) % NQF;
                    fid = faces[f];
                    ax = fid / 2;
                    side = fid % 2;
                    int tq[2] = {q % NQ, DIM == 3 ? q / NQ : 0}, t = 0;
                    for (int d = 0; d < 3; ++d) ix[d] = 0;
                    for (int d = 0; d < DIM; ++d) ix[d] = (d == ax) ? (side ? -2 : -1) : tq[t++];
                }
                T xi[3] = {0, 0, 0};
                for (int d = 0; d < DIM; ++d) xi[d] = ix[d] >= 0 ? qx[ix[d]] : (ix[d] == -1 ? T(0) : T(1));
                T Jit[3][3], det;
                if (mapped) {
                    T J[3][3];
                    map_jac_v<DIM>(geo, xi, J);
                    det = inv_t_v<DIM>(J, Jit);
                } else {
                    det = 1;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) Jit[a][b] = 0;
                    for (int d = 0; d < DIM; ++d) {
                        Jit[d][d] = T(1) / hcar[d];
                        det *= hcar[d];
                    }
                }
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) P[P_JIT + 3 * a + b] = Jit[a][b];
                // state value
                T v[3] = {0, 0, 0};
                for (int l = 0; l < NL; ++l) {
                    int li[3] = {l % N1, (l / N1) % N1, DIM == 3 ? l / (N1 * N1) : 0};
                    T nv = 1;
                    for (int d = 0; d < DIM; ++d) nv *= sv(ix[d], li[d]);
                    for (int c = 0; c < DIM; ++c) v[c] += vloc[c * NL + l] * nv;
                }
                for (int c = 0; c < 3; ++c) P[P_V + c] = v[c];
                if (fid < 0) {
                    T w = det;
                    for (int d = 0; d < DIM; ++d) w *= qw[ix[d]];
                    P[P_W] = w;
                    P[P_FACE] = T(-1);
                } else {
                    T sg = side ? T(1) : T(-1), nv[3] = {0, 0, 0}, len = 0;
                    for (int d = 0; d < DIM; ++d) {
                        nv[d] = sg * Jit[d][ax];
                        len += nv[d] * nv[d];
                    }
                    len = sqrt(len);
                    T w = fabs(det) * len;
                    for (int d = 0; d < DIM; ++d)
                        if (d != ax) w *= qw[ix[d]];
                    T vn = 0;
                    for (int d = 0; d < DIM; ++d) {
                        nv[d] /= len;
                        vn += v[d] * nv[d];
                    }
                    for (int d = 0; d < 3; ++d) P[P_N + d] = nv[d];
                    P[P_W] = w;
                    P[P_FACE] = T(fid);
                    P[P_ISD] = ((A.dmask >> fid) & 1u) ? T(1) : T(0);
                    P[P_VN] = vn;
                    P[P_OM] = om_(vn);
                    P[P_DOM] = dom_(vn);
                    T h = hF[fid] / T((R + 1) * (R + 1)); // penalty length: over the squared velocity degree
                    P[P_PEN1] = A.nu * A.g1 / h;
                    P[P_PEN2] = A.g2 / h;
                }
            }
        }
    };
    // chunk ch of the point records (threads < PCH), or all at once
    auto build_chunk = [&](int ch) {
        if constexpr (!PRE)
            if (tid < PCH) build_point(ch * PCH + tid, prec + tid * PREC, pidx + tid * 3);
    };
    if constexpr (PRE) {
        for (int p0 = tid; p0 < nchunks * PCH; p0 += NT) build_point(p0, prec + p0 * PREC, pidx + p0 * 3);
        __syncthreads();
    }
    // basis values/gradients of node l at point record p -> B[(p*TILE + slot)*4 ..]
    auto basis = [&](int p, int l, T *out) {
        const int *ix = pidx + p * 3;
        const T *P = prec + p * PREC;
        int li[3] = {l % N1, (l / N1) % N1, DIM == 3 ? l / (N1 * N1) : 0};
        T s[3] = {1, 1, 1}, d[3] = {0, 0, 0};
        for (int a = 0; a < DIM; ++a) {
            s[a] = sv(ix[a], li[a]);
            d[a] = dv(ix[a], li[a]);
        }
        T val = 1, gref[3];
        for (int a = 0; a < DIM; ++a) val *= s[a];
        for (int a = 0; a < DIM; ++a) {
            T g = d[a];
            for (int b = 0; b < DIM; ++b)
                if (b != a) g *= s[b];
            gref[a] = g;
        }
        out[0] = val;
        for (int a = 0; a < DIM; ++a) {
            T g = 0;
            for (int b = 0; b < DIM; ++b) g += P[P_JIT + 3 * a + b] * gref[b];
            out[1 + a] = g;
        }
        if (DIM == 2) out[3] = 0;
    };

    T *rec = A.out + (long long)cell * A.rec_words;
    T *Avv = rec;
    T *Mv = rec + DIM * DIM * NL * NL;
    T *Avp = Mv + NL * NL;
    const T nu = A.nu;
    constexpr int NTILE = (NL + TILE - 1) / TILE;
    const int tx = tid % 16, ty = tid / 16;

    for (int ti = 0; ti < NTILE; ++ti)
        for (int tj = 0; tj < NTILE; ++tj) {
            const int ib = ti * TILE, jb = tj * TILE;
            T acc[2][2][11];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int k = 0; k < 11; ++k) acc[a][b][k] = 0;
            for (int ch = 0; ch < nchunks; ++ch) {
                build_chunk(ch);
                __syncthreads();
                const int cb0 = PRE ? ch * PCH : 0;   // first record of the chunk
                for (int e = tid; e < PCH * TILE; e += NT) {
                    int p = e / TILE, s = e % TILE;
                    T tmp[4];
                    int li = ib + s, lj = jb + s;
                    if (li < NL) basis(cb0 + p, li, tmp);
                    else tmp[0] = tmp[1] = tmp[2] = tmp[3] = 0;
                    for (int k = 0; k < 4; ++k) Bi[(p * TILE + s) * 4 + k] = tmp[k];
                    if (lj < NL) basis(cb0 + p, lj, tmp);
                    else tmp[0] = tmp[1] = tmp[2] = tmp[3] = 0;
                    for (int k = 0; k < 4; ++k) Bj[(p * TILE + s) * 4 + k] = tmp[k];
                }
                __syncthreads();
                for (int p = 0; p < PCH; ++p) {
                    const T *P = prec + (cb0 + p) * PREC;
                    const T w = P[P_W];
                    if (w == T(0)) continue;
                    const T face = P[P_FACE];
                    const T v0 = P[P_V], v1 = P[P_V + 1], v2 = P[P_V + 2];
                    const T vv[3] = {v0, v1, v2};
                    for (int a = 0; a < 2; ++a) {
                        const T *bi = Bi + (p * TILE + ty + 16 * a) * 4;
                        const T Ni = bi[0], Gi[3] = {bi[1], bi[2], bi[3]};
                        for (int b = 0; b < 2; ++b) {
                            const T *bj = Bj + (p * TILE + tx + 16 * b) * 4;
                            const T Nj = bj[0], Gj[3] = {bj[1], bj[2], bj[3]};
                            T *ac = acc[a][b];
                            if (face < T(-0.5)) {
                                // volume: nu grad.grad - Nj (v.grad Ni)  |  -v_c Nj d_e Ni  |  mass
                                T gg = Gi[0] * Gj[0] + Gi[1] * Gj[1] + Gi[2] * Gj[2];
                                T vgi = v0 * Gi[0] + v1 * Gi[1] + v2 * Gi[2];
                                ac[0] += w * (nu * gg - Nj * vgi);
                                T wn = w * Nj;
                                for (int c = 0; c < DIM; ++c)
                                    for (int e2 = 0; e2 < DIM; ++e2) ac[1 + c * 3 + e2] -= wn * vv[c] * Gi[e2];
                                ac[10] += w * Ni * Nj;
                            } else {
                                const T n[3] = {P[P_N], P[P_N + 1], P[P_N + 2]};
                                const T isD = P[P_ISD], vn = P[P_VN];
                                T NN = Ni * Nj;
                                T Gnj = Gj[0] * n[0] + Gj[1] * n[1] + Gj[2] * n[2];
                                T Gni = Gi[0] * n[0] + Gi[1] * n[1] + Gi[2] * n[2];
                                T sc = vn * NN;
                                if (isD != T(0))
                                    sc += -nu * Gnj * Ni - P[P_OM] * NN - nu * Nj * Gni + P[P_PEN1] * NN;
                                ac[0] += w * sc;
                                T f1 = isD != T(0) ? (T(1) - P[P_DOM]) : T(1);
                                T f2 = isD != T(0) ? P[P_PEN2] : T(0);
                                for (int c = 0; c < DIM; ++c)
                                    for (int e2 = 0; e2 < DIM; ++e2)
                                        ac[1 + c * 3 + e2] += w * NN * (n[e2] * vv[c] * f1 + f2 * n[e2] * n[c]);
                            }
                        }
                    }
                }
                __syncthreads();
            }
            for (int a = 0; a < 2; ++a) {
                int i = ib + ty + 16 * a;
                if (i >= NL) continue;
                for (int b = 0; b < 2; ++b) {
                    int j = jb + tx + 16 * b;
                    if (j >= NL) continue;
                    const T *ac = acc[a][b];
                    for (int c = 0; c < DIM; ++c)
                        for (int e2 = 0; e2 < DIM; ++e2) {
                            T val = ac[1 + c * 3 + e2] + (c == e2 ? ac[0] : T(0));
                            if constexpr (FACE_ONLY) Avv[((long long)(c * DIM + e2) * NL + i) * NL + j] += val;
                            else Avv[((long long)(c * DIM + e2) * NL + i) * NL + j] = val;
                        }
                    if constexpr (!FACE_ONLY) Mv[(long long)i * NL + j] = ac[10];
                }
            }
        }

    // velocity-pressure coupling: (c,i) x m
    {
        constexpr int NPAIR = NL * NPM;
        constexpr int PPT = (NPAIR + NT - 1) / NT;
        T acc[PPT][3];
        for (int s = 0; s < PPT; ++s) acc[s][0] = acc[s][1] = acc[s][2] = 0;
        for (int ch = 0; ch < nchunks; ++ch) {
            build_chunk(ch);
            __syncthreads();
            const int cb0 = PRE ? ch * PCH : 0;   // first record of the chunk
            for (int s = 0; s < PPT; ++s) {
                int pr = tid + s * NT;
                if (pr >= NPAIR) break;
                int i = pr / NPM, m = pr % NPM;
                int al[3] = {0, 0, 0};
                pmode<DIM, R>(m, al);
                for (int p = 0; p < PCH; ++p) {
                    const T *P = prec + (cb0 + p) * PREC;
                    T w = P[P_W];
                    if (w == T(0)) continue;
                    const int *ix = pidx + (cb0 + p) * 3;
                    T psi = 1;
                    for (int a = 0; a < DIM; ++a) psi *= lv(ix[a], al[a]);
                    T b[4];
                    basis(cb0 + p, i, b);
                    if (P[P_FACE] < T(-0.5)) {
                        for (int c = 0; c < DIM; ++c) acc[s][c] -= w * psi * b[1 + c];
                    } else if (P[P_ISD] != T(0)) {
                        for (int c = 0; c < DIM; ++c) acc[s][c] += w * psi * P[P_N + c] * b[0];
                    }
                }
            }
            __syncthreads();
        }
        for (int s = 0; s < PPT; ++s) {
            int pr = tid + s * NT;
            if (pr >= NPAIR) break;
            int i = pr / NPM, m = pr % NPM;
            for (int c = 0; c < DIM; ++c) {
                if constexpr (FACE_ONLY) Avp[((long long)c * NL + i) * NPM + m] += acc[s][c];
                else Avp[((long long)c * NL + i) * NPM + m] = acc[s][c];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Volume part of the element matrices of 3D cells on MFMA (FP32 or FP64).  Every entry
// is a contraction over the Gauss points, A_ij = sum_q X_i(q) Y_j(q), with
//   K_ij    = sum_q w (nu grad phi_i . grad phi_j - (v . grad phi_i) phi_j)
//   N^ce_ij = -sum_q w v_c d_e phi_i phi_j
//   M_ij    = sum_q w phi_i phi_j
//   B^c_im  = -sum_q w d_c phi_i psi_m,
// so each 32 x 32 output tile is a set of small GEMMs (16 x 16 x 4 MFMA)
// whose k dimension runs over the points.  Operands are generated per
// chunk of points (16 in FP32, 8 in FP64 to bound the LDS) from the 1D tables and the per-point record (weight, J^{-T},
// state v); wave w owns 16 x 16 subtile w of all eleven blocks (K is added to
// the diagonal component blocks in registers).  Boundary-face terms follow in
// a second kernel over the boundary cells.
// ---------------------------------------------------------------------------
constexpr int EM_THREADS = 256;
template <typename T> constexpr int em_kc() { return sizeof(T) == 8 ? 8 : 16; }   // points per chunk
constexpr int EM_NX = 5, EM_NY = 8;       // X {phi, g0, g1, g2, v.g};  Y {nu w g0..2, -w phi, -w v_c phi, w phi}
constexpr int EM_PR = 13;                 // point record: w, J^{-T} (9), v (3)

template <int R, int NQ, typename T>
__global__ void __launch_bounds__(EM_THREADS) elem_mfma_kernel(ElemArgs<T> A)
{
    constexpr int EM_KC = em_kc<T>();
    using ACC = typename Mfma<T>::acc;
    using Z = VS<3, R>;
    constexpr int N1 = Z::N1, NL = Z::NL, RP1 = Z::RP1, NPM = Z::NPM;
    constexpr int NQV = NQ * NQ * NQ;
    constexpr int NTI = (NL + 31) / 32;
    constexpr int NCH = (NQV + EM_KC - 1) / EM_KC;
    __shared__ T tS[NQ * N1], tD[NQ * N1], tL[NQ * RP1], sqw[NQ], sqx[NQ];
    __shared__ T vloc[3 * NL];
    __shared__ T geo[24];
    __shared__ T prec[NQV * EM_PR];
    __shared__ T Xs[EM_NX][EM_KC][32];
    __shared__ T Ys[EM_NY][EM_KC][32];
    __shared__ int pal[32 * 3];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int cell = xcd_cell(blockIdx.x, gridDim.x);
    TableLayout lay;
    lay.init(R, NQ);
    for (int i = tid; i < NQ * N1; i += EM_THREADS) {
        tS[i] = A.tab[lay.S + i];
        tD[i] = A.tab[lay.D + i];
    }
    for (int i = tid; i < NQ * RP1; i += EM_THREADS) tL[i] = A.tab[lay.L + i];
    for (int i = tid; i < NQ; i += EM_THREADS) {
        sqw[i] = A.tab[lay.qw + i];
        sqx[i] = A.tab[lay.qx + i];
    }
    if (tid < 32) {
        int al[3] = {0, 0, 0};
        if (tid < NPM) pmode<3, R>(tid, al);
        pal[tid * 3] = al[0];
        pal[tid * 3 + 1] = al[1];
        pal[tid * 3 + 2] = al[2];
    }
    const int c0 = cell % A.n0, c1 = (cell / A.n0) % A.n1, c2 = cell / (A.n0 * A.n1);
    const long long N0 = (long long)(R + 1) * A.n0 + 1, N1g = (long long)(R + 1) * A.n1 + 1;
    for (int e = tid; e < 3 * NL; e += EM_THREADS) {
        const int l = e % NL, c = e / NL;
        const int i0 = l % N1, i1 = (l / N1) % N1, i2 = l / (N1 * N1);
        const long long g = ((long long)(R + 1) * c0 + i0) +
                            N0 * (((long long)(R + 1) * c1 + i1) + N1g * ((long long)(R + 1) * c2 + i2));
        vloc[e] = A.vstar[c * A.Nn + g];
    }
    const bool mapped = A.mapped != 0;
    if (mapped && tid < 8) {
        const int v = tid, o0 = v & 1, o1 = (v >> 1) & 1, o2 = (v >> 2) & 1;
        const long long vi = (c0 + o0) + (long long)(A.n0 + 1) * ((c1 + o1) + (long long)(A.n1 + 1) * (c2 + o2));
        for (int a = 0; a < 3; ++a) geo[v * 3 + a] = T(A.vert[vi * 3 + a]);
    }
    __syncthreads();
    // point records
    const T hcar[3] = {T(1) / A.n0, T(1) / A.n1, T(1) / A.n2};
    for (int q = tid; q < NQV; q += EM_THREADS) {
        const int qi[3] = {q % NQ, (q / NQ) % NQ, q / (NQ * NQ)};
        T xi[3], Jit[3][3], det;
        for (int d = 0; d < 3; ++d) xi[d] = sqx[qi[d]];
        if (mapped) {
            T J[3][3];
            map_jac_v<3>(geo, xi, J);
            det = inv_t_v<3>(J, Jit);
        } else {
            det = T(1);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Jit[a][b] = T(0);
            for (int d = 0; d < 3; ++d) {
                Jit[d][d] = T(1) / hcar[d];
                det *= hcar[d];
            }
        }
        T *P = prec + q * EM_PR;
        P[0] = det * sqw[qi[0]] * sqw[qi[1]] * sqw[qi[2]];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) P[1 + 3 * a + b] = Jit[a][b];
        T v[3] = {T(0), T(0), T(0)};
#pragma unroll 1
        for (int l2 = 0; l2 < N1; ++l2) {
            const T s2 = tS[qi[2] * N1 + l2];
#pragma unroll 1
            for (int l1 = 0; l1 < N1; ++l1) {
                const T s12 = s2 * tS[qi[1] * N1 + l1];
                for (int l0 = 0; l0 < N1; ++l0) {
                    const T s = s12 * tS[qi[0] * N1 + l0];
                    const int l = (l2 * N1 + l1) * N1 + l0;
                    for (int c = 0; c < 3; ++c) v[c] += vloc[c * NL + l] * s;
                }
            }
        }
        for (int c = 0; c < 3; ++c) P[10 + c] = v[c];
    }
    __syncthreads();

    // basis value and physical gradient of node l at point q (zero outside)
    auto basis = [&](int q, int l, T &phi, T g[3], const T *&P) {
        phi = T(0);
        g[0] = g[1] = g[2] = T(0);
        P = nullptr;
        if (q >= NQV || l >= NL) return;
        const int qi0 = q % NQ, qi1 = (q / NQ) % NQ, qi2 = q / (NQ * NQ);
        const int l0 = l % N1, l1 = (l / N1) % N1, l2 = l / (N1 * N1);
        const T s0 = tS[qi0 * N1 + l0], s1 = tS[qi1 * N1 + l1], s2 = tS[qi2 * N1 + l2];
        const T d0 = tD[qi0 * N1 + l0], d1 = tD[qi1 * N1 + l1], d2 = tD[qi2 * N1 + l2];
        const T gr[3] = {d0 * s1 * s2, s0 * d1 * s2, s0 * s1 * d2};
        P = prec + q * EM_PR;
        phi = s0 * s1 * s2;
        for (int e = 0; e < 3; ++e) g[e] = P[1 + 3 * e] * gr[0] + P[2 + 3 * e] * gr[1] + P[3 + 3 * e] * gr[2];
    };

    T *Avv = A.out + (long long)cell * A.rec_words;
    T *Mv = Avv + 9 * NL * NL;
    T *Avp = Mv + NL * NL;
    const T nu = A.nu;
    const int si = wv >> 1, sj = wv & 1;
    const int ar = si * 16 + (lane & 15), bc = sj * 16 + (lane & 15), kl = lane >> 4;

    for (int ti = 0; ti < NTI; ++ti)
        for (int tj = 0; tj < NTI; ++tj) {
            ACC acc[11];
            for (int b = 0; b < 11; ++b) acc[b] = ACC{T(0), T(0), T(0), T(0)};
            for (int ch = 0; ch < NCH; ++ch) {
                const int q0 = ch * EM_KC;
#pragma unroll 1
                for (int e = tid; e < 2 * EM_KC * 32; e += EM_THREADS) {
                    const int side = e / (EM_KC * 32), rr = e - side * EM_KC * 32, kq = rr >> 5, col = rr & 31;
                    T phi, g[3];
                    const T *P;
                    basis(q0 + kq, (side ? tj : ti) * 32 + col, phi, g, P);
                    const T w = P ? P[0] : T(0);
                    const T v[3] = {P ? P[10] : T(0), P ? P[11] : T(0), P ? P[12] : T(0)};
                    if (side == 0) {
                        Xs[0][kq][col] = phi;
                        Xs[1][kq][col] = g[0];
                        Xs[2][kq][col] = g[1];
                        Xs[3][kq][col] = g[2];
                        Xs[4][kq][col] = v[0] * g[0] + v[1] * g[1] + v[2] * g[2];
                    } else {
                        Ys[0][kq][col] = nu * w * g[0];
                        Ys[1][kq][col] = nu * w * g[1];
                        Ys[2][kq][col] = nu * w * g[2];
                        Ys[3][kq][col] = -w * phi;
                        Ys[4][kq][col] = -w * v[0] * phi;
                        Ys[5][kq][col] = -w * v[1] * phi;
                        Ys[6][kq][col] = -w * v[2] * phi;
                        Ys[7][kq][col] = w * phi;
                    }
                }
                __syncthreads();
#pragma unroll
                for (int k0 = 0; k0 < EM_KC; k0 += 4) {
                    const int kk = k0 + kl;
                    const T aphi = Xs[0][kk][ar], ag0 = Xs[1][kk][ar], ag1 = Xs[2][kk][ar], ag2 = Xs[3][kk][ar];
                    const T avg = Xs[4][kk][ar];
                    T b[EM_NY];
#pragma unroll
                    for (int t = 0; t < EM_NY; ++t) b[t] = Ys[t][kk][bc];
                    acc[0] = Mfma<T>::fma(ag0, b[0], acc[0]);
                    acc[0] = Mfma<T>::fma(ag1, b[1], acc[0]);
                    acc[0] = Mfma<T>::fma(ag2, b[2], acc[0]);
                    acc[0] = Mfma<T>::fma(avg, b[3], acc[0]);
                    const T ag[3] = {ag0, ag1, ag2};
#pragma unroll
                    for (int c = 0; c < 3; ++c)
#pragma unroll
                        for (int e = 0; e < 3; ++e)
                            acc[1 + 3 * c + e] = Mfma<T>::fma(ag[e], b[4 + c], acc[1 + 3 * c + e]);
                    acc[10] = Mfma<T>::fma(aphi, b[7], acc[10]);
                }
                __syncthreads();
            }
            // accumulator register i of lane l -> (row Mfma::row(l/16, i), col l%16)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = ti * 32 + si * 16 + Mfma<T>::row(kl, i), col = tj * 32 + sj * 16 + (lane & 15);
                if (row < NL && col < NL) {
#pragma unroll
                    for (int c = 0; c < 3; ++c)
#pragma unroll
                        for (int e = 0; e < 3; ++e)
                            Avv[((long long)(c * 3 + e) * NL + row) * NL + col] =
                                acc[1 + 3 * c + e][i] + (c == e ? acc[0][i] : T(0));
                    Mv[(long long)row * NL + col] = acc[10][i];
                }
            }
        }

    // velocity-pressure coupling B^c_im = -sum_q w d_c phi_i psi_m (32 mode columns, NPM valid)
    for (int ti = 0; ti < NTI; ++ti) {
        ACC acc[3];
        for (int c = 0; c < 3; ++c) acc[c] = ACC{T(0), T(0), T(0), T(0)};
        for (int ch = 0; ch < NCH; ++ch) {
            const int q0 = ch * EM_KC;
            for (int e = tid; e < 2 * EM_KC * 32; e += EM_THREADS) {
                const int side = e / (EM_KC * 32), rr = e - side * EM_KC * 32, kq = rr >> 5, col = rr & 31;
                const int q = q0 + kq;
                if (side == 0) {
                    T phi, g[3];
                    const T *P;
                    basis(q, ti * 32 + col, phi, g, P);
                    Xs[1][kq][col] = g[0];
                    Xs[2][kq][col] = g[1];
                    Xs[3][kq][col] = g[2];
                } else {
                    T val = T(0);
                    if (q < NQV && col < NPM) {
                        const int qi0 = q % NQ, qi1 = (q / NQ) % NQ, qi2 = q / (NQ * NQ);
                        val = -prec[q * EM_PR] * tL[qi0 * RP1 + pal[col * 3]] * tL[qi1 * RP1 + pal[col * 3 + 1]] *
                              tL[qi2 * RP1 + pal[col * 3 + 2]];
                    }
                    Ys[0][kq][col] = val;
                }
            }
            __syncthreads();
#pragma unroll
            for (int k0 = 0; k0 < EM_KC; k0 += 4) {
                const int kk = k0 + kl;
                const T bp = Ys[0][kk][bc];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    acc[c] = Mfma<T>::fma(Xs[1 + c][kk][ar], bp, acc[c]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = ti * 32 + si * 16 + Mfma<T>::row(kl, i), m = sj * 16 + (lane & 15);
            if (row < NL && m < NPM)
                for (int c = 0; c < 3; ++c) Avp[((long long)c * NL + row) * NPM + m] = acc[c][i];
        }
    }
}

// ---------------------------------------------------------------------------
// patch assembly (principal submatrix of the surrogate, space-time expansion)
// ---------------------------------------------------------------------------
template <int DIM, int R, typename TE, typename TP>
__global__ void __launch_bounds__(256) patch_kernel(PatchArgs<TE, TP> A)
{
    using Z = VS<DIM, R>;
    constexpr int N1 = Z::N1, NL = Z::NL, NPM = Z::NPM;
    const int cell = A.cell0 >= 0 ? A.cell0 : xcd_cell(blockIdx.x, gridDim.x);
    const int nt = A.nt;
    const int nv = nt * DIM * NL;
    const int m = nv + nt * NPM;
    const int cc[3] = {cell % A.n0, (cell / A.n0) % A.n1, DIM == 3 ? cell / (A.n0 * A.n1) : 0};
    const int nn[3] = {A.n0, A.n1, A.n2};
    TP *out = A.patches + (A.cell0 >= 0 ? 0LL : (long long)cell * m * m);
    const long long rw = A.rec_words;
    for (long long e = threadIdx.x; e < (long long)m * m; e += blockDim.x) {
        int row = (int)(e / m), col = (int)(e % m);
        double val = 0;
        if (row < nv && col < nv) {
            int i = row % NL, c = (row / NL) % DIM, a = row / (NL * DIM);
            int j = col % NL, e2 = (col / NL) % DIM, b = col / (NL * DIM);
            double kab = A.K[a * nt + b];
            bool need_m = (c == e2) && kab != 0.0;
            bool need_l = (a == b);
            if (need_m || need_l) {
                int li[3] = {i % N1, (i / N1) % N1, DIM == 3 ? i / (N1 * N1) : 0};
                int lj[3] = {j % N1, (j / N1) % N1, DIM == 3 ? j / (N1 * N1) : 0};
                // allowed neighbour offsets per axis: both nodes must lie in the neighbour
                int opts[3][3], nopt[3];
                for (int ax = 0; ax < 3; ++ax) {
                    nopt[ax] = 0;
                    opts[ax][nopt[ax]++] = 0;
                    if (ax >= DIM) continue;
                    if (li[ax] == 0 && lj[ax] == 0 && cc[ax] > 0) opts[ax][nopt[ax]++] = -1;
                    if (li[ax] == R + 1 && lj[ax] == R + 1 && cc[ax] < nn[ax] - 1) opts[ax][nopt[ax]++] = 1;
                }
                double ms = 0, ls = 0;
                for (int o2 = 0; o2 < nopt[2]; ++o2)
                    for (int o1 = 0; o1 < nopt[1]; ++o1)
                        for (int o0 = 0; o0 < nopt[0]; ++o0) {
                            int dd[3] = {opts[0][o0], opts[1][o1], opts[2][o2]};
                            long long nb = (cc[0] + dd[0]) + (long long)A.n0 * ((cc[1] + dd[1]) + (long long)A.n1 * (cc[2] + dd[2]));
                            int ip = 0, jp = 0, st = 1;
                            for (int ax = 0; ax < DIM; ++ax) {
                                ip += st * (li[ax] - dd[ax] * (R + 1));
                                jp += st * (lj[ax] - dd[ax] * (R + 1));
                                st *= N1;
                            }
                            const TE *rec = A.elem + nb * rw;
                            if (need_m) ms += (double)rec[DIM * DIM * NL * NL + (long long)ip * NL + jp];
                            if (need_l) ls += (double)rec[((long long)(c * DIM + e2) * NL + ip) * NL + jp];
                        }
                if (need_m) val += kab * ms;
                if (need_l) val += A.w[a] * ls;
            }
        } else if (row < nv && col >= nv) {
            int i = row % NL, c = (row / NL) % DIM, a = row / (NL * DIM);
            int q = col - nv, b = q / NPM, mm = q % NPM;
            if (a == b) {
                const TE *rec = A.elem + (long long)cell * rw + DIM * DIM * NL * NL + NL * NL;
                val = A.w[a] * (double)rec[((long long)c * NL + i) * NPM + mm];
            }
        } else if (row >= nv && col < nv) {
            int j = col % NL, e2 = (col / NL) % DIM, b = col / (NL * DIM);
            int q = row - nv, a = q / NPM, mm = q % NPM;
            if (a == b) {
                const TE *rec = A.elem + (long long)cell * rw + DIM * DIM * NL * NL + NL * NL;
                val = A.w[a] * (double)rec[((long long)e2 * NL + j) * NPM + mm];
            }
        }
        out[(long long)row * m + col] = (TP)val;
    }
}

// ---------------------------------------------------------------------------
// batched blocked LU with partial pivoting, row-major, one workgroup per
// matrix; the matrices of one launch may have different sizes
// ---------------------------------------------------------------------------
constexpr int LU_THREADS = 256;
constexpr int LU_CB = 64;        // column block of the trailing update
constexpr int LU_SWC = 64;       // column chunk of the row interchanges
constexpr int LU_NBO_MIN_M = 192; // larger matrices: outer blocks of LU_CB columns

// outer block width of an m x m factorization with panels of nb columns
// (32-column panels stay on one level: their register arrays leave no room
// for the code of the second level)
__host__ __device__ constexpr int lu_outer_block(int m, int nb) { return m > LU_NBO_MIN_M && nb < 32 ? LU_CB : nb; }
constexpr int LU_CBD = 32;       // column block of the complex once-per-block update
constexpr int LU_C2_ROWS = 4;    // panel rows per thread of lu_kernel_c2 (m <= LU_C2_ROWS LU_THREADS)
// words per plane of the complex U block: the panels' [NB][LU_CB] and the
// outer block's [nbo][LU_CBD]
__host__ __device__ constexpr int lu_c_u_words(int nb, int nbo)
{
    return nb * LU_CB > nbo * LU_CBD ? nb * LU_CB : nbo * LU_CBD;
}


// trailing update A22 -= L21 U12 of one column block, FP32 on MFMA
// (v_mfma_f32_16x16x4f32: A lane l -> (row l%16, k l/16), B lane l ->
// (k l/16, col l%16), D lane l reg i -> (row 4(l/16)+i, col l%16)).
// OP = 1 / 2: the L21 and U12 operands rounded to BF16 / FP16, products
// accumulated in FP32 (v_mfma_f32_16x16x16{bf16,f16}: A lane l -> (row l%16,
// k 4(l/16)+j), B lane l -> (k 4(l/16)+j, col l%16), j < 4; D as above);
// A22 stays FP32
template <int OP, int NTH = LU_THREADS, int PF = 1, typename LOP>
__device__ __forceinline__ void trailing_update(float *A, int r0, int m, int ld, int nb, int cb, int ncb, LOP lop,
                                                const float *ut, int ldu = LU_CB)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nrt = (m - r0 + 31) / 32, nct = (ncb + 31) / 32, ntile = nrt * nct;
    // each wave walks its tiles t = wv, wv + 4, ...; the next tile's C block is
    // loaded before the current one is computed (tiles are disjoint)
    auto load = [&](int t, floatx4_t (&c)[2][2]) {
        const int R = r0 + 32 * (t / nct), C = cb + 32 * (t % nct);
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
            for (int sj = 0; sj < 2; ++sj)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = R + 16 * si + 4 * (lane >> 4) + i, col = C + 16 * sj + (lane & 15);
                    c[si][sj][i] = (row < m && col < cb + ncb) ? A[(long long)row * ld + col] : 0.0f;
                }
    };
    // PF tiles ahead: the C blocks of the next PF tiles of this wave are in
    // flight while the current one is computed
    constexpr int S = NTH / 64;
    floatx4_t acc[2][2], nxt[2][2], nxt2[2][2];
    if (wv < ntile) load(wv, acc);
    if constexpr (PF > 1)
        if (wv + S < ntile) load(wv + S, nxt);
    for (int t = wv; t < ntile; t += S) {
        const int R = r0 + 32 * (t / nct), C = cb + 32 * (t % nct);
        const int tn = t + S;
        if constexpr (PF > 1) {
            if (t + 2 * S < ntile) load(t + 2 * S, nxt2);
        } else {
            if (tn < ntile) load(tn, nxt);
        }
        if constexpr (OP == 0) {
            // L operands of UK k-steps loaded before their products (the
            // once-per-block update reads L from global memory: one latency
            // per UK steps instead of one per step)
            constexpr int UK = 8;
            for (int k0 = 0; k0 < nb; k0 += 4 * UK) {
                float a[UK][2];
#pragma unroll
                for (int u = 0; u < UK; ++u) {
                    const int k = k0 + 4 * u + (lane >> 4);
#pragma unroll
                    for (int si = 0; si < 2; ++si) {
                        const int row = R + 16 * si + (lane & 15);
                        const float v = lop(min(row, m - 1), min(k, nb - 1));
                        a[u][si] = (row < m && k < nb) ? -v : 0.0f;
                    }
                }
#pragma unroll
                for (int u = 0; u < UK; ++u) {
                    const int k = k0 + 4 * u + (lane >> 4), kc = min(k, nb - 1);
                    float b[2];
#pragma unroll
                    for (int sj = 0; sj < 2; ++sj)
                        b[sj] = k < nb ? ut[kc * ldu + (C - cb) + 16 * sj + (lane & 15)] : 0.0f;
#pragma unroll
                    for (int si = 0; si < 2; ++si)
#pragma unroll
                        for (int sj = 0; sj < 2; ++sj)
                            acc[si][sj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][si], b[sj], acc[si][sj], 0, 0, 0);
                }
            }
        } else {
            for (int k0 = 0; k0 < nb; k0 += 16) {
                shortx4_t as[2], bs[2];
                halfx4_t ah[2], bh[2];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = k0 + 4 * (lane >> 4) + j, kc = min(k, nb - 1);
#pragma unroll
                    for (int si = 0; si < 2; ++si) {
                        const int row = R + 16 * si + (lane & 15);
                        const float v = -lop(min(row, m - 1), kc);
                        const float a = (row < m && k < nb) ? v : 0.0f;
                        if constexpr (OP == 1) as[si][j] = bf16_rne(a);
                        else ah[si][j] = (_Float16)a;
                    }
#pragma unroll
                    for (int sj = 0; sj < 2; ++sj) {
                        const float v = ut[kc * ldu + (C - cb) + 16 * sj + (lane & 15)];
                        const float b = k < nb ? v : 0.0f;
                        if constexpr (OP == 1) bs[sj][j] = bf16_rne(b);
                        else bh[sj][j] = (_Float16)b;
                    }
                }
#pragma unroll
                for (int si = 0; si < 2; ++si)
#pragma unroll
                    for (int sj = 0; sj < 2; ++sj) {
                        if constexpr (OP == 1)
                            acc[si][sj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(as[si], bs[sj], acc[si][sj], 0, 0, 0);
                        else
                            acc[si][sj] = __builtin_amdgcn_mfma_f32_16x16x16f16(ah[si], bh[sj], acc[si][sj], 0, 0, 0);
                    }
            }
        }
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
            for (int sj = 0; sj < 2; ++sj)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = R + 16 * si + 4 * (lane >> 4) + i, col = C + 16 * sj + (lane & 15);
                    if (row < m && col < cb + ncb) A[(long long)row * ld + col] = acc[si][sj][i];
                }
        if (tn < ntile) {
#pragma unroll
            for (int si = 0; si < 2; ++si)
#pragma unroll
                for (int sj = 0; sj < 2; ++sj) {
                    acc[si][sj] = nxt[si][sj];
                    if constexpr (PF > 1) nxt[si][sj] = nxt2[si][sj];
                }
        }
    }
}

// FP64 on MFMA (v_mfma_f64_16x16x4f64; operands as in FP32, accumulator lane
// l register i -> (row l/16 + 4i, col l%16)): each wave walks 32 x 32 tiles
// of the column block, the next tile's C block loaded before the current one
// is computed
template <int OP, int NTH = LU_THREADS, int PF = 1, typename LOP>
__device__ __forceinline__ void trailing_update(double *A, int r0, int m, int ld, int nb, int cb, int ncb, LOP lop,
                                                const double *ut, int ldu = LU_CB)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nrt = (m - r0 + 31) / 32, nct = (ncb + 31) / 32, ntile = nrt * nct;
    auto load = [&](int t, doublex4_t (&c)[2][2]) {
        const int R = r0 + 32 * (t / nct), C = cb + 32 * (t % nct);
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
            for (int sj = 0; sj < 2; ++sj)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = R + 16 * si + (lane >> 4) + 4 * i, col = C + 16 * sj + (lane & 15);
                    c[si][sj][i] = (row < m && col < cb + ncb) ? A[(long long)row * ld + col] : 0.0;
                }
    };
    constexpr int S = NTH / 64;
    doublex4_t acc[2][2], nxt[2][2], nxt2[2][2];
    if (wv < ntile) load(wv, acc);
    if constexpr (PF > 1)
        if (wv + S < ntile) load(wv + S, nxt);
    for (int t = wv; t < ntile; t += S) {
        const int R = r0 + 32 * (t / nct), C = cb + 32 * (t % nct);
        const int tn = t + S;
        if constexpr (PF > 1) {
            if (t + 2 * S < ntile) load(t + 2 * S, nxt2);
        } else {
            if (tn < ntile) load(tn, nxt);
        }
        // L operands of UK k-steps loaded before their products (see FP32)
        constexpr int UK = 4;
        for (int k0 = 0; k0 < nb; k0 += 4 * UK) {
            double a[UK][2];
#pragma unroll
            for (int u = 0; u < UK; ++u) {
                const int k = k0 + 4 * u + (lane >> 4);
#pragma unroll
                for (int si = 0; si < 2; ++si) {
                    const int row = R + 16 * si + (lane & 15);
                    const double v = lop(min(row, m - 1), min(k, nb - 1));
                    a[u][si] = (row < m && k < nb) ? -v : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < UK; ++u) {
                const int k = k0 + 4 * u + (lane >> 4), kc = min(k, nb - 1);
                double b[2];
#pragma unroll
                for (int sj = 0; sj < 2; ++sj)
                    b[sj] = k < nb ? ut[kc * ldu + (C - cb) + 16 * sj + (lane & 15)] : 0.0;
#pragma unroll
                for (int si = 0; si < 2; ++si)
#pragma unroll
                    for (int sj = 0; sj < 2; ++sj)
                        acc[si][sj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][si], b[sj], acc[si][sj], 0, 0, 0);
            }
        }
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
            for (int sj = 0; sj < 2; ++sj)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = R + 16 * si + (lane >> 4) + 4 * i, col = C + 16 * sj + (lane & 15);
                    if (row < m && col < cb + ncb) A[(long long)row * ld + col] = acc[si][sj][i];
                }
        if (tn < ntile) {
#pragma unroll
            for (int si = 0; si < 2; ++si)
#pragma unroll
                for (int sj = 0; sj < 2; ++sj) {
                    acc[si][sj] = nxt[si][sj];
                    if constexpr (PF > 1) nxt[si][sj] = nxt2[si][sj];
                }
        }
    }
}

// Composition of the row interchanges of one panel (row c swapped with row
// sw[c], c = 0 .. nb-1, in order) into one permutation of the affected panel
// rows: afterwards row aff_dst[i] holds what was in row aff_src[i].  Run by
// one wavefront: lane i owns entry i (position, content) of the at most 2 nb
// affected rows, lookups by ballot, swaps by shuffles.
template <int NB>
__device__ __forceinline__ void compose_panel_swaps(const int *sw, int nb, int *aff_dst, int *aff_src, int *n_aff)
{
    static_assert(2 * NB <= 64, "affected rows of a panel fit one wavefront");
    const int lane = threadIdx.x & 63;
    int pos = -1, cont = -1, n = 0;
    for (int c = 0; c < nb; ++c) {
        const int p = sw[c];
        if (p == c) continue;
        const unsigned long long mc = __ballot(pos == c), mp = __ballot(pos == p);
        int ic, ip;
        if (mc) {
            ic = __builtin_ctzll(mc);
        } else {
            ic = n++;
            if (lane == ic) pos = cont = c;
        }
        if (mp) {
            ip = __builtin_ctzll(mp);
        } else {
            ip = n++;
            if (lane == ip) pos = cont = p;
        }
        const int vc = __shfl(cont, ic, 64), vp = __shfl(cont, ip, 64);
        if (lane == ic) cont = vp;
        if (lane == ip) cont = vc;
    }
    const bool moved = lane < n && pos != cont;
    const unsigned long long mm = __ballot(moved);
    if (moved) {
        const int k = __popcll(mm & ((1ull << lane) - 1ull));
        aff_dst[k] = pos;
        aff_src[k] = cont;
    }
    if (lane == 0) *n_aff = __popcll(mm);
}

// LU with partial pivoting of one m x m matrix (row stride ld) by the whole
// workgroup with panels of NB columns in LDS (lds_raw: lu_lds_bytes<NB, T>(m)).
// Matrices larger than LU_NBO_MIN_M are blocked on two levels: the panels of
// one outer block of LU_CB columns update only the rest of that block (all
// rows) and the block's own rows; the rows and columns behind the block then
// receive one update with K = LU_CB (L from the factored block columns, U
// staged in LDS), so the trailing matrix crosses HBM once per LU_CB columns
// instead of once per panel.
template <typename T, int NB, int OP, int NTH = LU_THREADS, int PF = 1>
__device__ __forceinline__ void lu_one(T *__restrict__ A, int m, int ld, int *__restrict__ piv, int *info,
                                       unsigned char *lds_raw)
{
    constexpr int NBP = NB + 1;
    const int nbo = lu_outer_block(m, NB);
    T *pan = reinterpret_cast<T *>(lds_raw);          // [m][NBP] panel rows
    T *ut = pan + (size_t)m * NBP;                     // [nbo][LU_CB] U12 block
    T *stg = ut + (size_t)nbo * LU_CB;                 // [2 NB][LU_SWC] row interchange staging
    __shared__ T rv[NTH / 64];
    __shared__ int ri[NTH / 64];
    __shared__ int sw[NB];
    __shared__ int aff_src[2 * NB], aff_dst[2 * NB];
    __shared__ int n_aff;
    __shared__ int bsw[LU_CB];                         // local pivots of the outer block's panels
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    auto from_panel = [&](int j0) { return [=](int row, int k) { return pan[(row - j0) * NBP + k]; }; };
    // interchanges of one panel (local pivots sw[0 .. nb)), composed into one
    // permutation of the affected rows, applied to columns [c_lo, c_hi)
    auto apply_swaps = [&](int j0, int nb, int c_lo, int c_hi) {
        if (wv == 0) compose_panel_swaps<NB>(sw, nb, aff_dst, aff_src, &n_aff);
        __syncthreads();
        const int na = n_aff;
        if (na > 0) {
            if constexpr (NB <= 16) {
                // one column per thread: the column's affected entries to
                // registers, then to their new rows (columns are independent:
                // no staging, no barrier between column chunks)
                for (int col = c_lo + tid; col < c_hi; col += NTH) {
                    T v[2 * NB];
#pragma unroll
                    for (int i = 0; i < 2 * NB; ++i)
                        if (i < na) v[i] = A[(long long)(j0 + aff_src[i]) * ld + col];
#pragma unroll
                    for (int i = 0; i < 2 * NB; ++i)
                        if (i < na) A[(long long)(j0 + aff_dst[i]) * ld + col] = v[i];
                }
                __syncthreads();
            } else {
                for (int c0 = c_lo; c0 < c_hi; c0 += LU_SWC) {
                    const int nc = min(LU_SWC, c_hi - c0);
                    for (int e = tid; e < na * LU_SWC; e += NTH) {
                        int i = e / LU_SWC, j = e % LU_SWC;
                        if (j < nc) stg[i * LU_SWC + j] = A[(long long)(j0 + aff_src[i]) * ld + c0 + j];
                    }
                    __syncthreads();
                    for (int e = tid; e < na * LU_SWC; e += NTH) {
                        int i = e / LU_SWC, j = e % LU_SWC;
                        if (j < nc) A[(long long)(j0 + aff_dst[i]) * ld + c0 + j] = stg[i * LU_SWC + j];
                    }
                    __syncthreads();
                }
            }
        }
    };
    // U12 = L11^{-1} A12 on columns [c_lo, c_hi) of the rows j0 .. j0+nb (L11
    // from the panel rows in LDS), one column block at a time, each followed
    // by A22 -= L21 U12 on the rows [j0+nb, rend)
    auto u12_update = [&](int j0, int nb, int c_lo, int c_hi, int rend) {
        for (int cb = c_lo; cb < c_hi; cb += LU_CB) {
            const int ncb = min(LU_CB, c_hi - cb);
            for (int e = tid; e < NB * LU_CB; e += NTH) ut[e] = T(0);
            __syncthreads();
            if (tid < ncb) {
                const int col = cb + tid;
                T u[NB];
                for (int c = 0; c < NB; ++c) u[c] = c < nb ? A[(long long)(j0 + c) * ld + col] : T(0);
                // fully unrolled (register array); rows c >= nb stay zero
#pragma unroll
                for (int c = 1; c < NB; ++c) {
                    T s = u[c];
#pragma unroll
                    for (int k = 0; k < c; ++k) s -= pan[c * NBP + k] * u[k];
                    if (c < nb) u[c] = s;
                }
                for (int c = 0; c < NB; ++c)
                    if (c < nb) {
                        A[(long long)(j0 + c) * ld + col] = u[c];
                        ut[c * LU_CB + tid] = u[c];
                    }
            }
            __syncthreads();
            trailing_update<OP, NTH, PF>(A, j0 + nb, rend, ld, nb, cb, ncb, from_panel(j0), ut);
            __syncthreads();
        }
    };
    for (int J0 = 0; J0 < m; J0 += nbo) {
      const int jend = min(J0 + nbo, m);             // end of the outer block
      const int cmax = nbo == NB ? m : jend;         // columns the panels of the block touch
      for (int j0 = J0; j0 < jend; j0 += NB) {
        const int nb = min(NB, m - j0), mr = m - j0;
        for (int e = tid; e < mr * nb; e += NTH) {
            int r = e / nb, c = e % nb;
            pan[r * NBP + c] = A[(long long)(j0 + r) * ld + j0 + c];
        }
        __syncthreads();
        for (int c = 0; c < nb; ++c) {
            T best = T(-1);
            int bi = c;
            for (int r = c + tid; r < mr; r += NTH) {
                T v = fabs(pan[r * NBP + c]);
                if (v > best) { best = v; bi = r; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                T ov = __shfl_xor(best, off, 64);
                int oi = __shfl_xor(bi, off, 64);
                if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
            }
            if (lane == 0) { rv[wv] = best; ri[wv] = bi; }
            __syncthreads();
            T bv = rv[0];
            int p = ri[0];
            for (int w = 1; w < NTH / 64; ++w)
                if (rv[w] > bv || (rv[w] == bv && ri[w] < p)) { bv = rv[w]; p = ri[w]; }
            if (tid == 0) {
                piv[j0 + c] = j0 + p;
                sw[c] = p;
                bsw[j0 - J0 + c] = p;
                if (bv == T(0) && info) atomicAdd(info, 1);
            }
            if (p != c && tid < nb) {
                T t = pan[c * NBP + tid];
                pan[c * NBP + tid] = pan[p * NBP + tid];
                pan[p * NBP + tid] = t;
            }
            __syncthreads();
            const T d = pan[c * NBP + c];
            const T inv = d != T(0) ? T(1) / d : T(0);
            for (int r = c + 1 + tid; r < mr; r += NTH) {
                T l = pan[r * NBP + c] * inv;
                pan[r * NBP + c] = l;
                for (int cc = c + 1; cc < nb; ++cc) pan[r * NBP + cc] -= l * pan[c * NBP + cc];
            }
            __syncthreads();
        }
        // the panel's interchanges on the columns it touches (the panel columns
        // themselves are rewritten below)
        apply_swaps(j0, nb, 0, cmax);
        // write the factored panel back
        for (int e = tid; e < mr * nb; e += NTH) {
            int r = e / nb, c = e % nb;
            A[(long long)(j0 + r) * ld + j0 + c] = pan[r * NBP + c];
        }
        __syncthreads();
        u12_update(j0, nb, j0 + nb, cmax, m);
      }
      if constexpr (NB < 32) if (cmax < m) {
        // columns behind the block, untouched so far: the block's interchanges
        // in panel order, then U of the block's rows (blocked forward
        // substitution with the block's L11), then one update of the rows and
        // columns behind the block with K = jend - J0 (L from global memory, U
        // staged in LDS one column block at a time)
        for (int j0 = J0; j0 < jend; j0 += NB) {
            const int nb = min(NB, m - j0);
            if (tid < nb) sw[tid] = bsw[j0 - J0 + tid];
            __syncthreads();
            apply_swaps(j0, nb, jend, m);
        }
        for (int j0 = J0; j0 < jend; j0 += NB) {
            const int nb = min(NB, m - j0), nr = jend - j0;
            for (int e = tid; e < nr * nb; e += NTH) {
                int r = e / nb, c = e % nb;
                pan[r * NBP + c] = A[(long long)(j0 + r) * ld + j0 + c];
            }
            __syncthreads();
            u12_update(j0, nb, jend, m, jend);
        }
        // U staged in the panel and U regions (free here), in column blocks
        // as wide as they hold: every column block reads L once more from
        // global memory
        const int kk = jend - J0;
        const int cbw = max(LU_CB, min((int)(((size_t)m * NBP + (size_t)nbo * LU_CB) / kk) & ~31, (m - jend + 31) & ~31));
        T *uw = pan;
        for (int cb = jend; cb < m; cb += cbw) {
            const int ncb = min(cbw, m - cb);
            for (int e = tid; e < kk * cbw; e += NTH) {
                const int c = e / cbw, j = e - c * cbw;
                uw[e] = j < ncb ? A[(long long)(J0 + c) * ld + cb + j] : T(0);
            }
            __syncthreads();
            trailing_update<OP, NTH, PF>(A, jend, m, ld, kk, cb, ncb,
                                         [=](int row, int k) { return A[(long long)row * ld + J0 + k]; }, uw, cbw);
            __syncthreads();
        }
      }
    }
}


template <typename T, int NB, int OP = 0>
__global__ void __launch_bounds__(LU_THREADS) lu_kernel(T *__restrict__ Aall, int *__restrict__ pivall, LuBatch B,
                                                        int *info)
{
    extern __shared__ unsigned char lds_raw[];
    const int bid = blockIdx.x;
    const int m = B.m_of ? B.m_of[bid] : B.uniform_m;
    const int ld = B.uniform_ld > 0 ? B.uniform_ld : m;   // row stride
    T *A = Aall + (B.a_off ? B.a_off[bid] : (long long)bid * m * ld);
    int *piv = pivall + (B.p_off ? B.p_off[bid] : (long long)bid * m);
    lu_one<T, NB, OP>(A, m, ld, piv, info, lds_raw);
}

// Persistent batched LU of matrices of mixed sizes: a fixed grid of
// workgroups takes matrices from a device work queue (the metadata sorted by
// decreasing size, a counter that starts at zero) until the queue is empty;
// each matrix is factored with the panel width nb_of[i] (16, 8 or 4) chosen
// on the host, whose panel fits the launch's LDS (32-wide panels are left
// out: their register arrays would set the register count, and with it the
// occupancy, of every matrix of the launch).  Every thread of a workgroup reads the
// same queue position, so the whole workgroup leaves the loop together.
template <typename T, int OP, int NTH>
__global__ void __launch_bounds__(NTH) lu_queue_kernel(T *__restrict__ Aall, int *__restrict__ pivall,
                                                              LuQueue Q, int *info)
{
    extern __shared__ unsigned char lds_raw[];
    __shared__ int item;
    for (;;) {
        if (threadIdx.x == 0) item = atomicAdd(Q.counter, 1);
        __syncthreads();
        const int i = item;
        __syncthreads();
        if (i >= Q.batch) break;
        const int m = Q.m_of[i];
        T *A = Aall + Q.a_off[i];
        int *piv = pivall + Q.p_off[i];
        switch (Q.nb_of[i]) {
        case 16: lu_one<T, 16, OP, NTH, 2>(A, m, m, piv, info, lds_raw); break;
        case 8: lu_one<T, 8, OP, NTH, 2>(A, m, m, piv, info, lds_raw); break;
        default: lu_one<T, 4, OP, NTH, 2>(A, m, m, piv, info, lds_raw); break;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// triangular solves with a row-major LU (unit lower L, upper U), rhs b in LDS
// ---------------------------------------------------------------------------
constexpr int SV_THREADS = 256;

// b[r] -= L[r, kb:kb+nbk] . b[kb:kb+nbk] for rows r in [rbeg, rend) of a
// row-major factor with row stride ld (complex planar when CX: Lr/Li and br/bi), nbk <= KB.
// One 16-lane group per row, KB/16 columns per lane; each group keeps RU rows of
// loads in flight before it reduces, so a pass over the rows costs about one
// memory latency instead of one per row.  Per row the summation order is
// fixed: columns l16, l16+16, ..., then a 16-lane xor tree.
template <typename T, bool CX, int KB = 64, int RU = 4, typename TF = T>
__device__ __forceinline__ void block_gemv_update(const TF *__restrict__ Lr, const TF *__restrict__ Li, int ld, int kb,
                                                  int nbk, int rbeg, int rend, T *br, T *bi)
{
    constexpr int NG = SV_THREADS / 16, CPL = KB / 16;   // columns per lane
    const int tid = threadIdx.x, g = tid >> 4, l16 = tid & 15;
    T xr[CPL], xi[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
        const int c = l16 + 16 * i;
        const bool ok = c < nbk;
        xr[i] = ok ? br[kb + c] : T(0);
        xi[i] = CX && ok ? bi[kb + c] : T(0);
    }
#pragma unroll 1
    for (int r0 = rbeg + g; r0 < rend; r0 += RU * NG) {
        T lr[RU][CPL], li[RU][CPL];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            // unconditional loads from a clamped in-range address, then a
            // select: every load of the pass is issued before the first wait
            const int r = r0 + u * NG;
            const long long o = (long long)min(r, rend - 1) * ld + kb;
#pragma unroll
            for (int i = 0; i < CPL; ++i) {
                const int c = l16 + 16 * i;
                const bool ok = r < rend && c < nbk;
                const long long oc = o + min(c, nbk - 1);
                const T vr = ld_factor<T>(Lr + oc);
                lr[u][i] = ok ? vr : T(0);
                if constexpr (CX) {
                    const T vi = ld_factor<T>(Li + oc);
                    li[u][i] = ok ? vi : T(0);
                } else {
                    li[u][i] = T(0);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            T sr = 0, si = 0;
#pragma unroll
            for (int i = 0; i < CPL; ++i) {
                if constexpr (CX) {
                    sr += lr[u][i] * xr[i] - li[u][i] * xi[i];
                    si += lr[u][i] * xi[i] + li[u][i] * xr[i];
                } else {
                    sr += lr[u][i] * xr[i];
                }
            }
            for (int off = 8; off > 0; off >>= 1) {
                sr += __shfl_xor(sr, off, 16);
                if constexpr (CX) si += __shfl_xor(si, off, 16);
            }
            const int r = r0 + u * NG;
            if (l16 == 0 && r < rend) {
                br[r] -= sr;
                if constexpr (CX) bi[r] -= si;
            }
        }
    }
}

template <typename T, int KB = 64, typename TF = T>
__device__ __forceinline__ void lu_substitute(const TF *__restrict__ LU, int m, int ld, T *b, T *dblk)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = tid >> 4, l16 = tid & 15;
    // forward: unit lower
    for (int kb = 0; kb < m; kb += KB) {
        const int nbk = min(KB, m - kb);
        for (int e = tid; e < nbk * KB; e += SV_THREADS) {
            int i = e / KB, j = e % KB;
            if (j < nbk) dblk[i * (KB + 1) + j] = ld_factor<T>(LU + (long long)(kb + i) * ld + kb + j);
        }
        __syncthreads();
        if (wv == 0) {
            T y = lane < nbk ? b[kb + lane] : T(0);
            for (int c = 0; c < nbk; ++c) {
                T yc = __shfl(y, c, 64);
                if (lane > c && lane < nbk) y -= dblk[lane * (KB + 1) + c] * yc;
            }
            if (lane < nbk) b[kb + lane] = y;
        }
        __syncthreads();
        block_gemv_update<T, false, KB, 4, TF>(LU, (const TF *)nullptr, ld, kb, nbk, kb + nbk, m, b, nullptr);
        __syncthreads();
    }
    // backward: upper with diagonal
    const int nblk = (m + KB - 1) / KB;
    for (int bk = nblk - 1; bk >= 0; --bk) {
        const int kb = bk * KB, nbk = min(KB, m - kb);
        for (int e = tid; e < nbk * KB; e += SV_THREADS) {
            int i = e / KB, j = e % KB;
            if (j < nbk) dblk[i * (KB + 1) + j] = ld_factor<T>(LU + (long long)(kb + i) * ld + kb + j);
        }
        __syncthreads();
        if (wv == 0) {
            T x = lane < nbk ? b[kb + lane] : T(0);
            for (int c = nbk - 1; c >= 0; --c) {
                T xc = __shfl(x, c, 64) / dblk[c * (KB + 1) + c];
                if (lane == c) x = xc;
                if (lane < c) x -= dblk[lane * (KB + 1) + c] * xc;
            }
            if (lane < nbk) b[kb + lane] = x;
        }
        __syncthreads();
        block_gemv_update<T, false, KB, 4, TF>(LU, (const TF *)nullptr, ld, kb, nbk, 0, kb, b, nullptr);
        __syncthreads();
    }
}

template <int DIM, int R, typename T, typename TP>
__global__ void __launch_bounds__(SV_THREADS) solve_kernel(SolveArgs<T, TP> A)
{
    using Z = VS<DIM, R>;
    constexpr int N1 = Z::N1, NL = Z::NL, NPM = Z::NPM;
    extern __shared__ unsigned char lds_raw[];
    TP *b = reinterpret_cast<TP *>(lds_raw);
    const int cell = xcd_cell(blockIdx.x, gridDim.x), tid = threadIdx.x;
    const int nt = A.nt, nv = nt * DIM * NL, m = nv + nt * NPM;
    TP *dblk = b + ((m + 1) & ~1);
    const int c0 = cell % A.n0, c1 = (cell / A.n0) % A.n1, c2 = DIM == 3 ? cell / (A.n0 * A.n1) : 0;
    const long long N0 = (long long)(R + 1) * A.n0 + 1, N1g = (long long)(R + 1) * A.n1 + 1;
    auto gnode = [&](int l) -> long long {
        int i0 = l % N1, i1 = (l / N1) % N1, i2 = DIM == 3 ? l / (N1 * N1) : 0;
        return ((long long)(R + 1) * c0 + i0) + N0 * (((long long)(R + 1) * c1 + i1) + N1g * ((long long)(R + 1) * c2 + i2));
    };
    const long long pbase = (long long)nt * A.Nv1;
    for (int row = tid; row < m; row += SV_THREADS) {
        long long g;
        if (row < nv) {
            int l = row % NL, c = (row / NL) % DIM, a = row / (NL * DIM);
            g = a * A.Nv1 + c * A.Nn + gnode(l);
        } else {
            int q = row - nv, a = q / NPM, mm = q % NPM;
            g = pbase + a * A.Np1 + (long long)cell * NPM + mm;
        }
        b[row] = (TP)A.defect[g];
    }
    __syncthreads();
    const int *piv = A.piv + (long long)cell * m;
    if (tid == 0)
        for (int j = 0; j < m; ++j) {
            int p = piv[j];
            if (p != j) {
                TP t = b[j];
                b[j] = b[p];
                b[p] = t;
            }
        }
    __syncthreads();
    lu_substitute<TP>(A.patches + (long long)cell * m * m, m, m, b, dblk);
    // velocity -> cell-local buffer [cell][a][c][l]; pressure += omega * x
    T *Ec = A.E + (long long)cell * nv;
    for (int row = tid; row < m; row += SV_THREADS) {
        if (row < nv) Ec[row] = (T)b[row];
        else {
            int q = row - nv, a = q / NPM, mm = q % NPM;
            long long g = pbase + a * A.Np1 + (long long)cell * NPM + mm;
            A.d[g] += A.omega * (T)b[row];
        }
    }
}

// ---------------------------------------------------------------------------
// Time-decoupled patches.  With the midpoint surrogate the patch matrix is
// K (x) Mhat + W (x) Ahat (one spatial core for all time nodes); after the
// spectral splitting of W^{-1} K every eigenvalue lambda of the splitting
// needs the spatial matrix lambda Mhat + Ahat only: real for a real
// eigenvalue, complex (planar: real plane, then imaginary plane) for a
// conjugate pair.  Spatial patch order: velocity [c][l], then pressure modes.
// ---------------------------------------------------------------------------
template <int DIM, int R, typename TE, typename TP>
__global__ void __launch_bounds__(256) patch_td_kernel(PatchTdArgs<TE, TP> A)
{
    using Z = VS<DIM, R>;
    constexpr int N1 = Z::N1, NL = Z::NL, NPM = Z::NPM;
    constexpr int NV = DIM * NL, MS = NV + NPM;
    constexpr int LDM = td_ld(MS);
    constexpr long long MAT = (long long)MS * LDM;
    const int cell = xcd_cell(blockIdx.x, gridDim.x);
    const int cc[3] = {cell % A.n0, (cell / A.n0) % A.n1, DIM == 3 ? cell / (A.n0 * A.n1) : 0};
    const int nn[3] = {A.n0, A.n1, A.n2};
    const long long rw = A.rec_words;
    const TE *own = A.elem + (long long)cell * rw + DIM * DIM * NL * NL + NL * NL;
    // velocity index -> component, node and the node's per-axis positions,
    // packed (bits 0-3, 4-7, 8-11: positions; 12-19: node; 20-21: component)
    static_assert(N1 <= 16 && NL <= 256, "patch index packing");
    __shared__ int dec[NV];
    for (int t = threadIdx.x; t < NV; t += blockDim.x) {
        const int i = t % NL, c = t / NL;
        dec[t] = (i % N1) | (((i / N1) % N1) << 4) | ((DIM == 3 ? i / (N1 * N1) : 0) << 8) | (i << 12) | (c << 20);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < MS * MS; e += blockDim.x) {
        const int row = e / MS, col = e - (e / MS) * MS;
        double mv = 0, lv = 0;
        if (row < NV && col < NV) {
            const int dr = dec[row], dc = dec[col];
            const int i = (dr >> 12) & 255, c = dr >> 20, j = (dc >> 12) & 255, e2 = dc >> 20;
            const bool need_m = c == e2;
            int li[3] = {dr & 15, (dr >> 4) & 15, (dr >> 8) & 15};
            int lj[3] = {dc & 15, (dc >> 4) & 15, (dc >> 8) & 15};
            // neighbour offsets per axis that hold both nodes
            int opts[3][3], nopt[3];
            for (int ax = 0; ax < 3; ++ax) {
                nopt[ax] = 0;
                opts[ax][nopt[ax]++] = 0;
                if (ax >= DIM) continue;
                if (li[ax] == 0 && lj[ax] == 0 && cc[ax] > 0) opts[ax][nopt[ax]++] = -1;
                if (li[ax] == R + 1 && lj[ax] == R + 1 && cc[ax] < nn[ax] - 1) opts[ax][nopt[ax]++] = 1;
            }
            for (int o2 = 0; o2 < nopt[2]; ++o2)
                for (int o1 = 0; o1 < nopt[1]; ++o1)
                    for (int o0 = 0; o0 < nopt[0]; ++o0) {
                        const int dd[3] = {opts[0][o0], opts[1][o1], opts[2][o2]};
                        const long long nb = (cc[0] + dd[0]) +
                                             (long long)A.n0 * ((cc[1] + dd[1]) + (long long)A.n1 * (cc[2] + dd[2]));
                        int ip = 0, jp = 0, st = 1;
                        for (int ax = 0; ax < DIM; ++ax) {
                            ip += st * (li[ax] - dd[ax] * (R + 1));
                            jp += st * (lj[ax] - dd[ax] * (R + 1));
                            st *= N1;
                        }
                        const TE *rec = A.elem + nb * rw;
                        if (need_m) mv += (double)rec[DIM * DIM * NL * NL + (long long)ip * NL + jp];
                        lv += (double)rec[((long long)(c * DIM + e2) * NL + ip) * NL + jp];
                    }
        } else if (row < NV) {
            lv = (double)own[(long long)row * NPM + (col - NV)];     // row = c * NL + i
        } else if (col < NV) {
            lv = (double)own[(long long)col * NPM + (row - NV)];
        }
        for (int s = 0; s < A.nsys; ++s) {
            TP *o = A.sys[s] + (long long)cell * (A.cplx[s] ? 2 : 1) * MAT + (long long)row * LDM + col;
            o[0] = (TP)(A.lre[s] * mv + lv);
            if (A.cplx[s]) o[MAT] = (TP)(A.lim[s] * mv);
        }
    }
}

// complex trailing update C -= L21 U12 of one column block (planar), FP32 on
// MFMA: four real products per k step
template <int NBP>
__device__ __forceinline__ void trailing_update_c(float *Ar, float *Ai, int m, int ld, int j0, int nb, int cb, int ncb,
                                                  const float *pr, const float *pi, const float *ur, const float *ui)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r0 = j0 + nb;
    const int nrt = (m - r0 + 31) / 32, nct = (ncb + 31) / 32, ntile = nrt * nct;
    // the next tile's C block (both planes) is loaded before the current one
    // is computed (tiles are disjoint)
    auto load = [&](int t, floatx4_t (&xr)[2][2], floatx4_t (&xi)[2][2]) {
        const int R = r0 + 32 * (t / nct), C = cb + 32 * (t % nct);
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
            for (int sj = 0; sj < 2; ++sj)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = R + 16 * si + 4 * (lane >> 4) + i, col = C + 16 * sj + (lane & 15);
                    const bool ok = row < m && col < cb + ncb;
                    xr[si][sj][i] = ok ? Ar[(long long)row * ld + col] : 0.0f;
                    xi[si][sj][i] = ok ? Ai[(long long)row * ld + col] : 0.0f;
                }
    };
    floatx4_t cr[2][2], ci[2][2], nr[2][2], ni[2][2];
    if (wv < ntile) load(wv, cr, ci);
    for (int t = wv; t < ntile; t += LU_THREADS / 64) {
        const int R = r0 + 32 * (t / nct), C = cb + 32 * (t % nct);
        const int tn = t + LU_THREADS / 64;
        if (tn < ntile) load(tn, nr, ni);
        for (int k0 = 0; k0 < nb; k0 += 4) {
            const int k = k0 + (lane >> 4);
            float ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
            for (int si = 0; si < 2; ++si) {
                const int row = R + 16 * si + (lane & 15);
                const bool ok = row < m && k < nb;
                ar[si] = ok ? -pr[(row - j0) * NBP + k] : 0.0f;
                ai[si] = ok ? -pi[(row - j0) * NBP + k] : 0.0f;
                nai[si] = -ai[si];
            }
#pragma unroll
            for (int sj = 0; sj < 2; ++sj) {
                br[sj] = ur[k * LU_CB + (C - cb) + 16 * sj + (lane & 15)];
                bi[sj] = ui[k * LU_CB + (C - cb) + 16 * sj + (lane & 15)];
            }
#pragma unroll
            for (int si = 0; si < 2; ++si)
#pragma unroll
                for (int sj = 0; sj < 2; ++sj) {
                    cr[si][sj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[si], br[sj], cr[si][sj], 0, 0, 0);
                    cr[si][sj] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai[si], bi[sj], cr[si][sj], 0, 0, 0);
                    ci[si][sj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[si], bi[sj], ci[si][sj], 0, 0, 0);
                    ci[si][sj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[si], br[sj], ci[si][sj], 0, 0, 0);
                }
        }
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
            for (int sj = 0; sj < 2; ++sj)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = R + 16 * si + 4 * (lane >> 4) + i, col = C + 16 * sj + (lane & 15);
                    if (row < m && col < cb + ncb) {
                        Ar[(long long)row * ld + col] = cr[si][sj][i];
                        Ai[(long long)row * ld + col] = ci[si][sj][i];
                    }
                }
        if (tn < ntile) {
#pragma unroll
            for (int si = 0; si < 2; ++si)
#pragma unroll
                for (int sj = 0; sj < 2; ++sj) {
                    cr[si][sj] = nr[si][sj];
                    ci[si][sj] = ni[si][sj];
                }
        }
    }
}

// FP64: complex register tiles of 4 x 4 per thread on the vector ALUs
template <int NBP>
__device__ __forceinline__ void trailing_update_c(double *Ar, double *Ai, int m, int ld, int j0, int nb, int cb, int ncb,
                                                  const double *pr, const double *pi, const double *ur,
                                                  const double *ui)
{
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int r0 = j0 + nb;
    for (int R = r0; R < m; R += 64) {
        for (int C = cb; C < cb + ncb; C += 64) {
            double cr[4][4], ci[4][4];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    const int row = R + ty + 16 * i, col = C + tx + 16 * j;
                    const bool ok = row < m && col < cb + ncb;
                    cr[i][j] = ok ? Ar[(long long)row * ld + col] : 0.0;
                    ci[i][j] = ok ? Ai[(long long)row * ld + col] : 0.0;
                }
            for (int k = 0; k < nb; ++k) {
                double ar[4], ai[4], br[4], bi[4];
                for (int i = 0; i < 4; ++i) {
                    const int row = R + ty + 16 * i;
                    ar[i] = row < m ? pr[(row - j0) * NBP + k] : 0.0;
                    ai[i] = row < m ? pi[(row - j0) * NBP + k] : 0.0;
                }
                for (int j = 0; j < 4; ++j) {
                    br[j] = ur[k * LU_CB + (C - cb) + tx + 16 * j];
                    bi[j] = ui[k * LU_CB + (C - cb) + tx + 16 * j];
                }
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) {
                        cr[i][j] -= ar[i] * br[j] - ai[i] * bi[j];
                        ci[i][j] -= ar[i] * bi[j] + ai[i] * br[j];
                    }
            }
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    const int row = R + ty + 16 * i, col = C + tx + 16 * j;
                    if (row < m && col < cb + ncb) {
                        Ar[(long long)row * ld + col] = cr[i][j];
                        Ai[(long long)row * ld + col] = ci[i][j];
                    }
                }
        }
    }
}

// the composed interchanges of one panel (row j0 + aff_src[i] moves to row
// j0 + aff_dst[i], i < na) on columns [c_lo, c_hi), one plane after the
// other: one column per thread, its affected entries through registers
// (columns are independent: no staging and no barrier between column chunks)
template <int NB, typename T>
__device__ __forceinline__ void swap_columns_c(T *Ar, T *Ai, int ld, int j0, int na, const int *aff_src,
                                               const int *aff_dst, int c_lo, int c_hi)
{
#pragma unroll 1
    for (int col = c_lo + (int)threadIdx.x; col < c_hi; col += LU_THREADS)
#pragma unroll 1
        for (int plane = 0; plane < 2; ++plane) {
            // compiler-only barrier: keeps the row indices' LDS reads inside
            // the loop (hoisted, 4 NB row offsets would stay in registers)
            asm volatile("" ::: "memory");
            T *A = plane ? Ai : Ar;
            T v[2 * NB];
#pragma unroll
            for (int i = 0; i < 2 * NB; ++i)
                if (i < na) v[i] = A[(long long)(j0 + aff_src[i]) * ld + col];
#pragma unroll
            for (int i = 0; i < 2 * NB; ++i)
                if (i < na) A[(long long)(j0 + aff_dst[i]) * ld + col] = v[i];
        }
}

// batched blocked complex LU with partial pivoting (largest modulus), planar
// row-major storage: matrix b at Aall + b * a_stride, real plane then
// imaginary plane; same panel / interchange / update structure as the real
// kernel
template <typename T, int NB>
__global__ void __launch_bounds__(LU_THREADS) lu_kernel_c(T *__restrict__ Aall, int *__restrict__ pivall, int m,
                                                          int ld, long long a_stride, int *info)
{
    constexpr int NBP = NB + 1;
    extern __shared__ unsigned char lds_raw[];
    const int bid = blockIdx.x;
    T *Ar = Aall + (long long)bid * a_stride;
    T *Ai = Ar + (long long)m * ld;
    int *piv = pivall + (long long)bid * m;
    T *pr = reinterpret_cast<T *>(lds_raw);           // [m][NBP] panel, real
    T *pi = pr + (size_t)m * NBP;                      // [m][NBP] panel, imaginary
    T *ur = pi + (size_t)m * NBP;                      // [NB][LU_CB] U12 block
    T *ui = ur + (size_t)NB * LU_CB;
    T *stg = ui + (size_t)NB * LU_CB;                  // [2 NB][LU_SWC] interchange staging
    __shared__ T rv[LU_THREADS / 64];
    __shared__ int ri[LU_THREADS / 64];
    __shared__ int sw[NB];
    __shared__ int aff_src[2 * NB], aff_dst[2 * NB];
    __shared__ int n_aff;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int j0 = 0; j0 < m; j0 += NB) {
        const int nb = min(NB, m - j0), mr = m - j0;
        for (int e = tid; e < mr * nb; e += LU_THREADS) {
            const int r = e / nb, c = e % nb;
            const long long g = (long long)(j0 + r) * ld + j0 + c;
            pr[r * NBP + c] = Ar[g];
            pi[r * NBP + c] = Ai[g];
        }
        __syncthreads();
        for (int c = 0; c < nb; ++c) {
            T best = T(-1);
            int bi = c;
            for (int r = c + tid; r < mr; r += LU_THREADS) {
                const T x = pr[r * NBP + c], y = pi[r * NBP + c];
                const T v = x * x + y * y;
                if (v > best) { best = v; bi = r; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                T ov = __shfl_xor(best, off, 64);
                int oi = __shfl_xor(bi, off, 64);
                if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
            }
            if (lane == 0) { rv[wv] = best; ri[wv] = bi; }
            __syncthreads();
            T bv = rv[0];
            int p = ri[0];
            for (int w = 1; w < LU_THREADS / 64; ++w)
                if (rv[w] > bv || (rv[w] == bv && ri[w] < p)) { bv = rv[w]; p = ri[w]; }
            if (tid == 0) {
                piv[j0 + c] = j0 + p;
                sw[c] = p;
                if (bv == T(0) && info) atomicAdd(info, 1);
            }
            if (p != c && tid < nb) {
                T t = pr[c * NBP + tid];
                pr[c * NBP + tid] = pr[p * NBP + tid];
                pr[p * NBP + tid] = t;
                t = pi[c * NBP + tid];
                pi[c * NBP + tid] = pi[p * NBP + tid];
                pi[p * NBP + tid] = t;
            }
            __syncthreads();
            const T dr = pr[c * NBP + c], di = pi[c * NBP + c];
            const T den = dr * dr + di * di;
            const T ir = den != T(0) ? dr / den : T(0), ii = den != T(0) ? -di / den : T(0);
            for (int r = c + 1 + tid; r < mr; r += LU_THREADS) {
                const T xr = pr[r * NBP + c], xi = pi[r * NBP + c];
                const T lr = xr * ir - xi * ii, li = xr * ii + xi * ir;
                pr[r * NBP + c] = lr;
                pi[r * NBP + c] = li;
                for (int cc = c + 1; cc < nb; ++cc) {
                    const T vr = pr[c * NBP + cc], vi = pi[c * NBP + cc];
                    pr[r * NBP + cc] -= lr * vr - li * vi;
                    pi[r * NBP + cc] -= lr * vi + li * vr;
                }
            }
            __syncthreads();
        }
        if (wv == 0) compose_panel_swaps<NB>(sw, nb, aff_dst, aff_src, &n_aff);
        __syncthreads();
        const int na = n_aff;
        if constexpr (NB <= 16) {
            if (na > 0) {
                swap_columns_c<NB>(Ar, Ai, ld, j0, na, aff_src, aff_dst, 0, m);
                __syncthreads();
            }
        } else if (na > 0) {
            for (int plane = 0; plane < 2; ++plane) {
                T *A = plane ? Ai : Ar;
                for (int c0 = 0; c0 < m; c0 += LU_SWC) {
                    const int nc = min(LU_SWC, m - c0);
                    for (int e = tid; e < na * LU_SWC; e += LU_THREADS) {
                        const int i = e / LU_SWC, j = e % LU_SWC;
                        if (j < nc) stg[i * LU_SWC + j] = A[(long long)(j0 + aff_src[i]) * ld + c0 + j];
                    }
                    __syncthreads();
                    for (int e = tid; e < na * LU_SWC; e += LU_THREADS) {
                        const int i = e / LU_SWC, j = e % LU_SWC;
                        if (j < nc) A[(long long)(j0 + aff_dst[i]) * ld + c0 + j] = stg[i * LU_SWC + j];
                    }
                    __syncthreads();
                }
            }
        }
        for (int e = tid; e < mr * nb; e += LU_THREADS) {
            const int r = e / nb, c = e % nb;
            const long long g = (long long)(j0 + r) * ld + j0 + c;
            Ar[g] = pr[r * NBP + c];
            Ai[g] = pi[r * NBP + c];
        }
        __syncthreads();
        // U12 = L11^{-1} A12 for every column right of the panel at once (one
        // thread per column, all waves), written back to A; each trailing
        // update then takes its U12 block from there
#pragma unroll 1
        for (int col = j0 + nb + tid; col < m; col += LU_THREADS) {
            // compiler-only barrier: keeps the L11 reads from LDS inside the
            // loop (hoisted, they would hold NB(NB-1) values in registers)
            asm volatile("" ::: "memory");
            T vr[NB], vi[NB];
            for (int c = 0; c < NB; ++c) {
                const bool ok = c < nb;
                vr[c] = ok ? Ar[(long long)(j0 + c) * ld + col] : T(0);
                vi[c] = ok ? Ai[(long long)(j0 + c) * ld + col] : T(0);
            }
            // fully unrolled (register arrays); rows c >= nb stay zero
#pragma unroll
            for (int c = 1; c < NB; ++c) {
                T sr = vr[c], si = vi[c];
#pragma unroll
                for (int k = 0; k < c; ++k) {
                    const T lr = pr[c * NBP + k], li = pi[c * NBP + k];
                    sr -= lr * vr[k] - li * vi[k];
                    si -= lr * vi[k] + li * vr[k];
                }
                if (c < nb) {
                    vr[c] = sr;
                    vi[c] = si;
                }
            }
            for (int c = 0; c < NB; ++c)
                if (c < nb) {
                    Ar[(long long)(j0 + c) * ld + col] = vr[c];
                    Ai[(long long)(j0 + c) * ld + col] = vi[c];
                }
        }
        __syncthreads();
        for (int cb = j0 + nb; cb < m; cb += LU_CB) {
            const int ncb = min(LU_CB, m - cb);
            for (int e = tid; e < NB * LU_CB; e += LU_THREADS) {
                const int c = e / LU_CB, j = e % LU_CB;
                const bool ok = c < nb && j < ncb;
                const long long g = (long long)(j0 + min(c, nb - 1)) * ld + cb + min(j, ncb - 1);
                const T a = Ar[g], b = Ai[g];
                ur[e] = ok ? a : T(0);
                ui[e] = ok ? b : T(0);
            }
            __syncthreads();
            trailing_update_c<NBP>(Ar, Ai, m, ld, j0, nb, cb, ncb, pr, pi, ur, ui);
            __syncthreads();
        }
    }
}

// complex trailing update C -= L21 U12 of one column block (planar), FP32 on
// MFMA, for the second blocking level: rows [r0, m), K = nb, L21 from an
// accessor (the LDS panel or global memory), U12 from LDS with row stride ldu
template <typename LOP>
__device__ __forceinline__ void trailing_update_cg(float *Ar, float *Ai, int r0, int m, int ld, int nb, int cb, int ncb,
                                                  LOP lop, const float *ur, const float *ui, int ldu)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nrt = (m - r0 + 31) / 32, nct = (ncb + 31) / 32, ntile = nrt * nct;
    // the next tile's C block (both planes) is loaded before the current one
    // is computed (tiles are disjoint)
    auto load = [&](int t, floatx4_t (&xr)[2][2], floatx4_t (&xi)[2][2]) {
        const int R = r0 + 32 * (t / nct), C = cb + 32 * (t % nct);
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
            for (int sj = 0; sj < 2; ++sj)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = R + 16 * si + 4 * (lane >> 4) + i, col = C + 16 * sj + (lane & 15);
                    const bool ok = row < m && col < cb + ncb;
                    xr[si][sj][i] = ok ? Ar[(long long)row * ld + col] : 0.0f;
                    xi[si][sj][i] = ok ? Ai[(long long)row * ld + col] : 0.0f;
                }
    };
    floatx4_t cr[2][2], ci[2][2], nr[2][2], ni[2][2];
    if (wv < ntile) load(wv, cr, ci);
    for (int t = wv; t < ntile; t += LU_THREADS / 64) {
        const int R = r0 + 32 * (t / nct), C = cb + 32 * (t % nct);
        const int tn = t + LU_THREADS / 64;
        if (tn < ntile) load(tn, nr, ni);
        // L operands of UK k-steps loaded before their products (the L of
        // the once-per-block update comes from global memory)
        constexpr int UK = 4;
        for (int k0 = 0; k0 < nb; k0 += 4 * UK) {
            float ar[UK][2], ai[UK][2];
#pragma unroll
            for (int u = 0; u < UK; ++u) {
                const int k = k0 + 4 * u + (lane >> 4);
#pragma unroll
                for (int si = 0; si < 2; ++si) {
                    const int row = R + 16 * si + (lane & 15);
                    const bool ok = row < m && k < nb;
                    float lr, li;
                    lop(min(row, m - 1), min(k, nb - 1), lr, li);
                    ar[u][si] = ok ? -lr : 0.0f;
                    ai[u][si] = ok ? -li : 0.0f;
                }
            }
#pragma unroll
            for (int u = 0; u < UK; ++u) {
                const int k = k0 + 4 * u + (lane >> 4), kc = min(k, nb - 1);
                float br[2], bi[2];
#pragma unroll
                for (int sj = 0; sj < 2; ++sj) {
                    const int col = (C - cb) + 16 * sj + (lane & 15);
                    br[sj] = k < nb ? ur[kc * ldu + col] : 0.0f;
                    bi[sj] = k < nb ? ui[kc * ldu + col] : 0.0f;
                }
#pragma unroll
                for (int si = 0; si < 2; ++si)
#pragma unroll
                    for (int sj = 0; sj < 2; ++sj) {
                        cr[si][sj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[u][si], br[sj], cr[si][sj], 0, 0, 0);
                        cr[si][sj] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[u][si], bi[sj], cr[si][sj], 0, 0, 0);
                        ci[si][sj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[u][si], bi[sj], ci[si][sj], 0, 0, 0);
                        ci[si][sj] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[u][si], br[sj], ci[si][sj], 0, 0, 0);
                    }
            }
        }
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
            for (int sj = 0; sj < 2; ++sj)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = R + 16 * si + 4 * (lane >> 4) + i, col = C + 16 * sj + (lane & 15);
                    if (row < m && col < cb + ncb) {
                        Ar[(long long)row * ld + col] = cr[si][sj][i];
                        Ai[(long long)row * ld + col] = ci[si][sj][i];
                    }
                }
        if (tn < ntile) {
#pragma unroll
            for (int si = 0; si < 2; ++si)
#pragma unroll
                for (int sj = 0; sj < 2; ++sj) {
                    cr[si][sj] = nr[si][sj];
                    ci[si][sj] = ni[si][sj];
                }
        }
    }
}

// FP32 complex LU on two levels (matrices larger than LU_NBO_MIN_M): the
// panels of an outer block of LU_CB columns touch only the block's columns;
// then the block's interchanges, U of its rows (blocked forward substitution)
// and one update of the rows and columns behind it with K = LU_CB (LU_CBD
// columns at a time), as in lu_one.  Storage as in lu_kernel_c.
template <typename T, int NB>
__global__ void __launch_bounds__(LU_THREADS) lu_kernel_c2(T *__restrict__ Aall, int *__restrict__ pivall, int m,
                                                          int ld, long long a_stride, int *info)
{
    constexpr int NBP = NB + 1;
    extern __shared__ unsigned char lds_raw[];
    const int bid = blockIdx.x;
    T *Ar = Aall + (long long)bid * a_stride;
    T *Ai = Ar + (long long)m * ld;
    int *piv = pivall + (long long)bid * m;
    static_assert(NB < 32 && sizeof(T) == 4, "two-level complex LU: FP32, panels under 32 columns");
    constexpr int nbo = LU_CB;
    constexpr int ubw = lu_c_u_words(NB, nbo);
    T *pr = reinterpret_cast<T *>(lds_raw);           // [m][NBP] panel, real
    T *pi = pr + (size_t)m * NBP;                      // [m][NBP] panel, imaginary
    T *ur = pi + (size_t)m * NBP;                      // U block: [NB][LU_CB] or [nbo][LU_CBD]
    T *ui = ur + (size_t)ubw;
    int *pa = reinterpret_cast<int *>(ui + ubw);     // [m] panel row holding each logical row
    __shared__ T rv[2][LU_THREADS / 64];               // pivot candidates per wave, by column parity
    __shared__ int rl[2][LU_THREADS / 64], rp[2][LU_THREADS / 64];
    __shared__ int sw[NB];
    __shared__ int aff_src[2 * NB], aff_dst[2 * NB];
    __shared__ int n_aff;
    __shared__ int bsw[LU_CB];                         // local pivots of the outer block's panels
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    auto from_panel = [&](int j0) {
        return [=](int row, int k, T &lr, T &li) {
            const int o = pa[row - j0] * NBP + k;
            lr = pr[o];
            li = pi[o];
        };
    };
    // interchanges of one panel (local pivots sw[0 .. nb)) on columns [c_lo, c_hi), both planes
    auto apply_swaps = [&](int j0, int nb, int c_lo, int c_hi) {
        if (wv == 0) compose_panel_swaps<NB>(sw, nb, aff_dst, aff_src, &n_aff);
        __syncthreads();
        const int na = n_aff;
        if (na > 0) {
            swap_columns_c<NB>(Ar, Ai, ld, j0, na, aff_src, aff_dst, c_lo, c_hi);
            __syncthreads();
        }
    };
    // U12 = L11^{-1} A12 on columns [c_lo, c_hi) of the rows j0 .. j0+nb (L11
    // from the panel rows in LDS; one thread per column, all waves), written
    // back to A, then A22 -= L21 U12 on the rows [j0+nb, rend), one column
    // block at a time (U12 block staged from A)
    auto u12_update = [&](int j0, int nb, int c_lo, int c_hi, int rend) {
#pragma unroll 1
        for (int col = c_lo + tid; col < c_hi; col += LU_THREADS) {
            // compiler-only barrier: keeps the L11 reads from LDS inside the
            // loop (hoisted, they would hold NB(NB-1) values in registers)
            asm volatile("" ::: "memory");
            T vr[NB], vi[NB];
            for (int c = 0; c < NB; ++c) {
                const bool ok = c < nb;
                vr[c] = ok ? Ar[(long long)(j0 + c) * ld + col] : T(0);
                vi[c] = ok ? Ai[(long long)(j0 + c) * ld + col] : T(0);
            }
            // fully unrolled (register arrays); rows c >= nb stay zero
#pragma unroll
            for (int c = 1; c < NB; ++c) {
                T sr = vr[c], si = vi[c];
                const int pc = c < nb ? pa[c] * NBP : 0;
#pragma unroll
                for (int k = 0; k < c; ++k) {
                    const T lr = pr[pc + k], li = pi[pc + k];
                    sr -= lr * vr[k] - li * vi[k];
                    si -= lr * vi[k] + li * vr[k];
                }
                if (c < nb) {
                    vr[c] = sr;
                    vi[c] = si;
                }
            }
            for (int c = 0; c < NB; ++c)
                if (c < nb) {
                    Ar[(long long)(j0 + c) * ld + col] = vr[c];
                    Ai[(long long)(j0 + c) * ld + col] = vi[c];
                }
        }
        __syncthreads();
        if (rend <= j0 + nb) return;
        for (int cb = c_lo; cb < c_hi; cb += LU_CB) {
            const int ncb = min(LU_CB, c_hi - cb);
            for (int e = tid; e < NB * LU_CB; e += LU_THREADS) {
                const int c = e / LU_CB, j = e % LU_CB;
                const bool ok = c < nb && j < ncb;
                const long long g = (long long)(j0 + min(c, nb - 1)) * ld + cb + min(j, ncb - 1);
                const T a = Ar[g], b = Ai[g];
                ur[e] = ok ? a : T(0);
                ui[e] = ok ? b : T(0);
            }
            __syncthreads();
            trailing_update_cg(Ar, Ai, j0 + nb, rend, ld, nb, cb, ncb, from_panel(j0), ur, ui, LU_CB);
            __syncthreads();
        }
    };
    for (int J0 = 0; J0 < m; J0 += nbo) {
      const int jend = min(J0 + nbo, m);             // end of the outer block
      const int cmax = jend;                         // columns the panels of the block touch
      for (int j0 = J0; j0 < jend; j0 += NB) {
        const int nb = min(NB, m - j0), mr = m - j0;
        for (int e = tid; e < mr * nb; e += LU_THREADS) {
            const int r = e / nb, c = e % nb;
            const long long g = (long long)(j0 + r) * ld + j0 + c;
            pr[r * NBP + c] = Ar[g];
            pi[r * NBP + c] = Ai[g];
        }
        __syncthreads();
        // The panel rows stay where they are: each thread owns the rows
        // tid + i LU_THREADS and keeps their logical positions (lg, moved by
        // the interchanges) and whether they are pivotal yet (dn) in
        // registers.  A pivot row is not written while its column is
        // eliminated, and each thread searches only the rows it updated
        // itself, so each column takes one barrier; ties go to the smaller
        // logical row, so the pivots and factors are those of the panel with
        // its rows interchanged.
        int lg[LU_C2_ROWS];
        unsigned dn = 0;
#pragma unroll
        for (int i = 0; i < LU_C2_ROWS; ++i) lg[i] = tid + i * LU_THREADS;
        for (int c = 0; c < nb; ++c) {
            const int buf = c & 1;
            T best = T(-1);
            int bl = 0x7fffffff, bp = 0;
#pragma unroll
            for (int i = 0; i < LU_C2_ROWS; ++i) {
                const int r = tid + i * LU_THREADS;
                if (r < mr && !((dn >> i) & 1u)) {
                    const T x = pr[r * NBP + c], y = pi[r * NBP + c];
                    const T v = x * x + y * y;
                    if (v > best || (v == best && lg[i] < bl)) { best = v; bl = lg[i]; bp = r; }
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const T ov = __shfl_xor(best, off, 64);
                const int ol = __shfl_xor(bl, off, 64), op = __shfl_xor(bp, off, 64);
                if (ov > best || (ov == best && ol < bl)) { best = ov; bl = ol; bp = op; }
            }
            if (lane == 0) { rv[buf][wv] = best; rl[buf][wv] = bl; rp[buf][wv] = bp; }
            __syncthreads();
            T bv = rv[buf][0];
            int p = rl[buf][0], P = rp[buf][0];
            for (int w = 1; w < LU_THREADS / 64; ++w)
                if (rv[buf][w] > bv || (rv[buf][w] == bv && rl[buf][w] < p)) { bv = rv[buf][w]; p = rl[buf][w]; P = rp[buf][w]; }
            if (tid == 0) {
                piv[j0 + c] = j0 + p;
                sw[c] = p;
                bsw[j0 - J0 + c] = p;
                if (bv == T(0) && info) atomicAdd(info, 1);
            }
            const T dr = pr[P * NBP + c], di = pi[P * NBP + c];
            const T den = dr * dr + di * di;
            const T ir = den != T(0) ? dr / den : T(0), ii = den != T(0) ? -di / den : T(0);
#pragma unroll
            for (int i = 0; i < LU_C2_ROWS; ++i) {
                const int r = tid + i * LU_THREADS;
                if (r >= mr || ((dn >> i) & 1u)) continue;
                if (r == P) {
                    lg[i] = c;
                    dn |= 1u << i;
                    continue;
                }
                if (lg[i] == c) lg[i] = p;
                const T xr = pr[r * NBP + c], xi = pi[r * NBP + c];
                const T lr = xr * ir - xi * ii, li = xr * ii + xi * ir;
                pr[r * NBP + c] = lr;
                pi[r * NBP + c] = li;
                for (int cc = c + 1; cc < nb; ++cc) {
                    const T vr = pr[P * NBP + cc], vi = pi[P * NBP + cc];
                    pr[r * NBP + cc] -= lr * vr - li * vi;
                    pi[r * NBP + cc] -= lr * vi + li * vr;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < LU_C2_ROWS; ++i) {
            const int r = tid + i * LU_THREADS;
            if (r < mr) pa[lg[i]] = r;
        }
        __syncthreads();
        // the panel's interchanges on the columns it touches (its own columns
        // are rewritten below)
        apply_swaps(j0, nb, 0, cmax);
        for (int e = tid; e < mr * nb; e += LU_THREADS) {
            const int r = e / nb, c = e % nb;
            const long long g = (long long)(j0 + r) * ld + j0 + c;
            Ar[g] = pr[pa[r] * NBP + c];
            Ai[g] = pi[pa[r] * NBP + c];
        }
        __syncthreads();
        u12_update(j0, nb, j0 + nb, cmax, m);
      }
      if (cmax < m) {
        // columns behind the block, untouched so far: the block's interchanges
        // in panel order, U of the block's rows (blocked forward substitution
        // with the block's L11), then one update of the rows and columns
        // behind the block with K = jend - J0 (L from global memory, U staged
        // in LDS LU_CBD columns at a time)
        for (int j0 = J0; j0 < jend; j0 += NB) {
            const int nb = min(NB, m - j0);
            if (tid < nb) sw[tid] = bsw[j0 - J0 + tid];
            __syncthreads();
            apply_swaps(j0, nb, jend, m);
        }
        for (int j0 = J0; j0 < jend; j0 += NB) {
            const int nb = min(NB, m - j0), nr = jend - j0;
            for (int e = tid; e < nr * nb; e += LU_THREADS) {
                const int r = e / nb, c = e % nb;
                const long long g = (long long)(j0 + r) * ld + j0 + c;
                pr[r * NBP + c] = Ar[g];
                pi[r * NBP + c] = Ai[g];
            }
            for (int r = tid; r < nr; r += LU_THREADS) pa[r] = r;   // rows reloaded in logical order
            __syncthreads();
            u12_update(j0, nb, jend, m, jend);
        }
        // the U rows are staged in the panel and U regions (free here), in
        // column blocks as wide as they hold: every column block reads L once
        // more from global memory
        const int kk = jend - J0;
        const int cbw = max(LU_CBD, min(((2 * m * NBP + 2 * ubw) / (2 * kk)) & ~31, (m - jend + 31) & ~31));
        T *vr = pr, *vi = pr + (size_t)kk * cbw;
        for (int cb = jend; cb < m; cb += cbw) {
            const int ncb = min(cbw, m - cb);
            for (int e = tid; e < kk * cbw; e += LU_THREADS) {
                const int c = e / cbw, j = e - c * cbw;
                const long long g = (long long)(J0 + c) * ld + cb + min(j, ncb - 1);
                const T a = Ar[g], b = Ai[g];
                vr[e] = j < ncb ? a : T(0);
                vi[e] = j < ncb ? b : T(0);
            }
            __syncthreads();
            trailing_update_cg(Ar, Ai, jend, m, ld, kk, cb, ncb,
                              [=](int row, int k, T &lr, T &li) {
                                  const long long g = (long long)row * ld + J0 + k;
                                  lr = Ar[g];
                                  li = Ai[g];
                              },
                              vr, vi, cbw);
            __syncthreads();
        }
      }
    }
}

// sequential LAPACK-style row interchanges -> one gather permutation per
// matrix: (P b)[i] = b[perm[i]]
__global__ void piv_to_perm_kernel(const int *__restrict__ piv, int *__restrict__ perm, int m, long long nmat)
{
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nmat) return;
    const int *p = piv + b * m;
    int *q = perm + b * m;
    for (int i = 0; i < m; ++i) q[i] = i;
    for (int j = 0; j < m; ++j) {
        const int k = p[j];
        const int t = q[j];
        q[j] = q[k];
        q[k] = t;
    }
}

// triangular solves with a planar complex row-major LU (unit lower L, upper
// U), rhs (br, bi) in LDS.  Diagonal blocks of KB rows are solved by one
// wavefront from LDS; SB of them form a super-block whose rows are updated
// block by block, while the rows outside the super-block are updated once
// with all SB*KB columns (longer contiguous row segments per load, two rows
// per 16-lane group in flight for SB = 2: the same registers as KB columns
// and four rows).  With PF the next diagonal block is loaded into registers
// while the current one is solved and the rows are updated, and stored into
// the second LDS block (dr[2 KB(KB+1)] and di likewise must then hold two
// blocks): the factors are read-only, so its load never waits for the solve.
template <typename T, int KB = 64, int SB = 1, typename TF = T, bool PF = false>
__device__ __forceinline__ void lu_substitute_c(const TF *__restrict__ Lr, const TF *__restrict__ Li, int m, int ld, T *br, T *bi,
                                                T *dr, T *di)
{
    constexpr int SW = SB * KB, RUS = SB == 1 ? 4 : (SB == 2 ? 2 : 1);
    constexpr int DPT = (KB * KB + SV_THREADS - 1) / SV_THREADS, DB = KB * (KB + 1);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    T pr[DPT], pi[DPT];
    // clamped unconditional loads of a diagonal block into registers
    auto diag_regs = [&](int kb, int nbk) {
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            const int e = tid + q * SV_THREADS, i = min(e / KB, nbk - 1), j = min(e % KB, nbk - 1);
            const long long o = (long long)(kb + i) * ld + kb + j;
            pr[q] = ld_factor<T>(Lr + o);
            pi[q] = ld_factor<T>(Li + o);
        }
    };
    auto diag_store = [&](int buf, int nbk) {
#pragma unroll
        for (int q = 0; q < DPT; ++q) {
            const int e = tid + q * SV_THREADS, i = e / KB, j = e % KB;
            if (e < KB * KB && i < nbk && j < nbk) {
                dr[buf * DB + i * (KB + 1) + j] = pr[q];
                di[buf * DB + i * (KB + 1) + j] = pi[q];
            }
        }
    };
    auto load_diag = [&](int kb, int nbk) {
        for (int e = tid; e < nbk * KB; e += SV_THREADS) {
            const int i = e / KB, j = e % KB;
            if (j < nbk) {
                dr[i * (KB + 1) + j] = ld_factor<T>(Lr + (long long)(kb + i) * ld + kb + j);
                di[i * (KB + 1) + j] = ld_factor<T>(Li + (long long)(kb + i) * ld + kb + j);
            }
        }
    };
    // forward: unit lower
    int cur = 0;
    if constexpr (PF) {
        diag_regs(0, min(KB, m));
        diag_store(0, min(KB, m));
    }
    for (int sb = 0; sb < m; sb += SW) {
        const int se = min(sb + SW, m);
        for (int kb = sb; kb < se; kb += KB) {
            const int nbk = min(KB, se - kb), kn = kb + KB;
            if constexpr (PF) {
                if (kn < m) diag_regs(kn, min(KB, m - kn));
            } else {
                load_diag(kb, nbk);
            }
            __syncthreads();
            if (wv == 0) {
                const T *cr_ = dr + cur * DB, *ci_ = di + cur * DB;
                T yr = lane < nbk ? br[kb + lane] : T(0), yi = lane < nbk ? bi[kb + lane] : T(0);
                for (int c = 0; c < nbk; ++c) {
                    const T cr = __shfl(yr, c, 64), ci = __shfl(yi, c, 64);
                    if (lane > c && lane < nbk) {
                        const T lr = cr_[lane * (KB + 1) + c], li = ci_[lane * (KB + 1) + c];
                        yr -= lr * cr - li * ci;
                        yi -= lr * ci + li * cr;
                    }
                }
                if (lane < nbk) {
                    br[kb + lane] = yr;
                    bi[kb + lane] = yi;
                }
            }
            __syncthreads();
            if (kb + nbk < se) {
                block_gemv_update<T, true, KB, 4, TF>(Lr, Li, ld, kb, nbk, kb + nbk, se, br, bi);
            }
            if constexpr (PF) {
                if (kn < m) diag_store(cur ^ 1, min(KB, m - kn));
                cur ^= 1;
            }
            __syncthreads();
        }
        block_gemv_update<T, true, SW, RUS, TF>(Lr, Li, ld, sb, se - sb, se, m, br, bi);
        __syncthreads();
    }
    // backward: upper with diagonal
    const int nsb = (m + SW - 1) / SW;
    const int nblk = (m + KB - 1) / KB;
    if constexpr (PF) {
        const int kl = (nblk - 1) * KB;
        diag_regs(kl, m - kl);
        diag_store(cur, m - kl);
    }
    for (int bs = nsb - 1; bs >= 0; --bs) {
        const int sb = bs * SW, se = min(sb + SW, m);
        const int nin = (se - sb + KB - 1) / KB;
        for (int j = nin - 1; j >= 0; --j) {
            const int kb = sb + j * KB, nbk = min(KB, se - kb), kn = kb - KB;
            if constexpr (PF) {
                if (kn >= 0) diag_regs(kn, KB);
            } else {
                load_diag(kb, nbk);
            }
            __syncthreads();
            if (wv == 0) {
                const T *cr_ = dr + cur * DB, *ci_ = di + cur * DB;
                T xr = lane < nbk ? br[kb + lane] : T(0), xi = lane < nbk ? bi[kb + lane] : T(0);
                for (int c = nbk - 1; c >= 0; --c) {
                    const T vr = __shfl(xr, c, 64), vi = __shfl(xi, c, 64);
                    const T ur = cr_[c * (KB + 1) + c], ui = ci_[c * (KB + 1) + c];
                    const T den = ur * ur + ui * ui;
                    const T qr = (vr * ur + vi * ui) / den, qi = (vi * ur - vr * ui) / den;
                    if (lane == c) {
                        xr = qr;
                        xi = qi;
                    }
                    if (lane < c) {
                        const T lr = cr_[lane * (KB + 1) + c], li = ci_[lane * (KB + 1) + c];
                        xr -= lr * qr - li * qi;
                        xi -= lr * qi + li * qr;
                    }
                }
                if (lane < nbk) {
                    br[kb + lane] = xr;
                    bi[kb + lane] = xi;
                }
            }
            __syncthreads();
            if (kb > sb) {
                block_gemv_update<T, true, KB, 4, TF>(Lr, Li, ld, kb, nbk, sb, kb, br, bi);
            }
            if constexpr (PF) {
                if (kn >= 0) diag_store(cur ^ 1, KB);
                cur ^= 1;
            }
            __syncthreads();
        }
        block_gemv_update<T, true, SW, RUS, TF>(Lr, Li, ld, sb, se - sb, 0, sb, br, bi);
        __syncthreads();
    }
}

// one time-decoupled patch solve per cell: gather the patch defect of all
// time nodes, per eigen-system transform (with the LU row permutation),
// substitute, transform back; velocity to the cell buffer E, pressure
// updated in place (pressure unknowns belong to one cell)
template <int DIM, int R, typename T, typename TP, typename TF = TP>
__global__ void __launch_bounds__(SV_THREADS) solve_td_kernel(SolveTdArgs<T, TP, TF> A)
{
    using Z = VS<DIM, R>;
    constexpr int N1 = Z::N1, NL = Z::NL, NPM = Z::NPM;
    constexpr int NV = DIM * NL, MS = NV + NPM, MSP = (MS + 1) & ~1;
    constexpr int LDM = td_ld(MS);
    constexpr long long MAT = (long long)MS * LDM;
    extern __shared__ unsigned char lds_raw[];
    const int nt = A.nt;
    TP *rl = reinterpret_cast<TP *>(lds_raw);   // [nt][MS] patch defect
    TP *out = rl + nt * MSP;                    // [nt][MS] patch correction
    TP *br = out + nt * MSP;
    TP *bi = br + MSP;
    TP *dr = bi + MSP;
    // diagonal-block width of the substitutions: 32 keeps the LDS at a size
    // that lets several workgroups share a CU (32^3, r = 3, k = 1, finest
    // level: FP64 four instead of one, FP32 six instead of three); the
    // complex substitution updates the rows outside pairs of blocks with 64
    // columns at once (4 % faster sweeps than 32)
    constexpr int KBT = 32;
    // FP32, patches above 128 unknowns: two diagonal blocks per plane (the
    // next one is prefetched)
    constexpr bool PFD = sizeof(TP) == 4 && MS > 128;
    TP *di = dr + (PFD ? 2 : 1) * KBT * (KBT + 1);
    const int cell = xcd_cell(blockIdx.x, gridDim.x), tid = threadIdx.x;
    const int c0 = cell % A.n0, c1 = (cell / A.n0) % A.n1, c2 = DIM == 3 ? cell / (A.n0 * A.n1) : 0;
    const long long N0 = (long long)(R + 1) * A.n0 + 1, N1g = (long long)(R + 1) * A.n1 + 1;
    const long long pbase = (long long)nt * A.Nv1;
    for (int e = tid; e < nt * MS; e += SV_THREADS) {
        const int a = e / MS, j = e - (e / MS) * MS;
        long long g;
        if (j < NV) {
            const int l = j % NL, c = j / NL;
            const int i0 = l % N1, i1 = (l / N1) % N1, i2 = DIM == 3 ? l / (N1 * N1) : 0;
            g = a * A.Nv1 + c * A.Nn +
                (((long long)(R + 1) * c0 + i0) + N0 * (((long long)(R + 1) * c1 + i1) + N1g * ((long long)(R + 1) * c2 + i2)));
        } else {
            g = pbase + a * A.Np1 + (long long)cell * NPM + (j - NV);
        }
        rl[a * MSP + j] = (TP)A.defect[g];
        out[a * MSP + j] = TP(0);
    }
    __syncthreads();
    for (int s = 0; s < A.nsys; ++s) {
        const bool cx = A.cplx[s] != 0;
        const int *perm = A.perm[s] + (long long)cell * MS;
        for (int i = tid; i < MS; i += SV_THREADS) {
            const int src = perm[i];
            TP sr = 0, si = 0;
            for (int a = 0; a < nt; ++a) {
                sr += A.Tre[s * 4 + a] * rl[a * MSP + src];
                si += A.Tim[s * 4 + a] * rl[a * MSP + src];
            }
            br[i] = sr;
            bi[i] = si;
        }
        __syncthreads();
        const TF *LU = A.sys[s] + (long long)cell * (cx ? 2 : 1) * MAT;
        if (cx) lu_substitute_c<TP, KBT, 2, TF, PFD>(LU, LU + MAT, MS, LDM, br, bi, dr, di);
        else lu_substitute<TP, KBT, TF>(LU, MS, LDM, br, dr);
        for (int e = tid; e < nt * MS; e += SV_THREADS) {
            const int a = e / MS, j = e - (e / MS) * MS;
            TP v = A.Fre[a * 4 + s] * br[j];
            if (cx) v -= A.Fim[a * 4 + s] * bi[j];
            out[a * MSP + j] += v;
        }
        __syncthreads();
    }
    T *Ec = A.E + (long long)cell * nt * NV;
    for (int e = tid; e < nt * MS; e += SV_THREADS) {
        const int a = e / MS, j = e - (e / MS) * MS;
        if (j < NV) Ec[a * NV + j] = (T)out[a * MSP + j];
        else A.d[pbase + a * A.Np1 + (long long)cell * NPM + (j - NV)] += A.omega * (T)out[a * MSP + j];
    }
}

// ---------------------------------------------------------------------------
// Diagonal Vanka on the time-decoupled patch systems (the cheaper smoother the
// paper's conclusions point to): each spatial system [[A, B^T], [B, C]] of a
// cell is replaced by [[diag(A), B^T], [B, C]] and solved through the
// pressure Schur complement S = C - B diag(A)^{-1} B^T.  Complex systems are
// planar (re plane, then im plane); real systems have no im plane.
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ void cmul(T ar, T ai, T br, T bi, T &cr, T &ci)
{
    cr = ar * br - ai * bi;
    ci = ar * bi + ai * br;
}

// inverse of a small complex N x N block in registers (Gauss-Jordan with
// partial pivoting); a singular block gives zeros
template <int N, typename T> __device__ __forceinline__ void cinv_small(T (&ar)[N][N], T (&ai)[N][N])
{
    T xr[N][N], xi[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            xr[i][j] = i == j ? T(1) : T(0);
            xi[i][j] = T(0);
        }
    bool ok = true;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        int p = c;
        T best = ar[c][c] * ar[c][c] + ai[c][c] * ai[c][c];
#pragma unroll
        for (int r = c + 1; r < N; ++r) {
            const T v = ar[r][c] * ar[r][c] + ai[r][c] * ai[r][c];
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (best == T(0)) ok = false;
#pragma unroll
        for (int r = c + 1; r < N; ++r)
            if (r == p) {
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    T t = ar[c][j]; ar[c][j] = ar[r][j]; ar[r][j] = t;
                    t = ai[c][j]; ai[c][j] = ai[r][j]; ai[r][j] = t;
                    t = xr[c][j]; xr[c][j] = xr[r][j]; xr[r][j] = t;
                    t = xi[c][j]; xi[c][j] = xi[r][j]; xi[r][j] = t;
                }
            }
        const T den = ar[c][c] * ar[c][c] + ai[c][c] * ai[c][c];
        const T ir = den != T(0) ? ar[c][c] / den : T(0), ii = den != T(0) ? -ai[c][c] / den : T(0);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            T tr, ti;
            cmul(ar[c][j], ai[c][j], ir, ii, tr, ti);
            ar[c][j] = tr;
            ai[c][j] = ti;
            cmul(xr[c][j], xi[c][j], ir, ii, tr, ti);
            xr[c][j] = tr;
            xi[c][j] = ti;
        }
#pragma unroll
        for (int r = 0; r < N; ++r)
            if (r != c) {
                const T fr = ar[r][c], fi = ai[r][c];
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    T tr, ti;
                    cmul(fr, fi, ar[c][j], ai[c][j], tr, ti);
                    ar[r][j] -= tr;
                    ai[r][j] -= ti;
                    cmul(fr, fi, xr[c][j], xi[c][j], tr, ti);
                    xr[r][j] -= tr;
                    xi[r][j] -= ti;
                }
            }
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            ar[i][j] = ok ? xr[i][j] : T(0);
            ai[i][j] = ok ? xi[i][j] : T(0);
        }
}

// rebuild: D^{-1} (diagonal, or BLK: DIM x DIM node blocks), S and its LU
// (partial pivoting, one wavefront) per (cell, system); grid (ncell, nsys)
template <int DIM, int R, typename T, bool BLK>
__global__ void __launch_bounds__(SV_THREADS) dv_setup_kernel(DvArgs<T> A)
{
    using Z = VS<DIM, R>;
    constexpr int NL = Z::NL, NV = DIM * NL, NPM = Z::NPM, MS = NV + NPM;
    constexpr int ND = BLK ? NL * DIM * DIM : NV;   // stored D^{-1} entries per plane
    constexpr int LDM = td_ld(MS);
    constexpr long long MAT = (long long)MS * LDM;
    static_assert(NPM <= 64, "one lane per Schur row");
    __shared__ T dvr[ND], dvi[ND], sr[NPM * NPM], si[NPM * NPM];
    const int cell = blockIdx.x, sy = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const bool cx = A.cplx[sy] != 0;
    const T *Mr = A.sys[sy] + (long long)cell * (cx ? 2 : 1) * MAT;
    const T *Mi = Mr + MAT;   // read only when cx
    T *gd = A.dinv[sy] + (long long)cell * 2 * ND;
    if constexpr (BLK) {
        // node l: unknowns c NL + l, c < DIM; block stored [l][c][c']
        for (int l = tid; l < NL; l += SV_THREADS) {
            T br_[DIM][DIM], bi_[DIM][DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c)
#pragma unroll
                for (int c2 = 0; c2 < DIM; ++c2) {
                    const long long o = (long long)(c * NL + l) * LDM + c2 * NL + l;
                    br_[c][c2] = Mr[o];
                    bi_[c][c2] = cx ? Mi[o] : T(0);
                }
            cinv_small<DIM, T>(br_, bi_);
#pragma unroll
            for (int c = 0; c < DIM; ++c)
#pragma unroll
                for (int c2 = 0; c2 < DIM; ++c2) {
                    const int q = (l * DIM + c) * DIM + c2;
                    dvr[q] = br_[c][c2];
                    dvi[q] = bi_[c][c2];
                    gd[q] = br_[c][c2];
                    gd[ND + q] = bi_[c][c2];
                }
        }
    } else {
        for (int i = tid; i < NV; i += SV_THREADS) {
            const T ar = Mr[(long long)i * LDM + i], ai = cx ? Mi[(long long)i * LDM + i] : T(0);
            const T den = ar * ar + ai * ai;
            const T ir = den != T(0) ? ar / den : T(0), ii = den != T(0) ? -ai / den : T(0);
            dvr[i] = ir;
            dvi[i] = ii;
            gd[i] = ir;
            gd[ND + i] = ii;
        }
    }
    __syncthreads();
    for (int e = tid; e < NPM * NPM; e += SV_THREADS) {
        const int j = e / NPM, k = e - (e / NPM) * NPM;
        const long long rj = (long long)(NV + j) * LDM;
        T acr = Mr[rj + NV + k], aci = cx ? Mi[rj + NV + k] : T(0);
        if constexpr (BLK) {
            for (int l = 0; l < NL; ++l) {
                T wr[DIM], wi[DIM];   // (D_l^{-1} B^T[:, k]) for the node's components
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    wr[c] = 0;
                    wi[c] = 0;
#pragma unroll
                    for (int c2 = 0; c2 < DIM; ++c2) {
                        const long long o = (long long)(c2 * NL + l) * LDM + NV + k;
                        T tr, ti;
                        cmul(dvr[(l * DIM + c) * DIM + c2], dvi[(l * DIM + c) * DIM + c2], Mr[o], cx ? Mi[o] : T(0),
                             tr, ti);
                        wr[c] += tr;
                        wi[c] += ti;
                    }
                }
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    T tr, ti;
                    cmul(Mr[rj + c * NL + l], cx ? Mi[rj + c * NL + l] : T(0), wr[c], wi[c], tr, ti);
                    acr -= tr;
                    aci -= ti;
                }
            }
        } else {
            for (int i = 0; i < NV; ++i) {
                const long long ci_ = (long long)i * LDM + NV + k;
                const T bre = Mr[rj + i], bim = cx ? Mi[rj + i] : T(0);          // B[j][i]
                const T cre = Mr[ci_], cim = cx ? Mi[ci_] : T(0);                   // B^T[i][k]
                T tr, ti, ur, ui;
                cmul(bre, bim, dvr[i], dvi[i], tr, ti);
                cmul(tr, ti, cre, cim, ur, ui);
                acr -= ur;
                aci -= ui;
            }
        }
        sr[e] = acr;
        si[e] = aci;
    }
    __syncthreads();
    if (wv == 0) {
        int *pv = A.spiv[sy] + (long long)cell * NPM;
        for (int c = 0; c < NPM; ++c) {
            T best = T(-1);
            int bi = c;
            if (lane >= c && lane < NPM) {
                const T x = sr[lane * NPM + c], y = si[lane * NPM + c];
                best = x * x + y * y;
                bi = lane;
            }
            for (int off = 32; off > 0; off >>= 1) {
                const T ov = __shfl_xor(best, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ov > best || (ov == best && oi < bi)) {
                    best = ov;
                    bi = oi;
                }
            }
            const int p = bi;
            if (lane == 0) {
                pv[c] = p;
                if (best == T(0) && A.info) atomicAdd(A.info, 1);
            }
            if (p != c && lane < NPM) {
                T t = sr[c * NPM + lane];
                sr[c * NPM + lane] = sr[p * NPM + lane];
                sr[p * NPM + lane] = t;
                t = si[c * NPM + lane];
                si[c * NPM + lane] = si[p * NPM + lane];
                si[p * NPM + lane] = t;
            }
            __builtin_amdgcn_wave_barrier();
            const T dr = sr[c * NPM + c], di = si[c * NPM + c];
            const T den = dr * dr + di * di;
            const T ir = den != T(0) ? dr / den : T(0), ii = den != T(0) ? -di / den : T(0);
            if (lane > c && lane < NPM) {
                T lr, li;
                cmul(sr[lane * NPM + c], si[lane * NPM + c], ir, ii, lr, li);
                sr[lane * NPM + c] = lr;
                si[lane * NPM + c] = li;
                for (int cc = c + 1; cc < NPM; ++cc) {
                    T ur, ui;
                    cmul(lr, li, sr[c * NPM + cc], si[c * NPM + cc], ur, ui);
                    sr[lane * NPM + cc] -= ur;
                    si[lane * NPM + cc] -= ui;
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
    T *gs = A.schur[sy] + (long long)cell * 2 * NPM * NPM;
    for (int e = tid; e < NPM * NPM; e += SV_THREADS) {
        gs[e] = sr[e];
        gs[NPM * NPM + e] = si[e];
    }
}

// one diagonal-Vanka patch solve per cell: gather the patch defect of all
// time nodes, per eigen-system transform, t = D^{-1} f, h = g - B t,
// p = S^{-1} h, u = t - D^{-1} B^T p, transform back; velocity to the cell
// buffer E, pressure updated in place
template <int DIM, int R, typename T, bool BLK>
__global__ void __launch_bounds__(SV_THREADS) solve_dv_kernel(DvArgs<T> A)
{
    using Z = VS<DIM, R>;
    constexpr int N1 = Z::N1, NL = Z::NL, NPM = Z::NPM;
    constexpr int NV = DIM * NL, MS = NV + NPM, MSP = (MS + 1) & ~1;
    constexpr int LDM = td_ld(MS);
    constexpr long long MAT = (long long)MS * LDM;
    static_assert(NPM <= 64, "one lane per Schur row");
    extern __shared__ unsigned char lds_raw[];
    const int nt = A.nt;
    T *rl = reinterpret_cast<T *>(lds_raw);   // [nt][MS] patch defect
    T *out = rl + nt * MSP;                   // [nt][MS] patch correction
    T *br = out + nt * MSP;                   // system right-hand side / solution
    T *bi = br + MSP;
    T *hr = bi + MSP;                         // [NPM] Schur right-hand side
    T *hi = hr + NPM;
    const int cell = xcd_cell(blockIdx.x, gridDim.x), tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int c0 = cell % A.n0, c1 = (cell / A.n0) % A.n1, c2 = DIM == 3 ? cell / (A.n0 * A.n1) : 0;
    const long long N0 = (long long)(R + 1) * A.n0 + 1, N1g = (long long)(R + 1) * A.n1 + 1;
    const long long pbase = (long long)nt * A.Nv1;
    for (int e = tid; e < nt * MS; e += SV_THREADS) {
        const int a = e / MS, j = e - (e / MS) * MS;
        long long g;
        if (j < NV) {
            const int l = j % NL, c = j / NL;
            const int i0 = l % N1, i1 = (l / N1) % N1, i2 = DIM == 3 ? l / (N1 * N1) : 0;
            g = a * A.Nv1 + c * A.Nn +
                (((long long)(R + 1) * c0 + i0) + N0 * (((long long)(R + 1) * c1 + i1) + N1g * ((long long)(R + 1) * c2 + i2)));
        } else {
            g = pbase + a * A.Np1 + (long long)cell * NPM + (j - NV);
        }
        rl[a * MSP + j] = A.defect[g];
        out[a * MSP + j] = T(0);
    }
    __syncthreads();
    for (int sy = 0; sy < A.nsys; ++sy) {
        const bool cx = A.cplx[sy] != 0;
        const T *Mr = A.sys[sy] + (long long)cell * (cx ? 2 : 1) * MAT;
        const T *Mi = Mr + MAT;   // read only when cx
        constexpr int ND = BLK ? NL * DIM * DIM : NV;
        const T *dv = A.dinv[sy] + (long long)cell * 2 * ND;
        // transform, then t = D^{-1} f on the velocity part
        for (int i = tid; i < MS; i += SV_THREADS) {
            T xr = 0, xi = 0;
            for (int a = 0; a < nt; ++a) {
                xr += A.Tre[sy * 4 + a] * rl[a * MSP + i];
                xi += A.Tim[sy * 4 + a] * rl[a * MSP + i];
            }
            if (!BLK && i < NV) cmul(xr, xi, dv[i], dv[ND + i], xr, xi);
            br[i] = xr;
            bi[i] = xi;
        }
        __syncthreads();
        if constexpr (BLK) {
            // node blocks: t_l = D_l^{-1} f_l (one thread per node)
            for (int l = tid; l < NL; l += SV_THREADS) {
                T fr[DIM], fi[DIM];
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    fr[c] = br[c * NL + l];
                    fi[c] = bi[c * NL + l];
                }
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    T sr_ = 0, si_ = 0;
#pragma unroll
                    for (int c2 = 0; c2 < DIM; ++c2) {
                        const int q = (l * DIM + c) * DIM + c2;
                        T tr, ti;
                        cmul(dv[q], dv[ND + q], fr[c2], fi[c2], tr, ti);
                        sr_ += tr;
                        si_ += ti;
                    }
                    br[c * NL + l] = sr_;
                    bi[c * NL + l] = si_;
                }
            }
            __syncthreads();
        }
        // h = g - B t: one wavefront per pressure row
        for (int j = wv; j < NPM; j += SV_THREADS / 64) {
            const long long rj = (long long)(NV + j) * LDM;
            T sr_ = 0, si_ = 0;
            for (int i = lane; i < NV; i += 64) {
                T ur, ui;
                cmul(Mr[rj + i], cx ? Mi[rj + i] : T(0), br[i], bi[i], ur, ui);
                sr_ += ur;
                si_ += ui;
            }
            for (int off = 32; off > 0; off >>= 1) {
                sr_ += __shfl_xor(sr_, off, 64);
                si_ += __shfl_xor(si_, off, 64);
            }
            if (lane == 0) {
                hr[j] = br[NV + j] - sr_;
                hi[j] = bi[NV + j] - si_;
            }
        }
        __syncthreads();
        // p = S^{-1} h (row interchanges, unit lower, upper): one wavefront
        if (wv == 0) {
            const T *Sr = A.schur[sy] + (long long)cell * 2 * NPM * NPM, *Si = Sr + NPM * NPM;
            const int *pv = A.spiv[sy] + (long long)cell * NPM;
            if (lane == 0)
                for (int j = 0; j < NPM; ++j) {
                    const int p = pv[j];
                    if (p != j) {
                        T t = hr[j];
                        hr[j] = hr[p];
                        hr[p] = t;
                        t = hi[j];
                        hi[j] = hi[p];
                        hi[p] = t;
                    }
                }
            __builtin_amdgcn_wave_barrier();
            T xr = lane < NPM ? hr[lane] : T(0), xi = lane < NPM ? hi[lane] : T(0);
            for (int c = 0; c < NPM; ++c) {
                const T cr = __shfl(xr, c, 64), ci = __shfl(xi, c, 64);
                if (lane > c && lane < NPM) {
                    T ur, ui;
                    cmul(Sr[lane * NPM + c], Si[lane * NPM + c], cr, ci, ur, ui);
                    xr -= ur;
                    xi -= ui;
                }
            }
            for (int c = NPM - 1; c >= 0; --c) {
                const T vr = __shfl(xr, c, 64), vi = __shfl(xi, c, 64);
                const T ur = Sr[c * NPM + c], ui = Si[c * NPM + c];
                const T den = ur * ur + ui * ui;
                const T qr = (vr * ur + vi * ui) / den, qi = (vi * ur - vr * ui) / den;
                if (lane == c) {
                    xr = qr;
                    xi = qi;
                }
                if (lane < c) {
                    T wr, wi;
                    cmul(Sr[lane * NPM + c], Si[lane * NPM + c], qr, qi, wr, wi);
                    xr -= wr;
                    xi -= wi;
                }
            }
            if (lane < NPM) {
                br[NV + lane] = xr;
                bi[NV + lane] = xi;
            }
        }
        __syncthreads();
        // u = t - D^{-1} B^T p
        if constexpr (BLK) {
            for (int l = tid; l < NL; l += SV_THREADS) {
                T qr[DIM], qi[DIM];   // (B^T p) at the node's components
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    const long long ri = (long long)(c * NL + l) * LDM + NV;
                    T sr_ = 0, si_ = 0;
#pragma unroll 4
                    for (int j = 0; j < NPM; ++j) {
                        T ur, ui;
                        cmul(Mr[ri + j], cx ? Mi[ri + j] : T(0), br[NV + j], bi[NV + j], ur, ui);
                        sr_ += ur;
                        si_ += ui;
                    }
                    qr[c] = sr_;
                    qi[c] = si_;
                }
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    T sr_ = 0, si_ = 0;
#pragma unroll
                    for (int c2 = 0; c2 < DIM; ++c2) {
                        const int q = (l * DIM + c) * DIM + c2;
                        T tr, ti;
                        cmul(dv[q], dv[ND + q], qr[c2], qi[c2], tr, ti);
                        sr_ += tr;
                        si_ += ti;
                    }
                    br[c * NL + l] -= sr_;
                    bi[c * NL + l] -= si_;
                }
            }
        } else {
            for (int i = tid; i < NV; i += SV_THREADS) {
                const long long ri = (long long)i * LDM + NV;
                T sr_ = 0, si_ = 0;
#pragma unroll 4
                for (int j = 0; j < NPM; ++j) {
                    T ur, ui;
                    cmul(Mr[ri + j], cx ? Mi[ri + j] : T(0), br[NV + j], bi[NV + j], ur, ui);
                    sr_ += ur;
                    si_ += ui;
                }
                T wr, wi;
                cmul(sr_, si_, dv[i], dv[ND + i], wr, wi);
                br[i] -= wr;
                bi[i] -= wi;
            }
        }
        __syncthreads();
        for (int e = tid; e < nt * MS; e += SV_THREADS) {
            const int a = e / MS, j = e - (e / MS) * MS;
            T v = A.Fre[a * 4 + sy] * br[j];
            if (cx) v -= A.Fim[a * 4 + sy] * bi[j];
            out[a * MSP + j] += v;
        }
        __syncthreads();
    }
    T *Ec = A.E + (long long)cell * nt * NV;
    for (int e = tid; e < nt * MS; e += SV_THREADS) {
        const int a = e / MS, j = e - (e / MS) * MS;
        if (j < NV) Ec[a * NV + j] = out[a * MSP + j];
        else A.d[pbase + a * A.Np1 + (long long)cell * NPM + (j - NV)] += A.omega * out[a * MSP + j];
    }
}

// batched solves with variable sizes: one workgroup per system
template <typename T>
__global__ void __launch_bounds__(SV_THREADS) batched_solve_kernel(const T *LUall, const int *pivall, LuBatch B,
                                                                    const long long *b_off, T *ball)
{
    extern __shared__ unsigned char lds_raw[];
    T *b = reinterpret_cast<T *>(lds_raw);
    const int bid = blockIdx.x, tid = threadIdx.x;
    const int m = B.m_of[bid];
    T *dblk = b + ((m + 1) & ~1);
    const T *LU = LUall + B.a_off[bid];
    const int *piv = pivall + B.p_off[bid];
    T *x = ball + b_off[bid];
    for (int r = tid; r < m; r += SV_THREADS) b[r] = x[r];
    __syncthreads();
    if (tid == 0)
        for (int j = 0; j < m; ++j) {
            const int p = piv[j];
            if (p != j) {
                const T t = b[j];
                b[j] = b[p];
                b[p] = t;
            }
        }
    __syncthreads();
    lu_substitute<T>(LU, m, m, b, dblk);
    for (int r = tid; r < m; r += SV_THREADS) x[r] = b[r];
}

// dense solve of one LU-factored system (coarse level): x = A^{-1} rhs
template <typename T>
__global__ void __launch_bounds__(SV_THREADS) dense_solve_kernel(const T *LU, const int *piv, int m, const T *rhs,
                                                                  T *x, int nout)
{
    extern __shared__ unsigned char lds_raw[];
    T *b = reinterpret_cast<T *>(lds_raw);
    T *dblk = b + ((m + 1) & ~1);
    const int tid = threadIdx.x;
    for (int r = tid; r < m; r += SV_THREADS) b[r] = r < nout ? rhs[r] : T(0);
    __syncthreads();
    if (tid == 0)
        for (int j = 0; j < m; ++j) {
            int p = piv[j];
            if (p != j) {
                T t = b[j];
                b[j] = b[p];
                b[p] = t;
            }
        }
    __syncthreads();
    lu_substitute<T>(LU, m, m, b, dblk);
    for (int r = tid; r < nout; r += SV_THREADS) x[r] = b[r];
}

// coarse matrix from the columns J e_i (batched vmult output, row-major
// columns) and the border of constant pressures
__global__ void coarse_matrix_kernel(const double *Y, int n, int nb, int nt, long long pbase, long long Np1, int npm,
                                     long long ncell, double *A)
{
    const int m = n + nb;
    long long total = (long long)m * m;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        int row = (int)(e % m), col = (int)(e / m);
        double v = 0;
        if (row < n && col < n) v = Y[(long long)col * n + row];
        else if (row < n && col >= n) {
            int a = col - n;
            long long q = row - pbase;
            if (q >= a * Np1 && q < (a + 1) * Np1 && ((q - a * Np1) % npm) == 0) v = 1.0;
        } else if (row >= n && col < n) {
            int a = row - n;
            long long q = col - pbase;
            if (q >= a * Np1 && q < (a + 1) * Np1 && ((q - a * Np1) % npm) == 0) v = 1.0;
        }
        A[(long long)row * m + col] = v;
    }
    (void)nt;
    (void)ncell;
}

__global__ void identity_kernel(double *X, int n)
{
    long long total = (long long)n * n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x)
        X[e] = (e / n == e % n) ? 1.0 : 0.0;
}

// V* = sum_a phimid_a V^a (velocity of one time node)
template <typename T>
__global__ void midpoint_kernel(const T *state, long long Nv1, int nt, const double *phim_unused, T pm0, T pm1, T pm2,
                                T pm3, T *vstar)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nv1) return;
    T pm[4] = {pm0, pm1, pm2, pm3};
    T s = 0;
    for (int a = 0; a < nt; ++a) s += pm[a] * state[a * Nv1 + i];
    vstar[i] = s;
    (void)phim_unused;
}

template <int NB, typename T> size_t lu_lds_bytes(int m)
{
    return ((size_t)m * (NB + 1) + (size_t)lu_outer_block(m, NB) * LU_CB + (size_t)2 * NB * LU_SWC) * sizeof(T);
}

template <int NB, typename T> size_t lu_c_lds_bytes(int m)
{
    return ((size_t)2 * m * (NB + 1) + (size_t)2 * NB * LU_CB + (size_t)2 * NB * LU_SWC) * sizeof(T);
}

// LDS of lu_kernel_c2 (panel, U block, logical-to-panel row map)
template <int NB> size_t lu_c2_lds_bytes(int m)
{
    return ((size_t)2 * m * (NB + 1) + (size_t)2 * lu_c_u_words(NB, LU_CB) + (size_t)m) * sizeof(float);
}

} // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int elem_record_words(int dim, int r)
{
    int nl = 1;
    for (int a = 0; a < dim; ++a) nl *= r + 2;
    int npm = dim == 2 ? (r + 1) * (r + 2) / 2 : (r + 1) * (r + 2) * (r + 3) / 6;
    return dim * dim * nl * nl + nl * nl + dim * nl * npm;
}

template <typename T>
hipError_t launch_elem(int dim, int r, int nq, const ElemArgs<T> &a, int ncell, hipStream_t s)
{
    {
        // 3D: volume on MFMA, then the boundary faces
#define EMC(RR, Q)                                                                                                     \
    if (dim == 3 && r == RR && nq == Q) {                                                                              \
        hipLaunchKernelGGL((elem_mfma_kernel<RR, Q, T>), dim3(ncell), dim3(EM_THREADS), 0, s, a);                     \
        hipError_t e = hipGetLastError();                                                                              \
        if (e != hipSuccess || a.nbcell <= 0) return e;                                                                \
        hipLaunchKernelGGL((elem_kernel<3, RR, Q, T, true>), dim3(a.nbcell), dim3(EL_THREADS), 0, s, a);              \
        return hipGetLastError();                                                                                      \
    }
        EMC(1, 4) EMC(1, 3) EMC(2, 5) EMC(2, 4) EMC(3, 7) EMC(3, 5)
#undef EMC
    }
#define ELC(D, RR, Q)                                                                                                  \
    if (dim == D && r == RR && nq == Q) {                                                                              \
        hipLaunchKernelGGL((elem_kernel<D, RR, Q, T>), dim3(ncell), dim3(EL_THREADS), 0, s, a);                       \
        return hipGetLastError();                                                                                      \
    }
    ELC(2, 1, 4) ELC(2, 1, 3) ELC(2, 2, 5) ELC(2, 2, 4) ELC(2, 3, 7) ELC(2, 3, 5)
    ELC(3, 1, 4) ELC(3, 1, 3) ELC(3, 2, 5) ELC(3, 2, 4) ELC(3, 3, 7) ELC(3, 3, 5)
#undef ELC
    return hipErrorInvalidValue;
}

template <typename TE, typename TP>
hipError_t launch_patch(int dim, int r, const PatchArgs<TE, TP> &a, int ncell, hipStream_t s)
{
#define PC(D, RR)                                                                                                      \
    if (dim == D && r == RR) {                                                                                         \
        hipLaunchKernelGGL((patch_kernel<D, RR, TE, TP>), dim3(ncell), dim3(256), 0, s, a);                           \
        return hipGetLastError();                                                                                      \
    }
    PC(2, 1) PC(2, 2) PC(2, 3) PC(3, 1) PC(3, 2) PC(3, 3)
#undef PC
    return hipErrorInvalidValue;
}

// dynamic-LDS limit of a kernel, raised only when a launch needs more than
// any earlier one (keeps driver calls out of replayed or captured launches)
static hipError_t lds_attr(const void *kern, size_t bytes)
{
    static std::mutex mu;
    static std::unordered_map<const void *, size_t> set;
    std::lock_guard<std::mutex> lk(mu);
    size_t &have = set[kern];
    if (bytes <= have) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) have = bytes;
    return e;
}

// largest panel width the patch factorizations may use: 32, or the value of
// the tuning override STMG_LU_NB (32, 16, 8 or 4)
static int lu_nb_cap()
{
    const char *e = std::getenv("STMG_LU_NB");
    const int v = e ? std::atoi(e) : 32;
    return v == 16 || v == 8 || v == 4 ? v : 32;
}

// LDS of one CU: the panel width is chosen so that two factorizations share
// a CU when a panel of at least 16 columns allows it (measured on the complex
// FP32 m = 395 patches: NB 16 with two workgroups per CU is 27 % faster than
// NB 32 with one; NB 8 with four is slower, and so are the FP64 and the
// mixed-size real batches when pushed to NB 8)
constexpr size_t CU_LDS = 160 * 1024;

template <typename T>
hipError_t launch_lu(T *A, int *piv, int m, int batch, int *info, size_t max_lds, hipStream_t s, const LuBatch *vb,
                     int op)
{
    if (op < 0 || op > 2 || (op != 0 && !std::is_same<T, float>::value)) return hipErrorInvalidValue;
    LuBatch B{};
    if (vb) B = *vb;
    else B.uniform_m = m;
    int cap = lu_nb_cap();
    // widest panel (at least 16) with two workgroups per CU, else the widest
    // that fits (narrower panels lose more than the second workgroup gains)
    for (int nb = cap; nb >= 16; nb /= 2) {
        const size_t b = nb == 32 ? lu_lds_bytes<32, T>(m) : nb == 16 ? lu_lds_bytes<16, T>(m)
                       : nb == 8 ? lu_lds_bytes<8, T>(m) : lu_lds_bytes<4, T>(m);
        if (2 * b <= CU_LDS && b <= max_lds) { cap = nb; break; }
    }
#define LUK(NBV, OPV)                                                                                                  \
    {                                                                                                                  \
        size_t bytes = lu_lds_bytes<NBV, T>(m);                                                                        \
        hipError_t e = lds_attr((const void *)lu_kernel<T, NBV, OPV>, bytes);                                          \
        if (e != hipSuccess) return e;                                                                                 \
        hipLaunchKernelGGL((lu_kernel<T, NBV, OPV>), dim3(batch), dim3(LU_THREADS), bytes, s, A, piv, B, info);       \
        return hipGetLastError();                                                                                      \
    }
#define LUC(NBV)                                                                                                       \
    if (NBV <= cap && lu_lds_bytes<NBV, T>(m) <= max_lds) {                                                            \
        if constexpr (std::is_same<T, float>::value) {                                                                 \
            if (op == 1) LUK(NBV, 1)                                                                                   \
            if (op == 2) LUK(NBV, 2)                                                                                   \
        }                                                                                                              \
        LUK(NBV, 0)                                                                                                    \
    }
    LUC(32) LUC(16) LUC(8) LUC(4)
#undef LUC
#undef LUK
    return hipErrorInvalidConfiguration;
}

size_t lu_panel_lds_bytes(int nb, int m, bool f64)
{
    if (f64)
        return nb == 32 ? lu_lds_bytes<32, double>(m) : nb == 16 ? lu_lds_bytes<16, double>(m)
             : nb == 8 ? lu_lds_bytes<8, double>(m) : lu_lds_bytes<4, double>(m);
    return nb == 32 ? lu_lds_bytes<32, float>(m) : nb == 16 ? lu_lds_bytes<16, float>(m)
         : nb == 8 ? lu_lds_bytes<8, float>(m) : lu_lds_bytes<4, float>(m);
}

template <typename T>
hipError_t launch_lu_queue(T *A, int *piv, const LuQueue &q, size_t lds_bytes, int grid, int threads, int *info,
                           hipStream_t s, int op)
{
    if (op < 0 || op > 2 || (op != 0 && !std::is_same<T, float>::value) || grid < 1) return hipErrorInvalidValue;
    if (threads != 256 && threads != 512) return hipErrorInvalidValue;
    if (q.batch <= 0) return hipSuccess;
#define LUQ(OPV, NTV)                                                                                                  \
    {                                                                                                                  \
        hipError_t e = lds_attr((const void *)lu_queue_kernel<T, OPV, NTV>, lds_bytes);                                \
        if (e != hipSuccess) return e;                                                                                 \
        hipLaunchKernelGGL((lu_queue_kernel<T, OPV, NTV>), dim3(grid), dim3(NTV), lds_bytes, s, A, piv, q, info);      \
        return hipGetLastError();                                                                                      \
    }
    if constexpr (std::is_same<T, float>::value) {
        if (op == 1) {
            if (threads == 512) LUQ(1, 512)
            LUQ(1, 256)
        }
        if (op == 2) {
            if (threads == 512) LUQ(2, 512)
            LUQ(2, 256)
        }
    }
    if (threads == 512) LUQ(0, 512)
    LUQ(0, 256)
#undef LUQ
}

template <typename T, typename TP>
hipError_t launch_solve(int dim, int r, const SolveArgs<T, TP> &a, int ncell, int m, hipStream_t s)
{
    size_t bytes = ((size_t)((m + 1) & ~1) + 64 * 65) * sizeof(TP);
#define SC(D, RR)                                                                                                      \
    if (dim == D && r == RR) {                                                                                         \
        hipError_t e = lds_attr((const void *)solve_kernel<D, RR, T, TP>, bytes);                    \
        if (e != hipSuccess) return e;                                                                                 \
        hipLaunchKernelGGL((solve_kernel<D, RR, T, TP>), dim3(ncell), dim3(SV_THREADS), bytes, s, a);                 \
        return hipGetLastError();                                                                                      \
    }
    SC(2, 1) SC(2, 2) SC(2, 3) SC(3, 1) SC(3, 2) SC(3, 3)
#undef SC
    return hipErrorInvalidValue;
}

template <typename TE, typename TP>
hipError_t launch_patch_td(int dim, int r, const PatchTdArgs<TE, TP> &a, int ncell, hipStream_t s)
{
#define PC(D, RR)                                                                                                      \
    if (dim == D && r == RR) {                                                                                         \
        hipLaunchKernelGGL((patch_td_kernel<D, RR, TE, TP>), dim3(ncell), dim3(256), 0, s, a);                        \
        return hipGetLastError();                                                                                      \
    }
    PC(2, 1) PC(2, 2) PC(2, 3) PC(3, 1) PC(3, 2) PC(3, 3)
#undef PC
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_lu_c(T *A, int *piv, int m, int ld, long long a_stride, int batch, int *info, size_t max_lds,
                       hipStream_t s)
{
    if constexpr (std::is_same<T, float>::value) {
        if (m > LU_NBO_MIN_M && m <= LU_C2_ROWS * LU_THREADS) {
            // two blocking levels: the widest panel (16 or 8, within the
            // STMG_LU_NB cap) with two workgroups per CU, else the widest that fits
            int cap2 = std::min(lu_nb_cap(), 16);
            for (int nb = cap2; nb >= 8; nb /= 2) {
                const size_t b = nb == 16 ? lu_c2_lds_bytes<16>(m) : lu_c2_lds_bytes<8>(m);
                if (2 * b <= CU_LDS && b <= max_lds) { cap2 = nb; break; }
            }
#define LUC2(NBV)                                                                                                      \
    if (NBV <= cap2 && lu_c2_lds_bytes<NBV>(m) <= max_lds) {                                                           \
        size_t bytes = lu_c2_lds_bytes<NBV>(m);                                                                        \
        hipError_t e = lds_attr((const void *)lu_kernel_c2<float, NBV>, bytes);                                        \
        if (e != hipSuccess) return e;                                                                                 \
        hipLaunchKernelGGL((lu_kernel_c2<float, NBV>), dim3(batch), dim3(LU_THREADS), bytes, s, A, piv, m, ld, a_stride, \
                           info);                                                                                      \
        return hipGetLastError();                                                                                      \
    }
            LUC2(16) LUC2(8) LUC2(4)
#undef LUC2
        }
    }
    int cap = lu_nb_cap();
    for (int nb = cap; nb >= 16; nb /= 2) {
        const size_t b = nb == 32 ? lu_c_lds_bytes<32, T>(m) : nb == 16 ? lu_c_lds_bytes<16, T>(m)
                       : nb == 8 ? lu_c_lds_bytes<8, T>(m) : lu_c_lds_bytes<4, T>(m);
        if (2 * b <= CU_LDS && b <= max_lds) { cap = nb; break; }
    }
#define LUC(NBV)                                                                                                       \
    if (NBV <= cap && lu_c_lds_bytes<NBV, T>(m) <= max_lds) {                                                          \
        size_t bytes = lu_c_lds_bytes<NBV, T>(m);                                                                      \
        hipError_t e = lds_attr((const void *)lu_kernel_c<T, NBV>, bytes);                    \
        if (e != hipSuccess) return e;                                                                                 \
        hipLaunchKernelGGL((lu_kernel_c<T, NBV>), dim3(batch), dim3(LU_THREADS), bytes, s, A, piv, m, ld, a_stride, info); \
        return hipGetLastError();                                                                                      \
    }
    LUC(32) LUC(16) LUC(8) LUC(4)
#undef LUC
    return hipErrorInvalidConfiguration;
}

hipError_t launch_piv_to_perm(const int *piv, int *perm, int m, long long nmat, hipStream_t s)
{
    if (nmat <= 0) return hipSuccess;
    const int th = 256;
    hipLaunchKernelGGL(piv_to_perm_kernel, dim3((unsigned)((nmat + th - 1) / th)), dim3(th), 0, s, piv, perm, m, nmat);
    return hipGetLastError();
}

size_t solve_td_lds_bytes(int ms, int nt, size_t word)
{
    const size_t msp = (size_t)((ms + 1) & ~1);
    const size_t kb = 32;   // diagonal-block width of solve_td_kernel
    const size_t nd = word == 4 && ms > 128 ? 4 : 2;   // FP32 (ms > 128): the next block is prefetched
    return (2 * nt * msp + 2 * msp + nd * kb * (kb + 1)) * word;
}

template <typename T, typename TP>
hipError_t launch_solve_td(int dim, int r, const SolveTdArgs<T, TP> &a, int ncell, int ms, hipStream_t s)
{
    size_t bytes = solve_td_lds_bytes(ms, a.nt, sizeof(TP));
#define SC(D, RR)                                                                                                      \
    if (dim == D && r == RR) {                                                                                         \
        hipError_t e = lds_attr((const void *)solve_td_kernel<D, RR, T, TP>, bytes);                    \
        if (e != hipSuccess) return e;                                                                                 \
        hipLaunchKernelGGL((solve_td_kernel<D, RR, T, TP>), dim3(ncell), dim3(SV_THREADS), bytes, s, a);              \
        return hipGetLastError();                                                                                      \
    }
    SC(2, 1) SC(2, 2) SC(2, 3) SC(3, 1) SC(3, 2) SC(3, 3)
#undef SC
    return hipErrorInvalidValue;
}

hipError_t launch_solve_td_bf16(int dim, int r, const SolveTdArgs<float, float, unsigned short> &a, int ncell, int ms,
                                hipStream_t s)
{
    using T = float;
    using TP = float;
    size_t bytes = solve_td_lds_bytes(ms, a.nt, sizeof(TP));
#define SC(D, RR)                                                                                                      \
    if (dim == D && r == RR) {                                                                                         \
        hipError_t e = lds_attr((const void *)solve_td_kernel<D, RR, T, TP, unsigned short>, bytes);                    \
        if (e != hipSuccess) return e;                                                                                 \
        hipLaunchKernelGGL((solve_td_kernel<D, RR, T, TP, unsigned short>), dim3(ncell), dim3(SV_THREADS), bytes, s, a);              \
        return hipGetLastError();                                                                                      \
    }
    SC(2, 1) SC(2, 2) SC(2, 3) SC(3, 1) SC(3, 2) SC(3, 3)
#undef SC
    return hipErrorInvalidValue;
}

__global__ void pack_bf16_kernel(const float *__restrict__ src, unsigned short *__restrict__ dst, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = (unsigned short)bf16_rne(src[i]);
}

hipError_t launch_pack_bf16(const float *src, unsigned short *dst, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int th = 256;
    const long long nb = std::min<long long>((n + th - 1) / th, 65536);
    hipLaunchKernelGGL(pack_bf16_kernel, dim3((unsigned)nb), dim3(th), 0, s, src, dst, n);
    return hipGetLastError();
}

template <typename T> hipError_t launch_dv_setup(int dim, int r, const DvArgs<T> &a, int ncell, hipStream_t s)
{
    if (ncell <= 0) return hipSuccess;
    if (a.nsys < 1 || a.nsys > 4) return hipErrorInvalidValue;
#define DC(D, RR)                                                                                                      \
    if (dim == D && r == RR) {                                                                                         \
        if (a.block)                                                                                                   \
            hipLaunchKernelGGL((dv_setup_kernel<D, RR, T, true>), dim3(ncell, a.nsys), dim3(SV_THREADS), 0, s, a);     \
        else                                                                                                           \
            hipLaunchKernelGGL((dv_setup_kernel<D, RR, T, false>), dim3(ncell, a.nsys), dim3(SV_THREADS), 0, s, a);    \
        return hipGetLastError();                                                                                      \
    }
    DC(2, 1) DC(2, 2) DC(2, 3) DC(3, 1) DC(3, 2) DC(3, 3)
#undef DC
    return hipErrorInvalidValue;
}

template <typename T> hipError_t launch_solve_dv(int dim, int r, const DvArgs<T> &a, int ncell, hipStream_t s)
{
    if (ncell <= 0) return hipSuccess;
    const int npm = dim == 2 ? (r + 1) * (r + 2) / 2 : (r + 1) * (r + 2) * (r + 3) / 6;
    const int ms = dim * (dim == 2 ? (r + 2) * (r + 2) : (r + 2) * (r + 2) * (r + 2)) + npm;
    const size_t msp = (size_t)((ms + 1) & ~1);
    const size_t bytes = (2 * (size_t)a.nt * msp + 2 * msp + 2 * (size_t)npm) * sizeof(T);
#define SC(D, RR)                                                                                                      \
    if (dim == D && r == RR) {                                                                                         \
        if (a.block) {                                                                                                 \
            hipError_t e = lds_attr((const void *)solve_dv_kernel<D, RR, T, true>, bytes);                             \
            if (e != hipSuccess) return e;                                                                             \
            hipLaunchKernelGGL((solve_dv_kernel<D, RR, T, true>), dim3(ncell), dim3(SV_THREADS), bytes, s, a);         \
        } else {                                                                                                       \
            hipError_t e = lds_attr((const void *)solve_dv_kernel<D, RR, T, false>, bytes);                            \
            if (e != hipSuccess) return e;                                                                             \
            hipLaunchKernelGGL((solve_dv_kernel<D, RR, T, false>), dim3(ncell), dim3(SV_THREADS), bytes, s, a);        \
        }                                                                                                              \
        return hipGetLastError();                                                                                      \
    }
    SC(2, 1) SC(2, 2) SC(2, 3) SC(3, 1) SC(3, 2) SC(3, 3)
#undef SC
    return hipErrorInvalidValue;
}

template hipError_t launch_dv_setup<double>(int, int, const DvArgs<double> &, int, hipStream_t);
template hipError_t launch_dv_setup<float>(int, int, const DvArgs<float> &, int, hipStream_t);
template hipError_t launch_solve_dv<double>(int, int, const DvArgs<double> &, int, hipStream_t);
template hipError_t launch_solve_dv<float>(int, int, const DvArgs<float> &, int, hipStream_t);

template <typename T>
hipError_t launch_batched_solve(const T *LU, const int *piv, int max_m, int batch, const LuBatch &vb,
                                const long long *b_off, T *b, hipStream_t s)
{
    if (batch <= 0) return hipSuccess;
    const size_t bytes = ((size_t)((max_m + 1) & ~1) + 64 * 65) * sizeof(T);
    hipError_t e = lds_attr((const void *)batched_solve_kernel<T>, bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batched_solve_kernel<T>, dim3(batch), dim3(SV_THREADS), bytes, s, LU, piv, vb, b_off, b);
    return hipGetLastError();
}

template hipError_t launch_batched_solve<double>(const double *, const int *, int, int, const LuBatch &,
                                                 const long long *, double *, hipStream_t);
template hipError_t launch_batched_solve<float>(const float *, const int *, int, int, const LuBatch &,
                                                const long long *, float *, hipStream_t);

// ---------------------------------------------------------------------------
// Device-wide blocked LU with partial pivoting of ONE dense FP64 matrix (the
// coarsest-level system): per 32-column panel, a one-workgroup panel
// factorization, the panel's row interchanges on the other columns, the U12
// triangular solve and a tiled trailing update over many workgroups.  Same
// in-place format and pivot convention as lu_kernel (row j swapped with row
// piv[j], applied in order j = 0, 1, ...).
// ---------------------------------------------------------------------------
constexpr int DLU_NB = 32, DLU_PANEL_THREADS = 1024, DLU_TILE = 64;

__global__ void __launch_bounds__(DLU_PANEL_THREADS) dlu_panel_kernel(double *__restrict__ A, int m, int j0, int nb,
                                                                       int *__restrict__ piv, int *info)
{
    __shared__ double rv[DLU_PANEL_THREADS / 64];
    __shared__ int ri[DLU_PANEL_THREADS / 64];
    __shared__ double urow[DLU_NB];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int c = 0; c < nb; ++c) {
        const int col = j0 + c;
        // pivot: largest modulus in column col on rows col .. m-1 (ties: lowest row)
        double best = -1.0;
        int bi = col;
        for (int r = col + tid; r < m; r += DLU_PANEL_THREADS) {
            const double v = fabs(A[(long long)r * m + col]);
            if (v > best) {
                best = v;
                bi = r;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ov > best || (ov == best && oi < bi)) {
                best = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            rv[wv] = best;
            ri[wv] = bi;
        }
        __syncthreads();
        double bv = rv[0];
        int p = ri[0];
        for (int w = 1; w < DLU_PANEL_THREADS / 64; ++w)
            if (rv[w] > bv || (rv[w] == bv && ri[w] < p)) {
                bv = rv[w];
                p = ri[w];
            }
        if (tid == 0) {
            piv[col] = p;
            if (bv == 0.0 && info) atomicAdd(info, 1);
        }
        // interchange inside the panel columns, then the pivot row to LDS
        if (p != col && tid < nb) {
            const long long a = (long long)col * m + j0 + tid, b = (long long)p * m + j0 + tid;
            const double t = A[a];
            A[a] = A[b];
            A[b] = t;
        }
        __syncthreads();
        if (tid < nb - c) urow[tid] = A[(long long)col * m + col + tid];
        __syncthreads();
        const double d = urow[0];
        const double inv = d != 0.0 ? 1.0 / d : 0.0;
        for (int r = col + 1 + tid; r < m; r += DLU_PANEL_THREADS) {
            double *row = A + (long long)r * m;
            const double l = row[col] * inv;
            row[col] = l;
            for (int cc = 1; cc < nb - c; ++cc) row[col + cc] -= l * urow[cc];
        }
        __syncthreads();
    }
}

// the panel's interchanges on every column outside the panel, in order
__global__ void dlu_swap_kernel(double *__restrict__ A, int m, int j0, int nb, const int *__restrict__ piv)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m || (j >= j0 && j < j0 + nb)) return;
    for (int c = 0; c < nb; ++c) {
        const int r = j0 + c, p = piv[r];
        if (p != r) {
            const double t = A[(long long)r * m + j];
            A[(long long)r * m + j] = A[(long long)p * m + j];
            A[(long long)p * m + j] = t;
        }
    }
}

// U12 = L11^{-1} A12 (unit lower L11), one column per thread
__global__ void __launch_bounds__(256) dlu_trsm_kernel(double *__restrict__ A, int m, int j0, int nb)
{
    __shared__ double L[DLU_NB][DLU_NB + 1];
    for (int e = threadIdx.x; e < DLU_NB * DLU_NB; e += blockDim.x) {
        const int i = e / DLU_NB, k = e % DLU_NB;
        L[i][k] = i < nb && k < nb ? A[(long long)(j0 + i) * m + j0 + k] : 0.0;
    }
    __syncthreads();
    const int j = j0 + nb + blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    double u[DLU_NB];
#pragma unroll
    for (int c = 0; c < DLU_NB; ++c) u[c] = c < nb ? A[(long long)(j0 + c) * m + j] : 0.0;
#pragma unroll
    for (int c = 1; c < DLU_NB; ++c) {
        double sacc = u[c];
#pragma unroll
        for (int k = 0; k < c; ++k) sacc -= L[c][k] * u[k];
        if (c < nb) u[c] = sacc;
    }
#pragma unroll
    for (int c = 0; c < DLU_NB; ++c)
        if (c < nb) A[(long long)(j0 + c) * m + j] = u[c];
}

// A22 -= L21 U12 on 64 x 64 tiles, 4 x 4 outputs per thread
__global__ void __launch_bounds__(256) dlu_update_kernel(double *__restrict__ A, int m, int j0, int nb)
{
    __shared__ double Ls[DLU_TILE][DLU_NB + 1];
    __shared__ double Us[DLU_NB][DLU_TILE + 1];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int base = j0 + nb;
    const int r0 = base + blockIdx.y * DLU_TILE, c0 = base + blockIdx.x * DLU_TILE;
    for (int e = tid; e < DLU_TILE * DLU_NB; e += 256) {
        const int i = e / DLU_NB, k = e % DLU_NB, r = r0 + i;
        Ls[i][k] = r < m && k < nb ? A[(long long)r * m + j0 + k] : 0.0;
    }
    for (int e = tid; e < DLU_NB * DLU_TILE; e += 256) {
        const int k = e / DLU_TILE, jj = e % DLU_TILE, c = c0 + jj;
        Us[k][jj] = k < nb && c < m ? A[(long long)(j0 + k) * m + c] : 0.0;
    }
    __syncthreads();
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
#pragma unroll 4
    for (int k = 0; k < DLU_NB; ++k) {
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = Ls[ty + 16 * i][k];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = Us[k][tx + 16 * j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + ty + 16 * i, c = c0 + tx + 16 * j;
            if (r < m && c < m) A[(long long)r * m + c] -= acc[i][j];
        }
}

hipError_t launch_lu_dense(double *A, int *piv, int m, int *info, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    for (int j0 = 0; j0 < m; j0 += DLU_NB) {
        const int nb = min(DLU_NB, m - j0);
        hipLaunchKernelGGL(dlu_panel_kernel, dim3(1), dim3(DLU_PANEL_THREADS), 0, s, A, m, j0, nb, piv, info);
        hipLaunchKernelGGL(dlu_swap_kernel, dim3((m + 255) / 256), dim3(256), 0, s, A, m, j0, nb, (const int *)piv);
        const int rest = m - j0 - nb;
        if (rest > 0) {
            hipLaunchKernelGGL(dlu_trsm_kernel, dim3((rest + 255) / 256), dim3(256), 0, s, A, m, j0, nb);
            const int nt = (rest + DLU_TILE - 1) / DLU_TILE;
            hipLaunchKernelGGL(dlu_update_kernel, dim3(nt, nt), dim3(256), 0, s, A, m, j0, nb);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_dense_solve(const double *LU, const int *piv, int m, const double *rhs, double *x, int nout,
                              hipStream_t s)
{
    size_t bytes = ((size_t)((m + 1) & ~1) + 64 * 65) * sizeof(double);
    hipError_t e = lds_attr((const void *)dense_solve_kernel<double>, bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(dense_solve_kernel<double>, dim3(1), dim3(SV_THREADS), bytes, s, LU, piv, m, rhs, x, nout);
    return hipGetLastError();
}

hipError_t launch_identity(double *X, int n, hipStream_t s)
{
    hipLaunchKernelGGL(identity_kernel, dim3(256), dim3(256), 0, s, X, n);
    return hipGetLastError();
}

hipError_t launch_coarse_matrix(const double *Y, int n, int nb, int nt, long long pbase, long long Np1, int npm,
                                long long ncell, double *A, hipStream_t s)
{
    hipLaunchKernelGGL(coarse_matrix_kernel, dim3(256), dim3(256), 0, s, Y, n, nb, nt, pbase, Np1, npm, ncell, A);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_midpoint(const T *state, long long Nv1, int nt, const double *pm, T *vstar, hipStream_t s)
{
    T p[4] = {0, 0, 0, 0};
    for (int a = 0; a < nt && a < 4; ++a) p[a] = (T)pm[a];
    int th = 256;
    hipLaunchKernelGGL(midpoint_kernel<T>, dim3((unsigned)((Nv1 + th - 1) / th)), dim3(th), 0, s, state, Nv1, nt,
                       (const double *)nullptr, p[0], p[1], p[2], p[3], vstar);
    return hipGetLastError();
}

template hipError_t launch_elem<double>(int, int, int, const ElemArgs<double> &, int, hipStream_t);
template hipError_t launch_elem<float>(int, int, int, const ElemArgs<float> &, int, hipStream_t);
template hipError_t launch_patch<double, double>(int, int, const PatchArgs<double, double> &, int, hipStream_t);
template hipError_t launch_patch<float, float>(int, int, const PatchArgs<float, float> &, int, hipStream_t);
template hipError_t launch_patch<double, float>(int, int, const PatchArgs<double, float> &, int, hipStream_t);
template hipError_t launch_lu<double>(double *, int *, int, int, int *, size_t, hipStream_t, const LuBatch *, int);
template hipError_t launch_lu_queue<double>(double *, int *, const LuQueue &, size_t, int, int, int *, hipStream_t,
                                            int);
template hipError_t launch_lu_queue<float>(float *, int *, const LuQueue &, size_t, int, int, int *, hipStream_t, int);
template hipError_t launch_lu<float>(float *, int *, int, int, int *, size_t, hipStream_t, const LuBatch *, int);
template hipError_t launch_solve<double, double>(int, int, const SolveArgs<double, double> &, int, int, hipStream_t);
template hipError_t launch_solve<float, float>(int, int, const SolveArgs<float, float> &, int, int, hipStream_t);
template hipError_t launch_solve<double, float>(int, int, const SolveArgs<double, float> &, int, int, hipStream_t);
template hipError_t launch_patch_td<double, double>(int, int, const PatchTdArgs<double, double> &, int, hipStream_t);
template hipError_t launch_patch_td<float, float>(int, int, const PatchTdArgs<float, float> &, int, hipStream_t);
template hipError_t launch_lu_c<double>(double *, int *, int, int, long long, int, int *, size_t, hipStream_t);
template hipError_t launch_lu_c<float>(float *, int *, int, int, long long, int, int *, size_t, hipStream_t);
template hipError_t launch_solve_td<double, double>(int, int, const SolveTdArgs<double, double> &, int, int,
                                                    hipStream_t);
template hipError_t launch_solve_td<float, float>(int, int, const SolveTdArgs<float, float> &, int, int, hipStream_t);
template hipError_t launch_midpoint<double>(const double *, long long, int, const double *, double *, hipStream_t);
template hipError_t launch_midpoint<float>(const float *, long long, int, const double *, float *, hipStream_t);

} // namespace stmg
