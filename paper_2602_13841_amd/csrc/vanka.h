// Vanka smoother kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

namespace stmg {

template <typename T> struct ElemArgs {
    int n0, n1, n2;
    long long Nn;
    const T *vstar;        // midpoint velocity, one time node [c][node]
    const T *tab;          // table block of the level
    const double *vert;    // vertices or null
    int mapped;
    unsigned dmask;
    T nu, g1, g2;
    T *out;                // element records
    long long rec_words;
    const int *bcells;     // cells with a face on the domain boundary
    int nbcell;
};

template <typename TE, typename TP> struct PatchArgs {
    int n0, n1, n2;
    int nt;
    const TE *elem;
    long long rec_words;
    double K[16];
    double w[4];
    TP *patches;           // [cell][m*m] row-major
    int cell0;             // >= 0: assemble this cell only, into patches[0..m*m)
};

template <typename T, typename TP> struct SolveArgs {
    int n0, n1, n2;
    int nt;
    long long Nn, Nv1, Np1;
    const T *defect;       // slab vector
    const TP *patches;     // row-major LU factors
    const int *piv;
    T *E;                  // [cell][a][c][l] velocity part of the patch solution
    T *d;                  // slab vector: pressure part updated in place
    T omega;
};

// time-decoupled patches (one spatial matrix per eigen-system of the time
// coupling, ms rows of stride td_ld(ms); complex systems planar: real plane
// then imaginary plane)
template <typename TE, typename TP> struct PatchTdArgs {
    int n0, n1, n2;
    const TE *elem;
    long long rec_words;
    int nsys;
    int cplx[4];
    double lre[4], lim[4];
    TP *sys[4];            // per system: [cell][plane][ms][ms] row-major
};

// TF: storage type of the LU factors (TP, or unsigned short = BF16 bits of
// FP32 factors, widened to TP on load)
template <typename T, typename TP, typename TF = TP> struct SolveTdArgs {
    int n0, n1, n2;
    int nt;
    long long Nn, Nv1, Np1;
    const T *defect;
    int nsys;
    int cplx[4];
    const TF *sys[4];      // LU factors per system
    const int *perm[4];    // row permutation per system: [cell][ms]
    TP Tre[16], Tim[16];   // [s * 4 + a]
    TP Fre[16], Fim[16];   // [a * 4 + s]
    T *E;
    T *d;
    T omega;
};

// a batch of LU factorizations: uniform size m, or per-matrix sizes and
// offsets (elements of A, entries of the pivot array)
// row stride of the time-decoupled patch systems (elements): above 128
// unknowns every row starts on a 32-element boundary (128 bytes in FP32, 64 in
// the BF16 copy), so the 32-column blocks the substitutions read cover whole
// memory sectors instead of sharing their edge sectors with the neighbouring
// block; smaller systems stay unpadded (the padded form of their sweep needs
// more registers than it saves in bytes)
constexpr int td_ld(int ms) { return ms > 128 ? (ms + 31) & ~31 : ms; }

struct LuBatch {
    int uniform_m;
    const int *m_of;
    const long long *a_off;
    const long long *p_off;
    int uniform_ld;   // row stride of every matrix (0: its size m)
};

// a batch of LU factorizations taken from a device work queue by a fixed grid
// of workgroups (metadata sorted by decreasing size; counter zero at launch)
struct LuQueue {
    int batch;
    const int *m_of;          // matrix sizes
    const long long *a_off;   // element offsets of the matrices (row stride = size)
    const long long *p_off;   // offsets of their pivots
    const int *nb_of;         // panel width per matrix: 32, 16, 8 or 4
    int *counter;             // next queue position
};

// LDS bytes of one factorization of an m x m matrix with panel width nb
size_t lu_panel_lds_bytes(int nb, int m, bool f64);
// persistent launch: `grid` workgroups of `threads` (256 or 512) threads with
// `lds_bytes` of dynamic LDS each (>= lu_panel_lds_bytes of every matrix); op
// as for launch_lu
template <typename T>
hipError_t launch_lu_queue(T *A, int *piv, const LuQueue &q, size_t lds_bytes, int grid, int threads, int *info,
                           hipStream_t s, int op = 0);

int elem_record_words(int dim, int r);
template <typename T> hipError_t launch_elem(int dim, int r, int nq, const ElemArgs<T> &a, int ncell, hipStream_t s);
template <typename TE, typename TP>
hipError_t launch_patch(int dim, int r, const PatchArgs<TE, TP> &a, int ncell, hipStream_t s);
// m: the (largest) matrix size; vb: variable sizes (nullptr = all m x m,
// contiguous); op (FP32 only): operands of the trailing-update MFMA in FP32
// (0), BF16 (1) or FP16 (2), accumulation in FP32
template <typename T>
hipError_t launch_lu(T *A, int *piv, int m, int batch, int *info, size_t max_lds, hipStream_t s,
                     const LuBatch *vb = nullptr, int op = 0);
template <typename T, typename TP>
hipError_t launch_solve(int dim, int r, const SolveArgs<T, TP> &a, int ncell, int m, hipStream_t s);
template <typename TE, typename TP>
hipError_t launch_patch_td(int dim, int r, const PatchTdArgs<TE, TP> &a, int ncell, hipStream_t s);
// batched complex LU: matrix b at A + b * a_stride (real plane, imaginary plane)
template <typename T>
hipError_t launch_lu_c(T *A, int *piv, int m, int ld, long long a_stride, int batch, int *info, size_t max_lds,
                       hipStream_t s);
hipError_t launch_piv_to_perm(const int *piv, int *perm, int m, long long nmat, hipStream_t s);
size_t solve_td_lds_bytes(int ms, int nt, size_t word);
template <typename T, typename TP>
hipError_t launch_solve_td(int dim, int r, const SolveTdArgs<T, TP> &a, int ncell, int ms, hipStream_t s);
// the same with BF16-stored FP32 factors
hipError_t launch_solve_td_bf16(int dim, int r, const SolveTdArgs<float, float, unsigned short> &a, int ncell, int ms,
                                hipStream_t s);
// FP32 -> BF16 bits (round to nearest even), n elements
hipError_t launch_pack_bf16(const float *src, unsigned short *dst, long long n, hipStream_t s);

// diagonal Vanka on the time-decoupled patch systems: in every (possibly
// complex) spatial system of a cell the velocity-velocity block is replaced
// by its diagonal D (or its node blocks: all velocity components of one
// node), so the system is solved by the pressure Schur complement
// S = C - B D^{-1} B^T (npm x npm).  sys: the unfactored systems (ms x ms
// row-major with row stride td_ld(ms), planar complex); dinv: [cell][2][nv] D^{-1} (re, im); schur:
// [cell][2][npm npm] LU of S; spiv: [cell][npm] its row interchanges.
template <typename T> struct DvArgs {
    int n0, n1, n2;
    int nt;
    long long Nn, Nv1, Np1;
    const T *defect;
    int nsys;
    int cplx[4];
    const T *sys[4];
    T *dinv[4];
    T *schur[4];
    int *spiv[4];
    T Tre[16], Tim[16];    // [s * 4 + a]
    T Fre[16], Fim[16];    // [a * 4 + s]
    T *E;
    T *d;
    T omega;
    int *info;             // incremented per exactly zero Schur pivot (may be NULL)
    int block;             // 0: diagonal D; 1: DIM x DIM node blocks (all
                           // components of a node); dinv then [cell][2][nl][DIM][DIM]
};
template <typename T> hipError_t launch_dv_setup(int dim, int r, const DvArgs<T> &a, int ncell, hipStream_t s);
template <typename T> hipError_t launch_solve_dv(int dim, int r, const DvArgs<T> &a, int ncell, hipStream_t s);
// batched triangular solves with the factors of launch_lu (variable sizes:
// vb gives sizes and offsets; b_off the element offsets of the right-hand sides)
template <typename T>
hipError_t launch_batched_solve(const T *LU, const int *piv, int max_m, int batch, const LuBatch &vb,
                                const long long *b_off, T *b, hipStream_t s);
hipError_t launch_dense_solve(const double *LU, const int *piv, int m, const double *rhs, double *x, int nout,
                              hipStream_t s);
// LU with partial pivoting of one dense FP64 m x m matrix over the whole
// device (same format and pivots as launch_lu)
hipError_t launch_lu_dense(double *A, int *piv, int m, int *info, hipStream_t s);
hipError_t launch_identity(double *X, int n, hipStream_t s);
hipError_t launch_coarse_matrix(const double *Y, int n, int nb, int nt, long long pbase, long long Np1, int npm,
                                long long ncell, double *A, hipStream_t s);
template <typename T>
hipError_t launch_midpoint(const T *state, long long Nv1, int nt, const double *pm, T *vstar, hipStream_t s);

} // namespace stmg
