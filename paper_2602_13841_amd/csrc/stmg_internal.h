// Internal declarations of the stmg library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace stmg {

constexpr int MAX_K = 3;       // time degree k <= 3 (k+1 <= 4 Radau nodes)
constexpr int MAX_NT = MAX_K + 1;

struct TimeCoefs {
    int nt;
    double K[MAX_NT * MAX_NT];   // K[a*nt + b], reference slab (tau independent)
    double w[MAX_NT];            // diagonal of M_n^tau: tau/2 omega_a
    double phi0[MAX_NT];         // phi_a(t_{n-1}^+)
    double phimid[MAX_NT];       // phi_a(midpoint of I_n)
    double s[MAX_NT];            // Radau nodes on [0,1]
};

// Spectral splitting of the time coupling W^{-1} K of a midpoint-surrogate
// patch: nsys distinct eigen-systems (real eigenvalues first, then one
// member of each conjugate pair).  Patch solve: y_s = sum_a T[s][a] r_a,
// (lambda_s Mhat + Ahat) z_s = y_s, d_a = sum_s Re(F[a][s] z_s).
struct TimeDiag {
    int nsys;
    int cplx[MAX_NT];
    double lre[MAX_NT], lim[MAX_NT];
    double Tre[MAX_NT * MAX_NT], Tim[MAX_NT * MAX_NT];   // [s * MAX_NT + a]
    double Fre[MAX_NT * MAX_NT], Fim[MAX_NT * MAX_NT];   // [a * MAX_NT + s]
};

// host tables (tables.cpp)
void gauss_rule(int nq, std::vector<double> &x01, std::vector<double> &w01);
void lobatto_points(int npts, std::vector<double> &x01);
void radau_right(int k, std::vector<double> &x, std::vector<double> &w);
void lagrange_tables(const std::vector<double> &nodes, const std::vector<double> &pts,
                     std::vector<double> &L, std::vector<double> &dL);
void legendre01_table(int r, const std::vector<double> &pts, std::vector<double> &out);
std::vector<int> pressure_multi_indices(int r, int dim);
TimeCoefs time_coefficients(int k, double tau);
TimeDiag time_diagonalization(const TimeCoefs &tc);
std::vector<double> time_embedding(int kf, int kc);
int default_nq(int r);

enum class Mode : int { Jac = 0, Res = 1, Mass = 2 };

// Per-level discretization data visible to kernels.  Tables live in one
// device buffer per precision; offsets are fixed functions of (r, nq).
struct TableLayout {
    int n1 = 0, nq = 0, rp1 = 0;
    int S = 0, St = 0, D = 0, Dt = 0, Dq = 0, Dqt = 0, Se = 0, De = 0, L = 0, Lt = 0, Le = 0, qw = 0, qx = 0,
        total = 0;
    __host__ __device__ constexpr void init(int r, int nq_)
    {
        n1 = r + 2;
        nq = nq_;
        rp1 = r + 1;
        int o = 0;
        S = o;   o += nq * n1;
        St = o;  o += n1 * nq;
        D = o;   o += nq * n1;
        Dt = o;  o += n1 * nq;
        Dq = o;  o += nq * nq;
        Dqt = o; o += nq * nq;
        Se = o;  o += 2 * n1;
        De = o;  o += 2 * n1;
        L = o;   o += nq * rp1;
        Lt = o;  o += rp1 * nq;
        Le = o;  o += 2 * rp1;
        qw = o;  o += nq;
        qx = o;  o += nq;
        total = o;
    }
};

// host-side computation of the table block (in double)
std::vector<double> build_table_block(int r, int nq, const TableLayout &lay);

template <typename T>
struct CellArgs {
    int n0, n1, n2;          // cells per direction (n2 = 1 in 2D)
    int nt;                  // time nodes
    int ncell;
    long long Nn;            // velocity nodes per component
    long long Nv1;           // velocity unknowns per time node (d * Nn)
    long long Np1;           // pressure unknowns per time node
    long long Nslab;         // nt * (Nv1 + Np1)
    const T *x;              // slab vector input (Jac: direction; Res: iterate; Mass: x)
    const T *state;          // Jac: slab vector holding the state velocity
    const T *vprev;          // Res: velocity of one time node at t_{n-1} (may be null)
    const T *rhs;            // Res: slab right-hand side (may be null)
    T *E;                    // cell-local velocity results [cell][a][c][l]
    T *y;                    // slab output (pressure part written directly)
    const T *tab;            // table block
    const double *vert;      // vertex coordinates (null: Cartesian unit grid)
    int mapped;
    unsigned dmask;
    T nu, g1, g2;
    T K[MAX_NT * MAX_NT];
    T w[MAX_NT];
    T phi0[MAX_NT];
    long long xstride, ystride, sstride;   // batch strides (vectors along grid.y)
    const int *bcells;       // cells with a face on the domain boundary
    int nbcell;
};

template <typename T>
struct GatherArgs {
    int n0, n1, n2;
    int r;
    int nt;
    int dim;
    long long Nn, Nv1, Nslab;
    const T *E;
    const T *rhs;
    T *y;
    long long ystride;
    int nl;     // (r+2)^dim
    T alpha;        // y = alpha * sum (+ y if accumulate) (- rhs)
    int accumulate;
    int inv_mult;   // divide the sum by the number of cells holding the node
};

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2; give every XCD a contiguous range of cells so neighbouring cells (which
// share nodes) read through the same L2.  A bijection of [0, n).
__device__ __forceinline__ int xcd_cell(int b, int n)
{
    const int q = n >> 3, rem = n & 7, x = b & 7, k = b >> 3;
    return x * q + (x < rem ? x : rem) + k;
}

// launchers (cell_ops.hip)
template <typename T>
hipError_t launch_cell_op(Mode mode, int dim, int r, int nq, const CellArgs<T> &a, int nvec, hipStream_t s);
// boundary-face terms of the Jacobian / residual, added after launch_cell_op
template <typename T>
hipError_t launch_face_op(Mode mode, int dim, int r, int nq, const CellArgs<T> &a, int nvec, hipStream_t s);
template <typename T>
hipError_t launch_gather(const GatherArgs<T> &g, int nvec, hipStream_t s);
// 3D Jacobian: volume and boundary-face terms in one launch (replaces
// launch_cell_op + launch_face_op for Mode::Jac, dim 3)
template <typename T>
hipError_t launch_jac_fused_op(int r, int nq, const CellArgs<T> &a, int nvec, hipStream_t s);
bool jac_fuse_faces(int r, int nq, bool f64);

} // namespace stmg
