/*
 * Plain FP64 CPU oracle of the spatial forms of one space-time slab.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code,
 * header or table with the HIP library; all 1D tables are handed in by the
 * Python side of the oracle (oracle/tables.py).
 *
 * What is computed (per time node, i.e. for one spatial state):
 *
 *   residual   s(v,p)(z,q)  = <nu grad v - p I - v (x) v, grad z>
 *                            + <(v.n) v, z>_Gamma
 *                            - <(nu grad v - p I) n, z>_GD
 *                            - <(v.n)^- v, z>_GD
 *                            - <v, nu (grad z) n>_GD
 *                            + nu g1/h <v,z>_GD + g2/h <v.n, z.n>_GD
 *              continuity row (negated weak divergence, reading of the
 *              sign of B_h and G^p in the appendix on assembly):
 *                            - <div v, q> + <v.n, q>_GD
 *   (semilinear form A^tp_gamma of eq. def-a-gam-tp with B_gamma of
 *    eq. def-b-gam, convective form c of eq. Defc; g = 0 here, data enter
 *    through the right-hand side vector.)
 *
 *   Jacobian   the Gateaux derivative of the above at v in direction
 *              (xv, xp): eq. Defcp for the convective terms, and
 *              d/dy y^- = (sgn y - 1)/2 with sgn 0 = 0 for the inflow term.
 *
 *   mass       M_h (velocity) and M_h^p (pressure) of eq. DefMAB.
 *
 * Geometry: cells of a structured n0 x n1 (x n2) grid of [0,1]^d, each the
 * image of [0,1]^d under the multilinear map T_K through its 2^d vertices.
 * Velocity: Q_{r+1} Lagrange basis at Gauss-Lobatto points, pushed forward
 * by T_K (eq. Def:VKQK).  Pressure: mapped P_r^disc, orthonormal shifted
 * Legendre products of total degree <= r in reference coordinates.
 * h_{Gamma_D} of a boundary face = |K| / |F| (reading).
 *
 * Global numbering of one time node: velocity component c, node
 * (i0,i1,i2) on the ((r+1)n+1)^d grid, x fastest: c*Nn + i0 + N0*(i1 + N1*i2);
 * then pressure cell*npm + mode with cell = c0 + n0*(c1 + n1*c2).
 *
 * Integration is plain: every basis function is evaluated at every
 * quadrature point as a product of 1D values; no sum factorization.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int dim;            /* 2 or 3 */
    int n[3];           /* cells per direction */
    int r;              /* pressure degree; velocity degree r+1 */
    int nq;             /* Gauss points per direction */
    int npm;            /* number of pressure modes */
    int dmask;          /* bit f set: face f in Gamma_D (f = 2*axis + side) */
    double nu, gamma1, gamma2;
    const double *vert; /* ((n0+1)(n1+1)(n2+1)) x dim, NULL = Cartesian */
    const double *qw;   /* [nq] Gauss weights on [0,1] */
    const double *qx;   /* [nq] Gauss points on [0,1] */
    const double *S;    /* [nq][r+2] velocity 1D Lagrange values at Gauss points */
    const double *D;    /* [nq][r+2] their derivatives */
    const double *Se;   /* [2][r+2] values at s=0 and s=1 */
    const double *De;   /* [2][r+2] derivatives at s=0 and s=1 */
    const double *L;    /* [nq][r+1] orthonormal Legendre values at Gauss points */
    const double *Le;   /* [2][r+1] at s=0 and s=1 */
    const int *modes;   /* [npm][3] */
} ospace;

#define MAXN1 8      /* up to r = 6 */
#define MAXLOC (3 * MAXN1 * MAXN1 * MAXN1 + 100)

static int nnodes1(const ospace *s, int ax) { return (s->r + 1) * s->n[ax] + 1; }

static long nnodes(const ospace *s)
{
    long N = 1;
    for (int a = 0; a < s->dim; ++a) N *= nnodes1(s, a);
    return N;
}

static long ncells(const ospace *s)
{
    long N = 1;
    for (int a = 0; a < s->dim; ++a) N *= s->n[a];
    return N;
}

static int nloc1(const ospace *s)
{
    int n1 = s->r + 2, N = 1;
    for (int a = 0; a < s->dim; ++a) N *= n1;
    return N;
}

long orc_nv(const ospace *s) { return (long)s->dim * nnodes(s); }
long orc_np(const ospace *s) { return ncells(s) * s->npm; }
int orc_nloc(const ospace *s) { return s->dim * nloc1(s) + s->npm; }

/* cell index -> its coordinates */
static void cell_coords(const ospace *s, long cell, int cc[3])
{
    cc[0] = (int)(cell % s->n[0]);
    long rest = cell / s->n[0];
    cc[1] = s->dim > 1 ? (int)(rest % s->n[1]) : 0;
    cc[2] = s->dim > 2 ? (int)(rest / s->n[1]) : 0;
}

/* local-to-global map of a cell: velocity (c, l) then pressure modes */
static void cell_dofs(const ospace *s, long cell, long *g)
{
    int cc[3];
    cell_coords(s, cell, cc);
    int n1 = s->r + 2, nl = nloc1(s);
    long N0 = nnodes1(s, 0), N1 = s->dim > 1 ? nnodes1(s, 1) : 1;
    long Nn = nnodes(s);
    for (int l = 0; l < nl; ++l) {
        int i0 = l % n1, i1 = (l / n1) % n1, i2 = l / (n1 * n1);
        long gi0 = (long)(s->r + 1) * cc[0] + i0;
        long gi1 = (long)(s->r + 1) * cc[1] + i1;
        long gi2 = (long)(s->r + 1) * cc[2] + i2;
        long node = s->dim == 2 ? gi0 + N0 * gi1 : gi0 + N0 * (gi1 + N1 * gi2);
        for (int c = 0; c < s->dim; ++c) g[c * nl + l] = c * Nn + node;
    }
    long pbase = (long)s->dim * Nn;
    for (int m = 0; m < s->npm; ++m) g[s->dim * nl + m] = pbase + cell * s->npm + m;
}

/* vertex coordinates of a cell, X[v][dim], v = v0 + 2 v1 + 4 v2 */
static void cell_vertices(const ospace *s, long cell, double X[8][3])
{
    int cc[3];
    cell_coords(s, cell, cc);
    int nv = 1 << s->dim;
    for (int v = 0; v < nv; ++v) {
        int o[3] = {v & 1, (v >> 1) & 1, (v >> 2) & 1};
        long i0 = cc[0] + o[0], i1 = cc[1] + o[1], i2 = cc[2] + o[2];
        if (s->vert) {
            long idx = s->dim == 2 ? i0 + (s->n[0] + 1) * i1
                                   : i0 + (s->n[0] + 1) * (i1 + (long)(s->n[1] + 1) * i2);
            for (int a = 0; a < s->dim; ++a) X[v][a] = s->vert[idx * s->dim + a];
        } else {
            long ii[3] = {i0, i1, i2};
            for (int a = 0; a < s->dim; ++a) X[v][a] = (double)ii[a] / s->n[a];
        }
    }
}

/* Jacobian J[a][b] = d x_a / d xi_b of the multilinear map at xi */
static void map_jacobian(const ospace *s, double X[8][3], const double xi[3], double J[3][3])
{
    int d = s->dim, nv = 1 << d;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) J[a][b] = 0.0;
    for (int v = 0; v < nv; ++v) {
        int o[3] = {v & 1, (v >> 1) & 1, (v >> 2) & 1};
        double f[3], df[3];
        for (int b = 0; b < d; ++b) {
            f[b] = o[b] ? xi[b] : 1.0 - xi[b];
            df[b] = o[b] ? 1.0 : -1.0;
        }
        for (int b = 0; b < d; ++b) {
            double g = df[b];
            for (int e = 0; e < d; ++e)
                if (e != b) g *= f[e];
            for (int a = 0; a < d; ++a) J[a][b] += X[v][a] * g;
        }
    }
}

static void map_point(const ospace *s, double X[8][3], const double xi[3], double x[3])
{
    int d = s->dim, nv = 1 << d;
    for (int a = 0; a < 3; ++a) x[a] = 0.0;
    for (int v = 0; v < nv; ++v) {
        int o[3] = {v & 1, (v >> 1) & 1, (v >> 2) & 1};
        double f = 1.0;
        for (int b = 0; b < d; ++b) f *= o[b] ? xi[b] : 1.0 - xi[b];
        for (int a = 0; a < d; ++a) x[a] += X[v][a] * f;
    }
}

/* det and inverse transpose: Jit[a][b] = (J^{-1})[b][a] */
static double invert_transpose(int d, double J[3][3], double Jit[3][3])
{
    double det;
    if (d == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        Jit[0][0] = J[1][1] / det;
        Jit[0][1] = -J[1][0] / det;
        Jit[1][0] = -J[0][1] / det;
        Jit[1][1] = J[0][0] / det;
    } else {
        double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        double c10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        double c12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        double c20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        double c21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        /* cofactor matrix / det = J^{-T} */
        Jit[0][0] = c00 / det; Jit[0][1] = c01 / det; Jit[0][2] = c02 / det;
        Jit[1][0] = c10 / det; Jit[1][1] = c11 / det; Jit[1][2] = c12 / det;
        Jit[2][0] = c20 / det; Jit[2][1] = c21 / det; Jit[2][2] = c22 / det;
    }
    return det;
}

/* ------------------------------------------------------------------------
 * Evaluation points of a cell: volume Gauss points, then the Gauss points of
 * each boundary face (f = 2*axis + side).  For every point we hold the
 * physical gradients of all scalar velocity basis functions, their values,
 * the pressure mode values, the weight (JxW or dS), and for face points the
 * outward unit normal and the face kind.
 * --------------------------------------------------------------------- */
typedef struct {
    int nl;                     /* scalar velocity basis functions per cell */
    double N[MAXN1 * MAXN1 * MAXN1];
    double G[MAXN1 * MAXN1 * MAXN1][3];
    double psi[100];
    double wt;
    double nrm[3];
    int face;                   /* -1 volume, else face id */
} qpoint;

/* reference 1D values at a volume or face coordinate: idx >= 0 -> Gauss
 * point idx, idx = -1 -> s = 0, idx = -2 -> s = 1 */
static double vS(const ospace *s, int idx, int i)
{
    int n1 = s->r + 2;
    if (idx >= 0) return s->S[idx * n1 + i];
    return s->Se[(idx == -1 ? 0 : 1) * n1 + i];
}
static double vD(const ospace *s, int idx, int i)
{
    int n1 = s->r + 2;
    if (idx >= 0) return s->D[idx * n1 + i];
    return s->De[(idx == -1 ? 0 : 1) * n1 + i];
}
static double vL(const ospace *s, int idx, int i)
{
    int r1 = s->r + 1;
    if (idx >= 0) return s->L[idx * r1 + i];
    return s->Le[(idx == -1 ? 0 : 1) * r1 + i];
}
static double vxi(const ospace *s, int idx)
{
    if (idx >= 0) return s->qx[idx];
    return idx == -1 ? 0.0 : 1.0;
}

/* fill one evaluation point given per-axis 1D indices */
static void eval_point(const ospace *s, double X[8][3], const int idx[3], qpoint *P)
{
    int d = s->dim, n1 = s->r + 2;
    double xi[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) xi[a] = vxi(s, idx[a]);
    double J[3][3], Jit[3][3];
    map_jacobian(s, X, xi, J);
    double det = invert_transpose(d, J, Jit);
    P->nl = nloc1(s);
    for (int l = 0; l < P->nl; ++l) {
        int ii[3] = {l % n1, (l / n1) % n1, l / (n1 * n1)};
        double val = 1.0, gref[3];
        for (int a = 0; a < d; ++a) val *= vS(s, idx[a], ii[a]);
        for (int b = 0; b < d; ++b) {
            double g = 1.0;
            for (int a = 0; a < d; ++a) g *= (a == b) ? vD(s, idx[a], ii[a]) : vS(s, idx[a], ii[a]);
            gref[b] = g;
        }
        P->N[l] = val;
        for (int a = 0; a < d; ++a) {
            double g = 0.0;
            for (int b = 0; b < d; ++b) g += Jit[a][b] * gref[b];
            P->G[l][a] = g;
        }
    }
    for (int m = 0; m < s->npm; ++m) {
        double v = 1.0;
        for (int a = 0; a < d; ++a) v *= vL(s, idx[a], s->modes[3 * m + a]);
        P->psi[m] = v;
    }
    P->wt = det; /* caller multiplies by the reference weight */
    P->face = -1;
    /* stash J^{-T} rows for Nanson's formula in nrm (used by face points) */
    for (int a = 0; a < 3; ++a) P->nrm[a] = 0.0;
    (void)Jit;
}

/* Build the list of evaluation points of one cell.  Returns count; also the
 * cell volume.  pts must hold nq^d + 2d nq^(d-1) entries. */
static int cell_points(const ospace *s, long cell, qpoint *pts, double *volume)
{
    int d = s->dim, nq = s->nq;
    double X[8][3];
    cell_vertices(s, cell, X);
    int cc[3];
    cell_coords(s, cell, cc);
    int np = 0;
    double vol = 0.0;
    int nvol = 1;
    for (int a = 0; a < d; ++a) nvol *= nq;
    for (int q = 0; q < nvol; ++q) {
        int idx[3] = {q % nq, (q / nq) % nq, q / (nq * nq)};
        if (d == 2) idx[2] = 0;
        qpoint *P = &pts[np++];
        eval_point(s, X, idx, P);
        double w = 1.0;
        for (int a = 0; a < d; ++a) w *= s->qw[idx[a]];
        P->wt *= w;
        vol += P->wt;
    }
    *volume = vol;
    /* boundary faces of the domain that belong to this cell */
    int nfq = 1;
    for (int a = 0; a < d - 1; ++a) nfq *= nq;
    for (int ax = 0; ax < d; ++ax) {
        for (int side = 0; side < 2; ++side) {
            int onb = side == 0 ? (cc[ax] == 0) : (cc[ax] == s->n[ax] - 1);
            if (!onb) continue;
            int f = 2 * ax + side;
            for (int q = 0; q < nfq; ++q) {
                int idx[3], t = 0, qq = q;
                for (int a = 0; a < d; ++a) {
                    if (a == ax) idx[a] = side ? -2 : -1;
                    else { idx[a] = qq % nq; qq /= nq; ++t; }
                }
                if (d == 2) idx[2] = 0;
                qpoint *P = &pts[np++];
                eval_point(s, X, idx, P);
                /* Nanson: n dS = det J J^{-T} Nhat dShat */
                double xi[3] = {0, 0, 0};
                for (int a = 0; a < d; ++a) xi[a] = vxi(s, idx[a]);
                double J[3][3], Jit[3][3];
                map_jacobian(s, X, xi, J);
                double det = invert_transpose(d, J, Jit);
                double sgn = side ? 1.0 : -1.0, nv[3], len = 0.0;
                for (int a = 0; a < d; ++a) {
                    nv[a] = sgn * Jit[a][ax];
                    len += nv[a] * nv[a];
                }
                len = sqrt(len);
                double w = 1.0;
                for (int a = 0; a < d; ++a)
                    if (a != ax) w *= s->qw[idx[a]];
                P->wt = fabs(det) * len * w;
                for (int a = 0; a < d; ++a) P->nrm[a] = nv[a] / len;
                P->face = f;
            }
        }
    }
    return np;
}

static int max_points(const ospace *s)
{
    int d = s->dim, nq = s->nq, nv = 1, nf = 1;
    for (int a = 0; a < d; ++a) nv *= nq;
    for (int a = 0; a < d - 1; ++a) nf *= nq;
    return nv + 2 * d * nf;
}

/* Penalty length h_{Gamma_D} of face f (Nitsche penalty B^r_gamma, eq. def-b-gam):
 * the paper leaves it undefined.  Reading: the cell's normal extent |K|/|F|
 * divided by the square of the velocity degree r+1, the usual interior-penalty
 * scaling.  Without the degree factor the viscous Nitsche form with
 * gamma_1 = 10 is not coercive for Q4 velocities (its threshold is about
 * (r+1)^2 on Cartesian cells). */
static void face_h(const ospace *s, const qpoint *pts, int np, double vol, double hf[6])
{
    double area[6] = {0, 0, 0, 0, 0, 0};
    const double p2 = (double)(s->r + 1) * (double)(s->r + 1);
    for (int p = 0; p < np; ++p)
        if (pts[p].face >= 0) area[pts[p].face] += pts[p].wt;
    for (int f = 0; f < 2 * s->dim; ++f) hf[f] = area[f] > 0 ? vol / area[f] / p2 : 0.0;
}

static double ominus(double y) { return 0.5 * (fabs(y) - y); }
static double dominus(double y) { double sg = y > 0 ? 1.0 : (y < 0 ? -1.0 : 0.0); return 0.5 * (sg - 1.0); }

/* ------------------------------------------------------------------------
 * Element Jacobian (one time node) at the state given by local velocity
 * coefficients vloc[c*nl + l].  A is nloc x nloc, row = test, col = trial.
 * --------------------------------------------------------------------- */
static void element_jacobian(const ospace *s, long cell, const double *vloc, double *A, qpoint *pts)
{
    int d = s->dim, nl = nloc1(s), npm = s->npm, nloc = d * nl + npm;
    double nu = s->nu;
    memset(A, 0, sizeof(double) * nloc * nloc);
    double vol;
    int np = cell_points(s, cell, pts, &vol);
    double hf[6];
    face_h(s, pts, np, vol, hf);
    for (int p = 0; p < np; ++p) {
        const qpoint *P = &pts[p];
        double v[3] = {0, 0, 0};
        for (int c = 0; c < d; ++c)
            for (int l = 0; l < nl; ++l) v[c] += vloc[c * nl + l] * P->N[l];
        double w = P->wt;
        if (P->face < 0) {
            for (int i = 0; i < nl; ++i) {
                double vgi = 0.0;
                for (int a = 0; a < d; ++a) vgi += v[a] * P->G[i][a];
                for (int j = 0; j < nl; ++j) {
                    double gg = 0.0;
                    for (int a = 0; a < d; ++a) gg += P->G[j][a] * P->G[i][a];
                    double diag = nu * gg - P->N[j] * vgi;      /* viscous, -(xv (x) v):grad z */
                    for (int c = 0; c < d; ++c)
                        for (int e = 0; e < d; ++e) {
                            double val = -v[c] * P->N[j] * P->G[i][e]; /* -(v (x) xv):grad z */
                            if (c == e) val += diag;
                            A[(c * nl + i) * nloc + e * nl + j] += w * val;
                        }
                }
                for (int m = 0; m < npm; ++m)
                    for (int c = 0; c < d; ++c)
                        A[(c * nl + i) * nloc + d * nl + m] += w * (-P->psi[m] * P->G[i][c]);
            }
            for (int m = 0; m < npm; ++m)
                for (int j = 0; j < nl; ++j)
                    for (int e = 0; e < d; ++e)
                        A[(d * nl + m) * nloc + e * nl + j] += w * (-P->psi[m] * P->G[j][e]);
        } else {
            int isD = (s->dmask >> P->face) & 1;
            const double *n = P->nrm;
            double vn = 0.0;
            for (int a = 0; a < d; ++a) vn += v[a] * n[a];
            double h = hf[P->face];
            for (int i = 0; i < nl; ++i) {
                double Gni = 0.0;
                for (int a = 0; a < d; ++a) Gni += P->G[i][a] * n[a];
                for (int j = 0; j < nl; ++j) {
                    double Gnj = 0.0;
                    for (int a = 0; a < d; ++a) Gnj += P->G[j][a] * n[a];
                    double NN = P->N[j] * P->N[i];
                    for (int c = 0; c < d; ++c)
                        for (int e = 0; e < d; ++e) {
                            /* <(xv.n) v + (v.n) xv, z>_Gamma */
                            double val = n[e] * v[c] * NN;
                            if (c == e) val += vn * NN;
                            if (isD) {
                                if (c == e) {
                                    val += -nu * Gnj * P->N[i];          /* -(nu grad xv n).z */
                                    val += -ominus(vn) * NN;             /* -(v.n)^- xv.z */
                                    val += -nu * P->N[j] * Gni;          /* -nu xv.(grad z n) */
                                    val += nu * s->gamma1 / h * NN;      /* penalty */
                                }
                                val += -dominus(vn) * n[e] * v[c] * NN;  /* derivative of (v.n)^- */
                                val += s->gamma2 / h * n[e] * n[c] * NN;
                            }
                            A[(c * nl + i) * nloc + e * nl + j] += w * val;
                        }
                }
                if (isD)
                    for (int m = 0; m < npm; ++m)
                        for (int c = 0; c < d; ++c)
                            A[(c * nl + i) * nloc + d * nl + m] += w * P->psi[m] * n[c] * P->N[i];
            }
            if (isD)
                for (int m = 0; m < npm; ++m)
                    for (int j = 0; j < nl; ++j)
                        for (int e = 0; e < d; ++e)
                            A[(d * nl + m) * nloc + e * nl + j] += w * n[e] * P->N[j] * P->psi[m];
        }
    }
}

/* element residual (one time node) at local velocity vloc and pressure ploc */
static void element_residual(const ospace *s, long cell, const double *vloc, const double *ploc,
                             double *out, qpoint *pts)
{
    int d = s->dim, nl = nloc1(s), npm = s->npm, nloc = d * nl + npm;
    double nu = s->nu;
    memset(out, 0, sizeof(double) * nloc);
    double vol;
    int np = cell_points(s, cell, pts, &vol);
    double hf[6];
    face_h(s, pts, np, vol, hf);
    for (int p = 0; p < np; ++p) {
        const qpoint *P = &pts[p];
        double v[3] = {0, 0, 0}, g[3][3] = {{0}}, pr = 0.0;
        for (int c = 0; c < d; ++c)
            for (int l = 0; l < nl; ++l) {
                v[c] += vloc[c * nl + l] * P->N[l];
                for (int a = 0; a < d; ++a) g[c][a] += vloc[c * nl + l] * P->G[l][a];
            }
        for (int m = 0; m < npm; ++m) pr += ploc[m] * P->psi[m];
        double w = P->wt;
        if (P->face < 0) {
            /* flux F = nu grad v - p I - v (x) v, tested with grad z */
            double F[3][3];
            for (int c = 0; c < d; ++c)
                for (int a = 0; a < d; ++a) F[c][a] = nu * g[c][a] - v[c] * v[a] - (c == a ? pr : 0.0);
            for (int c = 0; c < d; ++c)
                for (int i = 0; i < nl; ++i) {
                    double t = 0.0;
                    for (int a = 0; a < d; ++a) t += F[c][a] * P->G[i][a];
                    out[c * nl + i] += w * t;
                }
            double div = 0.0;
            for (int a = 0; a < d; ++a) div += g[a][a];
            for (int m = 0; m < npm; ++m) out[d * nl + m] += w * (-div * P->psi[m]);
        } else {
            int isD = (s->dmask >> P->face) & 1;
            const double *n = P->nrm;
            double vn = 0.0, h = hf[P->face];
            for (int a = 0; a < d; ++a) vn += v[a] * n[a];
            double gn[3];
            for (int c = 0; c < d; ++c) {
                gn[c] = 0.0;
                for (int a = 0; a < d; ++a) gn[c] += g[c][a] * n[a];
            }
            for (int c = 0; c < d; ++c)
                for (int i = 0; i < nl; ++i) {
                    double Gni = 0.0;
                    for (int a = 0; a < d; ++a) Gni += P->G[i][a] * n[a];
                    double t = vn * v[c] * P->N[i];
                    if (isD) {
                        t += -nu * gn[c] * P->N[i] + pr * n[c] * P->N[i];
                        t += -ominus(vn) * v[c] * P->N[i];
                        t += -nu * v[c] * Gni;
                        t += nu * s->gamma1 / h * v[c] * P->N[i] + s->gamma2 / h * vn * n[c] * P->N[i];
                    }
                    out[c * nl + i] += w * t;
                }
            if (isD)
                for (int m = 0; m < npm; ++m) out[d * nl + m] += w * vn * P->psi[m];
        }
    }
}

/* element mass matrices: velocity (one scalar block, nl x nl) and pressure */
static void element_mass(const ospace *s, long cell, double *Mv, double *Mp, qpoint *pts)
{
    int nl = nloc1(s), npm = s->npm;
    memset(Mv, 0, sizeof(double) * nl * nl);
    memset(Mp, 0, sizeof(double) * npm * npm);
    double vol;
    int np = cell_points(s, cell, pts, &vol);
    for (int p = 0; p < np; ++p) {
        const qpoint *P = &pts[p];
        if (P->face >= 0) continue;
        for (int i = 0; i < nl; ++i)
            for (int j = 0; j < nl; ++j) Mv[i * nl + j] += P->wt * P->N[i] * P->N[j];
        for (int i = 0; i < npm; ++i)
            for (int j = 0; j < npm; ++j) Mp[i * npm + j] += P->wt * P->psi[i] * P->psi[j];
    }
}

static void gather_local(const ospace *s, const long *g, const double *V, const double *P,
                         double *vloc, double *ploc)
{
    int d = s->dim, nl = nloc1(s);
    long Mv = orc_nv(s);
    for (int i = 0; i < d * nl; ++i) vloc[i] = V[g[i]];
    if (ploc)
        for (int m = 0; m < s->npm; ++m) ploc[m] = P[g[d * nl + m] - Mv];
}

/* ======================================================================== */
/* exported entry points                                                     */
/* ======================================================================== */

/* local-to-global maps of all cells: G[cell][nloc] (spatial numbering) */
void orc_dof_map(const ospace *s, long *G)
{
    long nc = ncells(s);
    int nloc = orc_nloc(s);
    for (long c = 0; c < nc; ++c) cell_dofs(s, c, G + c * nloc);
}

/* all element Jacobians at velocity state V (spatial vector of one time
 * node, length Nv): A[cell][nloc][nloc] */
void orc_element_jacobians(const ospace *s, const double *V, double *A)
{
    long nc = ncells(s);
    int nloc = orc_nloc(s), mp = max_points(s);
#pragma omp parallel
    {
        qpoint *pts = (qpoint *)malloc(sizeof(qpoint) * mp);
        long g[MAXLOC];
        double vloc[MAXLOC];
#pragma omp for schedule(dynamic, 4)
        for (long c = 0; c < nc; ++c) {
            cell_dofs(s, c, g);
            gather_local(s, g, V, NULL, vloc, NULL);
            element_jacobian(s, c, vloc, A + c * (long)nloc * nloc, pts);
        }
        free(pts);
    }
}

/* element mass matrices: Mv[cell][nl][nl], Mp[cell][npm][npm] */
void orc_element_masses(const ospace *s, double *Mv, double *Mp)
{
    long nc = ncells(s);
    int nl = nloc1(s), npm = s->npm, mp = max_points(s);
#pragma omp parallel
    {
        qpoint *pts = (qpoint *)malloc(sizeof(qpoint) * mp);
#pragma omp for schedule(dynamic, 4)
        for (long c = 0; c < nc; ++c)
            element_mass(s, c, Mv + c * (long)nl * nl, Mp + c * (long)npm * npm, pts);
        free(pts);
    }
}

/* spatial residual of one time node: out (length Nv+Np) = s(V,P), assembled
 * cell by cell in cell order (deterministic). */
void orc_spatial_residual(const ospace *s, const double *V, const double *P, double *out)
{
    long nc = ncells(s), Nt = orc_nv(s) + orc_np(s);
    int nloc = orc_nloc(s), mp = max_points(s);
    double *loc = (double *)malloc(sizeof(double) * nc * nloc);
    long *G = (long *)malloc(sizeof(long) * nc * nloc);
#pragma omp parallel
    {
        qpoint *pts = (qpoint *)malloc(sizeof(qpoint) * mp);
        double vloc[MAXLOC], ploc[128];
#pragma omp for schedule(dynamic, 4)
        for (long c = 0; c < nc; ++c) {
            cell_dofs(s, c, G + c * nloc);
            gather_local(s, G + c * nloc, V, P, vloc, ploc);
            element_residual(s, c, vloc, ploc, loc + c * nloc, pts);
        }
        free(pts);
    }
    memset(out, 0, sizeof(double) * Nt);
    for (long c = 0; c < nc; ++c)
        for (int i = 0; i < nloc; ++i) out[G[c * nloc + i]] += loc[c * nloc + i];
    free(loc);
    free(G);
}

/* matrix-free spatial Jacobian action of one time node, by element matrices
 * applied cell by cell:  out = L(V) X,  X and out of length Nv+Np.
 * If Y != NULL, also  outm = M_h Y (velocity mass on Y's velocity part). */
void orc_spatial_action(const ospace *s, const double *V, const double *X, double *out,
                        const double *Y, double *outm)
{
    long nc = ncells(s), Nv = orc_nv(s), Nt = Nv + orc_np(s);
    int d = s->dim, nl = nloc1(s), nloc = orc_nloc(s), mp = max_points(s);
    double *loc = (double *)malloc(sizeof(double) * nc * nloc);
    double *locm = Y ? (double *)malloc(sizeof(double) * nc * d * nl) : NULL;
    long *G = (long *)malloc(sizeof(long) * nc * nloc);
#pragma omp parallel
    {
        qpoint *pts = (qpoint *)malloc(sizeof(qpoint) * mp);
        double *A = (double *)malloc(sizeof(double) * nloc * nloc);
        double *Mvv = (double *)malloc(sizeof(double) * nl * nl);
        double *Mpp = (double *)malloc(sizeof(double) * s->npm * s->npm);
        double vloc[MAXLOC], xloc[MAXLOC];
#pragma omp for schedule(dynamic, 4)
        for (long c = 0; c < nc; ++c) {
            long *g = G + c * nloc;
            cell_dofs(s, c, g);
            gather_local(s, g, V, NULL, vloc, NULL);
            element_jacobian(s, c, vloc, A, pts);
            for (int i = 0; i < nloc; ++i) xloc[i] = X[g[i]];
            for (int i = 0; i < nloc; ++i) {
                double t = 0.0;
                for (int j = 0; j < nloc; ++j) t += A[i * nloc + j] * xloc[j];
                loc[c * nloc + i] = t;
            }
            if (Y) {
                element_mass(s, c, Mvv, Mpp, pts);
                for (int e = 0; e < d; ++e)
                    for (int i = 0; i < nl; ++i) {
                        double t = 0.0;
                        for (int j = 0; j < nl; ++j) t += Mvv[i * nl + j] * Y[g[e * nl + j]];
                        locm[c * d * nl + e * nl + i] = t;
                    }
            }
        }
        free(pts);
        free(A);
        free(Mvv);
        free(Mpp);
    }
    memset(out, 0, sizeof(double) * Nt);
    for (long c = 0; c < nc; ++c)
        for (int i = 0; i < nloc; ++i) out[G[c * nloc + i]] += loc[c * nloc + i];
    if (Y) {
        memset(outm, 0, sizeof(double) * Nv);
        for (long c = 0; c < nc; ++c)
            for (int i = 0; i < d * nl; ++i) outm[G[c * nloc + i]] += locm[c * d * nl + i];
    }
    free(loc);
    free(locm);
    free(G);
}

/* The same action restricted to a list of cells: per-cell local results
 * loc[ic][nloc] (L(V)X) and locm[ic][d*nl] (M_h Y) with their maps.  Used to
 * evaluate sampled output rows at sizes where a full pass is too slow. */
void orc_cell_actions(const ospace *s, const double *V, const double *X, const double *Y,
                      long ncl, const long *cells, double *loc, double *locm, long *G)
{
    int d = s->dim, nl = nloc1(s), nloc = orc_nloc(s), mp = max_points(s);
#pragma omp parallel
    {
        qpoint *pts = (qpoint *)malloc(sizeof(qpoint) * mp);
        double *A = (double *)malloc(sizeof(double) * nloc * nloc);
        double *Mvv = (double *)malloc(sizeof(double) * nl * nl);
        double *Mpp = (double *)malloc(sizeof(double) * s->npm * s->npm);
        double vloc[MAXLOC], xloc[MAXLOC];
#pragma omp for schedule(dynamic, 1)
        for (long ic = 0; ic < ncl; ++ic) {
            long c = cells[ic];
            long *g = G + ic * nloc;
            cell_dofs(s, c, g);
            gather_local(s, g, V, NULL, vloc, NULL);
            element_jacobian(s, c, vloc, A, pts);
            for (int i = 0; i < nloc; ++i) xloc[i] = X[g[i]];
            for (int i = 0; i < nloc; ++i) {
                double t = 0.0;
                for (int j = 0; j < nloc; ++j) t += A[i * nloc + j] * xloc[j];
                loc[ic * nloc + i] = t;
            }
            element_mass(s, c, Mvv, Mpp, pts);
            for (int e = 0; e < d; ++e)
                for (int i = 0; i < nl; ++i) {
                    double t = 0.0;
                    for (int j = 0; j < nl; ++j) t += Mvv[i * nl + j] * Y[g[e * nl + j]];
                    locm[ic * d * nl + e * nl + i] = t;
                }
        }
        free(pts);
        free(A);
        free(Mvv);
        free(Mpp);
    }
}

/* physical coordinates of the volume Gauss points: xq[cell][q][dim] */
void orc_quadrature_points(const ospace *s, double *xq)
{
    long nc = ncells(s);
    int d = s->dim, nq = s->nq, nvol = 1;
    for (int a = 0; a < d; ++a) nvol *= nq;
    for (long c = 0; c < nc; ++c) {
        double X[8][3];
        cell_vertices(s, c, X);
        for (int q = 0; q < nvol; ++q) {
            int idx[3] = {q % nq, (q / nq) % nq, q / (nq * nq)};
            double xi[3] = {0, 0, 0}, x[3];
            for (int a = 0; a < d; ++a) xi[a] = s->qx[idx[a]];
            map_point(s, X, xi, x);
            for (int a = 0; a < d; ++a) xq[(c * nvol + q) * d + a] = x[a];
        }
    }
}

/* load vector <f, chi_i> from f given at the volume Gauss points fq[cell][q][dim] */
void orc_load_vector(const ospace *s, const double *fq, double *out)
{
    long nc = ncells(s);
    int d = s->dim, nl = nloc1(s), nloc = orc_nloc(s), mp = max_points(s);
    qpoint *pts = (qpoint *)malloc(sizeof(qpoint) * mp);
    long g[MAXLOC];
    memset(out, 0, sizeof(double) * orc_nv(s));
    int nvol = 1;
    for (int a = 0; a < d; ++a) nvol *= s->nq;
    for (long c = 0; c < nc; ++c) {
        cell_dofs(s, c, g);
        double vol;
        cell_points(s, c, pts, &vol);
        for (int q = 0; q < nvol; ++q)
            for (int e = 0; e < d; ++e)
                for (int i = 0; i < nl; ++i)
                    out[g[e * nl + i]] += pts[q].wt * fq[(c * nvol + q) * d + e] * pts[q].N[i];
    }
    (void)nloc;
    free(pts);
}

/* nodal coordinates of the velocity nodes (x fastest), computed through the
 * cell maps; the Gauss-Lobatto points are passed in gll[r+2]. */
void orc_node_coordinates(const ospace *s, const double *gll, double *xn)
{
    long nc = ncells(s);
    int d = s->dim, nl = nloc1(s), n1 = s->r + 2, nloc = orc_nloc(s);
    long g[MAXLOC];
    for (long c = 0; c < nc; ++c) {
        double X[8][3];
        cell_vertices(s, c, X);
        cell_dofs(s, c, g);
        for (int l = 0; l < nl; ++l) {
            int ii[3] = {l % n1, (l / n1) % n1, l / (n1 * n1)};
            double xi[3] = {0, 0, 0}, x[3];
            for (int a = 0; a < d; ++a) xi[a] = gll[ii[a]];
            map_point(s, X, xi, x);
            for (int a = 0; a < d; ++a) xn[g[l] * d + a] = x[a];
        }
    }
    (void)nloc;
}
