"""Oracle of the hp space-time multigrid preconditioned Newton-FGMRES solver.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Plain numpy/scipy, FP64, following Sec. "Solution of the nonlinear system of
equations" and the algorithms of the appendix:

* hierarchy (Sec. "Multilevel hierarchies"): p-coarsening first,
  (k, r) -> (k//2 if k >= 2 else k, max(1, r//2)), then h-coarsening of the
  spatial mesh (n -> n/2) while every n is even and >= 4; coarser meshes take
  every second vertex of the finer one;
* grid transfers (Sec. "Grid transfer operators"): prolongation = canonical
  embedding, evaluated cell by cell in reference coordinates (space) and at
  the fine Radau nodes (time); restriction = its transpose;
* level states: the finer state evaluated at the coarser nodes (space) and
  Radau nodes (time); level operators rediscretized there;
* inexact space-time Vanka smoother (eq. LVS, eq. DefTildeHn, eq. vanka0):
  patch = all unknowns of one cell at all time nodes, local matrix = the
  principal submatrix of the midpoint-frozen surrogate Jacobian, LU with
  partial pivoting, additive sweep d += omega W sum_K R^T S^{-1} R (r - J d)
  with W = diag(1 / number of patches holding the unknown) (default) or
  W = I (literal plain sum, option);
* V-cycle with nu1 = nu2 = 1, coarsest level solved directly (bordered by
  the constant pressures of each time node when Gamma_D is the whole
  boundary);
* FGMRES, right preconditioned, Arnoldi in the M_n inner product with
  classical Gram-Schmidt and one reorthogonalization, Givens rotations,
  zero initial guess, no restart;
* inexact Newton with Eisenstat-Walker forcing, nonmonotone Armijo
  backtracking and smoother rebuild triggers (Alg. "Inexact Newton-Krylov",
  Alg. "Armijo").
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import comb

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import tables as T
from .core import Problem, Slab


# --------------------------------------------------------------------------
# hierarchy
# --------------------------------------------------------------------------
def level_specs(prob: Problem, max_levels: int = 0, time_coarsening: bool = False):
    """List of (k, r, n) from finest to coarsest (Sec. "Preconditioning of GMRES
    by hp-STMG", cycle and coarsening order): first p in space, r -> max(1,
    floor(r/2)); in time either k -> floor(k/2) with the spatial steps
    (time_coarsening, the order the paper states) or k kept on every level
    (default); then h while every n is even and >= 4."""
    specs = [(prob.k, prob.r, tuple(prob.n))]
    k, r, n = prob.k, prob.r, tuple(prob.n)
    while (r > 1 or (time_coarsening and k > 1)) and (max_levels == 0 or len(specs) < max_levels):
        r = max(1, r // 2)
        if time_coarsening:
            k = k // 2 if k >= 2 else k
        specs.append((k, r, n))
    while all(x % 2 == 0 and x >= 4 for x in n) and (max_levels == 0 or len(specs) < max_levels):
        n = tuple(x // 2 for x in n)
        specs.append((k, r, n))
    return specs


def coarse_vertices(vert, dim, n):
    """Every second vertex of a vertex array of an n-cell grid (x fastest)."""
    if vert is None:
        return None
    shape = tuple(x + 1 for x in n)[::-1] + (dim,)
    V = np.asarray(vert).reshape(shape)
    if dim == 2:
        return V[::2, ::2].reshape(-1, dim).copy()
    return V[::2, ::2, ::2].reshape(-1, dim).copy()


def _lattice_index(node, N):
    out = []
    for a in range(len(N)):
        out.append(node % N[a])
        node //= N[a]
    return out


def _locate(g, r, ncell):
    """Cell and Gauss-Lobatto local index of lattice coordinate g along one axis
    (a node on a cell interface is assigned to the cell above it, the last
    node to the last cell)."""
    c = g // (r + 1)
    loc = g - (r + 1) * c
    if c >= ncell:
        c, loc = ncell - 1, r + 1
    return c, loc


def velocity_prolongation(fine: Slab, coarse: Slab, kind: str) -> sp.csr_matrix:
    """Scalar-node matrix: fine node values of the coarse Q_{rc+1} field."""
    pf, pc = fine.prob, coarse.prob
    d = pf.dim
    glf = T.gauss_lobatto01(pf.r + 2)
    glc = T.gauss_lobatto01(pc.r + 2)
    Nf = [(pf.r + 1) * pf.n[a] + 1 for a in range(d)]
    Nc = [(pc.r + 1) * pc.n[a] + 1 for a in range(d)]
    # 1D maps: for each fine lattice coordinate, (coarse cell, coarse reference coordinate)
    per_axis = []
    for a in range(d):
        rows = []
        for g in range(Nf[a]):
            cf, lf = _locate(g, pf.r, pf.n[a])
            xi_f = glf[lf]
            if kind == "p":
                cc, xi_c = cf, xi_f
            else:
                cc, o = cf // 2, cf % 2
                xi_c = 0.5 * (o + xi_f)
            vals = T.lagrange_values(glc, [xi_c])[0]
            rows.append([((pc.r + 1) * cc + j, vals[j]) for j in range(pc.r + 2)])
        per_axis.append(rows)
    # tensor product
    rr, cc_, vv = [], [], []
    for node in range(int(np.prod(Nf))):
        gi = _lattice_index(node, Nf)
        entries = [(0, 1.0)]
        stride = 1
        for a in range(d):
            new = []
            for (ci, vi) in entries:
                for (gj, vj) in per_axis[a][gi[a]]:
                    new.append((ci + stride * gj, vi * vj))
            entries = new
            stride *= Nc[a]
        for (ci, vi) in entries:
            if vi != 0.0:
                rr.append(node)
                cc_.append(ci)
                vv.append(vi)
    return sp.csr_matrix((vv, (rr, cc_)), shape=(int(np.prod(Nf)), int(np.prod(Nc))))


def pressure_prolongation(fine: Slab, coarse: Slab, kind: str) -> sp.csr_matrix:
    pf, pc = fine.prob, coarse.prob
    d = pf.dim
    mf, mc = fine.space.modes, coarse.space.modes
    nf, nc = len(mf), len(mc)
    ncf = int(np.prod(pf.n))
    rows, cols, vals = [], [], []
    if kind == "p":
        # embedding P_rc in P_rf: same orthonormal functions
        for j, a in enumerate(mc):
            i = [ii for ii, b in enumerate(mf) if tuple(b) == tuple(a)][0]
            for cell in range(ncf):
                rows.append(cell * nf + i)
                cols.append(cell * nc + j)
                vals.append(1.0)
    else:
        gx, gw = T.gauss_legendre01(pf.r + 2)
        pts = np.stack(np.meshgrid(*([gx] * d), indexing="ij"), axis=-1).reshape(-1, d)
        wts = np.prod(np.stack(np.meshgrid(*([gw] * d), indexing="ij"), axis=-1).reshape(-1, d), axis=1)

        def psi(modes, r, x):
            L = [T.legendre_orthonormal01(r, x[:, a]) for a in range(d)]
            return np.stack([np.prod([L[a][:, m[a]] for a in range(d)], axis=0) for m in modes], axis=1)

        child = {}
        for o in np.ndindex(*(2,) * d):
            xc = (np.array(o)[None, :] + pts) / 2.0
            Mo = (psi(mf, pf.r, pts) * wts[:, None]).T @ psi(mc, pc.r, xc)     # [fine mode, coarse mode]
            child[o] = Mo
        for cell in range(ncf):
            cf = _lattice_index(cell, list(pf.n))
            o = tuple(x % 2 for x in cf)
            ccell = 0
            stride = 1
            for a in range(d):
                ccell += stride * (cf[a] // 2)
                stride *= pc.n[a]
            Mo = child[o]
            for i in range(nf):
                for j in range(nc):
                    if Mo[i, j] != 0.0:
                        rows.append(cell * nf + i)
                        cols.append(ccell * nc + j)
                        vals.append(Mo[i, j])
    return sp.csr_matrix((vals, (rows, cols)), shape=(fine.Np, coarse.Np))


def time_prolongation(kf, kc):
    """Pt[a, b] = phi^coarse_b(t^fine_a) on the reference slab."""
    tf = T.time_tables(kf, 1.0)
    tc = T.time_tables(kc, 1.0)
    return T.lagrange_values(tc.t, tf.t)


def slab_prolongation(fine: Slab, coarse: Slab, kind: str) -> sp.csr_matrix:
    d = fine.prob.dim
    Pn = velocity_prolongation(fine, coarse, kind)
    Pp = pressure_prolongation(fine, coarse, kind)
    Pt = sp.csr_matrix(time_prolongation(fine.prob.k, coarse.prob.k))
    Pv = sp.kron(Pt, sp.kron(sp.identity(d), Pn))
    Ppp = sp.kron(Pt, Pp)
    return sp.block_diag([Pv, Ppp], format="csr")


def state_interpolation(fine: Slab, coarse: Slab, kind: str) -> sp.csr_matrix:
    """Coarse velocity state (all time nodes) from the fine one: the fine field
    evaluated at the coarse nodes and Radau nodes."""
    pf, pc = fine.prob, coarse.prob
    d = pf.dim
    glf = T.gauss_lobatto01(pf.r + 2)
    glc = T.gauss_lobatto01(pc.r + 2)
    Nf = [(pf.r + 1) * pf.n[a] + 1 for a in range(d)]
    Nc = [(pc.r + 1) * pc.n[a] + 1 for a in range(d)]
    per_axis = []
    for a in range(d):
        rows = []
        for g in range(Nc[a]):
            cc, lc = _locate(g, pc.r, pc.n[a])
            xi_c = glc[lc]
            if kind == "p":
                cf, xi_f = cc, xi_c
            else:
                o = min(int(np.floor(2 * xi_c)), 1)
                cf, xi_f = 2 * cc + o, 2 * xi_c - o
            vals = T.lagrange_values(glf, [xi_f])[0]
            rows.append([((pf.r + 1) * cf + j, vals[j]) for j in range(pf.r + 2)])
        per_axis.append(rows)
    rr, cc_, vv = [], [], []
    for node in range(int(np.prod(Nc))):
        gi = _lattice_index(node, Nc)
        entries = [(0, 1.0)]
        stride = 1
        for a in range(d):
            new = []
            for (ci, vi) in entries:
                for (gj, vj) in per_axis[a][gi[a]]:
                    new.append((ci + stride * gj, vi * vj))
            entries = new
            stride *= Nf[a]
        for (ci, vi) in entries:
            if vi != 0.0:
                rr.append(node)
                cc_.append(ci)
                vv.append(vi)
    In = sp.csr_matrix((vv, (rr, cc_)), shape=(int(np.prod(Nc)), int(np.prod(Nf))))
    tf = T.time_tables(pf.k, 1.0)
    tc = T.time_tables(pc.k, 1.0)
    It = sp.csr_matrix(T.lagrange_values(tf.t, tc.t))          # [coarse b, fine a]
    return sp.kron(It, sp.kron(sp.identity(d), In), format="csr")


class Level:
    def __init__(self, slab: Slab):
        self.slab = slab
        self.state = None          # slab vector (velocity part used)
        self.J = None              # exact level Jacobian at the state (CSR)
        self.patches = None        # list of (indices, lu factors)
        self.coarse_lu = None


class Hierarchy:
    """hp-STMG hierarchy of one slab problem."""

    def __init__(self, prob: Problem, max_levels: int = 0, omega: float | None = None, weighting: int = 1,
                 time_coarsening: bool = False, diagonal: int = 0):
        self.prob = prob
        self.weighting = weighting
        self.diagonal = diagonal
        if omega is None:
            omega = 1.0 if weighting else default_omega(prob.dim)
        self.omega = omega
        specs = level_specs(prob, max_levels, time_coarsening)
        self.levels = []
        self.kinds = []
        vert = prob.vertices
        n_prev = tuple(prob.n)
        for i, (k, r, n) in enumerate(specs):
            if i > 0 and n != n_prev:
                vert = coarse_vertices(vert, prob.dim, n_prev)
                self.kinds.append("h")
            elif i > 0:
                self.kinds.append("p")
            nq = prob.nq if r == prob.r else T.default_nq(r)
            p = Problem(dim=prob.dim, n=n, r=r, k=k, nu=prob.nu, tau=prob.tau, nq=nq,
                        dirichlet_mask=prob.dirichlet_mask, gamma1=prob.gamma1, gamma2=prob.gamma2,
                        vertices=vert)
            self.levels.append(Level(Slab(p)))
            n_prev = n
        self.P = [slab_prolongation(self.levels[i].slab, self.levels[i + 1].slab, self.kinds[i])
                  for i in range(len(self.levels) - 1)]
        self.I = [state_interpolation(self.levels[i].slab, self.levels[i + 1].slab, self.kinds[i])
                  for i in range(len(self.levels) - 1)]
        d = prob.dim
        self.pure_dirichlet = prob.dirichlet_mask == (1 << (2 * d)) - 1

    # ---- set-up at a Newton state ----------------------------------------
    def set_state(self, U):
        """Level states and exact level Jacobians at U (finest slab vector)."""
        lv = self.levels
        lv[0].state = np.array(U, dtype=float)
        for i in range(1, len(lv)):
            fs = lv[i - 1].slab
            Vf = lv[i - 1].state[: fs.nt * fs.Nv]
            cs = lv[i].slab
            Vc = self.I[i - 1] @ Vf
            lv[i].state = np.concatenate([Vc, np.zeros(cs.nt * cs.Np)])
        for L in lv:
            L.J = L.slab.jacobian(L.state)
        self._coarse_factor()

    def rebuild_smoother(self):
        """Midpoint-frozen surrogate patches on every level but the coarsest."""
        for li in range(len(self.levels) - 1):
            self.build_patches(li)

    def build_patches(self, li):
        L = self.levels[li]
        s = L.slab
        V, _ = s.split(L.state)
        vstar = s.tt.phimid @ V                   # eq. DefVnAst
        Jt = s.jacobian(L.state, surrogate_state=vstar)
        mats = [Jt[idx][:, idx].toarray() for idx in patch_indices(s)]
        if self.diagonal:
            mats = [diagonal_velocity_block(s, A, self.diagonal == 2) for A in mats]
        L.patches = [(idx, sla.lu_factor(A)) for idx, A in zip(patch_indices(s), mats)]
        mult = np.zeros(s.N)
        for idx, _ in L.patches:
            mult[idx] += 1.0
        L.mult = mult

    def _coarse_factor(self):
        L = self.levels[-1]
        s = L.slab
        A = L.J.toarray()
        if self.pure_dirichlet:
            E = constant_pressure_vectors(s)
            n, m = A.shape[0], E.shape[1]
            B = np.zeros((n + m, n + m))
            B[:n, :n] = A
            B[:n, n:] = E
            B[n:, :n] = E.T
            A = B
        L.coarse_lu = sla.lu_factor(A)

    def coarse_solve(self, r):
        L = self.levels[-1]
        n = len(r)
        rhs = np.concatenate([r, np.zeros(L.coarse_lu[0].shape[0] - n)])
        return sla.lu_solve(L.coarse_lu, rhs)[:n]

    # ---- smoother and cycle ----------------------------------------------
    def smooth(self, li, r, d):
        """One additive Vanka sweep (eq. vanka0) on level li.  weighting = 1:
        each unknown's update is divided by the number of patches holding it
        (partition of unity) before the relaxation omega."""
        L = self.levels[li]
        defect = r - L.J @ d
        upd = np.zeros_like(d)
        for idx, lu in L.patches:
            upd[idx] += sla.lu_solve(lu, defect[idx])
        if self.weighting:
            upd = upd / L.mult
        return d + self.omega * upd

    def vcycle(self, r, li=0, nu1=1, nu2=1):
        if li == len(self.levels) - 1:
            return self.coarse_solve(r)
        L = self.levels[li]
        d = np.zeros_like(r)
        for _ in range(nu1):
            d = self.smooth(li, r, d)
        res = r - L.J @ d
        e = self.vcycle(self.P[li].T @ res, li + 1, nu1, nu2)
        d = d + self.P[li] @ e
        for _ in range(nu2):
            d = self.smooth(li, r, d)
        return d


def default_omega(dim: int) -> float:
    """Scalar relaxation of the plain additive sweep (eq. vanka0 with
    weighting = 0; the paper leaves omega open): 1.4 / 2^d, about 1.4 over
    the number of patches that share a vertex (fixed by a sweep on 2D and 3D
    test problems).  The default sweep (weighting = 1) instead divides each
    unknown's correction by the number of patches holding it, with omega = 1."""
    return 1.4 / (1 << dim)


def patch_indices(s: Slab):
    """Slab indices of each cell patch: velocity [a][c][local node], then
    pressure [a][mode]."""
    G = s.space.dof_map()
    d, nl, npm = s.prob.dim, s.space.nl, s.space.npm
    Nv, Np, nt = s.Nv, s.Np, s.nt
    out = []
    for cell in range(s.space.ncell):
        g = G[cell]
        vel = g[: d * nl]
        pre = g[d * nl:] - Nv
        idx = [a * Nv + vel for a in range(nt)] + [nt * Nv + a * Np + pre for a in range(nt)]
        out.append(np.concatenate(idx))
    return out


def diagonal_velocity_block(s: Slab, A, node_blocks: bool = False):
    """Diagonal Vanka (the cheaper smoother the paper's conclusions point to,
    after John's diagonal Vanka): in the patch matrix (velocity [a][c][node],
    then pressure [a][mode]) every velocity-velocity time block keeps only its
    spatial diagonal (same component and node), or with node_blocks the
    entries of the same node (all component pairs); the time coupling and the
    pressure blocks stay."""
    nl = s.space.nl
    nv = s.prob.dim * nl
    n = s.nt * nv
    vi = np.arange(n) % nv
    key = vi % nl if node_blocks else vi
    B = np.array(A, dtype=float)
    B[:n, :n] *= key[:, None] == key[None, :]
    return B


def constant_pressure_vectors(s: Slab):
    E = np.zeros((s.N, s.nt))
    for a in range(s.nt):
        base = s.nt * s.Nv + a * s.Np
        E[base + np.arange(s.space.ncell) * s.space.npm, a] = 1.0
    return E


# --------------------------------------------------------------------------
# FGMRES in the M inner product
# --------------------------------------------------------------------------
@dataclass
class GmresResult:
    x: np.ndarray
    its: int
    history: list
    converged: bool


def fgmres(Jop, Bop, Mop, b, rtol, maxit=50):
    """Right-preconditioned flexible GMRES, zero initial guess.  Arnoldi in
    <x,y>_M = x^T M y with classical Gram-Schmidt and one reorthogonalization;
    the Givens residual estimate is ||b - J x||_M.  Stops when it is
    <= rtol * ||b||_M or after maxit iterations."""
    r = b.copy()
    Mr = Mop(r)
    beta = np.sqrt(max(r @ Mr, 0.0))
    hist = [beta]
    if beta == 0.0:
        return GmresResult(np.zeros_like(b), 0, hist, True)
    V, MV, Z = [r / beta], [Mr / beta], []
    H = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    its = 0
    converged = False
    for j in range(maxit):
        z = Bop(V[j])
        Z.append(z)
        w = Jop(z)
        u = Mop(w)
        h = np.array([u @ V[i] for i in range(j + 1)])
        for i in range(j + 1):
            w = w - h[i] * V[i]
            u = u - h[i] * MV[i]
        h2 = np.array([u @ V[i] for i in range(j + 1)])
        for i in range(j + 1):
            w = w - h2[i] * V[i]
            u = u - h2[i] * MV[i]
        h = h + h2
        hn = np.sqrt(max(w @ u, 0.0))
        col = np.concatenate([h, [hn]])
        for i in range(j):
            t = cs[i] * col[i] + sn[i] * col[i + 1]
            col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1]
            col[i] = t
        den = np.hypot(col[j], col[j + 1])
        cs[j], sn[j] = (col[j] / den, col[j + 1] / den) if den > 0 else (1.0, 0.0)
        col[j] = cs[j] * col[j] + sn[j] * col[j + 1]
        col[j + 1] = 0.0
        H[: j + 2, j] = col
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        its = j + 1
        res = abs(g[j + 1])
        hist.append(res)
        if res <= rtol * beta or hn == 0.0:
            converged = res <= rtol * beta
            break
        V.append(w / hn)
        MV.append(u / hn)
    y = sla.solve_triangular(H[:its, :its], g[:its])
    x = np.zeros_like(b)
    for i in range(its):
        x = x + y[i] * Z[i]
    return GmresResult(x, its, hist, converged)


# --------------------------------------------------------------------------
# Newton (Alg. "Inexact Newton-Krylov") with Armijo (Alg. "Armijo")
# --------------------------------------------------------------------------
@dataclass
class NewtonParams:
    rtol: float = 1e-8
    atol: float = 1e-12
    maxit: int = 30
    eta0: float = 0.4
    c_eta: float = 0.5
    theta: float = 1.5
    eta_min: float = 1e-3
    eta_max: float = 0.8
    lambda0: float = 1.0
    c: float = 1e-4
    tau: float = 0.5
    alpha_min: float = 1e-3
    window: int = 5
    max_backtracks: int = 5
    theta_N: float = 0.5
    theta_L: float = 2.0
    kappa_abs: float = 10.0
    stag_s: int = 3
    stag_theta: float = 0.9
    fgmres_maxit: int = 50
    eps: float = 1e-30


@dataclass
class NewtonStats:
    newton_its: int = 0
    fgmres_its: list = field(default_factory=list)
    rebuilds: int = 0
    backtracks: int = 0
    res0: float = 0.0
    res: float = 0.0
    history: list = field(default_factory=list)
    etas: list = field(default_factory=list)
    alphas: list = field(default_factory=list)
    converged: bool = False


def forcing_term(eta_prev, res_norm, res_norm_prev, p: NewtonParams):
    """Eisenstat-Walker forcing term of the next linear solve (eq. ew): the
    ratio of the current to the previous residual M-norm (denominator kept
    above eps), raised to theta.  Reading: the factor c_eta multiplies the
    previous forcing term and the result is held in [eta_min, eta_max], the
    form the appendix's Newton algorithm states with the parameter names of
    Sec. "Numerical experiments"."""
    ratio = res_norm / max(res_norm_prev, p.eps)
    return float(np.clip(p.c_eta * eta_prev * ratio ** p.theta, p.eta_min, p.eta_max))


class MeritMemory:
    """The nonmonotone reference of the line search (Grippo-Lampariello-Lucidi,
    Sec. "Inexact Newton-Krylov method"): the largest of the last `size`
    accepted merit values of the slab's Newton iteration, seeded with the
    initial merit value; size 0 = the monotone rule (reference = phi(0))."""

    def __init__(self, phi_initial, size):
        self.size = size
        self.values = [phi_initial]

    def reference(self, phi0):
        return max(self.values) if self.size > 0 else phi0

    def remember(self, phi):
        if self.size > 0:
            self.values = (self.values + [phi])[-self.size:]


def model_minimizer(phi0, g0, failures):
    """Trial step from a polynomial model of the merit function along the
    Newton direction (reading: quadratic after the first rejected step,
    cubic after later ones).  The quadratic q(a) = phi0 + g0 a + b a^2 takes
    phi at the last rejected step; the cubic phi0 + g0 a + b a^2 + c a^3 takes
    phi at the last two rejected steps.  Returns the model's local minimizer,
    or None when the model has none (a concave quadratic, a singular fit, no
    real critical point)."""
    a1, p1 = failures[-1]
    if len(failures) == 1:
        curv = p1 - phi0 - g0 * a1                    # b a1^2
        if curv <= 0.0:
            return None
        return -g0 * a1 * a1 / (2.0 * curv)
    a2, p2 = failures[-2]
    # solve [a1^2 a1^3; a2^2 a2^3] [b; c] = [e1; e2] by Cramer's rule
    e1 = p1 - phi0 - g0 * a1
    e2 = p2 - phi0 - g0 * a2
    det = a1 * a1 * a2 * a2 * (a1 - a2)
    if det == 0.0:
        return None
    c3 = (a2 * a2 * e1 - a1 * a1 * e2) / det
    b2 = (a1 ** 3 * e2 - a2 ** 3 * e1) / det
    if c3 == 0.0:
        return -g0 / (2.0 * b2) if b2 > 0.0 else None
    # phi'(a) = g0 + 2 b a + 3 c a^2 = 0; the root where phi'' > 0
    disc = b2 * b2 - 3.0 * c3 * g0
    if disc < 0.0:
        return None
    return (-b2 + np.sqrt(disc)) / (3.0 * c3)


def line_search(phi, phi0, g0, memory: MeritMemory, p: NewtonParams):
    """Step length by the nonmonotone Armijo condition (eq. armijo against the
    remembered reference): the first trial is lambda0; a rejected step is
    replaced by the model minimizer held in [0.1 alpha, 0.5 alpha] (tau alpha
    when the model has none); after max_backtracks rejections, or once the
    step would fall to alpha_min, the step is alpha_min.  Returns (alpha,
    accepted merit value or None, number of rejected steps)."""
    alpha = p.lambda0
    failures = []
    while alpha > p.alpha_min:
        phit = phi(alpha)
        if phit <= memory.reference(phi0) + p.c * alpha * g0:
            memory.remember(phit)
            return alpha, phit, len(failures)
        failures.append((alpha, phit))
        if len(failures) > p.max_backtracks:
            break
        trial = model_minimizer(phi0, g0, failures)
        alpha = p.tau * alpha if trial is None or not np.isfinite(trial) else \
            min(max(trial, 0.1 * alpha), 0.5 * alpha)
    return p.alpha_min, None, len(failures)


def fgmres_stagnated(history, s, theta):
    """Stagnation of the FGMRES residual estimates: s consecutive ratios
    r_{j+1} / r_j of at least theta (the third rebuild criterion of the
    remark after Lemma "patch perturbation")."""
    run = 0
    for a, b in zip(history[:-1], history[1:]):
        if a <= 0:
            continue
        run = run + 1 if b / a >= theta else 0
        if run >= s:
            return True
    return False


class RebuildPolicy:
    """When the midpoint-frozen smoother is rebuilt (the criteria of the
    remark after Lemma "patch perturbation"; thresholds are reading S9).
    Before a Newton step: when none is built yet, on Newton deterioration
    (the last residual contraction rho >= theta_N) or on linear
    deterioration (the last FGMRES count kappa >= max(theta_L kappa_ref,
    kappa_abs), kappa_ref = the count recorded at the last rebuild of this
    kind).  After a step: when the step's FGMRES residuals stagnated."""

    def __init__(self, p: NewtonParams):
        self.p = p
        self.rho = 1.0
        self.kappa = 1
        self.kappa_ref = 1
        self.built = False

    def due_before_step(self):
        p = self.p
        return (not self.built) or self.rho >= p.theta_N or \
            self.kappa >= max(p.theta_L * self.kappa_ref, p.kappa_abs)

    def rebuilt_before_step(self):
        self.built = True
        self.kappa_ref = max(1, self.kappa)

    def record_step(self, res_norm, res_norm_prev, fgmres_its):
        self.rho = res_norm / max(res_norm_prev, self.p.eps)
        self.kappa = max(1, fgmres_its)

    def due_after_step(self, fgmres_history):
        return fgmres_stagnated(fgmres_history, self.p.stag_s, self.p.stag_theta)


def newton_solve(slab: Slab, hier: Hierarchy, U0, rhs=None, vprev=None, p: NewtonParams = NewtonParams(),
                 nu1=1, nu2=1):
    """Inexact Newton method for R_n(U; V_{n-1}) = 0 (Sec. "Inexact
    Newton-Krylov method"): the correction solves eq. lin-sys by FGMRES to
    the relative M-norm accuracy of eq. inexact with the forcing term of
    eq. ew, preconditioned by one hp-STMG V-cycle; the step length comes from
    the nonmonotone Armijo rule on phi(a) = 1/2 ||R(U + a dU)||_M^2 with
    phi'(0) = (M R)^T J dU (reading S6); the smoother follows RebuildPolicy.
    Stops when ||R||_M <= max(atol, rtol ||R_0||_M) or after maxit steps."""
    M = slab.slab_mass()
    U = np.array(U0, dtype=float)
    st = NewtonStats()

    def R(X):
        return slab.residual(X, rhs, vprev)

    def mnorm(v):
        return np.sqrt(max(v @ (M @ v), 0.0))

    r = R(U)
    res = mnorm(r)
    st.res0 = res
    st.history.append(res)
    target = max(p.atol, p.rtol * res)
    memory = MeritMemory(0.5 * res * res, p.window)
    policy = RebuildPolicy(p)
    eta, res_before = p.eta0, res
    while res > target and st.newton_its < p.maxit:
        hier.set_state(U)
        if policy.due_before_step():
            hier.rebuild_smoother()
            st.rebuilds += 1
            policy.rebuilt_before_step()
        if st.newton_its > 0:
            eta = forcing_term(eta, res, res_before, p)
        st.etas.append(eta)
        J = hier.levels[0].J
        lin = fgmres(lambda z: J @ z, lambda v: hier.vcycle(v, 0, nu1, nu2), lambda v: M @ v, -r, eta,
                     p.fgmres_maxit)
        dU = lin.x
        st.fgmres_its.append(lin.its)
        g0 = (M @ r) @ (J @ dU)
        alpha, _, nback = line_search(lambda a: 0.5 * mnorm(R(U + a * dU)) ** 2, 0.5 * res * res, g0, memory, p)
        st.backtracks += nback
        st.alphas.append(alpha)
        U = U + alpha * dU
        res_before = res
        r = R(U)
        res = mnorm(r)
        st.history.append(res)
        policy.record_step(res, res_before, lin.its)
        if policy.due_after_step(lin.history):
            hier.set_state(U)
            hier.rebuild_smoother()
            st.rebuilds += 1
        st.newton_its += 1
    st.res = res
    st.converged = res <= target
    return U, st
