"""Plain FP64 oracle of one space-time slab: residual, Jacobian, mass.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of the benchmark, never by the product path.

The element integrals are computed by the C part (oracle/stmg_oracle.c,
plain loops, no sum factorization); this module holds the problem data,
hands the 1D tables to C and builds the space-time operators of Problem
LocAlgNS (eq. InAlgNS) and of the Jacobian (eq. JacobianLocal) with
scipy.sparse Kronecker products:

    R_v^a = sum_b K_ab M_h V^b + w_a s_v(V^a, P^a) - rhs_v^a - phi_a(0+) M_h v_prev
    R_p^a = w_a s_p(V^a)                            - rhs_p^a
    J     = [[K (x) M_h + blockdiag_a(w_a L_vv(V^a)), blockdiag_a(w_a L_vp)],
             [blockdiag_a(w_a L_pv),                  0                   ]]

where s and L are the spatial form of A^tp_gamma and its derivative at one
time node, w_a = tau/2 omega_a are the entries of the diagonal M_n^tau, and
the slab vector is ordered U = (V^1..V^{k+1}, P^1..P^{k+1}) (eq. DefSubvec).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from math import comb

import numpy as np
import scipy.sparse as sp

from . import tables as T

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stmg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", _LIB, _SRC, "-lm"])
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        sp_ = ctypes.c_void_p
        _lib.orc_nv.restype = ctypes.c_long
        _lib.orc_np.restype = ctypes.c_long
        _lib.orc_nloc.restype = ctypes.c_int
        for name in ("orc_nv", "orc_np", "orc_nloc"):
            getattr(_lib, name).argtypes = [sp_]
        _lib.orc_dof_map.argtypes = [sp_, lp]
        _lib.orc_element_jacobians.argtypes = [sp_, dp, dp]
        _lib.orc_element_masses.argtypes = [sp_, dp, dp]
        _lib.orc_spatial_residual.argtypes = [sp_, dp, dp, dp]
        _lib.orc_spatial_action.argtypes = [sp_, dp, dp, dp, dp, dp]
        _lib.orc_cell_actions.argtypes = [sp_, dp, dp, dp, ctypes.c_long, lp, dp, dp, lp]
        _lib.orc_quadrature_points.argtypes = [sp_, dp]
        _lib.orc_load_vector.argtypes = [sp_, dp, dp]
        _lib.orc_node_coordinates.argtypes = [sp_, dp, dp]
    return _lib


class _OSpace(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("r", ctypes.c_int),
                ("nq", ctypes.c_int), ("npm", ctypes.c_int), ("dmask", ctypes.c_int),
                ("nu", ctypes.c_double), ("gamma1", ctypes.c_double), ("gamma2", ctypes.c_double),
                ("vert", ctypes.c_void_p), ("qw", ctypes.c_void_p), ("qx", ctypes.c_void_p),
                ("S", ctypes.c_void_p), ("D", ctypes.c_void_p), ("Se", ctypes.c_void_p),
                ("De", ctypes.c_void_p), ("L", ctypes.c_void_p), ("Le", ctypes.c_void_p),
                ("modes", ctypes.c_void_p)]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _lp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


@dataclass
class Problem:
    """Data of one slab (Problem LocAlgNS): mesh, degrees, parameters."""
    dim: int
    n: tuple
    r: int
    k: int
    nu: float
    tau: float
    nq: int | None = None
    dirichlet_mask: int | None = None      # default: all faces Dirichlet
    gamma1: float = 10.0
    gamma2: float = 10.0
    vertices: np.ndarray | None = None      # ((n0+1)(n1+1)(n2+1), dim) or None

    def __post_init__(self):
        self.n = tuple(int(x) for x in self.n)[: self.dim]
        if self.nq is None:
            self.nq = T.default_nq(self.r)
        if self.dirichlet_mask is None:
            self.dirichlet_mask = (1 << (2 * self.dim)) - 1


class Space:
    """Spatial tables of a Problem plus the ctypes structure for the C part."""

    def __init__(self, prob: Problem):
        self.prob = prob
        d, r, nq = prob.dim, prob.r, prob.nq
        self.dim = d
        self.n1 = r + 2
        self.gll = T.gauss_lobatto01(r + 2)
        self.qx, self.qw = T.gauss_legendre01(nq)
        S = T.lagrange_values(self.gll, self.qx)
        D = T.lagrange_derivatives(self.gll, self.qx)
        Se = T.lagrange_values(self.gll, [0.0, 1.0])
        De = T.lagrange_derivatives(self.gll, [0.0, 1.0])
        L = T.legendre_orthonormal01(r, self.qx)
        Le = T.legendre_orthonormal01(r, [0.0, 1.0])
        self.modes = np.ascontiguousarray(T.pressure_modes(r, d))
        self.npm = len(self.modes)
        self._keep = [np.ascontiguousarray(a, dtype=np.float64) for a in (self.qw, self.qx, S, D, Se, De, L, Le)]
        vert = None
        if prob.vertices is not None:
            vert = np.ascontiguousarray(prob.vertices, dtype=np.float64)
            self._keep.append(vert)
        st = _OSpace()
        st.dim = d
        for a in range(3):
            st.n[a] = prob.n[a] if a < d else 1
        st.r = r
        st.nq = nq
        st.npm = self.npm
        st.dmask = prob.dirichlet_mask
        st.nu = prob.nu
        st.gamma1 = prob.gamma1
        st.gamma2 = prob.gamma2
        st.vert = vert.ctypes.data if vert is not None else None
        st.qw, st.qx, st.S, st.D, st.Se, st.De, st.L, st.Le = [a.ctypes.data for a in self._keep[:8]]
        st.modes = self.modes.ctypes.data
        self.st = st
        self.ref = ctypes.byref(st)
        self.Nv = lib().orc_nv(self.ref)
        self.Np = lib().orc_np(self.ref)
        self.nloc = lib().orc_nloc(self.ref)
        self.ncell = int(np.prod(prob.n))
        self.nnodes = self.Nv // d
        self.nl = self.n1 ** d

    # ---- maps and geometry ------------------------------------------------
    def dof_map(self) -> np.ndarray:
        G = np.zeros((self.ncell, self.nloc), dtype=np.int64)
        lib().orc_dof_map(self.ref, _lp(G))
        return G

    def node_coordinates(self) -> np.ndarray:
        xn = np.zeros((self.nnodes, self.dim))
        g = np.ascontiguousarray(self.gll)
        lib().orc_node_coordinates(self.ref, _dp(g), _dp(xn))
        return xn

    def quadrature_points(self) -> np.ndarray:
        nvol = self.prob.nq ** self.dim
        xq = np.zeros((self.ncell, nvol, self.dim))
        lib().orc_quadrature_points(self.ref, _dp(xq))
        return xq

    def load_vector(self, fq: np.ndarray) -> np.ndarray:
        fq = np.ascontiguousarray(fq, dtype=np.float64)
        out = np.zeros(self.Nv)
        lib().orc_load_vector(self.ref, _dp(fq), _dp(out))
        return out

    # ---- spatial forms of one time node -----------------------------------
    def spatial_residual(self, V: np.ndarray, P: np.ndarray) -> np.ndarray:
        V = np.ascontiguousarray(V, dtype=np.float64)
        P = np.ascontiguousarray(P, dtype=np.float64)
        out = np.zeros(self.Nv + self.Np)
        lib().orc_spatial_residual(self.ref, _dp(V), _dp(P), _dp(out))
        return out

    def element_jacobians(self, V: np.ndarray) -> np.ndarray:
        V = np.ascontiguousarray(V, dtype=np.float64)
        A = np.zeros((self.ncell, self.nloc, self.nloc))
        lib().orc_element_jacobians(self.ref, _dp(V), _dp(A))
        return A

    def spatial_jacobian(self, V: np.ndarray) -> sp.csr_matrix:
        """L(V) as a CSR matrix of size (Nv+Np)^2 assembled from element matrices."""
        A = self.element_jacobians(V)
        G = self.dof_map()
        rows = np.repeat(G, self.nloc, axis=1).ravel()
        cols = np.tile(G, (1, self.nloc)).ravel()
        n = self.Nv + self.Np
        M = sp.coo_matrix((A.ravel(), (rows, cols)), shape=(n, n)).tocsr()
        M.sum_duplicates()
        return M

    def spatial_action(self, V, X, Y=None):
        V = np.ascontiguousarray(V, dtype=np.float64)
        X = np.ascontiguousarray(X, dtype=np.float64)
        out = np.zeros(self.Nv + self.Np)
        if Y is None:
            lib().orc_spatial_action(self.ref, _dp(V), _dp(X), _dp(out), None, None)
            return out
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        outm = np.zeros(self.Nv)
        lib().orc_spatial_action(self.ref, _dp(V), _dp(X), _dp(out), _dp(Y), _dp(outm))
        return out, outm

    def cell_actions(self, V, X, Y, cells):
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        ncl = len(cells)
        loc = np.zeros((ncl, self.nloc))
        locm = np.zeros((ncl, self.dim * self.nl))
        G = np.zeros((ncl, self.nloc), dtype=np.int64)
        lib().orc_cell_actions(self.ref, _dp(np.ascontiguousarray(V, dtype=np.float64)),
                               _dp(np.ascontiguousarray(X, dtype=np.float64)),
                               _dp(np.ascontiguousarray(Y, dtype=np.float64)),
                               ncl, _lp(cells), _dp(loc), _dp(locm), _lp(G))
        return loc, locm, G

    def masses(self):
        """(M_h for all d components, M_h^p) as CSR matrices (eq. DefMAB)."""
        nl, npm = self.nl, self.npm
        Mv = np.zeros((self.ncell, nl, nl))
        Mp = np.zeros((self.ncell, npm, npm))
        lib().orc_element_masses(self.ref, _dp(Mv), _dp(Mp))
        G = self.dof_map()
        blocks = []
        rows, cols, vals = [], [], []
        for c in range(self.dim):
            g = G[:, c * nl:(c + 1) * nl]
            rows.append(np.repeat(g, nl, axis=1).ravel())
            cols.append(np.tile(g, (1, nl)).ravel())
            vals.append(Mv.ravel())
        Mh = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                           shape=(self.Nv, self.Nv)).tocsr()
        gp = G[:, self.dim * nl:] - self.Nv
        Mhp = sp.coo_matrix((Mp.ravel(), (np.repeat(gp, npm, axis=1).ravel(), np.tile(gp, (1, npm)).ravel())),
                            shape=(self.Np, self.Np)).tocsr()
        del blocks
        return Mh, Mhp


class Slab:
    """One space-time slab: Space + time tables + slab operators."""

    def __init__(self, prob: Problem):
        self.prob = prob
        self.space = Space(prob)
        self.tt = T.time_tables(prob.k, prob.tau)
        self.nt = prob.k + 1
        self.Nv = self.space.Nv
        self.Np = self.space.Np
        self.N = self.nt * (self.Nv + self.Np)
        self._mass = None

    @property
    def mass(self):
        if self._mass is None:
            self._mass = self.space.masses()
        return self._mass

    # ---- slab vector helpers ---------------------------------------------
    def split(self, U):
        nt, Nv, Np = self.nt, self.Nv, self.Np
        V = U[: nt * Nv].reshape(nt, Nv)
        P = U[nt * Nv:].reshape(nt, Np)
        return V, P

    def join(self, V, P):
        return np.concatenate([np.asarray(V).ravel(), np.asarray(P).ravel()])

    # ---- eq. InAlgNS -------------------------------------------------------
    def residual(self, U, rhs=None, vprev=None):
        V, P = self.split(U)
        K, w, phi0 = self.tt.K, self.tt.w, self.tt.phi0
        Mh, _ = self.mass
        MV = np.array([Mh @ V[b] for b in range(self.nt)])
        Rv = np.zeros_like(V)
        Rp = np.zeros_like(P)
        for a in range(self.nt):
            s = self.space.spatial_residual(V[a], P[a])
            Rv[a] = K[a] @ MV + w[a] * s[: self.Nv]
            Rp[a] = w[a] * s[self.Nv:]
            if vprev is not None:
                Rv[a] -= phi0[a] * (Mh @ vprev)
        R = self.join(Rv, Rp)
        if rhs is not None:
            R = R - rhs
        return R

    # ---- eq. JacobianLocal, explicit sparse matrix -------------------------
    def jacobian(self, U, surrogate_state=None) -> sp.csr_matrix:
        """Explicit CSR space-time Jacobian at U.  If surrogate_state is given
        (a velocity vector of one time node), every time node uses it as the
        state: this is the midpoint surrogate of eq. DefTildeHn."""
        V, _ = self.split(U)
        nt, Nv, Np = self.nt, self.Nv, self.Np
        K, w = self.tt.K, self.tt.w
        Mh, _ = self.mass
        Lvv, Lvp, Lpv = [], [], []
        cache = {}
        for a in range(nt):
            state = V[a] if surrogate_state is None else surrogate_state
            key = id(surrogate_state) if surrogate_state is not None else a
            if key not in cache:
                cache[key] = self.space.spatial_jacobian(state)
            L = cache[key]
            Lvv.append(w[a] * L[:Nv, :Nv])
            Lvp.append(w[a] * L[:Nv, Nv:])
            Lpv.append(w[a] * L[Nv:, :Nv])
        Jvv = sp.kron(sp.csr_matrix(K), Mh) + sp.block_diag(Lvv)
        Jvp = sp.block_diag(Lvp)
        Jpv = sp.block_diag(Lpv)
        J = sp.bmat([[Jvv, Jvp], [Jpv, None]], format="csr")
        J.sum_duplicates()
        return J

    def slab_mass(self) -> sp.csr_matrix:
        """The weight matrix of the M-norm of eq. inexact:
        blockdiag(M^tau (x) M_h, M^tau (x) M_h^p)."""
        Mh, Mhp = self.mass
        Mt = sp.csr_matrix(self.tt.M)
        return sp.block_diag([sp.kron(Mt, Mh), sp.kron(Mt, Mhp)], format="csr")

    def vmult(self, U, X):
        """y = J(U) x evaluated element by element without forming J."""
        V, _ = self.split(U)
        Xv, Xp = self.split(X)
        nt, Nv = self.nt, self.Nv
        K, w = self.tt.K, self.tt.w
        Yv = np.zeros((nt, Nv))
        Yp = np.zeros((nt, self.Np))
        for a in range(nt):
            mix = K[a] @ Xv                       # sum_b K_ab x^b
            Xa = np.concatenate([Xv[a], Xp[a]])
            out, outm = self.space.spatial_action(V[a], Xa, mix)
            Yv[a] = outm + w[a] * out[:Nv]
            Yp[a] = w[a] * out[Nv:]
        return self.join(Yv, Yp)

    def vmult_rows(self, U, X, rows):
        """Selected entries of y = J(U) x, each from the element contributions
        of the cells that hold the row's degree of freedom."""
        rows = np.asarray(rows, dtype=np.int64)
        V, _ = self.split(U)
        Xv, Xp = self.split(X)
        nt, Nv, Np = self.nt, self.Nv, self.Np
        K, w = self.tt.K, self.tt.w
        sp_ = self.space
        # decode rows into (time node a, spatial index)
        out = np.zeros(len(rows))
        G_all_cells = None
        need = {}
        for i, g in enumerate(rows):
            if g < nt * Nv:
                a, loc = divmod(int(g), Nv)
            else:
                a, loc = divmod(int(g) - nt * Nv, Np)
                loc += Nv
            need.setdefault(a, []).append((i, loc))
        for a, items in need.items():
            cells = set()
            for _, loc in items:
                cells.update(self._cells_of(loc))
            cells = np.array(sorted(cells), dtype=np.int64)
            mix = K[a] @ Xv
            Xa = np.concatenate([Xv[a], Xp[a]])
            loc_, locm, G = sp_.cell_actions(V[a], Xa, mix, cells)
            for i, l in items:
                val = 0.0
                for ic in range(len(cells)):
                    hit = np.nonzero(G[ic] == l)[0]
                    for h in hit:
                        val += w[a] * loc_[ic, h]
                        if h < sp_.dim * sp_.nl:
                            val += locm[ic, h]
                out[i] = val
        del G_all_cells
        return out

    def _cells_of(self, loc):
        """Cells whose local map contains spatial index loc."""
        sp_ = self.space
        prob = self.prob
        d = prob.dim
        if loc >= sp_.Nv:
            return [(loc - sp_.Nv) // sp_.npm]
        node = loc % sp_.nnodes
        Nn = [(prob.r + 1) * prob.n[a] + 1 for a in range(d)]
        idx = []
        for a in range(d):
            idx.append(node % Nn[a])
            node //= Nn[a]
        cand = []
        for a in range(d):
            i = idx[a]
            c = i // (prob.r + 1)
            opts = {min(c, prob.n[a] - 1)}
            if i % (prob.r + 1) == 0 and c > 0:
                opts.add(c - 1)
            cand.append(sorted(opts))
        cells = []
        if d == 2:
            for c1 in cand[1]:
                for c0 in cand[0]:
                    cells.append(c0 + prob.n[0] * c1)
        else:
            for c2 in cand[2]:
                for c1 in cand[1]:
                    for c0 in cand[0]:
                        cells.append(c0 + prob.n[0] * (c1 + prob.n[1] * c2))
        return cells


def dof_count(dim: int, n: int, r: int, k: int) -> int:
    """Space-time unknowns of one slab: (k+1)[d((r+1)n+1)^d + C(r+d,d) n^d]."""
    return (k + 1) * (dim * ((r + 1) * n + 1) ** dim + comb(r + dim, dim) * n ** dim)
