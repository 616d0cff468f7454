"""Space-time error norms of slab solutions against the manufactured solution
of Sec. "Convergence test" (Table tab:conv-ns).

TEST INFRASTRUCTURE ONLY: used by tests/ to compare discrete solutions (from
the oracle or from the HIP library) with the exact fields and with the
errors the paper prints.

Definitions, summed over the slabs I_n = (t0, t0 + tau] of [0, T]:
    e_v^2   = int int |v_h - v|^2                    (L2(L2) velocity error)
    e_H1^2  = int int |v_h - v|^2 + |grad(v_h - v)|^2 (L2(H1) velocity error)
    e_div^2 = int int (div v_h)^2                    (L2(L2) divergence)
    e_p^2   = int int ((p_h - pbar_h) - (p - pbar))^2 (L2(L2) pressure error)
with pbar the spatial mean at each time (the pressure is fixed only up to a
constant when all of the boundary carries Dirichlet data).  Readings: the
L2(H1) error is the full H1 norm (value plus gradient); the discrete solution
in time is the DG(k) polynomial through the Radau node values,
v_h(t) = sum_a phi_a(t) V^a.

Integration: Gauss-Legendre with r+4 points per spatial direction on every
cell and k+3 points per slab in time (exact for the discrete parts, the error
of the exact parts is far below the discretization error).  Uniform Cartesian
2D meshes of the unit square only (the setting of the convergence test).
"""
from __future__ import annotations

import numpy as np
import sympy as sy

from . import manufactured as MS
from . import tables as T
from .core import Slab

_EXACT = None


def _exact():
    """Lambdified exact velocity, its gradient and the pressure."""
    global _EXACT
    if _EXACT is None:
        x, y, t = MS._x, MS._y, MS._t
        v = MS.V_EXPR
        grads = [[sy.diff(v[c], s) for s in (x, y)] for c in range(2)]
        fv = [sy.lambdify((x, y, t), vc, "numpy") for vc in v]
        fg = [[sy.lambdify((x, y, t), g, "numpy") for g in row] for row in grads]
        fp = sy.lambdify((x, y, t), MS.P_EXPR, "numpy")
        _EXACT = (fv, fg, fp)
    return _EXACT


def slab_errors(slab: Slab, U: np.ndarray, t0: float) -> dict:
    """Squared error contributions of one slab solution U (slab vector) on
    (t0, t0 + tau]: keys 'v', 'h1', 'div', 'p'."""
    prob, sp = slab.prob, slab.space
    if prob.dim != 2 or prob.vertices is not None:
        raise ValueError("2D Cartesian meshes only")
    r, k, tau = prob.r, prob.k, prob.tau
    n0, n1 = prob.n
    hx, hy = 1.0 / n0, 1.0 / n1
    N1 = r + 2
    nl = N1 * N1
    # spatial error points and 1D tables on [0, 1]
    qx, qw = T.gauss_legendre01(r + 4)
    S = T.lagrange_values(sp.gll, qx)          # [q, i]
    D = T.lagrange_derivatives(sp.gll, qx)     # [q, i], reference derivative
    L = T.legendre_orthonormal01(r, qx)        # [q, alpha]
    modes = sp.modes
    G = sp.dof_map()
    ncell = G.shape[0]
    cx = np.arange(ncell) % n0
    cy = np.arange(ncell) // n0
    # physical coordinates of the points [cell, qy, qx]
    X = (cx[:, None, None] + qx[None, None, :]) * hx + 0.0 * qx[None, :, None]
    Y = (cy[:, None, None] + qx[None, :, None]) * hy + 0.0 * qx[None, None, :]
    W = np.outer(qw, qw)[None] * hx * hy      # [1, qy, qx]
    area = float(np.sum(np.broadcast_to(W, X.shape)))
    # pressure basis at the points [m, qy, qx]
    Pb = np.array([np.outer(L[:, a1], L[:, a0]) for (a0, a1, _a2) in modes])
    # time points and the DG basis through the Radau nodes
    tg, tw = T.gauss_legendre01(k + 3)
    phi = T.lagrange_values(slab.tt.t / tau, tg)   # [tq, a]
    V, P = slab.split(np.asarray(U, dtype=np.float64))
    fv, fg, fp = _exact()
    out = {"v": 0.0, "h1": 0.0, "div": 0.0, "p": 0.0}
    gv = G[:, : 2 * nl]
    gp = G[:, 2 * nl:] - sp.Nv
    for tq in range(len(tg)):
        t = t0 + tau * tg[tq]
        wt = tau * tw[tq]
        Vt = phi[tq] @ V                       # [Nv]
        Pt = phi[tq] @ P                       # [Np]
        Vl = Vt[gv].reshape(ncell, 2, N1, N1)  # [cell, c, j (y), i (x)]
        Pl = Pt[gp]                            # [cell, m]
        vh = np.einsum("yj,xi,ncji->ncyx", S, S, Vl)
        dxh = np.einsum("yj,xi,ncji->ncyx", S, D, Vl) / hx
        dyh = np.einsum("yj,xi,ncji->ncyx", D, S, Vl) / hy
        ph = np.einsum("myx,nm->nyx", Pb, Pl)
        ev = [vh[:, c] - fv[c](X, Y, t) for c in range(2)]
        eg = [[dxh[:, c] - fg[c][0](X, Y, t), dyh[:, c] - fg[c][1](X, Y, t)] for c in range(2)]
        pe = np.broadcast_to(fp(X, Y, t), X.shape)
        pbar_h = float(np.sum(W * ph)) / area
        pbar = float(np.sum(W * pe)) / area
        ep = (ph - pbar_h) - (pe - pbar)
        div = dxh[:, 0] + dyh[:, 1]
        sv = float(np.sum(W * (ev[0] ** 2 + ev[1] ** 2)))
        sg = float(np.sum(W * sum(e ** 2 for row in eg for e in row)))
        out["v"] += wt * sv
        out["h1"] += wt * (sv + sg)
        out["div"] += wt * float(np.sum(W * div ** 2))
        out["p"] += wt * float(np.sum(W * ep ** 2))
    return out


def final_velocity(slab: Slab, U: np.ndarray) -> np.ndarray:
    """Velocity at the slab end t0 + tau: the right Radau rule has its last
    node there, so it is the last node's velocity block."""
    V, _ = slab.split(np.asarray(U))
    return np.array(V[-1])
