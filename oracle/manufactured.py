"""Manufactured 2D solution of Sec. "Convergence test" (test data only).

TEST INFRASTRUCTURE ONLY.

Reading: the printed velocity field is not divergence free; with the sign of
its second component flipped,
    v = sin t ( sin^2(pi x) sin(pi y) cos(pi y), -sin(pi x) cos(pi x) sin^2(pi y) ),
    p = sin t sin(pi x) cos(pi x) sin(pi y) cos(pi y),
v is divergence free, vanishes on the boundary of the unit square and at
t = 0, and p has zero mean.  The body force f = dv/dt + (v.grad) v - nu lap v
+ grad p is derived symbolically.  The slab load vector F_n^a =
w_a <f(t_a), chi> (eq. DefFn with the Radau rule) is assembled by the oracle.
"""
from __future__ import annotations

import numpy as np
import sympy as sy

from .core import Slab

_x, _y, _t, _nu = sy.symbols("x y t nu")
_pi = sy.pi
V_EXPR = (sy.sin(_t) * sy.sin(_pi * _x) ** 2 * sy.sin(_pi * _y) * sy.cos(_pi * _y),
          -sy.sin(_t) * sy.sin(_pi * _x) * sy.cos(_pi * _x) * sy.sin(_pi * _y) ** 2)
P_EXPR = sy.sin(_t) * sy.sin(_pi * _x) * sy.cos(_pi * _x) * sy.sin(_pi * _y) * sy.cos(_pi * _y)


def _force():
    v = V_EXPR
    f = []
    for c in range(2):
        conv = v[0] * sy.diff(v[c], _x) + v[1] * sy.diff(v[c], _y)
        lap = sy.diff(v[c], _x, 2) + sy.diff(v[c], _y, 2)
        gp = sy.diff(P_EXPR, (_x, _y)[c])
        f.append(sy.simplify(sy.diff(v[c], _t) + conv - _nu * lap + gp))
    return f


_F = None


def force(x, y, t, nu):
    global _F
    if _F is None:
        _F = [sy.lambdify((_x, _y, _t, _nu), fc, "numpy") for fc in _force()]
    return np.stack([np.broadcast_to(fn(x, y, t, nu), np.shape(x)) for fn in _F], axis=-1)


def velocity(x, y, t):
    fn = [sy.lambdify((_x, _y, _t), vc, "numpy") for vc in V_EXPR]
    return np.stack([np.broadcast_to(f(x, y, t), np.shape(x)) for f in fn], axis=-1)


def slab_rhs(slab: Slab, t0: float) -> np.ndarray:
    """Slab right-hand side: F^a = w_a <f(t0 + t_a), chi> for the velocity
    rows, zero continuity data (g = 0)."""
    sp_ = slab.space
    xq = sp_.quadrature_points()
    out = np.zeros(slab.N)
    for a in range(slab.nt):
        fq = force(xq[..., 0], xq[..., 1], t0 + slab.tt.t[a], slab.prob.nu)
        out[a * slab.Nv:(a + 1) * slab.Nv] = slab.tt.w[a] * sp_.load_vector(fq)
    return out
