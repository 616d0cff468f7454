"""One-dimensional tables of the space-time discretization (oracle side).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
module; it exists so that the tests, the smoke check and the CPU baseline of
the benchmark can compare the HIP library against a plain FP64 definition.

Everything here is computed straight from its definition with numpy
polynomial routines (library primitives), in float64:

* right-sided Gauss-Radau rule on [-1, 1] with k+1 points, last node +1,
  exact for polynomials of degree 2k (Sec. "Preliminaries", eq. GF);
* Lagrange basis in time at the Radau nodes (eq. BasYk) and the time
  matrices K, M, C of the appendix on assembly (eq. DefKMC);
* Gauss-Lobatto points (velocity nodes of Q_{r+1}) and Gauss-Legendre rules;
* the orthonormal shifted Legendre basis used for the mapped P_r^disc
  pressure (reading: orthonormal on the unit reference cube, total degree
  <= r, multi-indices ordered lexicographically with the first index
  fastest).
"""
from __future__ import annotations

from fractions import Fraction
from math import comb

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


# --------------------------------------------------------------------------
# quadrature rules
# --------------------------------------------------------------------------
def gauss_legendre01(nq: int):
    """Gauss-Legendre rule with nq points mapped from [-1,1] to [0,1]."""
    x, w = npleg.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto01(npts: int) -> np.ndarray:
    """Gauss-Lobatto points on [0,1]: the end points and the roots of P'_{npts-1}."""
    N = npts - 1
    if N < 1:
        raise ValueError("need at least two Lobatto points")
    inner = npleg.Legendre.basis(N).deriv().roots() if N >= 2 else np.array([])
    x = np.concatenate(([-1.0], np.sort(np.real(inner)), [1.0]))
    return 0.5 * (x + 1.0)


def radau_right(k: int):
    """Right-sided (k+1)-point Gauss-Radau rule on [-1,1] (eq. GF).

    Nodes: the roots of P_{k+1} - P_k (these include +1).  Weights: the
    integrals of the Lagrange polynomials through the nodes, integrated
    exactly with a Gauss-Legendre rule of sufficient degree.
    """
    n = k + 1
    c = np.zeros(n + 1)
    c[n] = 1.0
    c[n - 1] = -1.0
    x = np.sort(np.real(npleg.legroots(c)))
    x[-1] = 1.0
    gx, gw = npleg.leggauss(n + 2)
    w = np.array([np.sum(gw * lagrange_values(x, gx)[:, i]) for i in range(n)])
    return x, w


# --------------------------------------------------------------------------
# Lagrange bases
# --------------------------------------------------------------------------
def lagrange_values(nodes: np.ndarray, x) -> np.ndarray:
    """L[p, j] = ell_j(x_p) for the Lagrange polynomials through `nodes`."""
    x = np.atleast_1d(np.asarray(x, dtype=float))
    n = len(nodes)
    L = np.ones((len(x), n))
    for j in range(n):
        for m in range(n):
            if m != j:
                L[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return L


def lagrange_derivatives(nodes: np.ndarray, x) -> np.ndarray:
    """D[p, j] = ell_j'(x_p), by differentiating the power-form polynomial."""
    x = np.atleast_1d(np.asarray(x, dtype=float))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for j in range(n):
        coef = np.array([1.0])
        for m in range(n):
            if m != j:
                coef = nppoly.polymul(coef, np.array([-nodes[m], 1.0]) / (nodes[j] - nodes[m]))
        D[:, j] = nppoly.polyval(x, nppoly.polyder(coef))
    return D


# --------------------------------------------------------------------------
# time matrices of one slab (appendix on assembly, eq. DefKMC)
# --------------------------------------------------------------------------
class TimeTables:
    """Radau rule, Lagrange basis and K, M, C for DG(k) on I_n = (0, tau]."""

    def __init__(self, k: int, tau: float):
        self.k = k
        self.tau = float(tau)
        that, what = radau_right(k)
        self.that = that                           # reference nodes on [-1,1]
        self.what = what                           # reference weights
        self.nodes01 = 0.5 * (that + 1.0)          # nodes on [0,1]
        self.t = self.tau * self.nodes01           # nodes on (0, tau]
        self.w = 0.5 * self.tau * what             # w_mu = tau/2 * omega_mu
        n = k + 1
        # exact integration on (0,tau] with a Gauss rule of degree >= 2k
        gx, gw = gauss_legendre01(n + 2)
        phi_g = lagrange_values(self.t, self.tau * gx)          # [g, a]
        dphi_g = lagrange_derivatives(self.t, self.tau * gx)    # [g, a]
        wg = self.tau * gw
        self.phi0 = lagrange_values(self.t, [0.0])[0]           # phi_a(t_{n-1}^+)
        self.phimid = lagrange_values(self.t, [0.5 * self.tau])[0]
        K = np.zeros((n, n))
        M = np.zeros((n, n))
        for a in range(n):
            for b in range(n):
                K[a, b] = np.sum(wg * dphi_g[:, b] * phi_g[:, a]) + self.phi0[b] * self.phi0[a]
                M[a, b] = np.sum(wg * phi_g[:, b] * phi_g[:, a])
        C = np.zeros((n, n))
        C[:, n - 1] = self.phi0                                  # delta_{b,k+1}
        self.K, self.M, self.C = K, M, C

    def values(self, t) -> np.ndarray:
        """phi_a(t) for t in (0, tau]."""
        return lagrange_values(self.t, t)


def time_tables(k: int, tau: float) -> TimeTables:
    return TimeTables(k, tau)


# --------------------------------------------------------------------------
# spatial bases
# --------------------------------------------------------------------------
def legendre_orthonormal01(r: int, s) -> np.ndarray:
    """Lt[p, i] = sqrt(2i+1) P_i(2 s_p - 1), i = 0..r (orthonormal on [0,1])."""
    s = np.atleast_1d(np.asarray(s, dtype=float))
    out = np.zeros((len(s), r + 1))
    for i in range(r + 1):
        c = np.zeros(i + 1)
        c[i] = 1.0
        out[:, i] = np.sqrt(2 * i + 1) * npleg.legval(2.0 * s - 1.0, c)
    return out


def pressure_modes(r: int, d: int) -> np.ndarray:
    """Multi-indices alpha with |alpha| <= r, first index fastest (shape [npm, 3])."""
    out = []
    if d == 2:
        for a1 in range(r + 1):
            for a0 in range(r + 1):
                if a0 + a1 <= r:
                    out.append((a0, a1, 0))
    else:
        for a2 in range(r + 1):
            for a1 in range(r + 1):
                for a0 in range(r + 1):
                    if a0 + a1 + a2 <= r:
                        out.append((a0, a1, a2))
    m = np.array(out, dtype=np.int32)
    assert len(m) == comb(r + d, d)
    return m


def default_nq(r: int) -> int:
    """Gauss points per direction that integrate the cubic convective product of
    Q_{r+1} fields exactly on affine cells: 2 nq - 1 >= 3 (r+1)."""
    return (3 * r + 4 + 1) // 2


# --------------------------------------------------------------------------
# exact closed forms printed in terms of fractions (used by pins only)
# --------------------------------------------------------------------------
def fraction_table(values):
    return [Fraction(v).limit_denominator(10**6) for v in values]
