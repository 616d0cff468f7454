"""Pins of the oracle's 1D tables against closed forms and exactness
properties (Sec. Preliminaries, eq. GF, eq. BasYk; appendix eq. DefKMC)."""
import os
from math import comb, sqrt

import numpy as np
import pytest

from oracle import tables as T
from oracle import dof_count

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_radau_closed_forms():
    # textbook right Radau rules on [-1,1]: roots of P_{k+1} - P_k
    x, w = T.radau_right(0)
    assert np.allclose(x, [1.0]) and np.allclose(w, [2.0])
    x, w = T.radau_right(1)
    assert np.allclose(x, [-1 / 3, 1.0], atol=1e-15)
    assert np.allclose(w, [1.5, 0.5], atol=1e-15)
    x, w = T.radau_right(2)
    s6 = sqrt(6.0)
    assert np.allclose(x, [(-1 - s6) / 5, (-1 + s6) / 5, 1.0], atol=1e-14)
    assert np.allclose(w, [(16 - s6) / 18, (16 + s6) / 18, 2 / 9], atol=1e-14)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_radau_exactness(k):
    # exact for degree 2k, not for 2k+1 (eq. GF); last node is +1
    x, w = T.radau_right(k)
    assert x[-1] == 1.0
    for deg in range(2 * k + 1):
        exact = (1 - (-1) ** (deg + 1)) / (deg + 1)
        assert abs(np.sum(w * x ** deg) - exact) < 1e-13
    deg = 2 * k + 1
    exact = (1 - (-1) ** (deg + 1)) / (deg + 1)
    assert abs(np.sum(w * x ** deg) - exact) > 1e-3


def test_time_matrices_k1_closed_form():
    tt = T.time_tables(1, 0.3)
    assert np.allclose(tt.K, [[9 / 8, 3 / 8], [-9 / 8, 5 / 8]], atol=1e-14)
    assert np.allclose(tt.M, np.diag([0.75 * 0.3, 0.25 * 0.3]), atol=1e-15)
    assert np.allclose(tt.C, [[0, 1.5], [0, -0.5]], atol=1e-14)
    assert np.allclose(tt.phimid, [0.75, 0.25], atol=1e-14)


def test_time_matrices_k2_midpoint():
    tt = T.time_tables(2, 1.0)
    s6 = sqrt(6.0)
    assert np.allclose(tt.phimid, [7 / 12 - s6 / 6, 7 / 12 + s6 / 6, -1 / 6], atol=1e-13)
    assert np.allclose(tt.C[:, 2], [1 / 3 + s6 / 2, 1 / 3 - s6 / 2, 1 / 3], atol=1e-13)
    assert np.allclose(np.diag(tt.M), [4 / 9 - s6 / 36, 4 / 9 + s6 / 36, 1 / 9], atol=1e-14)


def test_dg0_is_implicit_euler():
    # k = 0: K = 1, M = tau, C = 1: one backward Euler step
    tt = T.time_tables(0, 0.25)
    assert np.allclose(tt.K, [[1.0]]) and np.allclose(tt.M, [[0.25]]) and np.allclose(tt.C, [[1.0]])


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_time_matrix_identities(k):
    tau = 0.7
    tt = T.time_tables(k, tau)
    # M diagonal with the scaled Radau weights
    assert np.allclose(tt.M, np.diag(tt.w), atol=1e-15)
    assert np.allclose(tt.w, 0.5 * tau * T.radau_right(k)[1])
    # a constant-in-time field is reproduced: K 1 = C[:, k]
    assert np.allclose(tt.K @ np.ones(k + 1), tt.C[:, k], atol=1e-13)
    # DG energy identity x^T K x = 1/2 (p(tau)^2 + p(0+)^2)
    rng = np.random.default_rng(k)
    for _ in range(5):
        x = rng.standard_normal(k + 1)
        p_end = x[-1]                       # last node is t_n
        p0 = tt.phi0 @ x
        assert abs(x @ tt.K @ x - 0.5 * (p_end ** 2 + p0 ** 2)) < 1e-12


def test_gauss_lobatto_closed_forms():
    assert np.allclose(T.gauss_lobatto01(2), [0, 1])
    assert np.allclose(T.gauss_lobatto01(3), [0, 0.5, 1])
    a = 1 / sqrt(5)
    assert np.allclose(T.gauss_lobatto01(4), [0, (1 - a) / 2, (1 + a) / 2, 1], atol=1e-15)
    b = sqrt(3 / 7)
    assert np.allclose(T.gauss_lobatto01(5), [0, (1 - b) / 2, 0.5, (1 + b) / 2, 1], atol=1e-15)


@pytest.mark.parametrize("nq", [1, 2, 4, 7])
def test_gauss_exactness(nq):
    x, w = T.gauss_legendre01(nq)
    for deg in range(2 * nq):
        assert abs(np.sum(w * x ** deg) - 1 / (deg + 1)) < 1e-14


@pytest.mark.parametrize("d,r", [(2, 1), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_pressure_basis_orthonormal(d, r):
    modes = T.pressure_modes(r, d)
    assert len(modes) == comb(r + d, d)
    assert np.all(modes.sum(axis=1) <= r)
    x, w = T.gauss_legendre01(r + 2)
    L = T.legendre_orthonormal01(r, x)
    G = np.zeros((len(modes), len(modes)))
    for i, a in enumerate(modes):
        for j, b in enumerate(modes):
            val = 1.0
            for ax in range(d):
                val *= np.sum(w * L[:, a[ax]] * L[:, b[ax]])
            G[i, j] = val
    assert np.allclose(G, np.eye(len(modes)), atol=1e-13)


def test_lagrange_derivatives_exact():
    nodes = T.gauss_lobatto01(5)
    x = np.linspace(0, 1, 7)
    # interpolate x^4 and differentiate: exact
    f = nodes ** 4
    assert np.allclose(T.lagrange_derivatives(nodes, x) @ f, 4 * x ** 3, atol=1e-12)
    assert np.allclose(T.lagrange_values(nodes, x) @ f, x ** 4, atol=1e-13)


def test_dof_count_matches_paper_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "st_sizes.txt")) if not l.startswith("#") and l.strip()]
    assert len(rows) == 6
    for c, r, ndof in rows:
        c, r, ndof = int(c), int(r), int(ndof)
        n_slabs = 2 ** (c + 4)
        assert n_slabs * dof_count(3, 2 ** c, r, r) == ndof


def test_dof_count_configs():
    assert dof_count(2, 4, 1, 1) == 420
    assert dof_count(2, 8, 1, 1) == 1540
    assert dof_count(3, 16, 2, 2) == 1181721
    assert dof_count(3, 32, 3, 1) == 14190854
