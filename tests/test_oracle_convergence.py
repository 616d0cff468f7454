"""The oracle's slab-by-slab solution of the manufactured problem of Sec.
"Convergence test" against the errors the paper prints (Table tab:conv-ns,
r = 3, k = r, nu = 1e-2, tau = h, T = 1), fixture tests/golden/conv_ns_r3.txt.

Pins the whole discretization (forms, boundary terms and the penalty reading,
time rule, slab hand-off) to printed numbers: velocity, pressure, H1 and
divergence errors within 3 % at h = 1/2 and 1 % at h = 1/4 (measured: at
most 2.3 % and 0.8 %), and the observed orders between them within 0.08 of
the printed ones.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import errors as E
from oracle import manufactured as MS
from oracle import solver as S

GOLD = os.path.join(os.path.dirname(__file__), "golden", "conv_ns_r3.txt")
KEYS = ("v", "p", "h1", "div")


def paper_errors():
    rows = np.loadtxt(GOLD)
    return {float(r[0]): dict(zip(KEYS, r[1:])) for r in rows}


def oracle_march(n, r=3, k=3, nu=1e-2, T=1.0):
    h = 1.0 / n
    prob = oracle.Problem(dim=2, n=(n, n), r=r, k=k, nu=nu, tau=h)
    slab = oracle.Slab(prob)
    H = S.Hierarchy(prob)
    vprev = np.zeros(slab.space.Nv)
    U = np.zeros(slab.N)
    acc = dict.fromkeys(KEYS, 0.0)
    for s in range(int(round(T / h))):
        t0 = s * h
        U, st = S.newton_solve(slab, H, U.copy(), MS.slab_rhs(slab, t0), vprev)
        assert st.converged
        e = E.slab_errors(slab, U, t0)
        for key in KEYS:
            acc[key] += e[key]
        vprev = E.final_velocity(slab, U)
    return {key: float(np.sqrt(v)) for key, v in acc.items()}


def test_golden_fixture_orders():
    """The fixture's own observed orders are the ones the paper prints
    (guards the transcription)."""
    g = paper_errors()
    hs = sorted(g, reverse=True)
    printed_v = [4.46, 4.69, 4.93, 4.98]
    printed_p = [4.18, 3.95, 4.00, 4.00]
    for i in range(4):
        eoc_v = np.log2(g[hs[i]]["v"] / g[hs[i + 1]]["v"])
        eoc_p = np.log2(g[hs[i]]["p"] / g[hs[i + 1]]["p"])
        assert abs(eoc_v - printed_v[i]) < 0.006 and abs(eoc_p - printed_p[i]) < 0.006


def test_oracle_errors_match_paper():
    g = paper_errors()
    e2, e4 = oracle_march(2), oracle_march(4)
    for key in KEYS:
        assert abs(e2[key] / g[0.5][key] - 1) < 0.03, (key, e2[key], g[0.5][key])
        assert abs(e4[key] / g[0.25][key] - 1) < 0.01, (key, e4[key], g[0.25][key])
        eoc = np.log2(e2[key] / e4[key])
        eoc_paper = np.log2(g[0.5][key] / g[0.25][key])
        assert abs(eoc - eoc_paper) < 0.08, (key, eoc, eoc_paper)
