"""Pins of the solver part of the oracle: grid transfers, level states,
Vanka smoother, V-cycle, FGMRES and Newton (Sec. "Solution of the nonlinear
system of equations", eq. MatGeomProl, eq. LVS, eq. vanka0, eq. inexact,
Alg. "Inexact Newton-Krylov", Alg. "Armijo")."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
from numpy.polynomial import polynomial as P

from oracle import Problem, Slab
from oracle import manufactured as MS
from oracle import solver as S
from oracle import tables as T
from paper_2602_13841_amd import inputs as I


def pval(c, x):
    if x.shape[1] == 2:
        return P.polyval2d(x[:, 0], x[:, 1], c)
    return P.polyval3d(x[:, 0], x[:, 1], x[:, 2], c)


def _pair(d, n, r, k, kind):
    fine = Slab(Problem(dim=d, n=n, r=r, k=k, nu=1.0, tau=1.0))
    if kind == "h":
        coarse = Slab(Problem(dim=d, n=tuple(x // 2 for x in n), r=r, k=k, nu=1.0, tau=1.0))
    else:
        rc, kc = max(1, r // 2), (k // 2 if k >= 2 else k)
        coarse = Slab(Problem(dim=d, n=n, r=rc, k=kc, nu=1.0, tau=1.0))
    return fine, coarse


@pytest.mark.parametrize("d,n,r,k,kind", [(2, (4, 2), 1, 1, "h"), (2, (2, 2), 3, 2, "p"),
                                          (3, (2, 2, 4), 1, 0, "h"), (3, (1, 2, 1), 2, 2, "p")])
def test_prolongation_reproduces_coarse_polynomials(d, n, r, k, kind):
    """Canonical embedding: a coarse space-time polynomial is reproduced
    exactly on the fine level (velocity nodal values, pressure modes)."""
    fine, coarse = _pair(d, n, r, k, kind)
    rng = np.random.default_rng(1)
    rc, kc = coarse.prob.r, coarse.prob.k
    Pm = S.slab_prolongation(fine, coarse, kind)
    # velocity: v(x,t) = sum_j t^j q_j(x), q_j in Q_{rc+1}, degree kc in t
    xc, xf = coarse.space.node_coordinates(), fine.space.node_coordinates()
    coefs = [[rng.uniform(-1, 1, (rc + 2,) * d) for _ in range(d)] for _ in range(kc + 1)]

    def vel(xn, tnodes):
        return np.concatenate([np.concatenate([sum(t ** j * pval(coefs[j][c], xn) for j in range(kc + 1))
                                               for c in range(d)]) for t in tnodes])
    tc, tf = T.time_tables(kc, 1.0).t, T.time_tables(k, 1.0).t
    Vc, Vf = vel(xc, tc), vel(xf, tf)
    Uc = np.concatenate([Vc, np.zeros(coarse.nt * coarse.Np)])
    Uf = Pm @ Uc
    assert np.max(np.abs(Uf[: fine.nt * fine.Nv] - Vf)) < 1e-12
    # pressure: a coarse-cell-wise polynomial (coarse modes random) maps to the
    # fine modes of the same function: check by point evaluation in every fine cell
    Pc = rng.uniform(-1, 1, coarse.nt * coarse.Np)
    Uc = np.concatenate([np.zeros(coarse.nt * coarse.Nv), Pc])
    Pf = (Pm @ Uc)[fine.nt * fine.Nv:]
    pts = rng.uniform(0, 1, (5, d))

    def peval(slab, modes_vec, cell, xi):
        L = [T.legendre_orthonormal01(slab.prob.r, xi[:, a]) for a in range(d)]
        psi = np.stack([np.prod([L[a][:, m[a]] for a in range(d)], axis=0) for m in slab.space.modes], axis=1)
        return psi @ modes_vec[cell * slab.space.npm:(cell + 1) * slab.space.npm]

    Ptime = S.time_prolongation(k, kc)
    for a in range(fine.nt):
        pc_a = sum(Ptime[a, b] * Pc[b * coarse.Np:(b + 1) * coarse.Np] for b in range(coarse.nt))
        pf_a = Pf[a * fine.Np:(a + 1) * fine.Np]
        for cell in range(fine.space.ncell):
            cf = [(cell // int(np.prod(fine.prob.n[:ax]))) % fine.prob.n[ax] for ax in range(d)]
            if kind == "h":
                o = np.array([c % 2 for c in cf])
                cc = [c // 2 for c in cf]
                xi_c = (o[None, :] + pts) / 2
            else:
                cc, xi_c = cf, pts
            ccell = sum(cc[ax] * int(np.prod(coarse.prob.n[:ax])) for ax in range(d))
            assert np.allclose(peval(fine, pf_a, cell, pts), peval(coarse, pc_a, ccell, xi_c), atol=1e-12)


@pytest.mark.parametrize("d,n,r,k,kind", [(2, (4, 4), 2, 2, "h"), (2, (2, 3), 3, 2, "p"), (3, (2, 2, 2), 2, 1, "p")])
def test_state_interpolation_reproduces_polynomials(d, n, r, k, kind):
    fine, coarse = _pair(d, n, r, k, kind)
    rng = np.random.default_rng(2)
    rc, kc = coarse.prob.r, coarse.prob.k
    coefs = [[rng.uniform(-1, 1, (rc + 2,) * d) for _ in range(d)] for _ in range(kc + 1)]
    xc, xf = coarse.space.node_coordinates(), fine.space.node_coordinates()

    def vel(xn, tnodes):
        return np.concatenate([np.concatenate([sum(t ** j * pval(coefs[j][c], xn) for j in range(kc + 1))
                                               for c in range(d)]) for t in tnodes])
    Im = S.state_interpolation(fine, coarse, kind)
    assert np.max(np.abs(Im @ vel(xf, T.time_tables(k, 1.0).t) - vel(xc, T.time_tables(kc, 1.0).t))) < 1e-12


def test_level_specs():
    assert S.level_specs(Problem(dim=2, n=(4, 4), r=1, k=1, nu=1, tau=1)) == [(1, 1, (4, 4)), (1, 1, (2, 2))]
    sp3 = S.level_specs(Problem(dim=3, n=(32, 32, 32), r=3, k=1, nu=1, tau=1))
    assert sp3 == [(1, 3, (32,) * 3), (1, 1, (32,) * 3), (1, 1, (16,) * 3), (1, 1, (8,) * 3), (1, 1, (4,) * 3),
                   (1, 1, (2,) * 3)]
    assert S.level_specs(Problem(dim=3, n=(16,) * 3, r=2, k=2, nu=1, tau=1))[1] == (2, 1, (16,) * 3)
    assert S.level_specs(Problem(dim=3, n=(16,) * 3, r=2, k=2, nu=1, tau=1), time_coarsening=True)[1] == \
        (1, 1, (16,) * 3)
    assert S.level_specs(Problem(dim=2, n=(8, 8), r=1, k=3, nu=1, tau=1)) == [(3, 1, (8, 8)), (3, 1, (4, 4)),
                                                                              (3, 1, (2, 2))]
    assert S.level_specs(Problem(dim=2, n=(8, 8), r=1, k=3, nu=1, tau=1), time_coarsening=True)[:2] == \
        [(3, 1, (8, 8)), (1, 1, (8, 8))]
    assert S.level_specs(Problem(dim=2, n=(8, 8), r=1, k=1, nu=1, tau=1), max_levels=2) == [(1, 1, (8, 8)),
                                                                                            (1, 1, (4, 4))]


def _hier(d=2, n=(4, 4), r=1, k=1, nu=0.1, tau=0.1, mask=None, pert=False, max_levels=0, omega=None, seed=3):
    vert = I.perturbed_vertices(d, n, 0.2, 9) if pert else None
    prob = Problem(dim=d, n=n, r=r, k=k, nu=nu, tau=tau, dirichlet_mask=mask, vertices=vert)
    H = S.Hierarchy(prob, max_levels=max_levels, omega=omega)
    slab = H.levels[0].slab
    U = I.uniform(slab.N, seed)
    H.set_state(U)
    return H, slab, U


def test_surrogate_equals_exact_for_k0_and_constant_state():
    # k = 0: the midpoint value is the single time node
    H, slab, U = _hier(k=0)
    V, _ = slab.split(U)
    vstar = slab.tt.phimid @ V
    assert np.allclose(vstar, V[0])
    assert abs(slab.jacobian(U, surrogate_state=vstar) - slab.jacobian(U)).max() == 0.0
    # a state constant in time: surrogate = exact
    H, slab, U = _hier(k=2)
    V, Pp = slab.split(U)
    Uc = slab.join(np.tile(V[0], (slab.nt, 1)), Pp)
    Vc, _ = slab.split(Uc)
    vstar = slab.tt.phimid @ Vc
    assert abs(slab.jacobian(Uc, surrogate_state=vstar) - slab.jacobian(Uc)).max() < 1e-13


def test_patch_solve_matches_dense_solve():
    H, slab, U = _hier(d=2, n=(3, 2), r=2, k=1, pert=True)
    H.rebuild_smoother()
    L = H.levels[0]
    V, _ = slab.split(L.state)
    Jt = slab.jacobian(L.state, surrogate_state=slab.tt.phimid @ V).toarray()
    rng = np.random.default_rng(4)
    for idx, lu in L.patches[:3]:
        b = rng.uniform(-1, 1, len(idx))
        import scipy.linalg as sla
        assert np.allclose(sla.lu_solve(lu, b), np.linalg.solve(Jt[np.ix_(idx, idx)], b), rtol=1e-10, atol=1e-12)


def test_one_cell_sweep_is_exact_solve():
    # one cell with Neumann faces: the patch is the whole system
    H, slab, U = _hier(d=2, n=(1, 1), r=1, k=1, mask=0b0011, omega=1.0, max_levels=1)
    prob = slab.prob
    H2 = S.Hierarchy(prob, max_levels=2, omega=1.0)
    H2.set_state(U)
    H2.build_patches(0)
    r = I.uniform(slab.N, 5)
    d = H2.smooth(0, r, np.zeros(slab.N))
    V, _ = slab.split(U)
    Jt = slab.jacobian(U, surrogate_state=slab.tt.phimid @ V).toarray()
    assert np.allclose(d, np.linalg.solve(Jt, r), rtol=1e-10, atol=1e-12)


def test_surrogate_perturbation_linear_in_tau():
    """Lemma patch-perturbation: ||S_tilde - S|| = O(tau) for a state that is
    smooth in time."""
    d, n, r, k = 2, (2, 2), 1, 2
    errs = []
    for tau in (0.1, 0.05, 0.025):
        prob = Problem(dim=d, n=n, r=r, k=k, nu=0.1, tau=tau)
        slab = Slab(prob)
        v0 = I.smooth_velocity(d, n, r, 1, m=2)
        v1 = I.smooth_velocity(d, n, r, 2, m=2)
        V = np.array([v0 + np.sin(3 * t) * v1 for t in slab.tt.t])
        U = slab.join(V, np.zeros((slab.nt, slab.Np)))
        vstar = slab.tt.phimid @ V
        A = slab.jacobian(U).toarray()
        B = slab.jacobian(U, surrogate_state=vstar).toarray()
        idx = S.patch_indices(slab)[0]
        errs.append(np.linalg.norm(A[np.ix_(idx, idx)] - B[np.ix_(idx, idx)], 2))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 0.9), rates


def test_vcycle_linear_and_one_level_exact():
    H, slab, U = _hier(d=2, n=(4, 4), r=1, k=1)
    H.rebuild_smoother()
    r1, r2 = I.uniform(slab.N, 6), I.uniform(slab.N, 7)
    B = H.vcycle
    assert np.allclose(B(2.0 * r1 - 3.0 * r2), 2.0 * B(r1) - 3.0 * B(r2), rtol=1e-10, atol=1e-12)
    # one level with Neumann faces: the cycle is the direct solve
    H1, slab1, U1 = _hier(d=2, n=(2, 2), r=1, k=1, mask=0b0101, max_levels=1)
    x = H1.vcycle(r1[: slab1.N])
    assert np.allclose(slab1.jacobian(U1) @ x, r1[: slab1.N], rtol=1e-9, atol=1e-11)
    # pure Dirichlet coarse solve: bordered system solves consistent right-hand sides
    H2, slab2, U2 = _hier(d=2, n=(2, 2), r=1, k=1, max_levels=1)
    J = slab2.jacobian(U2)
    b = J @ I.uniform(slab2.N, 8)
    assert np.allclose(J @ H2.vcycle(b), b, rtol=1e-9, atol=1e-11)


def test_fgmres_exact_preconditioner_and_m_norm_residual():
    H, slab, U = _hier(d=2, n=(2, 2), r=1, k=1, mask=0b0101, max_levels=1)
    J = slab.jacobian(U)
    M = slab.slab_mass()
    b = I.uniform(slab.N, 9)
    res = S.fgmres(lambda z: J @ z, H.vcycle, lambda v: M @ v, b, 1e-10)
    assert res.its == 1
    assert np.allclose(J @ res.x, b, rtol=1e-9, atol=1e-11)
    # unpreconditioned, Euclidean inner product: same Krylov solution as a
    # direct solve, monotone residual estimates, estimate = true residual
    res = S.fgmres(lambda z: J @ z, lambda v: v, lambda v: v, b, 1e-9, maxit=200)
    hist = np.array(res.history)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])
    true = np.linalg.norm(b - J @ res.x)
    assert abs(true - hist[-1]) < 1e-8 * hist[0]
    x_ref = spla.spsolve(J.tocsc(), b)
    assert np.allclose(res.x, x_ref, rtol=1e-6, atol=1e-8 * np.abs(x_ref).max())


def test_armijo_quadratic_interpolation_exact():
    p = S.NewtonParams(window=0)
    # phi(a) = (a - 0.3)^2: phi0 = 0.09, g0 = -0.6; full step fails, the
    # quadratic model is exact, its minimizer 0.3 is inside [0.1, 0.5]
    phi = lambda a: (a - 0.3) ** 2
    alpha, val, nback = S.line_search(phi, 0.09, -0.6, S.MeritMemory(0.09, 0), p)
    assert abs(alpha - 0.3) < 1e-14 and nback == 1


def test_newton_c1_manufactured_converges():
    """C1: 2D 4x4, Q2/P1disc x DG(1), tau = 0.1, nu = 1, manufactured field,
    2 levels.  Converges to ||R||_M <= 1e-8 ||R_0||_M with quadratic-like
    final contraction; the discrete solution at t = 0.1 is close to the
    exact field."""
    prob = Problem(dim=2, n=(4, 4), r=1, k=1, nu=1.0, tau=0.1)
    slab = Slab(prob)
    rhs = MS.slab_rhs(slab, 0.0)
    H = S.Hierarchy(prob, max_levels=2)
    U, st = S.newton_solve(slab, H, np.zeros(slab.N), rhs, np.zeros(slab.Nv))
    assert st.converged and st.res <= 1e-8 * st.res0
    assert np.linalg.norm(slab.residual(U, rhs, np.zeros(slab.Nv))) < 1e-9
    h = st.history
    assert h[-1] / h[-2] < 0.1 * (h[-2] / h[-3]) or h[-1] < 1e-12
    xn = slab.space.node_coordinates()
    vex = MS.velocity(xn[:, 0], xn[:, 1], 0.1)
    V, _ = slab.split(U)
    vend = V[-1].reshape(2, -1).T
    assert np.max(np.abs(vend - vex)) < 0.05 * np.max(np.abs(vex))


@pytest.mark.parametrize("mode", [1, 2])
def test_diagonal_vanka_patch_is_schur_elimination(mode):
    """Diagonal Vanka patch (velocity-velocity blocks reduced to their spatial
    diagonal, or mode 2 to their node blocks, time coupling kept) solved
    directly equals the block elimination written from its definition: per
    spatial velocity unknown i (mode 2: per node, all components) the block D_i
    of the exact patch over the time nodes, S = C - B D^{-1} B^T,
    p = S^{-1}(g - B D^{-1} f), u = D^{-1}(f - B^T p)."""
    import scipy.linalg as sla
    for k in (0, 1, 2):
        prob = Problem(dim=2, n=(4, 4), r=1, k=k, nu=0.05, tau=0.1)
        H = S.Hierarchy(prob, max_levels=2, diagonal=mode)
        s = H.levels[0].slab
        U = I.uniform(s.N, 70 + k)
        H.set_state(U)
        V, _ = s.split(U)
        Jt = s.jacobian(U, surrogate_state=s.tt.phimid @ V)
        idx = S.patch_indices(s)[5]
        P = Jt[idx][:, idx].toarray()
        nv = prob.dim * s.space.nl
        nt = s.nt
        n = nt * nv
        rhs = I.uniform(len(idx), 80 + k)
        f, g = rhs[:n], rhs[n:]
        Dinv = np.zeros((n, n))
        nl = s.space.nl
        groups = [[i] for i in range(nv)] if mode == 1 else [[c * nl + l for c in range(prob.dim)] for l in range(nl)]
        for grp in groups:
            ii = [a * nv + i for a in range(nt) for i in grp]
            Dinv[np.ix_(ii, ii)] = np.linalg.inv(P[np.ix_(ii, ii)])
        B, BT, C = P[n:, :n], P[:n, n:], P[n:, n:]
        p = np.linalg.solve(C - B @ Dinv @ BT, g - B @ Dinv @ f)
        u = Dinv @ (f - BT @ p)
        x = sla.lu_solve(sla.lu_factor(S.diagonal_velocity_block(s, P, mode == 2)), rhs)
        assert np.allclose(x, np.concatenate([u, p]), rtol=1e-9, atol=1e-12 * np.max(np.abs(x)))
        # the smoother uses exactly these patches
        H.rebuild_smoother()
        lu = H.levels[0].patches[5][1]
        assert np.allclose(sla.lu_solve(lu, rhs), x, rtol=1e-12, atol=1e-14 * np.max(np.abs(x)))
