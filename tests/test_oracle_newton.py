"""Pins of the oracle's Newton control and of the Vanka overlap weighting,
each against values fixed by the definitions rather than by the oracle's
own code: the Eisenstat-Walker forcing term (eq. ew, reading S5), the
nonmonotone Armijo line search with its interpolation models (eq. armijo,
reading S7), the smoother rebuild criteria (the remark after Lemma "patch
perturbation", reading S9) and the partition-of-unity weighting of the
additive Vanka sweep (eq. vanka0, reading S3)."""
import numpy as np
import pytest

from oracle import Problem, Slab
from oracle import manufactured as MS
from oracle import solver as S
from paper_2602_13841_amd import inputs as I


# ---------------------------------------------------------------- forcing term
def test_forcing_term_hand_values():
    p = S.NewtonParams()                 # c_eta 0.5, theta 1.5, [1e-3, 0.8]
    # 0.5 * 0.4 * (0.25)^1.5 = 0.2 * 0.125
    assert S.forcing_term(0.4, 0.25, 1.0, p) == pytest.approx(0.025, rel=1e-15)
    # 0.5 * 0.025 * (0.04)^1.5 = 1e-4, held at eta_min
    assert S.forcing_term(0.025, 0.01, 0.25, p) == 1e-3
    # 0.5 * 0.8 * 4^1.5 = 3.2, held at eta_max
    assert S.forcing_term(0.8, 4.0, 1.0, p) == 0.8
    # a vanishing previous norm is replaced by eps = 1e-30: 0.2 * 0.1^1.5
    assert S.forcing_term(0.4, 1e-31, 0.0, p) == pytest.approx(0.2 * 10 ** -1.5, rel=1e-12)
    # theta enters as the exponent: theta = 2 gives 0.5 * 0.4 * 0.0625
    assert S.forcing_term(0.4, 0.25, 1.0, S.NewtonParams(theta=2.0)) == pytest.approx(0.0125, rel=1e-15)


def test_newton_uses_forcing_sequence():
    """The tolerances handed to FGMRES: eta0 first, then the forcing term of
    the residual norms before and after each step (values recomputed here
    from the recorded norms with the hand formula 0.5 eta (n_k / n_{k-1})^1.5
    held in [1e-3, 0.8])."""
    prob = Problem(dim=2, n=(4, 4), r=1, k=1, nu=1.0, tau=0.1)
    slab = Slab(prob)
    U, st = S.newton_solve(slab, S.Hierarchy(prob, max_levels=2), np.zeros(slab.N), MS.slab_rhs(slab, 0.0),
                           np.zeros(slab.Nv))
    assert st.etas[0] == 0.4 and len(st.etas) == st.newton_its >= 3
    for k in range(1, st.newton_its):
        want = min(max(0.5 * st.etas[k - 1] * (st.history[k] / st.history[k - 1]) ** 1.5, 1e-3), 0.8)
        assert st.etas[k] == pytest.approx(want, rel=1e-14)


# ---------------------------------------------------------------- line search
def test_line_search_cubic_step():
    """phi(a) = 1 - a - a^2 + 300 a^3 (phi0 = 1, g0 = -1).  a = 1 fails
    (phi = 299); the quadratic model's minimizer 1/598 is raised to 0.1,
    which fails too (phi = 1.19); the cubic through the two failures is phi
    itself, so the third trial is phi's local minimizer (1 + sqrt(901))/900,
    inside [0.01, 0.05], and it is accepted."""
    phi = lambda a: 1.0 - a - a * a + 300.0 * a ** 3
    calls = []

    def rec(a):
        calls.append(a)
        return phi(a)
    alpha, val, nback = S.line_search(rec, 1.0, -1.0, S.MeritMemory(1.0, 0), S.NewtonParams(window=0))
    astar = (1.0 + 901 ** 0.5) / 900.0
    assert calls[:2] == [1.0, 0.1] and nback == 2
    assert alpha == pytest.approx(astar, rel=1e-12) and val == pytest.approx(phi(astar), rel=1e-12)
    # the same minimizer from the model alone
    assert S.model_minimizer(1.0, -1.0, [(1.0, phi(1.0)), (0.1, phi(0.1))]) == pytest.approx(astar, rel=1e-12)


def test_line_search_quadratic_step_and_upper_clamp():
    """First trial lambda0 = 0.5 on phi(a) = (a - 0.1)^2 (phi0 = 0.01, g0 =
    -0.2): phi(0.5) = 0.16 fails, the quadratic model is phi itself, its
    minimizer 0.1 lies in [0.05, 0.25] and is accepted.  Then a merit
    function given by its values only: phi(1) = 50, phi(0.1) = 1 (phi0 = 1,
    g0 = -1) puts the cubic model's minimizer near 0.054, above half of the
    last step, so the third trial is 0.05."""
    calls = []

    def q(a):
        calls.append(a)
        return (a - 0.1) ** 2
    alpha, val, nback = S.line_search(q, 0.01, -0.2, S.MeritMemory(0.01, 0), S.NewtonParams(window=0, lambda0=0.5))
    assert calls == [0.5, pytest.approx(0.1, rel=1e-13)] and nback == 1
    table = {1.0: 50.0, 0.1: 1.0}
    calls.clear()

    def t(a):
        calls.append(a)
        return table.get(a, 0.5)
    S.line_search(t, 1.0, -1.0, S.MeritMemory(1.0, 0), S.NewtonParams(window=0))
    assert calls == [1.0, 0.1, 0.05]
    assert S.model_minimizer(1.0, -1.0, [(1.0, 50.0), (0.1, 1.0)]) > 0.05


def test_line_search_model_without_minimizer_halves():
    """A concave quadratic model (phi above phi0 + g0 a is required for a
    minimizer) has none: the step is multiplied by tau."""
    assert S.model_minimizer(1.0, -1.0, [(1.0, -0.5)]) is None
    # phi0 = 0, g0 = -1, phi(1) = -5 < phi0 + g0: concave model; the step is
    # rejected against a remembered reference of -10
    mem = S.MeritMemory(-10.0, 1)
    calls = []

    def rec(a):
        calls.append(a)
        return -5.0 if a > 0.9 else -20.0
    S.line_search(rec, 0.0, -1.0, mem, S.NewtonParams(window=1, tau=0.5))
    assert calls[:2] == [1.0, 0.5]


def test_line_search_nonmonotone_reference_and_cap():
    p = S.NewtonParams()                          # window 5, c = 1e-4, 5 backtracks, alpha_min 1e-3
    mem = S.MeritMemory(5.0, 5)
    # phi(1) = 2 exceeds phi0 = 1 but not the remembered maximum 5
    alpha, val, nback = S.line_search(lambda a: 2.0, 1.0, -1.0, mem, p)
    assert alpha == 1.0 and nback == 0 and mem.values == [5.0, 2.0]
    # the memory keeps the last 5 accepted values
    for v in (1.5, 1.4, 1.3, 1.2):
        mem.remember(v)
    assert mem.values == [2.0, 1.5, 1.4, 1.3, 1.2] and mem.reference(0.0) == 2.0
    # the monotone rule (size 0) rejects the same step
    trials = []

    def flat(a):
        trials.append(a)
        return 2.0
    alpha, val, nback = S.line_search(flat, 1.0, -1.0, S.MeritMemory(5.0, 0), p)
    # every step is rejected; the steps shrink by at least half until the next
    # one would not exceed alpha_min, whose value is returned
    assert val is None and alpha == p.alpha_min and nback == len(trials) <= p.max_backtracks
    assert all(b <= 0.5 * a for a, b in zip(trials[:-1], trials[1:])) and trials[-1] > p.alpha_min
    # with a tiny alpha_min the cap of max_backtracks + 1 rejected trials ends it
    trials.clear()
    p2 = S.NewtonParams(alpha_min=1e-12)
    alpha, val, nback = S.line_search(flat, 1.0, -1.0, S.MeritMemory(5.0, 0), p2)
    assert alpha == 1e-12 and nback == len(trials) == p2.max_backtracks + 1


# ------------------------------------------------------------ rebuild policy
def test_rebuild_policy_criteria():
    p = S.NewtonParams()                          # theta_N 0.5, theta_L 2, kappa_abs 10, s 3, 0.9
    pol = S.RebuildPolicy(p)
    assert pol.due_before_step()                  # nothing built yet
    pol.rebuilt_before_step()
    pol.record_step(0.3, 1.0, 4)                  # rho 0.3, kappa 4 < max(2, 10)
    assert not pol.due_before_step()
    pol.record_step(0.5, 1.0, 4)                  # Newton deterioration: rho = theta_N
    assert pol.due_before_step()
    pol.record_step(0.1, 1.0, 12)                 # kappa_ref still 1: 12 >= max(2, 10)
    assert pol.due_before_step()
    pol.rebuilt_before_step()                     # kappa_ref = 12
    pol.record_step(0.1, 1.0, 23)                 # 23 < max(24, 10)
    assert not pol.due_before_step()
    pol.record_step(0.1, 1.0, 24)
    assert pol.due_before_step()
    pol.record_step(0.1, 1.0, 0)                  # kappa counts at least 1
    assert pol.kappa == 1 and not pol.due_before_step()
    # stagnation: s = 3 consecutive ratios >= 0.9
    assert pol.due_after_step([1.0, 0.95, 0.9, 0.86])
    assert not pol.due_after_step([1.0, 0.95, 0.5, 0.48, 0.44])
    assert pol.due_after_step([1.0, 0.5, 0.48, 0.44, 0.43])
    assert not pol.due_after_step([1.0, 0.95, 0.9])


def _c1_solve(**kw):
    prob = Problem(dim=2, n=(4, 4), r=1, k=1, nu=1.0, tau=0.1)
    slab = Slab(prob)
    p = S.NewtonParams(**kw)
    return S.newton_solve(slab, S.Hierarchy(prob, max_levels=2), np.zeros(slab.N), MS.slab_rhs(slab, 0.0),
                          np.zeros(slab.Nv), p)[1]


def test_rebuild_triggers_forced():
    never = dict(theta_N=1e9, theta_L=1e9, kappa_abs=1e9, stag_theta=2.0)
    st = _c1_solve(**never)
    assert st.converged and st.rebuilds == 1
    # Newton deterioration always: a rebuild before every step
    st = _c1_solve(**{**never, "theta_N": 0.0})
    assert st.converged and st.rebuilds == st.newton_its
    # linear deterioration always (kappa >= 1 = max(0 * kappa_ref, 1))
    st = _c1_solve(**{**never, "theta_L": 0.0, "kappa_abs": 1.0})
    assert st.converged and st.rebuilds == st.newton_its
    # stagnation always (every ratio >= 0, one suffices): one rebuild after
    # every step with at least one FGMRES iteration, plus the first
    st = _c1_solve(**{**never, "stag_theta": 0.0, "stag_s": 1})
    assert st.converged and st.rebuilds == 1 + sum(1 for i in st.fgmres_its if i >= 1)


# ------------------------------------------------ Vanka overlap multiplicity
@pytest.mark.parametrize("d,n,r,k", [(2, (3, 3), 1, 1), (2, (3, 2), 2, 0), (3, (2, 3, 2), 1, 0)])
def test_vanka_multiplicity_and_weighted_sweep(d, n, r, k):
    """Each velocity unknown lies in as many cell patches as cells share its
    node: per axis 2 on an interior cell interface, else 1 (counted here from
    the node lattice); a pressure unknown lies in one.  The default sweep is
    d + (sum over cells of the dense patch solves) / multiplicity."""
    prob = Problem(dim=d, n=n, r=r, k=k, nu=0.1, tau=0.1, vertices=I.perturbed_vertices(d, n, 0.2, 4))
    H = S.Hierarchy(prob, max_levels=2)
    slab = H.levels[0].slab
    U = I.uniform(slab.N, 11)
    H.set_state(U)
    H.build_patches(0)
    Nax = [(r + 1) * x + 1 for x in n]
    per_axis = [np.array([2 if (g % (r + 1) == 0 and 0 < g < Nax[a] - 1) else 1 for g in range(Nax[a])])
                for a in range(d)]
    node_mult = per_axis[0]
    for a in range(1, d):
        node_mult = np.multiply.outer(per_axis[a], node_mult).reshape(-1)   # x fastest
    want = np.concatenate([np.tile(node_mult, d * slab.nt), np.ones(slab.nt * slab.Np)])
    assert np.array_equal(H.levels[0].mult, want)
    # sweep = weighted sum of dense patch solves of the surrogate's principal submatrices
    V, _ = slab.split(U)
    Jt = slab.jacobian(U, surrogate_state=slab.tt.phimid @ V).toarray()
    J = H.levels[0].J.toarray()
    r_ = I.uniform(slab.N, 12)
    d0 = I.uniform(slab.N, 13)
    defect = r_ - J @ d0
    acc = np.zeros(slab.N)
    for idx in S.patch_indices(slab):
        acc[idx] += np.linalg.solve(Jt[np.ix_(idx, idx)], defect[idx])
    assert np.allclose(H.smooth(0, r_, d0), d0 + acc / want, rtol=1e-10, atol=1e-12 * np.abs(acc).max())
    # the literal plain sum with omega
    H0 = S.Hierarchy(prob, max_levels=2, weighting=0, omega=0.3)
    H0.set_state(U)
    H0.build_patches(0)
    assert np.allclose(H0.smooth(0, r_, d0), d0 + 0.3 * acc, rtol=1e-10, atol=1e-12 * np.abs(acc).max())
