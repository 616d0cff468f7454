"""Parity of the HIP slab operators with the oracle (GPU).

Bar: FP64 results equal the oracle to 1e-12 relative (max-abs error over
max-abs value), FP32 to 1e-5 relative, on seeded inputs.  Small meshes are
compared element by element over the whole vector (several cells, ragged
cell counts, perturbed vertices, mixed Dirichlet/Neumann faces, one-cell
meshes); the full-size workloads (16^3 Q3/P2/DG(2) and the perturbed 32^3
Q4/P3/DG(1)) on rows sampled from every block of the slab vector.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2602_13841_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def stmg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_13841_amd import stmg as S
    return S


def dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


CASES = [
    # (dim, n, r, k, nu, tau, perturbed, dirichlet mask, nq)
    ("c1_4x4", 2, (4, 4), 1, 1, 1.0, 0.1, False, None, None),
    ("2d_ragged_pert_mixed", 2, (3, 5), 2, 2, 0.01, 0.05, True, 0b1011, None),
    ("2d_r3_k0", 2, (2, 3), 3, 0, 0.1, 0.2, True, None, None),
    ("3d_r1_k0_pert", 3, (2, 3, 2), 1, 0, 0.02, 0.1, True, None, None),
    ("3d_r2_k2", 3, (3, 2, 2), 2, 2, 0.01, 1 / 32, False, None, None),
    ("3d_r3_k1_pert", 3, (2, 2, 3), 3, 1, 1e-3, 1 / 64, True, 0b101011, None),
    ("3d_r2_k1_nqperf", 3, (2, 2, 2), 2, 1, 0.1, 0.1, True, None, 4),
    ("3d_one_cell", 3, (1, 1, 1), 2, 1, 0.5, 0.1, False, None, None),
    ("3d_r1_k3", 3, (2, 2, 2), 1, 3, 0.05, 0.1, False, None, None),
]


def make(case, stmg):
    name, d, n, r, k, nu, tau, pert, mask, nq = case
    vert = I.perturbed_vertices(d, n, 0.2, 40 + d * 10 + r) if pert else None
    prob = oracle.Problem(dim=d, n=n, r=r, k=k, nu=nu, tau=tau, vertices=vert, dirichlet_mask=mask, nq=nq)
    slab = oracle.Slab(prob)
    ctx = stmg.Context(d, n, r, k, nu, tau, vertices=vert, dirichlet_faces=prob.dirichlet_mask, n_q=nq or 0)
    assert ctx.N == slab.N
    return slab, ctx


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_jacobian_vmult_fp64_fp32(case, stmg):
    slab, ctx = make(case, stmg)
    U = I.uniform(slab.N, 1)
    X = I.uniform(slab.N, 2)
    want = slab.jacobian(U) @ X
    got = ctx.jacobian_vmult(dev(U), dev(X)).cpu().numpy()
    assert rel(got, want) < TOL64
    got32 = ctx.jacobian_vmult(dev(U, torch.float32), dev(X, torch.float32)).cpu().numpy()
    assert rel(got32, want) < TOL32


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_residual_fp64(case, stmg):
    slab, ctx = make(case, stmg)
    U = I.uniform(slab.N, 3)
    rhs = I.uniform(slab.N, 4)
    vprev = I.uniform(slab.Nv, 5)
    want = slab.residual(U, rhs, vprev)
    ctx.set_slab_data(dev(rhs), dev(vprev))
    got = ctx.residual(dev(U)).cpu().numpy()
    assert rel(got, want) < TOL64
    # no slab data: plain operator part
    ctx.set_slab_data(None, None)
    got0 = ctx.residual(dev(U)).cpu().numpy()
    assert rel(got0, slab.residual(U)) < TOL64


@pytest.mark.parametrize("case", CASES[:5], ids=[c[0] for c in CASES[:5]])
def test_mass_vmult(case, stmg):
    slab, ctx = make(case, stmg)
    X = I.uniform(slab.N, 6)
    want = slab.slab_mass() @ X
    got = ctx.mass_vmult(dev(X)).cpu().numpy()
    assert rel(got, want) < TOL64
    got32 = ctx.mass_vmult(dev(X, torch.float32)).cpu().numpy()
    assert rel(got32, want) < TOL32


def test_batched_vmult_matches_single(stmg):
    slab, ctx = make(CASES[5], stmg)
    U = dev(I.uniform(slab.N, 7))
    X = torch.stack([dev(I.uniform(slab.N, 8 + i)) for i in range(3)])
    Y = ctx.jacobian_vmult_batched(U, X)
    for i in range(3):
        yi = ctx.jacobian_vmult(U, X[i].contiguous())
        assert torch.equal(Y[i], yi)


def test_deterministic_repeat(stmg):
    slab, ctx = make(CASES[4], stmg)
    U = dev(I.uniform(slab.N, 9))
    X = dev(I.uniform(slab.N, 10))
    y1 = ctx.jacobian_vmult(U, X)
    y2 = ctx.jacobian_vmult(U, X)
    assert torch.equal(y1, y2)


def _sample_rows(slab, nper, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    nt, Nv, Np = slab.nt, slab.Nv, slab.Np
    rows = []
    for a in range(nt):
        rows += list(a * Nv + rng.choice(Nv, nper, replace=False))
        rows += list(nt * Nv + a * Np + rng.choice(Np, max(2, nper // 4), replace=False))
    rows += [0, nt * Nv - 1, slab.N - 1]
    return np.array(sorted(set(int(r) for r in rows)))


@pytest.mark.parametrize("which", ["c2_16cube_r2_k2", "c3_32cube_pert_r3_k1"])
def test_full_size_sampled_rows(which, stmg):
    if which.startswith("c2"):
        d, n, r, k, nu, tau, vert = 3, (16, 16, 16), 2, 2, 1e-2, 1 / 32, None
        U = I.slab_state(d, n, r, k, 3, kind="smooth")
        nper = 12
    else:
        d, n, r, k, nu, tau = 3, (32, 32, 32), 3, 1, 1e-3, 1 / 64
        vert = I.perturbed_vertices(d, n, 0.2, 4)
        U = I.slab_state(d, n, r, k, 5, kind="smooth")
        nper = 6
    prob = oracle.Problem(dim=d, n=n, r=r, k=k, nu=nu, tau=tau, vertices=vert)
    slab = oracle.Slab(prob)
    ctx = stmg.Context(d, n, r, k, nu, tau, vertices=vert)
    X = I.uniform(slab.N, 2)
    rows = _sample_rows(slab, nper, 11)
    want = slab.vmult_rows(U, X, rows)
    Ud, Xd = dev(U), dev(X)
    got = ctx.jacobian_vmult(Ud, Xd).cpu().numpy()
    scale = np.max(np.abs(got))
    assert np.max(np.abs(got[rows] - want)) / scale < TOL64
    got32 = ctx.jacobian_vmult(Ud.float(), Xd.float()).cpu().numpy()
    assert np.max(np.abs(got32[rows] - want)) / scale < TOL32
    # FP32 against FP64 over the whole vector
    assert np.max(np.abs(got32 - got)) / scale < TOL32


def test_full_c2_vmult_whole_vector(stmg):
    """The 16^3 Q3/P2disc x DG(2) vmult benchmark workload (smooth
    divergence-free state, nu = 1e-2, tau = 1/32) over the WHOLE slab vector
    (1,181,721 entries, every cell, node and time node) against the oracle's
    element-by-element action: FP64 <= 1e-12, FP32 <= 1e-5 relative, in the
    launch configuration the benchmark times."""
    import time
    d, n, r, k, nu, tau = 3, (16, 16, 16), 2, 2, 1e-2, 1 / 32
    U = I.slab_state(d, n, r, k, 3, kind="smooth")
    slab = oracle.Slab(oracle.Problem(dim=d, n=n, r=r, k=k, nu=nu, tau=tau))
    X = I.uniform(slab.N, 2)
    t0 = time.time()
    want = slab.vmult(U, X)
    print(f"oracle element action over {slab.N} rows: {time.time() - t0:.1f} s", flush=True)
    ctx = stmg.Context(d, n, r, k, nu, tau)
    Ud, Xd = dev(U), dev(X)
    got = ctx.jacobian_vmult(Ud, Xd).cpu().numpy()
    assert rel(got, want) < TOL64
    got32 = ctx.jacobian_vmult(Ud.float(), Xd.float()).double().cpu().numpy()
    assert rel(got32, want) < TOL32
