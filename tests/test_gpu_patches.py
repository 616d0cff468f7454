"""Vanka patches on the GPU: assembly of the surrogate principal submatrices
against the oracle, and the batched mixed-size patch factorizations (C ABI
stmg_batched_lu / stmg_batched_lu_solve) on real surrogate patches of
3D cells, r in {1, 2, 3}, k in {0, 1, 2}."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import solver as S  # noqa: E402
from paper_2602_13841_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stmg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_13841_amd import stmg as Sm
    return Sm


def surrogate_patch(prob, U, cell):
    """Oracle: principal submatrix of the midpoint surrogate (eq. DefTildeHn)
    on the unknowns of `cell` (dense, FP64)."""
    slab = oracle.Slab(prob)
    V, _ = slab.split(U)
    vstar = slab.tt.phimid @ V
    Jt = slab.jacobian(U, surrogate_state=vstar)
    idx = S.patch_indices(slab)[cell]
    return Jt[idx][:, idx].toarray()


@pytest.mark.parametrize("d,n,r,k,pert", [(3, (4, 4, 4), 1, 1, True), (3, (3, 2, 2), 2, 2, False),
                                          (3, (2, 2, 2), 3, 1, True), (2, (3, 3), 3, 2, True)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_level_patch_matches_oracle(d, n, r, k, pert, prec, stmg):
    p = stmg.STMG_F64 if prec == "f64" else stmg.STMG_F32
    vert = I.perturbed_vertices(d, n, 0.2, 71) if pert else None
    prob = oracle.Problem(dim=d, n=n, r=r, k=k, nu=0.01, tau=0.05, vertices=vert)
    ctx = stmg.Context(d, n, r, k, 0.01, 0.05, vertices=vert, prec_mg=p, max_levels=2)
    U = I.uniform(ctx.N, 72)
    ctx.smoother_rebuild(torch.tensor(U, device="cuda"))
    ncell = int(np.prod(n))
    for cell in sorted({0, ncell // 2, ncell - 1}):
        got = ctx.level_patch(0, cell).double().cpu().numpy()
        want = surrogate_patch(prob, U, cell)
        err = np.max(np.abs(got - want)) / np.max(np.abs(want))
        assert err < (1e-12 if prec == "f64" else 1e-5), (cell, err)


def c4_batch(seed=6, count=9):
    """Centre-cell surrogate patches of 3x3x3-cell meshes with h = 1/8,
    nodal state U(-1, 1), nu from {1, 1e-2, 1e-3}, tau = h/2 (oracle)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = 1.0 / 8
    axes = np.arange(4) * h
    g = np.stack(np.meshgrid(axes, axes, axes, indexing="ij"), axis=-1)
    vert = g.transpose(2, 1, 0, 3).reshape(-1, 3)      # x fastest
    mats = []
    combos = [(1, 0), (1, 2), (2, 1), (3, 0), (3, 1), (3, 2), (2, 0), (1, 1), (2, 2)][:count]
    for i, (r, k) in enumerate(combos):
        nu = float(rng.choice([1.0, 1e-2, 1e-3]))
        prob = oracle.Problem(dim=3, n=(3, 3, 3), r=r, k=k, nu=nu, tau=h / 2, vertices=vert)
        U = I.uniform(oracle.Slab(prob).N, 100 + i)
        mats.append(surrogate_patch(prob, U, 13))
    return mats


def test_batched_lu_mixed_sizes(stmg):
    mats = c4_batch()
    sizes = np.array([A.shape[0] for A in mats], dtype=np.int32)
    assert sizes.min() <= 100 and sizes.max() >= 1100
    a_off = np.concatenate([[0], np.cumsum(sizes.astype(np.int64) ** 2)[:-1]])
    p_off = np.concatenate([[0], np.cumsum(sizes.astype(np.int64))[:-1]])
    rng = np.random.Generator(np.random.PCG64(7))
    rhs = [rng.uniform(-1, 1, m) for m in sizes]
    for dt, tol in ((torch.float64, 1e-13), (torch.float32, 2e-6)):
        A = torch.tensor(np.concatenate([M.ravel() for M in mats]), dtype=dt, device="cuda")
        piv = torch.zeros(int(sizes.sum()), dtype=torch.int32, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        stmg.batched_lu(A, a_off, sizes, piv, p_off, info)
        b = torch.tensor(np.concatenate(rhs), dtype=dt, device="cuda")
        stmg.batched_lu_solve(A, a_off, sizes, piv, p_off, b, p_off)
        x = b.double().cpu().numpy()
        assert int(info.item()) == 0
        for i, M in enumerate(mats):
            xi = x[p_off[i]: p_off[i] + sizes[i]]
            # normwise backward error of the computed solution
            be = np.max(np.abs(M @ xi - rhs[i])) / (np.max(np.abs(M).sum(1)) * np.max(np.abs(xi)) +
                                                    np.max(np.abs(rhs[i])))
            assert be < tol, (i, sizes[i], be)
            if dt == torch.float64:
                ref = np.linalg.solve(M, rhs[i])
                assert np.max(np.abs(xi - ref)) <= 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("which", ["bf16", "f16"])
def test_batched_lu_16bit_update_operands(which, stmg):
    """FP32 factorizations whose trailing updates take BF16 / FP16 operands
    (FP32 accumulation).  Rounding the L21 and U12 entries perturbs every
    product by at most 2u relative (u = 2^-8 for BF16, 2^-11 for FP16), so the
    computed factors are exact for A + dA with |dA| <= 2u |L||U|: the normwise
    backward error of each solve is bounded by 2u rho, rho = || |L||U| || /
    ||A|| of the matrix's partial-pivoting LU (from scipy, in FP64); checked
    with a factor 2 of slack plus the FP32 floor."""
    import scipy.linalg as sla
    mats = c4_batch()
    sizes = np.array([A.shape[0] for A in mats], dtype=np.int32)
    a_off = np.concatenate([[0], np.cumsum(sizes.astype(np.int64) ** 2)[:-1]])
    p_off = np.concatenate([[0], np.cumsum(sizes.astype(np.int64))[:-1]])
    rng = np.random.Generator(np.random.PCG64(8))
    rhs = [rng.uniform(-1, 1, m) for m in sizes]
    prec, u = (stmg.STMG_F32_BF16, 2.0 ** -8) if which == "bf16" else (stmg.STMG_F32_F16, 2.0 ** -11)
    xs = {}
    for name, p in (("f32", None), (which, prec)):
        A = torch.tensor(np.concatenate([M.ravel() for M in mats]), dtype=torch.float32, device="cuda")
        piv = torch.zeros(int(sizes.sum()), dtype=torch.int32, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        stmg.batched_lu(A, a_off, sizes, piv, p_off, info, prec=p)
        b = torch.tensor(np.concatenate(rhs), dtype=torch.float32, device="cuda")
        stmg.batched_lu_solve(A, a_off, sizes, piv, p_off, b, p_off)
        assert int(info.item()) == 0
        xs[name] = b.double().cpu().numpy()
    assert not np.array_equal(xs["f32"], xs[which])     # the 16-bit path really ran
    for i, M in enumerate(mats):
        _, L, U = sla.lu(M)
        rho = np.max((np.abs(L) @ np.abs(U)).sum(1)) / np.max(np.abs(M).sum(1))
        xi = xs[which][p_off[i]: p_off[i] + sizes[i]]
        be = np.max(np.abs(M @ xi - rhs[i])) / (np.max(np.abs(M).sum(1)) * np.max(np.abs(xi)) +
                                                np.max(np.abs(rhs[i])))
        assert be < 4 * u * rho + 2e-6, (i, sizes[i], be, rho)


@pytest.mark.parametrize("config", [(0, None), (1, [16] * 5), (2, [8] * 5, 512), (3, [4, 8, 16, 16, 8]),
                                    (1, [16] * 5, 512), (4, [16, 16, 8, 4, 4])],
                         ids=lambda c: f"wg{c[0]}_t{c[2] if len(c) > 2 else 256}")
def test_batched_lu_launch_configurations(config, stmg):
    """The persistent work-queue factorization with any workgroups-per-CU /
    panel-width setting the tuner may choose (and the one-launch-per-size-
    class reference): every solve has a normwise backward error at the
    precision's level, and the zero-pivot count is zero."""
    rng = np.random.Generator(np.random.PCG64(19))
    sizes = [int(m) for m in rng.choice([85, 170, 202, 255, 395, 404, 606, 790, 1185], 23)] + [1, 2, 33]
    mats = []
    for i, m in enumerate(sizes):
        A = I.uniform(m * m, 500 + i).reshape(m, m)
        A[np.arange(m), np.arange(m)] += 0.5 * m ** 0.5
        mats.append(A)
    m64 = np.array(sizes, dtype=np.int64)
    a_off = np.concatenate([[0], np.cumsum(m64 ** 2)[:-1]])
    p_off = np.concatenate([[0], np.cumsum(m64)[:-1]])
    rhs = [I.uniform(m, 900 + i) for i, m in enumerate(sizes)]
    for dt, tol in ((torch.float64, 1e-13), (torch.float32, 2e-6)):
        A = torch.tensor(np.concatenate([M.ravel() for M in mats]), dtype=dt, device="cuda")
        piv = torch.zeros(int(m64.sum()), dtype=torch.int32, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        stmg.batched_lu(A, a_off, sizes, piv, p_off, info, config=config)
        b = torch.tensor(np.concatenate(rhs), dtype=dt, device="cuda")
        stmg.batched_lu_solve(A, a_off, sizes, piv, p_off, b, p_off)
        x = b.double().cpu().numpy()
        assert int(info.item()) == 0
        for i, M in enumerate(mats):
            xi = x[p_off[i]: p_off[i] + sizes[i]]
            be = np.max(np.abs(M @ xi - rhs[i])) / (np.max(np.abs(M).sum(1)) * np.max(np.abs(xi)) +
                                                    np.max(np.abs(rhs[i])))
            assert be < tol, (config, dt, i, sizes[i], be)
