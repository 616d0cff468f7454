"""The allocation-free batched LU entry point (stmg_batched_lu_noalloc) on
the GPU: through the C ABI it gives the same factors, pivots and zero-pivot
count as stmg_batched_lu on the same batch, on two calls in a row (the
second with a smaller batch, so stale metadata from the first call in the
library's fixed array would show), and it rejects a batch above its fixed
capacity."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2602_13841_amd import inputs as I  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stmg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_13841_amd import stmg as Sm
    return Sm


def _batch(sizes, seed, dt):
    mats = []
    for i, m in enumerate(sizes):
        A = I.uniform(m * m, seed + i).reshape(m, m)
        A[np.arange(m), np.arange(m)] += 0.1 * m ** 0.5      # not too ill-conditioned
        mats.append(A)
    a_off = np.concatenate([[0], np.cumsum(np.asarray(sizes, dtype=np.int64) ** 2)[:-1]])
    p_off = np.concatenate([[0], np.cumsum(np.asarray(sizes, dtype=np.int64))[:-1]])
    A = torch.tensor(np.concatenate([M.ravel() for M in mats]), dtype=dt, device="cuda")
    return mats, A, a_off, p_off


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_noalloc_equals_batched_lu_on_two_calls(dt, stmg):
    rng = np.random.Generator(np.random.PCG64(17))
    first = [int(m) for m in rng.integers(20, 1200, 40)] + [1185, 85]
    second = [int(m) for m in rng.integers(10, 300, 7)]
    for call, sizes in enumerate((first, second)):
        print(f"call {call}: {len(sizes)} matrices, m {min(sizes)}..{max(sizes)}, {dt}", flush=True)
        mats, A0, a_off, p_off = _batch(sizes, 300 + 50 * call, dt)
        A1 = A0.clone()
        npiv = int(sum(sizes))
        piv0 = torch.full((npiv,), -7, dtype=torch.int32, device="cuda")
        piv1 = piv0.clone()
        info0 = torch.zeros(1, dtype=torch.int32, device="cuda")
        info1 = torch.zeros(1, dtype=torch.int32, device="cuda")
        stmg.batched_lu(A0, a_off, sizes, piv0, p_off, info0)
        stmg.batched_lu(A1, a_off, sizes, piv1, p_off, info1, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(piv0, piv1)
        assert torch.equal(A0, A1)
        assert int(info0.item()) == int(info1.item()) == 0
        # and the factors are those of the matrices: P A = L U on two of them
        for i in (0, len(sizes) - 1):
            m = sizes[i]
            F = A1[a_off[i]: a_off[i] + m * m].double().cpu().numpy().reshape(m, m)
            L = np.tril(F, -1) + np.eye(m)
            U = np.triu(F)
            PA = mats[i].copy()
            pv = piv1[p_off[i]: p_off[i] + m].cpu().numpy()
            for j in range(m):
                PA[[j, pv[j]]] = PA[[pv[j], j]]
            tol = 1e-12 if dt == torch.float64 else 2e-5
            assert np.max(np.abs(L @ U - PA)) <= tol * np.max(np.abs(PA)) * m ** 0.5


def test_noalloc_rejects_batches_above_capacity(stmg):
    n = stmg.STMG_NOALLOC_MAX_BATCH + 1
    sizes = np.ones(n, dtype=np.int32)
    offs = np.arange(n, dtype=np.int64)
    A = torch.zeros(n, dtype=torch.float32, device="cuda")
    piv = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(stmg.StmgError):
        stmg.batched_lu(A, offs, sizes, piv, offs, noalloc=True)
