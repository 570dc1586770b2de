"""Block Davidson (the lowest k roots in one subspace) against dense eigh of
the oracle's H, and against the locking solver and the oracle sigma on the
4.0e6-determinant workload, through the C ABI.

Bars: FP64 energies <= 1e-8 Ha and 1 - |<x_j, x_ref_j>| <= 1e-9 for roots
separated from their neighbours by more than 1e-6 Ha; mixed precision
energies <= 1e-6 Ha.
"""
import functools

import numpy as np
import pytest

from paper_2601_16169_amd import inputs as I
from oracle import core
from tests.gpu_util import banner, need_gpu

pytestmark = pytest.mark.gpu

CASES = {
    "cfg1": I.cfg1,
    "ragged_8_3_4": lambda: I.small_problem(8, 3, 4, 37, 53, 3),
    "sab_neq_10_4_3": lambda: I.small_problem(10, 4, 3, 70, 97, 4),
}


@functools.lru_cache(maxsize=None)
def _dense(name):
    p = CASES[name]()
    w, v = np.linalg.eigh(core.Space.from_problem(p).dense())
    return w, v


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_2601_16169_amd import sqd
    c = sqd.Context(0)
    yield c
    c.close()


def _space(ctx, p):
    ctx.set_hamiltonian(p.ints.h, p.ints.eri, p.ints.ecore)
    return ctx.build_space(p.nalpha, p.nbeta, p.astr, p.bstr)


def _check(E, X, w, v, tolE, vec_bar):
    k = len(E)
    assert np.abs(np.asarray(E) - w[:k]).max() <= tolE, (E, w[:k])
    if vec_bar is None:
        return
    for j in range(k):
        gap = min(abs(w[j] - w[j - 1]) if j > 0 else np.inf, abs(w[j + 1] - w[j]))
        x = X[j]
        assert abs(np.linalg.norm(x) - 1) <= 1e-12
        i = int(np.argmax(np.abs(x)))
        assert x[i] > 0
        if gap > 1e-6:
            assert 1 - abs(x @ v[:, j]) <= vec_bar, (j, 1 - abs(x @ v[:, j]))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("nroots", [1, 4])
def test_block_fp64_matches_dense(ctx, name, nroots):
    banner(f"block davidson fp64 {name} k={nroots}")
    p = CASES[name]()
    sp = _space(ctx, p)
    w, v = _dense(name)
    E, X, reps = sp.davidson_block(nroots, tol=1e-9, max_iter=400)
    print("iterations", reps[0]["iterations"], "products", reps[0]["products"])
    assert all(r["converged"] for r in reps), [r["residual"] for r in reps]
    _check(E, X.cpu().numpy(), w, v, 1e-8, 1e-9)
    sp.close()


@pytest.mark.parametrize("name", ["cfg1", "sab_neq_10_4_3"])
def test_block_mixed_matches_dense(ctx, name):
    from paper_2601_16169_amd import sqd
    banner(f"block davidson mixed {name}")
    p = CASES[name]()
    sp = _space(ctx, p)
    w, v = _dense(name)
    E, X, reps = sp.davidson_block(4, tol=1e-8, max_iter=400, mode=sqd.DAV_MIXED, switch_tol=1e-4)
    assert all(r["converged"] for r in reps)
    assert reps[0]["switch_iter"] > 0 and reps[0]["iterations_fp32"] > 0
    _check(E, X.cpu().numpy(), w, v, 1e-6, None)
    sp.close()


@pytest.mark.parametrize("nroots,m_max", [(8, 32), (4, 12)])
def test_block_many_roots_and_restarts(ctx, nroots, m_max):
    banner(f"block davidson {nroots} roots, m_max {m_max}")
    p = CASES["cfg1"]()
    sp = _space(ctx, p)
    w, v = _dense("cfg1")
    E, X, reps = sp.davidson_block(nroots, tol=1e-9, m_max=m_max, max_iter=600)
    print("iterations", reps[0]["iterations"], "products", reps[0]["products"], "status", reps[0]["status"],
          "residuals", [r["residual"] for r in reps])
    assert all(r["converged"] for r in reps)
    _check(E, X.cpu().numpy(), w, v, 1e-8, 1e-9)
    sp.close()


def test_block_on_stored_product(ctx):
    from paper_2601_16169_amd import sqd
    banner("block davidson on the stored H")
    p = CASES["ragged_8_3_4"]()
    sp = _space(ctx, p)
    sp.store_hamiltonian()
    w, v = _dense("ragged_8_3_4")
    E, X, reps = sp.davidson_block(4, tol=1e-9, product=sqd.PRODUCT_STORED)
    assert all(r["converged"] for r in reps)
    _check(E, X.cpu().numpy(), w, v, 1e-8, 1e-9)
    sp.close()


def test_block_cfg2_matches_locking_and_oracle_rows(ctx):
    """4 roots of the 4.0e6-determinant workload: energies against the
    locking solver (<= 1e-8 Ha), and every vector's residual under the
    oracle sigma on 512 seeded rows."""
    torch = need_gpu()
    banner("block davidson cfg2, 4 roots")
    p = I.cfg2()
    sp = _space(ctx, p)
    E, X, reps = sp.davidson_block(4, tol=1e-8, max_iter=600)
    assert all(r["converged"] for r in reps)
    El, Xl, _ = sp.davidson_roots(4, tol=1e-8, noise=torch.tensor(I.guess_noise(sp.dim), device="cuda:0"),
                                  max_iter=600)
    assert np.abs(np.asarray(E) - np.asarray(El)).max() <= 1e-8, (E, El)
    osp = core.Space.from_problem(p)
    rows = np.random.default_rng(6).choice(sp.dim, 512, replace=False)
    Xn = X.cpu().numpy()
    for j in range(4):
        hx = osp.sigma_rows(Xn[j], rows)
        assert np.abs(hx - E[j] * Xn[j][rows]).max() <= 1e-8
    G = Xn @ Xn.T
    assert np.abs(G - np.eye(4)).max() <= 1e-10
    sp.close()


def test_block_argument_errors(ctx):
    from paper_2601_16169_amd import sqd
    p = CASES["cfg1"]()
    sp = _space(ctx, p)
    with pytest.raises(sqd.SQDError) as ei:
        sp.davidson_block(4, m_max=6)
    assert ei.value.code == -1
    with pytest.raises(sqd.SQDError) as ei:
        sp.davidson_block(9)
    assert ei.value.code == -1
    sp.close()
