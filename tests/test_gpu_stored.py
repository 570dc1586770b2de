"""Stored-H mode (H restricted to S built once into CSR on the device, then a
sparse product per iteration) against the oracle, through the C ABI.

* The stored matrix itself against the oracle's memoised H (the definition-
  based elements, pinned to the dense H and the matrix-free product on the
  CPU): row pointers identical, each row's column set identical (bit-exact),
  the diagonal first, values within 1e-12 of max |H_IJ|.
* The product against the oracle sigma (small spaces) and against the
  matrix-free product and sampled oracle rows (the 4.0e6-determinant
  workload, 2.66e9 stored elements): max-norm and 2-norm relative <= 1e-12.
* Davidson on the stored product against dense eigh and the stored oracle
  energy: <= 1e-8 Ha.
* Error paths: product before the build or after a Hamiltonian change
  (SQD_E_STATE), the stored product in mixed precision (SQD_E_INVALID_ARG).
"""
import json
import os

import numpy as np
import pytest

from paper_2601_16169_amd import inputs as I
from oracle import core, davidson
from tests.gpu_util import banner, need_gpu, rel_err

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

SMALL = [
    ("complete_4_2_2", lambda: I.small_problem(4, 2, 2, 6, 6, 1)),
    ("ragged_8_3_4", lambda: I.small_problem(8, 3, 4, 37, 53, 3)),
    ("sab_neq_10_4_3", lambda: I.small_problem(10, 4, 3, 70, 97, 4)),
    ("one_alpha_string", lambda: I.small_problem(6, 2, 3, 1, 20, 5)),
    ("one_beta_string", lambda: I.small_problem(6, 2, 3, 15, 1, 6)),
    ("zero_alpha_electrons", lambda: I.small_problem(5, 0, 2, 1, 10, 7)),
    ("cfg1", I.cfg1),
]


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


@pytest.mark.parametrize("name,make", SMALL)
def test_stored_matrix_matches_oracle(ctx, name, make):
    banner(f"stored H {name}")
    p = make()
    sp = _space(ctx, p)
    nnz = sp.store_hamiltonian()
    assert nnz == sp.info()["conn_per_sigma"]
    rp, cols, vals = sp.stored_hamiltonian(nnz)
    ref = core.MemoisedH(core.Space.from_problem(p))
    assert np.array_equal(rp, ref.rowptr)
    scale = np.abs(ref.vals).max()
    for r in range(sp.dim):
        a, b = rp[r], rp[r + 1]
        assert cols[a] == r and ref.cols[a] == r            # diagonal first
        og, orf = np.argsort(cols[a:b], kind="stable"), np.argsort(ref.cols[a:b], kind="stable")
        assert np.array_equal(cols[a:b][og], ref.cols[a:b][orf]), f"row {r} columns"
        assert np.abs(vals[a:b][og] - ref.vals[a:b][orf]).max() <= 1e-12 * scale, f"row {r} values"
    sp.close()


@pytest.mark.parametrize("name,make", SMALL)
def test_spmv_matches_oracle_sigma(ctx, name, make):
    torch = need_gpu()
    banner(f"spmv {name}")
    p = make()
    sp = _space(ctx, p)
    sp.store_hamiltonian()
    c = I.random_vector(sp.dim, 5)
    got = sp.spmv(torch.tensor(c, device="cuda:0")).cpu().numpy()
    ref = core.Space.from_problem(p).sigma(c)
    e_inf, e_2 = rel_err(got, ref)
    assert e_inf <= 1e-12 and e_2 <= 1e-12, (e_inf, e_2)
    sp.close()


@pytest.mark.parametrize("name,make", [SMALL[1], SMALL[2], SMALL[6]])
def test_davidson_on_stored_h_matches_dense(ctx, name, make):
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner(f"davidson stored {name}")
    p = make()
    sp = _space(ctx, p)
    sp.store_hamiltonian()
    E_ref, x_ref, _ = davidson.dense_lowest(core.Space.from_problem(p).dense())
    E, x, rep = sp.davidson(tol=1e-10, noise=torch.tensor(I.guess_noise(sp.dim), device="cuda:0"),
                            product=sqd.PRODUCT_STORED)
    assert rep["converged"]
    assert abs(E - E_ref) <= 1e-8, (E, E_ref)
    assert 1 - abs(x.cpu().numpy() @ x_ref) <= 1e-12
    sp.close()


def test_stored_cfg2_product_and_davidson(ctx):
    """The 4.0e6-determinant workload: 2.66e9 stored elements (32 GB)."""
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner("stored H cfg2: build, product vs matrix-free and oracle rows, Davidson")
    p = I.cfg2()
    sp = _space(ctx, p)
    nnz = sp.store_hamiltonian()
    assert nnz == sp.info()["conn_per_sigma"]
    c = torch.tensor(I.random_vector(sp.dim, 9), device="cuda:0")
    got = sp.spmv(c)
    ref = sp.sigma(c)
    e_inf, e_2 = rel_err(got.cpu().numpy(), ref.cpu().numpy())
    assert e_inf <= 1e-12 and e_2 <= 1e-12, (e_inf, e_2)
    rows = np.random.default_rng(4).choice(sp.dim, 2048, replace=False)
    oref = core.Space.from_problem(p).sigma_rows(c.cpu().numpy(), rows)
    g = got.cpu().numpy()[rows]
    assert np.abs(g - oref).max() <= 1e-12 * np.abs(oref).max()
    gold = json.load(open(os.path.join(GOLDEN, "cfg2_oracle.json")))
    E, x, rep = sp.davidson(tol=1e-8, noise=torch.tensor(I.guess_noise(sp.dim), device="cuda:0"),
                            product=sqd.PRODUCT_STORED)
    assert rep["converged"]
    assert abs(E - gold["energy"]) <= 1e-8, (E, gold["energy"])
    sp.release_hamiltonian()
    sp.close()


def test_stored_error_paths(ctx):
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner("stored H error paths")
    p = I.small_problem(8, 3, 4, 37, 53, 3)
    sp = _space(ctx, p)
    c = torch.tensor(I.random_vector(sp.dim, 1), device="cuda:0")
    with pytest.raises(sqd.SQDError) as ei:
        sp.spmv(c)
    assert ei.value.code == -8
    with pytest.raises(sqd.SQDError) as ei:
        sp.davidson(product=sqd.PRODUCT_STORED)
    assert ei.value.code == -8
    sp.store_hamiltonian()
    with pytest.raises(sqd.SQDError) as ei:
        sp.davidson(mode=sqd.DAV_MIXED, product=sqd.PRODUCT_STORED)
    assert ei.value.code == -1
    # a new Hamiltonian (same norb) makes the stored H stale until rebuilt
    ctx.set_hamiltonian(p.ints.h * 0.5, p.ints.eri, p.ints.ecore)
    with pytest.raises(sqd.SQDError) as ei:
        sp.spmv(c)
    assert ei.value.code == -8
    sp.store_hamiltonian()
    got = sp.spmv(c).cpu().numpy()
    ref = core.Space(p.norb, p.astr, p.bstr, p.ints.h * 0.5, p.ints.eri).sigma(c.cpu().numpy())
    e_inf, e_2 = rel_err(got, ref)
    assert e_inf <= 1e-12 and e_2 <= 1e-12
    sp.release_hamiltonian()
    with pytest.raises(sqd.SQDError) as ei:
        sp.spmv(c)
    assert ei.value.code == -8
    sp.close()
