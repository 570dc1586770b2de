"""GPU Davidson (FP64 and FP32-sigma + FP64 refinement) against the oracle:
dense eigh where the space is small, the stored oracle Davidson result for the
4.0e6-determinant workload, and residual checks with the oracle sigma.

Bars: FP64 energy <= 1e-8 Ha, vector 1 - |<x, x_ref>| <= 1e-12 (when the
reference vector is available); mixed energy <= 1e-6 Ha.
"""
import json
import os

import numpy as np
import pytest

from paper_2601_16169_amd import inputs as I
from oracle import core, davidson
from tests.gpu_util import banner, need_gpu

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def _noise(torch, dim):
    return torch.tensor(I.guess_noise(dim), device="cuda:0")


CASES = [
    ("cfg1", I.cfg1, 1e-10),
    ("ragged_8_3_4", lambda: I.small_problem(8, 3, 4, 37, 53, 3), 1e-10),
    ("sab_neq_10_4_3", lambda: I.small_problem(10, 4, 3, 70, 97, 4), 1e-9),
    ("tiny_dim_6", lambda: I.small_problem(4, 1, 1, 2, 3, 8), 1e-10),
]


@pytest.mark.parametrize("name,make,tol", CASES)
def test_fp64_matches_dense(ctx, name, make, tol):
    torch = need_gpu()
    banner(f"davidson fp64 {name}")
    p = make()
    sp = _space(ctx, p)
    E_ref, x_ref, _ = davidson.dense_lowest(core.Space.from_problem(p).dense())
    E, x, rep = sp.davidson(tol=tol, noise=_noise(torch, sp.dim))
    assert rep["converged"], rep["status"]
    assert abs(E - E_ref) <= 1e-8, (E, E_ref)
    xv = x.cpu().numpy()
    assert abs(np.linalg.norm(xv) - 1) <= 1e-12
    assert 1 - abs(xv @ x_ref) <= 1e-12
    sp.close()


@pytest.mark.parametrize("m_max", [2, 4, 7])
def test_collapse_paths(ctx, m_max):
    torch = need_gpu()
    p = I.small_problem(8, 3, 4, 37, 53, 3)
    sp = _space(ctx, p)
    E_ref = np.linalg.eigvalsh(core.Space.from_problem(p).dense())[0]
    E, x, rep = sp.davidson(tol=1e-9, m_max=m_max, max_iter=400, noise=_noise(torch, sp.dim))
    assert rep["converged"] and abs(E - E_ref) <= 1e-8
    sp.close()


def test_explicit_guess_and_phase(ctx):
    torch = need_gpu()
    p = I.cfg1()
    sp = _space(ctx, p)
    osp = core.Space.from_problem(p)
    E_ref, x_ref, _ = davidson.dense_lowest(osp.dense())
    g = torch.tensor(I.random_vector(sp.dim, 3), device="cuda:0")
    E, x, rep = sp.davidson(tol=1e-10, guess=g)
    xv = x.cpu().numpy()
    assert abs(E - E_ref) <= 1e-8
    k = int(np.argmax(np.abs(xv)))
    assert xv[k] > 0 and np.allclose(xv, x_ref, atol=1e-9)
    sp.close()


@pytest.mark.parametrize("name,make,tol", CASES[:3])
def test_mixed_matches_dense(ctx, name, make, tol):
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner(f"davidson mixed {name}")
    p = make()
    sp = _space(ctx, p)
    E_ref = np.linalg.eigvalsh(core.Space.from_problem(p).dense())[0]
    E, x, rep = sp.davidson(tol=tol, mode=sqd.DAV_MIXED, switch_tol=1e-4, noise=_noise(torch, sp.dim))
    assert rep["converged"]
    assert rep["switch_iter"] >= 1
    assert abs(E - E_ref) <= 1e-6
    sp.close()


def test_max_iter_cap_reports_not_converged(ctx):
    torch = need_gpu()
    p = I.cfg1()
    sp = _space(ctx, p)
    E, x, rep = sp.davidson(tol=1e-14, max_iter=3, noise=_noise(torch, sp.dim))
    assert not rep["converged"] and rep["status_code"] == 1 and rep["iterations"] == 3
    sp.close()


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}_oracle.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return json.load(open(path))


@pytest.mark.parametrize("mode", [0, 1])
def test_cfg2_against_stored_oracle(ctx, mode):
    """4.0e6 determinants against the oracle's Davidson over the memoised H
    (converged to 1e-11; stored by tests/golden/make_golden.py): the energy,
    and the vector element by element on its 4096 largest entries plus 65,536
    seeded rows.  FP64 solves to 1e-11 like the oracle: energy <= 1e-8 Ha,
    vector entries <= 1e-9.  Mixed precision solves to the benchmark's 1e-8:
    energy <= 1e-6 Ha, vector entries <= 1e-6 (the benchmark spec states the
    mixed vector error rather than gating it; this bound is a sanity check).
    Also the residual of the GPU vector under the oracle sigma on sampled
    rows."""
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    gold = _golden("cfg2")
    z = np.load(os.path.join(GOLDEN, gold["vector_file"]))
    idx, ref = z["index"], z["value"]
    banner(f"davidson cfg2 mode={mode}")
    p = I.cfg2()
    sp = _space(ctx, p)
    tol = 1e-11 if mode == 0 else 1e-8
    E, x, rep = sp.davidson(tol=tol, mode=mode, noise=_noise(torch, sp.dim), max_iter=1000)
    assert rep["converged"]
    tolE = 1e-8 if mode == 0 else 1e-6
    assert abs(E - gold["energy"]) <= tolE, (E, gold["energy"])
    xv = x.cpu().numpy()
    # Phase: the largest-magnitude entry is positive.  When the two largest
    # magnitudes agree to within the solver tolerance (a flip-odd state puts
    # equal weight on (ia, ib) and (ib, ia)), either choice satisfies the rule,
    # so the vectors are compared up to that one global sign and the rule is
    # checked on the GPU vector itself.
    k = int(np.argmax(np.abs(xv)))
    assert xv[k] > 0
    order = np.argsort(-np.abs(ref))
    mag = np.abs(ref[order])
    sgn = 1.0
    if mag[0] - mag[1] <= 1e-6 * mag[0]:
        sgn = float(np.sign(xv[idx] @ ref))
    err = float(np.abs(sgn * xv[idx] - ref).max())
    print(f"cfg2 mode {mode}: |dE| {abs(E - gold['energy']):.2e}, max vector error on {len(idx)} rows {err:.2e}")
    assert err <= (1e-9 if mode == 0 else 1e-6), err
    rows = np.unique(np.concatenate([idx[order[:64]], np.random.default_rng(3).choice(sp.dim, 512, replace=False)]))
    hx = core.Space.from_problem(p).sigma_rows(xv, rows)
    assert np.abs(hx - E * xv[rows]).max() <= (1e-9 if mode == 0 else 1e-7)
    sp.close()


def test_default_start_reaches_flip_odd_ground_state(ctx):
    """norb 6, 3+3, all strings, integral seed 9: the lowest state is odd under
    the exchange of alpha and beta strings, which the start e_argmin(H_II) alone
    (even) cannot reach.  With neither noise nor a guess passed, the library's
    own start noise reaches it, in the single-space and the batched solver."""
    need_gpu()
    s = I.all_strings(6, 3)
    p = I.Problem("flip_odd_6_3", I.make_integrals(6, 12, seed=9), 3, 3, s, s.copy())
    sp = _space(ctx, p)
    w = np.linalg.eigvalsh(core.Space.from_problem(p).dense())
    E, x, rep = sp.davidson(tol=1e-10)
    assert rep["converged"] and abs(E - w[0]) <= 1e-8, (E, w[:2])
    xv = x.cpu().numpy().reshape(sp.na, sp.nb)
    assert np.abs(xv + xv.T).max() <= 1e-8
    Eb, _, reps, rc = ctx.davidson_batched([sp], tol=1e-10)
    assert rc == 0 and abs(Eb[0] - w[0]) <= 1e-8
    sp.close()


def test_workspace_reuse_and_release(ctx):
    """Solves on spaces of different sizes reuse and grow the context's
    workspaces; after sqd_release_workspace the next solve allocates again and
    gives the same result."""
    torch = need_gpu()
    big = I.small_problem(8, 3, 4, 37, 53, 3)
    small = I.small_problem(6, 3, 2, 13, 11, 2)
    res = []
    for p in (big, small, big):
        sp = _space(ctx, p)
        E, x, rep = sp.davidson(tol=1e-10, noise=_noise(torch, sp.dim))
        res.append(E)
        sp.close()
    assert res[0] == res[2]
    ctx.release_workspace()
    sp = _space(ctx, big)
    E, x, rep = sp.davidson(tol=1e-10, noise=_noise(torch, sp.dim))
    assert E == res[0]
    Eb, _, reps, rc = ctx.davidson_batched([sp], tol=1e-10)
    ctx.release_workspace()
    Eb2, _, reps, rc = ctx.davidson_batched([sp], tol=1e-10)
    assert Eb == Eb2
    sp.close()


ROOT_CASES = [CASES[0], CASES[1], CASES[2]]


@pytest.mark.parametrize("name,make,tol", ROOT_CASES)
@pytest.mark.parametrize("mode", [0, 1])
def test_roots_match_dense(ctx, name, make, tol, mode):
    """Four lowest roots by locking against dense eigh: energies (1e-8 Ha FP64,
    1e-6 Ha mixed), orthonormal vectors, each vector along its eigenvector
    where the root is separated from its neighbours."""
    torch = need_gpu()
    banner(f"roots {name} mode={mode}")
    p = make()
    sp = _space(ctx, p)
    w, U = np.linalg.eigh(core.Space.from_problem(p).dense())
    k = 4
    E, X, reps = sp.davidson_roots(k, tol=tol, mode=mode, max_iter=400, noise=_noise(torch, sp.dim))
    assert all(r["converged"] for r in reps)
    tolE = 1e-8 if mode == 0 else 1e-6
    assert np.abs(np.array(E) - w[:k]).max() <= tolE, (E, w[:k])
    Xn = X.cpu().numpy()
    assert np.abs(Xn @ Xn.T - np.eye(k)).max() <= 1e-9
    for j in range(k):
        gap = min(abs(w[j] - w[j - 1]) if j else np.inf, abs(w[j + 1] - w[j]))
        if gap > 1e-4:
            assert 1 - abs(Xn[j] @ U[:, j]) <= (1e-8 if mode == 0 else 1e-5), (j, gap)
        assert Xn[j][np.argmax(np.abs(Xn[j]))] > 0
    sp.close()
