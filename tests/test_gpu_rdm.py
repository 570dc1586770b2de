"""GPU reduced density matrices and the autograd energy against the oracle.

RDMs: elementwise against the oracle's operator-by-operator RDMs of the same
vector (<= 1e-12 relative to the largest entry); at the full 1.6e7-determinant
workload, properties that hold at any size (traces, symmetry, the energy they
reproduce).  Gradients: central finite differences of the GPU energy over
symmetry orbits of integral entries (step 1e-5), |FD - analytic| <=
1e-6 + 1e-5 |analytic|.
"""
import numpy as np
import pytest

from paper_2601_16169_amd import inputs as I
from oracle import core, davidson
from tests.gpu_util import banner, need_gpu

pytestmark = pytest.mark.gpu


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


CASES = [
    ("ragged_6_3_2", lambda: I.small_problem(6, 3, 2, 13, 11, 2)),
    ("sab_neq_10_4_3", lambda: I.small_problem(10, 4, 3, 70, 97, 4)),
    ("cfg1", I.cfg1),
    ("norb20_n7_300", lambda: I.Problem("norb20_n7_300", I.make_integrals(20, 50, seed=5), 7, 7,
                                        I.sample_strings(20, 7, 300, seed=105),
                                        I.sample_strings(20, 7, 300, seed=105))),
    ("norb36_n12_120", lambda: I.small_problem(36, 12, 12, 120, 90, 6)),
]


@pytest.mark.parametrize("name,make", CASES)
def test_rdm_matches_oracle(ctx, name, make):
    torch = need_gpu()
    banner(f"rdm {name}")
    p = make()
    sp = _space(ctx, p)
    c = I.random_vector(sp.dim, 31)
    c /= np.linalg.norm(c)
    g1, g2 = sp.rdm(torch.tensor(c, device="cuda:0"))
    o1, o2 = core.Space.from_problem(p).rdm(c)
    g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
    assert np.abs(g1 - o1).max() <= 1e-12 * max(1.0, np.abs(o1).max())
    assert np.abs(g2 - o2).max() <= 1e-12 * max(1.0, np.abs(o2).max())
    sp.close()


def test_rdm_energy_and_invariants_cfg1(ctx):
    torch = need_gpu()
    p = I.cfg1()
    sp = _space(ctx, p)
    E, x, rep = sp.davidson(tol=1e-10, noise=torch.tensor(I.guess_noise(sp.dim), device="cuda:0"))
    g1, g2 = sp.rdm(x)
    g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
    E_rdm = float(np.sum(p.ints.h * g1) + 0.5 * np.sum(p.ints.eri * g2))
    assert abs(E_rdm - E) <= 1e-10
    assert abs(np.trace(g1) - 8) <= 1e-12
    assert abs(np.einsum("pprr->", g2) - 8 * 7) <= 1e-10
    assert np.abs(g2 - g2.transpose(2, 3, 0, 1)).max() <= 1e-12
    w = np.linalg.eigvalsh(g1)
    assert w.min() >= -1e-12 and w.max() <= 2 + 1e-12
    sp.close()


def test_one_body_only(ctx):
    torch = need_gpu()
    p = I.small_problem(8, 3, 4, 37, 53, 3)
    sp = _space(ctx, p)
    c = I.random_vector(sp.dim, 2)
    c /= np.linalg.norm(c)
    g1, g2 = sp.rdm(torch.tensor(c, device="cuda:0"), two_body=False)
    o1, _ = core.Space.from_problem(p).rdm(c)
    assert g2 is None and np.abs(g1.cpu().numpy() - o1).max() <= 1e-13
    sp.close()


def _orbits(norb, count, seed):
    """Symmetry orbits of h pairs and (pq|rs) 8-tuples, chosen uniformly."""
    rng = np.random.default_rng(seed)
    hs = [("h", (p, q)) for p in range(norb) for q in range(p, norb)]
    vs = set()
    while len(vs) < 4 * count:
        p, q, r, s = (int(v) for v in rng.integers(0, norb, 4))
        key = min([(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                   (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)])
        vs.add(key)
    pool = hs + [("v", k) for k in sorted(vs)]
    idx = rng.choice(len(pool), size=count, replace=False)
    return [pool[i] for i in idx]


def _members(kind, k):
    if kind == "h":
        p, q = k
        return {(p, q), (q, p)}
    p, q, r, s = k
    return {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
            (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}


def _fd_check(ctx, p, norbits, seed, tol):
    torch = need_gpu()
    from paper_2601_16169_amd import autograd
    sp = _space(ctx, p)
    h = torch.tensor(p.ints.h, requires_grad=True)
    eri = torch.tensor(p.ints.eri, requires_grad=True)
    noise = torch.tensor(I.guess_noise(sp.dim), device="cuda:0")
    E = autograd.energy(h, eri, sp, tol=tol, noise=noise)
    E.backward()
    gh, ge = h.grad.numpy(), eri.grad.numpy()
    _, x0, _ = sp.davidson(tol=tol, noise=noise)
    d = 1e-5
    worst = 0.0
    for kind, k in _orbits(p.norb, norbits, seed):
        mem = _members(kind, k)
        out = []
        for sgn in (+1, -1):
            hh, ee = p.ints.h.copy(), p.ints.eri.copy()
            for m in mem:
                if kind == "h":
                    hh[m] += sgn * d
                else:
                    ee[m] += sgn * d
            ctx.set_hamiltonian(hh, ee)
            Ei, _, rep = sp.davidson(tol=tol, guess=x0)
            assert rep["converged"]
            out.append(Ei)
        fd = (out[0] - out[1]) / (2 * d)
        an = sum((gh if kind == "h" else ge)[m] for m in mem)
        worst = max(worst, abs(fd - an) - 1e-5 * abs(an))
        assert abs(fd - an) <= 1e-6 + 1e-5 * abs(an), (kind, k, fd, an)
    sp.close()
    return worst


def test_autograd_matches_finite_differences_cfg1(ctx):
    banner("autograd FD cfg1")
    _fd_check(ctx, I.cfg1(), 50, 55, 1e-11)


def test_autograd_matches_oracle_rdm(ctx):
    """Gradients equal the oracle's RDMs of the oracle's own eigenvector."""
    torch = need_gpu()
    from paper_2601_16169_amd import autograd
    p = I.small_problem(8, 3, 3, 40, 40, 12)
    sp = _space(ctx, p)
    osp = core.Space.from_problem(p)
    _, xr, _ = davidson.dense_lowest(osp.dense())
    o1, o2 = osp.rdm(xr)
    h = torch.tensor(p.ints.h, requires_grad=True)
    eri = torch.tensor(p.ints.eri, requires_grad=True)
    E = autograd.energy(h, eri, sp, tol=1e-11, noise=torch.tensor(I.guess_noise(sp.dim), device="cuda:0"))
    E.backward()
    assert np.abs(h.grad.numpy() - o1).max() <= 1e-8
    assert np.abs(eri.grad.numpy() - 0.5 * o2).max() <= 1e-8
    sp.close()


@pytest.mark.slow
def test_cfg5_rdm_and_finite_differences(ctx):
    """Full 1.6e7-determinant workload: RDM properties at the converged vector
    and central differences on 50 symmetry orbits (warm-started solves)."""
    torch = need_gpu()
    banner("rdm cfg5")
    p = I.cfg5()
    sp = _space(ctx, p)
    E, x, rep = sp.davidson(tol=1e-9, noise=torch.tensor(I.guess_noise(sp.dim), device="cuda:0"), max_iter=600)
    assert rep["converged"]
    g1, g2 = sp.rdm(x)
    g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
    N = p.nalpha + p.nbeta
    assert abs(np.trace(g1) - N) <= 1e-10
    assert abs(np.einsum("pprr->", g2) - N * (N - 1)) <= 1e-8
    assert abs(float(np.sum(p.ints.h * g1) + 0.5 * np.sum(p.ints.eri * g2)) - E) <= 1e-8
    assert np.abs(g2 - g2.transpose(2, 3, 0, 1)).max() <= 1e-11
    sp.close()
    _fd_check(ctx, p, 50, 55, 1e-9)


def test_cfg5_rdm_matches_stored_oracle(ctx):
    """1.6e7-determinant workload: the 1- and 2-RDM of a seeded normalised
    vector against the oracle's (definition-based enumeration, stored by
    tests/golden/make_golden.py cfg5_rdm), element by element within 1e-12
    of the largest entry of each."""
    torch = need_gpu()
    import json
    import os
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    meta = json.load(open(os.path.join(golden, "cfg5_oracle_rdm.json")))
    assert meta["vector"] == "random_vector(dim, 55) normalised"
    ref = np.load(os.path.join(golden, "cfg5_oracle_rdm.npz"))
    banner("rdm cfg5 vs stored oracle")
    p = I.cfg5()
    sp = _space(ctx, p)
    c = I.random_vector(sp.dim, 55)
    c /= np.linalg.norm(c)
    g1, g2 = sp.rdm(torch.tensor(c, device="cuda:0"))
    g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
    r1, r2 = ref["rdm1"], ref["rdm2"]
    e1 = np.abs(g1 - r1).max() / np.abs(r1).max()
    e2 = np.abs(g2 - r2).max() / np.abs(r2).max()
    print("cfg5 rdm relative max differences", e1, e2)
    assert e1 <= 1e-12 and e2 <= 1e-12, (e1, e2)
    sp.close()
