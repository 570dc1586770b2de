"""Two-word strings (norb 72 and 96) through the C ABI against the oracle's
two-word path (itself pinned on the CPU to the one-word path by orbital
relabelling): excitation tables bit-exact, sigma per term (FP64 <= 1e-12,
FP32 <= 2e-6), the relabelled problem's sigma equal to the original's,
Davidson against dense eigh (<= 1e-8 Ha), RDMs element by element
(<= 1e-12 of the largest entry), the stored H, and block Davidson.
"""
import functools

import numpy as np
import pytest

from paper_2601_16169_amd import inputs as I
from oracle import core, tables
from tests.gpu_util import banner, need_gpu, rel_err

pytestmark = pytest.mark.gpu

MAP72 = [3, 17, 40, 63, 64, 65, 70, 71]

CASES = {
    "words_72_6_5": lambda: I.words_problem(72, 6, 5, 60, 70, 7),
    "words_96_4_4": lambda: I.words_problem(96, 4, 4, 80, 80, 8),
    "embedded_8_in_72": lambda: I.embed_problem(I.small_problem(8, 3, 4, 37, 53, 3), 72, MAP72, 11),
}


@functools.lru_cache(maxsize=None)
def _problem(name):
    return CASES[name]()


@functools.lru_cache(maxsize=None)
def _oracle(name):
    return core.Space.from_problem(_problem(name))


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


@pytest.mark.parametrize("name", list(CASES))
def test_words_tables_bit_exact(ctx, name):
    banner(f"two-word tables {name}")
    p = _problem(name)
    sp = _space(ctx, p)
    for spin, strs in ((0, p.astr), (1, p.bstr)):
        so, se, do, de = tables.build_tables(strs, p.norb)
        off, ent = sp.tables(spin, 0)
        assert np.array_equal(off, so) and np.array_equal(ent, se), f"singles spin {spin}"
        off, ent = sp.tables(spin, 1)
        assert np.array_equal(off, do) and np.array_equal(ent, de), f"doubles spin {spin}"
    sp.close()


@pytest.mark.parametrize("name", list(CASES))
def test_words_sigma_terms(ctx, name):
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner(f"two-word sigma {name}")
    p = _problem(name)
    sp = _space(ctx, p)
    osp = _oracle(name)
    c = I.random_vector(sp.dim, 2)
    ct = torch.tensor(c, device="cuda:0")
    for mask in (1, 2, 4, 8, 15):
        ref = osp.sigma(c, mask)
        for prec, bar in ((sqd.FP64, 1e-12), (sqd.FP32, 2e-6)):
            got = sp.sigma(ct, precision=prec, terms=mask).cpu().numpy()
            e_inf, e_2 = rel_err(got, ref)
            assert e_inf <= bar and e_2 <= bar, (mask, prec, e_inf, e_2)
    d = sp.diag().cpu().numpy()
    assert np.abs(d - osp.diag()).max() <= 1e-12 * np.abs(d).max()
    sp.close()


def test_embedded_sigma_equals_one_word_sigma(ctx):
    torch = need_gpu()
    banner("two-word embedding: sigma equals the one-word sigma")
    p = I.small_problem(8, 3, 4, 37, 53, 3)
    q = _problem("embedded_8_in_72")
    c = torch.tensor(I.random_vector(p.dim, 6), device="cuda:0")
    sp = _space(ctx, p)
    a = sp.sigma(c).cpu().numpy()
    sp.close()
    sq = _space(ctx, q)
    b = sq.sigma(c).cpu().numpy()
    e_inf, e_2 = rel_err(b, a)
    assert e_inf <= 1e-12 and e_2 <= 1e-12
    sq.close()


@pytest.mark.parametrize("name", ["words_72_6_5", "embedded_8_in_72"])
def test_words_davidson_and_block(ctx, name):
    torch = need_gpu()
    banner(f"two-word Davidson {name}")
    p = _problem(name)
    sp = _space(ctx, p)
    w, v = np.linalg.eigh(_oracle(name).dense())
    E, x, rep = sp.davidson(tol=1e-10, noise=torch.tensor(I.guess_noise(sp.dim), device="cuda:0"))
    assert rep["converged"] and abs(E - w[0]) <= 1e-8
    assert 1 - abs(x.cpu().numpy() @ v[:, 0]) <= 1e-10
    Eb, X, reps = sp.davidson_block(3, tol=1e-9, max_iter=400)
    assert all(r["converged"] for r in reps)
    assert np.abs(np.asarray(Eb) - w[:3]).max() <= 1e-8
    sp.close()


@pytest.mark.parametrize("name", ["words_72_6_5", "embedded_8_in_72"])
def test_words_rdms(ctx, name):
    torch = need_gpu()
    banner(f"two-word RDMs {name}")
    p = _problem(name)
    sp = _space(ctx, p)
    c = I.random_vector(sp.dim, 3)
    c /= np.linalg.norm(c)
    g1, g2 = sp.rdm(torch.tensor(c, device="cuda:0"))
    r1, r2 = _oracle(name).rdm(c)
    assert np.abs(g1.cpu().numpy() - r1).max() <= 1e-12 * np.abs(r1).max()
    assert np.abs(g2.cpu().numpy() - r2).max() <= 1e-12 * np.abs(r2).max()
    sp.close()


def test_words_stored_h(ctx):
    torch = need_gpu()
    banner("two-word stored H")
    p = _problem("words_72_6_5")
    sp = _space(ctx, p)
    nnz = sp.store_hamiltonian()
    rp, cols, vals = sp.stored_hamiltonian(nnz)
    ref = core.MemoisedH(_oracle("words_72_6_5"))
    assert np.array_equal(rp, ref.rowptr)
    c = I.random_vector(sp.dim, 8)
    got = sp.spmv(torch.tensor(c, device="cuda:0")).cpu().numpy()
    e_inf, e_2 = rel_err(got, _oracle("words_72_6_5").sigma(c))
    assert e_inf <= 1e-12 and e_2 <= 1e-12
    sp.close()


def test_words_error_codes(ctx):
    need_gpu()
    from paper_2601_16169_amd import sqd
    p = _problem("words_72_6_5")
    ctx.set_hamiltonian(p.ints.h, p.ints.eri)
    lo = np.ascontiguousarray(p.astr[:, 0])
    with pytest.raises(sqd.SQDError) as e:          # one-word strings at norb 72
        ctx.build_space(p.nalpha, p.nbeta, lo, lo)
    assert e.value.code == -4
    bad = p.astr.copy()
    bad[-1, 1] |= np.uint64(1 << 20)                # orbital 84 >= norb 72
    with pytest.raises(sqd.SQDError) as e:
        ctx.build_space(p.nalpha, p.nbeta, bad, p.bstr)
    assert e.value.code == -4
    with pytest.raises(sqd.SQDError) as e:          # descending in the high word
        ctx.build_space(p.nalpha, p.nbeta, p.astr[::-1].copy(), p.bstr)
    assert e.value.code == -2
