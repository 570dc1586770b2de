"""sqd_sigma_noalloc (the product with no device allocation, scratch in the
library's static array) against sqd_sigma, through the C ABI.

Two calls in a row, the second on a smaller space, each compared with the
allocating entry point on the same input: FP64 max-norm and 2-norm relative
difference <= 1e-12 (the sigma bar; the two entry points run different
alpha-beta kernels, so the summation order differs), FP32 <= 2e-6.  The smaller
space is also checked against the oracle.  Sizes above the documented maximum
are rejected with SQD_E_LIMIT before anything is enqueued.  A fresh space
needs no allocating product first; one whose beta rows take the windowed
same-spin kernel (12,000 strings) answers SQD_E_STATE until an allocating
product has built its windowed tables, and is then compared the same way.
"""
import numpy as np
import pytest

from paper_2601_16169_amd import inputs as I
from oracle import core
from tests.gpu_util import banner, need_gpu, rel_err

pytestmark = pytest.mark.gpu

MAX_DIM = 16777152   # SQD_NOALLOC_MAX_DIM


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


def _compare(sp, c, precision, terms, bar):
    torch = need_gpu()
    ref = sp.sigma(c, precision=precision, terms=terms)
    out = torch.full_like(c, float("nan"))
    sp.sigma_noalloc(c, out, precision=precision, terms=terms)
    torch.cuda.synchronize()
    e_inf, e_2 = rel_err(out.cpu().numpy(), ref.cpu().numpy())
    assert e_inf <= bar and e_2 <= bar, (precision, terms, e_inf, e_2)
    return out


def test_noalloc_matches_sigma_two_calls(ctx):
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner("sigma_noalloc: 4.0e6-determinant space, then a ragged 70 x 97 space")
    p = I.cfg2()
    sp = _space(ctx, p)
    c = torch.tensor(I.random_vector(sp.dim, 11), device="cuda:0")
    for prec, bar in ((sqd.FP64, 1e-12), (sqd.FP32, 2e-6)):
        _compare(sp, c, prec, sqd.TERM_ALL, bar)
    sp.close()
    # second call: a smaller space (fewer determinants than the first call's
    # scratch holds), unequal spin sets, each term alone and all together
    q = I.small_problem(10, 4, 3, 70, 97, 4)
    sq = _space(ctx, q)
    c2 = torch.tensor(I.random_vector(sq.dim, 12), device="cuda:0")
    for prec, bar in ((sqd.FP64, 1e-12), (sqd.FP32, 2e-6)):
        for terms in (sqd.TERM_AA, sqd.TERM_BB, sqd.TERM_AB, sqd.TERM_DIAG, sqd.TERM_ALL):
            _compare(sq, c2, prec, terms, bar)
    out = torch.empty_like(c2)
    sq.sigma_noalloc(c2, out)
    ref = core.Space.from_problem(q).sigma(c2.cpu().numpy())
    e_inf, e_2 = rel_err(out.cpu().numpy(), ref)
    assert e_inf <= 1e-12 and e_2 <= 1e-12, (e_inf, e_2)
    sq.close()


def test_noalloc_rejects_sizes_beyond_the_limit(ctx):
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner("sigma_noalloc: dimension above the limit")
    n = 4097                                    # 4097^2 > MAX_DIM
    strs = np.sort(I.random_subset(I.all_strings(16, 8), n, 21))
    ints = I.make_integrals(16, 8, 31)
    ctx.set_hamiltonian(ints.h, ints.eri, ints.ecore)
    sp = ctx.build_space(8, 8, strs, strs)
    assert sp.dim > MAX_DIM
    c = torch.zeros(sp.dim, dtype=torch.float64, device="cuda:0")
    out = torch.zeros_like(c)
    with pytest.raises(sqd.SQDError) as ei:
        sp.sigma_noalloc(c, out)
    assert ei.value.code == -9
    sp.close()


def test_noalloc_fresh_space_and_windowed_rows(ctx):
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner("sigma_noalloc: fresh space, then a space with windowed beta rows")
    # a space straight from build_space (diagonal built there) needs no
    # allocating product first
    q = I.small_problem(10, 4, 3, 70, 97, 4)
    sq = _space(ctx, q)
    c = torch.tensor(I.random_vector(sq.dim, 13), device="cuda:0")
    out = torch.full_like(c, float("nan"))
    sq.sigma_noalloc(c, out)
    torch.cuda.synchronize()
    e_inf, e_2 = rel_err(out.cpu().numpy(), core.Space.from_problem(q).sigma(c.cpu().numpy()))
    assert e_inf <= 1e-12 and e_2 <= 1e-12, (e_inf, e_2)
    sq.close()
    # 40 alpha strings x 12,000 beta strings of norb 16: two staged FP64 beta
    # rows exceed one workgroup's LDS, so the beta-beta term is windowed, and
    # its tables come with the first allocating product
    allb = I.all_strings(16, 8)
    bstr = np.sort(I.random_subset(allb, 12000, 41))
    astr = np.sort(I.random_subset(allb, 40, 42))
    ints = I.make_integrals(16, 8, 43)
    ctx.set_hamiltonian(ints.h, ints.eri, ints.ecore)
    sw = ctx.build_space(8, 8, astr, bstr)
    c = torch.tensor(I.random_vector(sw.dim, 14), device="cuda:0")
    out = torch.empty_like(c)
    with pytest.raises(sqd.SQDError) as ei:
        sw.sigma_noalloc(c, out, terms=sqd.TERM_BB)
    assert ei.value.code == -8
    for prec, bar in ((sqd.FP64, 1e-12), (sqd.FP32, 2e-6)):
        _compare(sw, c, prec, sqd.TERM_ALL, bar)
    sw.close()
