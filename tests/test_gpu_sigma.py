"""GPU parity of the excitation tables (bit-exact) and of sigma (per term and
in total) against the CPU oracle, through the C ABI.

Tolerance (FP64): max-norm and 2-norm relative error <= 1e-12, the bar set
for sigma; the oracle sums in a different order, so results are not
bit-identical.  FP32 sigma: <= 2e-6 relative (single-precision storage and
accumulation over a few hundred terms per row).
"""
import json
import numpy as np
import pytest

from paper_2601_16169_amd import inputs as I
from oracle import core, tables
from tests.gpu_util import banner, need_gpu, rel_err

pytestmark = pytest.mark.gpu

TERMS = {"DIAG": 1, "AA": 2, "BB": 4, "AB": 8, "ALL": 15}


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


SMALL = [
    ("complete_4_2_2", lambda: I.small_problem(4, 2, 2, 6, 6, 1)),
    ("ragged_6_3_2", lambda: I.small_problem(6, 3, 2, 13, 11, 2)),
    ("ragged_8_3_4", lambda: I.small_problem(8, 3, 4, 37, 53, 3)),
    ("sab_neq_10_4_3", lambda: I.small_problem(10, 4, 3, 70, 97, 4)),
    ("one_alpha_string", lambda: I.small_problem(6, 2, 3, 1, 20, 5)),
    ("one_beta_string", lambda: I.small_problem(6, 2, 3, 15, 1, 6)),
    ("zero_alpha_electrons", lambda: I.small_problem(5, 0, 2, 1, 10, 7)),
    ("full_alpha_shell", lambda: I.small_problem(5, 5, 2, 1, 10, 10)),
    ("cfg1", I.cfg1),
]


@pytest.mark.parametrize("name,make", SMALL)
def test_tables_bit_exact(ctx, name, make):
    banner(f"tables {name}")
    p = make()
    sp = _space(ctx, p)
    for spin, strs in ((0, p.astr), (1, p.bstr)):
        so, se, do, de = tables.build_tables(strs, p.norb)
        off, ent = sp.tables(spin, 0)
        assert np.array_equal(off, so) and np.array_equal(ent, se), f"singles spin {spin}"
        off, ent = sp.tables(spin, 1)
        assert np.array_equal(off, do) and np.array_equal(ent, de), f"doubles spin {spin}"
    sp.close()


def test_tables_bit_exact_cfg2(ctx):
    banner("tables cfg2")
    p = I.cfg2()
    sp = _space(ctx, p)
    so, se, do, de = tables.build_tables(p.astr, p.norb)
    for spin in (0, 1):
        off, ent = sp.tables(spin, 0)
        assert np.array_equal(off, so) and np.array_equal(ent, se)
        off, ent = sp.tables(spin, 1)
        assert np.array_equal(off, do) and np.array_equal(ent, de)
    info = sp.info()
    assert info["nnz_single"][0] == len(se) and info["nnz_double"][1] == len(de)
    sp.close()


@pytest.mark.parametrize("name,make", SMALL)
def test_diag_parity(ctx, name, make):
    torch = need_gpu()
    p = make()
    sp = _space(ctx, p)
    d = sp.diag().cpu().numpy()
    o = core.Space.from_problem(p).diag()
    assert rel_err(d, o)[0] <= 1e-13
    sp.close()


@pytest.mark.parametrize("name,make", SMALL)
@pytest.mark.parametrize("term", ["DIAG", "AA", "BB", "AB", "ALL"])
def test_sigma_terms_fp64(ctx, name, make, term):
    torch = need_gpu()
    banner(f"sigma fp64 {name} {term}")
    p = make()
    sp = _space(ctx, p)
    c = I.random_vector(sp.dim, 11)
    o = core.Space.from_problem(p).sigma(c, TERMS[term])
    ct = torch.tensor(c, device="cuda:0")
    s = sp.sigma(ct, terms=TERMS[term]).cpu().numpy()
    if np.abs(o).max() == 0.0:
        assert np.abs(s).max() == 0.0
    else:
        e_inf, e_2 = rel_err(s, o)
        assert e_inf <= 1e-12 and e_2 <= 1e-12, (e_inf, e_2)
    sp.close()


@pytest.mark.parametrize("name,make", SMALL[2:4] + SMALL[-1:])
@pytest.mark.parametrize("term", ["AA", "BB", "AB", "ALL"])
def test_sigma_terms_fp32(ctx, name, make, term):
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    p = make()
    sp = _space(ctx, p)
    c = I.random_vector(sp.dim, 12)
    o = core.Space.from_problem(p).sigma(c, TERMS[term])
    s = sp.sigma(torch.tensor(c, device="cuda:0"), precision=sqd.FP32, terms=TERMS[term]).cpu().numpy()
    e_inf, e_2 = rel_err(s, o)
    assert e_inf <= 2e-6 and e_2 <= 2e-6, (e_inf, e_2)
    sp.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("ab_variant", [0, 3])
def test_sigma_graph_capture_replays(precision, ab_variant):
    """sqd_sigma captured in a HIP graph (after a warm-up call has set up the
    tables and scratch) replays to the eager result, every replay, with eager
    library work and synchronisations between the replays; with the automatic
    alpha-beta kernel and with the source-grouped one."""
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner(f"sigma graph capture precision {precision} ab variant {ab_variant}")
    stream = torch.cuda.Stream()
    gctx = sqd.Context(0, stream)
    gctx.set_tuning(sqd.TUNE_AB_VARIANT, ab_variant)
    try:
        p = I.small_problem(10, 4, 3, 70, 97, 4)
        big_a = I.small_problem(10, 4, 3, 210, 120, 4).astr
        big_b = I.small_problem(10, 4, 3, 210, 120, 4).bstr
        sp = _space(gctx, p)
        with torch.cuda.stream(stream):
            c = torch.tensor(I.random_vector(sp.dim, 23), device="cuda:0")
            c2 = torch.tensor(I.random_vector(sp.dim, 24), device="cuda:0")
            out = torch.empty_like(c)
            other = torch.empty_like(c)
            eager = sp.sigma(c, precision=precision).clone()
            sp.sigma(c, out, precision=precision)    # warm-up of this exact call
        stream.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            sp.sigma(c, out, precision=precision)
        for rep in range(4):
            out.fill_(float("nan"))
            graph.replay()
            stream.synchronize()
            assert torch.equal(out, eager), f"replay {rep} differs"
            with torch.cuda.stream(stream):
                sp.sigma(c2, other, precision=precision)   # eager work between replays
                # eager calls that need a larger scratch than the captured one
                # (FP64 after an FP32 capture, the RDM, a larger space): the
                # buffer the graph uses must stay alive
                sp.sigma(c2, other, precision=0)
                sp.rdm(c2 / torch.linalg.norm(c2))
                if rep == 1:
                    big = gctx.build_space(p.nalpha, p.nbeta, big_a, big_b)
                    big.sigma(torch.ones(big.dim, dtype=torch.float64, device="cuda:0"))
                    big.close()
            stream.synchronize()
        o = core.Space.from_problem(p).sigma(I.random_vector(sp.dim, 23))
        assert max(rel_err(eager.cpu().numpy(), o)) <= (1e-12 if precision == 0 else 2e-6)
        sp.close()
    finally:
        gctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_sigma_graph_capture_windowed(precision):
    """The windowed same-spin kernel (forced, 64-string windows: 2 windows
    of beta sources, 4 of alpha sources) with its slot-order scratch and the
    placing passes (row-major with the diagonal, column-major adding into
    sigma) captured in a HIP graph: every replay equals the eager product,
    with eager products of another vector between the replays, and the eager
    product matches the oracle."""
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner(f"sigma graph capture windowed precision {precision}")
    stream = torch.cuda.Stream()
    gctx = sqd.Context(0, stream)
    gctx.set_tuning(sqd.TUNE_SS_WINDOW, 64)
    try:
        p = I.small_problem(10, 4, 3, 210, 120, 4)
        sp = _space(gctx, p)
        with torch.cuda.stream(stream):
            c = torch.tensor(I.random_vector(sp.dim, 25), device="cuda:0")
            c2 = torch.tensor(I.random_vector(sp.dim, 26), device="cuda:0")
            out = torch.empty_like(c)
            other = torch.empty_like(c)
            eager = sp.sigma(c, precision=precision).clone()
            sp.sigma(c, out, precision=precision)
        stream.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            sp.sigma(c, out, precision=precision)
        for rep in range(4):
            out.fill_(float("nan"))
            graph.replay()
            stream.synchronize()
            assert torch.equal(out, eager), f"replay {rep} differs"
            with torch.cuda.stream(stream):
                sp.sigma(c2, other, precision=precision)
                sp.sigma(c2, other, precision=0)
            stream.synchronize()
        o = core.Space.from_problem(p).sigma(I.random_vector(sp.dim, 25))
        assert max(rel_err(eager.cpu().numpy(), o)) <= (1e-12 if precision == 0 else 2e-6)
        sp.close()
    finally:
        gctx.close()


def test_sigma_capture_without_warmup_is_refused():
    """Under stream capture sqd_sigma allocates nothing: on a space whose
    product has never run eagerly it returns SQD_E_STATE."""
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner("sigma capture without warm-up")
    stream = torch.cuda.Stream()
    gctx = sqd.Context(0, stream)
    try:
        p = I.small_problem(8, 3, 4, 37, 53, 3)
        sp = _space(gctx, p)
        with torch.cuda.stream(stream):
            c = torch.tensor(I.random_vector(sp.dim, 1), device="cuda:0")
            out = torch.empty_like(c)
        stream.synchronize()
        graph = torch.cuda.CUDAGraph()
        code = None
        try:
            with torch.cuda.graph(graph, stream=stream):
                try:
                    sp.sigma(c, out)
                except sqd.SQDError as e:
                    code = e.code
        except RuntimeError:
            pass   # an empty capture may be rejected by torch itself
        assert code == -8
        stream.synchronize()
        with torch.cuda.stream(stream):
            sp.sigma(c, out)           # eager afterwards: works
        stream.synchronize()
        o = core.Space.from_problem(p).sigma(I.random_vector(sp.dim, 1))
        assert max(rel_err(out.cpu().numpy(), o)) <= 1e-12
        sp.close()
    finally:
        gctx.close()


def test_space_outlives_context_abi():
    """Through the raw C ABI: a space still open when its context is
    destroyed becomes an orphan; its info call fails with SQD_E_STATE and
    sqd_space_free on it only frees the host record (no crash)."""
    torch = need_gpu()
    import ctypes
    from paper_2601_16169_amd import sqd
    banner("space outlives context")
    L = sqd.lib()
    p = I.small_problem(6, 3, 2, 13, 11, 2)
    h = ctypes.c_void_p()
    assert L.sqd_create(0, ctypes.c_void_p(torch.cuda.current_stream(0).cuda_stream), ctypes.byref(h)) == 0
    hh = np.ascontiguousarray(p.ints.h)
    ee = np.ascontiguousarray(p.ints.eri)
    assert L.sqd_set_hamiltonian(h, p.norb, hh.ctypes.data_as(ctypes.c_void_p), ee.ctypes.data_as(ctypes.c_void_p),
                                 0.0) == 0
    a = np.ascontiguousarray(p.astr)
    b = np.ascontiguousarray(p.bstr)
    spaces = []
    for _ in range(2):
        s_ = ctypes.c_void_p()
        assert L.sqd_build_space(h, p.nalpha, p.nbeta, a.ctypes.data_as(ctypes.c_void_p), len(a),
                                 b.ctypes.data_as(ctypes.c_void_p), len(b), ctypes.byref(s_)) == 0
        spaces.append(s_)
    L.sqd_space_free(spaces[0])        # freed while the context lives
    L.sqd_destroy(h)                   # spaces[1] is still open
    info = sqd.SpaceInfo()
    assert L.sqd_space_info(spaces[1], ctypes.byref(info)) == -8
    L.sqd_space_free(spaces[1])        # orphan: host record only
    L.sqd_space_free(None)


def test_rdm_rejects_space_of_other_norb(ctx):
    """A space built for norb 8 fails every call once the integrals are
    replaced by norb-6 ones, the RDM call included (it would otherwise index
    the new integrals and outputs with the old norb)."""
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner("rdm norb guard")
    p = I.small_problem(8, 3, 4, 37, 53, 3)
    sp = _space(ctx, p)
    c = torch.tensor(I.random_vector(sp.dim, 1), device="cuda:0")
    c /= torch.linalg.norm(c)
    q = I.small_problem(6, 3, 2, 13, 11, 2)
    ctx.set_hamiltonian(q.ints.h, q.ints.eri)
    g1 = torch.empty((8, 8), dtype=torch.float64, device="cuda:0")
    g2 = torch.empty((8, 8, 8, 8), dtype=torch.float64, device="cuda:0")
    import ctypes
    rc = sqd.lib().sqd_rdm(ctx._h, sp._h, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(g1.data_ptr()),
                           ctypes.c_void_p(g2.data_ptr()))
    assert rc == -8
    for fn in (lambda: sp.sigma(c), lambda: sp.diag(), lambda: sp.davidson(max_iter=2)):
        with pytest.raises(sqd.SQDError) as e:
            fn()
        assert e.value.code == -8
    sp.close()


def test_sigma_norb64_edge(ctx):
    """norb = 64: orbital indices up to 63 and the full 64-bit string."""
    torch = need_gpu()
    banner("sigma norb64")
    ints = I.make_integrals(64, 3, seed=40)
    rng = np.random.default_rng(41)
    def strings(n, count):
        out = set()
        while len(out) < count:
            occ = rng.choice(64, n, replace=False)
            if rng.random() < 0.5:
                occ[0] = 63
                occ = np.unique(occ)
                if len(occ) < n:
                    continue
            out.add(int(sum(1 << int(o) for o in occ)))
        return np.array(sorted(out), dtype=np.uint64)
    a, b = strings(2, 40), strings(1, 64)
    p = I.Problem("norb64", ints, 2, 1, a, b)
    sp = _space(ctx, p)
    so, se, do, de = tables.build_tables(a, 64)
    off, ent = sp.tables(0, 0)
    assert np.array_equal(off, so) and np.array_equal(ent, se)
    c = I.random_vector(sp.dim, 13)
    o = core.Space.from_problem(p).sigma(c)
    s = sp.sigma(torch.tensor(c, device="cuda:0")).cpu().numpy()
    assert max(rel_err(s, o)) <= 1e-12
    sp.close()


def _sampled_rows(dim, k, seed):
    rng = np.random.default_rng(seed)
    rows = rng.choice(dim, size=min(k, dim), replace=False)
    return np.unique(np.concatenate([rows, [0, dim - 1]]))


@pytest.mark.parametrize("precision", [0, 1])
def test_sigma_cfg2_sampled_rows(ctx, precision):
    """Full-size 4.0e6-determinant workload, in the launch shape the benchmark
    times; the oracle evaluates sampled rows one by one."""
    torch = need_gpu()
    banner(f"sigma cfg2 sampled precision={precision}")
    p = I.cfg2()
    sp = _space(ctx, p)
    c = I.random_vector(sp.dim, 21)
    s = sp.sigma(torch.tensor(c, device="cuda:0"), precision=precision).cpu().numpy()
    rows = _sampled_rows(sp.dim, 4096, 5)
    o = core.Space.from_problem(p).sigma_rows(c, rows)
    tol = 1e-12 if precision == 0 else 2e-6
    err = np.abs(s[rows] - o) / np.abs(o).max()
    assert err.max() <= tol, err.max()
    sp.close()


def test_sigma_cfg2_hermitian_and_linear(ctx):
    torch = need_gpu()
    p = I.cfg2()
    sp = _space(ctx, p)
    x = torch.tensor(I.random_vector(sp.dim, 1), device="cuda:0")
    y = torch.tensor(I.random_vector(sp.dim, 2), device="cuda:0")
    sx, sy = sp.sigma(x), sp.sigma(y)
    lhs, rhs = float(torch.dot(x, sy)), float(torch.dot(y, sx))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    sxy = sp.sigma(x + 2.0 * y)
    assert float((sxy - sx - 2.0 * sy).abs().max()) <= 1e-11 * float(sxy.abs().max())
    sp.close()


def test_error_codes(ctx):
    need_gpu()
    from paper_2601_16169_amd import sqd
    p = I.small_problem(6, 3, 2, 10, 10, 9)
    ctx.set_hamiltonian(p.ints.h, p.ints.eri)
    with pytest.raises(sqd.SQDError) as e:
        ctx.build_space(3, 2, p.astr[::-1].copy(), p.bstr)
    assert e.value.code == -2
    with pytest.raises(sqd.SQDError) as e:
        ctx.build_space(2, 2, p.astr, p.bstr)
    assert e.value.code == -3
    bad = p.astr.copy()
    bad[-1] = np.uint64(int(bad[-1]) | (1 << 7))
    with pytest.raises(sqd.SQDError):
        ctx.build_space(3, 2, bad, p.bstr)
    h = p.ints.h.copy()
    h[0, 1] += 1e-3
    with pytest.raises(sqd.SQDError) as e:
        ctx.set_hamiltonian(h, p.ints.eri)
    assert e.value.code == -5
    eri = p.ints.eri.copy()
    eri[0, 1, 2, 3] += 1e-3
    with pytest.raises(sqd.SQDError) as e:
        ctx.set_hamiltonian(p.ints.h, eri)
    assert e.value.code == -5
    ctx.set_hamiltonian(p.ints.h, p.ints.eri)
    # empty string list, electron count above norb
    with pytest.raises(sqd.SQDError) as e:
        ctx.build_space(3, 2, np.zeros(0, dtype=np.uint64), p.bstr)
    assert e.value.code == -1
    with pytest.raises(sqd.SQDError) as e:
        ctx.build_space(7, 2, p.astr, p.bstr)
    assert e.value.code == -3
    # tuning values outside the allowed sets
    with pytest.raises(sqd.SQDError) as e:
        ctx.set_tuning(sqd.TUNE_SS_ROWS, 3)
    assert e.value.code == -1
    with pytest.raises(sqd.SQDError) as e:
        ctx.set_tuning(99, 1)
    assert e.value.code == -1
    # the space still works after the rejected calls
    sp = ctx.build_space(3, 2, p.astr, p.bstr)
    with pytest.raises(sqd.SQDError) as e:
        sp.davidson_roots(9)           # more than SQD_MAXLOCK roots
    assert e.value.code == -1
    sp.close()
    q = I.small_problem(3, 1, 1, 2, 2, 11)
    ctx.set_hamiltonian(q.ints.h, q.ints.eri)
    sq = ctx.build_space(1, 1, q.astr, q.bstr)
    assert sq.dim == 4
    with pytest.raises(sqd.SQDError) as e:
        sq.davidson_roots(5)           # more roots than determinants
    assert e.value.code == -1
    sq.close()


# ragged tiles (53 and 97 beta strings), one alpha string, a beta side with no
# singles (every tile has an empty pair union), no alpha electrons, full CI
KH_CASES = [c for c in SMALL if c[0] in ("ragged_8_3_4", "sab_neq_10_4_3", "one_alpha_string", "one_beta_string",
                                         "zero_alpha_electrons", "cfg1")]
# 8008-string beta rows: in FP64 the source row no longer fits beside the
# tiles at two workgroups per CU, so the kernel reads it from global memory
KH_CASES.append(("kh_long_rows_16_3_6", lambda: I.small_problem(16, 3, 6, 24, 8008, 12)))


@pytest.mark.parametrize("name,make", KH_CASES)
@pytest.mark.parametrize("precision", [0, 1])
def test_sigma_ab_knowles_handy(ctx, name, make, precision):
    """The MFMA Knowles-Handy alpha-beta path against the oracle."""
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner(f"sigma KH {name} p={precision}")
    p = make()
    sp = _space(ctx, p)
    c = I.random_vector(sp.dim, 14)
    o = core.Space.from_problem(p).sigma(c, TERMS["AB"])
    s = sp.sigma(torch.tensor(c, device="cuda:0"), precision=precision, terms=TERMS["AB"],
                 ab_path=sqd.AB_KH).cpu().numpy()
    if np.abs(o).max() == 0.0:
        assert np.abs(s).max() == 0.0
    else:
        tol = 1e-12 if precision == 0 else 2e-6
        assert max(rel_err(s, o)) <= tol
    sp.close()


@pytest.mark.parametrize("name,make", SMALL + [("src_long_rows_16_3_6", lambda: I.small_problem(16, 3, 6, 24, 8008, 12))])
def test_sigma_ab_source_grouped(ctx, name, make):
    """The alpha-beta kernel grouped by source string (SQD_TUNE_AB_VARIANT 3)
    against the oracle, FP64 <= 1e-12 and FP32 <= 2e-6, and bit for bit
    against the pair-grouped kernel (same products, same summation order),
    on ragged and degenerate spaces and on 8008-string beta rows."""
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner(f"sigma ab source-grouped {name}")
    p = make()
    sp = _space(ctx, p)
    c = I.random_vector(sp.dim, 25)
    ct = torch.tensor(c, device="cuda:0")
    o = core.Space.from_problem(p).sigma(c, TERMS["AB"])
    for prec, tol in ((0, 1e-12), (1, 2e-6)):
        try:
            ctx.set_tuning(sqd.TUNE_AB_VARIANT, 3)
            s3 = sp.sigma(ct, precision=prec, terms=TERMS["AB"]).cpu().numpy()
            ctx.set_tuning(sqd.TUNE_AB_VARIANT, 1)
            s1 = sp.sigma(ct, precision=prec, terms=TERMS["AB"]).cpu().numpy()
        finally:
            ctx.set_tuning(sqd.TUNE_AB_VARIANT, 0)
        assert np.array_equal(s3, s1), (prec, np.abs(s3 - s1).max())
        if np.abs(o).max() == 0.0:
            assert np.abs(s3).max() == 0.0
        else:
            assert max(rel_err(s3, o)) <= tol, (prec, rel_err(s3, o))
    sp.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_sigma_full14_sampled_rows(ctx, precision):
    """The full-CI 14-orbital space (3432 strings per spin, dim 1.18e7),
    where the automatic alpha-beta path groups the singles by source string
    (pair groups would hold two source rows): 320 sampled rows of the whole
    product and of the alpha-beta term against the oracle."""
    torch = need_gpu()
    banner(f"sigma full14 sampled precision={precision}")
    p = I.full14()
    sp = _space(ctx, p)
    c = I.random_vector(sp.dim, 26)
    ct = torch.tensor(c, device="cuda:0")
    rows = _sampled_rows(sp.dim, 320, 9)
    osp = core.Space.from_problem(p)
    tol = 1e-12 if precision == 0 else 2e-6
    for mask in (TERMS["ALL"], TERMS["AB"]):
        got = sp.sigma(ct, precision=precision, terms=mask)[torch.tensor(rows, device="cuda:0")].cpu().numpy()
        o = osp.sigma_rows(c, rows, mask)
        err = np.abs(got - o).max() / np.abs(o).max()
        assert err <= tol, (mask, err)
    sp.close()


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_sigma_ab_variants_cfg2(ctx, variant):
    """The direct alpha-beta kernels (grouped by pair, row-staged, grouped by
    source) and KH agree on the 4.0e6-determinant workload (sampled rows
    against the oracle)."""
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    p = I.cfg2()
    sp = _space(ctx, p)
    c = I.random_vector(sp.dim, 22)
    ct = torch.tensor(c, device="cuda:0")
    ctx.set_tuning(sqd.TUNE_AB_VARIANT, variant)
    try:
        s = sp.sigma(ct, terms=TERMS["AB"]).cpu().numpy()
    finally:
        ctx.set_tuning(sqd.TUNE_AB_VARIANT, 0)
    k = sp.sigma(ct, terms=TERMS["AB"], ab_path=sqd.AB_KH).cpu().numpy()
    rows = _sampled_rows(sp.dim, 2048, 6)
    o = core.Space.from_problem(p).sigma_rows(c, rows, TERMS["AB"])
    scale = np.abs(o).max()
    assert np.abs(s[rows] - o).max() <= 1e-12 * scale
    assert np.abs(k[rows] - o).max() <= 1e-12 * scale
    assert np.abs(s - k).max() <= 1e-12 * np.abs(k).max()
    sp.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_sigma_long_beta_rows(ctx, precision):
    """Rows of 16500 beta strings: in FP64 a row (132,000 bytes) is longer
    than the gather assembles in LDS, so the alpha-beta sums are added into
    sigma in place, and the beta-beta term takes the windowed kernel in both
    precisions (fewer than four rows fit); sampled rows against the oracle,
    all terms and the alpha-beta term alone."""
    torch = need_gpu()
    banner(f"sigma long beta rows precision={precision}")
    p = I.small_problem(18, 3, 9, 6, 16500, 31)
    sp = _space(ctx, p)
    assert sp.nb == 16500 and sp.nb * 8 > 128 * 1024
    c = I.random_vector(sp.dim, 24)
    ct = torch.tensor(c, device="cuda:0")
    rows = _sampled_rows(sp.dim, 384, 8)
    osp = core.Space.from_problem(p)
    tol = 1e-12 if precision == 0 else 2e-6
    for mask in (TERMS["ALL"], TERMS["AB"]):
        got = sp.sigma(ct, precision=precision, terms=mask).cpu().numpy()[rows]
        o = osp.sigma_rows(c, rows, mask)
        err = np.abs(got - o).max() / np.abs(o).max()
        assert err <= tol, (mask, err)
    sp.close()


@pytest.mark.slow
@pytest.mark.parametrize("precision", [0, 1])
def test_sigma_cfg3_sampled_rows(ctx, precision):
    """The 2.56e8-determinant single-GPU share (norb 36, 12+12 electrons,
    16000 strings per spin) in the launch shape of a full product; the oracle
    evaluates 512 sampled rows (plus the first and last) one by one."""
    torch = need_gpu()
    banner(f"sigma cfg3 sampled precision={precision}")
    p = I.cfg3()
    sp = _space(ctx, p)
    c = I.random_vector(sp.dim, 23)
    ct = torch.tensor(c, device="cuda:0")
    s = sp.sigma(ct, precision=precision)
    rows = _sampled_rows(sp.dim, 512, 6)
    got = s[torch.tensor(rows, device="cuda:0")].cpu().numpy()
    del s, ct
    o = core.Space.from_problem(p).sigma_rows(c, rows)
    tol = 1e-12 if precision == 0 else 2e-6
    err = np.abs(got - o) / np.abs(o).max()
    assert err.max() <= tol, err.max()
    sp.close()


def test_autotune_keeps_results(ctx, tmp_path, monkeypatch):
    """The autotuner's search leaves a setting applied that still reproduces
    the oracle's sigma, caches it, and re-applies it from the cache."""
    torch = need_gpu()
    from paper_2601_16169_amd import autotune, sqd
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    p = SMALL[3][1]()
    sp = _space(ctx, p)
    r = autotune.tune(sp, precision=sqd.FP64, reps=2)
    assert set(r) == {"ss", "ab"}
    c = I.random_vector(sp.dim, 31)
    ref = core.Space.from_problem(p).sigma(c)
    got = sp.sigma(torch.tensor(c, device="cuda:0")).cpu().numpy()
    assert max(rel_err(got, ref)) <= 1e-12
    autotune.reset(ctx)
    assert autotune.tune(sp, precision=sqd.FP64) == json.loads(json.dumps(r))
    autotune.reset(ctx)
    sp.close()


@pytest.mark.parametrize("name,make,width", [
    ("sab_neq_10_4_3", lambda: I.small_problem(10, 4, 3, 70, 97, 4), 64),      # 2 windows each way, ragged
    ("ragged_8_3_4", lambda: I.small_problem(8, 3, 4, 37, 53, 3), 64),         # one short window
    ("one_beta_string", lambda: I.small_problem(6, 2, 3, 15, 1, 6), 64),       # fewer rows than staged
])
def test_sigma_windowed_same_spin(ctx, name, make, width):
    """The same-spin term by windows of source strings (the path taken for
    rows too long to stage whole), forced on small spaces with a narrow
    window, against the oracle per term: FP64 <= 1e-12, FP32 <= 2e-6."""
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner(f"windowed same-spin {name} width {width}")
    p = make()
    sp = _space(ctx, p)
    osp = core.Space.from_problem(p)
    c = I.random_vector(sp.dim, 17)
    ct = torch.tensor(c, device="cuda:0")
    ctx.set_tuning(sqd.TUNE_SS_WINDOW, width)
    try:
        for mask in (TERMS["AA"], TERMS["BB"], TERMS["BB"] | TERMS["DIAG"], TERMS["AA"] | TERMS["DIAG"],
                     TERMS["ALL"]):
            ref = osp.sigma(c, mask)
            for prec, bar in ((sqd.FP64, 1e-12), (sqd.FP32, 2e-6)):
                got = sp.sigma(ct, precision=prec, terms=mask).cpu().numpy()
                e_inf, e_2 = rel_err(got, ref)
                assert e_inf <= bar and e_2 <= bar, (mask, prec, e_inf, e_2)
    finally:
        ctx.set_tuning(sqd.TUNE_SS_WINDOW, 0)
    sp.close()


def test_sigma_windowed_cfg2_matches_row_staged(ctx):
    """4.0e6 determinants: windows of 256 source strings (8 windows per row)
    against the row-staged kernels, FP64 and FP32, all terms."""
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner("windowed same-spin cfg2, width 256")
    p = I.cfg2()
    sp = _space(ctx, p)
    c = torch.tensor(I.random_vector(sp.dim, 23), device="cuda:0")
    for prec, bar in ((sqd.FP64, 1e-12), (sqd.FP32, 2e-6)):
        ref = sp.sigma(c, precision=prec).cpu().numpy()
        ctx.set_tuning(sqd.TUNE_SS_WINDOW, 256)
        try:
            got = sp.sigma(c, precision=prec).cpu().numpy()
        finally:
            ctx.set_tuning(sqd.TUNE_SS_WINDOW, 0)
        e_inf, e_2 = rel_err(got, ref)
        assert e_inf <= bar and e_2 <= bar, (prec, e_inf, e_2)
    sp.close()


@pytest.mark.parametrize("name,make", [
    ("sab_neq_10_4_3", lambda: I.small_problem(10, 4, 3, 70, 97, 4)),     # 97 beta rows: a 1-row last block
    ("rows_64_8_3_4", lambda: I.small_problem(8, 3, 4, 53, 64, 5)),       # whole 8-row blocks, even rows
    ("rows_9_8_4_4", lambda: I.small_problem(8, 4, 4, 60, 9, 7)),         # two blocks, the second of one row
])
def test_sigma_alpha_alpha_column_major(ctx, name, make):
    """The alpha-alpha term read from C column-major (8 staged FP64 rows, the
    path of the 4.0e6 workload) on small ragged spaces, forced with
    SQD_TUNE_SS_ROWS = 8: against the oracle per term and in total, FP64
    <= 1e-12 (and FP32, which keeps the transposes at 8 rows, <= 2e-6)."""
    torch = need_gpu()
    from paper_2601_16169_amd import sqd
    banner(f"alpha-alpha column-major {name}")
    p = make()
    sp = _space(ctx, p)
    osp = core.Space.from_problem(p)
    c = I.random_vector(sp.dim, 19)
    ct = torch.tensor(c, device="cuda:0")
    ctx.set_tuning(sqd.TUNE_SS_ROWS, 8)
    try:
        for mask in (TERMS["AA"], TERMS["AA"] | TERMS["BB"], TERMS["ALL"], TERMS["AA"] | TERMS["DIAG"],
                     TERMS["DIAG"] | TERMS["AA"] | TERMS["BB"]):
            ref = osp.sigma(c, mask)
            for prec, bar in ((sqd.FP64, 1e-12), (sqd.FP32, 2e-6)):
                got = sp.sigma(ct, precision=prec, terms=mask).cpu().numpy()
                e_inf, e_2 = rel_err(got, ref)
                assert e_inf <= bar and e_2 <= bar, (mask, prec, e_inf, e_2)
    finally:
        ctx.set_tuning(sqd.TUNE_SS_ROWS, 0)
    sp.close()
