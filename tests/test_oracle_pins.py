"""Pins of the CPU oracle against facts fixed by the mathematics, not by the
oracle itself: Jordan-Wigner brute force, closed forms, invariants, bounds.

The paper prints no worked example or energy (its tables are timings and
counters), so every pin here is mathematical.
"""
import numpy as np
import pytest

from paper_2601_16169_amd import inputs as I
from oracle import core, davidson, fock, tables

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")


def _space(p):
    return core.Space.from_problem(p)


@pytest.mark.parametrize("norb,na_el,nb_el,na,nb,seed", [
    (4, 2, 2, 6, 6, 1),      # complete space
    (4, 2, 1, 5, 4, 2),      # n_alpha != n_beta, subsets
    (5, 3, 2, 7, 9, 3),      # S_alpha != S_beta, random subsets
    (5, 2, 2, 10, 10, 4),    # complete space, norb 5
    (5, 1, 3, 5, 6, 5),
])
def test_elements_match_jordan_wigner(norb, na_el, nb_el, na, nb, seed):
    """Every H_S[I, J] of the oracle, signs included, equals the projected
    Fock-space Hamiltonian built from Kronecker-product ladder operators."""
    p = I.small_problem(norb, na_el, nb_el, na, nb, seed)
    H = _space(p).dense()
    Hj = fock.projected_hamiltonian(norb, p.astr, p.bstr, p.ints.h, p.ints.eri)
    assert np.abs(H - Hj).max() <= 1e-14 * max(1.0, np.abs(Hj).max())


def test_ecore_shifts_diagonal():
    p = I.small_problem(4, 2, 2, 5, 5, 9)
    s0 = core.Space(p.norb, p.astr, p.bstr, p.ints.h, p.ints.eri, 0.0)
    s1 = core.Space(p.norb, p.astr, p.bstr, p.ints.h, p.ints.eri, 1.25)
    assert np.allclose(s1.dense() - s0.dense(), 1.25 * np.eye(s0.dim), atol=1e-14, rtol=0)


@pytest.mark.parametrize("t,U", [(1.0, 4.0), (0.5, 1.0), (1.3, 0.0), (0.2, 8.0)])
def test_two_site_hubbard_closed_form(t, U):
    """norb 2, one electron per spin, h = [[0,-t],[-t,0]], only (00|00) =
    (11|11) = U: E0 = (U - sqrt(U^2 + 16 t^2)) / 2."""
    h = np.array([[0.0, -t], [-t, 0.0]])
    eri = np.zeros((2, 2, 2, 2))
    eri[0, 0, 0, 0] = eri[1, 1, 1, 1] = U
    s = I.all_strings(2, 1)
    sp_ = core.Space(2, s, s, h, eri)
    E = np.linalg.eigvalsh(sp_.dense())[0]
    assert abs(E - (U - np.sqrt(U * U + 16 * t * t)) / 2) <= 1e-14 * max(1, U, t)


def test_noninteracting_complete_space_sum_of_orbital_energies():
    """V = 0, complete space: E0 = sum of the n_alpha + n_beta lowest
    eigenvalues of h (occupied separately per spin)."""
    norb, na_el, nb_el = 6, 3, 2
    ints = I.make_integrals(norb, 4, seed=21)
    eri = np.zeros_like(ints.eri)
    eps = np.linalg.eigvalsh(ints.h)
    sp_ = core.Space(norb, I.all_strings(norb, na_el), I.all_strings(norb, nb_el), ints.h, eri)
    E = np.linalg.eigvalsh(sp_.dense())[0]
    assert abs(E - (eps[:na_el].sum() + eps[:nb_el].sum())) <= 1e-12


def test_diagonal_h_no_interaction_any_subset_with_hf():
    """Diagonal h, V = 0, any space holding the HF strings: E0 = sum of the
    lowest h_ii per spin, and the vector is the HF determinant."""
    norb = 8
    ints = I.make_integrals(norb, 4, seed=22)
    h = np.diag(np.diag(ints.h))
    a = I.sample_strings(norb, 3, 20, seed=5)
    b = I.sample_strings(norb, 4, 25, seed=6)
    sp_ = core.Space(norb, a, b, h, np.zeros_like(ints.eri))
    E = np.linalg.eigvalsh(sp_.dense())[0]
    hd = np.sort(np.diag(h))
    assert abs(E - (hd[:3].sum() + hd[:4].sum())) <= 1e-13


def test_hermiticity_random_vectors():
    p = I.small_problem(8, 3, 4, 30, 40, 11)
    sp_ = _space(p)
    x = I.random_vector(sp_.dim, 1)
    y = I.random_vector(sp_.dim, 2)
    lhs, rhs = x @ sp_.sigma(y), y @ sp_.sigma(x)
    Hn = np.abs(sp_.dense()).sum(axis=1).max()
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(x) * np.linalg.norm(y) * Hn


def test_sigma_equals_dense_product_and_terms_sum():
    p = I.small_problem(6, 3, 2, 12, 15, 12)
    sp_ = _space(p)
    c = I.random_vector(sp_.dim, 3)
    H = sp_.dense()
    s = sp_.sigma(c)
    assert np.abs(s - H @ c).max() <= 1e-12 * np.abs(s).max()
    parts = [sp_.sigma(c, m) for m in (core.DIAG, core.AA, core.BB, core.AB)]
    assert np.abs(sum(parts) - s).max() <= 1e-12 * np.abs(s).max()
    assert np.allclose(parts[0], sp_.diag() * c, atol=1e-13, rtol=0)
    rows = np.array([0, 7, sp_.dim - 1, 33])
    assert np.allclose(sp_.sigma_rows(c, rows), s[rows], atol=1e-13, rtol=0)


def test_term_classes_touch_only_their_blocks():
    """AA couples only equal beta strings, BB only equal alpha strings,
    AB only pairs that differ in both (one electron each)."""
    p = I.small_problem(6, 2, 3, 10, 12, 13)
    sp_ = _space(p)
    na, nb = sp_.na, sp_.nb
    for mask in (core.AA, core.BB, core.AB):
        M = np.zeros((sp_.dim, sp_.dim))
        for j in range(sp_.dim):
            e = np.zeros(sp_.dim)
            e[j] = 1.0
            M[:, j] = sp_.sigma(e, mask)
        ii, jj = np.nonzero(M)
        ia, ib, ja, jb = ii // nb, ii % nb, jj // nb, jj % nb
        if mask == core.AA:
            assert np.all(ib == jb) and np.all(ia != ja)
        elif mask == core.BB:
            assert np.all(ia == ja) and np.all(ib != jb)
        else:
            assert np.all(ia != ja) and np.all(ib != jb)


def test_spin_flip_symmetry():
    """S_alpha = S_beta and n_alpha = n_beta: sigma(C^T) = sigma(C)^T."""
    p = I.small_problem(7, 3, 3, 20, 20, 14)
    s = p.astr
    sp_ = core.Space(p.norb, s, s, p.ints.h, p.ints.eri)
    n = len(s)
    C = I.random_vector(n * n, 4).reshape(n, n)
    a = sp_.sigma(C.T.reshape(-1)).reshape(n, n)
    b = sp_.sigma(C.reshape(-1)).reshape(n, n).T
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def test_variational_nested_subsets():
    """S1 c S2 c full: E(S1) >= E(S2) >= E_FCI (Cauchy interlacing)."""
    p = I.cfg1()
    full = p.astr
    rng = np.random.default_rng(3)
    hf = I.hf_string(4)
    rest = [int(x) for x in full if int(x) != hf]
    rng.shuffle(rest)
    energies = []
    for k in (10, 25, 45, 70):
        sub = np.array(sorted([hf] + rest[:k - 1]), dtype=np.uint64)
        sp_ = core.Space(8, sub, sub, p.ints.h, p.ints.eri)
        energies.append(np.linalg.eigvalsh(sp_.dense())[0])
    assert all(energies[i] >= energies[i + 1] - 1e-12 for i in range(3))


def test_orbital_permutation_invariance():
    norb = 6
    p = I.small_problem(norb, 3, 2, 20, 15, 15)
    E0 = np.linalg.eigvalsh(_space(p).dense())[0]
    perm = np.random.default_rng(2).permutation(norb)
    h2 = p.ints.h[np.ix_(perm, perm)]
    e2 = p.ints.eri[np.ix_(perm, perm, perm, perm)]
    inv = np.argsort(perm)  # new orbital k = old orbital perm[k]

    def relabel(strings):
        out = []
        for s in strings:
            t = 0
            for old in range(norb):
                if (int(s) >> old) & 1:
                    t |= 1 << int(inv[old])
            out.append(t)
        return np.array(sorted(out), dtype=np.uint64)

    sp2 = core.Space(norb, relabel(p.astr), relabel(p.bstr), h2, e2)
    E1 = np.linalg.eigvalsh(sp2.dense())[0]
    assert abs(E1 - E0) <= 1e-12


def test_phase_convention_does_not_change_spectrum():
    """Block (alpha-first) and interleaved spin-orbital orders differ by a
    +-1 per determinant: same spectrum."""
    p = I.small_problem(4, 2, 2, 5, 6, 16)
    Hb = fock.projected_hamiltonian(4, p.astr, p.bstr, p.ints.h, p.ints.eri)
    Hi = fock.projected_hamiltonian(4, p.astr, p.bstr, p.ints.h, p.ints.eri, interleaved=True)
    assert np.allclose(np.linalg.eigvalsh(Hb), np.linalg.eigvalsh(Hi), atol=1e-13)
    assert np.allclose(np.abs(Hb), np.abs(Hi), atol=1e-14)
    # the two orders really differ by determinant phases
    assert np.any(np.sign(Hb) * np.sign(Hi) < 0)


def test_davidson_matches_dense_cfg1():
    p = I.cfg1()
    sp_ = _space(p)
    E, x, _ = davidson.dense_lowest(sp_.dense())
    r = davidson.davidson(sp_.sigma, sp_.diag(), I.guess_noise(sp_.dim), tol=1e-10)
    assert r.converged
    assert abs(r.energy - E) <= 1e-10
    assert 1 - abs(r.vector @ x) <= 1e-12


def test_davidson_small_restart_path():
    """m_max small forces collapses; the answer must not change."""
    p = I.small_problem(6, 3, 3, 20, 20, 17)
    sp_ = _space(p)
    E = np.linalg.eigvalsh(sp_.dense())[0]
    r = davidson.davidson(sp_.sigma, sp_.diag(), I.guess_noise(sp_.dim), tol=1e-9, m_max=4)
    assert r.converged and abs(r.energy - E) <= 1e-9


@pytest.mark.parametrize("norb,na_el,nb_el,na,nb,seed", [
    (6, 3, 3, 20, 20, 31),    # complete-size subsets, equal electron counts
    (7, 3, 2, 25, 18, 32),    # S_alpha != S_beta, n_alpha != n_beta
    (8, 4, 1, 30, 8, 33),     # complete beta set of one electron
    (5, 0, 2, 1, 10, 34),     # no alpha electrons: a single empty alpha string
])
def test_memoised_h_matches_matrix_free_and_dense(norb, na_el, nb_el, na, nb, seed):
    """The CSR copy of H that the larger Davidson runs iterate with holds the
    same matrix as the matrix-free product and the dense H (itself pinned to
    Jordan-Wigner above): row pointers, column indices and values all checked
    by products with unit and random vectors, and the diagonal stored first."""
    p = I.small_problem(norb, na_el, nb_el, na, nb, seed)
    sp_ = _space(p)
    M = core.MemoisedH(sp_)
    H = sp_.dense()
    # the stored pattern is exactly the set of connected pairs
    assert M.nnz == int(sum(M.rowptr[r + 1] - M.rowptr[r] for r in range(sp_.dim)))
    assert np.all(M.cols[M.rowptr[:-1]] == np.arange(sp_.dim))
    D = np.zeros_like(H)
    for r in range(sp_.dim):
        k0, k1 = M.rowptr[r], M.rowptr[r + 1]
        assert len(set(M.cols[k0:k1].tolist())) == k1 - k0     # no column stored twice
        D[r, M.cols[k0:k1]] = M.vals[k0:k1]
    assert np.abs(D - H).max() <= 1e-15 * max(1.0, np.abs(H).max())
    for seed_c in (1, 2):
        c = I.random_vector(sp_.dim, seed_c)
        s = sp_.sigma(c)
        y = M.matvec(c)
        assert np.abs(y - s).max() <= 1e-14 * np.abs(s).max()
        assert np.abs(y - H @ c).max() <= 1e-13 * np.abs(s).max()


def test_memoised_h_only_doubles_and_isolated_strings():
    """Strings without any in-set single: alpha strings four bits apart
    (doubles only) and one beta string (no same-spin partner at all)."""
    norb = 8
    ints = I.make_integrals(norb, 8, seed=35)
    a = np.array(sorted([0b00001111, 0b00111100, 0b11110000]), dtype=np.uint64)
    b = np.array([0b00000111], dtype=np.uint64)
    sp_ = core.Space(norb, a, b, ints.h, ints.eri)
    M = core.MemoisedH(sp_)
    H = sp_.dense()
    c = I.random_vector(sp_.dim, 3)
    assert np.abs(M.matvec(c) - H @ c).max() <= 1e-14 * np.abs(H @ c).max()
    assert np.abs(M.matvec(c) - sp_.sigma(c)).max() <= 1e-14 * np.abs(H @ c).max()


def test_memoised_h_large_space_sampled_rows():
    """A space of dimension 1.6e5 (HF-biased strings, norb 16): the CSR
    product equals the matrix-free product on 2000 seeded rows."""
    norb = 16
    ints = I.make_integrals(norb, 20, seed=36)
    s = I.sample_strings(norb, 8, 400, seed=136)
    sp_ = core.Space(norb, s, s, ints.h, ints.eri)
    assert sp_.dim > 100000
    M = core.MemoisedH(sp_)
    c = I.random_vector(sp_.dim, 4)
    rows = np.sort(np.random.default_rng(5).choice(sp_.dim, size=2000, replace=False))
    ref = sp_.sigma_rows(c, rows)
    y = M.matvec(c)
    assert np.abs(y[rows] - ref).max() <= 1e-14 * np.abs(ref).max()
    assert np.all(M.cols[M.rowptr[:-1]] == np.arange(sp_.dim))


def test_davidson_collapse_reaches_dense_energy():
    """Plain collapse onto the current Ritz vector at m_max (the restart rule
    of the oracle) on cfg1 and two small spaces: the converged energy is the
    dense one to 1e-10, whatever m_max."""
    for p, tol in ((I.cfg1(), 1e-10), (I.small_problem(7, 3, 2, 25, 18, 32), 1e-10),
                   (I.small_problem(8, 4, 4, 40, 40, 37), 1e-10)):
        sp_ = _space(p)
        E = np.linalg.eigvalsh(sp_.dense())[0]
        M = core.MemoisedH(sp_)    # pinned to the matrix-free product above
        for m_max in (4, 12, 24):
            r = davidson.davidson(M.matvec, sp_.diag(), I.guess_noise(sp_.dim), tol=tol, m_max=m_max,
                                  max_iter=600)
            assert r.converged and abs(r.energy - E) <= 1e-10, (p.name, m_max, r.energy - E)


# ---------------------------------------------------------------- RDMs

def test_rdms_match_jordan_wigner():
    p = I.small_problem(4, 2, 1, 6, 4, 18)
    sp_ = _space(p)
    c = I.random_vector(sp_.dim, 7)
    c /= np.linalg.norm(c)
    g1, g2 = sp_.rdm(c)
    j1, j2 = fock.fock_rdms(4, p.astr, p.bstr, c)
    assert np.abs(g1 - j1).max() <= 1e-14
    assert np.abs(g2 - j2).max() <= 1e-14


def test_rdm_invariants_and_energy():
    p = I.small_problem(7, 3, 2, 25, 18, 19)
    sp_ = _space(p)
    H = sp_.dense()
    E, x, _ = davidson.dense_lowest(H)
    g1, g2 = sp_.rdm(x)
    N = 5
    assert abs(np.trace(g1) - N) <= 1e-12
    assert abs(np.einsum("pprr->", g2) - N * (N - 1)) <= 1e-11
    assert abs(sp_.energy_from_rdm(g1, g2) - E) <= 1e-10
    w = np.linalg.eigvalsh(g1)
    assert w.min() >= -1e-12 and w.max() <= 2 + 1e-12
    assert np.abs(g2 - g2.transpose(2, 3, 0, 1)).max() <= 1e-13
    assert np.abs(g1 - g1.T).max() <= 1e-13


def test_hellmann_feynman_finite_difference_small():
    """dE/dh_pq summed over the symmetric pair and dE/d(pq|rs) summed over
    its symmetry orbit equal the RDM contractions (central differences)."""
    p = I.small_problem(5, 2, 2, 8, 8, 20)
    sp_ = _space(p)
    E, x, _ = davidson.dense_lowest(sp_.dense())
    g1, g2 = sp_.rdm(x)
    d = 1e-5

    def energy(h, eri):
        return np.linalg.eigvalsh(core.Space(5, p.astr, p.bstr, h, eri).dense())[0]

    h, eri = p.ints.h, p.ints.eri
    for (a, b) in [(0, 1), (2, 2), (1, 4)]:
        hp, hm = h.copy(), h.copy()
        for (u, v) in {(a, b), (b, a)}:
            hp[u, v] += d
            hm[u, v] -= d
        fd = (energy(hp, eri) - energy(hm, eri)) / (2 * d)
        an = sum(g1[u, v] for (u, v) in {(a, b), (b, a)})
        assert abs(fd - an) <= 1e-6 + 1e-5 * abs(an)
    for (a, b, c_, e) in [(0, 1, 2, 3), (1, 1, 4, 4), (0, 2, 0, 2)]:
        orbit = {(a, b, c_, e), (b, a, c_, e), (a, b, e, c_), (b, a, e, c_),
                 (c_, e, a, b), (e, c_, a, b), (c_, e, b, a), (e, c_, b, a)}
        ep, em = eri.copy(), eri.copy()
        for o in orbit:
            ep[o] += d
            em[o] -= d
        fd = (energy(h, ep) - energy(h, em)) / (2 * d)
        an = sum(0.5 * g2[o] for o in orbit)
        assert abs(fd - an) <= 1e-6 + 1e-5 * abs(an)


# ---------------------------------------------------------------- tables

def test_tables_complete_space_counts():
    s = I.all_strings(8, 4)
    so, se, do, de = tables.build_tables(s, 8)
    assert np.all(np.diff(so) == 16)      # n (norb - n)
    assert np.all(np.diff(do) == 36)      # C(n,2) C(norb-n,2)


def test_table_signs_match_jordan_wigner():
    norb = 5
    s = I.all_strings(norb, 2)
    so, se, do, de = tables.build_tables(s, norb)
    for src in range(len(s)):
        for e in se[so[src]:so[src + 1]]:
            t, i, a, sign = tables.unpack(e, "single")
            assert fock.single_spin_element(norb, s[t], s[src], a, i) == sign
        for e in de[do[src]:do[src + 1]]:
            t, i, j, a, b, sign = tables.unpack(e, "double")
            assert fock.single_spin_double_element(norb, s[t], s[src], a, b, i, j) == sign


def test_tables_find_every_in_set_neighbour():
    s = I.sample_strings(10, 4, 60, seed=8)
    so, se, do, de = tables.build_tables(s, 10)
    for src in range(len(s)):
        got1 = {tables.unpack(e, "single")[0] for e in se[so[src]:so[src + 1]]}
        got2 = {tables.unpack(e, "double")[0] for e in de[do[src]:do[src + 1]]}
        want1 = {t for t in range(len(s)) if bin(int(s[t]) ^ int(s[src])).count("1") == 2}
        want2 = {t for t in range(len(s)) if bin(int(s[t]) ^ int(s[src])).count("1") == 4}
        assert got1 == want1 and got2 == want2
        # canonical order: ascending targets
        t1 = [tables.unpack(e, "single")[0] for e in se[so[src]:so[src + 1]]]
        assert t1 == sorted(t1)


def test_tables_symmetric_connectivity_same_sign():
    s = I.sample_strings(12, 5, 80, seed=9)
    so, se, do, de = tables.build_tables(s, 12)
    fwd = {}
    for src in range(len(s)):
        for e in se[so[src]:so[src + 1]]:
            t, i, a, sg = tables.unpack(e, "single")
            fwd[(src, t)] = sg
    for (src, t), sg in fwd.items():
        assert fwd[(t, src)] == sg


# ---------------------------------------------------------------- inputs

def test_generator_properties():
    p = I.cfg2()
    assert len(p.astr) == 2000 and np.all(p.astr[1:] > p.astr[:-1])
    assert all(bin(int(x)).count("1") == 8 for x in p.astr[:50])
    assert int(I.hf_string(8)) in set(int(x) for x in p.astr)
    e = p.ints.eri
    assert np.array_equal(e, e.transpose(1, 0, 2, 3))
    assert np.array_equal(e, e.transpose(2, 3, 0, 1))
    assert np.array_equal(p.ints.h, p.ints.h.T)
    d = np.diag(p.ints.h)
    assert np.all(np.diff(d) >= 0) and d.min() >= -2 and d.max() <= 0
    # reproducible
    assert np.array_equal(I.cfg2().astr, p.astr)


# ---------------------------------------------------------------- two-word strings (norb > 64)
# The two-word path of the oracle (and of its table builder) is pinned to the
# one-word path, itself pinned to Jordan-Wigner above: a problem on 8 orbitals
# relabelled onto 72 or 96 orbitals, the other orbitals never occupied, is the
# same Hamiltonian.  An increasing relabelling keeps the string order and
# every sign (no empty orbital changes an occupation count below another), so
# sigma agrees element by element; any relabelling keeps the spectrum and,
# up to the determinant permutation and signs, the matrix.

MAP72 = [3, 17, 40, 63, 64, 65, 70, 71]          # increasing, across the word boundary
MAP96 = [90, 5, 64, 33, 71, 2, 95, 60]           # not monotone


def _small8():
    return I.small_problem(8, 3, 4, 37, 53, 3)


def test_two_word_embedding_keeps_sigma_elementwise():
    p = _small8()
    q = I.embed_problem(p, 72, MAP72, seed=11)
    sp, sq = _space(p), _space(q)
    assert sq.nw == 2 and sq.norb == 72
    c = I.random_vector(sp.dim, 3)
    for mask in (core.DIAG, core.AA, core.BB, core.AB, core.ALL):
        a, b = sp.sigma(c, mask), sq.sigma(c, mask)
        assert np.abs(a - b).max() <= 1e-13 * max(1.0, np.abs(a).max()), mask
    assert np.abs(sp.diag() - sq.diag()).max() <= 1e-13


def test_two_word_embedding_keeps_spectrum_and_matrix_up_to_permutation():
    p = _small8()
    q = I.embed_problem(p, 96, MAP96, seed=12)
    Hp, Hq = _space(p).dense(), _space(q).dense()
    wp, wq = np.linalg.eigvalsh(Hp), np.linalg.eigvalsh(Hq)
    assert np.abs(wp - wq).max() <= 1e-10
    # determinant permutation: where each relabelled string landed
    def relabel(s):
        return sum(1 << MAP96[k] for k in range(8) if (int(s) >> k) & 1)
    ia = {v: k for k, v in enumerate(I.from_words(q.astr))}
    ib = {v: k for k, v in enumerate(I.from_words(q.bstr))}
    pa = [ia[relabel(s)] for s in p.astr]
    pb = [ib[relabel(s)] for s in p.bstr]
    perm = np.array([pa[i] * len(pb) + pb[j] for i in range(len(pa)) for j in range(len(pb))])
    Hq_back = Hq[np.ix_(perm, perm)]
    assert np.abs(np.abs(Hq_back) - np.abs(Hp)).max() <= 1e-13 * np.abs(Hp).max()
    # and the signs are a diagonal similarity H_q = D H_p D, D_I the parity of
    # the permutation that sorts the relabelled creators of I (per spin)
    def parity(s):
        occ = [MAP96[k] for k in range(8) if (int(s) >> k) & 1]
        inv = sum(1 for x in range(len(occ)) for y in range(x + 1, len(occ)) if occ[x] > occ[y])
        return -1.0 if inv % 2 else 1.0
    da = np.array([parity(s) for s in p.astr])
    db = np.array([parity(s) for s in p.bstr])
    d = np.outer(da, db).ravel()
    assert np.abs(Hq_back - np.outer(d, d) * Hp).max() <= 1e-13 * np.abs(Hp).max()


def test_two_word_tables_are_relabelled_one_word_tables():
    p = _small8()
    q = I.embed_problem(p, 72, MAP72, seed=11)
    for s1, s2 in ((p.astr, q.astr), (p.bstr, q.bstr)):
        so, se, do, de = tables.build_tables(s1, 8)
        so2, se2, do2, de2 = tables.build_tables(s2, 72)
        assert np.array_equal(so, so2) and np.array_equal(do, do2)
        for e, e2 in zip(se, se2):
            t, i, a, sg = tables.unpack(e, "single")
            assert tables.unpack(e2, "single") == (t, MAP72[i], MAP72[a], sg)
        for e, e2 in zip(de, de2):
            t, i, j, a, b, sg = tables.unpack(e, "double")
            assert tables.unpack(e2, "double") == (t, MAP72[i], MAP72[j], MAP72[a], MAP72[b], sg)


def test_two_word_rdms_are_relabelled():
    p = _small8()
    q = I.embed_problem(p, 72, MAP72, seed=11)
    c = I.random_vector(_space(p).dim, 4)
    c /= np.linalg.norm(c)
    g1, g2 = _space(p).rdm(c)
    h1, h2 = _space(q).rdm(c)
    m = np.array(MAP72)
    assert np.abs(h1[np.ix_(m, m)] - g1).max() <= 1e-13
    assert np.abs(h2[np.ix_(m, m, m, m)] - g2).max() <= 1e-13
    assert abs(np.abs(h1).sum() - np.abs(g1).sum()) <= 1e-12
    assert abs(np.abs(h2).sum() - np.abs(g2).sum()) <= 1e-10
