"""Seeded synthetic inputs for sample-based quantum diagonalization (SQD).

This module is the single source of workload data for both the CPU oracle and
the HIP path.  It holds no part of the method's arithmetic: it draws integrals
and occupation strings from fixed seeds and nothing else.

The paper's own molecules (H2O/cc-pVDZ, N2; Sec. VI and Sec. VII, Tables II-IV)
and its PySCF-derived configuration sets (Sec. II) are not available, so these
generators stand in for them:

* one-electron integrals h: symmetric, diagonal sorted ascending in a stated
  range, off-diagonal N(0, 0.05) (standard deviation);
* two-electron integrals (pq|rs) = sum_k L^k_pq L^k_rs with symmetric L^k whose
  upper-triangle entries are N(0, 0.1), which gives the full 8-fold symmetry of
  real chemists'-notation integrals;
* alpha/beta strings: the Hartree-Fock string plus strings that move k
  electrons from the HF occupied set to the HF virtual set, k ~ Geometric(0.4)
  (support 1, 2, ...), mimicking "keep configurations whose coefficient is
  above a cutoff" (Sec. II), which favours low excitation ranks.

Draw order (fixed, so that every consumer sees identical arrays): the h
diagonal, then the h upper triangle row-major, then L^k k-major with each
upper triangle (diagonal included) row-major.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Integrals:
    norb: int
    h: np.ndarray        # (norb, norb) float64, symmetric
    eri: np.ndarray      # (norb, norb, norb, norb) float64, (pq|rs) at [p, q, r, s]
    ecore: float = 0.0


@dataclasses.dataclass(frozen=True)
class Problem:
    """One SQD subspace: integrals plus sorted alpha and beta string sets."""
    name: str
    ints: Integrals
    nalpha: int
    nbeta: int
    astr: np.ndarray     # uint64, strictly ascending
    bstr: np.ndarray     # uint64, strictly ascending

    @property
    def norb(self) -> int:
        return self.ints.norb

    @property
    def dim(self) -> int:
        return int(len(self.astr)) * int(len(self.bstr))

    @property
    def nwords(self) -> int:
        return 1 if np.asarray(self.astr).ndim == 1 else int(np.asarray(self.astr).shape[1])


def make_integrals(norb: int, nchol: int, seed: int,
                   diag_range: Tuple[float, float] = (-2.0, 0.0),
                   offdiag_sd: float = 0.05, chol_sd: float = 0.1) -> Integrals:
    """Random real integrals with the symmetry of a molecular Hamiltonian."""
    rng = np.random.default_rng(seed)
    h = np.zeros((norb, norb))
    h[np.diag_indices(norb)] = np.sort(rng.uniform(diag_range[0], diag_range[1], norb))
    iu = np.triu_indices(norb, 1)
    off = rng.normal(0.0, offdiag_sd, len(iu[0]))
    h[iu] = off
    h[(iu[1], iu[0])] = off
    iu0 = np.triu_indices(norb, 0)
    L = np.zeros((nchol, norb, norb))
    for k in range(nchol):
        v = rng.normal(0.0, chol_sd, len(iu0[0]))
        L[k][iu0] = v
        L[k][(iu0[1], iu0[0])] = v
    Lm = L.reshape(nchol, norb * norb)
    eri = (Lm.T @ Lm).reshape(norb, norb, norb, norb)
    # exact symmetrisation of rounding noise so that (pq|rs)=(rs|pq) bit for bit
    eri = 0.5 * (eri + eri.transpose(2, 3, 0, 1))
    return Integrals(norb=norb, h=np.ascontiguousarray(h), eri=np.ascontiguousarray(eri))


def hf_string(n: int) -> int:
    return (1 << n) - 1


def sample_strings(norb: int, n: int, count: int, seed: int, p: float = 0.4,
                   max_draws: Optional[int] = None) -> np.ndarray:
    """HF-biased unique occupation strings, returned sorted ascending (uint64).

    The HF string (lowest n orbitals) is always included.  Each further draw
    takes k ~ Geometric(p) capped at min(n, norb - n), then flips k distinct
    HF-occupied and k distinct HF-virtual orbitals chosen uniformly; duplicates
    are rejected until ``count`` unique strings exist.
    """
    from math import comb
    if count > comb(norb, n):
        raise ValueError("requested more strings than C(norb, n)")
    rng = np.random.default_rng(seed)
    kmax = min(n, norb - n)
    hf = hf_string(n)
    seen = {hf}
    out = [hf]
    draws = 0
    limit = max_draws if max_draws is not None else 1000 * count + 10000
    while len(out) < count:
        draws += 1
        if draws > limit:
            raise RuntimeError("string sampler did not reach the requested count")
        k = min(int(rng.geometric(p)), kmax)
        occ = rng.choice(n, size=k, replace=False)
        vir = rng.choice(norb - n, size=k, replace=False) + n
        s = hf
        for o in occ:
            s &= ~(1 << int(o))
        for v in vir:
            s |= (1 << int(v))
        if s not in seen:
            seen.add(s)
            out.append(s)
    return np.array(sorted(out), dtype=np.uint64)


def to_words(strings, nw: int = 2) -> np.ndarray:
    """Strings (Python ints or a uint64 array) as an (n, nw) uint64 array, word
    q holding orbitals 64 q .. 64 q + 63."""
    vals = [int(x) for x in strings]
    out = np.zeros((len(vals), nw), dtype=np.uint64)
    for k, v in enumerate(vals):
        for q in range(nw):
            out[k, q] = (v >> (64 * q)) & 0xFFFFFFFFFFFFFFFF
    return out


def from_words(words: np.ndarray) -> list:
    """Inverse of to_words: Python ints."""
    a = np.asarray(words, dtype=np.uint64)
    if a.ndim == 1:
        return [int(x) for x in a]
    return [sum(int(w) << (64 * q) for q, w in enumerate(row)) for row in a]


def sample_strings_words(norb: int, n: int, count: int, seed: int, p: float = 0.4) -> np.ndarray:
    """HF-biased strings as sample_strings, for norb up to 128: an ascending
    (count, 2) uint64 array of two-word strings."""
    from math import comb
    if count > comb(norb, n):
        raise ValueError("requested more strings than C(norb, n)")
    rng = np.random.default_rng(seed)
    kmax = min(n, norb - n)
    hf = hf_string(n)
    seen = {hf}
    while len(seen) < count:
        k = min(int(rng.geometric(p)), kmax)
        occ = rng.choice(n, size=k, replace=False)
        vir = rng.choice(norb - n, size=k, replace=False) + n
        s = hf
        for o in occ:
            s &= ~(1 << int(o))
        for v in vir:
            s |= (1 << int(v))
        seen.add(s)
    return to_words(sorted(seen), 2)


def embed_problem(prob: "Problem", norb_big: int, orb_map, seed: int) -> "Problem":
    """The same problem on norb_big orbitals: orbital p becomes orb_map[p]
    (distinct, below norb_big); the other orbitals are never occupied.  The
    integrals among mapped orbitals are the original ones; every other
    integral is random (with the full symmetry), and none of them can enter
    H restricted to the embedded strings.  Strings are two-word arrays sorted
    ascending; with an increasing orb_map the order, and every sign, of the
    original is kept."""
    m = np.asarray(orb_map, dtype=np.int64)
    assert len(m) == prob.norb and len(set(m.tolist())) == prob.norb and m.max() < norb_big
    big = make_integrals(norb_big, 4, seed)
    h = big.h.copy()
    eri = big.eri.copy()
    h[np.ix_(m, m)] = prob.ints.h
    eri[np.ix_(m, m, m, m)] = prob.ints.eri

    def relabel(strs):
        out = []
        for s in from_words(strs):
            t = 0
            for q in range(prob.norb):
                if (s >> q) & 1:
                    t |= 1 << int(m[q])
            out.append(t)
        return to_words(sorted(out), 2)

    ints = Integrals(norb=norb_big, h=np.ascontiguousarray(h), eri=np.ascontiguousarray(eri), ecore=prob.ints.ecore)
    return Problem(f"{prob.name}_in{norb_big}", ints, prob.nalpha, prob.nbeta, relabel(prob.astr), relabel(prob.bstr))


def words_problem(norb: int, nalpha: int, nbeta: int, na: int, nb: int, seed: int) -> "Problem":
    """A random problem on norb (<= 128) orbitals with two-word strings
    (HF-biased alpha and beta sets drawn independently)."""
    ints = make_integrals(norb, 4, seed=seed)
    a = sample_strings_words(norb, nalpha, na, 1000 + seed)
    b = sample_strings_words(norb, nbeta, nb, 2000 + seed)
    return Problem(f"words_{norb}_{nalpha}_{nbeta}_{na}_{nb}_{seed}", ints, nalpha, nbeta, a, b)


def all_strings(norb: int, n: int) -> np.ndarray:
    """Every string with n of norb bits set, ascending."""
    from itertools import combinations
    vals = []
    for occ in combinations(range(norb), n):
        s = 0
        for o in occ:
            s |= 1 << o
        vals.append(s)
    return np.array(sorted(vals), dtype=np.uint64)


def random_subset(strings: np.ndarray, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(strings), size=count, replace=False)
    return np.array(sorted(strings[idx].tolist()), dtype=np.uint64)


def random_vector(dim: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) vector (float64)."""
    return np.random.default_rng(seed).standard_normal(dim)


def guess_noise(dim: int, seed: int = 7, norm: float = 1e-3) -> np.ndarray:
    """Seeded noise added to the Davidson start vector (norm ``norm``).

    The start vector is the unit vector on the lowest diagonal element plus
    this noise, so that a guess with the spin-flip symmetry of an S_a = S_b
    space can still reach a flip-odd lowest state.
    """
    v = np.random.default_rng(seed).standard_normal(dim)
    return v * (norm / np.linalg.norm(v))


# ---------------------------------------------------------------------------
# Named workloads.  Integral seed = workload number; string seed = 100 + number;
# the batched workload draws its counts from seed 104 and batch b uses 400 + b.
# ---------------------------------------------------------------------------

def cfg1() -> Problem:
    """norb 8, 4+4 electrons, all 70 strings per spin (full CI, dim 4900)."""
    ints = make_integrals(8, 16, seed=1)
    s = all_strings(8, 4)
    return Problem("cfg1_norb8_n4_full", ints, 4, 4, s, s.copy())


def cfg2() -> Problem:
    """norb 16, 8+8, 2000 HF-biased strings shared by both spins (dim 4.0e6)."""
    ints = make_integrals(16, 40, seed=2)
    s = sample_strings(16, 8, 2000, seed=102)
    return Problem("cfg2_norb16_n8_2000", ints, 8, 8, s, s.copy())


def cfg3(nstr: int = 16000) -> Problem:
    """norb 36, 12+12, 16000 HF-biased strings per spin (dim 2.56e8)."""
    ints = make_integrals(36, 120, seed=3, diag_range=(-20.0, 2.0))
    s = sample_strings(36, 12, nstr, seed=103)
    return Problem(f"cfg3_norb36_n12_{nstr}", ints, 12, 12, s, s.copy())


def cfg4_counts() -> np.ndarray:
    return np.random.default_rng(104).integers(200, 3001, size=64)


def cfg4(nbatch: int = 64) -> List[Problem]:
    """64 independent subspaces, norb 24, 8+8, N_b ~ U{200..3000}, shared integrals."""
    ints = make_integrals(24, 60, seed=4)
    counts = cfg4_counts()[:nbatch]
    out = []
    for b, nb in enumerate(counts):
        s = sample_strings(24, 8, int(nb), seed=400 + b)
        out.append(Problem(f"cfg4_b{b}_n{nb}", ints, 8, 8, s, s.copy()))
    return out


def cfg5() -> Problem:
    """norb 20, 7+7, 4000 HF-biased strings per spin (dim 1.6e7), FP64 + RDMs."""
    ints = make_integrals(20, 50, seed=5)
    s = sample_strings(20, 7, 4000, seed=105)
    return Problem("cfg5_norb20_n7_4000", ints, 7, 7, s, s.copy())


def small_problem(norb: int, nalpha: int, nbeta: int, na: int, nb: int, seed: int,
                  nchol: Optional[int] = None, diag_range=(-2.0, 0.0)) -> Problem:
    """A small random problem with independent alpha and beta string sets."""
    from math import comb
    ints = make_integrals(norb, nchol or max(2, 2 * norb), seed=seed, diag_range=diag_range)
    def pick(n, count, sd):
        total = comb(norb, n)
        if count >= total:
            return all_strings(norb, n)
        if total <= 20000:
            return random_subset(all_strings(norb, n), count, sd)
        return sample_strings(norb, n, count, sd)
    a = pick(nalpha, na, 1000 + seed)
    b = pick(nbeta, nb, 2000 + seed)
    return Problem(f"small_{norb}_{nalpha}_{nbeta}_{na}_{nb}_{seed}", ints, nalpha, nbeta, a, b)


def full14() -> Problem:
    """norb 14, 7+7, all 3432 strings per spin (full CI, dim 1.18e7): the
    regime the Knowles-Handy form was made for, used to compare the two
    alpha-beta paths."""
    ints = make_integrals(14, 28, seed=9)
    s = all_strings(14, 7)
    return Problem("full_norb14_n7", ints, 7, 7, s, s.copy())


WORKLOADS = {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3, "cfg5": cfg5, "full14": full14}
