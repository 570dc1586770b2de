"""Jordan-Wigner brute force on the full Fock space (test infrastructure only).

For norb <= 5 (2*norb <= 10 spin-orbitals, 1024 Fock states) the ladder
operators are built as Kronecker products of 2x2 matrices (a parity string of
Z factors on all lower modes, the lowering matrix on the mode itself), and the
Hamiltonian of Sec. I / Sec. II is assembled from them term by term:

    H = Ecore + sum_{PQ} h_pq [sP==sQ] a+_P a_Q
              + 1/2 sum_{PQRS} (pq|rs) [sP==sQ][sR==sS] a+_P a+_R a_S a_Q .

Spin-orbital P = p for alpha and norb + p for beta; Fock state index = bit
pattern D = Ialpha | (Ibeta << norb).  With this mode order the determinant
a+_{P1} a+_{P2} ... |0> (P1 < P2 < ...) is exactly +|D>, so H_S[I, J] =
<D_I| H |D_J>.  The sign of every matrix element therefore comes from the
tensor-product parity strings, not from any bit-counting code, which makes
this an independent check of the oracle's operator application.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def ladder_ops(nmodes: int):
    """Annihilation operators a_P (P = 0..nmodes-1) as sparse matrices on
    2**nmodes states, state index = sum_P n_P 2**P."""
    I2 = sp.identity(2, format="csr", dtype=np.float64)
    Z = sp.csr_matrix(np.diag([1.0, -1.0]))
    low = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))  # |1> -> |0>
    ops = []
    for P in range(nmodes):
        # kron order: most significant mode first
        m = None
        for k in range(nmodes - 1, -1, -1):
            f = I2 if k > P else (low if k == P else Z)
            m = f if m is None else sp.kron(m, f, format="csr")
        ops.append(m.tocsr())
    return ops


def mode_labels(norb, interleaved=False):
    """(spin, orbital) of each mode.  Block order: alpha 0..norb-1 then beta;
    interleaved order: 0a, 0b, 1a, 1b, ..."""
    if interleaved:
        return [k % 2 for k in range(2 * norb)], [k // 2 for k in range(2 * norb)]
    return [0] * norb + [1] * norb, list(range(norb)) * 2


def fock_hamiltonian(norb, h, eri, ecore=0.0, interleaved=False):
    M = 2 * norb
    a = ladder_ops(M)
    ad = [x.T.tocsr() for x in a]
    dim = 1 << M
    H = sp.csr_matrix((dim, dim))
    spin, orb = mode_labels(norb, interleaved)
    for P in range(M):
        for Q in range(M):
            if spin[P] == spin[Q] and h[orb[P], orb[Q]] != 0.0:
                H = H + h[orb[P], orb[Q]] * (ad[P] @ a[Q])
    mid = {}
    for R in range(M):
        for S in range(M):
            if spin[R] == spin[S]:
                mid[(R, S)] = (ad[R] @ a[S]).tocsr()
    for P in range(M):
        for Q in range(M):
            if spin[P] != spin[Q]:
                continue
            inner = sp.csr_matrix((dim, dim))
            for (R, S), m in mid.items():
                v = eri[orb[P], orb[Q], orb[R], orb[S]]
                if v != 0.0:
                    inner = inner + v * m
            H = H + 0.5 * (ad[P] @ inner @ a[Q])
    if ecore:
        H = H + ecore * sp.identity(dim, format="csr")
    return H.tocsr()


def det_index(norb, astr, bstr, interleaved=False):
    """Fock-state indices of the product space, alpha-major."""
    a = np.asarray(astr, dtype=np.uint64).astype(np.int64)
    b = np.asarray(bstr, dtype=np.uint64).astype(np.int64)
    if not interleaved:
        return (a[:, None] | (b[None, :] << norb)).reshape(-1)
    def spread(x, off):
        out = np.zeros_like(x)
        for k in range(norb):
            out |= ((x >> k) & 1) << (2 * k + off)
        return out
    return (spread(a, 0)[:, None] | spread(b, 1)[None, :]).reshape(-1)


def projected_hamiltonian(norb, astr, bstr, h, eri, ecore=0.0, interleaved=False):
    H = fock_hamiltonian(norb, h, eri, ecore, interleaved)
    idx = det_index(norb, astr, bstr, interleaved)
    return np.asarray(H[idx][:, idx].todense())


def fock_rdms(norb, astr, bstr, c):
    """Spin-summed 1- and 2-RDMs of the space vector c embedded in Fock space."""
    M = 2 * norb
    a = ladder_ops(M)
    ad = [x.T.tocsr() for x in a]
    psi = np.zeros(1 << M)
    psi[det_index(norb, astr, bstr)] = c
    spin = [0] * norb + [1] * norb
    orb = list(range(norb)) * 2
    g1 = np.zeros((norb, norb))
    g2 = np.zeros((norb, norb, norb, norb))
    aq = [a[Q] @ psi for Q in range(M)]
    for P in range(M):
        for Q in range(M):
            if spin[P] == spin[Q]:
                g1[orb[P], orb[Q]] += psi @ (ad[P] @ aq[Q])
    for P in range(M):
        for Q in range(M):
            if spin[P] != spin[Q]:
                continue
            for R in range(M):
                for S in range(M):
                    if spin[R] != spin[S]:
                        continue
                    v = ad[P] @ (ad[R] @ (a[S] @ aq[Q]))
                    g2[orb[P], orb[Q], orb[R], orb[S]] += psi @ v
    return g1, g2


def single_spin_element(norb, target, source, create, annihilate):
    """<target| a+_create a_annihilate |source> on a single spin's Fock space
    (norb modes), by the Kronecker-product operators."""
    a = ladder_ops(norb)
    ad = [x.T.tocsr() for x in a]
    op = ad[create] @ a[annihilate]
    return float(op[int(target), int(source)])


def single_spin_double_element(norb, target, source, a_, b_, i_, j_):
    """<target| a+_a a+_b a_j a_i |source> on one spin's Fock space."""
    a = ladder_ops(norb)
    ad = [x.T.tocsr() for x in a]
    op = ad[a_] @ ad[b_] @ a[j_] @ a[i_]
    return float(op[int(target), int(source)])
