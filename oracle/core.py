"""ctypes front end of the plain C oracle (test infrastructure only).

Every function follows the definition of the Hamiltonian in second
quantization (Sec. I; the matrix elements H_ij of Sec. II recomputed from the
integrals with a sign) restricted to the product space of alpha and beta
strings (Sec. IV).  Vectors are indexed d = ia * nb + ib over the ascending
string lists.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

DIAG, AA, BB, AB = 1, 2, 4, 8
ALL = DIAG | AA | BB | AB

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build_oracle
            build_oracle.build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        d = ctypes.c_double
        ci = ctypes.c_int
        L.oracle_sigma.argtypes = [ci, ci, P, i64, P, i64, P, P, d, P, P, ctypes.c_uint]
        L.oracle_sigma_rows.argtypes = [ci, ci, P, i64, P, i64, P, P, d, P, P, i64, P, ctypes.c_uint]
        L.oracle_diag.argtypes = [ci, ci, P, i64, P, i64, P, P, d, P]
        L.oracle_dense.argtypes = [ci, ci, P, i64, P, i64, P, P, d, P]
        L.oracle_rdm.argtypes = [ci, ci, P, i64, P, i64, P, P, P]
        L.oracle_h_elem.argtypes = [ci, ci, P, i64, P, i64, P, P, d, i64, i64, i64, i64]
        L.oracle_h_elem.restype = d
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_csr_count.argtypes = [ci, ci, P, i64, P, i64, P]
        L.oracle_csr_fill.argtypes = [ci, ci, P, i64, P, i64, P, P, d, P, P, P]
        L.oracle_csr_matvec.argtypes = [i64, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ascending(words: np.ndarray) -> bool:
    """Strings (n x nw words, word 0 lowest) strictly ascending as integers."""
    vals = [sum(int(w) << (64 * q) for q, w in enumerate(row)) for row in words]
    return all(b > a for a, b in zip(vals, vals[1:]))


class Space:
    """Integrals plus ascending string sets, held as contiguous numpy arrays.

    A string is one uint64 (norb <= 64; arrays of shape (n,)) or nw words
    (arrays of shape (n, nw), word q holding orbitals 64 q .. 64 q + 63)."""

    def __init__(self, norb, astr, bstr, h, eri, ecore=0.0):
        self.norb = int(norb)
        a = np.asarray(astr, dtype=np.uint64)
        b = np.asarray(bstr, dtype=np.uint64)
        self.nw = 1 if a.ndim == 1 else int(a.shape[1])
        self.astr = np.ascontiguousarray(a.reshape(len(a), self.nw))
        self.bstr = np.ascontiguousarray(b.reshape(len(b), self.nw))
        self.h = np.ascontiguousarray(h, dtype=np.float64)
        self.eri = np.ascontiguousarray(eri, dtype=np.float64)
        self.ecore = float(ecore)
        if not _ascending(self.astr):
            raise ValueError("alpha strings must be strictly ascending")
        if not _ascending(self.bstr):
            raise ValueError("beta strings must be strictly ascending")

    @classmethod
    def from_problem(cls, prob):
        return cls(prob.norb, prob.astr, prob.bstr, prob.ints.h, prob.ints.eri, prob.ints.ecore)

    @property
    def na(self):
        return len(self.astr)

    @property
    def nb(self):
        return len(self.bstr)

    @property
    def dim(self):
        return self.na * self.nb

    def _args(self):
        return (self.norb, self.nw, _p(self.astr), self.na, _p(self.bstr), self.nb,
                _p(self.h), _p(self.eri), ctypes.c_double(self.ecore))

    def sigma(self, c: np.ndarray, mask: int = ALL) -> np.ndarray:
        c = np.ascontiguousarray(c, dtype=np.float64)
        assert c.shape == (self.dim,)
        out = np.zeros(self.dim)
        rc = lib().oracle_sigma(*self._args(), _p(c), _p(out), ctypes.c_uint(mask))
        if rc:
            raise RuntimeError(f"oracle_sigma failed ({rc})")
        return out

    def sigma_rows(self, c: np.ndarray, rows: np.ndarray, mask: int = ALL) -> np.ndarray:
        c = np.ascontiguousarray(c, dtype=np.float64)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros(len(rows))
        rc = lib().oracle_sigma_rows(*self._args(), _p(c), _p(rows), len(rows), _p(out),
                                     ctypes.c_uint(mask))
        if rc:
            raise RuntimeError(f"oracle_sigma_rows failed ({rc})")
        return out

    def diag(self) -> np.ndarray:
        out = np.zeros(self.dim)
        rc = lib().oracle_diag(*self._args(), _p(out))
        if rc:
            raise RuntimeError("oracle_diag failed")
        return out

    def dense(self) -> np.ndarray:
        if self.dim > 30000:
            raise ValueError("dense H only for small spaces")
        H = np.zeros((self.dim, self.dim))
        rc = lib().oracle_dense(*self._args(), _p(H))
        if rc:
            raise RuntimeError("oracle_dense failed")
        return H

    def h_elem(self, ia, ib, ja, jb) -> float:
        return lib().oracle_h_elem(*self._args(), ia, ib, ja, jb)

    def rdm(self, c: np.ndarray):
        """(gamma, Gamma) spin-summed: gamma[p,q] = sum_s <a+_ps a_qs>,
        Gamma[p,q,r,s] = sum_st <a+_ps a+_rt a_st a_qs>."""
        c = np.ascontiguousarray(c, dtype=np.float64)
        n = self.norb
        g1 = np.zeros((n, n))
        g2 = np.zeros((n, n, n, n))
        rc = lib().oracle_rdm(self.norb, self.nw, _p(self.astr), self.na, _p(self.bstr), self.nb,
                              _p(c), _p(g1), _p(g2))
        if rc:
            raise RuntimeError("oracle_rdm failed")
        return g1, g2

    def energy_from_rdm(self, g1, g2) -> float:
        return self.ecore + float(np.sum(self.h * g1)) + 0.5 * float(np.sum(self.eri * g2))


class MemoisedH:
    """H of a Space evaluated once (by the same definition-based elements) and
    kept as CSR, for repeated products on spaces too large for the matrix-free
    oracle to revisit hundreds of times."""

    def __init__(self, space: "Space"):
        dim = space.dim
        self.dim = dim
        self.rowptr = np.zeros(dim + 1, dtype=np.int64)
        rc = lib().oracle_csr_count(space.norb, space.nw, _p(space.astr), space.na, _p(space.bstr), space.nb,
                                    _p(self.rowptr))
        if rc:
            raise RuntimeError("oracle_csr_count failed")
        nnz = int(self.rowptr[-1])
        self.cols = np.empty(nnz, dtype=np.int32)
        self.vals = np.empty(nnz, dtype=np.float64)
        rc = lib().oracle_csr_fill(space.norb, space.nw, _p(space.astr), space.na, _p(space.bstr), space.nb,
                                   _p(space.h), _p(space.eri), ctypes.c_double(space.ecore),
                                   _p(self.rowptr), _p(self.cols), _p(self.vals))
        if rc:
            raise RuntimeError(f"oracle_csr_fill failed ({rc})")

    @property
    def nnz(self):
        return int(self.rowptr[-1])

    def matvec(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.dim)
        lib().oracle_csr_matvec(self.dim, _p(self.rowptr), _p(self.cols), _p(self.vals), _p(x), _p(y))
        return y


def num_threads() -> int:
    return int(lib().oracle_num_threads())
