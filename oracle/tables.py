"""Per-string excitation lists built with Python sets and dicts (test
infrastructure only).

For every string s of a sorted set (Sec. V-A: flattened per-string excitation
lists, offset + entries), list the in-set strings t reachable by

  * a single excitation  t = a+_a a_i s           (i in s, a not in s),
  * a double excitation  t = a+_a a+_b a_j a_i s  (i < j in s, a < b not in s),

with the sign s_t = <t| op |s> obtained by applying the ladder operators one
at a time (each contributes (-1)^(occupied orbitals below it)).

Canonical order: rows by source index; inside a row, entries by target index
ascending.  Entry packing (uint64; orbitals in 7-bit fields, norb <= 128):

  singles: bits 0-31 target | 32-38 i | 39-45 a | bit 63 sign (1 = negative)
  doubles: bits 0-31 target | 32-38 i | 39-45 j | 46-52 a | 53-59 b | bit 63 sign

Strings are Python integers (bit p = orbital p); a numpy array of shape
(n, nw) holds string k as words [k, 0], [k, 1], ... (word q = orbitals
64 q .. 64 q + 63).
"""
from __future__ import annotations

from itertools import combinations
from typing import Tuple

import numpy as np


def _apply(string: int, ops) -> Tuple[int, int]:
    """Apply ladder operators right to left.  ops is a list of (kind, orbital)
    in the order they act ('a' annihilate, 'c' create).  Returns (sign, result)
    or (0, None) if the result vanishes."""
    sign = 1
    s = int(string)
    for kind, k in ops:
        below = bin(s & ((1 << k) - 1)).count("1")
        occupied = (s >> k) & 1
        if kind == "a":
            if not occupied:
                return 0, None
            s &= ~(1 << k)
        else:
            if occupied:
                return 0, None
            s |= 1 << k
        if below % 2:
            sign = -sign
    return sign, s


def pack_single(target, i, a, sign):
    v = int(target) | (int(i) << 32) | (int(a) << 39)
    if sign < 0:
        v |= 1 << 63
    return v


def pack_double(target, i, j, a, b, sign):
    v = int(target) | (int(i) << 32) | (int(j) << 39) | (int(a) << 46) | (int(b) << 53)
    if sign < 0:
        v |= 1 << 63
    return v


def as_ints(strings) -> list:
    """Strings as Python integers, from shape (n,) or (n, nw) uint64 arrays."""
    a = np.asarray(strings, dtype=np.uint64)
    if a.ndim == 1:
        return [int(x) for x in a]
    return [sum(int(w) << (64 * q) for q, w in enumerate(row)) for row in a]


def build_tables(strings: np.ndarray, norb: int):
    """Return (s_off, s_ent, d_off, d_ent): CSR offsets (int64) and packed
    uint64 entries for singles and doubles, canonical order."""
    strs = as_ints(strings)
    index = {s: k for k, s in enumerate(strs)}
    s_rows, d_rows = [], []
    for s in strs:
        occ = [k for k in range(norb) if (s >> k) & 1]
        vir = [k for k in range(norb) if not (s >> k) & 1]
        singles = []
        for i in occ:
            for a in vir:
                sign, t = _apply(s, [("a", i), ("c", a)])
                if t in index:
                    singles.append((index[t], pack_single(index[t], i, a, sign)))
        doubles = []
        for i, j in combinations(occ, 2):
            for a, b in combinations(vir, 2):
                sign, t = _apply(s, [("a", i), ("a", j), ("c", b), ("c", a)])
                if t in index:
                    doubles.append((index[t], pack_double(index[t], i, j, a, b, sign)))
        s_rows.append([e for _, e in sorted(singles)])
        d_rows.append([e for _, e in sorted(doubles)])

    def csr(rows):
        off = np.zeros(len(rows) + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(r) for r in rows])
        ent = np.array([e for r in rows for e in r], dtype=np.uint64)
        return off, ent

    so, se = csr(s_rows)
    do, de = csr(d_rows)
    return so, se, do, de


def unpack(entry: int, kind: str):
    e = int(entry)
    target = e & 0xFFFFFFFF
    sign = -1 if (e >> 63) & 1 else 1
    if kind == "single":
        return target, (e >> 32) & 127, (e >> 39) & 127, sign
    return target, (e >> 32) & 127, (e >> 39) & 127, (e >> 46) & 127, (e >> 53) & 127, sign
