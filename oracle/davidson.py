"""Textbook Davidson-Liu for the lowest root (test infrastructure only).

The paper names the Davidson algorithm (Sec. I, Sec. VI: one matrix-vector
product per iteration, with vector updates, dot products and Gram-Schmidt
orthogonalisation around it) without fixing its details; this is the plain
textbook form with the readings stated here:

  start   x0 = e_k + noise, k = argmin H_II (lowest index on ties); v0 = x0/|x0|
  loop    G = V^T A V;  (theta, y) = lowest eigenpair of G (numpy.linalg.eigh)
          x = V y;  r = A x - theta x;  stop when |r|_2 <= tol
          if m == m_max: collapse the basis onto the current Ritz vector x
          (V = [x], AV = [A x])
          t_I = r_I / (theta - H_II), a denominator of size < 1e-8 replaced by
          1e-8 with the same sign (+ when it is exactly zero)
          two rounds of classical Gram-Schmidt against V, normalise, append
  result  theta and x normalised with its largest-|x| entry positive
          (lowest index on ties).

The dense route forms H_S explicitly and calls numpy.linalg.eigh.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np


@dataclasses.dataclass
class Result:
    energy: float
    vector: np.ndarray
    iterations: int
    residual: float
    converged: bool
    history: list


def fix_phase(x: np.ndarray) -> np.ndarray:
    k = int(np.argmax(np.abs(x)))
    return -x if x[k] < 0 else x


def precondition(r, theta, diag, floor=1e-8):
    den = theta - diag
    small = np.abs(den) < floor
    den = np.where(small, np.where(den < 0, -floor, floor), den)
    return r / den


def davidson(apply_h: Callable[[np.ndarray], np.ndarray], diag: np.ndarray,
             noise: Optional[np.ndarray] = None, tol: float = 1e-8, m_max: int = 24,
             max_iter: int = 200) -> Result:
    dim = len(diag)
    x0 = np.zeros(dim)
    x0[int(np.argmin(diag))] = 1.0
    if noise is not None:
        x0 = x0 + noise
    V = [x0 / np.linalg.norm(x0)]
    AV = [apply_h(V[0])]
    hist = []
    theta, x, rn = 0.0, V[0], np.inf
    for it in range(1, max_iter + 1):
        Vm = np.array(V)
        AVm = np.array(AV)
        G = Vm @ AVm.T
        G = 0.5 * (G + G.T)
        w, Y = np.linalg.eigh(G)
        theta, y = float(w[0]), Y[:, 0]
        x = y @ Vm
        ax = y @ AVm
        r = ax - theta * x
        rn = float(np.linalg.norm(r))
        hist.append((theta, rn))
        if rn <= tol:
            return Result(theta, fix_phase(x / np.linalg.norm(x)), it, rn, True, hist)
        if len(V) == m_max:
            V, AV = [x], [ax]
            Vm = np.array(V)
        t = precondition(r, theta, diag)
        for _ in range(2):
            t = t - (Vm @ t) @ Vm
        nt = np.linalg.norm(t)
        if nt == 0.0:
            break
        t = t / nt
        V.append(t)
        AV.append(apply_h(t))
    return Result(theta, fix_phase(x / np.linalg.norm(x)), len(hist), rn, False, hist)


def dense_lowest(H: np.ndarray):
    w, U = np.linalg.eigh(H)
    return float(w[0]), fix_phase(U[:, 0]), w
