"""Python binding of libsqd: argument marshalling only.

Every computation happens in the HIP library behind the C ABI declared in
``include/sqd.h``; this module converts numpy / torch objects to pointers and
sizes, and raises on error codes.  PyTorch supplies device memory and the
stream.  If the compiled library is missing the import of any entry point
fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsqd.so")

SQD_OK, SQD_NOT_CONVERGED = 0, 1
TERM_DIAG, TERM_AA, TERM_BB, TERM_AB, TERM_ALL = 1, 2, 4, 8, 15
FP64, FP32 = 0, 1
AB_AUTO, AB_DIRECT, AB_KH = 0, 1, 2
DAV_FP64, DAV_MIXED = 0, 1
PRODUCT_MATRIX_FREE, PRODUCT_STORED = 0, 1
SINGLES, DOUBLES = 0, 1
(TUNE_SS_ROWS, TUNE_AB_CHUNK, TUNE_AB_WAVES, TUNE_SS_WAVES, TUNE_AB_PATH, TUNE_KH_TILE, TUNE_AB_VARIANT,
 TUNE_AB_GROUP, TUNE_SS_WINDOW) = range(9)
MMAX, HIST = 32, 512

ERRORS = {
    -1: "SQD_E_INVALID_ARG", -2: "SQD_E_UNSORTED", -3: "SQD_E_POPCOUNT", -4: "SQD_E_NORB",
    -5: "SQD_E_ASYMMETRIC", -6: "SQD_E_OOM", -7: "SQD_E_HIP", -8: "SQD_E_STATE", -9: "SQD_E_LIMIT",
}


class SQDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class SpaceInfo(ctypes.Structure):
    _fields_ = [("norb", ctypes.c_int), ("nalpha", ctypes.c_int), ("nbeta", ctypes.c_int),
                ("na", ctypes.c_int64), ("nb", ctypes.c_int64), ("dim", ctypes.c_int64),
                ("nnz_single", ctypes.c_int64 * 2), ("nnz_double", ctypes.c_int64 * 2),
                ("conn_per_sigma", ctypes.c_int64), ("conn_terms", ctypes.c_int64 * 4),
                ("device_bytes", ctypes.c_int64), ("kh_columns", ctypes.c_int64)]


class DavidsonOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("m_max", ctypes.c_int),
                ("mode", ctypes.c_int), ("switch_tol", ctypes.c_double), ("ab_path", ctypes.c_int),
                ("guess_noise_dev", ctypes.c_void_p), ("guess_dev", ctypes.c_void_p),
                ("check_every", ctypes.c_int), ("product", ctypes.c_int)]


class Report(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("iterations_fp32", ctypes.c_int),
                ("switch_iter", ctypes.c_int), ("converged", ctypes.c_int), ("status", ctypes.c_int),
                ("nhist", ctypes.c_int), ("energy", ctypes.c_double), ("residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("residual_history", ctypes.c_double * HIST),
                ("energy_history", ctypes.c_double * HIST), ("products", ctypes.c_int)]

    def as_dict(self):
        n = min(self.nhist, HIST)
        return {"iterations": self.iterations, "iterations_fp32": self.iterations_fp32,
                "switch_iter": self.switch_iter, "converged": bool(self.converged),
                "status": self.status, "energy": self.energy, "residual": self.residual,
                "seconds": self.seconds,
                "products": self.products,
                "residual_history": list(self.residual_history[:n]),
                "energy_history": list(self.energy_history[:n])}


_lib = None

EXPORTS = [
    "sqd_version", "sqd_create", "sqd_destroy", "sqd_last_error", "sqd_synchronize", "sqd_set_tuning",
    "sqd_get_tuning", "sqd_set_hamiltonian", "sqd_build_space", "sqd_space_free", "sqd_space_info",
    "sqd_get_tables", "sqd_diag", "sqd_sigma", "sqd_davidson_default_opts", "sqd_davidson",
    "sqd_davidson_batched", "sqd_rdm", "sqd_profile", "sqd_profile_report", "sqd_release_workspace",
    "sqd_davidson_roots", "sqd_sigma_noalloc", "sqd_store_hamiltonian", "sqd_release_hamiltonian", "sqd_spmv",
    "sqd_get_stored_hamiltonian", "sqd_davidson_block", "sqd_build_space_words",
]


def lib():
    """Load libsqd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsqd.so not built at {LIB_PATH}; run python -m paper_2601_16169_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, i64, u32, c_int, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint, ctypes.c_int, ctypes.c_double
    L.sqd_version.restype = ctypes.c_char_p
    L.sqd_create.argtypes = [c_int, P, ctypes.POINTER(P)]
    L.sqd_destroy.argtypes = [P]
    L.sqd_destroy.restype = None
    L.sqd_last_error.argtypes = [P]
    L.sqd_last_error.restype = ctypes.c_char_p
    L.sqd_synchronize.argtypes = [P]
    L.sqd_set_tuning.argtypes = [P, c_int, c_int]
    L.sqd_get_tuning.argtypes = [P, c_int, ctypes.POINTER(c_int)]
    L.sqd_set_hamiltonian.argtypes = [P, c_int, P, P, d]
    L.sqd_build_space.argtypes = [P, c_int, c_int, P, i64, P, i64, ctypes.POINTER(P)]
    L.sqd_build_space_words.argtypes = [P, c_int, c_int, c_int, P, i64, P, i64, ctypes.POINTER(P)]
    L.sqd_space_free.argtypes = [P]
    L.sqd_space_free.restype = None
    L.sqd_space_info.argtypes = [P, ctypes.POINTER(SpaceInfo)]
    L.sqd_get_tables.argtypes = [P, c_int, c_int, P, P]
    L.sqd_diag.argtypes = [P, P, P]
    L.sqd_sigma.argtypes = [P, P, P, P, c_int, u32, c_int]
    L.sqd_sigma_noalloc.argtypes = [P, P, P, P, c_int, u32]
    L.sqd_store_hamiltonian.argtypes = [P, P, ctypes.POINTER(i64)]
    L.sqd_release_hamiltonian.argtypes = [P, P]
    L.sqd_spmv.argtypes = [P, P, P, P]
    L.sqd_get_stored_hamiltonian.argtypes = [P, P, P, P]
    L.sqd_davidson_default_opts.argtypes = [ctypes.POINTER(DavidsonOpts)]
    L.sqd_davidson_default_opts.restype = None
    L.sqd_davidson.argtypes = [P, P, ctypes.POINTER(DavidsonOpts), ctypes.POINTER(d), P,
                               ctypes.POINTER(Report)]
    L.sqd_davidson_batched.argtypes = [P, c_int, ctypes.POINTER(P), ctypes.POINTER(DavidsonOpts),
                                       ctypes.POINTER(d), ctypes.POINTER(P), ctypes.POINTER(Report)]
    L.sqd_rdm.argtypes = [P, P, P, P, P]
    L.sqd_profile.argtypes = [P, c_int]
    L.sqd_release_workspace.argtypes = [P]
    L.sqd_davidson_roots.argtypes = [P, P, P, c_int, P, P, P]
    L.sqd_davidson_block.argtypes = [P, P, P, c_int, P, P, P]
    L.sqd_profile_report.argtypes = [P, ctypes.c_char_p, c_int]
    _lib = L
    return L


def _torch():
    import torch
    return torch


def _dev_ptr(t, dtype_name="float64", numel=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device (cuda/hip) torch tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"expected {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A libsqd context bound to one device and one stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self._spaces = weakref.WeakSet()
        self._h = ctypes.c_void_p()
        rc = lib().sqd_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(self._h))
        if rc != 0:
            raise SQDError(rc, "sqd_create failed")
        self.norb = None

    def _check(self, rc: int, what: str) -> int:
        if rc < 0:
            msg = lib().sqd_last_error(self._h).decode()
            raise SQDError(rc, f"{what}: {msg}")
        return rc

    def close(self):
        """Free every space still open on this context, then the context."""
        if self._h:
            for sp in list(self._spaces):
                sp.close()
            lib().sqd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def synchronize(self):
        self._check(lib().sqd_synchronize(self._h), "sqd_synchronize")

    def release_workspace(self):
        """Free the device workspaces kept between calls (product, Davidson
        and batched-solver scratch)."""
        self._check(lib().sqd_release_workspace(self._h), "sqd_release_workspace")

    def profile(self, enable: bool = True):
        """Start/stop per-kernel HIP-event timers on this context's stream."""
        self._check(lib().sqd_profile(self._h, 1 if enable else 0), "sqd_profile")

    def profile_report(self) -> dict:
        """{kernel name: (calls, total ms)} since the last report."""
        buf = ctypes.create_string_buffer(1 << 16)
        self._check(lib().sqd_profile_report(self._h, buf, len(buf)), "sqd_profile_report")
        out = {}
        for line in buf.value.decode().splitlines():
            name, calls, ms = line.rsplit(" ", 2)
            out[name] = (int(calls), float(ms))
        return out

    def set_tuning(self, key: int, value: int):
        self._check(lib().sqd_set_tuning(self._h, key, value), "sqd_set_tuning")

    def get_tuning(self, key: int) -> int:
        v = ctypes.c_int()
        self._check(lib().sqd_get_tuning(self._h, key, ctypes.byref(v)), "sqd_get_tuning")
        return v.value

    def set_hamiltonian(self, h, eri, ecore: float = 0.0):
        h = np.ascontiguousarray(np.asarray(h, dtype=np.float64))
        eri = np.ascontiguousarray(np.asarray(eri, dtype=np.float64))
        norb = h.shape[0]
        if h.shape != (norb, norb) or eri.size != norb ** 4:
            raise ValueError("h must be (norb, norb) and eri norb^4")
        self._check(lib().sqd_set_hamiltonian(self._h, norb, h.ctypes.data_as(ctypes.c_void_p),
                                              eri.ctypes.data_as(ctypes.c_void_p), float(ecore)),
                    "sqd_set_hamiltonian")
        self.norb = norb

    def build_space(self, nalpha: int, nbeta: int, astr, bstr) -> "Space":
        """Strings as uint64 arrays of shape (n,) (one word) or (n, nwords)."""
        a = np.ascontiguousarray(np.asarray(astr, dtype=np.uint64))
        b = np.ascontiguousarray(np.asarray(bstr, dtype=np.uint64))
        h = ctypes.c_void_p()
        if a.ndim == 1 and b.ndim == 1:
            self._check(lib().sqd_build_space(self._h, nalpha, nbeta, a.ctypes.data_as(ctypes.c_void_p), len(a),
                                              b.ctypes.data_as(ctypes.c_void_p), len(b), ctypes.byref(h)),
                        "sqd_build_space")
        else:
            if a.ndim != 2 or b.ndim != 2 or a.shape[1] != b.shape[1]:
                raise ValueError("string arrays must both be (n,) or (n, nwords) with the same nwords")
            self._check(lib().sqd_build_space_words(self._h, nalpha, nbeta, int(a.shape[1]),
                                                    a.ctypes.data_as(ctypes.c_void_p), len(a),
                                                    b.ctypes.data_as(ctypes.c_void_p), len(b), ctypes.byref(h)),
                        "sqd_build_space_words")
        return Space(self, h, len(a), len(b))

    def davidson_batched(self, spaces: Sequence["Space"], tol=1e-8, max_iter=200, m_max=24, mode=DAV_FP64,
                         switch_tol=1e-4, ab_path=AB_AUTO, noises=None, check_every=4):
        torch = _torch()
        n = len(spaces)
        vecs = [torch.empty(s.dim, dtype=torch.float64, device=f"cuda:{self.device}") for s in spaces]
        energies = (ctypes.c_double * n)()
        reps = (Report * n)()
        sp_arr = (ctypes.c_void_p * n)(*[s._h.value for s in spaces])
        v_arr = (ctypes.c_void_p * n)(*[v.data_ptr() for v in vecs])
        o = _opts(tol, max_iter, m_max, mode, switch_tol, ab_path, None, None, check_every)
        keep = []
        if noises is not None:
            raise ValueError("batched solves take no guess noise")
        rc = self._check(lib().sqd_davidson_batched(self._h, n, sp_arr, ctypes.byref(o), energies, v_arr, reps),
                         "sqd_davidson_batched")
        return [energies[k] for k in range(n)], vecs, [reps[k].as_dict() for k in range(n)], rc


def _opts(tol, max_iter, m_max, mode, switch_tol, ab_path, noise_ptr, guess_ptr, check_every,
          product=PRODUCT_MATRIX_FREE):
    o = DavidsonOpts()
    lib().sqd_davidson_default_opts(ctypes.byref(o))
    o.product = int(product)
    o.tol, o.max_iter, o.m_max, o.mode = float(tol), int(max_iter), int(m_max), int(mode)
    o.switch_tol, o.ab_path, o.check_every = float(switch_tol), int(ab_path), int(check_every)
    o.guess_noise_dev = noise_ptr
    o.guess_dev = guess_ptr
    return o


class Space:
    """Strings and excitation tables of one product space on a context."""

    def __init__(self, ctx: Context, handle, na: int, nb: int):
        self.ctx = ctx
        self._h = handle
        self.na, self.nb = na, nb
        self.dim = na * nb
        ctx._spaces.add(self)

    def close(self):
        if self._h:
            # after the context was destroyed the space is an orphan and this
            # frees only its host record
            lib().sqd_space_free(self._h)
            self._h = ctypes.c_void_p()
            self.ctx._spaces.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _dev(self):
        return f"cuda:{self.ctx.device}"

    def info(self) -> dict:
        i = SpaceInfo()
        self.ctx._check(lib().sqd_space_info(self._h, ctypes.byref(i)), "sqd_space_info")
        return {"norb": i.norb, "nalpha": i.nalpha, "nbeta": i.nbeta, "na": i.na, "nb": i.nb, "dim": i.dim,
                "nnz_single": list(i.nnz_single), "nnz_double": list(i.nnz_double),
                "conn_per_sigma": i.conn_per_sigma, "conn_terms": list(i.conn_terms),
                "device_bytes": i.device_bytes, "kh_columns": i.kh_columns}

    def tables(self, spin: int, kind: int):
        n = self.na if spin == 0 else self.nb
        off = np.zeros(n + 1, dtype=np.int64)
        info = self.info()
        nnz = (info["nnz_single"] if kind == SINGLES else info["nnz_double"])[spin]
        ent = np.zeros(max(nnz, 1), dtype=np.uint64)
        self.ctx._check(lib().sqd_get_tables(self._h, spin, kind, off.ctypes.data_as(ctypes.c_void_p),
                                             ent.ctypes.data_as(ctypes.c_void_p)), "sqd_get_tables")
        return off, ent[:nnz]

    def diag(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self.dim, dtype=torch.float64, device=self._dev)
        self.ctx._check(lib().sqd_diag(self.ctx._h, self._h, _dev_ptr(out, numel=self.dim)), "sqd_diag")
        return out

    def sigma(self, c, out=None, precision=FP64, terms=TERM_ALL, ab_path=AB_AUTO):
        torch = _torch()
        if out is None:
            out = torch.empty(self.dim, dtype=torch.float64, device=self._dev)
        self.ctx._check(lib().sqd_sigma(self.ctx._h, self._h, _dev_ptr(c, numel=self.dim),
                                        _dev_ptr(out, numel=self.dim), int(precision), int(terms), int(ab_path)),
                        "sqd_sigma")
        return out

    def sigma_noalloc(self, c, out, precision=FP64, terms=TERM_ALL):
        """sigma into a caller-allocated `out` through sqd_sigma_noalloc (no
        device allocation: the library's static scratch)."""
        self.ctx._check(lib().sqd_sigma_noalloc(self.ctx._h, self._h, _dev_ptr(c, numel=self.dim),
                                                _dev_ptr(out, numel=self.dim), int(precision), int(terms)),
                        "sqd_sigma_noalloc")
        return out

    def store_hamiltonian(self) -> int:
        """Build the stored H (CSR on the device); returns its element count."""
        nnz = ctypes.c_int64()
        self.ctx._check(lib().sqd_store_hamiltonian(self.ctx._h, self._h, ctypes.byref(nnz)),
                        "sqd_store_hamiltonian")
        return nnz.value

    def release_hamiltonian(self):
        self.ctx._check(lib().sqd_release_hamiltonian(self.ctx._h, self._h), "sqd_release_hamiltonian")

    def spmv(self, c, out=None):
        """sigma = H c from the stored H."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.dim, dtype=torch.float64, device=self._dev)
        self.ctx._check(lib().sqd_spmv(self.ctx._h, self._h, _dev_ptr(c, numel=self.dim),
                                       _dev_ptr(out, numel=self.dim)), "sqd_spmv")
        return out

    def stored_hamiltonian(self, nnz: int):
        """Host copy (rowptr, cols, vals) of the stored H of nnz elements."""
        rp = np.zeros(self.dim + 1, dtype=np.int64)
        cols = np.zeros(max(nnz, 1), dtype=np.int32)
        vals = np.zeros(max(nnz, 1), dtype=np.float64)
        self.ctx._check(lib().sqd_get_stored_hamiltonian(self._h, rp.ctypes.data_as(ctypes.c_void_p),
                                                         cols.ctypes.data_as(ctypes.c_void_p),
                                                         vals.ctypes.data_as(ctypes.c_void_p)),
                        "sqd_get_stored_hamiltonian")
        return rp, cols[:nnz], vals[:nnz]

    def davidson(self, tol=1e-8, max_iter=200, m_max=24, mode=DAV_FP64, switch_tol=1e-4, ab_path=AB_AUTO,
                 noise=None, guess=None, check_every=4, out=None, product=PRODUCT_MATRIX_FREE):
        torch = _torch()
        if out is None:
            out = torch.empty(self.dim, dtype=torch.float64, device=self._dev)
        np_ = _dev_ptr(noise, numel=self.dim) if noise is not None else None
        gp = _dev_ptr(guess, numel=self.dim) if guess is not None else None
        o = _opts(tol, max_iter, m_max, mode, switch_tol, ab_path, np_, gp, check_every, product)
        e = ctypes.c_double()
        rep = Report()
        rc = self.ctx._check(lib().sqd_davidson(self.ctx._h, self._h, ctypes.byref(o), ctypes.byref(e),
                                                _dev_ptr(out, numel=self.dim), ctypes.byref(rep)), "sqd_davidson")
        r = rep.as_dict()
        r["status_code"] = rc
        return e.value, out, r

    def davidson_roots(self, nroots, tol=1e-8, max_iter=200, m_max=24, mode=DAV_FP64, switch_tol=1e-4,
                       ab_path=AB_AUTO, noise=None, check_every=4):
        """The nroots lowest eigenpairs: (energies, vectors (nroots x dim), reports)."""
        torch = _torch()
        vecs = torch.empty((nroots, self.dim), dtype=torch.float64, device=self._dev)
        np_ = _dev_ptr(noise, numel=self.dim) if noise is not None else None
        o = _opts(tol, max_iter, m_max, mode, switch_tol, ab_path, np_, None, check_every)
        e = (ctypes.c_double * nroots)()
        reps = (Report * nroots)()
        rc = self.ctx._check(lib().sqd_davidson_roots(self.ctx._h, self._h, ctypes.byref(o), nroots, e,
                                                      _dev_ptr(vecs, numel=nroots * self.dim), reps),
                             "sqd_davidson_roots")
        out = [r.as_dict() for r in reps]
        for r in out:
            r["status_code"] = rc
        return list(e), vecs, out

    def davidson_block(self, nroots, tol=1e-8, max_iter=200, m_max=24, mode=DAV_FP64, switch_tol=1e-4,
                       ab_path=AB_AUTO, product=PRODUCT_MATRIX_FREE):
        """The nroots lowest eigenpairs by block Davidson: (energies, vectors
        (nroots x dim), reports)."""
        torch = _torch()
        vecs = torch.empty((nroots, self.dim), dtype=torch.float64, device=self._dev)
        o = _opts(tol, max_iter, m_max, mode, switch_tol, ab_path, None, None, 1, product)
        e = (ctypes.c_double * nroots)()
        reps = (Report * nroots)()
        rc = self.ctx._check(lib().sqd_davidson_block(self.ctx._h, self._h, ctypes.byref(o), nroots, e,
                                                      _dev_ptr(vecs, numel=nroots * self.dim), reps),
                             "sqd_davidson_block")
        out = [r.as_dict() for r in reps]
        for r in out:
            r["status_code"] = rc
        return list(e), vecs, out

    def rdm(self, c, two_body=True):
        torch = _torch()
        n = self.ctx.norb
        g1 = torch.empty((n, n), dtype=torch.float64, device=self._dev)
        g2 = torch.empty((n, n, n, n), dtype=torch.float64, device=self._dev) if two_body else None
        self.ctx._check(lib().sqd_rdm(self.ctx._h, self._h, _dev_ptr(c, numel=self.dim), _dev_ptr(g1),
                                      _dev_ptr(g2) if two_body else None), "sqd_rdm")
        return g1, g2
