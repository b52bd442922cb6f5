"""Explicit Hamiltonian matrix elements for the oracle (test infrastructure).

<M_i|H|M_j> (Sec. 2, Eq. for H_ij) from the m-scheme terms of ``interaction``,
computed term by term with Jordan-Wigner signs over the combined
proton-then-neutron state index (C core ``oracle_core.c``). Nothing here uses
the proton x neutron factorisation of App. B; the GPU library does, and this
is what it is checked against.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build
from .basis import ProductBasis
from .interaction import mscheme_terms, one_body

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build()
        _lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        _lib.orc_lines.argtypes = [ctypes.c_int, P, i64, P, P, P, i64, ctypes.c_int, P, P, P, P, P, P,
                                   P, i64, P, P, P, i64, ctypes.c_int]
        _lib.orc_lines.restype = ctypes.c_int
        _lib.orc_apply_rows.argtypes = [P, i64, P, P, P, i64, ctypes.c_int, P, P, P, P, P, P, P, i64,
                                        P, ctypes.c_int, P]
        _lib.orc_apply_rows.restype = ctypes.c_int
        _lib.orc_num_threads.restype = ctypes.c_int
        _lib.orc_row_nnz.argtypes = [P, i64, P, P, P, i64, ctypes.c_int, P, P, P, P, P, P, P, i64, P]
        _lib.orc_row_nnz.restype = ctypes.c_int
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Model:
    """Basis + Hamiltonian of one workload, in the product-basis order of ``basis``."""

    def __init__(self, orbits, n_prot, n_neut, twoM, tbme, spe_p, spe_n, parity=0):
        self.orbits = tuple(orbits)
        self.basis = ProductBasis(orbits, n_prot, n_neut, twoM, parity)
        self.dim = self.basis.dim
        self.S = 2 * self.basis.nstates
        if self.S > 64:
            raise ValueError("oracle handles at most 64 combined single-particle states")
        self.words = self.basis.combined_words_array()
        order = np.argsort(self.words, kind="stable")
        self.sorted = np.ascontiguousarray(self.words[order])
        self.sidx = np.ascontiguousarray(order.astype(np.int64))
        self.e = np.array(one_body(orbits, spe_p, spe_n), dtype=np.float64)
        self.terms = mscheme_terms(orbits, tbme)
        self._prep()

    def with_interaction(self, tbme, spe_p, spe_n):
        """Same basis, another Hamiltonian (H is linear in e and V)."""
        new = object.__new__(Model)
        new.__dict__.update({k: self.__dict__[k] for k in ("basis", "dim", "S", "words", "sorted", "sidx")})
        new.orbits = self.orbits
        new.e = np.array(one_body(self.orbits, spe_p, spe_n), dtype=np.float64)
        new.terms = mscheme_terms(self.orbits, tbme)
        new._prep()
        return new

    def _group(self, key):
        S = self.S
        items = sorted(self.terms.items(), key=lambda kv: key(kv[0]))
        ta = np.array([k[0] for k, _ in items], dtype=np.int32)
        tb = np.array([k[1] for k, _ in items], dtype=np.int32)
        tc = np.array([k[2] for k, _ in items], dtype=np.int32)
        td = np.array([k[3] for k, _ in items], dtype=np.int32)
        th = np.array([v for _, v in items], dtype=np.float64)
        gp = np.array([key(k)[0] * S + key(k)[1] for k, _ in items], dtype=np.int64)
        start = np.searchsorted(gp, np.arange(S * S + 1), side="left").astype(np.int64)
        return ta, tb, tc, td, th, start

    def _prep(self):
        # rows: group by creation pair (a,b); columns: group by annihilation pair (c,d)
        self._rowterms = self._group(lambda k: (k[0], k[1]))
        self._colterms = self._group(lambda k: (k[2], k[3]))
        self.cap = int(max(1, len(self.terms))) + 1

    def _lines(self, idx, mode, merge=1):
        lib = _load()
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        ta, tb, tc, td, th, start = self._rowterms if mode == 0 else self._colterms
        cap_total = max(1, len(idx) * self.cap)
        ptr = np.zeros(len(idx) + 1, dtype=np.int64)
        col = np.zeros(cap_total, dtype=np.int64)
        val = np.zeros(cap_total, dtype=np.float64)
        rc = lib.orc_lines(mode, _ptr(idx), len(idx), _ptr(self.words), _ptr(self.sorted), _ptr(self.sidx),
                           self.dim, self.S, _ptr(self.e), _ptr(ta), _ptr(tb), _ptr(tc), _ptr(td), _ptr(th),
                           _ptr(start), self.cap, _ptr(ptr), _ptr(col), _ptr(val), cap_total, merge)
        if rc != 0:
            raise RuntimeError(f"orc_lines failed ({rc})")
        n = ptr[-1]
        return ptr, col[:n].copy(), val[:n].copy()

    def rows(self, idx):
        """CSR pieces (ptr, col, val) of rows ``idx``: <i|H|j>."""
        return self._lines(idx, 0)

    def rows_generated(self, idx):
        """Rows ``idx`` as the terms that generate them, unmerged (ptr, col, val): the
        single-particle-energy diagonal, then one entry per m-scheme term whose adjoint maps
        basis state i to a basis state. A per-element H.V adds exactly these products, so
        np.diff(ptr) is the number of terms its sum for row i has."""
        return self._lines(idx, 0, merge=0)

    def columns(self, idx):
        """CSR pieces of columns ``idx``: <j|H|i>, built by applying H to |i>."""
        return self._lines(idx, 1)

    def dense(self):
        if self.dim > 6000:
            raise ValueError("dense H only for small spaces")
        ptr, col, val = self.rows(np.arange(self.dim))
        H = np.zeros((self.dim, self.dim))
        for i in range(self.dim):
            H[i, col[ptr[i]:ptr[i + 1]]] = val[ptr[i]:ptr[i + 1]]
        return H

    def csr(self):
        import scipy.sparse as sp
        ptr, col, val = self.rows(np.arange(self.dim))
        return sp.csr_matrix((val, col, ptr), shape=(self.dim, self.dim))

    def apply_rows(self, V, idx):
        """(H V)[idx, :] with V of shape (D, nb), FP64."""
        lib = _load()
        V = np.ascontiguousarray(V, dtype=np.float64)
        if V.ndim == 1:
            V = V[:, None]
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        W = np.zeros((len(idx), V.shape[1]))
        ta, tb, tc, td, th, start = self._rowterms
        rc = lib.orc_apply_rows(_ptr(idx), len(idx), _ptr(self.words), _ptr(self.sorted), _ptr(self.sidx),
                                self.dim, self.S, _ptr(self.e), _ptr(ta), _ptr(tb), _ptr(tc), _ptr(td),
                                _ptr(th), _ptr(start), self.cap, _ptr(V), V.shape[1], _ptr(W))
        if rc != 0:
            raise RuntimeError(f"orc_apply_rows failed ({rc})")
        return W

    def row_nnz(self, idx=None):
        """Non-zero count of each row (all rows by default)."""
        lib = _load()
        idx = np.arange(self.dim) if idx is None else idx
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        out = np.zeros(len(idx), dtype=np.int64)
        ta, tb, tc, td, th, start = self._rowterms
        rc = lib.orc_row_nnz(_ptr(idx), len(idx), _ptr(self.words), _ptr(self.sorted), _ptr(self.sidx), self.dim,
                             self.S, _ptr(self.e), _ptr(ta), _ptr(tb), _ptr(tc), _ptr(td), _ptr(th), _ptr(start),
                             self.cap, _ptr(out))
        if rc != 0:
            raise RuntimeError(f"orc_row_nnz failed ({rc})")
        return out

    def apply(self, V):
        return self.apply_rows(V, np.arange(self.dim))


def threads() -> int:
    return int(_load().orc_num_threads())


def model_from_workload(w, tbme=None, twoM=None):
    tb = w.tbme() if tbme is None else tbme
    return Model(w.orbits, w.n_prot, w.n_neut, w.twoM if twoM is None else twoM, tb, w.spe, w.spe, w.parity)
