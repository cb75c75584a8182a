"""Plain FP64 CPU oracle for the M-scheme CI Hamiltonian (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg use this package; the product library never imports it, and it
imports nothing from the product library.

The C core (``ci_oracle.c``) is the plain definition written out: the basis is
enumerated, and each stored entry of a row is found by testing every column
``j >= i`` and evaluated with the Slater-Condon rules (paper Sec. 2: only half
of the symmetric matrix is generated and stored; Sec. 4.1: nonzeros are
located, counted and calculated and stored in compressed-row form; elements are
linear combinations of one-body and two-body interaction terms).
``brute.py`` applies the second-quantized operator directly on tiny bases and
``dimcount.py`` counts the basis by a generating function; both pin the C core.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ci_oracle.c")
_LIB = os.path.join(_HERE, "_ci_oracle.so")
_lib = None

HW_MEV = 15.0


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP over rows)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    L = ctypes.CDLL(_LIB)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.orc_new.restype = vp
    L.orc_new.argtypes = [i32, i32, i32, i32, i32, dbl, i32]
    L.orc_free.argtypes = [vp]
    L.orc_info.argtypes = [vp, vp]
    L.orc_orbits.argtypes = [vp, vp]
    L.orc_keys.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.orc_species.argtypes = [vp, vp, vp]
    L.orc_states.argtypes = [vp, vp]
    L.orc_tbme_keys.argtypes = [vp, vp]
    L.orc_set_tbme.argtypes = [vp, vp]
    L.orc_vget.restype = dbl
    L.orc_vget.argtypes = [vp, i32, i32, i32, i32]
    L.orc_row_counts.argtypes = [vp, vp, i64, vp]
    L.orc_rows.argtypes = [vp, vp, i64, vp, vp, vp]
    L.orc_row_counts_full.argtypes = [vp, vp, i64, vp]
    L.orc_rows_full.argtypes = [vp, vp, i64, vp, vp, vp]
    L.orc_element.restype = dbl
    L.orc_element.argtypes = [vp, i64, i64]
    L.orc_grad_rows.argtypes = [vp, vp, i64, vp, vp]
    L.orc_set_v3.argtypes = [vp, i32, ctypes.c_uint64, dbl]
    L.orc_set_threads.argtypes = [i32]
    L.orc_max_threads.restype = i32
    L.orc_v3.restype = dbl
    L.orc_v3.argtypes = [vp, i32, i32, i32, i32, i32, i32]
    L.orc_row_counts3.argtypes = [vp, vp, i64, vp]
    L.orc_rows3.argtypes = [vp, vp, i64, vp, vp, vp]
    L.orc_element3.restype = dbl
    L.orc_element3.argtypes = [vp, i64, i64]
    L.orc_row_counts3_full.argtypes = [vp, vp, i64, vp]
    L.orc_rows3_full.argtypes = [vp, vp, i64, vp, vp, vp]
    _lib = L
    return L


def set_threads(n: int) -> None:
    """OpenMP threads of the row-parallel oracle functions."""
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Problem:
    Z: int
    N: int
    nmax: int
    two_m: int
    parity: int = 1
    hw: float = HW_MEV
    kinetic: int = 0  # 1: off-diagonal harmonic-oscillator kinetic elements in the one-body term

    def astuple(self):
        return (self.Z, self.N, self.nmax, self.two_m, self.parity)


class Oracle:
    """One basis + two-body table, FP64.  Rows are computed on demand."""

    def __init__(self, prob: Problem):
        self.prob = prob
        L = _load()
        h = L.orc_new(prob.Z, prob.N, prob.nmax, prob.two_m, prob.parity, float(prob.hw), int(prob.kinetic))
        if not h:
            raise ValueError("invalid problem %r" % (prob,))
        self._h = ctypes.c_void_p(h)
        info = np.zeros(16, np.int64)
        L.orc_info(self._h, _ptr(info))
        (self.shell_max, self.n_sps, self.n_words, self.n0, self.n_pkeys, self.n_nkeys,
         self.n_blocks, self.n_psd, self.n_nsd, self.dim, self.n_tbme) = [int(x) for x in info[:11]]
        self._V = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                _load().orc_free(self._h)
                self._h = None
        except Exception:
            pass

    # ---- structure -------------------------------------------------------
    def orbits(self) -> np.ndarray:
        """[n_sps, 5] int32: N, n, l, 2j, 2m (order N, l, 2j, 2m ascending)."""
        o = np.zeros((self.n_sps, 5), np.int32)
        _load().orc_orbits(self._h, _ptr(o))
        return o

    def keys(self):
        pk = np.zeros((self.n_pkeys, 2), np.int32)
        nk = np.zeros((self.n_nkeys, 2), np.int32)
        pko = np.zeros(self.n_pkeys + 1, np.int64)
        nko = np.zeros(self.n_nkeys + 1, np.int64)
        blk = np.zeros((self.n_blocks, 2), np.int32)
        bo = np.zeros(self.n_blocks + 1, np.int64)
        _load().orc_keys(self._h, _ptr(pk), _ptr(nk), _ptr(pko), _ptr(nko), _ptr(blk), _ptr(bo))
        return dict(pkeys=pk, nkeys=nk, pkey_off=pko, nkey_off=nko, blocks=blk, block_off=bo)

    def species(self):
        p = np.zeros((self.n_psd, self.n_words), np.uint64)
        n = np.zeros((self.n_nsd, self.n_words), np.uint64)
        _load().orc_species(self._h, _ptr(p), _ptr(n))
        return p, n

    def states(self) -> np.ndarray:
        """[D, 2W] uint64: proton words then neutron words of every basis state."""
        s = np.zeros((self.dim, 2 * self.n_words), np.uint64)
        _load().orc_states(self._h, _ptr(s))
        return s

    def tbme_keys(self) -> np.ndarray:
        k = np.zeros((self.n_tbme, 4), np.int32)
        _load().orc_tbme_keys(self._h, _ptr(k))
        return k

    # ---- values ----------------------------------------------------------
    def set_tbme(self, v) -> None:
        if v is None:
            _load().orc_set_tbme(self._h, None)
            self._V = None
            return
        v = np.ascontiguousarray(v, dtype=np.float64)
        if v.shape != (self.n_tbme,):
            raise ValueError("expected %d two-body values, got %s" % (self.n_tbme, v.shape))
        _load().orc_set_tbme(self._h, _ptr(v))
        self._V = v

    def vget(self, a, b, c, d) -> float:
        return _load().orc_vget(self._h, a, b, c, d)

    def row_counts(self, rows) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros(len(rows), np.int64)
        if len(rows):
            _load().orc_row_counts(self._h, _ptr(rows), len(rows), _ptr(out))
        return out

    def rows(self, rows, values: bool = True):
        """(counts, cols int32, vals float64) for the given rows, concatenated."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        counts = self.row_counts(rows)
        offs = np.zeros(len(rows), np.int64)
        if len(rows):
            offs[1:] = np.cumsum(counts)[:-1]
        tot = int(counts.sum())
        cols = np.zeros(max(tot, 1), np.int32)
        vals = np.zeros(max(tot, 1), np.float64) if values else None
        if len(rows):
            _load().orc_rows(self._h, _ptr(rows), len(rows), _ptr(offs), _ptr(cols),
                             _ptr(vals) if values else None)
        return counts, cols[:tot], (vals[:tot] if values else None)

    def rows_full(self, rows, values: bool = True):
        """Like rows(), for the full symmetric matrix (every column of the row)."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        counts = np.zeros(len(rows), np.int64)
        if len(rows):
            _load().orc_row_counts_full(self._h, _ptr(rows), len(rows), _ptr(counts))
        offs = np.zeros(len(rows), np.int64)
        if len(rows):
            offs[1:] = np.cumsum(counts)[:-1]
        tot = int(counts.sum())
        cols = np.zeros(max(tot, 1), np.int32)
        vals = np.zeros(max(tot, 1), np.float64) if values else None
        if len(rows):
            _load().orc_rows_full(self._h, _ptr(rows), len(rows), _ptr(offs), _ptr(cols),
                                  _ptr(vals) if values else None)
        return counts, cols[:tot], (vals[:tot] if values else None)

    # ---- three-body term (d <= 3 structure)
    V3_NONE, V3_SYNTHETIC, V3_IDENTITY = 0, 1, 2

    def set_v3(self, kind: int, seed: int = 0, scale: float = 1.0) -> None:
        """Three-body interaction: none, synthetic (splitmix64 of the triple pair,
        uniform in [-scale, scale)), or identity (scale on equal triples)."""
        _load().orc_set_v3(self._h, int(kind), int(seed) & ((1 << 64) - 1), float(scale))

    def v3(self, a, b, c, d, e, f) -> float:
        return _load().orc_v3(self._h, a, b, c, d, e, f)

    def row_counts3(self, rows) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros(len(rows), np.int64)
        if len(rows):
            _load().orc_row_counts3(self._h, _ptr(rows), len(rows), _ptr(out))
        return out

    def rows3(self, rows, values: bool = True):
        """Like rows(), with the three-body term: columns j >= i with at most
        three nucleons different."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        counts = self.row_counts3(rows)
        offs = np.zeros(len(rows), np.int64)
        if len(rows):
            offs[1:] = np.cumsum(counts)[:-1]
        tot = int(counts.sum())
        cols = np.zeros(max(tot, 1), np.int32)
        vals = np.zeros(max(tot, 1), np.float64) if values else None
        if len(rows):
            _load().orc_rows3(self._h, _ptr(rows), len(rows), _ptr(offs), _ptr(cols),
                              _ptr(vals) if values else None)
        return counts, cols[:tot], (vals[:tot] if values else None)

    def rows3_full(self, rows, values: bool = True):
        """Like rows3(), for the full symmetric matrix (every column of the row)."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        counts = np.zeros(len(rows), np.int64)
        if len(rows):
            _load().orc_row_counts3_full(self._h, _ptr(rows), len(rows), _ptr(counts))
        offs = np.zeros(len(rows), np.int64)
        if len(rows):
            offs[1:] = np.cumsum(counts)[:-1]
        tot = int(counts.sum())
        cols = np.zeros(max(tot, 1), np.int32)
        vals = np.zeros(max(tot, 1), np.float64) if values else None
        if len(rows):
            _load().orc_rows3_full(self._h, _ptr(rows), len(rows), _ptr(offs), _ptr(cols),
                                   _ptr(vals) if values else None)
        return counts, cols[:tot], (vals[:tot] if values else None)

    def lowest_eigenpair3(self):
        """Lowest eigenvalue and eigenvector of the matrix with the three-body
        term (numpy's dense symmetric eigensolver)."""
        w, v = np.linalg.eigh(self.dense3())
        return float(w[0]), v[:, 0]

    def element3(self, i: int, j: int) -> float:
        return _load().orc_element3(self._h, int(i), int(j))

    def dense3(self) -> np.ndarray:
        """Dense symmetric H with the three-body term (small bases only)."""
        counts, cols, vals = self.rows3(np.arange(self.dim))
        H = np.zeros((self.dim, self.dim))
        rows = np.repeat(np.arange(self.dim), counts)
        H[rows, cols] = vals
        H[cols, rows] = vals
        return H

    def csr(self, values: bool = True):
        """Full upper-triangle CSR (row_ptr int64[D+1], col int32, val float64)."""
        counts, cols, vals = self.rows(np.arange(self.dim), values)
        rp = np.zeros(self.dim + 1, np.int64)
        rp[1:] = np.cumsum(counts)
        return rp, cols, vals

    def element(self, i: int, j: int) -> float:
        return _load().orc_element(self._h, int(i), int(j))

    def grad_rows(self, rows, G) -> np.ndarray:
        """d/dV of sum_e G_e H_e over the stored entries of `rows` (FP64)."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        G = np.ascontiguousarray(G, dtype=np.float64)
        g = np.zeros(max(self.n_tbme, 1), np.float64)
        _load().orc_grad_rows(self._h, _ptr(rows), len(rows), _ptr(G), _ptr(g))
        return g[: self.n_tbme]

    def lowest_eigenpair(self):
        """Lowest eigenvalue and a unit eigenvector of the full symmetric H:
        the plain definition, numpy's dense symmetric eigensolver on dense()
        (tiny bases only)."""
        w, v = np.linalg.eigh(self.dense())
        return float(w[0]), v[:, 0].copy()

    def hellmann_feynman(self, psi) -> np.ndarray:
        """dE/dV for the eigenvalue E = psi^T H psi of unit eigenvector psi:
        the gradient of the sum over the stored (upper) entries with upstream
        value psi_i psi_j, doubled off the diagonal (each off-diagonal entry
        stands for two matrix elements)."""
        rows = np.arange(self.dim)
        counts, cols, _ = self.rows(rows, values=False)
        ri = np.repeat(rows, counts)
        G = psi[ri] * psi[cols] * np.where(ri == cols, 1.0, 2.0)
        return self.grad_rows(rows, G)

    def dense(self) -> np.ndarray:
        """Full symmetric matrix (tiny bases only)."""
        rp, cols, vals = self.csr()
        H = np.zeros((self.dim, self.dim))
        for i in range(self.dim):
            for k in range(rp[i], rp[i + 1]):
                H[i, cols[k]] = vals[k]
                H[cols[k], i] = vals[k]
        return H
