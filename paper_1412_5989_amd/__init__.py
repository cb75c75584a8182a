"""MI355X construction of M-scheme CI / No-Core Shell Model Hamiltonians.

Thin Python binding of ``libci.so`` (C ABI in ``include/ci.h``).  Python only
marshals arguments: device memory comes from torch tensors and every step of
the construction runs in the library's HIP kernels.  There is no CPU fallback:
if the library is missing or no GPU is visible, the calls raise.

Entry points (same names as the C ABI):
  ci_basis_plan(problems)                      sizes, host only
  ci_tbme_keys(problem)                        two-body keys in table order, host only
  ci_basis_build(problems) -> Basis            basis indexing (paper Sec. 2)
  ci_hamiltonian_count(basis) -> (row_ptr, nnz)            count pass (Sec. 4.1)
  ci_hamiltonian_fill(basis, tbme, row_ptr) -> (col, val)  fill pass (Sec. 2, 4.1)
  ci_hamiltonian_vjp(basis, row_ptr, grad_val) -> grad_tbme  adjoint
  ci_hamiltonian_fill_keys / ci_hamiltonian_vjp_keys       the same with the structure stored per entry
  CIHamiltonian.apply(tbme, basis, row_ptr, col) -> val      autograd wrapper
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libci.so")

CI_OK, CI_EINVAL, CI_EUNSUPPORTED, CI_ESPACE, CI_EHIP = 0, -1, -2, -3, -4
_ERRNAMES = {CI_EINVAL: "CI_EINVAL", CI_EUNSUPPORTED: "CI_EUNSUPPORTED", CI_ESPACE: "CI_ESPACE",
             CI_EHIP: "CI_EHIP"}

HW_MEV = 15.0


class CIError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_ERRNAMES.get(code, str(code)), msg))
        self.code = code


class ci_problem(ctypes.Structure):
    _fields_ = [("Z", ctypes.c_int32), ("N", ctypes.c_int32), ("nmax", ctypes.c_int32),
                ("two_m", ctypes.c_int32), ("parity", ctypes.c_int32), ("kinetic", ctypes.c_int32),
                ("hw_mev", ctypes.c_double)]


class ci_basis_info(ctypes.Structure):
    _fields_ = [("shell_max", ctypes.c_int32), ("n_sps", ctypes.c_int32), ("n_words", ctypes.c_int32),
                ("n0", ctypes.c_int32), ("n_pkeys", ctypes.c_int32), ("n_nkeys", ctypes.c_int32),
                ("n_blocks", ctypes.c_int32), ("n_sectors", ctypes.c_int32),
                ("n_psd", ctypes.c_int64), ("n_nsd", ctypes.c_int64), ("dim", ctypes.c_int64),
                ("n_tbme", ctypes.c_int64), ("row_ptr_offset", ctypes.c_int64),
                ("tbme_offset", ctypes.c_int64), ("index_bytes", ctypes.c_int64),
                ("arena_bytes", ctypes.c_int64), ("list_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ci_v3(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("seed", ctypes.c_uint64), ("scale", ctypes.c_double)]


CI_V3_NONE, CI_V3_SYNTHETIC, CI_V3_IDENTITY = 0, 1, 2


class ci_tuning(ctypes.Structure):
    _fields_ = [("row_waves", ctypes.c_int32), ("row_grab", ctypes.c_int32), ("adj_rows", ctypes.c_int32),
                ("adj_tile_n", ctypes.c_int32), ("adj_persistent", ctypes.c_int32), ("adjk_rows", ctypes.c_int32),
                ("adjk_tile_n", ctypes.c_int32), ("adjk_persistent", ctypes.c_int32), ("row_xcd", ctypes.c_int32),
                ("adj_wide", ctypes.c_int32), ("adj_flush", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# every symbol include/ci.h declares
EXPORTS = ["ci_last_error", "ci_basis_plan", "ci_tbme_keys", "ci_basis_build", "ci_basis_list_bytes",
           "ci_basis_build_lists", "ci_basis_free",
           "ci_hamiltonian_count", "ci_hamiltonian_fill", "ci_hamiltonian_vjp", "ci_vjp_work_bytes",
           "ci_hamiltonian_fill_keys", "ci_hamiltonian_vjp_keys", "ci_hamiltonian_vjp_noalloc",
           "ci_vjp_noalloc_scratch_bytes",
           "ci_hamiltonian_count_full", "ci_hamiltonian_fill_full", "ci_hamiltonian3_count", "ci_hamiltonian3_fill",
           "ci_hamiltonian3_count_full", "ci_hamiltonian3_fill_full", "ci_hamiltonian_spmv", "ci_lanczos",
           "ci_hamiltonian_spmv_upper", "ci_lanczos_upper", "ci_lanczos_work_bytes",
           "ci_hamiltonian_tune", "ci_basis_get_tuning", "ci_basis_set_tuning", "ci_probe_ceilings",
           "ci_threebody_plan", "ci_threebody_build", "ci_threebody_free", "ci_threebody_info", "ci_threebody_keys",
           "ci_threebody_orbitals", "ci_threebody_decouple", "ci_threebody_work_bytes", "ci_clebsch_gordan",
           "ci_basis_count", "ci_basis_get_info", "ci_basis_states"]

_lib = None


def load_library():
    """Load libci.so (built by ``paper_1412_5989_amd.build``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libci.so is not built (run `python -m paper_1412_5989_amd.build`)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    P = ctypes.POINTER
    L.ci_last_error.restype = ctypes.c_char_p
    L.ci_basis_plan.argtypes = [P(ci_problem), i32, P(ci_basis_info)]
    L.ci_tbme_keys.argtypes = [P(ci_problem), vp, i64]
    L.ci_basis_build.argtypes = [P(ci_problem), i32, P(ci_basis_info), vp, sz, P(vp), vp]
    L.ci_basis_list_bytes.argtypes = [vp, P(sz), vp]
    L.ci_basis_build_lists.argtypes = [vp, vp, sz, vp]
    L.ci_basis_free.argtypes = [vp]
    L.ci_basis_free.restype = None
    L.ci_hamiltonian_count.argtypes = [vp, vp, vp, vp]
    L.ci_hamiltonian_fill.argtypes = [vp, vp, vp, vp, vp, vp]
    L.ci_hamiltonian_vjp.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    L.ci_hamiltonian_fill_keys.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.ci_hamiltonian_vjp_keys.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
    L.ci_hamiltonian_vjp_noalloc.argtypes = [vp, vp, vp, vp, vp]
    L.ci_vjp_noalloc_scratch_bytes.argtypes = []
    L.ci_vjp_noalloc_scratch_bytes.restype = sz
    L.ci_hamiltonian_count_full.argtypes = [vp, vp, vp, vp]
    L.ci_hamiltonian_fill_full.argtypes = [vp, vp, vp, vp, vp, vp]
    L.ci_hamiltonian_spmv.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    L.ci_hamiltonian_spmv_upper.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    L.ci_lanczos.argtypes = [vp, i32, vp, vp, vp, vp, i32, ctypes.c_double, P(ctypes.c_double), P(i32), vp, vp,
                             sz, vp]
    L.ci_lanczos_upper.argtypes = L.ci_lanczos.argtypes
    L.ci_lanczos_work_bytes.argtypes = [i64, i32]
    L.ci_lanczos_work_bytes.restype = sz
    L.ci_hamiltonian_tune.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, i32, vp]
    L.ci_basis_get_tuning.argtypes = [vp, P(ci_tuning)]
    L.ci_basis_set_tuning.argtypes = [vp, P(ci_tuning)]
    L.ci_probe_ceilings.argtypes = [vp, sz, P(ctypes.c_double), P(ctypes.c_double), vp]
    L.ci_threebody_plan.argtypes = [i32, i32, P(i64), P(i32)]
    L.ci_threebody_build.argtypes = [i32, i32, P(vp)]
    L.ci_threebody_free.argtypes = [vp]
    L.ci_threebody_free.restype = None
    L.ci_threebody_info.argtypes = [vp, P(i64), P(i32), P(i32), P(i32)]
    L.ci_threebody_keys.argtypes = [vp, vp, i64]
    L.ci_threebody_orbitals.argtypes = [vp, vp, vp, vp]
    L.ci_threebody_decouple.argtypes = [vp, vp, vp, i64, vp, vp, sz, vp]
    L.ci_hamiltonian3_count.argtypes = [vp, vp, vp, vp]
    L.ci_hamiltonian3_fill.argtypes = [vp, vp, P(ci_v3), vp, vp, vp, vp]
    L.ci_hamiltonian3_count_full.argtypes = [vp, vp, vp, vp]
    L.ci_hamiltonian3_fill_full.argtypes = [vp, vp, P(ci_v3), vp, vp, vp, vp]
    L.ci_clebsch_gordan.argtypes = [i32, i32, i32, i32, i32, i32, P(ctypes.c_double)]
    L.ci_threebody_work_bytes.argtypes = [i64]
    L.ci_threebody_work_bytes.restype = sz
    L.ci_vjp_work_bytes.argtypes = [vp]
    L.ci_vjp_work_bytes.restype = sz
    L.ci_basis_count.argtypes = [vp]
    L.ci_basis_count.restype = i32
    L.ci_basis_get_info.argtypes = [vp, i32, P(ci_basis_info)]
    L.ci_basis_states.argtypes = [vp, i32, vp, vp]
    for name in EXPORTS:
        if name not in ("ci_last_error", "ci_basis_free", "ci_vjp_work_bytes", "ci_basis_count",
                        "ci_vjp_noalloc_scratch_bytes",
                        "ci_lanczos_work_bytes", "ci_threebody_free", "ci_threebody_work_bytes"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != CI_OK:
        raise CIError(rc, load_library().ci_last_error().decode())


def _problems(problems) -> Tuple[ctypes.Array, int]:
    if isinstance(problems, tuple) and problems and isinstance(problems[0], (int, np.integer)):
        problems = [problems]
    ps = list(problems)
    arr = (ci_problem * len(ps))()
    for k, p in enumerate(ps):
        Z, N, nmax, two_m = (int(x) for x in p[:4])
        parity = int(p[4]) if len(p) > 4 else 1
        hw = float(p[5]) if len(p) > 5 else HW_MEV
        kinetic = int(p[6]) if len(p) > 6 else 0
        arr[k] = ci_problem(Z, N, nmax, two_m, parity, kinetic, hw)
    return arr, len(ps)


def ci_basis_plan(problems) -> List[dict]:
    """Sizes of each problem's basis (host only, no device call)."""
    arr, n = _problems(problems)
    info = (ci_basis_info * n)()
    _check(load_library().ci_basis_plan(arr, n, info))
    return [info[k].as_dict() for k in range(n)]


def ci_tbme_keys(problem) -> np.ndarray:
    """[n_tbme, 4] int32 two-body keys (a, b, c, d) in table order (host only)."""
    arr, _ = _problems([problem])
    n = ci_basis_plan([problem])[0]["n_tbme"]
    out = np.zeros((max(n, 1), 4), np.int32)
    _check(load_library().ci_tbme_keys(arr, out.ctypes.data_as(ctypes.c_void_p), n))
    return out[:n]


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: libci runs only on the device (no CPU fallback)")
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Basis:
    """Handle of one or more bases built on the current device.

    The device memory of the handle is two torch tensors owned here: the
    arena of the index tables (size from the build's size query) and the
    partner lists (size from ci_basis_list_bytes); the library allocates no
    device memory.  Both live as long as this object."""

    def __init__(self, problems, stream=None):
        torch = _torch()
        L = load_library()
        arr, n = _problems(problems)
        info = (ci_basis_info * n)()
        sp = _stream_ptr(stream)
        self.device = torch.device("cuda", torch.cuda.current_device())
        _check(L.ci_basis_build(arr, n, info, None, 0, None, sp))  # size query (host only)
        abytes = int(info[0].arena_bytes)
        self._arena = torch.empty(max(abytes, 1), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(L.ci_basis_build(arr, n, info, _ptr(self._arena), abytes, ctypes.byref(h), sp))
        self._h = h
        lb = ctypes.c_size_t()
        _check(L.ci_basis_list_bytes(h, ctypes.byref(lb), sp))
        self._lists = torch.empty(max(int(lb.value), 1), dtype=torch.uint8, device=self.device)
        _check(L.ci_basis_build_lists(h, _ptr(self._lists), int(lb.value), sp))
        for k in range(n):  # index_bytes / list_bytes are known now
            _check(L.ci_basis_get_info(h, k, ctypes.byref(info[k])))
        self.problems = [tuple(int(x) for x in (p.Z, p.N, p.nmax, p.two_m, p.parity)) for p in arr]
        self.info = [info[k].as_dict() for k in range(n)]
        self.n_probs = n
        self.n_rowptr = sum(i["dim"] + 1 for i in self.info)
        self.n_tbme = sum(i["n_tbme"] for i in self.info)
        self.nnz = None  # per basis, after count

    @property
    def handle(self):
        return self._h

    def free(self):
        """Frees the handle (host memory) and drops the tensors of its device
        memory; torch's allocator reuses them in stream order."""
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().ci_basis_free(self._h)
            self._h = None
        self._arena = None
        self._lists = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def vjp_work_bytes(self) -> int:
        return int(load_library().ci_vjp_work_bytes(self._h))

    @property
    def tuning(self) -> dict:
        """Launch shapes of the handle (see ci_tuning in include/ci.h)."""
        t = ci_tuning()
        _check(load_library().ci_basis_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    @tuning.setter
    def tuning(self, d: dict):
        t = ci_tuning()
        _check(load_library().ci_basis_get_tuning(self._h, ctypes.byref(t)))
        for k, v in d.items():
            setattr(t, k, int(v))
        _check(load_library().ci_basis_set_tuning(self._h, ctypes.byref(t)))

    def states(self, prob: int = 0):
        torch = _torch()
        i = self.info[prob]
        out = torch.empty((i["dim"], 2 * i["n_words"]), dtype=torch.int64, device=self.device)
        _check(load_library().ci_basis_states(self._h, prob, _ptr(out), _stream_ptr()))
        return out

    def row_ptr_slice(self, row_ptr, prob: int):
        """row_ptr of one basis (values are positions in the concatenated arrays)."""
        i = self.info[prob]
        return row_ptr[i["row_ptr_offset"]: i["row_ptr_offset"] + i["dim"] + 1]


def ci_basis_build(problems, stream=None) -> Basis:
    return Basis(problems, stream)


def ci_hamiltonian_count(basis: Basis, stream=None):
    """Count pass: (row_ptr int64 device tensor, nnz list per basis)."""
    torch = _torch()
    row_ptr = torch.empty(basis.n_rowptr, dtype=torch.int64, device=basis.device)
    nnz = np.zeros(basis.n_probs, np.int64)
    _check(load_library().ci_hamiltonian_count(basis.handle, _ptr(row_ptr),
                                               nnz.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream)))
    basis.nnz = [int(x) for x in nnz]
    return row_ptr, basis.nnz


def ci_hamiltonian_count_full(basis: Basis, stream=None):
    """Count pass of the full symmetric matrix: (row_ptr, nnz list per basis)."""
    torch = _torch()
    row_ptr = torch.empty(basis.n_rowptr, dtype=torch.int64, device=basis.device)
    nnz = np.zeros(basis.n_probs, np.int64)
    _check(load_library().ci_hamiltonian_count_full(basis.handle, _ptr(row_ptr),
                                                    nnz.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream)))
    basis.nnz_full = [int(x) for x in nnz]
    return row_ptr, basis.nnz_full


def ci_hamiltonian_fill_full(basis: Basis, tbme, row_ptr, col=None, val=None, stream=None):
    """Fill pass of the full symmetric matrix: (col int32, val float32)."""
    torch = _torch()
    tot = sum(basis.nnz_full)
    _check_tensor(tbme, torch.float32, basis.n_tbme, "tbme")
    _check_tensor(row_ptr, torch.int64, basis.n_rowptr, "row_ptr")
    if col is None:
        col = torch.empty(tot, dtype=torch.int32, device=basis.device)
    if val is None:
        val = torch.empty(tot, dtype=torch.float32, device=basis.device)
    _check_tensor(col, torch.int32, tot, "col")
    _check_tensor(val, torch.float32, tot, "val")
    _check(load_library().ci_hamiltonian_fill_full(basis.handle, _ptr(tbme), _ptr(row_ptr), _ptr(col), _ptr(val),
                                                   _stream_ptr(stream)))
    return col, val


def _h3_count(basis: Basis, full: bool, stream=None):
    torch = _torch()
    row_ptr = torch.empty(basis.n_rowptr, dtype=torch.int64, device=basis.device)
    nnz = np.zeros(basis.n_probs, np.int64)
    fn = load_library().ci_hamiltonian3_count_full if full else load_library().ci_hamiltonian3_count
    _check(fn(basis.handle, _ptr(row_ptr), nnz.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream)))
    counts = [int(x) for x in nnz]
    if full:
        basis.nnz3_full = counts
    else:
        basis.nnz3 = counts
    return row_ptr, counts


def _h3_fill(basis: Basis, tbme, v3, row_ptr, col, val, full: bool, stream=None):
    torch = _torch()
    tot = sum(basis.nnz3_full if full else basis.nnz3)
    _check_tensor(tbme, torch.float32, basis.n_tbme, "tbme")
    _check_tensor(row_ptr, torch.int64, basis.n_rowptr, "row_ptr")
    if col is None:
        col = torch.empty(tot, dtype=torch.int32, device=basis.device)
    if val is None:
        val = torch.empty(tot, dtype=torch.float32, device=basis.device)
    _check_tensor(col, torch.int32, tot, "col")
    _check_tensor(val, torch.float32, tot, "val")
    kind, seed, scale = v3
    p = ci_v3(int(kind), int(seed) & ((1 << 64) - 1), float(scale))
    fn = load_library().ci_hamiltonian3_fill_full if full else load_library().ci_hamiltonian3_fill
    _check(fn(basis.handle, _ptr(tbme), ctypes.byref(p), _ptr(row_ptr), _ptr(col), _ptr(val), _stream_ptr(stream)))
    return col, val


def ci_hamiltonian3_count(basis: Basis, stream=None):
    """Count pass of the matrix with a three-body term (states at most three
    nucleons apart, upper triangle): (row_ptr, nnz list per basis)."""
    return _h3_count(basis, False, stream)


def ci_hamiltonian3_fill(basis: Basis, tbme, v3, row_ptr, col=None, val=None, stream=None):
    """Fill pass with the three-body term: (col int32, val float32).
    v3 = (kind, seed, scale) with kind CI_V3_NONE / CI_V3_SYNTHETIC / CI_V3_IDENTITY."""
    return _h3_fill(basis, tbme, v3, row_ptr, col, val, False, stream)


def ci_hamiltonian3_count_full(basis: Basis, stream=None):
    """Count pass of the FULL symmetric matrix with the three-body term."""
    return _h3_count(basis, True, stream)


def ci_hamiltonian3_fill_full(basis: Basis, tbme, v3, row_ptr, col=None, val=None, stream=None):
    """Fill pass of the FULL symmetric matrix with the three-body term (for ci_lanczos)."""
    return _h3_fill(basis, tbme, v3, row_ptr, col, val, True, stream)


def ci_hamiltonian_spmv(basis: Basis, prob: int, row_ptr, col, val, x, y=None, stream=None, upper=False):
    """y = H x (float64) for problem `prob`, H in full CSR form, or (upper=True)
    the stored upper triangle of ci_hamiltonian_fill (ci_hamiltonian_spmv_upper)."""
    torch = _torch()
    D = basis.info[prob]["dim"]
    _check_tensor(x, torch.float64, D, "x")
    if y is None:
        y = torch.empty(D, dtype=torch.float64, device=basis.device)
    _check_tensor(y, torch.float64, D, "y")
    L = load_library()
    fn = L.ci_hamiltonian_spmv_upper if upper else L.ci_hamiltonian_spmv
    _check(fn(basis.handle, int(prob), _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y), _stream_ptr(stream)))
    return y


def ci_hamiltonian_spmv_upper(basis: Basis, prob: int, row_ptr, col, val, x, y=None, stream=None):
    """y = H x from the stored upper triangle (ci_hamiltonian_count / _fill output)."""
    return ci_hamiltonian_spmv(basis, prob, row_ptr, col, val, x, y, stream, upper=True)


def ci_lanczos_upper(basis: Basis, prob: int, row_ptr, col, val, x0=None, max_iter: int = 200, tol: float = 1e-12,
                     stream=None):
    """Lowest eigenpair of H from the stored upper triangle (ci_hamiltonian_fill output)."""
    return ci_lanczos(basis, prob, row_ptr, col, val, x0, max_iter, tol, stream, upper=True)


def ci_lanczos(basis: Basis, prob: int, row_ptr, col, val, x0=None, max_iter: int = 200, tol: float = 1e-12,
               stream=None, upper=False):
    """Lowest eigenpair of H (full CSR, or upper=True: the stored upper
    triangle): (eigenvalue, eigenvector float64 tensor, iterations)."""
    torch = _torch()
    D = basis.info[prob]["dim"]
    if x0 is None:
        x0 = torch.ones(D, dtype=torch.float64, device=basis.device)
    _check_tensor(x0, torch.float64, D, "x0")
    L = load_library()
    nwork = int(L.ci_lanczos_work_bytes(D, int(max_iter)))
    work = torch.empty(max(nwork, 8), dtype=torch.uint8, device=basis.device)
    evec = torch.empty(D, dtype=torch.float64, device=basis.device)
    ev, it = ctypes.c_double(), ctypes.c_int32()
    fn = L.ci_lanczos_upper if upper else L.ci_lanczos
    _check(fn(basis.handle, int(prob), _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x0), int(max_iter),
              float(tol), ctypes.byref(ev), ctypes.byref(it), _ptr(evec), _ptr(work),
              work.numel(), _stream_ptr(stream)))
    return ev.value, evec, it.value


def _check_tensor(t, dtype, n, name):
    torch = _torch()
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError("%s must be a contiguous %s CUDA tensor of %d elements" % (name, dtype, n))


def ci_hamiltonian_fill(basis: Basis, tbme, row_ptr, col=None, val=None, stream=None):
    """Fill pass: (col int32, val float32) device tensors of all stored entries."""
    torch = _torch()
    if basis.nnz is None:
        raise RuntimeError("call ci_hamiltonian_count first")
    tot = sum(basis.nnz)
    _check_tensor(tbme, torch.float32, basis.n_tbme, "tbme")
    _check_tensor(row_ptr, torch.int64, basis.n_rowptr, "row_ptr")
    if col is None:
        col = torch.empty(tot, dtype=torch.int32, device=basis.device)
    if val is None:
        val = torch.empty(tot, dtype=torch.float32, device=basis.device)
    _check_tensor(col, torch.int32, tot, "col")
    _check_tensor(val, torch.float32, tot, "val")
    _check(load_library().ci_hamiltonian_fill(basis.handle, _ptr(tbme), _ptr(row_ptr), _ptr(col), _ptr(val),
                                              _stream_ptr(stream)))
    return col, val


def ci_hamiltonian_vjp(basis: Basis, row_ptr, grad_val, grad_tbme=None, work=None, stream=None):
    """Adjoint: grad_tbme (float32 device) = d(sum grad_val * val)/d tbme."""
    torch = _torch()
    tot = sum(basis.nnz)
    _check_tensor(row_ptr, torch.int64, basis.n_rowptr, "row_ptr")
    _check_tensor(grad_val, torch.float32, tot, "grad_val")
    if grad_tbme is None:
        grad_tbme = torch.empty(basis.n_tbme, dtype=torch.float32, device=basis.device)
    nwork = basis.vjp_work_bytes()
    if work is None or work.numel() * work.element_size() < nwork:
        work = torch.empty(max(nwork, 8), dtype=torch.uint8, device=basis.device)
    _check(load_library().ci_hamiltonian_vjp(basis.handle, _ptr(row_ptr), _ptr(grad_val), _ptr(grad_tbme),
                                             _ptr(work), work.numel() * work.element_size(),
                                             _stream_ptr(stream)))
    return grad_tbme


def ci_hamiltonian_fill_keys(basis: Basis, tbme, row_ptr, col=None, val=None, keys=None, stream=None):
    """Fill pass that also stores one structure word per entry (int32 device
    tensor; opaque) for ci_hamiltonian_vjp_keys: (col, val, keys)."""
    torch = _torch()
    if basis.nnz is None:
        raise RuntimeError("call ci_hamiltonian_count first")
    tot = sum(basis.nnz)
    _check_tensor(tbme, torch.float32, basis.n_tbme, "tbme")
    _check_tensor(row_ptr, torch.int64, basis.n_rowptr, "row_ptr")
    if col is None:
        col = torch.empty(tot, dtype=torch.int32, device=basis.device)
    if val is None:
        val = torch.empty(tot, dtype=torch.float32, device=basis.device)
    if keys is None:
        keys = torch.empty(tot, dtype=torch.int32, device=basis.device)
    _check_tensor(col, torch.int32, tot, "col")
    _check_tensor(val, torch.float32, tot, "val")
    _check_tensor(keys, torch.int32, tot, "keys")
    _check(load_library().ci_hamiltonian_fill_keys(basis.handle, _ptr(tbme), _ptr(row_ptr), _ptr(col), _ptr(val),
                                                   _ptr(keys), _stream_ptr(stream)))
    return col, val, keys


def ci_hamiltonian_vjp_keys(basis: Basis, row_ptr, keys, grad_val, grad_tbme=None, work=None, stream=None):
    """Adjoint from the words of ci_hamiltonian_fill_keys: grad_tbme as ci_hamiltonian_vjp."""
    torch = _torch()
    tot = sum(basis.nnz)
    _check_tensor(row_ptr, torch.int64, basis.n_rowptr, "row_ptr")
    _check_tensor(keys, torch.int32, tot, "keys")
    _check_tensor(grad_val, torch.float32, tot, "grad_val")
    if grad_tbme is None:
        grad_tbme = torch.empty(basis.n_tbme, dtype=torch.float32, device=basis.device)
    nwork = basis.vjp_work_bytes()
    if work is None or work.numel() * work.element_size() < nwork:
        work = torch.empty(max(nwork, 8), dtype=torch.uint8, device=basis.device)
    _check(load_library().ci_hamiltonian_vjp_keys(basis.handle, _ptr(row_ptr), _ptr(keys), _ptr(grad_val),
                                                  _ptr(grad_tbme), _ptr(work), work.numel() * work.element_size(),
                                                  _stream_ptr(stream)))
    return grad_tbme


def ci_hamiltonian_tune(basis: Basis, tbme, row_ptr, col, val, grad_val, grad_tbme=None, work=None,
                        reps: int = 3, keys=None, stream=None) -> dict:
    """Autotuner: times the launch shapes of fill and adjoint on these buffers,
    keeps the fastest in the handle (and for later handles of the same
    problems); returns the chosen shapes.  keys: an int32 tensor of nnz
    elements to also tune the adjoint from stored words (it then holds the
    words), or None."""
    torch = _torch()
    tot = sum(basis.nnz)
    _check_tensor(tbme, torch.float32, basis.n_tbme, "tbme")
    _check_tensor(row_ptr, torch.int64, basis.n_rowptr, "row_ptr")
    _check_tensor(col, torch.int32, tot, "col")
    _check_tensor(val, torch.float32, tot, "val")
    _check_tensor(grad_val, torch.float32, tot, "grad_val")
    if keys is not None:
        _check_tensor(keys, torch.int32, tot, "keys")
    if grad_tbme is None:
        grad_tbme = torch.empty(basis.n_tbme, dtype=torch.float32, device=basis.device)
    nwork = basis.vjp_work_bytes()
    if work is None or work.numel() * work.element_size() < nwork:
        work = torch.empty(max(nwork, 8), dtype=torch.uint8, device=basis.device)
    _check(load_library().ci_hamiltonian_tune(basis.handle, _ptr(tbme), _ptr(row_ptr), _ptr(col), _ptr(val),
                                              _ptr(keys) if keys is not None else None,
                                              _ptr(grad_val), _ptr(grad_tbme), _ptr(work),
                                              work.numel() * work.element_size(), int(reps),
                                              _stream_ptr(stream)))
    return basis.tuning


def ci_probe_ceilings(mib: int = 1024, stream=None) -> dict:
    """Measured store bandwidth (GB/s) and XOR + popcount steps/s of the device."""
    torch = _torch()
    buf = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    gbs, steps = ctypes.c_double(), ctypes.c_double()
    _check(load_library().ci_probe_ceilings(_ptr(buf), buf.numel(), ctypes.byref(gbs), ctypes.byref(steps),
                                            _stream_ptr(stream)))
    return {"store_GBps": gbs.value, "xor_popcount_steps_per_s": steps.value, "store_bytes": int(mib) << 20}


def ci_clebsch_gordan(j1: int, m1: int, j2: int, m2: int, J: int, M: int) -> float:
    """<j1 m1 j2 m2 | J M>, doubled arguments (host; the decoupling's table routine)."""
    out = ctypes.c_double()
    _check(load_library().ci_clebsch_gordan(j1, m1, j2, m2, J, M, ctypes.byref(out)))
    return out.value


def ci_threebody_plan(n1max: int, n3max: int) -> dict:
    """Sizes of the three-body layout (host only)."""
    n, t = ctypes.c_int64(), ctypes.c_int32()
    _check(load_library().ci_threebody_plan(int(n1max), int(n3max), ctypes.byref(n), ctypes.byref(t)))
    return {"n_coupled": n.value, "n_triples": t.value}


class ThreeBody:
    """Three-body layout (coupled-JT input order, device tables) of shells
    0..n1max with triples inside n3max."""

    def __init__(self, n1max: int, n3max: int):
        _torch()
        L = load_library()
        h = ctypes.c_void_p()
        _check(L.ci_threebody_build(int(n1max), int(n3max), ctypes.byref(h)))
        self._h = h
        nc, ns, nn, nt = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(L.ci_threebody_info(h, ctypes.byref(nc), ctypes.byref(ns), ctypes.byref(nn), ctypes.byref(nt)))
        self.n_coupled, self.n_sps, self.n_nlj, self.n_triples = nc.value, ns.value, nn.value, nt.value
        self.nlj = np.zeros((self.n_nlj, 3), np.int32)
        self.morb = np.zeros((self.n_sps, 2), np.int32)
        self.triples = np.zeros((max(self.n_triples, 1), 3), np.int32)
        _check(L.ci_threebody_orbitals(h, self.nlj.ctypes.data_as(ctypes.c_void_p),
                                       self.morb.ctypes.data_as(ctypes.c_void_p),
                                       self.triples.ctypes.data_as(ctypes.c_void_p)))

    def keys(self) -> np.ndarray:
        """[n_coupled, 8] int32: (t, t', 2J, 2T, 2J_ab, 2T_ab, 2J_de, 2T_de) in storage order."""
        out = np.zeros((max(self.n_coupled, 1), 8), np.int32)
        _check(load_library().ci_threebody_keys(self._h, out.ctypes.data_as(ctypes.c_void_p), self.n_coupled))
        return out[: self.n_coupled]

    # below this many requests the cost order (four small launches, ~40 us) does not pay
    ORDER_MIN = 1 << 19

    def decouple(self, coupled, requests, out=None, order="auto", work=None, stream=None):
        """m-scheme elements (float32 device tensor) of requests (int32 [n, 6] device tensor).
        order: True to group the requests by cost first (a work buffer of
        ci_threebody_work_bytes(n) bytes, `work` or one the handle keeps),
        False for the given order, "auto" for True from ORDER_MIN requests."""
        torch = _torch()
        _check_tensor(coupled, torch.float32, self.n_coupled, "coupled")
        if requests.dtype != torch.int32 or not requests.is_cuda or not requests.is_contiguous():
            raise ValueError("requests must be a contiguous int32 CUDA tensor [n, 6]")
        n = requests.numel() // 6
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=coupled.device)
        _check_tensor(out, torch.float32, n, "out")
        L = load_library()
        if order == "auto":
            order = n >= self.ORDER_MIN
        wptr, wbytes = None, 0
        if order:
            need = int(L.ci_threebody_work_bytes(n))
            if work is None:
                if getattr(self, "_work", None) is None or self._work.numel() < need:
                    self._work = torch.empty(need, dtype=torch.uint8, device=coupled.device)
                work = self._work
            if not work.is_cuda or work.numel() * work.element_size() < need:
                raise ValueError("work must be a CUDA tensor of at least %d bytes" % need)
            wptr, wbytes = _ptr(work), work.numel() * work.element_size()
        _check(L.ci_threebody_decouple(self._h, _ptr(coupled), _ptr(requests), n, _ptr(out), wptr, wbytes,
                                       _stream_ptr(stream)))
        return out

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().ci_threebody_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _make_autograd():
    import torch

    class CIHamiltonian(torch.autograd.Function):
        """val = H(tbme) on a fixed structure; backward runs the adjoint kernel.

        The backward recomputes the pair and phase structure by walking the
        partner lists again (the default).  store_keys: the forward also
        stores one structure word per entry (4 bytes each, kept until
        backward) and the backward reads them instead."""

        @staticmethod
        def forward(ctx, tbme, basis, row_ptr, col=None, store_keys=False):
            ctx.basis = basis
            if store_keys:
                _, val, keys = ci_hamiltonian_fill_keys(basis, tbme.detach().contiguous(), row_ptr, col=col)
                ctx.save_for_backward(row_ptr, keys)
            else:
                _, val = ci_hamiltonian_fill(basis, tbme.detach().contiguous(), row_ptr, col=col)
                ctx.save_for_backward(row_ptr)
            return val

        @staticmethod
        def backward(ctx, gval):
            saved = ctx.saved_tensors
            gval = gval.contiguous().to(torch.float32)
            if len(saved) == 2:
                g = ci_hamiltonian_vjp_keys(ctx.basis, saved[0], saved[1], gval)
            else:
                g = ci_hamiltonian_vjp(ctx.basis, saved[0], gval)
            return g, None, None, None, None

    return CIHamiltonian


class _Lazy:
    def __init__(self):
        self._cls = None

    def __getattr__(self, k):
        if self._cls is None:
            self._cls = _make_autograd()
        return getattr(self._cls, k)


CIHamiltonian = _Lazy()
