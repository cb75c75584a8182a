"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds no arithmetic of the method: it only draws random numbers
and names the workloads.  Both the tests of the oracle and the tests/benchmark
of the HIP library take their inputs from here, so that each side is fed the
same bits.

Inputs (the interaction files of a real calculation are not available; these
stand in for them):
  * two-body table: N(0,1) MeV per stored element, drawn in table order with
    ``numpy.random.default_rng(seed).standard_normal(n_tbme)`` (FP64); the
    FP32 input of the library is its round-to-nearest;
  * one-body energies: (N + 3/2) * hbar*omega with hbar*omega = 15 MeV (these
    are computed by each side from the oscillator shell; only the 15 MeV is
    named here);
  * upstream gradient on the stored entries: G_e = fp32(psi_i * psi_j) for a
    seeded, unit-norm random vector psi of length D;
  * batch: 64 problems with (Z, N) uniform on {2,3,4}^2, Nmax uniform on
    {2,4,6}, the lowest allowed 2M = (Z + N) mod 2, positive parity.
"""
from __future__ import annotations

import numpy as np

HW_MEV = 15.0

# (Z, N, Nmax, 2M, parity) of the named workloads and their table seeds
WORKLOADS = {
    "he4_nmax2": dict(problem=(2, 2, 2, 0, 1), tbme_seed=0),
    "li6_nmax6": dict(problem=(3, 3, 6, 2, 1), tbme_seed=1),
    "b10_nmax4": dict(problem=(5, 5, 4, 0, 1), tbme_seed=2),
}
PSI_SEED = {"he4_nmax2": 101, "li6_nmax6": 102, "b10_nmax4": 104}
FD_SEED = 200
BATCH_SEED = 5
BATCH_SIZE = 64


def tbme_f64(seed: int, n_tbme: int) -> np.ndarray:
    """The two-body table in FP64 MeV, table order."""
    return np.random.default_rng(seed).standard_normal(n_tbme)


def tbme_f32(seed: int, n_tbme: int) -> np.ndarray:
    return tbme_f64(seed, n_tbme).astype(np.float32)


def psi(seed: int, dim: int) -> np.ndarray:
    """Seeded unit-norm FP64 vector of length dim."""
    v = np.random.default_rng(seed).standard_normal(dim)
    n = np.linalg.norm(v)
    return v / n if n > 0 else v


def upstream_grad(psi_vec: np.ndarray, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """G_e = fp32(psi_i * psi_j) for each stored entry (i, j)."""
    return (psi_vec[rows] * psi_vec[cols]).astype(np.float32)


def fd_keys(n_tbme: int, count: int = 64) -> np.ndarray:
    """Distinct table indices for the finite-difference check."""
    return np.sort(np.random.default_rng(FD_SEED).choice(n_tbme, size=min(count, n_tbme),
                                                         replace=False))


def batch_problems(seed: int = BATCH_SEED, count: int = BATCH_SIZE):
    """List of (Z, N, Nmax, 2M, parity) and table seeds / psi seeds per basis."""
    rng = np.random.default_rng(seed)
    zs = rng.integers(2, 5, size=count)
    ns = rng.integers(2, 5, size=count)
    nm = rng.choice([2, 4, 6], size=count)
    probs = [(int(z), int(n), int(m), int((z + n) % 2), 1) for z, n, m in zip(zs, ns, nm)]
    return probs, [1000 + b for b in range(count)], [2000 + b for b in range(count)]


def sample_rows(dim: int, count: int, seed: int) -> np.ndarray:
    """Sorted distinct row indices, always including the first and last row."""
    if dim <= count:
        return np.arange(dim, dtype=np.int64)
    r = np.random.default_rng(seed).choice(dim, size=count - 2, replace=False)
    return np.unique(np.concatenate([[0, dim - 1], r])).astype(np.int64)
