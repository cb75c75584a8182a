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


# ---------------------------------------------------------------- three-body inputs

def _mix64(x):
    """splitmix64 finalizer on uint64 arrays (wrapping arithmetic)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return x ^ (x >> np.uint64(31))


SPLITMIX64_GAMMA = 0x9E3779B97F4A7C15


def v3_synthetic(seed, a, b, c, d, e, f, scale=1.0):
    """Synthetic antisymmetrized m-scheme three-body elements V_{abc,def} for
    ascending triples of combined orbit indices (arrays): the (x+1)-th output
    of the splitmix64 generator (Steele, Lea & Flood 2014) started at `seed`,
    x = min(kb, kk) << 27 | max(kb, kk) with k = (a*512 + b)*512 + c per
    triple, mapped to scale * (2u - 1), u = top 53 bits / 2^53."""
    u = np.uint64
    with np.errstate(over="ignore"):
        kb = (np.asarray(a, dtype=u) * u(512) + np.asarray(b, dtype=u)) * u(512) + np.asarray(c, dtype=u)
        kk = (np.asarray(d, dtype=u) * u(512) + np.asarray(e, dtype=u)) * u(512) + np.asarray(f, dtype=u)
        x = (np.minimum(kb, kk) << u(27)) | np.maximum(kb, kk)
        z = _mix64(u(int(seed) & ((1 << 64) - 1)) + (x + u(1)) * u(SPLITMIX64_GAMMA))
    return scale * (2.0 * ((z >> u(11)).astype(np.float64) / float(1 << 53)) - 1.0)


def coupled3b_values(seed, bra, ket, J2, T2, Jab2, Tab2, Jde2, Tde2):
    """Synthetic coupled-JT three-body elements, N(0,1), from a counter-based
    hash of the labels (bra, ket: [n, 3] orbital triples; the rest [n] doubled
    quantum numbers).  Symmetric under exchanging (bra, J_ab, T_ab) with
    (ket, J_de, T_de), so the interaction is Hermitian."""
    u = np.uint64
    bra = np.asarray(bra, dtype=np.uint64).reshape(-1, 3)
    ket = np.asarray(ket, dtype=np.uint64).reshape(-1, 3)
    with np.errstate(over="ignore"):
        hb = _mix64((((bra[:, 0] * u(97) + bra[:, 1]) * u(97) + bra[:, 2]) * u(131) + np.asarray(Jab2, dtype=u)) * u(7)
                    + np.asarray(Tab2, dtype=u))
        hk = _mix64((((ket[:, 0] * u(97) + ket[:, 1]) * u(97) + ket[:, 2]) * u(131) + np.asarray(Jde2, dtype=u)) * u(7)
                    + np.asarray(Tde2, dtype=u))
        lo, hi = np.minimum(hb, hk), np.maximum(hb, hk)
        x = _mix64(lo ^ _mix64(hi + u(seed)) ^ (np.asarray(J2, dtype=u) * u(0x9E3779B97F4A7C15))
                   ^ (np.asarray(T2, dtype=u) << u(56)))
        y = _mix64(x + u(0x632BE59BD9B4E019))
    u1 = ((x >> u(11)).astype(np.float64) + 0.5) / float(1 << 53)
    u2 = ((y >> u(11)).astype(np.float64) + 0.5) / float(1 << 53)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def coupled3b_value(seed, bra, ket, J2, T2, Jab2, Tab2, Jde2, Tde2) -> float:
    return float(coupled3b_values(seed, [bra], [ket], [J2], [T2], [Jab2], [Tab2], [Jde2], [Tde2])[0])


def _morbits(n1max):
    out = []  # (N, l, 2j, 2m) of one species, ordered by N, l, 2j, 2m
    for N in range(n1max + 1):
        for l in range(N % 2, N + 1, 2):
            for j2 in (2 * l - 1, 2 * l + 1):
                if j2 > 0:
                    out.extend((N, l, j2, m2) for m2 in range(-j2, j2 + 1, 2))
    return out


def requests_3b(seed, n, n1max, n3max, mismatched=0):
    """n three-body requests [n, 6] int32 (combined orbit indices a b c d e f)
    with both triples inside n3max and equal M, M_T and parity, plus
    `mismatched` requests whose ket has a different M (their element is 0).
    Each orbit is drawn uniformly among those that still fit under n3max."""
    orb = _morbits(n1max)
    ns = len(orb)
    comb = [(o[0], o[1], o[3], 1 if s == 0 else -1) for s in range(2) for o in orb]  # N, l, 2m, 2t
    by_n = sorted(range(2 * ns), key=lambda k: comb[k][0])
    upto = [sum(1 for k in range(2 * ns) if comb[k][0] <= q) for q in range(n3max + 1)]
    by = {}
    for k, (N, l, m2, t2) in enumerate(comb):
        by.setdefault((m2, t2, l % 2), []).append((N, k))
    for v in by.values():
        v.sort()
    rng = np.random.default_rng(seed)

    def draw(room):
        return by_n[int(rng.integers(0, upto[room]))]

    out = []
    while len(out) < n:
        a = draw(n3max)
        b = draw(n3max - comb[a][0])
        c = draw(n3max - comb[a][0] - comb[b][0])
        d = draw(n3max)
        e = draw(n3max - comb[d][0])
        M = comb[a][2] + comb[b][2] + comb[c][2]
        MT = comb[a][3] + comb[b][3] + comb[c][3]
        par = (comb[a][1] + comb[b][1] + comb[c][1]) % 2
        key = (M - comb[d][2] - comb[e][2], MT - comb[d][3] - comb[e][3], (par - comb[d][1] - comb[e][1]) % 2)
        room = n3max - comb[d][0] - comb[e][0]
        cand = by.get(key, ())
        cnt = 0
        while cnt < len(cand) and cand[cnt][0] <= room:
            cnt += 1
        if cnt == 0:
            continue
        out.append((a, b, c, d, e, cand[int(rng.integers(0, cnt))][1]))
    for _ in range(mismatched):
        r = list(out[int(rng.integers(0, n))])  # a valid request
        # move f to another projection of the same orbital (a different M)
        N, l, j2, m2 = orb[r[5] % ns]
        if j2 > 1:
            m_new = m2 + 2 if m2 + 2 <= j2 else m2 - 2
            r[5] = (r[5] // ns) * ns + orb.index((N, l, j2, m_new))
            out.append(tuple(r))
    return np.asarray(out, dtype=np.int32).reshape(-1, 6)
