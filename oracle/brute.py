"""Pure-Python second-quantized operator application on tiny bases.

TEST INFRASTRUCTURE ONLY (pins the C oracle; never used by the product).

This is a second, independent route to the same matrix: it does not use the
Slater-Condon formulas at all.  Each basis state |Phi_j> is a product of
creation operators in ascending combined index acting on the vacuum; the
Hamiltonian

    H = sum_a e_a a+_a a_a + sum_{a<b, c<d} V_{ab,cd} a+_a a+_b a_d a_c

is applied term by term with explicit fermion signs, and <Phi_i|H|Phi_j> is read
off.  The paper (Sec. 2) states that elements are linear combinations of
kinetic and two-body interaction terms; the operator form above is the textbook
definition of that combination.  The basis is enumerated here independently
(itertools over orbit subsets), in the same key / colex order as the C oracle,
so that the two can be compared index by index.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def shell_cap(N: int) -> int:
    return (N + 1) * (N + 2)


def ntop(X: int) -> int:
    N, filled = 0, 0
    if X <= 0:
        return 0
    while filled + shell_cap(N) < X:
        filled += shell_cap(N)
        N += 1
    return N


def n0(X: int) -> int:
    s, N, left = 0, 0, X
    while left > 0:
        take = min(left, shell_cap(N))
        s += take * N
        left -= take
        N += 1
    return s


def orbits(S: int):
    """(N, n, l, 2j, 2m) for shells 0..S, ordered N, l, 2j, 2m ascending."""
    out = []
    for N in range(S + 1):
        for l in range(N % 2, N + 1, 2):
            for j2 in (2 * l - 1, 2 * l + 1):
                if j2 < 0:
                    continue
                for m2 in range(-j2, j2 + 1, 2):
                    out.append((N, (N - l) // 2, l, j2, m2))
    return out


class BruteBasis:
    def __init__(self, Z, N, nmax, two_m, parity=1, hw=15.0):
        self.Z, self.N, self.nmax, self.two_m, self.parity, self.hw = Z, N, nmax, two_m, parity, hw
        self.S = max(ntop(Z), ntop(N)) + nmax
        self.orb = orbits(self.S)
        self.nsps = len(self.orb)
        self.N0 = n0(Z) + n0(N)
        top = self.N0 + nmax
        # species subsets with their (Nq, 2M) key
        def species(X, other0):
            res = {}
            for occ in itertools.combinations(range(self.nsps), X):
                nq = sum(self.orb[o][0] for o in occ)
                if nq > top - other0:
                    continue
                m2 = sum(self.orb[o][4] for o in occ)
                res.setdefault((nq, m2), []).append(occ)
            return res

        sp, sn = species(Z, n0(N)), species(N, n0(Z))

        def ok(kp, kn):
            nq = kp[0] + kn[0]
            return nq <= top and (1 if nq % 2 == 0 else -1) == parity and kp[1] + kn[1] == two_m

        blocks = sorted((kp, kn) for kp in sp for kn in sn if ok(kp, kn))

        def colex(occ):  # the bitstring as an unsigned integer
            return sum(1 << o for o in occ)

        self.states = []  # combined-index occupation tuples
        for kp, kn in blocks:
            for P in sorted(sp[kp], key=colex):
                for Q in sorted(sn[kn], key=colex):
                    self.states.append(tuple(P) + tuple(self.nsps + q for q in Q))
        self.index = {s: i for i, s in enumerate(self.states)}
        self.dim = len(self.states)

    def spe(self, a: int, kinetic: bool = False) -> float:
        """Diagonal one-body energy of orbit a: the oscillator energy (N + 3/2) hw,
        or with the kinetic term the diagonal of T, (hw/2)(2n + l + 3/2)."""
        N, n, l = self.orb[a % self.nsps][:3]
        return 0.5 * (2 * n + l + 1.5) * self.hw if kinetic else (N + 1.5) * self.hw

    def state_words(self, W: int) -> np.ndarray:
        """[D, 2W] uint64 words (proton then neutron), for comparison."""
        out = np.zeros((self.dim, 2 * W), np.uint64)
        for i, s in enumerate(self.states):
            for a in s:
                sp, o = divmod(a, self.nsps)
                out[i, sp * W + o // 64] |= np.uint64(1) << np.uint64(o % 64)
        return out


def _annihilate(occ: tuple, c: int):
    if c not in occ:
        return None, 0
    k = occ.index(c)  # number of occupied orbits below c (occ is ascending)
    return occ[:k] + occ[k + 1:], (-1) ** k


def _create(occ: tuple, a: int):
    if a in occ:
        return None, 0
    k = sum(1 for x in occ if x < a)
    return occ[:k] + (a,) + occ[k:], (-1) ** k


def kinetic_offdiag(basis: BruteBasis, a: int, b: int) -> float:
    """Harmonic-oscillator kinetic energy between orbits a != b (combined
    index) of one species: nonzero only for the same (l, j, m) and radial
    quantum numbers n, n + 1, where it is (hw/2) sqrt((n+1)(n+l+3/2))."""
    if a == b or a // basis.nsps != b // basis.nsps:
        return 0.0
    Na, na, la, ja, ma = basis.orb[a % basis.nsps]
    Nb, nb, lb, jb, mb = basis.orb[b % basis.nsps]
    if (la, ja, ma) != (lb, jb, mb) or abs(na - nb) != 1:
        return 0.0
    n = min(na, nb)
    return 0.5 * basis.hw * math.sqrt((n + 1) * (n + la + 1.5))


def hamiltonian(basis: BruteBasis, keys: np.ndarray, values: np.ndarray, kinetic: bool = False) -> np.ndarray:
    """Dense <Phi_i|H|Phi_j> by operator application.

    `keys[t] = (a, b, c, d)` with a<b, c<d is the two-body table as a list of
    canonical elements V_{ab,cd} = V_{cd,ab}; anything not listed is zero.
    kinetic: the one-body term is the oscillator kinetic energy T, its
    diagonal (spe) plus sum_{a != b} t_ab a+_a a_b (kinetic_offdiag)."""
    D = basis.dim
    H = np.zeros((D, D))
    if kinetic:
        norb = 2 * basis.nsps
        for j, phi in enumerate(basis.states):
            for b in phi:
                x0, s1 = _annihilate(phi, b)
                for a in range(norb):
                    t = kinetic_offdiag(basis, a, b)
                    if t == 0.0:
                        continue
                    x, s2 = _create(x0, a)
                    if x is None:
                        continue
                    i = basis.index.get(x)
                    if i is not None:
                        H[i, j] += s1 * s2 * t
    # ket pair (c,d) -> list of (a, b, V_{ab,cd}); both orientations of each key
    by_ket = {}
    for (a, b, c, d), v in zip(map(tuple, keys), values):
        by_ket.setdefault((c, d), []).append((a, b, v))
        if (a, b) != (c, d):
            by_ket.setdefault((a, b), []).append((c, d, v))
    for j, phi in enumerate(basis.states):
        H[j, j] += sum(basis.spe(a, kinetic) for a in phi)
        for c, d in itertools.combinations(phi, 2):  # c < d, both occupied
            for a, b, v in by_ket.get((c, d), ()):
                x, s1 = _annihilate(phi, c)
                x, s2 = _annihilate(x, d)
                x, s3 = _create(x, b)
                if x is None:
                    continue
                x, s4 = _create(x, a)
                if x is None:
                    continue
                i = basis.index.get(x)
                if i is None:
                    continue  # leaves the truncated space
                H[i, j] += s1 * s2 * s3 * s4 * v
    return H


def hamiltonian3(basis: BruteBasis, v3) -> np.ndarray:
    """Dense <Phi_i|H3|Phi_j> by operator application, for

        H3 = sum_{a<b<c, d<e<f} V_{abc,def} a+_a a+_b a+_c a_f a_e a_d

    with v3(a, b, c, d, e, f) the element for ascending triples.  Each term
    removes d, e, f from |Phi_j> (in that order) and creates c, b, a, with the
    fermion sign of every step; created triples are drawn from those with the
    removed triple's species content, total 2m and parity (any other triple
    leaves the basis)."""
    D = basis.dim
    H = np.zeros((D, D))
    norb = 2 * basis.nsps

    def label(t):
        occ = [basis.orb[o % basis.nsps] for o in t]
        return (sum(1 for o in t if o < basis.nsps), sum(x[4] for x in occ), sum(x[2] for x in occ) % 2)

    by_label = {}
    for t in itertools.combinations(range(norb), 3):
        by_label.setdefault(label(t), []).append(t)
    for j, phi in enumerate(basis.states):
        for d, e, f in itertools.combinations(phi, 3):
            x, s1 = _annihilate(phi, d)
            x, s2 = _annihilate(x, e)
            x, s3 = _annihilate(x, f)
            for a, b, c in by_label[label((d, e, f))]:
                y, t1 = _create(x, c)
                if y is None:
                    continue
                y, t2 = _create(y, b)
                if y is None:
                    continue
                y, t3 = _create(y, a)
                if y is None:
                    continue
                i = basis.index.get(y)
                if i is not None:
                    H[i, j] += s1 * s2 * s3 * t1 * t2 * t3 * v3(a, b, c, d, e, f)
    return H
