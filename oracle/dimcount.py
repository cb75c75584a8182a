"""Basis dimension by a generating function (no enumeration of determinants).

TEST INFRASTRUCTURE ONLY (pins the C oracle's basis enumeration).

For one species, the number of ways to occupy X distinct harmonic-oscillator
orbits with total oscillator quanta Nq and total 2M is the coefficient of
x^X q^Nq y^M in prod_orbits (1 + x q^N y^m).  The dimension of the M-scheme
Nmax space is then the sum over compatible (proton, neutron) coefficients:
Nq_p + Nq_n <= N0 + Nmax, (-1)^(Nq_p + Nq_n) = parity, 2M_p + 2M_n = 2M.
The orbit multiset per shell is rebuilt here from the HO quantum numbers.
"""
from __future__ import annotations

from collections import defaultdict


def _shell_orbits(N):
    """(N, 2m) of every orbit in shell N: l = N, N-2, ..; j = l -+ 1/2; m = -j..j."""
    out = []
    for l in range(N % 2, N + 1, 2):
        for j2 in (2 * l - 1, 2 * l + 1):
            if j2 >= 0:
                out += [(N, m2) for m2 in range(-j2, j2 + 1, 2)]
    return out


def species_counts(X: int, shells: int, nq_max: int):
    """{(Nq, 2M): number of X-subsets} for orbits in shells 0..shells."""
    # poly[k] : dict (nq, m2) -> count, for k chosen orbits
    poly = [defaultdict(int) for _ in range(X + 1)]
    poly[0][(0, 0)] = 1
    for N in range(shells + 1):
        for (_, m2) in _shell_orbits(N):
            for k in range(X, 0, -1):
                for (nq, mm), c in list(poly[k - 1].items()):
                    if nq + N <= nq_max:
                        poly[k][(nq + N, mm + m2)] += c
    return dict(poly[X])


def dimension(Z, N, nmax, two_m, parity, shells, n0p, n0n):
    top = n0p + n0n + nmax
    cp = species_counts(Z, shells, top - n0n)
    cn = species_counts(N, shells, top - n0p)
    D = 0
    for (qp, mp), a in cp.items():
        for (qn, mn), b in cn.items():
            q = qp + qn
            if q <= top and (1 if q % 2 == 0 else -1) == parity and mp + mn == two_m:
                D += a * b
    return D
