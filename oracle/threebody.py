"""Plain oracle for the three-body basis transformation (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark's CPU baseline,
never by the product library, and it imports nothing from it.

The m-scheme element of a three-body interaction between product states
|a b c> and |d e f> (orbits with projections m and isospin projections t) is
the coupled-JT interaction transformed back with angular-momentum and isospin
coupling coefficients (paper Sec. 3.1: A' = D^T A D, the projections D built
from coupling coefficients and never formed):

    <abc|V|def> = sum_{J_ab T_ab J_de T_de J T}
        <j_a m_a j_b m_b|J_ab M_ab> <J_ab M_ab j_c m_c|J M>
        <1/2 t_a 1/2 t_b|T_ab M_Tab> <T_ab M_Tab 1/2 t_c|T M_T>
        (the same for d e f)  V^{J T}_{(ab) J_ab T_ab c, (de) J_de T_de f}

with V^{JT} diagonal in J, T and independent of M, M_T.  Here everything is a
direct sum over all quantum numbers the coefficients allow, with exact
rational Clebsch-Gordan coefficients (Racah's closed formula, Python
integers); the coupled elements come from a caller's function of the labels.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache


def nlj_orbitals(n1max: int):
    """[(N, l, 2j)] for shells 0..n1max, ordered by N, l, 2j."""
    out = []
    for N in range(n1max + 1):
        for l in range(N % 2, N + 1, 2):
            for j2 in (2 * l - 1, 2 * l + 1):
                if j2 > 0:
                    out.append((N, l, j2))
    return out


def m_orbitals(n1max: int):
    """[(orbital index, 2m)] of one species, ordered by N, l, 2j, 2m."""
    out = []
    for a, (N, l, j2) in enumerate(nlj_orbitals(n1max)):
        for m2 in range(-j2, j2 + 1, 2):
            out.append((a, m2))
    return out


def _tri(a2, b2, c2):
    return abs(a2 - b2) <= c2 <= a2 + b2 and (a2 + b2 + c2) % 2 == 0


@lru_cache(maxsize=None)
def cg(j1: int, m1: int, j2: int, m2: int, J: int, M: int) -> float:
    """<j1 m1 j2 m2|J M>, all arguments doubled (Condon-Shortley phases)."""
    if m1 + m2 != M or abs(m1) > j1 or abs(m2) > j2 or abs(M) > J or not _tri(j1, j2, J):
        return 0.0
    if (j1 + m1) % 2 or (j2 + m2) % 2 or (J + M) % 2:
        return 0.0
    f = math.factorial
    a, b, c = (j1 + j2 - J) // 2, (j1 - j2 + J) // 2, (-j1 + j2 + J) // 2
    pre = Fraction((J + 1) * f(a) * f(b) * f(c) * f((J + M) // 2) * f((J - M) // 2) * f((j1 - m1) // 2)
                   * f((j1 + m1) // 2) * f((j2 - m2) // 2) * f((j2 + m2) // 2), f((j1 + j2 + J) // 2 + 1))
    s = Fraction(0)
    for k in range(0, a + 1):
        d = [k, a - k, (j1 - m1) // 2 - k, (j2 + m2) // 2 - k, (J - j2 + m1) // 2 + k, (J - j1 - m2) // 2 + k]
        if min(d) < 0:
            continue
        den = 1
        for x in d:
            den *= f(x)
        s += Fraction((-1) ** k, den)
    return float(s) * math.sqrt(pre)


def channels(j2a, j2b, j2c, J2, T2):
    """(2J_ab, 2T_ab) channels of a triple coupled to (J, T)."""
    return [(jab, tab) for jab in range(abs(j2a - j2b), j2a + j2b + 1, 2) if _tri(jab, j2c, J2)
            for tab in (0, 2) if _tri(tab, 1, T2)]


class ThreeBody:
    """Oscillator space of shells 0..n1max, triples with N_a + N_b + N_c <= n3max."""

    def __init__(self, n1max: int, n3max: int):
        self.n1max, self.n3max = n1max, n3max
        self.nlj = nlj_orbitals(n1max)
        self.morb = m_orbitals(n1max)
        self.nsps = len(self.morb)

    def decode(self, o: int):
        """(orbital, 2m, 2t) of a combined index (proton k -> k, neutron n_sps + k)."""
        sp, k = divmod(o, self.nsps)
        a, m2 = self.morb[k]
        return a, m2, (1 if sp == 0 else -1)

    def element(self, req, value) -> float:
        """<abc|V|def> for one request (six combined orbit indices);
        value(bra, ket, J2, T2, Jab2, Tab2, Jde2, Tde2) gives the coupled
        element for orbital triples bra = (a, b, c), ket = (d, e, f)."""
        if any(o < 0 or o >= 2 * self.nsps for o in req):
            return 0.0
        q = [self.decode(o) for o in req]
        al = [x[0] for x in q]
        m = [x[1] for x in q]
        t = [x[2] for x in q]
        N = [self.nlj[a][0] for a in al]
        l = [self.nlj[a][1] for a in al]
        j = [self.nlj[a][2] for a in al]
        if sum(N[:3]) > self.n3max or sum(N[3:]) > self.n3max:
            return 0.0
        if sum(m[:3]) != sum(m[3:]) or sum(t[:3]) != sum(t[3:]) or sum(l[:3]) % 2 != sum(l[3:]) % 2:
            return 0.0
        M, MT = sum(m[:3]), sum(t[:3])
        bra, ket = tuple(al[:3]), tuple(al[3:])
        total = 0.0
        for J2 in range(1, min(sum(j[:3]), sum(j[3:])) + 1, 2):
            for T2 in (1, 3):
                for jab, tab in channels(j[0], j[1], j[2], J2, T2):
                    cb = (cg(j[0], m[0], j[1], m[1], jab, m[0] + m[1]) * cg(jab, m[0] + m[1], j[2], m[2], J2, M)
                          * cg(1, t[0], 1, t[1], tab, t[0] + t[1]) * cg(tab, t[0] + t[1], 1, t[2], T2, MT))
                    if cb == 0.0:
                        continue
                    for jde, tde in channels(j[3], j[4], j[5], J2, T2):
                        ck = (cg(j[3], m[3], j[4], m[4], jde, m[3] + m[4]) * cg(jde, m[3] + m[4], j[5], m[5], J2, M)
                              * cg(1, t[3], 1, t[4], tde, t[3] + t[4]) * cg(tde, t[3] + t[4], 1, t[5], T2, MT))
                        if ck != 0.0:
                            total += cb * ck * value(bra, ket, J2, T2, jab, tab, jde, tde)
        return total
