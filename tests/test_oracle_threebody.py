"""Pins of the three-body decoupling oracle (CPU): coupling coefficients
against known values and both orthogonality relations, and the transformation
against its closed forms (identity interaction -> identity, Hermiticity,
conservation zeros)."""
import math

import numpy as np
import pytest

import seeded_inputs as si
from oracle.threebody import ThreeBody, cg, channels


def test_cg_known_values():
    s = 1 / math.sqrt(2)
    assert cg(1, 1, 1, -1, 2, 0) == pytest.approx(s)
    assert cg(1, 1, 1, -1, 0, 0) == pytest.approx(s)
    assert cg(1, -1, 1, 1, 0, 0) == pytest.approx(-s)
    assert cg(2, 2, 2, -2, 0, 0) == pytest.approx(1 / math.sqrt(3))
    assert cg(2, 0, 2, 0, 0, 0) == pytest.approx(-1 / math.sqrt(3))
    assert cg(2, 2, 1, -1, 3, 1) == pytest.approx(math.sqrt(1 / 3))
    assert cg(2, 2, 1, -1, 1, 1) == pytest.approx(math.sqrt(2 / 3))
    assert cg(4, 4, 4, -4, 0, 0) == pytest.approx(1 / math.sqrt(5))
    assert cg(1, 1, 1, 1, 2, 2) == 1.0
    assert cg(1, 1, 1, 1, 0, 2) == 0.0  # |M| > J


@pytest.mark.parametrize("j1,j2", [(1, 1), (1, 2), (3, 2), (3, 5), (9, 7), (4, 4)])
def test_cg_orthogonality(j1, j2):
    Js = list(range(abs(j1 - j2), j1 + j2 + 1, 2))
    for M in range(-(j1 + j2), j1 + j2 + 1, 2):
        pairs = [(m1, M - m1) for m1 in range(-j1, j1 + 1, 2) if abs(M - m1) <= j2]
        for J in Js:
            for Jp in Js:
                s = sum(cg(j1, m1, j2, m2, J, M) * cg(j1, m1, j2, m2, Jp, M) for m1, m2 in pairs)
                assert s == pytest.approx(1.0 if (J == Jp and abs(M) <= J) else 0.0, abs=1e-12)
        for a in pairs:
            for b in pairs:
                s = sum(cg(j1, a[0], j2, a[1], J, M) * cg(j1, b[0], j2, b[1], J, M) for J in Js if abs(M) <= J)
                assert s == pytest.approx(1.0 if a == b else 0.0, abs=1e-12)


def identity(bra, ket, J2, T2, jab, tab, jde, tde):
    return 1.0 if (bra, jab, tab) == (ket, jde, tde) else 0.0


@pytest.mark.parametrize("n1,n3", [(2, 2), (3, 3), (4, 4)])
def test_identity_interaction_gives_the_identity(n1, n3):
    # the coupled states of one orbital triple form an orthonormal basis of its
    # m-scheme product states, so the identity stays the identity
    tb = ThreeBody(n1, n3)
    req = si.requests_3b(7, 300, n1, n3)
    for r in req:
        assert tb.element(r, identity) == pytest.approx(1.0 if tuple(r[:3]) == tuple(r[3:]) else 0.0, abs=1e-12)
    for r in req[:150]:
        d = np.concatenate([r[:3], r[:3]])
        assert tb.element(d, identity) == pytest.approx(1.0, abs=1e-12)


def test_hermitian_and_conserving():
    tb = ThreeBody(4, 4)

    def val(*k):
        return si.coupled3b_value(11, *k)

    req = si.requests_3b(8, 150, 4, 4, mismatched=30)
    n_ok = 150
    for r in req[:n_ok]:
        swapped = np.concatenate([r[3:], r[:3]])
        assert tb.element(r, val) == pytest.approx(tb.element(swapped, val), abs=1e-12)
    for r in req[n_ok:]:
        assert tb.element(r, val) == 0.0  # M differs
    assert tb.element([-1, 0, 0, 0, 0, 0], val) == 0.0


def test_channels_count_the_coupled_space():
    # sum over J, T of the channel counts of one triple is the number of its
    # product states with a fixed total projection summed over projections:
    # sum_{J T} (2J+1)(2T+1) n_ch(J, T) = prod (2j+1) * 2^3
    tb = ThreeBody(3, 3)
    for a, b, c in [(0, 1, 2), (3, 3, 1), (2, 4, 0), (5, 5, 5)]:
        if max(a, b, c) >= len(tb.nlj):
            continue
        j = [tb.nlj[x][2] for x in (a, b, c)]
        tot = sum((J + 1) * (T + 1) * len(channels(j[0], j[1], j[2], J, T))
                  for J in range(1, sum(j) + 1, 2) for T in (1, 3))
        assert tot == (j[0] + 1) * (j[1] + 1) * (j[2] + 1) * 8
