"""Pins of the oracle's three-body term (CPU).

The d <= 3 matrix with a synthetic three-body interaction is checked against
an independent route (operator application with explicit fermion signs,
oracle/brute.py), against closed forms (three nucleons of one species: the
matrix is the interaction itself; the identity interaction gives
A(A-1)(A-2)/6 times the identity), against the two-body oracle on d <= 2, and
for symmetry; the generator against its definition in seeded_inputs.
"""
import math

import numpy as np
import pytest

import seeded_inputs as si
from oracle import Oracle, Problem, brute

# (Z, N, nmax, 2M, parity), A >= 3
SMALL3 = [(2, 1, 2, 1, -1), (2, 1, 2, 1, 1), (1, 2, 2, -1, -1), (3, 0, 2, 1, 1), (0, 3, 2, 3, -1),
          (2, 2, 2, 0, 1), (3, 1, 2, 2, -1), (3, 2, 2, 1, 1)]
SEED, SCALE = 0x5EED3, 2.0


def oracle3(p, kind=Oracle.V3_SYNTHETIC, tbme_seed=31, kinetic=0, scale=SCALE):
    o = Oracle(Problem(*p, kinetic=kinetic))
    o.set_tbme(si.tbme_f64(tbme_seed, o.n_tbme) if tbme_seed is not None else np.zeros(o.n_tbme))
    o.set_v3(kind, SEED, scale)
    return o


def v3fn(a, b, c, d, e, f):
    return float(si.v3_synthetic(SEED, [a], [b], [c], [d], [e], [f], scale=SCALE)[0])


def test_generator_matches_its_definition():
    o = oracle3((2, 1, 2, 1, -1))
    rng = np.random.default_rng(1)
    for _ in range(200):
        t = np.sort(rng.choice(480, 3, replace=False))
        q = np.sort(rng.choice(480, 3, replace=False))
        ref = float(si.v3_synthetic(SEED, *t, *q, scale=SCALE))
        assert o.v3(*t, *q) == ref
        assert o.v3(*q, *t) == ref  # symmetric under bra <-> ket
        assert o.v3(t[1], t[0], t[2], *q) == -ref  # antisymmetric in each triple
        assert o.v3(t[0], t[1], t[2], q[2], q[1], q[0]) == -ref
        assert o.v3(t[0], t[0], t[2], *q) == 0.0
    vals = si.v3_synthetic(SEED, *np.sort(rng.integers(0, 480, (3, 20000)), axis=0),
                           *np.sort(rng.integers(0, 480, (3, 20000)), axis=0), scale=1.0)
    assert -1.0 <= vals.min() and vals.max() < 1.0 and abs(vals.mean()) < 0.02 and abs(vals.std() - 3 ** -0.5) < 0.01


@pytest.mark.parametrize("p", SMALL3)
def test_matrix_equals_operator_application(p):
    o = oracle3(p)
    b = brute.BruteBasis(*p)
    Hb = brute.hamiltonian(b, o.tbme_keys(), si.tbme_f64(31, o.n_tbme)) + brute.hamiltonian3(b, v3fn)
    Hc = o.dense3()
    assert np.abs(Hb - Hb.T).max() <= 1e-12
    np.testing.assert_allclose(Hc, Hb, rtol=0, atol=1e-11)


def test_matrix_equals_operator_application_with_kinetic():
    p = (2, 2, 2, 0, 1)
    o = oracle3(p, kinetic=1)
    b = brute.BruteBasis(*p)
    Hb = (brute.hamiltonian(b, o.tbme_keys(), si.tbme_f64(31, o.n_tbme), kinetic=True)
          + brute.hamiltonian3(b, v3fn))
    np.testing.assert_allclose(o.dense3(), Hb, rtol=0, atol=1e-11)


@pytest.mark.parametrize("p", [(3, 0, 2, 1, 1), (0, 3, 4, 3, 1), (3, 0, 3, 1, -1)])
def test_three_nucleons_of_one_species_see_the_interaction_itself(p):
    # |abc> = a+_a a+_b a+_c |0> with a < b < c: <abc|H3|def> = V_{abc,def}
    o = oracle3(p, tbme_seed=None)
    S = o.states()
    occ = [[w * 64 + k for w in range(S.shape[1]) for k in range(64) if (int(S[i, w]) >> k) & 1]
           for i in range(o.dim)]
    sp = 0 if p[0] == 3 else o.n_sps  # combined-index offset of the species
    H = o.dense3()
    for i in range(o.dim):
        a = [sp + (x % (64 * (S.shape[1] // 2))) for x in occ[i]]
        for j in range(o.dim):
            d = [sp + (x % (64 * (S.shape[1] // 2))) for x in occ[j]]
            ref = o.v3(*a, *d) + (sum((o.orbits()[x % o.n_sps][0] + 1.5) * 15.0 for x in a) if i == j else 0.0)
            assert H[i, j] == pytest.approx(ref, abs=1e-12)
            assert o.v3(*a, *d) == float(si.v3_synthetic(SEED, *a, *d, scale=SCALE))


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 2, 2, 1, 1), (3, 3, 2, 0, 1)])
def test_identity_interaction_counts_triples(p):
    # V = s * delta(abc, def): H3 = s * N(N-1)(N-2)/6, on A-nucleon states the
    # constant s * C(A, 3), with no off-diagonal part
    s = 0.75
    o3 = oracle3(p, kind=Oracle.V3_IDENTITY, scale=s)
    o2 = oracle3(p, kind=Oracle.V3_NONE)
    A = p[0] + p[1]
    np.testing.assert_allclose(o3.dense3() - o2.dense3(), s * math.comb(A, 3) * np.eye(o3.dim), rtol=0, atol=1e-12)


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 2, 2, 1, 1), (3, 3, 2, 0, 1)])
def test_without_three_body_it_is_the_two_body_matrix(p):
    o = oracle3(p, kind=Oracle.V3_NONE)
    rp, cols, vals = o.csr()
    counts3, cols3, vals3 = o.rows3(np.arange(o.dim))
    H2 = np.zeros((o.dim, o.dim))
    H2[np.repeat(np.arange(o.dim), np.diff(rp)), cols] = vals
    H3 = np.zeros((o.dim, o.dim))
    H3[np.repeat(np.arange(o.dim), counts3), cols3] = vals3
    np.testing.assert_array_equal(H2, H3)


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 2, 2, 1, 1), (2, 2, 4, 0, 1)])
def test_structure_is_every_pair_within_three(p):
    o = oracle3(p)
    S = o.states()
    counts, cols, _ = o.rows3(np.arange(o.dim), values=False)
    pop = np.vectorize(lambda x: bin(int(x)).count("1"))
    start = 0
    for i in range(o.dim):
        d = pop(S[i:] ^ S[i]).sum(axis=1) // 2
        ref = i + np.nonzero(d <= 3)[0]
        assert np.array_equal(cols[start:start + counts[i]], ref)
        start += counts[i]


@pytest.mark.parametrize("p", [(3, 2, 2, 1, 1), (3, 3, 2, 0, 1)])
def test_symmetric(p):
    o = oracle3(p)
    rng = np.random.default_rng(4)
    for _ in range(300):
        i, j = rng.integers(0, o.dim, 2)
        assert o.element3(i, j) == pytest.approx(o.element3(j, i), abs=1e-12)


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 2, 2, 1, 1), (2, 1, 2, 1, 1)])
def test_full_rows_are_upper_rows_and_their_transpose(p):
    # every element below the diagonal is computed directly; it must equal
    # the stored upper element (the matrix is symmetric)
    o = oracle3(p)
    D = o.dim
    counts, cols, vals = o.rows3(np.arange(D))
    U = np.zeros((D, D))
    U[np.repeat(np.arange(D), counts), cols] = vals
    H = U + np.triu(U, 1).T
    fc, fcols, fvals = o.rows3_full(np.arange(D))
    F = np.zeros((D, D))
    F[np.repeat(np.arange(D), fc), fcols] = fvals
    assert fc.sum() == 2 * counts.sum() - D
    np.testing.assert_allclose(F, H, rtol=0, atol=1e-11)
