"""Property tests of the oracle over random small problems (hypothesis,
derandomized so that every run checks the same cases).

For random (Z, N, Nmax, 2M, parity) with a small basis: the basis equals an
independent enumeration; the stored structure is exactly the pairs within two
(three, with the three-body term) nucleons, found by a direct pairwise scan;
the values are linear in the two-body table and the adjoint satisfies
<G, J V'> = <J^T G, V'>; the matrix is symmetric.
"""
import numpy as np
from hypothesis import HealthCheck, assume, given, settings, strategies as st

import seeded_inputs as si
from oracle import Oracle, Problem, brute

SETTINGS = dict(max_examples=30, deadline=None, derandomize=True,
                suppress_health_check=[HealthCheck.filter_too_much, HealthCheck.too_slow])


@st.composite
def problems(draw, max_dim=1500):
    Z = draw(st.integers(0, 4))
    N = draw(st.integers(0, 4))
    assume(Z + N >= 1)
    nmax = draw(st.integers(0, 4 if Z + N <= 4 else 2))
    two_m = draw(st.integers(-3, 3)) * 2 + (Z + N) % 2
    parity = draw(st.sampled_from([1, -1]))
    p = (Z, N, nmax, two_m, parity)
    o = Oracle(Problem(*p))
    assume(0 < o.dim <= max_dim)
    return p, o


def occupations(o):
    S = o.states()
    return np.array([[(int(w) >> k) & 1 for w in row for k in range(64)] for row in S], dtype=np.int8)


@settings(**SETTINGS)
@given(problems())
def test_basis_and_structure_match_pairwise_scan(po):
    p, o = po
    b = brute.BruteBasis(*p)
    assert b.dim == o.dim
    occ = occupations(o)
    d = (occ[:, None, :] != occ[None, :, :]).sum(axis=2) // 2
    rp, cols, _ = o.csr(values=False)
    counts3, cols3, _ = o.rows3(np.arange(o.dim), values=False)
    for i in range(o.dim):
        assert np.array_equal(cols[rp[i]:rp[i + 1]], i + np.nonzero(d[i, i:] <= 2)[0])
    assert np.array_equal(counts3, [(d[i, i:] <= 3).sum() for i in range(o.dim)])
    assert np.array_equal(np.concatenate([i + np.nonzero(d[i, i:] <= 3)[0] for i in range(o.dim)]), cols3)


@settings(**SETTINGS)
@given(problems(), st.integers(0, 2**31 - 1))
def test_linearity_and_adjoint_dot_product(po, seed):
    p, o = po
    assume(o.n_tbme > 0)
    rng = np.random.default_rng(seed)
    V = rng.standard_normal(o.n_tbme)
    o.set_tbme(np.zeros(o.n_tbme))
    _, _, v0 = o.csr()
    o.set_tbme(V)
    rp, cols, v1 = o.csr()
    o.set_tbme(2.0 * V)
    _, _, v2 = o.csr()
    np.testing.assert_allclose(v2 - v0, 2.0 * (v1 - v0), rtol=1e-12, atol=1e-12)
    G = rng.standard_normal(len(cols))
    g = o.grad_rows(np.arange(o.dim), G)
    lhs, rhs = float(G @ (v1 - v0)), float(g @ V)
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))


@settings(**SETTINGS)
@given(problems(max_dim=400), st.integers(0, 2**31 - 1))
def test_symmetric_with_three_body_term(po, seed):
    p, o = po
    o.set_tbme(si.tbme_f64(seed % 1000, o.n_tbme))
    o.set_v3(Oracle.V3_SYNTHETIC, seed, 1.0)
    H = np.array([[o.element3(i, j) for j in range(o.dim)] for i in range(o.dim)])
    np.testing.assert_allclose(H, H.T, rtol=0, atol=1e-11)
