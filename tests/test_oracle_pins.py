"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against mathematics that does not go through its
own code: a hand count, a generating-function count, a literature dimension, an
independent operator-application build, closed forms (A = 2; one-body only),
symmetry, conservation laws, and exact linearity of the two-body dependence.
"""
import itertools

import numpy as np
from scipy.integrate import quad
from scipy.special import genlaguerre
import pytest

import seeded_inputs as si
from oracle import Oracle, Problem, brute, dimcount

SMALL = [
    (2, 2, 2, 0, 1),
    (1, 1, 2, 0, 1),
    (2, 1, 2, 1, 1),
    (1, 2, 2, -1, -1),
    (3, 1, 2, 0, 1),
    (2, 0, 4, 0, 1),
    (0, 3, 2, 1, 1),
    (2, 2, 2, 2, -1),
    (3, 2, 2, 1, 1),
    (2, 2, 0, 0, 1),
    (1, 1, 4, 2, 1),
]


def _ndiff(a, b):
    return sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)) // 2


# ---------------------------------------------------------------- dimension


def test_he4_nmax2_dimension_by_hand():
    # 4He, Nmax=2, 2M=0, + : the positive-parity states with <= 2 quanta are
    #   (0s)^4                                     1
    #   one p-proton + one p-neutron (0s holes)    sum_M c(M) c(-M) with
    #     c = #(s,p) proton pairs of 2M = -4..4 = 1,3,4,3,1  ->  1+9+16+9+1 = 36
    #   two quanta in the protons, neutrons (0s)^2: p^2 with 2M=0 (5) plus
    #     s x (sd) with 2M=0 (6)                   11
    #   the same in the neutrons                   11
    o = Oracle(Problem(2, 2, 2, 0, 1))
    assert o.dim == 1 + 36 + 11 + 11 == 59
    assert o.n_sps == 20 and o.n_words == 1


def test_li6_nmax6_literature_dimension():
    # 6Li, Nmax = 6, M = 0, natural parity: the M-scheme dimension quoted in the
    # No-Core Shell Model literature is 197,822.
    o = Oracle(Problem(3, 3, 6, 0, 1))
    assert o.dim == 197822


@pytest.mark.parametrize(
    "p",
    SMALL
    + [(3, 3, 6, 2, 1), (5, 5, 4, 0, 1), (4, 4, 4, 0, 1), (2, 3, 6, 1, 1), (4, 2, 2, 0, 1)],
)
def test_dimension_generating_function(p):
    o = Oracle(Problem(*p))
    D = dimcount.dimension(*p, o.shell_max, brute.n0(p[0]), brute.n0(p[1]))
    assert o.dim == D


def test_named_workload_sizes():
    # orbit counts follow from the shell cut S = max(Ntop(Z), Ntop(N)) + Nmax:
    # sum_{N<=S} (N+1)(N+2) orbits per species
    for name, S, nsps, W in [("he4_nmax2", 2, 20, 1), ("li6_nmax6", 7, 240, 4),
                             ("b10_nmax4", 5, 112, 2)]:
        o = Oracle(Problem(*si.WORKLOADS[name]["problem"]))
        assert (o.shell_max, o.n_sps, o.n_words) == (S, nsps, W)
        assert nsps == sum((n + 1) * (n + 2) for n in range(S + 1))


# ---------------------------------------------------------------- basis


@pytest.mark.parametrize("p", SMALL)
def test_basis_matches_independent_enumeration(p):
    o = Oracle(Problem(*p))
    b = brute.BruteBasis(*p)
    assert b.dim == o.dim
    assert np.array_equal(b.state_words(o.n_words), o.states())


@pytest.mark.parametrize("p", SMALL + [(3, 3, 4, 0, 1)])
def test_basis_conserves_m_and_parity(p):
    o = Oracle(Problem(*p))
    orb = o.orbits()
    S = o.states()
    W = o.n_words
    seen = set()
    for row in S:
        occ = [k for k in range(o.n_sps) if (int(row[k // 64]) >> (k % 64)) & 1]
        occn = [k for k in range(o.n_sps) if (int(row[W + k // 64]) >> (k % 64)) & 1]
        assert len(occ) == p[0] and len(occn) == p[1]
        m2 = sum(orb[k, 4] for k in occ) + sum(orb[k, 4] for k in occn)
        nq = sum(orb[k, 0] for k in occ) + sum(orb[k, 0] for k in occn)
        assert m2 == p[3]
        assert (1 if nq % 2 == 0 else -1) == p[4]
        assert nq <= o.n0 + p[2]
        seen.add(tuple(int(x) for x in row))
    assert len(seen) == o.dim


def test_orbit_order():
    o = Oracle(Problem(3, 3, 2, 0, 1))
    orb = o.orbits()
    keys = [tuple(r[[0, 2, 3, 4]]) for r in orb]  # N, l, 2j, 2m
    assert keys == sorted(keys)
    for N, n, l, j2, m2 in orb:
        assert N == 2 * n + l and abs(j2 - 2 * l) == 1 and abs(m2) <= j2 and (m2 - j2) % 2 == 0


# ---------------------------------------------------------------- two-body table


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 2, 2, 1, 1), (2, 0, 4, 0, 1), (0, 3, 2, 1, 1),
                               (3, 3, 2, 0, 1)])
def test_tbme_table_structure(p):
    o = Oracle(Problem(*p))
    orb = o.orbits()
    n = o.n_sps
    K = o.tbme_keys()
    assert len({tuple(k) for k in K}) == len(K)

    def cls(a, b):  # number of neutrons in the pair -> 0 pp, 1 pn, 2 nn
        return int(a >= n) + int(b >= n)

    def q(a):
        return orb[a % n]

    n0 = brute.n0
    for a, b, c, d in K:
        assert a < b and c < d and (a, b) <= (c, d)
        assert cls(a, b) == cls(c, d)
        assert q(a)[4] + q(b)[4] == q(c)[4] + q(d)[4]
        assert (q(a)[0] + q(b)[0]) % 2 == (q(c)[0] + q(d)[0]) % 2
        z = 2 - cls(a, b)
        lim = o.n0 - (n0(p[0] - z) + n0(p[1] - (2 - z))) + p[2]
        assert q(a)[0] + q(b)[0] <= lim and q(c)[0] + q(d)[0] <= lim
    # independent count: sum over sectors of s(s+1)/2
    sectors = {}
    for a in range(2 * n):
        for b in range(a + 1, 2 * n):
            c = cls(a, b)
            z = 2 - c
            if p[0] - z < 0 or p[1] - (2 - z) < 0:
                continue
            lim = o.n0 - (n0(p[0] - z) + n0(p[1] - (2 - z))) + p[2]
            if q(a)[0] + q(b)[0] > lim:
                continue
            key = (c, q(a)[4] + q(b)[4], (q(a)[0] + q(b)[0]) % 2)
            sectors[key] = sectors.get(key, 0) + 1
    assert o.n_tbme == sum(s * (s + 1) // 2 for s in sectors.values())
    # table order: sector (class, 2M, parity) non-decreasing; pairs inside it lexicographic
    sec = [(cls(a, b), q(a)[4] + q(b)[4], (q(a)[0] + q(b)[0]) % 2) for a, b, _, _ in K]
    assert sec == sorted(sec)
    for t in range(1, len(K)):
        if sec[t] == sec[t - 1]:
            assert tuple(K[t - 1]) < tuple(K[t])


def test_named_table_sizes():
    assert Oracle(Problem(2, 2, 2, 0, 1)).n_tbme == 1298


def test_vget_antisymmetry():
    o = Oracle(Problem(2, 2, 2, 0, 1))
    v = si.tbme_f64(0, o.n_tbme)
    o.set_tbme(v)
    K = o.tbme_keys()
    rng = np.random.default_rng(7)
    for t in rng.choice(len(K), 50, replace=False):
        a, b, c, d = (int(x) for x in K[t])
        assert o.vget(a, b, c, d) == v[t]
        assert o.vget(b, a, c, d) == -v[t]
        assert o.vget(a, b, d, c) == -v[t]
        assert o.vget(d, c, b, a) == v[t]
        assert o.vget(c, d, a, b) == v[t]


# ---------------------------------------------------------------- matrix


@pytest.mark.parametrize("p", SMALL)
def test_matrix_equals_operator_application(p):
    o = Oracle(Problem(*p))
    v = si.tbme_f64(11, o.n_tbme)
    o.set_tbme(v)
    Hb = brute.hamiltonian(brute.BruteBasis(*p), o.tbme_keys(), v)
    Hc = o.dense()
    assert np.abs(Hb - Hb.T).max() == 0.0
    np.testing.assert_allclose(Hc, Hb, rtol=0, atol=1e-12)


def test_matrix_equals_operator_application_larger():
    p = (2, 2, 4, 0, 1)  # D = 952
    o = Oracle(Problem(*p))
    v = si.tbme_f64(12, o.n_tbme)
    o.set_tbme(v)
    Hb = brute.hamiltonian(brute.BruteBasis(*p), o.tbme_keys(), v)
    np.testing.assert_allclose(o.dense(), Hb, rtol=0, atol=1e-12)


@pytest.mark.parametrize("p", SMALL + [(2, 2, 4, 0, 1)])
def test_structure_is_every_pair_within_two(p):
    o = Oracle(Problem(*p))
    S = o.states()
    rp, cols, _ = o.csr(values=False)
    for i in range(o.dim):
        want = [j for j in range(i, o.dim) if _ndiff(S[i], S[j]) <= 2]
        assert list(cols[rp[i]:rp[i + 1]]) == want


def test_he4_nnz_by_class():
    # stored entries of the upper triangle by (proton, neutron) difference
    o = Oracle(Problem(2, 2, 2, 0, 1))
    S = o.states()
    rp, cols, _ = o.csr(values=False)
    assert rp[-1] == 875
    cnt = {}
    for i in range(o.dim):
        for j in cols[rp[i]:rp[i + 1]]:
            dp = bin(int(S[i, 0]) ^ int(S[j, 0])).count("1") // 2
            dn = bin(int(S[i, 1]) ^ int(S[j, 1])).count("1") // 2
            cnt[(dp, dn)] = cnt.get((dp, dn), 0) + 1
    assert cnt == {(0, 0): 59, (1, 0): 30, (0, 1): 30, (2, 0): 78, (0, 2): 78, (1, 1): 600}


def test_two_nucleon_closed_form():
    # A = 2: every state is a pair |ab>, H_(ab),(cd) = V_ab,cd + delta (e_a + e_b)
    p = (1, 1, 2, 0, 1)
    o = Oracle(Problem(*p))
    v = si.tbme_f64(5, o.n_tbme)
    o.set_tbme(v)
    H = o.dense()
    rp, cols, _ = o.csr(values=False)
    assert rp[-1] == o.dim * (o.dim + 1) // 2  # dense upper triangle
    S = o.states()
    orb = o.orbits()
    n = o.n_sps

    def pair(i):
        a = int(S[i, 0]).bit_length() - 1
        b = int(S[i, 1]).bit_length() - 1
        return a, n + b

    for i in range(o.dim):
        for j in range(o.dim):
            a, b = pair(i)
            c, d = pair(j)
            want = o.vget(a, b, c, d)
            if i == j:
                want += 15.0 * (orb[a % n, 0] + orb[b % n, 0] + 3)
            assert H[i, j] == pytest.approx(want, abs=1e-12)


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 2, 2, 1, 1), (3, 3, 2, 0, 1), (0, 3, 2, 1, 1)])
def test_one_body_closed_form(p):
    # V = 0: diagonal 15 (Nq + 3A/2) exactly, every off-diagonal stored entry 0
    o = Oracle(Problem(*p))
    o.set_tbme(None)
    rp, cols, vals = o.csr()
    S = o.states()
    orb = o.orbits()
    W = o.n_words
    A = p[0] + p[1]
    for i in range(o.dim):
        nq = 0
        for sp in range(2):
            for k in range(o.n_sps):
                if (int(S[i, sp * W + k // 64]) >> (k % 64)) & 1:
                    nq += orb[k, 0]
        seg = slice(rp[i], rp[i + 1])
        assert cols[seg][0] == i
        assert vals[seg][0] == 15.0 * (nq + 1.5 * A)
        assert np.all(vals[seg][1:] == 0.0)


def test_lower_triangle_symmetric():
    # H_ji computed with the roles of bra and ket exchanged equals H_ij
    o = Oracle(Problem(3, 3, 2, 0, 1))
    o.set_tbme(si.tbme_f64(9, o.n_tbme))
    rp, cols, vals = o.csr()
    rng = np.random.default_rng(3)
    for i in rng.choice(o.dim, 40, replace=False):
        for k in range(rp[i], rp[i + 1]):
            assert o.element(cols[k], i) == pytest.approx(vals[k], abs=1e-12)


def test_spectrum_invariant_under_orbit_relabeling():
    # A convention-free check of the phases: relabel the proton orbits by a
    # random permutation pi (a neutron orbit keeps its label), carry the
    # interaction along (V'_{pi a pi b, pi c pi d} = V_{ab,cd}), build the
    # relabelled matrix by operator application on the relabelled basis, and
    # compare spectra with the oracle's matrix.
    p = (2, 2, 2, 0, 1)
    o = Oracle(Problem(*p))
    v = si.tbme_f64(21, o.n_tbme)
    o.set_tbme(v)
    ev = np.linalg.eigvalsh(o.dense())
    b = brute.BruteBasis(*p)
    n = o.n_sps
    rng = np.random.default_rng(4)
    perm = rng.permutation(n)  # proton relabeling only (M, N of each orbit carried along)
    lab = lambda a: int(perm[a]) if a < n else a
    K = o.tbme_keys()
    keys2, vals2 = [], []
    for (a, b_, c, d), x in zip(K, v):
        A, B, C, Dd = lab(a), lab(b_), lab(c), lab(d)
        s = 1.0
        if A > B:
            A, B, s = B, A, -s
        if C > Dd:
            C, Dd, s = Dd, C, -s
        keys2.append((A, B, C, Dd))
        vals2.append(s * x)
    b.states = [tuple(sorted(lab(a) for a in st)) for st in b.states]
    b.index = {s: i for i, s in enumerate(b.states)}
    spe = b.spe
    inv = {int(perm[a]): a for a in range(n)}
    b.spe = lambda a, kinetic=False: spe(inv[a] if a < n else a, kinetic)
    H2 = brute.hamiltonian(b, np.array(keys2), np.array(vals2))
    np.testing.assert_allclose(np.linalg.eigvalsh(H2), ev, rtol=0, atol=1e-10)


# ---------------------------------------------------------------- gradient


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 2, 2, 1, 1)])
def test_gradient_finite_difference_exact(p):
    # L(V) = sum_e G_e H_e(V) is affine in V, so a central difference is exact
    o = Oracle(Problem(*p))
    v = si.tbme_f64(2, o.n_tbme)
    rows = np.arange(o.dim)
    o.set_tbme(v)
    _, cols, vals = o.rows(rows)
    counts = o.row_counts(rows)
    ri = np.repeat(rows, counts)
    ps = si.psi(104, o.dim)
    G = si.upstream_grad(ps, ri, cols).astype(np.float64)
    g = o.grad_rows(rows, G)
    h = 1e-3
    for k in si.fd_keys(o.n_tbme, 32):
        vp, vm = v.copy(), v.copy()
        vp[k] += h
        vm[k] -= h
        o.set_tbme(vp)
        Lp = G @ o.rows(rows)[2]
        o.set_tbme(vm)
        Lm = G @ o.rows(rows)[2]
        assert (Lp - Lm) / (2 * h) == pytest.approx(g[k], abs=1e-8)


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 3, 2, 0, 1)])
def test_gradient_dot_product_and_euler(p):
    o = Oracle(Problem(*p))
    rows = np.arange(o.dim)
    counts = o.row_counts(rows)
    o.set_tbme(None)
    _, cols, onebody = o.rows(rows)
    ri = np.repeat(rows, counts)
    G = si.upstream_grad(si.psi(7, o.dim), ri, cols).astype(np.float64)
    g = o.grad_rows(rows, G)
    # <G, J V'> = <J^T G, V'> with J V' = H(V') - H(0)
    vprime = np.random.default_rng(8).standard_normal(o.n_tbme)
    o.set_tbme(vprime)
    JV = o.rows(rows)[2] - onebody
    assert G @ JV == pytest.approx(g @ vprime, rel=1e-12, abs=1e-12)
    # Euler: sum_k g_k V_k = sum_e G_e (H_e - onebody_e)
    v = si.tbme_f64(1, o.n_tbme)
    o.set_tbme(v)
    assert g @ v == pytest.approx(G @ (o.rows(rows)[2] - onebody), rel=1e-12, abs=1e-12)


def test_gradient_row_subset_is_additive():
    # the gradient of a row subset is the restriction of the full sum: summing
    # the gradients of a partition of the rows gives the full gradient
    o = Oracle(Problem(2, 2, 2, 0, 1))
    rows = np.arange(o.dim)
    counts = o.row_counts(rows)
    _, cols, _ = o.rows(rows, values=False)
    ri = np.repeat(rows, counts)
    G = si.upstream_grad(si.psi(5, o.dim), ri, cols).astype(np.float64)
    full = o.grad_rows(rows, G)
    off = np.concatenate([[0], np.cumsum(counts)])
    parts = np.zeros_like(full)
    for chunk in np.array_split(rows, 5):
        Gc = np.concatenate([G[off[i]:off[i + 1]] for i in chunk])
        parts += o.grad_rows(chunk, Gc)
    np.testing.assert_allclose(parts, full, rtol=1e-13, atol=1e-15)


# ------------------------------------------------------------------ full matrix and lowest eigenpair


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 2, 2, 1, 1), (1, 1, 4, 2, 1), (0, 3, 2, 1, 1)])
def test_full_rows_are_upper_rows_plus_transposed_entries(p):
    o = Oracle(Problem(*p))
    o.set_tbme(si.tbme_f64(7, o.n_tbme))
    rows = np.arange(o.dim)
    cu, colu, valu = o.rows(rows)
    cf, colf, valf = o.rows_full(rows)
    assert int(cf.sum()) == 2 * int(cu.sum()) - o.dim
    # upper part of each full row is exactly the stored row
    ru = np.repeat(rows, cu)
    rf = np.repeat(rows, cf)
    up = colf >= rf
    assert np.array_equal(colf[up], colu) and np.array_equal(valf[up], valu)
    # lower part: row i, column j < i equals the stored entry (j, i), computed
    # independently (roles swapped) -- symmetric to rounding
    lower = {(int(j), int(i)): v for i, j, v in zip(rf[~up], colf[~up], valf[~up])}
    stored = {(int(i), int(j)): v for i, j, v in zip(ru, colu, valu) if i != j}
    assert lower.keys() == stored.keys()
    assert max(abs(lower[k] - stored[k]) for k in stored) <= 1e-12 * max(1.0, np.abs(valu).max())


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 3, 2, 0, 1), (2, 3, 2, 1, 1)])
def test_lowest_eigenvalue_one_body_closed_form(p):
    # with no two-body term H is diagonal: the lowest eigenvalue is the
    # smallest single-particle sum, 15 (Nq_min + 3A/2) with Nq_min = N0 for a
    # natural-parity space
    o = Oracle(Problem(*p))
    o.set_tbme(np.zeros(o.n_tbme))
    E, v = o.lowest_eigenpair()
    A = p[0] + p[1]

    def n0(X):  # quanta of the lowest filling: shells of (N+1)(N+2) states from the bottom
        s, N, left = 0, 0, X
        while left > 0:
            take = min(left, (N + 1) * (N + 2))
            s, left, N = s + take * N, left - take, N + 1
        return s

    N0 = n0(p[0]) + n0(p[1])
    nq_min = N0 if ((N0 % 2 == 0) == (p[4] == 1)) else N0 + 1
    assert E == pytest.approx(15.0 * (nq_min + 1.5 * A), abs=1e-9)


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 2, 2, 1, 1)])
def test_lowest_eigenpair_residual(p):
    o = Oracle(Problem(*p))
    o.set_tbme(si.tbme_f64(8, o.n_tbme))
    H = o.dense()
    E, v = o.lowest_eigenpair()
    assert abs(np.linalg.norm(v) - 1.0) < 1e-12
    assert np.linalg.norm(H @ v - E * v) <= 1e-10 * abs(E)
    assert E == pytest.approx(float(v @ H @ v), rel=1e-13)
    # variational: below every diagonal element
    assert E <= H.diagonal().min() + 1e-9


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 2, 2, 1, 1)])
def test_hellmann_feynman_matches_eigenvalue_differences(p):
    # dE/dV_k from the adjoint with upstream psi_i psi_j (doubled off the
    # diagonal) equals the central difference of the lowest eigenvalue
    o = Oracle(Problem(*p))
    V = si.tbme_f64(9, o.n_tbme)
    o.set_tbme(V)
    E, psi = o.lowest_eigenpair()
    w, _ = np.linalg.eigh(o.dense())
    assert w[1] - w[0] > 1e-3  # nondegenerate ground state
    g = o.hellmann_feynman(psi)
    keys = np.random.default_rng(10).choice(o.n_tbme, size=12, replace=False)
    h = 1e-4
    for k in keys:
        Vp, Vm = V.copy(), V.copy()
        Vp[k] += h
        Vm[k] -= h
        o.set_tbme(Vp)
        Ep, _ = o.lowest_eigenpair()
        o.set_tbme(Vm)
        Em, _ = o.lowest_eigenpair()
        assert (Ep - Em) / (2 * h) == pytest.approx(g[k], abs=1e-6 * max(1.0, np.abs(g).max()))
    o.set_tbme(V)


# ------------------------------------------------------------------ off-diagonal kinetic one-body term


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (1, 1, 4, 2, 1), (3, 2, 2, 1, 1), (2, 1, 4, 1, 1), (0, 3, 2, 1, 1),
                               (2, 2, 4, 0, 1)])
def test_kinetic_matrix_equals_operator_application(p):
    o = Oracle(Problem(*p, kinetic=1))
    v = si.tbme_f64(12, o.n_tbme)
    o.set_tbme(v)
    H = o.dense()
    Hb = brute.hamiltonian(brute.BruteBasis(*p), o.tbme_keys(), v, kinetic=True)
    assert np.abs(H - Hb).max() <= 1e-12 * max(1.0, np.abs(Hb).max())
    # the term changes the matrix where the space holds states two quanta
    # apart (a radial excitation n -> n + 1); otherwise it must vanish
    o0 = Oracle(Problem(*p))
    o0.set_tbme(v)
    words = o.states()
    nq = set()
    orbs = brute.orbits(o.shell_max)
    for row in words:
        q = 0
        for sp in range(2):
            for w in range(o.n_words):
                x = int(row[sp * o.n_words + w])
                while x:
                    b = (x & -x).bit_length() - 1
                    x &= x - 1
                    q += orbs[w * 64 + b][0]
        nq.add(q)
    # the diagonal one-body part is halved: (hw/2)(N + 3/2) per orbit
    H0 = o0.dense()
    off = H - H0
    np.fill_diagonal(off, 0.0)
    if len(nq) > 1:
        assert np.abs(off).max() > 1.0
    else:
        assert np.abs(off).max() == 0.0
    o00 = Oracle(Problem(*p))
    o00.set_tbme(np.zeros(o00.n_tbme))
    assert np.abs(np.diag(H) - np.diag(H0) + 0.5 * np.diag(o00.dense())).max() <= 1e-9


def _oscillator_radial(n, l):
    """Oscillator radial function R_nl(r) (lengths in oscillator units) and
    its derivative, normalized by quadrature and positive near the origin:
    r^l exp(-r^2/2) L_n^(l+1/2)(r^2) with scipy's generalized Laguerre
    polynomial."""
    L = genlaguerre(n, l + 0.5)
    dL = L.deriv()

    def f(r):
        return r ** l * np.exp(-0.5 * r * r) * L(r * r)

    def df(r):
        lead = l * r ** (l - 1) if l > 0 else 0.0
        return np.exp(-0.5 * r * r) * ((lead - r ** (l + 1)) * L(r * r) + 2.0 * r ** (l + 1) * dL(r * r))

    norm = np.sqrt(quad(lambda r: (f(r) * r) ** 2, 0.0, np.inf, limit=200)[0])
    return (lambda r: f(r) / norm), (lambda r: df(r) / norm)


def _kinetic_quadrature(n1, n2, l, hw):
    """<n1 l|T|n2 l> for T = -(hw/2) nabla^2 in oscillator units, as the
    quadratic form (hw/2) int (R1' R2' + l(l+1) R1 R2 / r^2) r^2 dr."""
    f1, d1 = _oscillator_radial(n1, l)
    f2, d2 = _oscillator_radial(n2, l)
    v = quad(lambda r: d1(r) * d2(r) * r * r + l * (l + 1) * f1(r) * f2(r), 0.0, np.inf, limit=200)[0]
    return 0.5 * hw * v


@pytest.mark.parametrize("parity", [1, -1])
def test_kinetic_single_nucleon_equals_quadrature(parity):
    # One proton in shells 0..7 (every (n, l) the workloads reach: 6Li Nmax=6
    # and the batch go up to shell 7): the matrix is the one-body operator
    # itself, here the kinetic energy T of the oscillator orbits.  Every
    # element, diagonal and off-diagonal, against T computed by quadrature
    # of the radial functions (no closed form used): this fails for a
    # missing hw/2, for n + l + 1/2 in place of n + l + 3/2, or for a
    # diagonal of (N + 3/2) hw.
    p = (1, 0, 7, 1, parity)
    o = Oracle(Problem(*p, kinetic=1))
    o.set_tbme(np.zeros(o.n_tbme))
    H = o.dense()
    orbs = brute.orbits(o.shell_max)
    want_par = 0 if parity == 1 else 1
    states = [a for a, (N, n, l, j2, m2) in enumerate(orbs) if m2 == 1 and N % 2 == want_par and N <= 7]
    assert o.dim == len(states)
    assert max(orbs[a][0] for a in states) >= 6
    T = np.zeros((o.dim, o.dim))
    cache = {}
    for x, a in enumerate(states):
        for y, b in enumerate(states):
            Na, na, la, ja, ma = orbs[a]
            Nb, nb, lb, jb, mb = orbs[b]
            if (la, ja, ma) != (lb, jb, mb):
                continue  # T is a scalar: no element between different (l, j, m)
            key = (min(na, nb), max(na, nb), la)
            if key not in cache:
                cache[key] = _kinetic_quadrature(key[0], key[1], la, 15.0)
            T[x, y] = cache[key]
    # the basis order of one proton is the orbit order (colex of one bit)
    assert np.abs(H - T).max() <= 1e-9 * np.abs(T).max()
    # the quadrature itself sees no element two radial quanta apart
    assert abs(_kinetic_quadrature(0, 2, 1, 15.0)) < 1e-9


def test_kinetic_term_is_oscillator_energy_minus_potential():
    # the same one-nucleon matrix, rebuilt from h_HO = T + r^2/2 hw: T equals
    # the oscillator energy on the diagonal minus (hw/2) <r^2>, with <r^2>
    # by quadrature (a second route to T, through the potential)
    p = (1, 0, 6, 1, 1)
    o = Oracle(Problem(*p, kinetic=1))
    o.set_tbme(np.zeros(o.n_tbme))
    H = o.dense()
    orbs = brute.orbits(o.shell_max)
    states = [a for a, (N, n, l, j2, m2) in enumerate(orbs) if m2 == 1 and N % 2 == 0 and N <= 6]
    for x, a in enumerate(states):
        for y, b in enumerate(states):
            Na, na, la, ja, ma = orbs[a]
            Nb, nb, lb, jb, mb = orbs[b]
            if (la, ja, ma) != (lb, jb, mb):
                assert H[x, y] == 0.0
                continue
            f1, _ = _oscillator_radial(na, la)
            f2, _ = _oscillator_radial(nb, la)
            r2 = quad(lambda r: f1(r) * f2(r) * r ** 4, 0.0, np.inf, limit=200)[0]
            want = (Na + 1.5) * 15.0 * (a == b) - 0.5 * 15.0 * r2
            assert abs(H[x, y] - want) <= 1e-9 * 15.0 * (Na + 1.5)


def test_kinetic_leaves_the_gradient_unchanged():
    # the one-body term does not depend on the two-body table
    p = (3, 2, 2, 1, 1)
    o1, o0 = Oracle(Problem(*p, kinetic=1)), Oracle(Problem(*p))
    v = si.tbme_f64(13, o1.n_tbme)
    o1.set_tbme(v)
    o0.set_tbme(v)
    rows = np.arange(o1.dim)
    counts, cols, _ = o1.rows(rows, values=False)
    G = np.random.default_rng(3).standard_normal(int(counts.sum()))
    assert np.array_equal(o1.grad_rows(rows, G), o0.grad_rows(rows, G))
