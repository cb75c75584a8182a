"""libci host-side checks that need no GPU.

The library loads, exports every symbol include/ci.h declares, and its host
planning (basis sizes, two-body key list) equals the oracle's; validation
errors are raised before any device call.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1412_5989_amd as ci
import seeded_inputs as si
from oracle import Oracle, Problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "ci.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ci_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = ci.load_library()
    decl = declared_symbols()
    assert decl, "no declarations found"
    assert sorted(ci.EXPORTS) == decl
    for name in decl:
        assert hasattr(L, name), name


PLAN = [(2, 2, 2, 0, 1), (1, 1, 2, 0, 1), (3, 3, 6, 2, 1), (5, 5, 4, 0, 1), (2, 3, 6, 1, 1),
        (0, 3, 2, 1, 1), (2, 0, 4, 0, 1), (3, 4, 4, 1, -1), (2, 2, 0, 0, -1)]


@pytest.mark.parametrize("p", PLAN)
def test_plan_matches_oracle(p):
    info = ci.ci_basis_plan([p])[0]
    o = Oracle(Problem(*p))
    assert (info["shell_max"], info["n_sps"], info["n_words"], info["n0"]) == (
        o.shell_max, o.n_sps, o.n_words, o.n0)
    assert (info["n_pkeys"], info["n_nkeys"], info["n_blocks"]) == (o.n_pkeys, o.n_nkeys, o.n_blocks)
    assert (info["n_psd"], info["n_nsd"], info["dim"], info["n_tbme"]) == (
        o.n_psd, o.n_nsd, o.dim, o.n_tbme)


@pytest.mark.parametrize("p", PLAN[:7])
def test_tbme_keys_match_oracle(p):
    assert np.array_equal(ci.ci_tbme_keys(p), Oracle(Problem(*p)).tbme_keys())


def test_batch_plan_offsets():
    probs, _, _ = si.batch_problems()
    info = ci.ci_basis_plan(probs)
    R = T = 0
    for i in info:
        assert i["row_ptr_offset"] == R and i["tbme_offset"] == T
        R += i["dim"] + 1
        T += i["n_tbme"]


@pytest.mark.parametrize("bad", [(-1, 2, 2, 0, 1), (0, 0, 2, 0, 1), (2, 2, -1, 0, 1), (2, 2, 2, 0, 0),
                                 (2, 2, 2, 1, 1), (2, 1, 2, 0, 1)])
def test_invalid_problem(bad):
    with pytest.raises(ci.CIError) as e:
        ci.ci_basis_plan([bad])
    assert e.value.code == ci.CI_EINVAL


def test_unsupported_problem():
    # 4He with Nmax = 8 needs shells 0..8 = 330 orbits per species (> 256)
    with pytest.raises(ci.CIError) as e:
        ci.ci_basis_plan([(2, 2, 8, 0, 1)])
    assert e.value.code == ci.CI_EUNSUPPORTED


def test_tbme_keys_capacity():
    L = ci.load_library()
    arr, _ = ci._problems([(2, 2, 2, 0, 1)])
    buf = np.zeros((10, 4), np.int32)
    rc = L.ci_tbme_keys(arr, buf.ctypes.data_as(ci.ctypes.c_void_p), 10)
    assert rc == ci.CI_ESPACE


def test_argument_errors_before_any_device_call():
    # null handles and short buffers are refused on the host
    L = ci.load_library()
    c = ci.ctypes
    d = c.c_double()
    assert L.ci_probe_ceilings(None, 1 << 30, c.byref(d), c.byref(d), None) == ci.CI_EINVAL
    # a non-null placeholder address is never dereferenced: the size check comes first
    assert L.ci_probe_ceilings(c.c_void_p(256), 1 << 20, c.byref(d), c.byref(d), None) == ci.CI_ESPACE
    t = ci.ci_tuning()
    assert L.ci_basis_get_tuning(None, c.byref(t)) == ci.CI_EINVAL
    assert L.ci_basis_set_tuning(None, c.byref(t)) == ci.CI_EINVAL
    assert L.ci_hamiltonian_tune(None, None, None, None, None, None, None, None, None, 0, 1, None) == ci.CI_EINVAL
    assert L.ci_hamiltonian_fill(None, None, None, None, None, None) == ci.CI_EINVAL
    assert L.ci_hamiltonian_vjp(None, None, None, None, None, 0, None) == ci.CI_EINVAL
    assert L.ci_hamiltonian_count(None, None, None, None) == ci.CI_EINVAL
    assert L.ci_hamiltonian_fill_keys(None, None, None, None, None, None, None) == ci.CI_EINVAL
    assert L.ci_hamiltonian_vjp_keys(None, None, None, None, None, None, 0, None) == ci.CI_EINVAL
    assert L.ci_vjp_work_bytes(None) == 0 and L.ci_basis_count(None) == 0


def test_build_size_query_is_host_only():
    # arena = NULL: the size query plans on the host and needs no device; a
    # short arena is refused before any device call (the placeholder address
    # is never touched), and so are the list calls without a handle
    L = ci.load_library()
    c = ci.ctypes
    for probs in ([(3, 3, 6, 2, 1)], [(2, 2, 2, 0, 1), (2, 3, 4, 1, 1), (2, 2, 2, 0, 1)]):
        arr, n = ci._problems(probs)
        info = (ci.ci_basis_info * n)()
        assert L.ci_basis_build(arr, n, info, None, 0, None, None) == ci.CI_OK
        need = info[0].arena_bytes
        assert need > 0 and all(info[k].arena_bytes == need for k in range(n))
        assert all(info[k].n_tbme == -1 and info[k].list_bytes == -1 for k in range(n))
        plan = ci.ci_basis_plan(probs)
        for k in range(n):
            assert info[k].dim == plan[k]["dim"] and info[k].n_blocks == plan[k]["n_blocks"]
            assert plan[k]["arena_bytes"] == need
        h = c.c_void_p()
        assert L.ci_basis_build(arr, n, info, c.c_void_p(256), need - 1, c.byref(h), None) == ci.CI_ESPACE
        assert not h.value
        assert str(need) in L.ci_last_error().decode()
    sz = c.c_size_t()
    assert L.ci_basis_list_bytes(None, c.byref(sz), None) == ci.CI_EINVAL
    assert L.ci_basis_build_lists(None, None, 0, None) == ci.CI_EINVAL


def test_kinetic_flag_validation():
    with pytest.raises(ci.CIError) as e:
        ci.ci_basis_plan([(2, 2, 2, 0, 1, ci.HW_MEV, 2)])
    assert e.value.code == ci.CI_EINVAL
    a = ci.ci_basis_plan([(2, 2, 2, 0, 1, ci.HW_MEV, 1)])[0]
    b = ci.ci_basis_plan([(2, 2, 2, 0, 1)])[0]
    assert a == b  # the one-body term changes values, not sizes


@pytest.mark.parametrize("n1,n3", [(2, 2), (3, 3), (4, 4)])
def test_threebody_layout_size_matches_the_oracle_count(n1, n3):
    # the coupled input holds one block per equal-parity triple pair and (J, T)
    # over the channels of both triples: count them from the oracle's channels
    from oracle.threebody import ThreeBody, channels

    tb = ThreeBody(n1, n3)
    nlj = tb.nlj
    T = [(a, b, c) for a in range(len(nlj)) for b in range(len(nlj)) for c in range(len(nlj))
         if nlj[a][0] + nlj[b][0] + nlj[c][0] <= n3]
    par = [(nlj[a][1] + nlj[b][1] + nlj[c][1]) % 2 for a, b, c in T]
    ch = []
    for t in T:
        j = [nlj[x][2] for x in t]
        ch.append({(J, TT): len(channels(j[0], j[1], j[2], J, TT)) for J in range(1, sum(j) + 1, 2) for TT in (1, 3)})
    tot = 0
    for x in range(len(T)):
        for y in range(len(T)):
            if par[x] == par[y]:
                tot += sum(n * ch[y].get(k, 0) for k, n in ch[x].items())
    plan = ci.ci_threebody_plan(n1, n3)
    assert plan["n_triples"] == len(T)
    assert plan["n_coupled"] == tot


def test_threebody_plan_validation():
    for bad in ((-1, 0), (13, 3), (2, 7)):
        with pytest.raises(ci.CIError) as e:
            ci.ci_threebody_plan(*bad)
        assert e.value.code == ci.CI_EINVAL


def test_threebody_decouple_argument_errors():
    # rejected before any device call: null handle / pointers, negative n
    L = ci.load_library()
    vp = ctypes.c_void_p
    assert L.ci_threebody_decouple(None, None, None, 0, None, None, 0, None) == ci.CI_EINVAL
    assert L.ci_threebody_decouple(vp(1), None, None, -1, None, None, 0, None) == ci.CI_EINVAL
    assert L.ci_threebody_decouple(vp(1), None, None, 5, None, None, 0, None) == ci.CI_EINVAL
    # the cost order's work buffer: counters, one byte and one int32 per request
    assert L.ci_threebody_work_bytes(0) == 0
    for n in (1, 255, 256, 1000, 1 << 20):
        assert L.ci_threebody_work_bytes(n) >= 5 * n


def test_three_body_term_argument_errors():
    L = ci.load_library()
    vp = ctypes.c_void_p
    v3 = ci.ci_v3(ci.CI_V3_SYNTHETIC, 1, 1.0)
    assert L.ci_hamiltonian3_count(None, None, None, None) == ci.CI_EINVAL
    assert L.ci_hamiltonian3_fill(None, None, ctypes.byref(v3), None, None, None, None) == ci.CI_EINVAL
    assert L.ci_hamiltonian3_fill(vp(1), None, None, vp(1), vp(1), vp(1), None) == ci.CI_EINVAL
    assert L.ci_hamiltonian3_fill(vp(1), None, ctypes.byref(v3), None, vp(1), vp(1), None) == ci.CI_EINVAL


def test_coefficient_routine_of_the_decoupling_tables_is_exact_enough():
    # the routine the decoupling's coefficient tables are built with (Racah's
    # formula in long double) against exact rationals, up to the largest
    # arguments of the largest supported space (n1max = 12: j <= 25/2, J_ab <= 25,
    # J <= 75/2): first coupling (odd j1, j2 <= 25) and second (even J12 <= 50, odd j3 <= 25)
    import random

    from oracle.threebody import cg

    rng = random.Random(12)
    worst, n = 0.0, 0
    for j1, j2 in [(a, b) for a in range(1, 26, 2) for b in range(1, 26, 2)] + \
                  [(a, b) for a in range(0, 51, 2) for b in range(1, 26, 2)]:
        for J in range(abs(j1 - j2), j1 + j2 + 1, 2):
            m1 = rng.randrange(-j1, j1 + 1, 2) if j1 else 0
            m2 = rng.randrange(-j2, j2 + 1, 2)
            M = m1 + m2
            v = ci.ci_clebsch_gordan(j1, m1, j2, m2, J, M)
            ref = cg(j1, m1, j2, m2, J, M) if abs(M) <= J else 0.0
            worst = max(worst, abs(v - ref))
            n += 1
    assert n > 5000 and worst <= 1e-14
    assert ci.ci_clebsch_gordan(3, 1, 3, 1, 0, 2) == 0.0  # |M| > J
    assert ci.ci_clebsch_gordan(1, 1, 1, 1, 4, 2) == 0.0  # outside the triangle
    with pytest.raises(ci.CIError):
        ci.ci_clebsch_gordan(121, 1, 1, 1, 120, 2)
