"""GPU parity: libci (HIP, through the C ABI) against the FP64 oracle.

Structure (row_ptr, col, basis bits, key list) must be bit-exact; values must
satisfy max|val - ref| / max|ref| <= 1e-5 (FP32 output of an FP64 reference);
gradients max|g - g_ref| / max|g_ref| <= 1e-5.  Full-size workloads are
checked on sampled rows against the oracle and on the whole structure against
SHA-256 digests the oracle wrote (tests/golden/structure.json).
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import seeded_inputs as si
from oracle import Oracle, Problem

pytestmark = pytest.mark.gpu

VAL_TOL = 1e-5
GRAD_TOL = 1e-5
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "structure.json")

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
    (2, 2, 4, 0, 1),
    (3, 3, 2, 0, 1),
    (2, 3, 4, 1, 1),
    (4, 4, 2, 0, 1),
    (3, 4, 2, 1, -1),
    (2, 2, 6, 0, 1),
]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ci():
    import torch

    import paper_1412_5989_amd as lib

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    lib.load_library()
    return lib


def run_forward(ci, problems, seeds):
    import torch

    say("build", problems)
    b = ci.ci_basis_build(problems)
    row_ptr, nnz = ci.ci_hamiltonian_count(b)
    tb = np.concatenate([si.tbme_f32(s, i["n_tbme"]) for s, i in zip(seeds, b.info)]) if b.n_tbme else \
        np.zeros(0, np.float32)
    tbme = torch.from_numpy(tb).cuda()
    col, val = ci.ci_hamiltonian_fill(b, tbme, row_ptr)
    torch.cuda.synchronize()
    return b, row_ptr.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy(), tb


def test_build_into_torch_memory_through_the_c_abi(ci):
    # The two-body path allocates no device memory: the index tables go into
    # an arena and the partner lists into a second buffer, both torch tensors
    # (filled with 0xFF first, so nothing may rely on their contents), sized
    # by the size query and by ci_basis_list_bytes.  The matrix built that way
    # equals the oracle's; calls before the lists exist are refused.
    import ctypes

    import torch

    L = ci.load_library()
    probs = [(2, 2, 4, 0, 1), (3, 2, 2, 1, 1)]
    say("raw build", probs)
    arr, n = ci._problems(probs)
    info = (ci.ci_basis_info * n)()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.ci_basis_build(arr, n, info, None, 0, None, s) == ci.CI_OK
    need = int(info[0].arena_bytes)
    arena = torch.full((need,), 255, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    assert L.ci_basis_build(arr, n, info, ctypes.c_void_p(arena.data_ptr()), need - 256, ctypes.byref(h), s) \
        == ci.CI_ESPACE
    assert L.ci_basis_build(arr, n, info, ctypes.c_void_p(arena.data_ptr()), need, ctypes.byref(h), s) == ci.CI_OK
    rows = sum(info[k].dim + 1 for k in range(n))
    rp = torch.empty(rows, dtype=torch.int64, device="cuda")
    nnz = np.zeros(n, np.int64)
    assert L.ci_hamiltonian_count(h, ctypes.c_void_p(rp.data_ptr()), nnz.ctypes.data_as(ctypes.c_void_p), s) \
        == ci.CI_EINVAL  # no partner lists yet
    lb = ctypes.c_size_t()
    assert L.ci_basis_list_bytes(h, ctypes.byref(lb), s) == ci.CI_OK
    lists = torch.full((int(lb.value),), 255, dtype=torch.uint8, device="cuda")
    assert L.ci_basis_build_lists(h, ctypes.c_void_p(lists.data_ptr()), int(lb.value) - 8, s) == ci.CI_ESPACE
    assert L.ci_basis_build_lists(h, ctypes.c_void_p(lists.data_ptr()), int(lb.value), s) == ci.CI_OK
    assert L.ci_hamiltonian_count(h, ctypes.c_void_p(rp.data_ptr()), nnz.ctypes.data_as(ctypes.c_void_p), s) \
        == ci.CI_OK
    ntb = sum(info[k].n_tbme for k in range(n))
    seeds = [5, 6]
    tb = torch.from_numpy(np.concatenate([si.tbme_f32(sd, info[k].n_tbme) for k, sd in enumerate(seeds)])).cuda()
    assert tb.numel() == ntb
    col = torch.empty(int(nnz.sum()), dtype=torch.int32, device="cuda")
    val = torch.empty(int(nnz.sum()), dtype=torch.float32, device="cuda")
    assert L.ci_hamiltonian_fill(h, ctypes.c_void_p(tb.data_ptr()), ctypes.c_void_p(rp.data_ptr()),
                                 ctypes.c_void_p(col.data_ptr()), ctypes.c_void_p(val.data_ptr()), s) == ci.CI_OK
    torch.cuda.synchronize()
    L.ci_basis_free(h)
    rpc, colc, valc = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
    for k, (p, sd) in enumerate(zip(probs, seeds)):
        r0 = int(info[k].row_ptr_offset)
        r = rpc[r0: r0 + info[k].dim + 1]
        o = Oracle(Problem(*p))
        o.set_tbme(si.tbme_f32(sd, o.n_tbme).astype(np.float64))
        rpo, co, vo = o.csr()
        assert np.array_equal(r - r[0], rpo)
        assert np.array_equal(colc[r[0]: r[-1]], co)
        assert np.abs(valc[r[0]: r[-1]].astype(np.float64) - vo).max() <= VAL_TOL * np.abs(vo).max()


def split(b, rp, col, val, k):
    i = b.info[k]
    r = rp[i["row_ptr_offset"]: i["row_ptr_offset"] + i["dim"] + 1]
    return r - r[0], col[r[0]: r[-1]], val[r[0]: r[-1]]


def rel_err(a, ref):
    den = np.abs(ref).max() if ref.size else 1.0
    return float(np.abs(a - ref).max() / den) if ref.size else 0.0


def test_states_match_oracle(ci):
    for p in SMALL + [si.WORKLOADS["li6_nmax6"]["problem"], si.WORKLOADS["b10_nmax4"]["problem"]]:
        say("states", p)
        b = ci.ci_basis_build([p])
        s = b.states(0).cpu().numpy().view(np.uint64)
        o = Oracle(Problem(*p))
        assert np.array_equal(s, o.states()), p


@pytest.mark.parametrize("p", SMALL)
def test_small_full_matrix(ci, p):
    b, rp, col, val, tb = run_forward(ci, [p], [7])
    o = Oracle(Problem(*p))
    o.set_tbme(tb.astype(np.float64))
    rpo, co, vo = o.csr()
    r, c, v = split(b, rp, col, val, 0)
    assert b.nnz[0] == rpo[-1]
    assert np.array_equal(r, rpo)
    assert np.array_equal(c, co)
    assert rel_err(v.astype(np.float64), vo) <= VAL_TOL


def test_batch_of_small_problems(ci):
    probs = SMALL[:12]
    seeds = [100 + k for k in range(len(probs))]
    b, rp, col, val, tb = run_forward(ci, probs, seeds)
    for k, p in enumerate(probs):
        o = Oracle(Problem(*p))
        o.set_tbme(si.tbme_f64(seeds[k], o.n_tbme).astype(np.float32).astype(np.float64))
        rpo, co, vo = o.csr()
        r, c, v = split(b, rp, col, val, k)
        assert np.array_equal(r, rpo), p
        assert np.array_equal(c, co), p
        assert rel_err(v.astype(np.float64), vo) <= VAL_TOL, p


def test_empty_basis(ci):
    # no positive-parity... here negative-parity state exists without excitation
    p = (2, 2, 0, 0, -1)
    b, rp, col, val, _ = run_forward(ci, [p], [0])
    assert b.info[0]["dim"] == 0 and b.nnz == [0]
    assert list(rp) == [0]


def sha(a, dt):
    return hashlib.sha256(np.ascontiguousarray(a.astype(dt)).tobytes()).hexdigest()


@pytest.mark.parametrize("name", ["he4_nmax2", "li6_nmax6", "b10_nmax4"])
def test_workload_structure_and_sampled_rows(ci, name):
    with open(GOLDEN) as f:
        gold = json.load(f)[name]
    w = si.WORKLOADS[name]
    b, rp, col, val, tb = run_forward(ci, [w["problem"]], [w["tbme_seed"]])
    r, c, v = split(b, rp, col, val, 0)
    assert b.info[0]["dim"] == gold["dim"]
    assert b.nnz[0] == gold["nnz"]
    assert sha(r, "<i8") == gold["row_ptr_sha256"]
    assert sha(c, "<i4") == gold["col_sha256"]
    o = Oracle(Problem(*w["problem"]))
    o.set_tbme(tb.astype(np.float64))
    rows = si.sample_rows(o.dim, 300, seed=11)
    cnt, co, vo = o.rows(rows)
    got_c = np.concatenate([c[r[i]: r[i + 1]] for i in rows])
    got_v = np.concatenate([v[r[i]: r[i + 1]] for i in rows]).astype(np.float64)
    assert np.array_equal(np.diff(r)[rows], cnt)
    assert np.array_equal(got_c, co)
    # the relative error is taken against the largest |value| of the sample
    assert rel_err(got_v, vo) <= VAL_TOL


def test_fill_is_deterministic(ci):
    import torch

    w = si.WORKLOADS["b10_nmax4"]
    b = ci.ci_basis_build([w["problem"]])
    rp, nnz = ci.ci_hamiltonian_count(b)
    tbme = torch.from_numpy(si.tbme_f32(w["tbme_seed"], b.n_tbme)).cuda()
    c1, v1 = ci.ci_hamiltonian_fill(b, tbme, rp)
    c2, v2 = ci.ci_hamiltonian_fill(b, tbme, rp)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2) and torch.equal(v1.view(torch.int32), v2.view(torch.int32))


# ------------------------------------------------------------------ adjoint


def run_vjp(ci, b, rp_t, G):
    import torch

    g = ci.ci_hamiltonian_vjp(b, rp_t, torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 2, 2, 1, 1), (2, 2, 4, 0, 1), (3, 3, 2, 0, 1),
                               (0, 3, 2, 1, 1), (2, 3, 4, 1, 1)])
def test_vjp_small_full(ci, p):
    import torch

    say("vjp", p)
    b = ci.ci_basis_build([p])
    rp_t, nnz = ci.ci_hamiltonian_count(b)
    o = Oracle(Problem(*p))
    rows = np.arange(o.dim)
    counts, cols, _ = o.rows(rows, values=False)
    G = si.upstream_grad(si.psi(3, o.dim), np.repeat(rows, counts), cols)
    g = run_vjp(ci, b, rp_t, G)
    gref = o.grad_rows(rows, G.astype(np.float64))
    assert rel_err(g, gref) <= GRAD_TOL


def test_vjp_b10_sampled_rows(ci):
    # upstream gradient nonzero only on the entries of sampled rows: the exact
    # FP64 gradient of those rows comes from the oracle row by row
    w = si.WORKLOADS["b10_nmax4"]
    p = w["problem"]
    b = ci.ci_basis_build([p])
    rp_t, nnz = ci.ci_hamiltonian_count(b)
    rp = rp_t.cpu().numpy()
    o = Oracle(Problem(*p))
    rows = si.sample_rows(o.dim, 400, seed=12)
    counts, cols, _ = o.rows(rows, values=False)
    ps = si.psi(si.PSI_SEED["b10_nmax4"], o.dim)
    Gs = si.upstream_grad(ps, np.repeat(rows, counts), cols)
    G = np.zeros(nnz[0], np.float32)
    o_ = 0
    for i, n in zip(rows, counts):
        G[rp[i]: rp[i] + n] = Gs[o_: o_ + n]
        o_ += n
    g = run_vjp(ci, b, rp_t, G)
    gref = o.grad_rows(rows, Gs.astype(np.float64))
    assert rel_err(g, gref) <= GRAD_TOL


def test_vjp_b10_full_identities(ci):
    # For the full psi psi^T upstream gradient (too large for the oracle's
    # row scan): the vjp is the exact adjoint of the fill,
    #   Euler:        sum_k g_k V_k   = sum_e G_e (H_e(V) - H_e(0))
    #   dot product:  sum_k g_k V'_k  = sum_e G_e (H_e(V') - H_e(0))
    import torch

    w = si.WORKLOADS["b10_nmax4"]
    b = ci.ci_basis_build([w["problem"]])
    rp_t, nnz = ci.ci_hamiltonian_count(b)
    rp = rp_t.cpu().numpy()
    col_t, _ = ci.ci_hamiltonian_fill(b, torch.zeros(b.n_tbme, dtype=torch.float32, device="cuda"), rp_t)
    col = col_t.cpu().numpy()
    rows = np.repeat(np.arange(b.info[0]["dim"]), np.diff(rp))
    G = si.upstream_grad(si.psi(si.PSI_SEED["b10_nmax4"], b.info[0]["dim"]), rows, col)
    g = run_vjp(ci, b, rp_t, G)
    Gd = torch.from_numpy(G.astype(np.float64)).cuda()

    def H(v):
        _, val = ci.ci_hamiltonian_fill(b, torch.from_numpy(v.astype(np.float32)).cuda(), rp_t)
        return val.double()

    h0 = H(np.zeros(b.n_tbme))
    for v in (si.tbme_f32(w["tbme_seed"], b.n_tbme), np.random.default_rng(9).standard_normal(b.n_tbme)):
        v32 = v.astype(np.float32)
        lhs = float(g @ v32.astype(np.float64))
        rhs = float(Gd @ (H(v32) - h0))
        assert lhs == pytest.approx(rhs, rel=1e-4)


def test_vjp_finite_difference_b10(ci):
    # central differences of L(V) = sum_e G_e val_e(V) with the GPU forward
    # (FP32 values, FP64 dot) at h = 1e-3 on 64 seeded table entries
    import torch

    w = si.WORKLOADS["b10_nmax4"]
    b = ci.ci_basis_build([w["problem"]])
    rp_t, nnz = ci.ci_hamiltonian_count(b)
    v = si.tbme_f32(w["tbme_seed"], b.n_tbme)
    col_t, _ = ci.ci_hamiltonian_fill(b, torch.from_numpy(v).cuda(), rp_t)
    rp = rp_t.cpu().numpy()
    rows = np.repeat(np.arange(b.info[0]["dim"]), np.diff(rp))
    G = si.upstream_grad(si.psi(si.PSI_SEED["b10_nmax4"], b.info[0]["dim"]), rows, col_t.cpu().numpy())
    g = run_vjp(ci, b, rp_t, G)
    Gd = torch.from_numpy(G.astype(np.float64)).cuda()
    vt = torch.from_numpy(v).cuda()
    h = 1e-3
    fd = []
    keys = si.fd_keys(b.n_tbme, 64)
    for k in keys:
        vp, vm = vt.clone(), vt.clone()
        vp[k] += h
        vm[k] -= h
        hp = (vp[k] - vt[k]).double()
        hm = (vt[k] - vm[k]).double()
        _, a = ci.ci_hamiltonian_fill(b, vp, rp_t)
        Lp = float(Gd @ a.double())
        _, a = ci.ci_hamiltonian_fill(b, vm, rp_t)
        Lm = float(Gd @ a.double())
        fd.append((Lp - Lm) / float(hp + hm))
    fd = np.array(fd)
    scale = np.abs(g[keys]).max()
    say("fd max err / scale", np.abs(fd - g[keys]).max() / scale)
    assert np.abs(fd - g[keys]).max() <= 2e-2 * scale


def test_autograd_function(ci):
    import torch

    p = (3, 2, 2, 1, 1)
    b = ci.ci_basis_build([p])
    rp_t, nnz = ci.ci_hamiltonian_count(b)
    v = torch.from_numpy(si.tbme_f32(4, b.n_tbme)).cuda().requires_grad_(True)
    val = ci.CIHamiltonian.apply(v, b, rp_t, None)
    w = torch.from_numpy(np.random.default_rng(1).standard_normal(val.numel()).astype(np.float32)).cuda()
    (val * w).sum().backward()
    g2 = ci.ci_hamiltonian_vjp(b, rp_t, w)
    torch.cuda.synchronize()
    # the adjoint sums in fixed point (integer sums have no order), so the
    # autograd path and a direct call at the same launch shape agree bit for bit
    assert torch.equal(v.grad.view(torch.int32), g2.view(torch.int32))


# ------------------------------------------------------------------ launch shapes and batches

SHAPES = [dict(row_waves=w, row_grab=g, row_xcd=0) for w in (4, 8) for g in (0, 1, 7)] + \
    [dict(row_waves=w, row_grab=0, row_xcd=1) for w in (4, 8)]
ADJ_SHAPES = [dict(adj_rows=r, adj_tile_n=n, adj_persistent=q, row_xcd=0, adj_wide=w, adj_flush=f)
              for r, n in ((1, 1), (17, 5), (64, 16), (32, 64)) for q in (0, 1) for w in (0, 1) for f in (0, 1)] + \
    [dict(adj_rows=r, adj_tile_n=n, adj_persistent=0, row_xcd=1, adj_wide=w) for r, n in ((17, 5), (128, 8))
     for w in (0, 1)] + [dict(adj_rows=512, adj_tile_n=32, adj_persistent=q, row_xcd=0, adj_wide=1) for q in (0, 1)]


def test_launch_shapes_give_the_same_result(ci):
    # every launch shape computes each row the same way: the fill is bit-exact
    # across shapes; the adjoint is bit-exact across runs, flushes, persistent
    # grids and workgroup orders at one tile shape (its fixed-point sums have no
    # order), and agrees to rounding across tile shapes (the fixed-point scale
    # depends on the rows of a tile)
    import torch

    w = si.WORKLOADS["b10_nmax4"]
    b = ci.ci_basis_build([w["problem"]])
    rp, nnz = ci.ci_hamiltonian_count(b)
    tbme = torch.from_numpy(si.tbme_f32(w["tbme_seed"], b.n_tbme)).cuda()
    c0, v0 = ci.ci_hamiltonian_fill(b, tbme, rp)
    G = torch.rand(nnz[0], device="cuda") - 0.5
    g0 = ci.ci_hamiltonian_vjp(b, rp, G)
    torch.cuda.synchronize()
    scale = float(g0.abs().max())
    for sh in SHAPES:
        say("fill shape", sh)
        b.tuning = sh
        rp2, nnz2 = ci.ci_hamiltonian_count(b)
        assert nnz2 == nnz and torch.equal(rp2, rp), sh
        c, v = ci.ci_hamiltonian_fill(b, tbme, rp)
        torch.cuda.synchronize()
        assert torch.equal(c, c0) and torch.equal(v.view(torch.int32), v0.view(torch.int32)), sh
    by_tile = {}
    for sh in ADJ_SHAPES:
        say("adjoint shape", sh)
        b.tuning = sh
        g = ci.ci_hamiltonian_vjp(b, rp, G)
        torch.cuda.synchronize()
        assert float((g - g0).abs().max()) <= GRAD_TOL * scale, sh
        bits = g.view(torch.int32).clone()
        tile = (sh["adj_rows"], sh["adj_tile_n"])
        if tile in by_tile:
            assert torch.equal(bits, by_tile[tile]), sh
        else:
            by_tile[tile] = bits
            g2 = ci.ci_hamiltonian_vjp(b, rp, G)  # the same shape again
            torch.cuda.synchronize()
            assert torch.equal(g2.view(torch.int32), bits), sh


def test_tuning_validation_and_tuner(ci):
    import torch

    probs = SMALL[:6]
    seeds = [300 + k for k in range(len(probs))]
    b, rp, col, val, tb = run_forward(ci, probs, seeds)
    for bad in (dict(row_waves=6), dict(row_grab=-1), dict(adj_rows=0), dict(adj_tile_n=0), dict(adj_persistent=2),
                dict(adjk_rows=0), dict(adjk_tile_n=4097), dict(row_xcd=2), dict(adjk_persistent=3), dict(adj_wide=2), dict(adj_flush=2)):
        with pytest.raises(ci.CIError):
            b.tuning = bad
    rp_t = torch.from_numpy(rp).cuda()
    tbme = torch.from_numpy(tb).cuda()
    c = torch.empty(len(col), dtype=torch.int32, device="cuda")
    v = torch.empty(len(col), dtype=torch.float32, device="cuda")
    G = torch.ones(len(col), device="cuda")
    g_ref = ci.ci_hamiltonian_vjp(b, rp_t, G)
    kw = torch.empty(len(col), dtype=torch.int32, device="cuda")
    t = ci.ci_hamiltonian_tune(b, tbme, rp_t, c, v, G, reps=1, keys=kw)
    say("tuned", t)
    assert t["row_waves"] in (4, 8) and t["row_grab"] in (0, 1, 4, 16)
    assert (t["adj_rows"], t["adj_tile_n"], t["adj_wide"]) in (
        (32, 8, 0), (64, 8, 0), (64, 16, 0), (128, 16, 0), (64, 16, 1), (96, 16, 1), (128, 16, 1), (192, 16, 1),
        (256, 16, 1), (256, 32, 1), (512, 32, 1))
    assert (t["adjk_rows"], t["adjk_tile_n"]) in ((64, 8), (96, 8), (128, 8), (96, 16), (192, 8), (256, 16))
    assert t["adj_persistent"] in (0, 1) and t["adjk_persistent"] in (0, 1)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), col)
    assert np.array_equal(v.cpu().numpy().view(np.int32), val.view(np.int32))
    # the words the tuner left are the fill's: the stored-word adjoint agrees
    gk = ci.ci_hamiltonian_vjp_keys(b, rp_t, kw, G)
    torch.cuda.synchronize()
    assert float((gk - g_ref).abs().max()) <= GRAD_TOL * float(g_ref.abs().max())
    # a new handle of the same problems starts from the tuned shapes
    b2 = ci.ci_basis_build(probs)
    assert b2.tuning == t
    g = ci.ci_hamiltonian_vjp(b, rp_t, G)
    torch.cuda.synchronize()
    assert float((g - g_ref).abs().max()) <= GRAD_TOL * float(g_ref.abs().max())


@pytest.mark.parametrize("stored", [False, True])
def test_batched_64_bases_sampled_rows(ci, stored):
    # The 64-basis batch at full size, tuned and run as one captured graph of
    # fill + adjoint (stored: the fill stores the structure words and the
    # adjoint reads them, as timed by the benchmark).  Values: sampled rows of every
    # basis against the oracle.  Adjoint: the upstream gradient is psi_i psi_j
    # on the sampled rows' entries and zero elsewhere, so the oracle's gradient
    # of those rows is the exact FP64 reference for every basis' table.
    import torch

    probs, tseeds, pseeds = si.batch_problems()
    say("batch build", len(probs))
    b = ci.ci_basis_build(probs)
    rp_t, nnz = ci.ci_hamiltonian_count(b)
    tb = np.concatenate([si.tbme_f32(s, i["n_tbme"]) for s, i in zip(tseeds, b.info)])
    tbme = torch.from_numpy(tb).cuda()
    tot = int(sum(nnz))
    say("batch nnz", tot)
    rp = rp_t.cpu().numpy()
    col = torch.empty(tot, dtype=torch.int32, device="cuda")
    val = torch.empty(tot, dtype=torch.float32, device="cuda")
    G = torch.zeros(tot, dtype=torch.float32, device="cuda")
    oracles, samples = [], []
    for k, (p, i) in enumerate(zip(probs, b.info)):
        o = Oracle(Problem(*p))
        assert o.dim == i["dim"], p
        o.set_tbme(tb[i["tbme_offset"]: i["tbme_offset"] + i["n_tbme"]].astype(np.float64))
        rows = si.sample_rows(o.dim, 12, seed=40 + k)
        counts, cols, vals = o.rows(rows)
        R = i["row_ptr_offset"]
        assert np.array_equal(rp[R + rows + 1] - rp[R + rows], counts), p
        pos = np.concatenate([np.arange(rp[R + r], rp[R + r + 1]) for r in rows])
        ps = si.psi(pseeds[k], o.dim)
        Gs = si.upstream_grad(ps, np.repeat(rows, counts), cols)
        G[torch.from_numpy(pos).cuda()] = torch.from_numpy(Gs).cuda()
        oracles.append(o)
        samples.append((rows, counts, cols, vals, pos, Gs))
    gt = torch.empty(b.n_tbme, dtype=torch.float32, device="cuda")
    keys = torch.empty(tot, dtype=torch.int32, device="cuda")
    say("batch tune")
    ci.ci_hamiltonian_tune(b, tbme, rp_t, col, val, G, gt, None, reps=1, keys=keys if stored else None)
    work = torch.empty(b.vjp_work_bytes(), dtype=torch.uint8, device="cuda")
    col.fill_(-1)
    val.fill_(float("nan"))
    gt.fill_(float("nan"))

    def step():
        if stored:
            ci.ci_hamiltonian_fill_keys(b, tbme, rp_t, col, val, keys)
            ci.ci_hamiltonian_vjp_keys(b, rp_t, keys, G, gt, work)
        else:
            ci.ci_hamiltonian_fill(b, tbme, rp_t, col, val)
            ci.ci_hamiltonian_vjp(b, rp_t, G, gt, work)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(2):
        col.fill_(-1)
        keys.fill_(-1)
        gt.fill_(float("nan"))
        say("batch graph replay", rep, "stored", stored)
        graph.replay()
        torch.cuda.synchronize()
        g = gt.cpu().numpy().astype(np.float64)
        for k, (o, (rows, counts, cols, vals, pos, Gs)) in enumerate(zip(oracles, samples)):
            pt = torch.from_numpy(pos).cuda()
            c = col[pt].cpu().numpy()
            v = val[pt].cpu().numpy().astype(np.float64)
            assert np.array_equal(c, cols), probs[k]
            assert rel_err(v, vals) <= VAL_TOL, probs[k]
            i = b.info[k]
            gref = o.grad_rows(rows, Gs.astype(np.float64))
            assert rel_err(g[i["tbme_offset"]: i["tbme_offset"] + i["n_tbme"]], gref) <= GRAD_TOL, probs[k]


def test_probe_ceilings(ci):
    # the measured ceilings are in the range the device's published figures allow
    c = ci.ci_probe_ceilings(256)
    say("ceilings", c)
    assert 500.0 < c["store_GBps"] < 8000.0 * 1.05
    assert 1e11 < c["xor_popcount_steps_per_s"] < 1e14


# ------------------------------------------------------------------ off-diagonal kinetic one-body term

KINETIC = [(2, 2, 2, 0, 1), (1, 1, 4, 2, 1), (2, 1, 4, 1, 1), (2, 2, 4, 0, 1), (1, 0, 6, 1, 1), (3, 3, 2, 0, 1)]


@pytest.mark.parametrize("p", [(1, 0, 4, 1, 1), (0, 1, 6, -1, 1), (1, 0, 2, 1, -1)])
def test_single_nucleon_full_matrix(ci, p):
    # one nucleon: no two-body terms at all; the diagonal is the single-particle
    # energy and one-nucleon differences are structural zeros
    b, rp, col, val, tb = run_forward(ci, [p], [42])
    o = Oracle(Problem(*p))
    o.set_tbme(tb.astype(np.float64))
    rpo, co, vo = o.csr()
    assert np.array_equal(rp, rpo)
    assert np.array_equal(col, co)
    assert rel_err(val.astype(np.float64), vo) <= VAL_TOL


@pytest.mark.parametrize("p", KINETIC)
def test_kinetic_full_matrix(ci, p):
    import torch

    say("kinetic", p)
    b = ci.ci_basis_build([p + (ci.HW_MEV, 1)])
    rp, nnz = ci.ci_hamiltonian_count(b)
    tb = si.tbme_f32(41, b.n_tbme)
    col, val = ci.ci_hamiltonian_fill(b, torch.from_numpy(tb).cuda(), rp)
    torch.cuda.synchronize()
    o = Oracle(Problem(*p, kinetic=1))
    o.set_tbme(tb.astype(np.float64))
    rpo, co, vo = o.csr()
    assert np.array_equal(rp.cpu().numpy(), rpo)
    assert np.array_equal(col.cpu().numpy(), co)
    assert rel_err(val.cpu().numpy().astype(np.float64), vo) <= VAL_TOL


def test_kinetic_leaves_the_adjoint_unchanged(ci):
    import torch

    p = (2, 2, 4, 0, 1)
    b0, b1 = ci.ci_basis_build([p]), ci.ci_basis_build([p + (ci.HW_MEV, 1)])
    rp0, nnz0 = ci.ci_hamiltonian_count(b0)
    rp1, nnz1 = ci.ci_hamiltonian_count(b1)
    assert nnz0 == nnz1 and torch.equal(rp0, rp1)
    G = torch.rand(nnz0[0], device="cuda") - 0.5
    g0 = ci.ci_hamiltonian_vjp(b0, rp0, G)
    g1 = ci.ci_hamiltonian_vjp(b1, rp1, G)
    torch.cuda.synchronize()
    assert float((g0 - g1).abs().max()) <= GRAD_TOL * float(g0.abs().max())
