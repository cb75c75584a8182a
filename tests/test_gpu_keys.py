"""Fill with stored structure words and the adjoint that reads them, on the GPU.

ci_hamiltonian_fill_keys must write the same col and val bits as
ci_hamiltonian_fill; ci_hamiltonian_vjp_keys must give the oracle's FP64
gradient within 1e-5 of its max norm (same bar as ci_hamiltonian_vjp), on
whole small problems, on sampled rows of the full-size workloads, across
adjoint launch shapes and with the oscillator kinetic term.
"""
import sys

import numpy as np
import pytest

import seeded_inputs as si
from oracle import Oracle, Problem

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-5


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


def rel_err(a, ref):
    den = np.abs(ref).max() if ref.size else 1.0
    return float(np.abs(a - ref).max() / den) if ref.size else 0.0


def vjp_keys(ci, b, rp, keys, G):
    import torch

    g = ci.ci_hamiltonian_vjp_keys(b, rp, keys, G if torch.is_tensor(G) else torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 1, 2, 0, 1), (2, 0, 4, 0, 1), (0, 3, 2, 1, 1),
                               (2, 2, 4, 0, 1, 15.0, 1), (3, 4, 2, 1, -1), "li6_nmax6", "b10_nmax4"])
def test_fill_keys_writes_the_fill_bits(ci, p):
    import torch

    tseed = 3
    if isinstance(p, str):
        tseed = si.WORKLOADS[p]["tbme_seed"]
        p = si.WORKLOADS[p]["problem"]
    say("fill_keys", p)
    b = ci.ci_basis_build([p])
    rp, nnz = ci.ci_hamiltonian_count(b)
    tbme = torch.from_numpy(si.tbme_f32(tseed, b.n_tbme)).cuda()
    c0, v0 = ci.ci_hamiltonian_fill(b, tbme, rp)
    c1, v1, k1 = ci.ci_hamiltonian_fill_keys(b, tbme, rp)
    torch.cuda.synchronize()
    assert torch.equal(c0, c1)
    assert torch.equal(v0.view(torch.int32), v1.view(torch.int32))
    # the first entry of every row is its diagonal (a multi-term entry)
    first = rp[:-1][rp[1:] > rp[:-1]]
    assert bool(((k1[first] >> 31) != 0).all())


@pytest.mark.parametrize("p", [(2, 2, 2, 0, 1), (3, 2, 2, 1, 1), (2, 2, 4, 0, 1), (3, 3, 2, 0, 1),
                               (0, 3, 2, 1, 1), (2, 3, 4, 1, 1), (1, 1, 4, 2, 1), (2, 2, 6, 0, 1)])
def test_vjp_keys_small_full(ci, p):
    import torch

    say("vjp_keys", p)
    b = ci.ci_basis_build([p])
    rp, nnz = ci.ci_hamiltonian_count(b)
    _, _, keys = ci.ci_hamiltonian_fill_keys(b, torch.zeros(b.n_tbme, dtype=torch.float32, device="cuda"), rp)
    o = Oracle(Problem(*p))
    rows = np.arange(o.dim)
    counts, cols, _ = o.rows(rows, values=False)
    G = si.upstream_grad(si.psi(3, o.dim), np.repeat(rows, counts), cols)
    g = vjp_keys(ci, b, rp, keys, G)
    gref = o.grad_rows(rows, G.astype(np.float64))
    assert rel_err(g, gref) <= GRAD_TOL


@pytest.mark.parametrize("name,nrows", [("b10_nmax4", 400), ("li6_nmax6", 60)])
def test_vjp_keys_workload_sampled_rows(ci, name, nrows):
    # upstream gradient psi_i psi_j on the entries of sampled rows, zero
    # elsewhere: the oracle's gradient of those rows is the exact reference
    import torch

    w = si.WORKLOADS[name]
    p = w["problem"]
    b = ci.ci_basis_build([p])
    rp_t, nnz = ci.ci_hamiltonian_count(b)
    rp = rp_t.cpu().numpy()
    _, _, keys = ci.ci_hamiltonian_fill_keys(b, torch.from_numpy(si.tbme_f32(w["tbme_seed"], b.n_tbme)).cuda(),
                                             rp_t)
    o = Oracle(Problem(*p))
    rows = si.sample_rows(o.dim, nrows, seed=13)
    say("vjp_keys sampled", name, len(rows))
    counts, cols, _ = o.rows(rows, values=False)
    Gs = si.upstream_grad(si.psi(si.PSI_SEED[name], o.dim), np.repeat(rows, counts), cols)
    G = np.zeros(nnz[0], np.float32)
    o_ = 0
    for i, n in zip(rows, counts):
        G[rp[i]: rp[i] + n] = Gs[o_: o_ + n]
        o_ += n
    g = vjp_keys(ci, b, rp_t, keys, G)
    gref = o.grad_rows(rows, Gs.astype(np.float64))
    assert rel_err(g, gref) <= GRAD_TOL


# tiles of the stored-word adjoint (its own fields of the launch shape)
ADJ_SHAPES = [dict(adjk_rows=r, adjk_tile_n=n, adjk_persistent=q, adj_flush=f)
              for r, n in ((1, 1), (17, 5), (64, 8), (128, 16)) for q in (0, 1) for f in (0, 1)]


def test_vjp_keys_agrees_with_vjp_across_shapes(ci):
    # the full psi psi^T upstream gradient of the measured workload: both
    # adjoints add the same FP32 terms into FP64 accumulators in no fixed
    # order, so they agree to rounding
    import torch

    w = si.WORKLOADS["li6_nmax6"]
    b = ci.ci_basis_build([w["problem"]])
    rp_t, nnz = ci.ci_hamiltonian_count(b)
    tbme = torch.from_numpy(si.tbme_f32(w["tbme_seed"], b.n_tbme)).cuda()
    col, _, keys = ci.ci_hamiltonian_fill_keys(b, tbme, rp_t)
    rp = rp_t.cpu().numpy()
    rows = np.repeat(np.arange(b.info[0]["dim"]), np.diff(rp))
    G = torch.from_numpy(si.upstream_grad(si.psi(si.PSI_SEED["li6_nmax6"], b.info[0]["dim"]), rows,
                                          col.cpu().numpy())).cuda()
    g0 = ci.ci_hamiltonian_vjp(b, rp_t, G)
    torch.cuda.synchronize()
    scale = float(g0.abs().max())
    for sh in ADJ_SHAPES:
        say("keys adjoint shape", sh)
        b.tuning = sh
        g = ci.ci_hamiltonian_vjp_keys(b, rp_t, keys, G)
        torch.cuda.synchronize()
        assert float((g - g0).abs().max()) <= GRAD_TOL * scale, sh


def test_vjp_keys_with_kinetic_term(ci):
    # the kinetic term is one-body: it changes values, not the adjoint
    import torch

    p = (2, 2, 4, 0, 1)
    b0, b1 = ci.ci_basis_build([p]), ci.ci_basis_build([p + (ci.HW_MEV, 1)])
    rp0, nnz0 = ci.ci_hamiltonian_count(b0)
    rp1, _ = ci.ci_hamiltonian_count(b1)
    t = torch.from_numpy(si.tbme_f32(5, b0.n_tbme)).cuda()
    _, _, k1 = ci.ci_hamiltonian_fill_keys(b1, t, rp1)
    G = torch.rand(nnz0[0], device="cuda") - 0.5
    g0 = ci.ci_hamiltonian_vjp(b0, rp0, G)
    g1 = ci.ci_hamiltonian_vjp_keys(b1, rp1, k1, G)
    torch.cuda.synchronize()
    assert float((g0 - g1).abs().max()) <= GRAD_TOL * float(g0.abs().max())


def test_autograd_with_and_without_stored_keys(ci):
    import torch

    p = (3, 2, 2, 1, 1)
    b = ci.ci_basis_build([p])
    rp_t, nnz = ci.ci_hamiltonian_count(b)
    w = torch.from_numpy(np.random.default_rng(1).standard_normal(int(nnz[0])).astype(np.float32)).cuda()
    grads = []
    for store in (True, False):
        v = torch.from_numpy(si.tbme_f32(4, b.n_tbme)).cuda().requires_grad_(True)
        val = ci.CIHamiltonian.apply(v, b, rp_t, None, store)
        (val * w).sum().backward()
        grads.append(v.grad.clone())
    torch.cuda.synchronize()
    o = Oracle(Problem(*p))
    rows = np.arange(o.dim)
    gref = o.grad_rows(rows, w.cpu().numpy().astype(np.float64))
    for g in grads:
        assert rel_err(g.cpu().numpy().astype(np.float64), gref) <= GRAD_TOL


def test_empty_basis_keys(ci):
    import torch

    b = ci.ci_basis_build([(2, 2, 0, 0, -1)])
    rp, nnz = ci.ci_hamiltonian_count(b)
    assert nnz == [0]
    t = torch.zeros(b.n_tbme, dtype=torch.float32, device="cuda")
    c, v, k = ci.ci_hamiltonian_fill_keys(b, t, rp)
    g = ci.ci_hamiltonian_vjp_keys(b, rp, k, torch.zeros(0, device="cuda"))
    g2 = ci.ci_hamiltonian_vjp(b, rp, torch.zeros(0, device="cuda"))
    torch.cuda.synchronize()
    assert c.numel() == 0 and k.numel() == 0 and bool((g == 0).all()) and bool((g2 == 0).all())
