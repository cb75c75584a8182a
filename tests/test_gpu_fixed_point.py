"""GPU: exact properties of the adjoint's fixed-point sums.

Each contribution g to a table position is summed as the integer
rint(g * 2^s), s per basis from max |G| and the rows of an adjoint tile, and
the integer totals are scaled back once.  What follows from that, bit for bit:
scaling G by a power of two scales the gradient by the same power (the shift
moves with the exponent of max |G|, the integers do not change); G -> -G gives
-gradient (rounding to nearest even is odd-symmetric); G = 0 gives 0; and the
two adjoints (partner-list walk and stored words) give the same bits when
their tiles have the same shape.  A G whose entries span six decades still
meets the max-norm bound against the FP64 oracle gradient.
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


def bits(t):
    import torch

    torch.cuda.synchronize()
    return t.view(torch.int32).cpu().numpy()


@pytest.mark.parametrize("p", [(3, 2, 4, 1, 1), (2, 2, 6, 0, 1)])
def test_power_of_two_scaling_sign_and_zero_are_exact(ci, p):
    import torch

    say("fixed point", p)
    b = ci.ci_basis_build([p])
    rp, nnz = ci.ci_hamiltonian_count(b)
    G = torch.from_numpy(np.random.default_rng(7).standard_normal(nnz[0]).astype(np.float32)).cuda()
    g = ci.ci_hamiltonian_vjp(b, rp, G).clone()
    g0 = bits(g)
    for k in (-7, -1, 3, 11):
        gk = ci.ci_hamiltonian_vjp(b, rp, G * (2.0 ** k))
        assert np.array_equal(bits(gk), bits(g * (2.0 ** k))), k
    gn = ci.ci_hamiltonian_vjp(b, rp, -G)
    assert np.array_equal(bits(gn), bits(-g + 0.0))  # + 0.0: a zero total is +0 either way
    gz = ci.ci_hamiltonian_vjp(b, rp, torch.zeros_like(G))
    assert not torch.any(gz != 0)
    # and twice the same call gives the same bits
    assert np.array_equal(bits(ci.ci_hamiltonian_vjp(b, rp, G)), g0)


def test_walk_and_stored_words_agree_bit_for_bit(ci):
    import torch

    w = si.WORKLOADS["li6_nmax6"]
    say("walk vs stored words", w["problem"])
    b = ci.ci_basis_build([w["problem"]])
    rp, nnz = ci.ci_hamiltonian_count(b)
    tbme = torch.from_numpy(si.tbme_f32(w["tbme_seed"], b.n_tbme)).cuda()
    col, val, keys = ci.ci_hamiltonian_fill_keys(b, tbme, rp)
    G = torch.rand(nnz[0], device="cuda") - 0.5
    for rows, tn in ((96, 8), (64, 16)):
        b.tuning = dict(adj_rows=rows, adj_tile_n=tn, adjk_rows=rows, adjk_tile_n=tn)
        gw = ci.ci_hamiltonian_vjp(b, rp, G)
        gk = ci.ci_hamiltonian_vjp_keys(b, rp, keys, G)
        assert np.array_equal(bits(gw), bits(gk)), (rows, tn)


def test_wide_dynamic_range_meets_the_bound(ci):
    import torch

    p = (2, 3, 4, 1, 1)
    say("dynamic range", p)
    o = Oracle(Problem(*p))
    b = ci.ci_basis_build([p])
    rp_t, nnz = ci.ci_hamiltonian_count(b)
    rp = rp_t.cpu().numpy()
    rng = np.random.default_rng(11)
    # magnitudes log-uniform over six decades, random signs; a few entries 1e6 x the smallest
    G = (rng.choice([-1.0, 1.0], nnz[0]) * 10.0 ** rng.uniform(-6, 0, nnz[0])).astype(np.float32)
    g = ci.ci_hamiltonian_vjp(b, rp_t, torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    rows = np.arange(o.dim)
    ref = o.grad_rows(rows, G.astype(np.float64))
    got = g.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= GRAD_TOL * np.abs(ref).max()
    assert rp[-1] == nnz[0]
