"""Three-body decoupling kernel on the GPU against the oracle, through the C ABI.

Bar: every request within 1e-5 relative (max norm over the requests) of the
oracle's direct sum, with the coupled input rounded to FP32 on both sides;
exact zeros where M, M_T or parity differ or an index is out of range; the
identity interaction gives the identity.
"""
import sys

import numpy as np
import pytest

import seeded_inputs as si
from oracle.threebody import ThreeBody as OracleTB

pytestmark = pytest.mark.gpu

TOL = 1e-5


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


def coupled_input(t, seed):
    """FP32 coupled elements in the library's storage order, from the labels."""
    k = t.keys()
    tri = t.triples
    return si.coupled3b_values(seed, tri[k[:, 0]], tri[k[:, 1]], k[:, 2], k[:, 3], k[:, 4], k[:, 5], k[:, 6],
                               k[:, 7]).astype(np.float32)


@pytest.mark.parametrize("order", [False, True])
@pytest.mark.parametrize("n1,n3,nreq", [(2, 2, 600), (3, 3, 600), (4, 4, 800)])
def test_decouple_matches_oracle(ci, n1, n3, nreq, order):
    import torch

    t = ci.ThreeBody(n1, n3)
    say("three-body", n1, n3, "coupled", t.n_coupled, "triples", t.n_triples, "cost order", order)
    A = coupled_input(t, 50 + n1)
    req = si.requests_3b(60 + n1, nreq, n1, n3, mismatched=40)
    bad = np.array([[-1, 0, 0, 0, 0, 0], [0, 0, 0, 0, 0, 2 * t.n_sps]], np.int32)
    req = np.concatenate([req, bad])
    out = t.decouple(torch.from_numpy(A).cuda(), torch.from_numpy(req).cuda(),
                     order=order).cpu().numpy().astype(np.float64)
    o = OracleTB(n1, n3)

    def val(*key):
        return float(np.float32(si.coupled3b_value(50 + n1, *key)))

    ref = np.array([o.element(r, val) for r in req])
    scale = np.abs(ref).max()
    say("max err / scale", np.abs(out - ref).max() / scale)
    assert np.abs(out - ref).max() <= TOL * scale
    zero = ref == 0.0
    assert zero[nreq:].all() and (out[zero] == 0.0).all()


def test_identity_interaction(ci):
    import torch

    t = ci.ThreeBody(3, 3)
    k = t.keys()
    tri = t.triples
    same = (k[:, 0] == k[:, 1]) & (k[:, 4] == k[:, 6]) & (k[:, 5] == k[:, 7])
    A = torch.from_numpy(same.astype(np.float32)).cuda()
    req = si.requests_3b(70, 400, 3, 3)
    diag = np.concatenate([req[:, :3], req[:, :3]], axis=1)
    out_r = t.decouple(A, torch.from_numpy(req).cuda()).cpu().numpy()
    out_d = t.decouple(A, torch.from_numpy(np.ascontiguousarray(diag)).cuda()).cpu().numpy()
    expect = (req[:, :3] == req[:, 3:]).all(axis=1).astype(np.float32)
    assert np.abs(out_r - expect).max() <= 1e-6
    assert np.abs(out_d - 1.0).max() <= 1e-6


def test_decouple_workload_sampled(ci):
    # the measured workload (shells 0..6, triples inside 6): sampled requests
    import torch

    t = ci.ThreeBody(6, 6)
    A = coupled_input(t, 56)
    req = si.requests_3b(66, 4000, 6, 6)
    out = t.decouple(torch.from_numpy(A).cuda(), torch.from_numpy(req).cuda()).cpu().numpy().astype(np.float64)
    o = OracleTB(6, 6)

    def val(*key):
        return float(np.float32(si.coupled3b_value(56, *key)))

    pick = np.random.default_rng(5).choice(len(req), size=200, replace=False)
    ref = np.array([o.element(req[i], val) for i in pick])
    say("workload max err / scale", np.abs(out[pick] - ref).max() / np.abs(ref).max())
    assert np.abs(out[pick] - ref).max() <= TOL * np.abs(ref).max()


def test_cost_order_gives_the_same_bits(ci):
    # each request is summed by one lane in a fixed order, so grouping the
    # requests by cost changes no bit of any result; ragged n, repeated calls
    # on one work buffer with a smaller n second
    import torch

    t = ci.ThreeBody(6, 6)
    A = torch.from_numpy(np.random.default_rng(3).standard_normal(t.n_coupled).astype(np.float32)).cuda()
    req = torch.from_numpy(si.requests_3b(67, 150001, 6, 6, mismatched=1000)).cuda()
    ref = t.decouple(A, req, order=False)
    work = torch.empty(ci.load_library().ci_threebody_work_bytes(150001), dtype=torch.uint8, device="cuda")
    for n in (150001, 70001, 1, 0):
        got = t.decouple(A, req[:n], order=True, work=work)
        torch.cuda.synchronize()
        say("cost order n", n)
        assert torch.equal(got, ref[:n])
    with pytest.raises(ValueError):
        t.decouple(A, req, order=True, work=work[:100])
