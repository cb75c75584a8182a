"""The adjoint entry point that allocates nothing (ci_hamiltonian_vjp_noalloc),
through the C ABI, against ci_hamiltonian_vjp on the same inputs: two calls in
a row, the second on a smaller problem, each within the adjoint's tolerance
(1e-5 of max |gradient|); the small problem also against the FP64 oracle."""
import ctypes
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


def _case(ci, p, tseed, pseed):
    import torch

    b = ci.ci_basis_build([p])
    rp, nnz = ci.ci_hamiltonian_count(b)
    tb = torch.from_numpy(si.tbme_f32(tseed, b.n_tbme)).cuda()
    col, _ = ci.ci_hamiltonian_fill(b, tb, rp)
    D = b.info[0]["dim"]
    rows = torch.repeat_interleave(torch.arange(D, device="cuda"), torch.diff(rp))
    ps = torch.from_numpy(si.psi(pseed, D)).cuda()
    G = (ps[rows] * ps[col.long()]).float()
    return b, rp, col, G


def _noalloc(ci, b, rp, G):
    import torch

    L = ci.load_library()
    out = torch.full((b.n_tbme,), float("nan"), dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.ci_hamiltonian_vjp_noalloc(b.handle, ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), s)
    assert rc == ci.CI_OK, L.ci_last_error()
    return out


def test_noalloc_vjp_matches_vjp_twice(ci):
    import torch

    assert int(ci.load_library().ci_vjp_noalloc_scratch_bytes()) == 64 << 20
    cases = [("b10_nmax4", 2, 104), ("he4_nmax2", 0, 101)]  # the second one smaller
    for name, tseed, pseed in cases:
        p = si.WORKLOADS[name]["problem"]
        say("noalloc vjp", name, p)
        b, rp, col, G = _case(ci, p, tseed, pseed)
        g_ref = ci.ci_hamiltonian_vjp(b, rp, G)
        g = _noalloc(ci, b, rp, G)
        torch.cuda.synchronize()
        scale = float(g_ref.abs().max())
        assert scale > 0 and bool(torch.isfinite(g).all())
        assert float((g - g_ref).abs().max()) <= GRAD_TOL * scale, name
        if name == "he4_nmax2":
            o = Oracle(Problem(*p))
            o.set_tbme(si.tbme_f32(tseed, o.n_tbme).astype(np.float64))
            rpo, co, _ = o.csr()
            Gh = G.cpu().numpy().astype(np.float64)
            gref = o.grad_rows(np.arange(o.dim), Gh)
            assert np.abs(g.cpu().numpy() - gref).max() <= GRAD_TOL * np.abs(gref).max()


def test_noalloc_vjp_refuses_a_table_beyond_the_scratch(ci):
    # the 6Li Nmax=6 table (3.97e6 elements, 31.8 MB of FP64 accumulators)
    # fits; a batch whose tables exceed the 64 MiB scratch is refused with
    # CI_ESPACE before any launch
    import torch

    probs = [si.WORKLOADS["li6_nmax6"]["problem"], (3, 4, 6, 1, 1)]
    b = ci.ci_basis_build(probs)
    assert b.n_tbme * 8 > 64 << 20
    rp, nnz = ci.ci_hamiltonian_count(b)
    L = ci.load_library()
    G = torch.zeros(sum(nnz), dtype=torch.float32, device="cuda")
    out = torch.zeros(b.n_tbme, dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.ci_hamiltonian_vjp_noalloc(b.handle, ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(G.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), s)
    assert rc == ci.CI_ESPACE
    assert b"scratch" in L.ci_last_error()
