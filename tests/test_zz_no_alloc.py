"""bfsft_execute_noalloc: the plain execute's result, bit for bit, with the
sweep's state in the library's static scratch array, on two calls in a row
(the second on a smaller plan, so the array holds the first call's state
when it starts), and a plan whose state does not fit is rejected."""
import ctypes

import numpy as np
import pytest

from paper_0801_1524_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_0801_1524_amd as bf
    bf.lib()
    return bf


def run_both(bf, P, precision):
    import torch
    with bf.Plan(P.d, P.N, P.p, P.x, P.k, precision) as plan:
        f = torch.from_numpy(P.f).to("cuda")
        ref = torch.empty(P.nx, dtype=torch.complex128, device="cuda")
        out = torch.full((P.nx,), complex(7.0, -7.0), dtype=torch.complex128, device="cuda")
        plan.execute(f, out=ref)
        plan.execute_noalloc(f, out=out)
        torch.cuda.synchronize()
        return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("precision", ["mixed", "fp64", "bf16x3"])
def test_noalloc_matches_execute_two_calls(bf, precision):
    big = synth.config("c1") if precision != "fp64" else synth.curve_problem(1024, 7, seed=3)
    small = synth.config("c0")
    for P in (big, small):  # the second call is the smaller input
        ref, got = run_both(bf, P, precision)
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), P.name


def test_noalloc_rejects_a_state_beyond_the_scratch(bf, monkeypatch):
    import torch
    monkeypatch.setenv("BFSFT_AUTOTUNE", "0")
    P = synth.curve_problem(16384, 9, seed=5)  # its largest level needs well over 64 MiB
    with bf.Plan(P.d, P.N, P.p, P.x, P.k, "mixed") as plan:
        info = plan.info()
        assert 2 * max(info["pairs"]) * 81 * 8 > 64 << 20
        out = torch.empty(P.nx, dtype=torch.complex128, device="cuda")
        with pytest.raises(bf.BfsftError) as e:
            plan.execute_noalloc(P.f, out=out)
        assert e.value.status == bf.EINVAL


def test_noalloc_through_the_c_abi(bf):
    """The entry point itself, called with raw device pointers."""
    import torch
    P = synth.config("c0")
    L = bf.lib()
    with bf.Plan(P.d, P.N, P.p, P.x, P.k, "mixed") as plan:
        f = torch.from_numpy(P.f).to("cuda")
        ref = plan.execute(f)
        out = torch.zeros_like(ref)
        torch.cuda.synchronize()
        rc = L.bfsft_execute_noalloc(plan._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()))
        assert rc == 0
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        assert L.bfsft_execute_noalloc(None, None, None) == bf.EINVAL
