"""The allocation-free entry point svdphat_locate_noalloc through the C ABI
against svdphat_locate on the same inputs: identical directions, powers,
reduced powers and margins (the same kernels on a fixed scratch array instead
of the plan's workspace), on two calls in a row, the second with fewer
frames (the array keeps the first call's contents), in every precision; and
a call that needs more scratch than the array holds is refused with
E_INVAL.  Needs an MI355X and the built library."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def amd(torch):
    import paper_1811_11785_amd as amd
    amd.lib()
    return amd


def _outs(torch, F):
    return [torch.full((F,), -7, dtype=torch.int32, device="cuda")] + \
           [torch.full((F,), -7.0, dtype=torch.float32, device="cuda") for _ in range(3)]


@pytest.mark.parametrize("prec,mode", [("fp16", "hilo"), ("bf16", "hilo"), ("fp32", "rescore"),
                                       ("fp16", "rescore")])
def test_noalloc_matches_locate(amd, torch, prec, mode):
    print(f"noalloc {prec} {mode}", flush=True)
    mics = synth.geometry("2d")
    grid = synth.icosphere(5)
    plan = amd.Plan(mics, grid, 16000.0, 343.0, 512, 1e-5)
    rng = np.random.default_rng(11785900)
    X, _, _ = synth.segments(mics, 13, 100, rng)
    X = torch.from_numpy(X).cuda()
    m = amd.RESCORE | (amd.HILO if mode == "hilo" else 0)
    P = amd.PRECISIONS[prec]
    for F in (1300, 301, 9):
        Xf = X[:F].contiguous()
        ref = _outs(torch, F)
        got = _outs(torch, F)
        amd.svdphat_locate(plan.handle, Xf, P, m, *ref)
        amd.svdphat_locate_noalloc(plan.handle, Xf, P, m, *got)
        torch.cuda.synchronize()
        for name, a, b in zip(("doa", "power", "yhat", "margin"), got, ref):
            assert torch.equal(a, b), f"F={F}: {name} differs from svdphat_locate"
    plan.close()


def test_noalloc_refuses_oversized_calls(amd, torch):
    print("noalloc oversized", flush=True)
    mics = synth.geometry("2d")
    grid = synth.icosphere(5)
    plan = amd.Plan(mics, grid, 16000.0, 343.0, 512, 1e-5)
    F = 40000
    X = torch.zeros((F, 7, 257), dtype=torch.complex64, device="cuda")
    out = _outs(torch, F)
    with pytest.raises(amd.SvdphatError) as e:
        amd.svdphat_locate_noalloc(plan.handle, X, amd.FP16, amd.RESCORE | amd.HILO, *out)
    assert e.value.code == amd.E_INVAL
    torch.cuda.synchronize()
    assert torch.all(out[0] == -7)       # nothing was enqueued
    assert amd.svdphat_noalloc_scratch_bytes() == 64 << 20
    plan.close()
