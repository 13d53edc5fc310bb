"""svdphat_locate captured into a HIP graph (through torch's graph API on a
side stream) and replayed several times, with eager work and host
synchronisation between the replays; every replay must reproduce the eager
call exactly.  Needs an MI355X and the built library."""
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


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_locate_graph_replays(torch, prec):
    import paper_1811_11785_amd as amd
    amd.lib()
    print(f"graph replays {prec}", flush=True)
    mics = synth.geometry("2d")
    grid = synth.icosphere(3)
    plan = amd.Plan(mics, grid, 16000.0, 343.0, 512, 1e-5)
    rng = np.random.default_rng(11785300)
    F = 300
    X1 = synth.plane_wave_fd(mics, synth.random_direction(rng), F, 512, 16000.0, 343.0, rng, snr_db=3.0)
    X2 = synth.plane_wave_fd(mics, synth.random_direction(rng), F, 512, 16000.0, 343.0, rng, snr_db=15.0)
    X1 = torch.from_numpy(X1.astype(np.complex64)).cuda()
    X2 = torch.from_numpy(X2.astype(np.complex64)).cuda()
    Xin = torch.empty_like(X1)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        # eager references (also sizes the stream's workspace before capture)
        Xin.copy_(X1)
        ref1 = {k: v.clone() for k, v in plan.locate(Xin, precision=prec, hilo=True, stream=s).items()}
        Xin.copy_(X2)
        ref2 = {k: v.clone() for k, v in plan.locate(Xin, precision=prec, hilo=True, stream=s).items()}
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        out = plan.locate(Xin, precision=prec, hilo=True, stream=s)
    torch.cuda.synchronize()
    for rep in range(4):
        src, ref = (X1, ref1) if rep % 2 == 0 else (X2, ref2)
        Xin.copy_(src)
        _ = (X1 * 2).sum().item()  # eager work between the replays
        g.replay()
        torch.cuda.synchronize()
        for k in ("doa", "power", "yhat", "margin"):
            assert torch.equal(out[k], ref[k]), f"replay {rep}: {k} differs from the eager call"
    plan.close()
