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


def test_replay_after_workspace_growth(torch):
    """A graph captured at 300 frames keeps working after an eager call of
    20000 frames on the same stream has grown the stream's workspace (the
    captured buffer is kept, not freed), and a call that would have to grow
    the workspace while the stream is being captured is refused with
    E_INVAL before anything is enqueued."""
    import ctypes

    import paper_1811_11785_amd as amd
    amd.lib()
    print("graph replay after workspace growth", flush=True)
    mics = synth.geometry("2d")
    grid = synth.icosphere(3)
    plan = amd.Plan(mics, grid, 16000.0, 343.0, 512, 1e-5)
    rng = np.random.default_rng(11785310)
    X1 = synth.plane_wave_fd(mics, synth.random_direction(rng), 300, 512, 16000.0, 343.0, rng, snr_db=5.0)
    X1 = torch.from_numpy(X1.astype(np.complex64)).cuda()
    Xbig = torch.from_numpy(np.tile(X1.cpu().numpy(), (67, 1, 1))[:20000]).cuda()
    Xin = torch.empty_like(X1)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        Xin.copy_(X1)
        ref = {k: v.clone() for k, v in plan.locate(Xin, precision="fp16", hilo=True, stream=s).items()}
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        out = plan.locate(Xin, precision="fp16", hilo=True, stream=s)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        big = plan.locate(Xbig, precision="fp16", hilo=True, stream=s)
    torch.cuda.synchronize()
    assert big["doa"].shape[0] == 20000
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        for k in ("doa", "power", "yhat", "margin"):
            assert torch.equal(out[k], ref[k]), f"replay {rep}: {k} differs from the eager call"
    # a fresh stream has no workspace: capturing a call on it is refused
    hip = ctypes.CDLL("libamdhip64.so")
    s2 = torch.cuda.Stream()
    h = ctypes.c_void_p(s2.cuda_stream)
    assert hip.hipStreamBeginCapture(h, ctypes.c_int(2)) == 0     # relaxed mode
    with pytest.raises(amd.SvdphatError) as e:
        plan.locate(Xin, precision="fp16", hilo=True, stream=s2)
    graph = ctypes.c_void_p()
    assert hip.hipStreamEndCapture(h, ctypes.byref(graph)) == 0
    if graph.value:
        hip.hipGraphDestroy(graph)
    assert e.value.code == amd.E_INVAL
    torch.cuda.synchronize()
    plan.close()
