"""The 3-D array workloads (the 3-D 7-microphone array of Table 2, two
simultaneous white-noise sources per 100-frame segment, power ratio U[0, 6]
dB, no sensor noise) at Q = 10242 (icosphere level 5) and Q = 40962
(level 6), delta = 1e-5 (K = 71), through the C ABI against the stored FP64
oracle answers: batches of 4096 frames and the whole 40960-frame batch,
single frames one call at a time (batch 1, the streaming use), BF16 with
FP32 rescoring and FP16 with hi/lo.  Needs an MI355X and the built library."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
# index exact above this oracle margin (FP32 rescoring, hi/lo where asked)
MARGIN_TOL = 1e-5
# reduced powers before rescoring, per frame max_q |y - y*| / max_q |y*|
# (the bounds of the planar parity tests)
Y_TOL = {"fp32": 1e-4, "fp16": 5e-4, "bf16": 5e-3}


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


def _load(name, frames):
    w = synth.workload(name, frames=frames)
    gold = dict(np.load(os.path.join(HERE, "golden", f"{name}_oracle.npz")))
    return w, gold


@pytest.fixture(scope="module")
def cube10(amd, torch):
    w, gold = _load("cube_q10242", None)
    plan = amd.Plan(w["mics"], w["grid"], w["fs"], w["c"], w["N"], w["delta"])
    X = torch.from_numpy(w["X"]).cuda()
    yield dict(w=w, gold=gold, plan=plan, X=X)
    plan.close()


def _check(doa, power, gold, L, n=None, tol=MARGIN_TOL):
    n = int(gold["frames"]) if n is None else n
    ref, margin = gold["doa"][:n], gold["margin"][:n]
    judged = margin > tol
    bad = np.flatnonzero(judged & (doa[:n] != ref))
    assert bad.size == 0, f"{bad.size} judged mismatches, e.g. frames {bad[:5]} margins {margin[bad[:5]]}"
    same = doa[:n] == ref
    want = gold["power"][:n][same]
    assert np.all(np.abs(power[:n][same] - want) <= 1e-5 * L + 2e-5 * np.abs(want))
    return float(np.mean(same)), float(np.mean(doa[:n][judged] == ref[judged]))


def test_cube_q10242_plan(cube10):
    info, g = cube10["plan"].info, cube10["gold"]
    assert info["K"] == int(g["K"]) == 71 and info["K_paper"] == int(g["K_paper"])
    assert info["n_classes"] == int(g["n_classes"]) == 10242
    assert abs(info["residual"] - float(g["residual"])) <= 1e-8


@pytest.mark.parametrize("prec,hilo", [("bf16", False), ("bf16", True), ("fp16", True), ("fp32", False)])
def test_cube_q10242_batches(cube10, torch, prec, hilo):
    """4096-frame batches and the whole 40960-frame batch in one call: the
    stored frames against the oracle, every frame in range."""
    print(f"cube_q10242 prec={prec} hilo={hilo}", flush=True)
    d, g = cube10, cube10["gold"]
    L = d["plan"].info["L"]
    whole = d["plan"].locate(d["X"], precision=prec, rescore=True, hilo=hilo)
    part = d["plan"].locate(d["X"][:4096].contiguous(), precision=prec, rescore=True, hilo=hilo)
    torch.cuda.synchronize()
    for out in (whole, part):
        doa, power = out["doa"].cpu().numpy(), out["power"].cpu().numpy()
        assert np.all((doa >= 0) & (doa < 10242)) and np.all(np.isfinite(power))
        m_all, m_j = _check(doa, power, g, L)
        print(f"  match all {m_all:.4%} judged {m_j:.4%}", flush=True)


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_cube_q10242_y_rows(cube10, torch, prec):
    d, g = cube10, cube10["gold"]
    out = d["plan"].locate(d["X"][:4096].contiguous(), precision=prec, rescore=True, want_y=True)
    torch.cuda.synchronize()
    rows = torch.from_numpy(g["y_rows"]).cuda()
    y = out["y"].index_select(0, rows).cpu().numpy().astype(np.float64)
    yr = g["y"].astype(np.float64)
    err = np.max(np.abs(y - yr), axis=1) / np.max(np.abs(yr), axis=1)
    print(f"  cube y error {prec} max {err.max():.3e}", flush=True)
    assert np.all(err <= Y_TOL[prec])


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_cube_q10242_single_frames(cube10, torch, amd, prec):
    """Batch 1: one call per frame on one stream (the streaming use), the
    first 160 frames (two segments), against the oracle."""
    print(f"cube_q10242 single frames {prec}", flush=True)
    d, g = cube10, cube10["gold"]
    n = 160
    X = d["X"][:n].contiguous()
    doa = torch.empty(n, dtype=torch.int32, device="cuda")
    power = torch.empty(n, dtype=torch.float32, device="cuda")
    P = amd.PRECISIONS[prec]
    for f in range(n):
        amd.svdphat_locate(d["plan"].handle, X[f:f + 1], P, amd.RESCORE | amd.HILO, doa[f:f + 1], power[f:f + 1])
    torch.cuda.synchronize()
    _check(doa.cpu().numpy(), power.cpu().numpy(), g, d["plan"].info["L"], n=n)


def test_cube_q40962(amd, torch):
    """Q = 40962: the stored 400 frames in one BF16 call with rescoring
    (and with hi/lo), the sampled frames' reduced powers, and single frames."""
    print("cube_q40962", flush=True)
    w, g = _load("cube_q40962", 400)
    plan = amd.Plan(w["mics"], w["grid"], w["fs"], w["c"], w["N"], w["delta"])
    info = plan.info
    assert info["K"] == int(g["K"]) == 71 and info["n_classes"] == 40962
    X = torch.from_numpy(w["X"]).cuda()
    L = info["L"]
    for hilo in (False, True):
        out = plan.locate(X, precision="bf16", rescore=True, hilo=hilo, want_y=not hilo)
        torch.cuda.synchronize()
        m_all, m_j = _check(out["doa"].cpu().numpy(), out["power"].cpu().numpy(), g, L)
        print(f"  bf16 hilo={hilo} match all {m_all:.4%} judged {m_j:.4%}", flush=True)
        if not hilo:
            rows = torch.from_numpy(g["y_rows"]).cuda()
            y = out["y"].index_select(0, rows).cpu().numpy().astype(np.float64)
            yr = g["y"].astype(np.float64)
            err = np.max(np.abs(y - yr), axis=1) / np.max(np.abs(yr), axis=1)
            print(f"  y error max {err.max():.3e}", flush=True)
            assert np.all(err <= Y_TOL["bf16"])
    n = 40
    doa = torch.empty(n, dtype=torch.int32, device="cuda")
    power = torch.empty(n, dtype=torch.float32, device="cuda")
    for f in range(n):
        amd.svdphat_locate(plan.handle, X[f:f + 1].contiguous(), amd.BF16, amd.RESCORE | amd.HILO,
                           doa[f:f + 1], power[f:f + 1])
    torch.cuda.synchronize()
    _check(doa.cpu().numpy(), power.cpu().numpy(), g, L, n=n)
    plan.close()
