"""Small batches (1 to 16 frames per call) run in GEMV form with FP32
projections and an exact FP32 argmax over every scored row: parity with the
FP64 oracle on tiny random arrays (3 to 16 microphones, K from a few to 294,
so every stacked-row count the kernels are instantiated for), every precision argument, single frames one call at a time,
silent and non-finite frames, and the step from 16 to 17 frames where the
batched path takes over.  Needs an MI355X and the built library."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FS, C = 16000.0, 343.0


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


def _case(seed, M, N, level, F, aperture=None):
    rng = np.random.default_rng(seed)
    mics = synth.random_array(M, aperture or rng.uniform(0.04, 0.2), rng)
    grid = synth.icosphere(level)
    X = np.concatenate([synth.plane_wave_fd(mics, synth.random_direction(rng), 1, N, FS, C, rng,
                                            snr_db=rng.uniform(0, 20)) for _ in range(F)])
    return mics, grid, X.astype(np.complex64)


def _check(out, ref, L):
    doa = out["doa"].cpu().numpy()
    judged = ref["margin"] > 1e-6
    bad = np.flatnonzero(judged & (doa != ref["doa"]))
    assert bad.size == 0, f"frames {bad} differ, margins {ref['margin'][bad]}"
    ymax = np.max(np.abs(ref["y"]), axis=1)
    same = doa == ref["doa"]
    yhat = out["yhat"].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(yhat[same] - ref["yhat"][same]) <= 1e-4 * ymax[same])
    p = out["power"].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(p[same] - ref["power"][same]) <= 1e-5 * L + 2e-5 * np.abs(ref["power"][same]))
    # the margin is exact in FP32 here (every row scored): close to the oracle's
    m = out["margin"].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(m[same] - ref["margin"][same]) <= 2e-4)


CASES = [  # seed, M, N, level, delta, F
    (1, 3, 16, 1, 1e-3, 5),
    (2, 4, 32, 2, 1e-5, 16),
    (3, 7, 512, 3, 1e-5, 9),
    (4, 8, 64, 2, 1e-5, 1),
    (5, 12, 32, 2, 1e-5, 13),
    (6, 16, 16, 2, 1e-4, 16),
    (7, 16, 64, 3, 1e-7, 3),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_small_batches_match_oracle(amd, torch, case, prec):
    seed, M, N, level, delta, F = case
    print(f"gemv case seed={seed} M={M} N={N} level={level} F={F} prec={prec}", flush=True)
    mics, grid, X = _case(seed, M, N, level, F)
    ref_plan = oracle.make_plan(mics, grid, FS, C, N, delta)
    ref = oracle.locate(ref_plan, X)
    plan = amd.Plan(mics, grid, FS, C, N, delta)
    print(f"  K={plan.info['K']}", flush=True)
    out = plan.locate(torch.from_numpy(X).cuda(), precision=prec, rescore=True, hilo=True)
    torch.cuda.synchronize()
    _check(out, ref, ref_plan.W.shape[1])
    plan.close()


def test_single_frames_stream(amd, torch):
    """One call per frame on one stream for 48 frames of the planar array at
    Q = 10242, against one call of all 48 frames through the same path in
    16-frame pieces, and against the oracle."""
    print("single frames stream", flush=True)
    w = synth.workload("planar_q10242", frames=48)
    plan = amd.Plan(w["mics"], w["grid"], w["fs"], w["c"], w["N"], w["delta"])
    X = torch.from_numpy(w["X"]).cuda()
    F = X.shape[0]
    doa = torch.empty(F, dtype=torch.int32, device="cuda")
    power = torch.empty(F, dtype=torch.float32, device="cuda")
    yhat = torch.empty(F, dtype=torch.float32, device="cuda")
    margin = torch.empty(F, dtype=torch.float32, device="cuda")
    for f in range(F):
        amd.svdphat_locate(plan.handle, X[f:f + 1], amd.BF16, amd.RESCORE | amd.HILO, doa[f:f + 1], power[f:f + 1],
                           yhat[f:f + 1], margin[f:f + 1])
    pieces = [plan.locate(X[a:a + 16].contiguous(), precision="fp16") for a in range(0, F, 16)]
    torch.cuda.synchronize()
    for k, v in (("doa", doa), ("power", power), ("yhat", yhat), ("margin", margin)):
        assert torch.equal(v, torch.cat([p[k] for p in pieces])), k
    import os
    gold = dict(np.load(os.path.join(os.path.dirname(__file__), "golden", "planar_q10242_oracle.npz")))
    judged = gold["margin"][:F] > 1e-6
    d = doa.cpu().numpy()
    assert np.array_equal(d[judged], gold["doa"][:F][judged])
    same = d == gold["doa"][:F]
    L = plan.info["L"]
    pw = power.cpu().numpy()
    assert np.all(np.abs(pw[same] - gold["power"][:F][same]) <= 1e-5 * L + 2e-5 * np.abs(gold["power"][:F][same]))
    plan.close()


def test_small_batch_edges(amd, torch):
    """Silent frames, a silent microphone, NaN / Inf in one frame (the other
    frames unchanged, every index in range), and 16 against 17 frames (GEMV
    form against the batched path) on the same frames."""
    print("gemv edges", flush=True)
    mics, grid, X = _case(11, 6, 64, 3, 17)
    plan = amd.Plan(mics, grid, FS, C, 64, 1e-5)
    Q = grid.shape[0]
    Xs = X.copy()
    Xs[2] = 0
    Xs[5, 3] = 0
    Xn = Xs.copy()
    Xn[7, 1, 4] = np.nan
    Xn[8, 0, 0] = np.inf
    a = plan.locate(torch.from_numpy(Xs[:16]).cuda(), precision="fp32")
    b = plan.locate(torch.from_numpy(Xn[:16]).cuda(), precision="fp32")
    full = plan.locate(torch.from_numpy(Xs).cuda(), precision="fp32")
    torch.cuda.synchronize()
    ad, bd = a["doa"].cpu().numpy(), b["doa"].cpu().numpy()
    keep = np.ones(16, bool)
    keep[[7, 8]] = False
    assert np.array_equal(ad[keep], bd[keep])
    assert np.all((bd >= 0) & (bd < Q))
    ref_plan = oracle.make_plan(mics, grid, FS, C, 64, 1e-5)
    ref = oracle.locate(ref_plan, Xs)
    assert ad[2] == ref["doa"][2] == 0          # a silent frame: every power 0, lowest index
    assert a["power"].cpu().numpy()[2] == 0.0
    judged = ref["margin"][:16] > 1e-5
    fd = full["doa"].cpu().numpy()[:16]
    assert np.array_equal(ad[judged], fd[judged])
    assert np.array_equal(ad[judged], ref["doa"][:16][judged])
    plan.close()
