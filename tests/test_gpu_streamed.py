"""GPU parity of the streamed GEMM1 form (6 to 8 microphones, 16-bit
operands, one persistent workgroup per CU) at the frame counts around its
64-frame tile, on degenerate frames and at a large batch, against the FP64
oracle.  Needs an MI355X and the built library."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

MARGIN_TOL = {"fp16": 1e-5, "bf16": 1e-5}
FS, C, N = 16000.0, 343.0, 512


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


@pytest.fixture(scope="module")
def planar642(amd):
    """Planar array of Table 2 on the level-3 grid (642 directions): the
    streamed layout (7 microphones, 2K = 96) with an oracle that builds in
    seconds."""
    mics = synth.geometry("2d")
    grid = synth.icosphere(3)
    plan = amd.Plan(mics, grid, FS, C, N, 1e-5)
    ref_plan = oracle.make_plan(mics, grid, FS, C, N, 1e-5)
    yield dict(mics=mics, grid=grid, plan=plan, ref=ref_plan)
    plan.close()


def _check(out, ref, sel, prec, L):
    doa = out["doa"].cpu().numpy()
    power = out["power"].cpu().numpy()
    rd, rm, rp = ref["doa"][sel], ref["margin"][sel], ref["power"][sel]
    judged = rm > MARGIN_TOL[prec]
    bad = np.flatnonzero(judged & (doa != rd))
    assert bad.size == 0, f"{prec}: {bad.size} judged frames differ, e.g. {bad[:5]}, margins {rm[bad[:5]]}"
    same = doa == rd
    assert np.all(np.abs(power[same] - rp[same]) <= 1e-5 * L + 2e-5 * np.abs(rp[same]))


@pytest.mark.parametrize("F", [1, 2, 63, 64, 65, 127, 200])
def test_streamed_tile_edges(amd, torch, planar642, F):
    """Frame counts below, at and just past one and two 64-frame tiles (the
    last tile ragged), with a silent frame, a silent microphone and a silent
    bin, in both 16-bit forms with the hi/lo pass."""
    print(f"streamed F={F}", flush=True)
    rng = np.random.default_rng(11785100 + F)
    X = synth.plane_wave_fd(planar642["mics"], synth.random_direction(rng), F, N, FS, C, rng,
                            snr_db=rng.uniform(0.0, 20.0)).astype(np.complex64)
    if F > 3:
        X[1] = 0             # silent frame
        X[2, 3, :] = 0       # silent microphone
        X[3, :, 100] = 0     # silent bin
    ref = oracle.locate(planar642["ref"], X)
    L = planar642["plan"].info["L"]
    Xd = torch.from_numpy(X).cuda()
    for prec in ("fp16", "bf16"):
        out = planar642["plan"].locate(Xd, precision=prec, rescore=True, hilo=True)
        torch.cuda.synchronize()
        _check(out, ref, slice(0, F), prec, L)
        if F > 3:
            assert out["doa"].cpu().numpy()[1] == ref["doa"][1]
            assert out["power"].cpu().numpy()[1] == 0.0


def test_streamed_nonfinite_frames_stay_local(amd, torch, planar642):
    """NaN or Inf in one frame's STFT leaves every other frame's answer as it
    was (the streamed tiles mix 64 frames in one MFMA block)."""
    rng = np.random.default_rng(11785199)
    X = synth.plane_wave_fd(planar642["mics"], synth.random_direction(rng), 130, N, FS, C, rng,
                            snr_db=10.0).astype(np.complex64)
    Xn = X.copy()
    Xn[5, 1, 7] = np.nan
    Xn[70, 0, 0] = np.inf
    plan = planar642["plan"]
    a = plan.locate(torch.from_numpy(X).cuda(), precision="fp16", hilo=True)["doa"].cpu().numpy()
    b = plan.locate(torch.from_numpy(Xn).cuda(), precision="fp16", hilo=True)["doa"].cpu().numpy()
    keep = np.ones(130, bool)
    keep[[5, 70]] = False
    assert np.array_equal(a[keep], b[keep])
    assert np.all((b >= 0) & (b < planar642["grid"].shape[0]))


def test_streamed_large_batch_sampled(amd, torch, planar642):
    """262,200 frames (3.8 GB of STFT) in one call: many frame tiles per
    workgroup and 64-bit offsets.  Sampled frames (first, last, tile
    boundaries, random) are checked against the oracle one by one; every
    frame against the grid's index range and finite powers."""
    print("streamed large batch", flush=True)
    X = synth.plane_wave_fd_torch(planar642["mics"], 2622, 100, N, FS, C, seed=11785177, snr_range=(0.0, 20.0))
    F = X.shape[0]
    out = planar642["plan"].locate(X, precision="fp16", rescore=True, hilo=True)
    torch.cuda.synchronize()
    doa = out["doa"].cpu().numpy()
    power = out["power"].cpu().numpy()
    assert np.all((doa >= 0) & (doa < planar642["grid"].shape[0]))
    assert np.all(np.isfinite(power))
    rng = np.random.default_rng(5)
    sel = np.unique(np.concatenate([[0, 63, 64, F // 2, F - 65, F - 64, F - 1],
                                    rng.integers(0, F, 185)]))
    Xs = X[torch.as_tensor(sel, device=X.device)].cpu().numpy()
    ref = oracle.locate(planar642["ref"], Xs)
    L = planar642["plan"].info["L"]
    sub = dict(doa=out["doa"][torch.as_tensor(sel, device=X.device)],
               power=out["power"][torch.as_tensor(sel, device=X.device)])
    _check(sub, ref, slice(None), "fp16", L)
    del X


@pytest.mark.parametrize("N_", [512, 1024])
def test_hilo_all_planar(amd, torch, N_):
    """Every frame of a 7-microphone batch through the hi/lo pass.  At N = 512
    the list rescoring stages the 33 partial slots of a frame in LDS; at
    N = 1024 (65 slots) it takes the general path.  Against the oracle, and
    equal to the default pass wherever the oracle's margin judges the frame."""
    print(f"hilo_all planar N={N_}", flush=True)
    mics = synth.geometry("2d")
    grid = synth.icosphere(3)
    rng = np.random.default_rng(11785400 + N_)
    F = 130 if N_ == 512 else 70
    X = np.concatenate([synth.plane_wave_fd(mics, synth.random_direction(rng), 10, N_, FS, C, rng,
                                            snr_db=rng.uniform(0.0, 20.0)) for _ in range(F // 10)])
    X = X.astype(np.complex64)
    X[3] = 0  # silent frame
    ref_plan = oracle.make_plan(mics, grid, FS, C, N_, 1e-5)
    ref = oracle.locate(ref_plan, X)
    plan = amd.Plan(mics, grid, FS, C, N_, 1e-5)
    L = plan.info["L"]
    Xd = torch.from_numpy(X).cuda()
    for prec in ("fp16", "bf16"):
        out = plan.locate(Xd, precision=prec, rescore=True, hilo_all=True)
        base = plan.locate(Xd, precision=prec, rescore=True, hilo=True)
        torch.cuda.synchronize()
        _check(out, ref, slice(None), prec, L)
        judged = ref["margin"] > MARGIN_TOL[prec]
        assert np.array_equal(out["doa"].cpu().numpy()[judged], base["doa"].cpu().numpy()[judged])
        assert out["power"].cpu().numpy()[3] == 0.0
    plan.close()
