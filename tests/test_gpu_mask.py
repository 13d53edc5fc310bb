"""The binary time-frequency mask (svdphat_locate_masked) through the C ABI
against the FP64 oracle with the same mask: random masks (including frames
with every bin dropped or kept), a band mask, every precision, batched and in
the GEMV form of small batches, eq. (14) and eq. (15), and the 7-microphone
planar array at Q = 10242.  Needs an MI355X and the built library."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FS, C = 16000.0, 343.0
MARGIN_TOL = {"fp32": 1e-6, "fp16": 1e-5, "bf16": 1e-5}


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


def _frames(mics, N, F, rng, snr=(0.0, 20.0)):
    X = np.concatenate([synth.plane_wave_fd(mics, synth.random_direction(rng), 10, N, FS, C, rng,
                                            snr_db=rng.uniform(*snr)) for _ in range(-(-F // 10))])[:F]
    return X.astype(np.complex64)


def _masks(rng, F, B):
    m = (rng.random((F, B)) > 0.3).astype(np.uint8)
    m[0] = 0                      # every bin dropped
    m[1] = 1                      # every bin kept
    m[2] = 0
    m[2, 20:60] = 1               # a band
    return m


def _check(out, ref, prec, L, key="margin"):
    doa = out["doa"].cpu().numpy()
    judged = ref[key] > MARGIN_TOL[prec]
    bad = np.flatnonzero(judged & (doa != ref["doa"]))
    assert bad.size == 0, f"{prec}: frames {bad[:5]} differ, margins {ref[key][bad[:5]]}"
    same = doa == ref["doa"]
    p = out["power"].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(p[same] - ref["power"][same]) <= 1e-5 * L + 2e-5 * np.abs(ref["power"][same]))
    return judged


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_mask_tiny(amd, torch, prec):
    print(f"mask tiny {prec}", flush=True)
    rng = np.random.default_rng(11785800)
    mics = synth.random_array(6, 0.1, rng)
    grid = synth.icosphere(3)
    N, F = 128, 90
    B = N // 2 + 1
    X = _frames(mics, N, F, rng)
    m = _masks(rng, F, B)
    ref_plan = oracle.make_plan(mics, grid, FS, C, N, 1e-5)
    plan = amd.Plan(mics, grid, FS, C, N, 1e-5)
    Xd, md = torch.from_numpy(X).cuda(), torch.from_numpy(m).cuda()
    L = ref_plan.W.shape[1]
    for normalized in (False, True):
        ref = (oracle.normalized_locate if normalized else oracle.locate)(ref_plan, X, mask=m)
        out = plan.locate(Xd, precision=prec, rescore=True, hilo=True, normalized=normalized, mask=md)
        small = plan.locate(Xd[:12].contiguous(), precision=prec, normalized=normalized, mask=md[:12].contiguous())
        torch.cuda.synchronize()
        _check(out, ref, prec, L)
        _check(small, {k: v[:12] for k, v in ref.items()}, "fp32", L)
        d = out["doa"].cpu().numpy()
        assert d[0] == ref["doa"][0] == 0 and out["power"].cpu().numpy()[0] == 0.0   # nothing kept
    # the unmasked call equals the mask of ones
    ones = torch.ones_like(md)
    a = plan.locate(Xd, precision=prec, hilo=True)
    b = plan.locate(Xd, precision=prec, hilo=True, mask=ones)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k
    plan.close()


def test_mask_planar_q10242(amd, torch):
    """The benchmark's array and grid with a random mask on 96 frames (FP16
    with rescoring and hi/lo), against the oracle (its SVD of W built here)."""
    print("mask planar q10242", flush=True)
    w = synth.workload("planar_q10242", frames=96)
    rng = np.random.default_rng(11785810)
    m = _masks(rng, 96, 257)
    ref_plan = oracle.make_plan(w["mics"], w["grid"], w["fs"], w["c"], w["N"], w["delta"])
    ref = oracle.locate(ref_plan, w["X"], mask=m)
    plan = amd.Plan(w["mics"], w["grid"], w["fs"], w["c"], w["N"], w["delta"])
    out = plan.locate(torch.from_numpy(w["X"]).cuda(), precision="fp16", hilo=True,
                      mask=torch.from_numpy(m).cuda())
    torch.cuda.synchronize()
    judged = _check(out, ref, "fp16", ref_plan.W.shape[1])
    print(f"  judged {judged.sum()}/96 frames match", flush=True)
    plan.close()


def _premasked(torch, Xd, md):
    """The frames with the dropped bins written as 0 (what the mask means)."""
    return torch.where(md.bool()[:, None, :], Xd, torch.zeros((), dtype=Xd.dtype, device=Xd.device)).contiguous()


@pytest.mark.parametrize("name,F", [("planar_q10242", 2000), ("cube_q10242", 4096)])
def test_mask_inside_kernels_equals_masked_frames(amd, torch, name, F):
    """Where the streamed GEMM1 serves the call, the mask is applied inside the
    kernels (the PHAT producers, the hi/lo pass's listed frames, the power)
    instead of on a masked copy of every frame.  Its results must be those
    of the unmasked call on the frames with the dropped bins set to 0, bit
    for bit: the planar array (one GEMM1 pass) on a ragged last frame tile,
    and the 3-D array at 4096 frames (GEMM1 in two row-group passes); FP16
    and BF16, eq. (14) with hi/lo on the close frames and on every frame,
    and eq. (15)."""
    print(f"mask fused {name} F={F}", flush=True)
    w = synth.workload(name, frames=F)
    X = w["X"][:F]
    B = X.shape[2]
    rng = np.random.default_rng(11785820)
    m = _masks(rng, F, B)
    m[3:40] = 1                     # frames kept whole among the random ones
    m[-1] = 0                       # the ragged tile's last frame: nothing kept
    plan = amd.Plan(w["mics"], w["grid"], w["fs"], w["c"], w["N"], w["delta"])
    Xd, md = torch.from_numpy(X).cuda(), torch.from_numpy(m).cuda()
    Xz = _premasked(torch, Xd, md)
    cases = [dict(precision="fp16", hilo=True), dict(precision="bf16", hilo=True),
             dict(precision="fp16", hilo_all=True), dict(precision="fp16", hilo=True, normalized=True),
             dict(precision="fp16", rescore=False)]
    for kw in cases:
        a = plan.locate(Xd, mask=md, **kw)
        b = plan.locate(Xz, **kw)
        torch.cuda.synchronize()
        for k in a:
            assert torch.equal(a[k], b[k]), (kw, k, (a[k] != b[k]).nonzero()[:5].flatten().tolist())
        if kw.get("rescore", True):  # a frame with nothing kept: every direction ties, the first wins
            assert a["doa"][-1].item() == 0 and a["power"][-1].item() == 0.0
    # every direction's reduced power as well (y_opt): the in-kernel form
    # serves it at any frame count, also below the GEMV form's 16 frames
    for n in (F, 12):
        kw = dict(precision="fp16", hilo=True, want_y=True)
        a = plan.locate(Xd[:n].contiguous(), mask=md[:n].contiguous(), **kw)
        b = plan.locate(Xz[:n].contiguous(), **kw)
        torch.cuda.synchronize()
        for k in a:
            assert torch.equal(a[k], b[k]), (n, k)
    plan.close()
