"""The normalised search of eq. (15) (mode SVDPHAT_NORMALIZED) through the C
ABI against the FP64 oracle's normalized_locate: tiny random arrays in every
precision, batched and in the GEMV form of small batches, and the full
20000-frame planar batch at Q = 10242 on the stored oracle frames.  Index
exact wherever the oracle's margin exceeds the tolerance of the precision;
yhat = Re{D_q Z} / ||D_q|| within the precision's bound relative to ||Z||;
power is the row power of the chosen direction.  Needs an MI355X and the
built library."""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FS, C = 16000.0, 343.0
MARGIN_TOL = {"fp32": 1e-6, "fp16": 1e-5, "bf16": 1e-5}
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


def _case(seed, M, N, level, F):
    rng = np.random.default_rng(seed)
    mics = synth.random_array(M, rng.uniform(0.04, 0.2), rng)
    grid = synth.icosphere(level)
    X = np.concatenate([synth.plane_wave_fd(mics, synth.random_direction(rng), 8, N, FS, C, rng,
                                            snr_db=rng.uniform(0, 20)) for _ in range(-(-F // 8))])[:F]
    return mics, grid, X.astype(np.complex64)


def _check(out, ref, prec, L):
    doa = out["doa"].cpu().numpy()
    judged = ref["margin"] > MARGIN_TOL[prec]
    bad = np.flatnonzero(judged & (doa != ref["doa"]))
    assert bad.size == 0, f"{prec}: frames {bad[:5]} differ, margins {ref['margin'][bad[:5]]}"
    same = doa == ref["doa"]
    zn = np.abs(ref["yhat"]) / np.maximum(np.abs(ref["score"]), 1e-30)
    yhat = out["yhat"].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(yhat[same] - ref["yhat"][same]) <= Y_TOL[prec] * zn[same] + 1e-6)
    p = out["power"].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(p[same] - ref["power"][same]) <= 1e-5 * L + 2e-5 * np.abs(ref["power"][same]))


CASES = [  # seed, M, N, level, delta, F
    (41, 3, 16, 1, 1e-3, 37),
    (42, 5, 32, 2, 1e-1, 70),
    (43, 7, 512, 3, 1e-5, 130),
    (44, 8, 64, 2, 1e-4, 11),
    (45, 12, 32, 2, 1e-5, 65),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_normalized_tiny(amd, torch, case, prec):
    seed, M, N, level, delta, F = case
    print(f"eq15 case seed={seed} M={M} N={N} level={level} F={F} prec={prec}", flush=True)
    mics, grid, X = _case(seed, M, N, level, F)
    ref_plan = oracle.make_plan(mics, grid, FS, C, N, delta)
    ref = oracle.normalized_locate(ref_plan, X)
    plan = amd.Plan(mics, grid, FS, C, N, delta)
    Xd = torch.from_numpy(X).cuda()
    out = plan.locate(Xd, precision=prec, rescore=True, hilo=True, normalized=True)
    small = plan.locate(Xd[:9].contiguous(), precision=prec, normalized=True)   # GEMV form
    torch.cuda.synchronize()
    L = ref_plan.W.shape[1]
    _check(out, ref, prec, L)
    _check(small, {k: v[:9] for k, v in ref.items()}, "fp32", L)
    plan.close()


def test_normalized_differs_from_eq14(amd, torch):
    """On a strongly truncated plan (delta = 0.1, unequal ||D_q||) eq. (15) and
    eq. (14) pick different directions on some frames, and each form matches
    its own oracle there."""
    mics, grid, X = _case(46, 6, 64, 3, 160)
    ref_plan = oracle.make_plan(mics, grid, FS, C, 64, 1e-1)
    r15 = oracle.normalized_locate(ref_plan, X)
    r14 = oracle.locate(ref_plan, X)
    plan = amd.Plan(mics, grid, FS, C, 64, 1e-1)
    Xd = torch.from_numpy(X).cuda()
    o15 = plan.locate(Xd, precision="fp32", normalized=True)
    o14 = plan.locate(Xd, precision="fp32")
    torch.cuda.synchronize()
    d15, d14 = o15["doa"].cpu().numpy(), o14["doa"].cpu().numpy()
    j = (r15["margin"] > 1e-6) & (r14["margin"] > 1e-6)
    assert np.array_equal(d15[j], r15["doa"][j]) and np.array_equal(d14[j], r14["doa"][j])
    assert np.any(r15["doa"][j] != r14["doa"][j])
    plan.close()


def test_normalized_planar_full_batch(amd, torch):
    print("eq15 planar full batch", flush=True)
    w = synth.workload("planar_q10242")
    gold = dict(np.load(os.path.join(HERE, "golden", "planar_q10242_oracle.npz")))
    plan = amd.Plan(w["mics"], w["grid"], w["fs"], w["c"], w["N"], w["delta"])
    X = torch.from_numpy(w["X"]).cuda()
    n = int(gold["frames"])
    for prec in ("fp16", "fp32"):
        out = plan.locate(X, precision=prec, rescore=True, hilo=True, normalized=True)
        torch.cuda.synchronize()
        doa = out["doa"].cpu().numpy()
        assert np.all((doa >= 0) & (doa < w["grid"].shape[0]))
        judged = gold["nn_margin"] > MARGIN_TOL[prec]
        bad = np.flatnonzero(judged & (doa[:n] != gold["nn_doa"]))
        print(f"  {prec}: match all {np.mean(doa[:n] == gold['nn_doa']):.4%}, "
              f"eq. (14) and (15) differ on {np.mean(gold['nn_doa'] != gold['doa']):.2%} of frames", flush=True)
        assert bad.size == 0, f"{bad.size} judged mismatches, margins {gold['nn_margin'][bad[:5]]}"
        same = doa[:n] == gold["nn_doa"]
        L = plan.info["L"]
        p = out["power"].cpu().numpy()[:n]
        assert np.all(np.abs(p[same] - gold["nn_power"][same]) <= 1e-5 * L + 2e-5 * np.abs(gold["nn_power"][same]))
    plan.close()
