"""Ragged batches (many arrays with their own microphones, grids and ranks in
one graph launch) against the FP64 oracle of each array.  GPU only."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

MARGIN_TOL = 1e-5  # FP16 with FP32 rescoring


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


def _arrays(seed, n, max_frames=160):
    """n random arrays: M in 4..16, aperture U[5, 20] cm, grid level 1..3,
    N in {64, 128}, delta in {1e-3, 1e-5}, 1..max_frames frames each."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        M = int(rng.integers(4, 17))
        mics = synth.random_array(M, rng.uniform(0.05, 0.20), rng)
        level = int(rng.integers(1, 4))
        N = int(rng.choice([64, 128]))
        delta = float(rng.choice([1e-3, 1e-5]))
        F = int(rng.integers(1, max_frames + 1))
        u = synth.random_direction(rng)
        X = synth.plane_wave_fd(mics, u, F, N, 16000.0, 343.0, rng, snr_db=rng.uniform(0, 20))
        out.append(dict(mics=mics, grid=synth.icosphere(level), N=N, delta=delta,
                        X=X.astype(np.complex64)))
    return out


@pytest.fixture(scope="module")
def batch(amd, torch):
    arrs = _arrays(4242, 14)
    refs, plans, Xs = [], [], []
    for a in arrs:
        rp = oracle.make_plan(a["mics"], a["grid"], 16000.0, 343.0, a["N"], a["delta"])
        refs.append((rp, oracle.locate(rp, a["X"])))
        plans.append(amd.Plan(a["mics"], a["grid"], 16000.0, 343.0, a["N"], a["delta"]))
        Xs.append(torch.from_numpy(a["X"]).cuda())
    yield dict(arrs=arrs, refs=refs, plans=plans, Xs=Xs)
    for p in plans:
        p.close()


def _check(amd, torch, d, doas, powers, frames=None):
    for i, (rp, ref) in enumerate(d["refs"]):
        n = d["Xs"][i].shape[0] if frames is None else frames[i]
        doa = doas[i].cpu().numpy()[:n]
        pw = powers[i].cpu().numpy()[:n].astype(np.float64)
        judged = ref["margin"][:n] > MARGIN_TOL
        bad = np.flatnonzero(judged & (doa != ref["doa"][:n]))
        assert bad.size == 0, f"array {i}: {bad.size} judged mismatches"
        same = doa == ref["doa"][:n]
        L = rp.W.shape[1]
        assert np.all(np.abs(pw[same] - ref["power"][:n][same]) <= 1e-5 * L + 2e-5 * np.abs(ref["power"][:n][same]))


def test_ragged_matches_oracle(amd, torch, batch):
    d = batch
    rg = amd.Ragged(d["plans"], [x.shape[0] for x in d["Xs"]])
    doas, powers = rg.locate(d["Xs"])
    torch.cuda.synchronize()
    _check(amd, torch, d, doas, powers)
    # the same graph again with fewer frames per array (descriptors change)
    short = [x[: max(0, x.shape[0] // 2)].contiguous() for x in d["Xs"]]
    doas2, powers2 = rg.locate(short)
    torch.cuda.synchronize()
    _check(amd, torch, d, doas2, powers2, frames=[x.shape[0] for x in short])
    # and the full batch once more: identical to the first call
    doas3, _ = rg.locate(d["Xs"])
    torch.cuda.synchronize()
    for a, b in zip(doas, doas3):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    rg.close()


def test_ragged_agrees_with_single_plan_calls(amd, torch, batch):
    d = batch
    rg = amd.Ragged(d["plans"], [x.shape[0] for x in d["Xs"]])
    doas, powers = rg.locate(d["Xs"])
    torch.cuda.synchronize()
    for i, p in enumerate(d["plans"]):
        one = p.locate(d["Xs"][i], precision="fp16", rescore=True, hilo=False)
        torch.cuda.synchronize()
        ref = d["refs"][i][1]
        judged = ref["margin"] > MARGIN_TOL
        assert np.array_equal(one["doa"].cpu().numpy()[judged], doas[i].cpu().numpy()[judged])
    rg.close()


def test_ragged_autotune_cache(amd, torch, batch, tmp_path):
    d = batch
    cache = tmp_path / "tune.jsonl"
    sub = d["plans"][:4]
    mf = [x.shape[0] for x in d["Xs"][:4]]
    rg = amd.Ragged(sub, mf, tune=True, tune_cache=cache)
    tuned, cached = rg.info()
    assert tuned >= 1 and cached == 0
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == tuned and all('"arch": "gfx' in l for l in lines)
    doas, _ = rg.locate(d["Xs"][:4])
    torch.cuda.synchronize()
    for i in range(4):
        ref = d["refs"][i][1]
        judged = ref["margin"] > MARGIN_TOL
        assert np.array_equal(doas[i].cpu().numpy()[judged], ref["doa"][judged])
    rg.close()
    rg2 = amd.Ragged(sub, mf, tune=True, tune_cache=cache)
    tuned2, cached2 = rg2.info()
    assert tuned2 == 0 and cached2 == tuned
    rg2.close()


def test_ragged_rejects(amd, torch, batch):
    d = batch
    rg = amd.Ragged(d["plans"][:2], [4, 4])
    with pytest.raises(amd.SvdphatError) as e:
        rg.locate(d["Xs"][:2] if d["Xs"][0].shape[0] > 4 else [d["Xs"][0][:1].repeat(5, 1, 1), d["Xs"][1][:1]])
    assert e.value.code == amd.E_INVAL
    rg.close()
    nd = amd.Plan(d["arrs"][0]["mics"], d["arrs"][0]["grid"], 16000.0, 343.0, d["arrs"][0]["N"], 1e-3,
                  dedup=False)
    with pytest.raises(amd.SvdphatError) as e:
        amd.Ragged([nd], [8])
    assert e.value.code == amd.E_UNSUPPORTED
    nd.close()
    # only FP16 (with FP32 rescoring) runs in a ragged batch
    rg = amd.Ragged(d["plans"][:2], [8, 8])
    doas = [torch.empty(1, dtype=torch.int32, device="cuda") for _ in range(2)]
    pows = [torch.empty(1, dtype=torch.float32, device="cuda") for _ in range(2)]
    with pytest.raises(amd.SvdphatError) as e:
        amd.svdphat_ragged_locate(rg._h, [x[:1] for x in d["Xs"][:2]], doas, pows, precision=amd.BF16)
    assert e.value.code == amd.E_UNSUPPORTED
    rg.close()


def test_ragged_c4_shapes(amd, torch):
    """Shapes at the ends of the 256-array workload in one batch: 16
    microphones over 20 cm (P = 120, L = 30840, K in the hundreds), 4
    microphones over 5 cm with Q = 10242, and a mid-size array, all at
    N = 512; sampled frames of each against its FP64 oracle."""
    print("ragged C4 shapes", flush=True)
    rng = np.random.default_rng(11785950)
    specs = [(16, 0.20, 3, 1e-5, 300), (4, 0.05, 5, 1e-3, 256), (11, 0.12, 3, 1e-5, 97)]
    plans, Xs, refs = [], [], []
    for M, ap, level, delta, F in specs:
        mics = synth.random_array(M, ap, rng)
        grid = synth.icosphere(level)
        X = np.concatenate([synth.plane_wave_fd(mics, synth.random_direction(rng), 25, 512, 16000.0, 343.0, rng,
                                                snr_db=rng.uniform(0, 20)) for _ in range(-(-F // 25))])[:F]
        X = X.astype(np.complex64)
        rp = oracle.make_plan(mics, grid, 16000.0, 343.0, 512, delta)
        sample = np.unique(np.concatenate([[0, 1, F - 1], np.arange(0, F, 7)]))
        refs.append((rp, sample, oracle.locate(rp, X[sample])))
        plans.append(amd.Plan(mics, grid, 16000.0, 343.0, 512, delta))
        Xs.append(torch.from_numpy(X).cuda())
    Ks = [p.info["K"] for p in plans]
    print(f"  K = {Ks}, Q = {[p.info['Q'] for p in plans]}", flush=True)
    assert max(Ks) >= 200 and [r[0].K for r in refs] == Ks
    rg = amd.Ragged(plans, [x.shape[0] for x in Xs])
    doas, pows = rg.locate(Xs)
    torch.cuda.synchronize()
    for (rp, sample, ref), d, pw in zip(refs, doas, pows):
        d, pw = d.cpu().numpy()[sample], pw.cpu().numpy()[sample]
        judged = ref["margin"] > MARGIN_TOL
        assert np.array_equal(d[judged], ref["doa"][judged])
        same = d == ref["doa"]
        L = rp.W.shape[1]
        assert np.all(np.abs(pw[same] - ref["power"][same]) <= 1e-5 * L + 2e-5 * np.abs(ref["power"][same]))
    rg.close()
    for p in plans:
        p.close()
