"""Learned coarse-cell proposal: cells, FP16 gradients against the FP64
oracle, training on the method's own labels, and proposal search against the
full search.  GPU only."""
import numpy as np
import pytest

import oracle
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


@pytest.fixture(scope="module")
def small(amd):
    mics = synth.geometry("2d")
    fine, coarse = synth.icosphere(4), synth.icosphere(2)
    plan = amd.Plan(mics, fine, 16000.0, 343.0, 256, 1e-5)
    prop = amd.Proposal(plan, coarse, hidden=128, seed=7)
    yield dict(mics=mics, fine=fine, coarse=coarse, plan=plan, prop=prop)
    prop.close()
    plan.close()


def test_cells_match_oracle(small):
    cells = small["prop"].cells()
    ref = oracle.coarse_cells(small["fine"], small["coarse"])
    assert np.array_equal(cells, ref)


def _unpack(flat, D, H, C):
    o = 0
    out = []
    for shape in ((H, D), (H,), (H, H), (H,), (C, H), (C,)):
        n = int(np.prod(shape))
        out.append(flat[o:o + n].reshape(shape).astype(np.float64))
        o += n
    assert o == flat.size
    return out


def test_gradients_match_fp64_oracle(small):
    """FP16 forward/backward kernels against the analytic FP64 backward."""
    prop, plan = small["prop"], small["plan"]
    D, H, C = 2 * plan.info["K"], 128, small["coarse"].shape[0]
    rng = np.random.default_rng(3)
    params = prop.get_params()
    # moderate random weights, exactly representable in FP16
    params = (rng.standard_normal(params.size) * 0.08).astype(np.float16).astype(np.float32)
    prop.set_params(params)
    F = 300
    feat = rng.standard_normal((F, D))
    feat /= np.linalg.norm(feat, axis=1, keepdims=True)
    feat = feat.astype(np.float16).astype(np.float64)
    lab = rng.integers(0, C, F).astype(np.int32)
    loss, g = prop.grad(feat.astype(np.float32), lab)
    P = _unpack(params.astype(np.float64), D, H, C)
    logits, cache = oracle.mlp_forward(P, feat)
    rloss, dl, _ = oracle.softmax_xent(logits, lab)
    ref = oracle.mlp_backward(P, cache, dl)
    assert abs(loss - rloss) <= 2e-3 * abs(rloss)
    G = _unpack(g.astype(np.float64), D, H, C)
    for name, a, b in zip(("W1", "b1", "W2", "b2", "W3", "b3"), G, ref):
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert rel <= 2e-2, f"{name}: relative gradient error {rel:.3e}"


def _frames(torch, mics, n_seg, seed, snr=(-5.0, 20.0), seg=64, N=256):
    rng = np.random.default_rng(seed)
    Xs = []
    for _ in range(n_seg):
        u = synth.random_direction(rng)
        Xs.append(synth.plane_wave_fd(mics, u, seg, N, 16000.0, 343.0, rng, snr_db=rng.uniform(*snr)))
    return torch.from_numpy(np.concatenate(Xs).astype(np.complex64)).cuda()


def test_training_and_proposal_search(amd, torch, small):
    plan = small["plan"]
    prop = amd.Proposal(plan, small["coarse"], hidden=128, seed=11)
    losses = []
    for step in range(120):
        X = _frames(torch, small["mics"], 48, 1000 + step, snr=(0.0, 20.0))
        losses.append(prop.train_step(X, lr=1e-2 if step < 80 else 3e-3))
    print("losses", np.round(losses[::10], 3))
    assert np.mean(losses[-5:]) < 0.35 * np.mean(losses[:3]), losses
    # evaluation on fresh frames against the full search and the FP64 oracle
    X = _frames(torch, small["mics"], 24, 99, snr=(0.0, 20.0))
    out = prop.locate(X, topk=4, conf_min=0.5)
    full = plan.locate(X, precision="fp16", rescore=True, hilo=True)
    torch.cuda.synchronize()
    doa, fell = out["doa"].cpu().numpy(), out["fell_back"].cpu().numpy().astype(bool)
    fdoa = full["doa"].cpu().numpy()
    # frames that fell back ran the full search: identical to it
    assert np.array_equal(doa[fell], fdoa[fell])
    assert fell.mean() < 0.5
    agree = np.mean(doa == fdoa)
    assert agree >= 0.95, agree
    # proposal answers are the exact FP32 rescored power of their direction
    p, fp = out["power"].cpu().numpy(), full["power"].cpu().numpy()
    same = doa == fdoa
    assert np.allclose(p[same], fp[same], rtol=1e-5, atol=1e-3)
    ref_plan = oracle.make_plan(small["mics"], small["fine"], 16000.0, 343.0, 256, 1e-5)
    ref = oracle.locate(ref_plan, X.cpu().numpy())
    judged = ref["margin"] > 1e-5
    print(f"proposal agreement {agree:.4f}, fell back {fell.mean():.3f}, "
          f"vs oracle {np.mean(doa[judged] == ref['doa'][judged]):.4f}")
    prop.close()


def test_proposal_rejects(amd, small):
    with pytest.raises(amd.SvdphatError) as e:
        amd.Proposal(small["plan"], small["coarse"], hidden=100)
    assert e.value.code == amd.E_INVAL
