"""Saved plans and proposals through the C ABI: a plan loaded from its file
locates bit for bit like the original (every precision, the GEMV form of
small batches, the plain form, every direction's reduced powers), reports
the same factorisation and input hash; a proposal saved after training and
loaded onto the loaded plan proposes the same directions and continues
training identically (Adam moments and step count restored), and loading it
onto a plan of other inputs is refused.  Needs an MI355X and the built
library."""
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


def _frames(torch, mics, seed, n_seg=6, seg=50, N=512):
    rng = np.random.default_rng(seed)
    X = np.concatenate([synth.plane_wave_fd(mics, synth.random_direction(rng), seg, N, 16000.0, 343.0, rng,
                                            snr_db=rng.uniform(0, 20)) for _ in range(n_seg)])
    return torch.from_numpy(X.astype(np.complex64)).cuda()


def test_plan_round_trip(amd, torch, tmp_path):
    print("plan save/load", flush=True)
    mics = synth.geometry("2d")
    grid = synth.icosphere(4)
    plan = amd.Plan(mics, grid, 16000.0, 343.0, 512, 1e-5, keep_w=True)
    path = tmp_path / "planar.plan"
    plan.save(path)
    loaded = amd.Plan.load(path)
    a, b = plan.info, loaded.info
    for k in ("M", "Q", "K", "K_paper", "n_classes", "L", "has_w", "residual", "sigma1", "sigmaK", "fro2",
              "u_rownorm_max", "device_bytes", "input_hash"):
        assert a[k] == b[k], k
    assert a["input_hash"] == amd.svdphat_plan_input_hash(mics, grid, 16000.0, 343.0, 512, 1e-5, amd.KEEP_W)
    for x, y in zip(plan.export(), loaded.export()):
        assert np.array_equal(x, y)
    X = _frames(torch, mics, 77)
    for prec, hilo in (("fp16", True), ("bf16", True), ("fp32", False)):
        o1 = plan.locate(X, precision=prec, hilo=hilo, want_y=True)
        o2 = loaded.locate(X, precision=prec, hilo=hilo, want_y=True)
        torch.cuda.synchronize()
        for k in o1:
            assert torch.equal(o1[k], o2[k]), f"{prec}: {k}"
    s1, s2 = plan.locate(X[:9].contiguous()), loaded.locate(X[:9].contiguous())
    r1, r2 = plan.srp_locate(X), loaded.srp_locate(X)
    torch.cuda.synchronize()
    for k in s1:
        assert torch.equal(s1[k], s2[k]), k
    for k in r1:
        assert torch.equal(r1[k], r2[k]), k
    loaded.close()
    plan.close()


def test_proposal_round_trip(amd, torch, tmp_path):
    print("proposal save/load", flush=True)
    mics = synth.geometry("2d")
    fine, coarse = synth.icosphere(4), synth.icosphere(2)
    plan = amd.Plan(mics, fine, 16000.0, 343.0, 256, 1e-5)
    prop = amd.Proposal(plan, coarse, hidden=64, seed=3)
    for step in range(5):
        prop.train_step(_frames(torch, mics, 100 + step, n_seg=8, seg=32, N=256), lr=1e-2)
    plan.save(tmp_path / "fine.plan")
    prop.save(tmp_path / "prop.bin")
    plan2 = amd.Plan.load(tmp_path / "fine.plan")
    prop2 = amd.Proposal.load(plan2, tmp_path / "prop.bin")
    assert np.array_equal(prop.get_params(), prop2.get_params())
    assert np.array_equal(prop.cells(), prop2.cells())
    X = _frames(torch, mics, 999, n_seg=8, seg=32, N=256)
    o1, o2 = prop.locate(X, topk=4, conf_min=0.3), prop2.locate(X, topk=4, conf_min=0.3)
    torch.cuda.synchronize()
    for k in o1:
        assert torch.equal(o1[k], o2[k]), k
    # training continues from the same Adam state and step count
    Xt = _frames(torch, mics, 555, n_seg=8, seg=32, N=256)
    l1, l2 = prop.train_step(Xt, lr=1e-2), prop2.train_step(Xt, lr=1e-2)
    assert l1 == l2
    assert np.array_equal(prop.get_params(), prop2.get_params())
    # a plan of other inputs: refused
    other = amd.Plan(mics, fine, 16000.0, 343.0, 256, 1e-4)
    with pytest.raises(amd.SvdphatError) as e:
        amd.Proposal.load(other, tmp_path / "prop.bin")
    assert e.value.code == amd.E_INVAL
    for o in (prop2, prop, other, plan2, plan):
        o.close()
