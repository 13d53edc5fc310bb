"""Forced faults (fault injection from the host): with SVDPHAT_FAULT=alloc
every device allocation of the library fails, with SVDPHAT_FAULT=eig the
eigensolver reports no convergence.  Each call must return its defined
status code (no crash, no half-built object), and the library must work
normally once the fault is lifted.  Needs an MI355X and the built library."""
import os

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


@pytest.fixture
def fault(monkeypatch):
    def set_fault(kind):
        if kind:
            monkeypatch.setenv("SVDPHAT_FAULT", kind)
        else:
            monkeypatch.delenv("SVDPHAT_FAULT", raising=False)
    yield set_fault
    monkeypatch.delenv("SVDPHAT_FAULT", raising=False)


def _case():
    rng = np.random.default_rng(606)
    mics = synth.random_array(6, 0.1, rng)
    grid = synth.icosphere(2)
    X = synth.plane_wave_fd(mics, synth.random_direction(rng), 40, 128, 16000.0, 343.0, rng, snr_db=15.0)
    return mics, grid, X.astype(np.complex64)


def test_forced_faults(amd, torch, fault):
    print("forced faults", flush=True)
    mics, grid, X = _case()
    # plan build: allocation failure, then eigensolver failure
    fault("alloc")
    with pytest.raises(amd.SvdphatError) as e:
        amd.Plan(mics, grid, 16000.0, 343.0, 128, 1e-5)
    assert e.value.code == amd.E_NOMEM
    fault("eig")
    with pytest.raises(amd.SvdphatError) as e:
        amd.Plan(mics, grid, 16000.0, 343.0, 128, 1e-5)
    assert e.value.code == amd.E_NUMERIC
    fault(None)
    plan = amd.Plan(mics, grid, 16000.0, 343.0, 128, 1e-5)
    Xd = torch.from_numpy(X).cuda()
    ref = plan.locate(Xd, precision="fp16")
    torch.cuda.synchronize()
    # a call whose workspace must grow fails cleanly and leaves the plan usable
    big = Xd.repeat(64, 1, 1)
    fault("alloc")
    with pytest.raises(amd.SvdphatError) as e:
        plan.locate(big, precision="fp16")
        torch.cuda.synchronize()
    assert e.value.code == amd.E_NOMEM
    # the proposal and a ragged batch report the same
    with pytest.raises(amd.SvdphatError) as e:
        amd.Proposal(plan, synth.icosphere(1), hidden=64, seed=1)
    assert e.value.code == amd.E_NOMEM
    with pytest.raises(amd.SvdphatError) as e:
        amd.Ragged([plan], [40])
    assert e.value.code == amd.E_NOMEM
    fault(None)
    out = plan.locate(Xd, precision="fp16")
    outb = plan.locate(big, precision="fp16")
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(ref[k], out[k]), k
    assert torch.equal(outb["doa"][:40], ref["doa"])
    # and against the oracle
    ro = oracle.locate(oracle.make_plan(mics, grid, 16000.0, 343.0, 128, 1e-5), X)
    judged = ro["margin"] > 1e-5
    assert np.array_equal(out["doa"].cpu().numpy()[judged], ro["doa"][judged])
    # teardown after a failed workspace growth frees every buffer once, and
    # leaves no error behind for the next call
    plan.close()
    again = amd.Plan(mics, grid, 16000.0, 343.0, 128, 1e-5)
    o2 = again.locate(Xd, precision="fp16")
    torch.cuda.synchronize()
    assert torch.equal(o2["doa"], ref["doa"])
    again.close()
