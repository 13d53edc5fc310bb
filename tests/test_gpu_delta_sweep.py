"""The rank of eq. (11) over delta (the sweep behind the paper's K(delta)
and gain Q/K curves, Section 4) for the three arrays of Table 2 at the
Table 1 configuration (Q = 2562, N = 256): the GPU plan build's K_paper and
K against the FP64 oracle's, exactly, and the residual energy within the
rule.  Prints the table.  Needs an MI355X and the built library."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

DELTAS = [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7]


@pytest.fixture(scope="module")
def amd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1811_11785_amd as amd
    amd.lib()
    return amd


@pytest.mark.parametrize("geo", ["1d", "2d", "3d"])
def test_delta_sweep_rank(amd, geo):
    t1 = synth.TABLE1
    mics = synth.geometry(geo)
    grid = synth.icosphere(4)
    assert grid.shape[0] == t1["Q"]
    tau = oracle.tdoa_farfield(mics, grid, t1["fs"], t1["c"])
    W = oracle.steering_matrix(tau, t1["N"])
    _, s, _, _, _ = oracle.truncated_svd(W, 1e-5)     # all singular values of W
    E = float(np.sum(np.abs(W) ** 2))
    rows = []
    for delta in DELTAS:
        print(f"delta sweep {geo} delta={delta}", flush=True)
        Kp, K = oracle.choose_rank(s, delta, energy=E)
        plan = amd.Plan(mics, grid, t1["fs"], t1["c"], t1["N"], delta)
        info = plan.info
        plan.close()
        assert info["K_paper"] == Kp, (geo, delta, info["K_paper"], Kp)
        assert info["K"] == K, (geo, delta, info["K"], K)
        assert info["residual"] <= delta * (1 + 1e-6) + 1e-12
        rows.append((delta, Kp, K, t1["Q"] / K))
    print(f"\n{geo}: delta, K_paper, K, Q/K")
    for r in rows:
        print(f"  {r[0]:.0e}  {r[1]:4d}  {r[2]:4d}  {r[3]:7.1f}")
    # K grows as delta shrinks
    assert all(a[2] <= b[2] for a, b in zip(rows, rows[1:]))
