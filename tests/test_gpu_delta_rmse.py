"""Synthetic stand-in for the paper's localisation error over delta (Section
4, eq. (20) with f_1, f_2, f_3): the paper measures speech in simulated
rooms; here seeded time-domain plane waves (12 segments of 24 frames, one
random direction each, 10 dB SNR) at the Table 1 configuration (Q = 2562,
N = 256, hop 128).  Per segment, RMSE_alpha of the GPU's SVD-PHAT (FP32
form, rescored) and of the GPU's plain FP32 SRP-PHAT, each weighted by the
frames' powers; Delta RMSE is their difference averaged over segments.
Prints the table.  Needs an MI355X and the built library."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

DELTAS = [1e-1, 1e-2, 1e-3, 1e-4, 1e-5]
ALPHA = {"1d": 1, "2d": 2, "3d": 3}


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


def _seg_rmse(grid, doa, power, dirs, seg, alpha):
    r = []
    for i, u in enumerate(dirs):
        sl = slice(i * seg, (i + 1) * seg)
        r.append(oracle.rmse_alpha(grid[doa[sl]], power[sl], u, alpha))
    return np.asarray(r)


@pytest.mark.parametrize("geo", ["1d", "2d", "3d"])
def test_delta_rmse(amd, torch, geo):
    print(f"delta rmse {geo}", flush=True)
    t1 = synth.TABLE1
    alpha = ALPHA[geo]
    mics = synth.geometry(geo)
    grid = synth.icosphere(4)
    rng = np.random.default_rng(11785600 + alpha)
    n_seg, seg = 12, 24
    dirs = [synth.random_direction(rng) for _ in range(n_seg)]
    X = np.concatenate([synth.plane_wave_td(mics, [u], seg, t1["N"], t1["hop"], t1["fs"], t1["c"], rng,
                                            snr_db=10.0) for u in dirs]).astype(np.complex64)
    X = np.ascontiguousarray(X)
    Xd = torch.from_numpy(X).cuda()
    ref = amd.Plan(mics, grid, t1["fs"], t1["c"], t1["N"], 1e-5, keep_w=True)
    s = ref.srp_locate(Xd)
    torch.cuda.synchronize()
    r_srp = _seg_rmse(grid, s["doa"].cpu().numpy(), s["power"].cpu().numpy().astype(np.float64), dirs, seg, alpha)
    ref.close()
    rows = []
    for delta in DELTAS:
        plan = amd.Plan(mics, grid, t1["fs"], t1["c"], t1["N"], delta)
        out = plan.locate(Xd, precision="fp32", rescore=True)
        torch.cuda.synchronize()
        K = plan.info["K"]
        plan.close()
        r_svd = _seg_rmse(grid, out["doa"].cpu().numpy(), out["power"].cpu().numpy().astype(np.float64), dirs,
                          seg, alpha)
        rows.append((delta, K, float(r_svd.mean()), float(r_srp.mean()), float((r_svd - r_srp).mean())))
    print(f"\n{geo} (alpha = {alpha}): delta, K, RMSE SVD-PHAT, RMSE SRP-PHAT, Delta RMSE")
    for r in rows:
        print(f"  {r[0]:.0e}  {r[1]:4d}  {r[2]:.4f}  {r[3]:.4f}  {r[4]:+.4f}")
    # at delta = 1e-5 the two methods localise alike (Section 4)
    assert abs(rows[-1][4]) <= 0.02, rows[-1]
    assert np.all(np.isfinite([r[2] for r in rows]))
