"""GPU parity of svdphat_peaks (several separated peaks per frame) with the
oracle's greedy peak picking on the same powers: on the reduced powers
svdphat_locate returns for frames of two simultaneous sources, and on
integer-valued powers full of ties with NaNs, n = 16 and the no-separation
and full-separation limits.  Needs an MI355X and the built library.

The oracle takes its separation decisions in FP64 from the FP64 directions;
the kernel forms the dot products in FP32 from FP32 directions.  Those
differ by at most about 5 u = 3e-7 (u = 2^-24: rounding of the unit vectors,
two of each product's factors, and three FP32 operations, each relative to
sum |x x'| <= 1), so a comparison is undecided only within BAND = 1e-6 of
cos_sep.  Peaks that precede any undecided comparison must equal the
oracle's bit for bit; every peak must pass the oracle's validity check, and
every value must be the frame's power at the returned index."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FS, C, N = 16000.0, 343.0, 512
BAND = 1e-6


def _check(idx, val, y, grid, n, cs):
    """idx/val from the GPU; y [F, Q] the powers the GPU was given."""
    idx = idx.cpu().numpy().astype(np.int64)
    val = val.cpu().numpy()
    ri, rv, dec = oracle.peaks(y, grid, n, float(cs), band=BAND)
    for f in range(y.shape[0]):
        k = dec[f]
        assert np.array_equal(idx[f, :k], ri[f, :k]), f"frame {f}: {idx[f]} vs {ri[f]} (decided {k})"
    assert np.all(oracle.valid_peaks(y, grid, float(cs), BAND, idx))
    rows = np.arange(y.shape[0])[:, None]
    want = np.where(idx >= 0, y[rows, np.maximum(idx, 0)], -np.inf).astype(np.float32)
    assert np.array_equal(val, want)
    return int(np.sum(dec == n))


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


def test_peaks_two_sources(amd, torch):
    print("peaks two sources", flush=True)
    mics = synth.geometry("3d")
    grid = synth.icosphere(3)
    rng = np.random.default_rng(11785700)
    X, dirs, _ = synth.segments(mics, 8, 12, rng, snr_range=(15.0, 15.0), n_src=2, ratio_db_range=(0.0, 0.0))
    X = np.ascontiguousarray(X)
    plan = amd.Plan(mics, grid, FS, C, N, 1e-5)
    out = plan.locate(torch.from_numpy(X).cuda(), precision="fp32", rescore=True, want_y=True)
    y = out["y"]
    d = torch.from_numpy(grid.astype(np.float32)).cuda()
    cs = np.float32(np.cos(np.deg2rad(25.0)))
    idx, val = amd.peaks(y, d, 3, cs)
    torch.cuda.synchronize()
    full = _check(idx, val, y.cpu().numpy(), grid, 3, cs)
    print(f"frames decided in full: {full}/{X.shape[0]}", flush=True)
    # the two leading peaks near the two sources (within 20 degrees) in most frames
    ii = idx.cpu().numpy()
    hit = 0
    for f in range(X.shape[0]):
        src = dirs[f // 12]
        got = grid[ii[f, :2]]
        near = (got @ src.T) >= np.cos(np.deg2rad(20.0))
        hit += bool(near[:, 0].any() and near[:, 1].any())
    print(f"frames with both sources among the two leading peaks: {hit}/{X.shape[0]}", flush=True)
    assert hit >= 0.5 * X.shape[0]
    plan.close()


@pytest.mark.parametrize("n,cos_sep", [(16, 0.9), (5, 1.5), (3, -1.5), (1, 0.5)])
def test_peaks_ties_and_limits(amd, torch, n, cos_sep):
    print(f"peaks ties n={n} cos={cos_sep}", flush=True)
    grid = synth.icosphere(3)
    Q = grid.shape[0]
    rng = np.random.default_rng(11785710 + n)
    F = 37
    y = rng.integers(0, 25, size=(F, Q)).astype(np.float32)   # many equal values
    y[3, rng.integers(0, Q, 50)] = np.nan
    y[4] = np.nan                                              # a frame with nothing to pick
    buf = torch.zeros((F, Q + 9), dtype=torch.float32, device="cuda")
    buf[:, :Q] = torch.from_numpy(y).cuda()
    d = torch.from_numpy(grid.astype(np.float32)).cuda()
    idx, val = amd.peaks(buf[:, :Q], d, n, cos_sep)
    torch.cuda.synchronize()
    _check(idx, val, y, grid, n, np.float32(cos_sep))
    assert np.all(idx.cpu().numpy()[4] == -1)


def test_peaks_large_grid(amd, torch):
    """The benchmark's 10,242-direction grid (161 lane-strided loads per pass),
    smooth random fields with several bumps, n = 8, 15 degrees apart."""
    print("peaks large grid", flush=True)
    grid = synth.icosphere(5)
    Q = grid.shape[0]
    rng = np.random.default_rng(11785720)
    F = 24
    centres = np.array([[synth.random_direction(rng) for _ in range(5)] for _ in range(F)])
    y = np.einsum("fcd,qd->fqc", centres, grid)
    y = np.exp(6.0 * (y - 1.0)).sum(axis=2) + 0.05 * rng.standard_normal((F, Q))
    y = y.astype(np.float32)
    d = torch.from_numpy(grid.astype(np.float32)).cuda()
    cs = np.float32(np.cos(np.deg2rad(15.0)))
    idx, val = amd.peaks(torch.from_numpy(y).cuda(), d, 8, cs)
    torch.cuda.synchronize()
    full = _check(idx, val, y, grid, 8, cs)
    print(f"frames decided in full: {full}/{F}", flush=True)
