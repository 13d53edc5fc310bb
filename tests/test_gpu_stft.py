"""GPU parity of the STFT front end (svdphat_stft) against the FP64 oracle
STFT, and of the whole path from microphone samples (GPU STFT, then
svdphat_locate) against the oracle's STFT and localisation.  Needs an
MI355X and the built library.

Tolerance: the kernel is an FP32 radix-2 FFT with FP32 twiddles, so each
bin's error is O(log2 N u) times the frame's windowed-signal norm (u =
2^-24; about 7e-7 at N = 2048).  The tests allow 1e-5 of that norm."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FS, C = 16000.0, 343.0
REL = 1e-5


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


def _check_stft(Xg, ref, pcm, N, hop):
    F = ref.shape[0]
    assert Xg.shape == ref.shape
    if F == 0:
        return
    w = oracle.sine_window(N)
    for f in range(F):
        nrm = np.linalg.norm(pcm[:, f * hop:f * hop + N] * w[None, :], axis=1)  # per microphone
        err = np.abs(Xg[f] - ref[f]).max(axis=1)
        assert np.all(err <= REL * np.maximum(nrm, 1e-30)), (f, err.max(), nrm.min())


# (M, N, hop, T, extra row stride)
CASES = [
    (7, 512, 256, 256 * 40 + 512 + 100, 0),   # ragged tail: 100 samples left over
    (1, 16, 8, 16, 0),                         # exactly one frame
    (3, 64, 16, 63, 0),                        # shorter than a frame: F = 0
    (4, 2048, 512, 2048 * 3 + 77, 5),          # largest N, odd row stride
    (2, 128, 100, 1000, 37),                   # hop not a power of two
    (16, 256, 128, 128 * 9 + 256, 0),          # many microphones
]


@pytest.mark.parametrize("case", CASES)
def test_stft_parity(amd, torch, case):
    M, N, hop, T, extra = case
    print(f"stft M={M} N={N} hop={hop} T={T} ld=T+{extra}", flush=True)
    rng = np.random.default_rng(11785500 + N + M)
    pcm = rng.standard_normal((M, T)).astype(np.float32)
    pcm[0, : min(T, N)] *= 1e-3                 # a quiet stretch
    if M > 2:
        pcm[2] = 0.0                            # a silent microphone
    ref = oracle.stft(pcm.astype(np.float64), N, hop)
    buf = torch.zeros((M, T + extra), dtype=torch.float32, device="cuda")
    buf[:, :T] = torch.from_numpy(pcm).cuda()
    view = buf[:, :T]
    assert amd.stft_frames(T, N, hop) == ref.shape[0]
    Xg = amd.stft(view, N, hop)
    torch.cuda.synchronize()
    Xg = Xg.cpu().numpy().astype(np.complex128)
    _check_stft(Xg, ref, pcm.astype(np.float64), N, hop)
    if M > 2 and ref.shape[0] > 0:
        assert np.all(Xg[:, 2, :] == 0)


def test_stft_invalid(amd, torch):
    pcm = torch.zeros((2, 1000), dtype=torch.float32, device="cuda")
    X = torch.zeros((4, 2, 251), dtype=torch.complex64, device="cuda")
    with pytest.raises(amd.SvdphatError) as e:
        amd.svdphat_stft(pcm, 500, 250, X)
    assert e.value.code == amd.E_UNSUPPORTED
    with pytest.raises(amd.SvdphatError) as e:
        amd.svdphat_stft(pcm, 4096, 256, X)
    assert e.value.code == amd.E_UNSUPPORTED
    with pytest.raises(amd.SvdphatError) as e:
        amd.svdphat_stft(pcm, 512, 0, X)
    assert e.value.code == amd.E_INVAL
    assert amd.stft_frames(-1, 512, 256) == -1


def test_stft_then_locate(amd, torch):
    """Microphone samples of moving plane-wave sources (segments of 16 frames
    from random directions at random SNR) through the GPU STFT and
    svdphat_locate (FP16, hi/lo), against the oracle's STFT and
    localisation; the GPU STFT also against the oracle's."""
    print("stft then locate", flush=True)
    mics = synth.geometry("2d")
    grid = synth.icosphere(3)
    N, hop, seg = 512, 256, 16
    rng = np.random.default_rng(11785560)
    pcm = np.concatenate([synth.plane_wave_pcm(mics, [synth.random_direction(rng)], seg * hop, FS, C, rng,
                                               snr_db=rng.uniform(0.0, 20.0)) for _ in range(8)], axis=1)
    pcm = np.concatenate([pcm, np.zeros((mics.shape[0], N))], axis=1).astype(np.float32)
    pcm[:, 3 * hop:3 * hop + N] = 0.0            # one silent frame (frame 3)
    ref_X = oracle.stft(pcm.astype(np.float64), N, hop)
    ref_plan = oracle.make_plan(mics, grid, FS, C, N, 1e-5)
    ref = oracle.locate(ref_plan, ref_X)
    plan = amd.Plan(mics, grid, FS, C, N, 1e-5)
    Xg = amd.stft(torch.from_numpy(pcm).cuda(), N, hop)
    out = plan.locate(Xg, precision="fp16", rescore=True, hilo=True)
    torch.cuda.synchronize()
    _check_stft(Xg.cpu().numpy().astype(np.complex128), ref_X, pcm.astype(np.float64), N, hop)
    doa = out["doa"].cpu().numpy()
    judged = ref["margin"] > 1e-5
    assert judged.sum() > 0.8 * len(doa)
    assert np.array_equal(doa[judged], ref["doa"][judged])
    assert doa[3] == ref["doa"][3] and out["power"].cpu().numpy()[3] == 0.0
    plan.close()


def test_stft_full_workload_sampled(amd, torch):
    """The 20,000-frame signal of the benchmark (7 microphones, 5.1M samples
    each) in one call; sampled frames (first, last, random) against the
    oracle frame by frame, every frame finite."""
    print("stft full workload", flush=True)
    N, hop, F = 512, 256, 20000
    pcm = synth.workload_pcm("planar_q10242", F)
    T = pcm.shape[1]
    assert amd.stft_frames(T, N, hop) == F
    Xg = amd.stft(torch.from_numpy(pcm).cuda(), N, hop)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(torch.view_as_real(Xg)).all())
    rng = np.random.default_rng(3)
    for f in np.unique(np.concatenate([[0, 1, F - 1], rng.integers(0, F, 40)])):
        seg = pcm[:, f * hop:f * hop + N].astype(np.float64)
        ref = oracle.stft(seg, N, hop)
        _check_stft(Xg[f:f + 1].cpu().numpy().astype(np.complex128), ref, seg, N, hop)
