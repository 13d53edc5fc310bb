"""Seeded synthetic inputs for SVD-PHAT (Grondin & Glass, arXiv 1811.11785).

This module holds only input generators: microphone geometries, the
candidate-direction grid and multichannel STFT frames of simulated plane
waves.  It contains none of the localisation method's arithmetic (no pair
delays, no steering matrix, no PHAT weighting, no projection) and is shared
by the FP64 oracle, the tests and the benchmark, which each use it to build
the same inputs from the same seed.

Conventions
-----------
* Positions are in metres, directions are unit 3-vectors (x, y, z).
* A plane wave arriving from unit direction ``u`` reaches a microphone at
  position ``r`` earlier by ``r . u / c`` seconds than it reaches the origin,
  so that microphone's signal is the source signal advanced by
  ``fs * r . u / c`` samples.
* STFT: frame length ``N``, hop ``hop``, periodic sine window
  ``w[n] = sin(pi n / N)`` (the square root of a periodic Hann window),
  forward transform ``X[k] = sum_n w[n] x[n] exp(-2 pi i k n / N)`` for
  ``k = 0 .. N/2`` (numpy ``rfft``).  Section 2 of the paper states only that
  a sine window is used; this is the reading adopted throughout.
* Frames are returned as complex64 arrays shaped ``[F, M, N/2+1]``.
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# Microphone geometries: Table 2 of the paper (positions in cm), converted to
# metres.  The planar array keeps the printed y = +-4.3 cm.
# --------------------------------------------------------------------------
_TABLE2_CM = {
    "1d": [(0, 0, -5.0), (0, 0, -3.3), (0, 0, -1.7), (0, 0, 0),
           (0, 0, 1.7), (0, 0, 3.3), (0, 0, 5.0)],
    "2d": [(0, 0, 0), (5, 0, 0), (2.5, 4.3, 0), (-2.5, 4.3, 0),
           (-5.0, 0, 0), (-2.5, -4.3, 0), (2.5, -4.3, 0)],
    "3d": [(0, 0, 0), (-5, 0, 0), (5, 0, 0), (0, -5, 0), (0, 5, 0),
           (0, 0, -5), (0, 0, 5)],
}


def geometry(name: str) -> np.ndarray:
    """Microphone positions (M x 3, metres) of one of the paper's arrays
    (Table 2): ``"1d"`` linear, ``"2d"`` planar, ``"3d"`` three-dimensional."""
    return np.asarray(_TABLE2_CM[name], dtype=np.float64) * 1e-2


# Table 1 of the paper.
TABLE1 = dict(fs=16000.0, c=343.0, N=256, hop=128, Q=2562)

# --------------------------------------------------------------------------
# Candidate-direction grid: recursively subdivided icosahedron.
# --------------------------------------------------------------------------
_PHI = (1.0 + 5.0 ** 0.5) / 2.0
_ICO_V = [(-1, _PHI, 0), (1, _PHI, 0), (-1, -_PHI, 0), (1, -_PHI, 0),
          (0, -1, _PHI), (0, 1, _PHI), (0, -1, -_PHI), (0, 1, -_PHI),
          (_PHI, 0, -1), (_PHI, 0, 1), (-_PHI, 0, -1), (-_PHI, 0, 1)]
_ICO_F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
          (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
          (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
          (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]


def icosphere(level: int) -> np.ndarray:
    """Unit vectors of an icosphere with ``10 * 4**level + 2`` points.

    Level 0 is the icosahedron (vertices at the cyclic permutations of
    (0, +-1, +-phi), normalised).  Each further level splits every triangle
    into four at its edge midpoints, pushed back onto the sphere.  New points
    are appended in order of first appearance, so the points of level ``l``
    are the first ``10 * 4**l + 2`` points of every finer level.

    The paper (Section 4) uses a recursively generated sphere of 2562 points;
    2562 = 10 * 4**4 + 2 is the icosahedral count, so level 4 is that grid.
    """
    if level < 0:
        raise ValueError("level must be >= 0")
    verts = [np.asarray(v, dtype=np.float64) / np.linalg.norm(v) for v in _ICO_V]
    faces = list(_ICO_F)
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        new_faces = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    return np.stack(verts)


def icosphere_count(level: int) -> int:
    return 10 * 4 ** level + 2


# --------------------------------------------------------------------------
# Random draws
# --------------------------------------------------------------------------
def random_direction(rng: np.random.Generator) -> np.ndarray:
    """Uniform direction on the unit sphere (normalised Gaussian 3-vector)."""
    while True:
        v = rng.standard_normal(3)
        n = np.linalg.norm(v)
        if n > 1e-12:
            return v / n


def random_array(M: int, aperture: float, rng: np.random.Generator) -> np.ndarray:
    """M positions uniform in a cube, centred, scaled so that the largest
    pairwise distance equals ``aperture`` metres."""
    r = rng.uniform(-0.5, 0.5, size=(M, 3))
    r -= r.mean(axis=0)
    d = np.sqrt(((r[:, None, :] - r[None, :, :]) ** 2).sum(-1)).max()
    return r * (aperture / d)


def _sine_window(N: int) -> np.ndarray:
    n = np.arange(N)
    return np.sin(np.pi * n / N)


def stft(sig: np.ndarray, N: int, hop: int) -> np.ndarray:
    """STFT of multichannel signals ``sig`` [M, T] -> [F, M, N/2+1] complex128."""
    M, T = sig.shape
    F = 1 + (T - N) // hop
    w = _sine_window(N)
    idx = np.arange(N)[None, :] + hop * np.arange(F)[:, None]        # F x N
    frames = sig[:, idx] * w[None, None, :]                            # M x F x N
    return np.fft.rfft(frames, axis=-1).transpose(1, 0, 2)


def _advance(sig: np.ndarray, adv: np.ndarray) -> np.ndarray:
    """Circularly advance a length-T signal by ``adv[m]`` (fractional) samples
    for every channel m, exactly, in the frequency domain."""
    T = sig.shape[-1]
    S = np.fft.rfft(sig)
    f = np.arange(S.shape[-1])
    ph = np.exp(2j * np.pi * f[None, :] * adv[:, None] / T)
    return np.fft.irfft(S[None, :] * ph, n=T)


def plane_wave_pcm(mics: np.ndarray, dirs, T: int, fs: float, c: float,
                   rng: np.random.Generator, snr_db=None, powers_db=None) -> np.ndarray:
    """Microphone signals [M, T] (float64) of white-Gaussian plane-wave
    source(s): each source advanced by fs r_m . u / c samples per microphone.

    ``dirs`` is one unit vector or a list of them (simultaneous independent
    sources).  ``powers_db`` gives each source's power relative to the first.
    If ``snr_db`` is given, independent white Gaussian noise is added to
    every microphone so that (total source variance) / (noise variance)
    equals that ratio.
    """
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    M = mics.shape[0]
    if powers_db is None:
        powers_db = np.zeros(len(dirs))
    sig = np.zeros((M, T))
    total_var = 0.0
    for u, pdb in zip(dirs, powers_db):
        amp = 10.0 ** (pdb / 20.0)
        s = amp * rng.standard_normal(T)
        adv = fs * (mics @ u) / c
        sig += _advance(s, adv)
        total_var += amp * amp
    if snr_db is not None:
        nvar = total_var / (10.0 ** (snr_db / 10.0))
        sig += np.sqrt(nvar) * rng.standard_normal((M, T))
    return sig


def plane_wave_td(mics: np.ndarray, dirs, F: int, N: int, hop: int, fs: float,
                  c: float, rng: np.random.Generator, snr_db=None,
                  powers_db=None) -> np.ndarray:
    """STFT frames of the signals of ``plane_wave_pcm`` over (F - 1) hop + N
    samples.  Returns complex128 [F, M, N/2+1]."""
    return stft(plane_wave_pcm(mics, dirs, (F - 1) * hop + N, fs, c, rng, snr_db, powers_db), N, hop)


def plane_wave_fd(mics: np.ndarray, u: np.ndarray, F: int, N: int, fs: float,
                  c: float, rng: np.random.Generator, snr_db=None) -> np.ndarray:
    """Frequency-domain plane wave: X_m[k] = S[k] exp(+2 pi i k a_m / N) + n_m[k]
    with a_m = fs r_m . u / c, S[k] complex Gaussian and, if ``snr_db`` is
    given, complex Gaussian noise of per-bin variance E|S|^2 / 10^(snr/10).
    Returns complex128 [F, M, N/2+1]."""
    B = N // 2 + 1
    M = mics.shape[0]
    k = np.arange(B)
    adv = fs * (mics @ np.asarray(u, dtype=np.float64)) / c
    S = (rng.standard_normal((F, B)) + 1j * rng.standard_normal((F, B))) / np.sqrt(2)
    X = S[:, None, :] * np.exp(2j * np.pi * np.outer(adv, k) / N)[None]
    if snr_db is not None:
        sd = np.sqrt(10.0 ** (-snr_db / 10.0) / 2.0)
        X = X + sd * (rng.standard_normal((F, M, B)) + 1j * rng.standard_normal((F, M, B)))
    return X


# --------------------------------------------------------------------------
# Workloads (seed = 11785000 + workload number)
# --------------------------------------------------------------------------
SEED0 = 11785000
STFT = dict(fs=16000.0, c=343.0, N=512, hop=256)


def segments(mics, n_seg: int, seg_frames: int, rng, snr_range=(0.0, 20.0),
             n_src: int = 1, ratio_db_range=(0.0, 6.0), noise=True,
             N=512, hop=256, fs=16000.0, c=343.0):
    """Concatenate ``n_seg`` segments of ``seg_frames`` frames, each with its
    own uniformly random source direction(s) and SNR.  Returns
    (X complex64 [F, M, B], dirs [n_seg, n_src, 3], snr [n_seg])."""
    Xs, D, S = [], [], []
    for _ in range(n_seg):
        dirs = [random_direction(rng) for _ in range(n_src)]
        pw = [0.0] + [-rng.uniform(*ratio_db_range) for _ in range(n_src - 1)]
        snr = rng.uniform(*snr_range) if noise else None
        Xs.append(plane_wave_td(mics, dirs, seg_frames, N, hop, fs, c, rng,
                                snr_db=snr, powers_db=pw))
        D.append(dirs)
        S.append(np.nan if snr is None else snr)
    return (np.concatenate(Xs).astype(np.complex64), np.asarray(D),
            np.asarray(S))


def workload(name: str, frames: int | None = None, seed_offset: int = 0):
    """Inputs of the named workload as a dict.

    ``"linear_q642"``   1-D array, Q=642 (level 3), delta=1e-5, 200 frames of one
                        source at one random direction, 10 dB SNR.
    ``"planar_q10242"`` planar array, Q=10242 (level 5), delta=1e-5, 20000 frames
                        in 100-frame segments, random direction and SNR U[0,20] dB
                        per segment.
    ``"cube_q10242"``   3-D array, Q=10242, delta=1e-5, two white sources with
                        power ratio U[0,6] dB, no sensor noise.
    ``"cube_q40962"``   as above at Q=40962 (level 6).
    ``"planar_q40962"`` planar array, Q=40962, SNR U[-5,20] dB.
    ``frames`` overrides the frame count (rounded up to whole segments).
    """
    spec = {
        "linear_q642": dict(geo="1d", level=3, frames=200, num=1),
        "planar_q10242": dict(geo="2d", level=5, frames=20000, num=2),
        "cube_q10242": dict(geo="3d", level=5, frames=40960, num=3),
        "cube_q40962": dict(geo="3d", level=6, frames=40960, num=3),
        "planar_q40962": dict(geo="2d", level=6, frames=20000, num=5),
    }[name]
    F = spec["frames"] if frames is None else frames
    rng = np.random.default_rng(SEED0 + spec["num"] + 1000 * seed_offset)
    mics = geometry(spec["geo"])
    grid = icosphere(spec["level"])
    if name == "linear_q642":
        u = random_direction(rng)
        X = plane_wave_td(mics, [u], F, STFT["N"], STFT["hop"], STFT["fs"],
                          STFT["c"], rng, snr_db=10.0).astype(np.complex64)
        dirs = np.asarray([[u]])
    else:
        seg = 100
        n_seg = max(1, -(-F // seg))
        if name.startswith("cube"):
            X, dirs, _ = segments(mics, n_seg, seg, rng, n_src=2, noise=False)
        elif name == "planar_q40962":
            X, dirs, _ = segments(mics, n_seg, seg, rng, snr_range=(-5.0, 20.0))
        else:
            X, dirs, _ = segments(mics, n_seg, seg, rng)
        X = X[:F]
    return dict(mics=mics, grid=grid, X=np.ascontiguousarray(X), dirs=dirs,
                delta=1e-5, **STFT)


def workload_pcm(name: str, frames: int | None = None) -> np.ndarray:
    """Microphone signals standing in for the named workload in the time
    domain: float32 [M, T] with T = F hop + (N - hop), so that exactly F
    frames fit.  The signal is a concatenation of 100-frame segments (100 hop
    samples each), each a plane wave from its own uniformly random direction
    at SNR U[0, 20] dB, as in ``segments`` (own seed stream: the workload's
    seed + 100)."""
    spec = {"planar_q10242": dict(geo="2d", frames=20000, num=2),
            "linear_q642": dict(geo="1d", frames=200, num=1)}[name]
    F = spec["frames"] if frames is None else frames
    N, hop = STFT["N"], STFT["hop"]
    rng = np.random.default_rng(SEED0 + spec["num"] + 100)
    mics = geometry(spec["geo"])
    seg = 100
    parts = []
    for _ in range(max(1, -(-F // seg))):
        u = random_direction(rng)
        parts.append(plane_wave_pcm(mics, [u], seg * hop, STFT["fs"], STFT["c"], rng,
                                    snr_db=rng.uniform(0.0, 20.0)))
    tail = plane_wave_pcm(mics, [random_direction(rng)], N - hop, STFT["fs"], STFT["c"], rng,
                          snr_db=rng.uniform(0.0, 20.0))
    sig = np.concatenate(parts + [tail], axis=1)[:, :F * hop + N - hop]
    return np.ascontiguousarray(sig.astype(np.float32))


def ragged_workload(n_arrays: int = 256, seed_offset: int = 0, frames_range=(64, 1024),
                    levels=(3, 4, 5)):
    """Many independent arrays: M ~ U{4..16} microphones at random positions
    within an aperture ~ U[5, 20] cm, grid level ~ U(levels) (642 / 2562 /
    10242 directions), delta ~ U{1e-3, 1e-5}, F ~ U[frames_range] frames of
    one plane-wave source at a random direction with SNR ~ U[0, 20] dB,
    N = 512, hop 256.  Returns a list of dicts (mics, grid_level, delta, X)."""
    rng = np.random.default_rng(SEED0 + 4 + 1000 * seed_offset)
    out = []
    for _ in range(n_arrays):
        M = int(rng.integers(4, 17))
        mics = random_array(M, rng.uniform(0.05, 0.20), rng)
        level = int(rng.choice(levels))
        delta = float(rng.choice([1e-3, 1e-5]))
        F = int(rng.integers(frames_range[0], frames_range[1] + 1))
        u = random_direction(rng)
        X = plane_wave_td(mics, [u], F, STFT["N"], STFT["hop"], STFT["fs"], STFT["c"], rng,
                          snr_db=rng.uniform(0.0, 20.0)).astype(np.complex64)
        out.append(dict(mics=mics, level=level, delta=delta, X=np.ascontiguousarray(X)))
    return out


def plane_wave_fd_torch(mics, n_seg: int, seg_frames: int, N: int, fs: float, c: float, seed: int,
                        snr_range=(-5.0, 20.0), device="cuda"):
    """Frequency-domain plane waves generated directly on a torch device:
    ``n_seg`` segments of ``seg_frames`` frames, each segment with its own
    uniformly random direction and SNR (dB, uniform in ``snr_range``);
    X_m[k] = S[k] exp(+2 pi i k a_m / N) + n_m[k], a_m = fs r_m . u / c,
    S and n complex Gaussian.  Returns complex64 [n_seg * seg_frames, M, N/2+1]."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    M = mics.shape[0]
    B = N // 2 + 1
    F = n_seg * seg_frames
    u = torch.randn(n_seg, 3, generator=g, device=device, dtype=torch.float64)
    u = u / u.norm(dim=1, keepdim=True)
    snr = torch.rand(n_seg, generator=g, device=device, dtype=torch.float64) * (snr_range[1] - snr_range[0]) + snr_range[0]
    r = torch.as_tensor(np.asarray(mics, dtype=np.float64), device=device)
    adv = fs * (u @ r.T) / c                                   # [n_seg, M]
    k = torch.arange(B, device=device, dtype=torch.float64)
    ph = torch.exp(2j * np.pi * adv[:, :, None] * k[None, None, :] / N)   # [n_seg, M, B]
    ph = ph.repeat_interleave(seg_frames, dim=0)
    S = torch.complex(torch.randn(F, B, generator=g, device=device),
                      torch.randn(F, B, generator=g, device=device)) / np.sqrt(2.0)
    sd = torch.sqrt(10.0 ** (-snr / 10.0) / 2.0).repeat_interleave(seg_frames).to(torch.float32)
    noise = torch.complex(torch.randn(F, M, B, generator=g, device=device),
                          torch.randn(F, M, B, generator=g, device=device)) * sd[:, None, None]
    X = S[:, None, :] * ph.to(torch.complex64) + noise
    return X.contiguous()
