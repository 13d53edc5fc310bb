"""Pins of the FP64 oracle against what the paper and the mathematics fix,
independently of the oracle's own formulas (CPU only)."""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _small(M=4, N=16, level=1, seed=0, geo=None):
    rng = np.random.default_rng(seed)
    mics = synth.geometry(geo) if geo else synth.random_array(M, 0.08, rng)
    grid = synth.icosphere(level)
    return mics, grid, rng


# ------------------------------------------------------------------ P4
def _golden_gains():
    rows = {}
    with open(os.path.join(HERE, "golden", "table1_gains.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                g, v = line.split()
                rows[g] = int(v)
    return rows


@pytest.mark.parametrize("geo", ["1d", "2d", "3d"])
def test_p4_paper_gains(geo):
    """Section 4: delta = 1e-5 gives Q/K = 320 / 53 / 36 with the Table 1
    parameters and the Table 2 arrays."""
    t1 = synth.TABLE1
    mics = synth.geometry(geo)
    grid = synth.icosphere(4)
    assert grid.shape[0] == t1["Q"]
    tau = oracle.tdoa_farfield(mics, grid, t1["fs"], t1["c"])
    W = oracle.steering_matrix(tau, t1["N"])
    _, s, _, Kp, K = oracle.truncated_svd(W, 1e-5)
    assert int(t1["Q"] / Kp) == _golden_gains()[geo]
    # P1 on the same matrix: every entry of eq. (4) has unit modulus.
    assert abs(np.sum(s ** 2) / W.size - 1.0) < 1e-12


# ------------------------------------------------------------------ P1, P3
def test_p1_p3_energy_and_residual():
    mics, grid, _ = _small(M=5, N=32, level=2)
    tau = oracle.tdoa_farfield(mics, grid, 16000.0, 343.0)
    W = oracle.steering_matrix(tau, 32)
    Q, L = W.shape
    assert np.allclose(np.abs(W), 1.0, atol=1e-15)
    for delta in (1e-1, 1e-3, 1e-5):
        U, s, Vh, Kp, K = oracle.truncated_svd(W, delta)
        E = Q * L
        assert abs(np.sum(s ** 2) - E) < 1e-9 * E
        # explicit reconstruction residual, eq. (11)
        WK = (U * s[:K]) @ Vh
        res = np.sum(np.abs(W - WK) ** 2) / E
        assert res <= delta * (1 + 1e-9)
        assert abs(res - np.sum(s[K:] ** 2) / E) < 1e-10
        # K_paper is the smallest rank that satisfies eq. (11)
        if Kp > 1:
            assert np.sum(s[:Kp - 1] ** 2) < (1 - delta) * E
        # columns of U and V are orthonormal
        assert np.allclose(U.conj().T @ U, np.eye(K), atol=1e-10)
        assert np.allclose(Vh @ Vh.conj().T, np.eye(K), atol=1e-10)


def test_rank_rule_cluster_extension():
    s = np.array([5.0, 3.0, 2.0, 2.0, 2.0, 1.0, 0.1])
    E = np.sum(s ** 2)
    # cut at K=3 falls inside the cluster {2,2,2}: extended to 5
    delta = 1 - np.sum(s[:3] ** 2) / E
    Kp, K = oracle.choose_rank(s, delta * 1.000001)
    assert Kp == 3 and K == 5
    Kp, K = oracle.choose_rank(s, 1e-12)
    assert Kp == K == 7
    # eq. (11) takes a positive delta
    for bad in (0.0, -1e-5):
        with pytest.raises(ValueError):
            oracle.choose_rank(s, bad)


# ------------------------------------------------------------------ P2
def test_p2_full_rank_equals_srp():
    """With every singular value kept, eqs. (12)-(14) reproduce eq. (9) to
    rounding; with a tiny delta the difference is bounded by the first
    dropped singular value times ||x||."""
    for level, seed in ((0, 3), (2, 3)):
        mics, grid, rng = _small(M=4, N=16, level=level, seed=seed)
        tau = oracle.tdoa_farfield(mics, grid, 16000.0, 343.0)
        W = oracle.steering_matrix(tau, 16)
        U, s, Vh, Kp, K = oracle.truncated_svd(W, 1e-13)
        X = rng.standard_normal((6, 4, 9)) + 1j * rng.standard_normal((6, 4, 9))
        x = oracle.phat_vector(X)
        y_srp = oracle.srp_phat_power(W, x)
        y_svd = oracle.svd_phat_power(U, s, Vh, x)
        dropped = s[K] if K < s.size else 0.0
        bound = dropped * np.linalg.norm(x, axis=1)[:, None] + 1e-10 * W.shape[1]
        assert np.all(np.abs(y_srp - y_svd) <= bound)
        if level == 0:
            assert K == s.size  # full rank: equality to rounding
            assert np.max(np.abs(y_srp - y_svd)) <= 1e-10 * W.shape[1]
        # stacked real form gives the same numbers
        Ast, Ust = oracle.stacked_projection(U, s, Vh)
        xs = np.concatenate([x.real, x.imag], axis=1)
        assert np.allclose((xs @ Ast.T) @ Ust.T, y_svd, atol=1e-9)


# ------------------------------------------------------------------ P10 brute force
def test_p10_brute_force_eq5():
    """Eq. (5) written as three explicit loops with eqs. (2)-(4), against the
    matrix form of eq. (9) and the argmax of eq. (6)."""
    M, N, fs, c = 3, 8, 16000.0, 343.0
    mics, grid, rng = _small(M=M, N=N, level=1, seed=7)
    X = rng.standard_normal((2, M, N // 2 + 1)) + 1j * rng.standard_normal((2, M, N // 2 + 1))
    W = oracle.steering_matrix(oracle.tdoa_farfield(mics, grid, fs, c), N)
    y = oracle.srp_phat_power(W, oracle.phat_vector(X))
    for f in range(2):
        ybf = []
        for s in grid:
            sh = s / math.sqrt(sum(v * v for v in s))
            acc = 0j
            for i in range(M):
                for j in range(i + 1, M):
                    tau = fs / c * sum((mics[j][d] - mics[i][d]) * sh[d] for d in range(3))
                    for k in range(N // 2 + 1):
                        Xi, Xj = X[f, i, k], X[f, j, k]
                        xij = Xi * Xj.conjugate() / (abs(Xi) * abs(Xj))
                        acc += complex(math.cos(2 * math.pi * k * tau / N),
                                       math.sin(2 * math.pi * k * tau / N)) * xij
            ybf.append(acc.real)
        assert np.allclose(y[f], ybf, atol=1e-12)
        best = max(range(len(ybf)), key=lambda q: (ybf[q], -q))
        assert int(np.argmax(y[f])) == best


# ------------------------------------------------------------------ P6, P7
@pytest.mark.parametrize("geo", ["1d", "2d", "3d"])
def test_p7_dirichlet_closed_form(geo):
    """Noiseless off-grid plane wave: eq. (9) equals the Dirichlet-kernel sum."""
    N, fs, c = 512, 16000.0, 343.0
    mics = synth.geometry(geo)
    grid = synth.icosphere(2)
    rng = np.random.default_rng(11)
    u = synth.random_direction(rng)
    X = synth.plane_wave_fd(mics, u, 3, N, fs, c, rng)
    x = oracle.phat_vector(X)
    tau = oracle.tdoa_farfield(mics, grid, fs, c)
    y = oracle.srp_phat_power(oracle.steering_matrix(tau, N), x)
    # pair delays of the source direction, from the microphone advances
    a = fs * (mics @ u) / c
    tsrc = np.array([a[j] - a[i] for i, j in oracle.mic_pairs(7)])
    yc = oracle.dirichlet_power(tau, tsrc, N)
    L = 21 * (N // 2 + 1)
    for f in range(3):
        assert np.max(np.abs(y[f] - yc)) <= 1e-9 * L


@pytest.mark.parametrize("geo", ["1d", "2d", "3d"])
def test_p6_on_grid_plane_wave(geo):
    """A noiseless plane wave from grid direction q0 gives Y_q0 = L, the
    maximum, for SRP-PHAT and for the truncated SVD-PHAT at delta = 1e-5."""
    N, fs, c = 512, 16000.0, 343.0
    mics = synth.geometry(geo)
    grid = synth.icosphere(3)
    plan = oracle.make_plan(mics, grid, fs, c, N, 1e-5)
    rng = np.random.default_rng(5)
    L = plan.W.shape[1]
    for q0 in rng.choice(grid.shape[0], 12, replace=False):
        X = synth.plane_wave_fd(mics, grid[q0], 1, N, fs, c, rng)
        x = oracle.phat_vector(X)
        y = oracle.srp_phat_power(plan.W, x)[0]
        assert abs(y[q0] - L) < 1e-8 * L
        qbar, _, _ = oracle.argmax_with_margin(y, plan.rep)
        assert qbar[0] == plan.rep[q0]
        ysvd = oracle.svd_phat_power(plan.U, plan.s, plan.Vh, x)
        qs, _, _ = oracle.argmax_with_margin(ysvd, plan.rep)
        assert qs[0] == plan.rep[q0]


def test_p6_time_domain_generator():
    """The time-domain generator (fractional advance + sine-window STFT)
    agrees with the sign conventions: a noiseless wave from a grid direction
    is localised at that direction's class."""
    N, fs, c = 512, 16000.0, 343.0
    mics = synth.geometry("3d")
    grid = synth.icosphere(3)
    tau = oracle.tdoa_farfield(mics, grid, fs, c)
    W = oracle.steering_matrix(tau, N)
    rep = oracle.direction_classes(tau)
    rng = np.random.default_rng(2)
    for q0 in rng.choice(grid.shape[0], 6, replace=False):
        X = synth.plane_wave_td(mics, [grid[q0]], 4, N, 256, fs, c, rng)
        y = oracle.srp_phat_power(W, oracle.phat_vector(X))
        qbar, _, _ = oracle.argmax_with_margin(y, rep)
        assert np.all(qbar == rep[q0])


# ------------------------------------------------------------------ P8
def test_p8_row_bound():
    N, fs, c = 512, 16000.0, 343.0
    mics = synth.geometry("2d")
    grid = synth.icosphere(2)
    plan = oracle.make_plan(mics, grid, fs, c, N, 1e-3)
    rng = np.random.default_rng(8)
    X = synth.plane_wave_fd(mics, synth.random_direction(rng), 8, N, fs, c, rng, snr_db=5)
    x = oracle.phat_vector(X)
    ys = oracle.srp_phat_power(plan.W, x)
    yv = oracle.svd_phat_power(plan.U, plan.s, plan.Vh, x)
    D = plan.U * plan.s[:plan.K]
    r2 = plan.W.shape[1] - np.sum(np.abs(D) ** 2, axis=1)          # ||r_q||^2
    WK = D @ plan.Vh
    assert np.allclose(r2, np.sum(np.abs(plan.W - WK) ** 2, axis=1), atol=1e-8)
    bound = np.sqrt(np.maximum(r2, 0))[None, :] * np.linalg.norm(x, axis=1)[:, None]
    assert np.all(np.abs(ys - yv) <= bound + 1e-9)


# ------------------------------------------------------------------ P9
def test_p9_metamorphic():
    N, fs, c = 32, 16000.0, 343.0
    mics, grid, rng = _small(M=4, N=N, level=2, seed=9)
    B = N // 2 + 1
    X = rng.standard_normal((3, 4, B)) + 1j * rng.standard_normal((3, 4, B))
    x = oracle.phat_vector(X)
    # per-mic positive gains and a common per-bin phase leave x unchanged
    a = rng.uniform(0.1, 10, size=(1, 4, B))
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, size=(1, 1, B)))
    assert np.allclose(oracle.phat_vector(X * a * ph), x, atol=1e-12)
    tau = oracle.tdoa_farfield(mics, grid, fs, c)
    y = oracle.srp_phat_power(oracle.steering_matrix(tau, N), x)
    # relabelling the microphones leaves every power unchanged
    perm = [2, 0, 3, 1]
    tau2 = oracle.tdoa_farfield(mics[perm], grid, fs, c)
    y2 = oracle.srp_phat_power(oracle.steering_matrix(tau2, N), oracle.phat_vector(X[:, perm]))
    assert np.allclose(y, y2, atol=1e-10)
    # permuting the grid permutes the powers
    gp = rng.permutation(grid.shape[0])
    tau3 = oracle.tdoa_farfield(mics, grid[gp], fs, c)
    y3 = oracle.srp_phat_power(oracle.steering_matrix(tau3, N), x)
    assert np.allclose(y3, y[:, gp], atol=1e-10)
    # a silent bin of one microphone removes that bin's pairs
    Xz = X.copy()
    Xz[:, 1, 3] = 0
    xz = oracle.phat_vector(Xz).reshape(3, 6, B)
    for p, (i, j) in enumerate(oracle.mic_pairs(4)):
        if 1 in (i, j):
            assert np.all(xz[:, p, 3] == 0)


# ------------------------------------------------------------------ classes
def test_classes_follow_array_symmetry():
    """A linear array along z only sees s_z; a planar array in z = 0 cannot
    tell +z from -z.  The classes must be exactly those."""
    grid = synth.icosphere(3)
    fs, c = 16000.0, 343.0
    r1 = oracle.direction_classes(oracle.tdoa_farfield(synth.geometry("1d"), grid, fs, c))
    key = np.round(grid[:, 2], 9)
    for q in range(grid.shape[0]):
        assert r1[q] == np.flatnonzero(key == key[q])[0]
    r2 = oracle.direction_classes(oracle.tdoa_farfield(synth.geometry("2d"), grid, fs, c))
    kx, ky = np.round(grid[:, 0], 9), np.round(grid[:, 1], 9)
    for q in range(grid.shape[0]):
        assert r2[q] == np.flatnonzero((kx == kx[q]) & (ky == ky[q]))[0]
    r3 = oracle.direction_classes(oracle.tdoa_farfield(synth.geometry("3d"), grid, fs, c))
    assert np.all(r3 == np.arange(grid.shape[0]))


def test_margin_between_classes():
    y = np.array([[1.0, 3.0, 3.0, 2.0]])
    rep = np.array([0, 1, 1, 3])
    q, y1, m = oracle.argmax_with_margin(y, rep)
    assert q[0] == 1 and y1[0] == 3.0 and abs(m[0] - 1 / 3) < 1e-15


def test_exact_power_is_row_of_srp():
    N = 64
    mics, grid, rng = _small(M=4, N=N, level=1, seed=4)
    tau = oracle.tdoa_farfield(mics, grid, 16000.0, 343.0)
    W = oracle.steering_matrix(tau, N)
    X = rng.standard_normal((2, 4, N // 2 + 1)) + 1j * rng.standard_normal((2, 4, N // 2 + 1))
    x = oracle.phat_vector(X)
    y = oracle.srp_phat_power(W, x)
    for q in (0, 5, 41):
        assert abs(oracle.exact_power(tau[q], N, x[1]) - y[1, q]) < 1e-10


# ------------------------------------------------------------------ grid
def test_icosphere_counts_and_nesting():
    for lv in range(5):
        g = synth.icosphere(lv)
        assert g.shape == (synth.icosphere_count(lv), 3)
        assert np.allclose(np.linalg.norm(g, axis=1), 1.0)
    g3, g5 = synth.icosphere(3), synth.icosphere(5)
    assert np.array_equal(g5[:642], g3)
    # all points distinct
    d = g3 @ g3.T - 2 * np.eye(642)
    assert d.max() < 1 - 1e-6


# ------------------------------------------------------------------ MLP (proposal)
def _mlp(rng, i=6, h=5, o=4):
    return [rng.standard_normal((h, i)) * 0.5, rng.standard_normal(h) * 0.1,
            rng.standard_normal((h, h)) * 0.5, rng.standard_normal(h) * 0.1,
            rng.standard_normal((o, h)) * 0.5, rng.standard_normal(o) * 0.1]


def test_gelu_definition():
    from scipy.stats import norm
    x = np.linspace(-6, 6, 101)
    assert np.allclose(oracle.gelu(x), x * norm.cdf(x), atol=1e-14)
    h = 1e-6
    fd = (oracle.gelu(x + h) - oracle.gelu(x - h)) / (2 * h)
    assert np.allclose(oracle.gelu_grad(x), fd, atol=1e-8)


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(1)
    params = _mlp(rng)
    f = rng.standard_normal((7, 6))
    lab = rng.integers(0, 4, 7)
    logits, cache = oracle.mlp_forward(params, f)
    loss, dl, _ = oracle.softmax_xent(logits, lab)
    grads = oracle.mlp_backward(params, cache, dl)
    h = 1e-5
    for P, G in zip(params, grads):
        for idx in itertools.islice(np.ndindex(P.shape), 0, None, 3):
            old = P[idx]
            P[idx] = old + h
            lp, _, _ = oracle.softmax_xent(oracle.mlp_forward(params, f)[0], lab)
            P[idx] = old - h
            lm, _, _ = oracle.softmax_xent(oracle.mlp_forward(params, f)[0], lab)
            P[idx] = old
            assert abs((lp - lm) / (2 * h) - G[idx]) < 1e-7


def test_adam_first_step():
    """First Adam step moves each parameter by lr * g / (|g| + eps')."""
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = oracle.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-4)


def test_adam_constant_gradient_steps():
    """With the same gradient at every step the bias-corrected moments are
    m^ = g and v^ = g^2 at every t, so each of three steps moves a parameter
    by lr g / (|g| + eps); a missing or stale bias correction moves it by a
    different amount from the second step on."""
    g = np.array([0.5, -3.0, 2e-2, -1e-3])
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    lr, eps = 0.01, 1e-8
    for t in (1, 2, 3):
        p, m, v = oracle.adam_step(p, g, m, v, t, lr=lr, eps=eps)
        assert np.allclose(p, -t * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_proposal_features_pins():
    """The network input [Re z, Im z] / ||z||: a worked example, unit norm,
    invariance under a positive scale of z, zero for z = 0, and a Gram
    matrix over frames that a unitary change of the singular-vector basis
    (a phase per component) leaves unchanged."""
    z = np.array([[1 + 2j, 3 + 0j], [0j, 0j], [0j, -2j]])
    f = oracle.proposal_features(z)
    assert np.allclose(f[0], np.array([1.0, 3.0, 2.0, 0.0]) / np.sqrt(14.0), atol=1e-15)
    assert np.array_equal(f[1], np.zeros(4))
    assert np.allclose(f[2], [0.0, 0.0, 0.0, -1.0], atol=1e-15)
    rng = np.random.default_rng(24)
    z = rng.standard_normal((9, 6)) + 1j * rng.standard_normal((9, 6))
    f = oracle.proposal_features(z)
    assert np.allclose(np.linalg.norm(f, axis=1), 1.0, atol=1e-14)
    assert np.allclose(oracle.proposal_features(z * 37.5), f, atol=1e-14)
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, 6))
    g = oracle.proposal_features(z * ph[None, :])
    assert np.allclose(g @ g.T, f @ f.T, atol=1e-13)
    assert not np.allclose(g, f, atol=1e-3)


def test_coarse_cells_nesting():
    fine = synth.icosphere(4)
    coarse = synth.icosphere(2)
    cell = oracle.coarse_cells(fine, coarse)
    assert np.array_equal(cell[:coarse.shape[0]], np.arange(coarse.shape[0]))
    # brute force nearest by angle
    for q in range(0, fine.shape[0], 97):
        ang = np.arccos(np.clip(coarse @ fine[q], -1, 1))
        assert ang[cell[q]] <= ang.min() + 1e-9


# ------------------------------------------------------------ STFT front end
def _geom_sum(alpha, N):
    """sum_{n<N} exp(i alpha n), closed form (alpha not a multiple of 2 pi)."""
    return (1 - np.exp(1j * alpha * N)) / (1 - np.exp(1j * alpha))


@pytest.mark.parametrize("N,hop,k0", [(512, 256, 37.3), (64, 16, 5.0), (16, 8, 2.71)])
def test_stft_tone_closed_form(N, hop, k0):
    """A cosine A cos(theta t + phi) (on or off a bin) through the sine
    window: writing w[n] = (e^{i pi n/N} - e^{-i pi n/N}) / 2i makes every
    bin a sum of four geometric series, in closed form, frame by frame."""
    A, phi, F = 1.7, 0.4, 5
    theta = 2 * np.pi * k0 / N
    T = (F - 1) * hop + N
    pcm = (A * np.cos(theta * np.arange(T) + phi))[None, :]
    X = oracle.stft(pcm, N, hop)[:, 0, :]
    k = np.arange(N // 2 + 1)
    for f in range(F):
        pf = phi + theta * f * hop
        b = 2 * np.pi * k / N
        s = lambda a: _geom_sum(a, N)
        ref = A / (4j) * (np.exp(1j * pf) * (s(theta + np.pi / N - b) - s(theta - np.pi / N - b))
                          + np.exp(-1j * pf) * (s(-theta + np.pi / N - b) - s(-theta - np.pi / N - b)))
        assert np.abs(X[f] - ref).max() <= 1e-9 * N


def test_stft_brute_force_tiny():
    """Tiny case against the double sum written with math.cos / math.sin."""
    rng = np.random.default_rng(4)
    N, hop, M, T = 8, 3, 2, 20
    pcm = rng.standard_normal((M, T))
    X = oracle.stft(pcm, N, hop)
    F = 1 + (T - N) // hop
    assert X.shape == (F, M, N // 2 + 1)
    for f in range(F):
        for m in range(M):
            for k in range(N // 2 + 1):
                re = im = 0.0
                for n in range(N):
                    v = math.sin(math.pi * n / N) * pcm[m, f * hop + n]
                    re += v * math.cos(2 * math.pi * k * n / N)
                    im -= v * math.sin(2 * math.pi * k * n / N)
                assert abs(X[f, m, k] - complex(re, im)) < 1e-12


def test_stft_frames_and_shift():
    """Frame count 1 + (T - N) // hop (0 below one frame), and shifting the
    signal by one hop shifts the frames by one."""
    assert oracle.stft_frames(15, 16, 8) == 0
    assert oracle.stft_frames(16, 16, 8) == 1
    assert oracle.stft_frames(23, 16, 8) == 1
    assert oracle.stft_frames(24, 16, 8) == 2
    assert oracle.stft(np.zeros((3, 10)), 16, 8).shape == (0, 3, 9)
    rng = np.random.default_rng(8)
    pcm = rng.standard_normal((3, 200))
    X = oracle.stft(pcm, 32, 12)
    Xs = oracle.stft(pcm[:, 12:], 32, 12)
    assert np.allclose(X[1:1 + Xs.shape[0]], Xs, rtol=0, atol=1e-12)


# ------------------------------------------------- error measure, eq. (20)
def test_doa_maps():
    """f_1 keeps only the elevation (unit vectors in the x-z half plane,
    the same for every azimuth); f_2 folds z; f_3 is the identity."""
    rng = np.random.default_rng(12)
    s = np.array([synth.random_direction(rng) for _ in range(50)])
    f1 = oracle.doa_map(s, 1)
    assert np.allclose(np.linalg.norm(f1, axis=1), 1.0) and np.all(f1[:, 1] == 0) and np.all(f1[:, 0] >= 0)
    assert np.allclose(f1[:, 2], s[:, 2])                      # sin(elevation) = s_z on the unit sphere
    rot = s @ np.array([[0.6, -0.8, 0], [0.8, 0.6, 0], [0, 0, 1.0]]).T   # any azimuth rotation
    assert np.allclose(oracle.doa_map(rot, 1), f1)
    xz = np.array([[np.cos(a), 0.0, np.sin(a)] for a in np.linspace(-1.5, 1.5, 7)])
    assert np.allclose(oracle.doa_map(xz, 1), xz)
    f2 = oracle.doa_map(s, 2)
    assert np.allclose(f2[:, :2], s[:, :2]) and np.allclose(f2[:, 2], np.abs(s[:, 2]))
    assert np.array_equal(oracle.doa_map(s, 3), s)


def test_rmse_alpha_cases():
    """Eq. (20): zero when every estimate is the true direction, whatever
    the weights; the distance of the one estimate when all agree; the
    weighted mean for two estimates; mirror images count as equal for the
    planar array."""
    s0 = np.array([0.0, 0.6, 0.8])
    a = np.array([0.6, 0.0, 0.8])
    Y = np.array([1.0, 3.0, 0.5])
    for alpha in (1, 2, 3):
        assert oracle.rmse_alpha(np.tile(s0, (3, 1)), Y, s0, alpha) < 1e-15
    assert abs(oracle.rmse_alpha(np.tile(a, (3, 1)), Y, s0, 3) - np.linalg.norm(a - s0)) < 1e-15
    est = np.stack([s0, a])
    w = np.array([1.0, 3.0])
    want = np.linalg.norm((s0 * 1 + a * 3) / 4 - s0)
    assert abs(oracle.rmse_alpha(est, w, s0, 3) - want) < 1e-15
    mirror = np.array([[0.0, 0.6, -0.8]])
    assert oracle.rmse_alpha(mirror, np.ones(1), s0, 2) < 1e-15
    assert oracle.rmse_alpha(mirror, np.ones(1), s0, 3) > 1.5
    # the linear array sees azimuth as nothing: a = s0 rotated about z
    assert oracle.rmse_alpha(np.array([[0.6, 0.0, 0.8]]), np.ones(1), s0, 1) < 1e-15


# ---------------------------------------------------- several sources (peaks)
def test_peaks_no_separation_is_top_n():
    """With a separation no pair of directions meets (cos_sep > 1), the
    peaks are the n largest values in decreasing order, ties to the lower
    index (numpy's stable sort)."""
    rng = np.random.default_rng(21)
    grid = synth.icosphere(2)
    y = rng.integers(0, 40, size=(30, grid.shape[0])).astype(np.float32)   # many ties
    idx, val, dec = oracle.peaks(y, grid, 5, 1.5, band=1e-6)
    assert np.all(dec == 5)
    for f in range(30):
        order = np.argsort(-y[f], kind="stable")[:5]
        assert np.array_equal(idx[f], order) and np.array_equal(val[f], y[f, order])


def test_peaks_full_separation_and_separated_bumps():
    """cos_sep below -1 removes every direction after the first peak; two bumps
    far apart are both found, each at its own maximum, and a third peak
    never lies within the separation of the first two."""
    grid = synth.icosphere(3)
    rng = np.random.default_rng(22)
    y = rng.standard_normal((4, grid.shape[0])).astype(np.float32)
    idx, val, _ = oracle.peaks(y, grid, 3, -1.5)
    assert np.array_equal(idx[:, 0], np.argmax(y, axis=1)) and np.all(idx[:, 1:] == -1)
    assert np.all(np.isinf(val[:, 1:]))
    ia = 17
    ib = int(np.argmin(np.abs(grid @ grid[ia])))    # about 90 degrees away
    a, b = grid[ia], grid[ib]
    assert abs(a @ b) < 0.1
    yb = (np.exp(8 * (grid @ a - 1)) + 0.8 * np.exp(8 * (grid @ b - 1))).astype(np.float32)[None]
    idx, _, _ = oracle.peaks(yb, grid, 3, np.cos(np.deg2rad(30)))
    assert idx[0, 0] == ia and idx[0, 1] == ib
    assert grid[idx[0, 2]] @ a < np.cos(np.deg2rad(30)) and grid[idx[0, 2]] @ b < np.cos(np.deg2rad(30))


def test_peaks_pair_at_the_separation():
    """A direction whose dot product with the first peak is exactly cos_sep
    is too close (the comparison is 'below cos_sep' for a free direction);
    one ulp of cos_sep higher it is free.  The pair (1, 0, 0), (0.6, 0.8, 0)
    has the dot product fl(0.6) exactly in FP64.  Within a band around
    cos_sep the oracle reports only the first peak as decided, and the
    validity check accepts either choice there but rejects a peak that is
    clearly too close or clearly not the largest free power."""
    dirs = np.array([[1.0, 0.0, 0.0], [0.6, 0.8, 0.0], [-1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    assert dirs[1] @ dirs[0] == 0.6
    y = np.array([[4.0, 3.0, 1.0, 2.0]])
    idx, val, dec = oracle.peaks(y, dirs, 2, 0.6)
    assert idx[0].tolist() == [0, 3] and val[0].tolist() == [4.0, 2.0] and dec[0] == 2
    idx, _, _ = oracle.peaks(y, dirs, 2, np.nextafter(0.6, 1.0))
    assert idx[0].tolist() == [0, 1]
    _, _, dec = oracle.peaks(y, dirs, 2, 0.6, band=1e-6)
    assert dec[0] == 1
    for second, ok in ((1, True), (3, True), (2, False)):
        assert oracle.valid_peaks(y, dirs, 0.6, 1e-6, np.array([[0, second]]))[0] == ok
    # outside the band only the exact answer is valid
    assert oracle.valid_peaks(y, dirs, 0.5, 1e-6, np.array([[0, 3]]))[0]
    assert not oracle.valid_peaks(y, dirs, 0.5, 1e-6, np.array([[0, 1]]))[0]
    assert not oracle.valid_peaks(y, dirs, 0.7, 1e-6, np.array([[0, 3]]))[0]
    assert oracle.valid_peaks(y, dirs, 0.7, 1e-6, np.array([[0, 1]]))[0]


def test_peaks_brute_force_greedy():
    """The greedy reading by brute force on tiny random inputs: every
    ordered choice of n directions is enumerated and the one the rule
    selects (each peak the largest strictly separated power, lowest index on
    ties) compared with the oracle; the oracle's answer also passes the
    validity check and the check rejects every other enumerated choice
    away from the band."""
    rng = np.random.default_rng(23)
    for trial in range(40):
        Q = 7
        dirs = rng.standard_normal((Q, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        y = rng.integers(0, 4, size=(1, Q)).astype(np.float64)
        cs = float(rng.uniform(-0.5, 0.9))
        n = 3
        idx, _, dec = oracle.peaks(y, dirs, n, cs, band=1e-9)
        best = None
        for choice in itertools.permutations(range(Q), n):
            good = True
            for p, q in enumerate(choice):
                free = [r for r in range(Q) if r not in choice[:p]
                        and all(dirs[r] @ dirs[e] < cs for e in choice[:p])]
                if not free or q not in free:
                    good = False
                    break
                m = max(y[0, r] for r in free)
                if y[0, q] != m or q != min(r for r in free if y[0, r] == m):
                    good = False
                    break
            if good:
                best = choice
                break
        if best is None:   # fewer than n peaks exist: compare the leading ones
            k = int(np.sum(idx[0] >= 0))
            assert np.all(idx[0, k:] == -1)
        else:
            assert tuple(idx[0].tolist()) == best
        assert oracle.valid_peaks(y, dirs, cs, 1e-9, idx)[0]
        if dec[0] == n and best is not None:
            for choice in itertools.permutations(range(Q), n):
                if choice != best:
                    assert not oracle.valid_peaks(y, dirs, cs, 1e-9, np.array([choice]))[0]


# ------------------------------------------------ eq. (15), normalised search
def _nn_case(seed=31, M=4, N=16, level=2, delta=1e-3, F=12):
    mics, grid, rng = _small(M=M, N=N, level=level, seed=seed)
    plan = oracle.make_plan(mics, grid, 16000.0, 343.0, N, delta)
    X = rng.standard_normal((F, M, N // 2 + 1)) + 1j * rng.standard_normal((F, M, N // 2 + 1))
    return plan, X


def test_eq15_identity_and_brute_force():
    """For unit rows D^_q and the unit projection Z^, 1 - ||D^_q - Z^^H||^2 / 2
    equals Re(sum_k D^_qk Z^_k) (the product of eq. (14), no conjugate),
    checked with explicit loops over directions and components; the oracle's
    answer is the arg-max of y_q / ||D_q|| from the reduced powers of eqs.
    (12)-(14), a different route to the same number."""
    plan, X = _nn_case()
    K = plan.K
    D = plan.U * plan.s[:K][None, :]
    x = oracle.phat_vector(X)
    r = oracle.normalized_locate(plan, X)
    y = oracle.svd_phat_power(plan.U, plan.s, plan.Vh, x)
    rn = np.linalg.norm(D, axis=1)
    for f in range(X.shape[0]):
        Z = plan.Vh @ x[f]
        zn = math.sqrt(sum(abs(v) ** 2 for v in Z))
        best, bq = -2.0, -1
        for q in range(D.shape[0]):
            dn = [D[q, k] / rn[q] for k in range(K)]
            zh = [Z[k] / zn for k in range(K)]
            dist2 = sum(abs(dn[k] - zh[k].conjugate()) ** 2 for k in range(K))
            dot = sum(dn[k] * zh[k] for k in range(K)).real
            assert abs((1.0 - 0.5 * dist2) - dot) < 1e-12
            if dot > best + 1e-12:
                best, bq = dot, q
        assert plan.rep[bq] == r["doa"][f]
        assert abs(r["score"][f] - best) < 1e-12
        qn = int(np.argmax(y[f] / rn))
        assert plan.rep[qn] == r["doa"][f]
        assert abs(r["yhat"][f] - y[f, qn] / rn[qn]) < 1e-9 * max(1.0, abs(r["yhat"][f]))


def test_eq15_full_rank_equals_srp():
    """At full rank ||D_q||^2 = ||W_q||^2 = L for every direction (unit-modulus
    entries of eq. (4)), so eq. (15) picks the direction of eq. (9)."""
    mics, grid, rng = _small(M=4, N=16, level=0, seed=3)
    plan = oracle.make_plan(mics, grid, 16000.0, 343.0, 16, 1e-13)
    assert plan.K == min(plan.W.shape)
    D = plan.U * plan.s[:plan.K][None, :]
    assert np.allclose(np.sum(np.abs(D) ** 2, axis=1), plan.W.shape[1], rtol=1e-12)
    X = rng.standard_normal((20, 4, 9)) + 1j * rng.standard_normal((20, 4, 9))
    r = oracle.normalized_locate(plan, X)
    s = oracle.srp_locate(plan, X)
    judged = s["margin"] > 1e-9
    assert np.array_equal(r["doa"][judged], s["doa"][judged])
    # and a truncated plan's row norms differ, so eq. (15) is not eq. (14)
    plan2, X2 = _nn_case(delta=1e-1, F=40)
    D2 = plan2.U * plan2.s[:plan2.K][None, :]
    assert np.ptp(np.linalg.norm(D2, axis=1)) > 1e-3


# ------------------------------------------------ binary time-frequency mask
def test_mask_pins():
    """The mask of ones changes nothing; dropping bins equals silencing them
    in X (eq. (3) gives 0 for a silent bin); and for a noiseless plane wave
    with only bins k0..k1 kept, SRP-PHAT is the band-limited Dirichlet sum
    sum_p sum_{k=k0}^{k1} cos(k theta_p) = sum_p (D(k1) - D(k0 - 1)), with
    D(n) = 1/2 + sin((n + 1/2) t) / (2 sin(t / 2))."""
    N, fs, c = 64, 16000.0, 343.0
    mics = synth.geometry("2d")
    grid = synth.icosphere(2)
    plan = oracle.make_plan(mics, grid, fs, c, N, 1e-5)
    rng = np.random.default_rng(33)
    B = N // 2 + 1
    X = synth.plane_wave_fd(mics, synth.random_direction(rng), 6, N, fs, c, rng, snr_db=5.0)
    ones = np.ones((6, B), np.uint8)
    a, b = oracle.locate(plan, X), oracle.locate(plan, X, mask=ones)
    assert np.array_equal(a["y"], b["y"]) and np.array_equal(a["power"], b["power"])
    m = rng.integers(0, 2, size=(6, B)).astype(np.uint8)
    Xz = X * m[:, None, :]
    c1, c2 = oracle.locate(plan, X, mask=m), oracle.locate(plan, Xz)
    assert np.allclose(c1["y"], c2["y"], atol=1e-12) and np.allclose(c1["power"], c2["power"], atol=1e-12)
    # band-limited Dirichlet sum for a noiseless off-grid plane wave
    u = synth.random_direction(rng)
    Xp = synth.plane_wave_fd(mics, u, 1, N, fs, c, rng)
    k0, k1 = 5, 21
    band = np.zeros((1, B), np.uint8)
    band[0, k0:k1 + 1] = 1
    s = oracle.srp_locate(plan, Xp, mask=band)
    tau = plan.tau
    src = oracle.tdoa_farfield(mics, u[None, :], fs, c)[0]
    th = 2 * np.pi * (tau - src[None, :]) / N
    th = np.mod(th + np.pi, 2 * np.pi) - np.pi

    def dsum(n, t):
        small = np.abs(t) < 1e-12
        st = np.where(small, 1.0, t)
        return np.where(small, n + 1.0, 0.5 + np.sin((n + 0.5) * st) / (2 * np.sin(st / 2)))
    want = (dsum(k1, th) - dsum(k0 - 1, th)).sum(axis=1)
    assert np.max(np.abs(s["y"][0] - want)) < 1e-9 * plan.W.shape[1]


def test_eq15_silent_frame_ties():
    """A frame with every bin silent has Z = 0: every direction ties in
    eq. (15) and the lowest index is returned, as for eq. (14)."""
    plan, X = _nn_case(F=3)
    X[1] = 0
    r = oracle.normalized_locate(plan, X)
    assert r["doa"][1] == 0 and r["yhat"][1] == 0.0 and r["margin"][1] == 0.0
    assert oracle.locate(plan, X)["doa"][1] == 0
