"""FP64 oracle of SRP-PHAT and SVD-PHAT.  Test infrastructure only: see the
package docstring.  Every function follows the passage cited in its
docstring; there is no blocking, fusion or reordering beyond the paper's own
definitions."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla


# ---------------------------------------------------------------- Section 2
def mic_pairs(M: int) -> list[tuple[int, int]]:
    """All P = M(M-1)/2 pairs (i, j), i < j, in the order of the double sum
    of eq. (5) and of the vector of eq. (7): (0,1), (0,2), ..., (M-2, M-1)."""
    return [(i, j) for i in range(M) for j in range(i + 1, M)]


def tdoa_farfield(mics: np.ndarray, grid: np.ndarray, fs: float, c: float) -> np.ndarray:
    """Far-field TDOA in samples, eq. (2):
    tau[q, p] = fs/c * (r_j - r_i) . s_q / ||s_q||   for pair p = (i, j)."""
    s = grid / np.linalg.norm(grid, axis=1, keepdims=True)
    pairs = mic_pairs(mics.shape[0])
    tau = np.empty((grid.shape[0], len(pairs)))
    for p, (i, j) in enumerate(pairs):
        tau[:, p] = fs / c * (s @ (mics[j] - mics[i]))
    return tau


def steering_matrix(tau: np.ndarray, N: int) -> np.ndarray:
    """W of eq. (8), entries of eq. (4): W[q, p*(N/2+1) + k] =
    exp(2 pi i k tau[q, p] / N), columns ordered pair-major, bin-minor."""
    k = np.arange(N // 2 + 1)
    Q, P = tau.shape
    W = np.exp(2j * np.pi * tau[:, :, None] * k[None, None, :] / N)
    return W.reshape(Q, P * k.size)


def phat_vector(X: np.ndarray) -> np.ndarray:
    """PHAT-weighted cross-spectra, eqs. (3) and (7).

    X: [F, M, N/2+1] STFT frames.  Returns x: [F, P*(N/2+1)] complex128 with
    x[f, p*(N/2+1) + k] = X_i[k] X_j[k]^* / (|X_i[k]| |X_j[k]|), and 0 where
    the denominator is 0."""
    X = np.asarray(X, dtype=np.complex128)
    F, M, B = X.shape
    pairs = mic_pairs(M)
    x = np.zeros((F, len(pairs), B), dtype=np.complex128)
    for p, (i, j) in enumerate(pairs):
        num = X[:, i, :] * np.conj(X[:, j, :])
        den = np.abs(X[:, i, :]) * np.abs(X[:, j, :])
        nz = den > 0
        x[:, p, :][nz] = num[nz] / den[nz]
    return x.reshape(F, len(pairs) * B)


def apply_mask(x: np.ndarray, mask, B: int) -> np.ndarray:
    """Binary time-frequency mask (Section 5 names masks as future work):
    x [F, P*B] of eq. (7) with every pair's value at bin k of frame f set to
    0 where mask[f, k] == 0.  mask None leaves x unchanged."""
    if mask is None:
        return x
    F = x.shape[0]
    m = (np.asarray(mask)[:F] != 0).astype(x.real.dtype)
    return (x.reshape(F, -1, B) * m[:, None, :]).reshape(F, -1)


def srp_phat_power(W: np.ndarray, x: np.ndarray) -> np.ndarray:
    """SRP-PHAT powers, eq. (9): Y = Re{W X}, for a batch x [F, L] -> [F, Q]."""
    return np.real(x @ W.T)


def dirichlet_power(tau: np.ndarray, tau_src: np.ndarray, N: int) -> np.ndarray:
    """Closed form of eq. (5) for a noiseless plane wave whose pair delays are
    tau_src[p]: the PHAT spectrum is exp(-2 pi i k tau_src[p] / N), so
    Y_q = sum_p sum_{k=0}^{N/2} cos(k theta_p), theta_p = 2 pi (tau[q,p] -
    tau_src[p]) / N, and sum_{k=0}^{n} cos(k t) = 1/2 + sin((n+1/2) t) /
    (2 sin(t/2)) (Dirichlet kernel), equal to n+1 at t = 0 (mod 2 pi)."""
    n = N // 2
    th = 2.0 * np.pi * (tau - tau_src[None, :]) / N
    th = np.mod(th + np.pi, 2.0 * np.pi) - np.pi
    small = np.abs(th) < 1e-12
    safe = np.where(small, 1.0, th)
    val = 0.5 + np.sin((n + 0.5) * safe) / (2.0 * np.sin(safe / 2.0))
    val = np.where(small, n + 1.0, val)
    return val.sum(axis=1)


# ---------------------------------------------------------------- Section 3
def choose_rank(sigma: np.ndarray, delta: float, energy: float | None = None,
                cluster_rtol: float = 1e-9) -> tuple[int, int]:
    """Rank rule of eq. (11): K_paper is the smallest K >= 1 with
    sum_{k<=K} s_k^2 >= (1 - delta) * ||W||_F^2, for the small positive delta
    Section 3 defines (delta <= 0 raises ValueError).  K_used extends K_paper
    over a cluster of equal singular values at the cut.  Returns
    (K_paper, K_used)."""
    if not delta > 0.0:
        raise ValueError("eq. (11) takes a positive delta")
    s2 = sigma.astype(np.float64) ** 2
    E = s2.sum() if energy is None else energy
    cum = np.cumsum(s2)
    Kp = int(np.searchsorted(cum, (1.0 - delta) * E, side="left") + 1)
    Kp = min(max(Kp, 1), sigma.size)
    K = Kp
    while K < sigma.size and sigma[K] >= (1.0 - cluster_rtol) * sigma[K - 1]:
        K += 1
    return Kp, K


def truncated_svd(W: np.ndarray, delta: float):
    """Eqs. (10)-(11): W ~ U S V^H with the rank chosen by eq. (11).
    Uses LAPACK's divide-and-conquer SVD of W itself.  Returns
    (U_K [Q,K], s [min(Q,L)] all singular values, Vh_K [K, L], K_paper, K)."""
    U, s, Vh = sla.svd(W, full_matrices=False, lapack_driver="gesdd")
    Kp, K = choose_rank(s, delta, energy=float(np.sum(np.abs(W) ** 2)))
    return U[:, :K], s, Vh[:K, :], Kp, K


def svd_phat_power(U: np.ndarray, s: np.ndarray, Vh: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Reduced powers of eqs. (12)-(14): Z = V^H X, D = U S and
    Y_q = Re(sum_k D_qk Z_k).  x: [F, L] -> [F, Q]."""
    K = U.shape[1]
    D = U * s[:K][None, :]
    Z = x @ Vh.T                     # [F, K] = (V^H X)^T per frame
    return np.real(Z @ D.T)


def stacked_projection(U: np.ndarray, s: np.ndarray, Vh: np.ndarray):
    """Real stacked forms of the two products (with S folded into V^H):
    A = S V^H, z = A x gives [Re z; Im z] = [[Re A, -Im A], [Im A, Re A]]
    [Re x; Im x], and y = [Re U, -Im U] [Re z; Im z]."""
    K = U.shape[1]
    A = s[:K, None] * Vh
    Ast = np.block([[A.real, -A.imag], [A.imag, A.real]])
    Ust = np.concatenate([U.real, -U.imag], axis=1)
    return Ast, Ust


def direction_classes(tau: np.ndarray, tol: float = 1e-9) -> np.ndarray:
    """rep[q] = lowest index q' whose delay row equals row q within ``tol``
    samples in every pair (identical rows of W, hence identical powers).
    Brute force over all pairs of directions, in blocks."""
    Q = tau.shape[0]
    rep = np.arange(Q)
    blk = max(1, int(2e7 // max(1, Q * tau.shape[1])))
    for a in range(0, Q, blk):
        d = np.abs(tau[a:a + blk, None, :] - tau[None, :, :]).max(axis=2)  # b x Q
        for r in range(d.shape[0]):
            rep[a + r] = int(np.flatnonzero(d[r] <= tol)[0])
    return rep


def argmax_with_margin(y: np.ndarray, rep: np.ndarray):
    """Eq. (6)/(14) over classes.  For each frame: q* = argmax_q y_q (lowest
    index on exact ties), qbar = rep[q*]; margin = (y_(1) - y_(2)) / |y_(1)|
    where y_(2) is the largest y over directions of any other class."""
    y = np.atleast_2d(y)
    qstar = np.argmax(y, axis=1)
    qbar = rep[qstar]
    y1 = y[np.arange(y.shape[0]), qstar]
    other = rep[None, :] != qbar[:, None]
    y2 = np.where(other, y, -np.inf).max(axis=1)
    margin = (y1 - y2) / np.maximum(np.abs(y1), 1e-300)
    return qbar, y1, margin


def exact_power(tau_row: np.ndarray, N: int, x: np.ndarray) -> float:
    """Algorithm 1, online step 4: Y_qbar from row qbar of W, i.e.
    Re sum_{p,k} exp(2 pi i k tau[qbar, p] / N) x[p*(N/2+1)+k]."""
    w = steering_matrix(tau_row[None, :], N)[0]
    return float(np.real(w @ x))


# ------------------------------------------------------------ plan / locate
@dataclass
class OraclePlan:
    mics: np.ndarray
    grid: np.ndarray
    fs: float
    c: float
    N: int
    delta: float
    tau: np.ndarray
    W: np.ndarray
    U: np.ndarray
    s: np.ndarray
    Vh: np.ndarray
    K_paper: int
    K: int
    rep: np.ndarray

    @property
    def residual(self) -> float:
        """sum_{k>K} s_k^2 / ||W||_F^2 (the part eq. (11) lets go)."""
        E = float(np.sum(np.abs(self.W) ** 2))
        return float(np.sum(self.s[self.K:] ** 2) / E)


def make_plan(mics, grid, fs, c, N, delta, keep_all=False) -> OraclePlan:
    """Algorithm 1, offline steps 1-2 (steps 3-4, the normalised vectors and
    the k-d tree, are not part of the brute-force search of eq. (14))."""
    tau = tdoa_farfield(np.asarray(mics, float), np.asarray(grid, float), fs, c)
    W = steering_matrix(tau, N)
    U, s, Vh, Kp, K = truncated_svd(W, delta)
    rep = direction_classes(tau)
    return OraclePlan(np.asarray(mics, float), np.asarray(grid, float), fs, c, N,
                      delta, tau, W, U, s, Vh, Kp, K, rep)


def locate(plan: OraclePlan, X: np.ndarray, chunk: int = 256, mask=None):
    """Algorithm 1, online steps 1-4 with the brute-force search of eq. (14),
    on x masked by ``mask`` [F, N/2+1] (apply_mask) if given.
    Returns dict(doa, power, yhat, margin, y)."""
    out = {k: [] for k in ("doa", "power", "yhat", "margin", "y")}
    B = plan.N // 2 + 1
    for a in range(0, X.shape[0], chunk):
        x = apply_mask(phat_vector(X[a:a + chunk]), None if mask is None else mask[a:a + chunk], B)
        y = svd_phat_power(plan.U, plan.s, plan.Vh, x)
        qbar, y1, m = argmax_with_margin(y, plan.rep)
        out["doa"].append(qbar)
        out["yhat"].append(y1)
        out["margin"].append(m)
        out["power"].append(np.array([exact_power(plan.tau[q], plan.N, xv)
                                      for q, xv in zip(qbar, x)]))
        out["y"].append(y)
    return {k: np.concatenate(v) for k, v in out.items()}


def srp_locate(plan: OraclePlan, X: np.ndarray, chunk: int = 64, W: np.ndarray | None = None, mask=None):
    """Plain SRP-PHAT, eqs. (3), (9) and (6), on x masked by ``mask`` if
    given.  Returns dict(doa, power, margin, y)."""
    W = plan.W if W is None else W
    out = {k: [] for k in ("doa", "power", "margin", "y")}
    B = plan.N // 2 + 1
    for a in range(0, X.shape[0], chunk):
        x = apply_mask(phat_vector(X[a:a + chunk]), None if mask is None else mask[a:a + chunk], B)
        y = srp_phat_power(W, x)
        qbar, y1, m = argmax_with_margin(y, plan.rep)
        out["doa"].append(qbar)
        out["power"].append(y1)
        out["margin"].append(m)
        out["y"].append(y)
    return {k: np.concatenate(v) for k, v in out.items()}


def normalized_locate(plan: OraclePlan, X: np.ndarray, chunk: int = 256, mask=None):
    """The search of eq. (15), Section 3: with D = U S (eq. (13)), unit rows
    D^_q = D_q / ||D_q|| and the unit projection Z^ = Z / ||Z|| (Z = V^H X,
    eq. (12)), q_bar minimises ||D^_q - Z^^H||^2 over the directions (lowest
    index on exact ties, then the class representative), which equals
    maximising 1 - ||D^_q - Z^^H||^2 / 2 = Re(D^_q . Z^).  For Z = 0 (a
    silent frame) Z^ is undefined and every direction ties.  Returns
    dict(doa, score, margin, yhat, power): score the normalised value at
    q_bar, margin (s1 - s2) / |s1| to the best other class, yhat =
    ||Z|| score = Re(D_q Z) / ||D_q|| at q_bar, power the row power of
    Algorithm 1 online step 4."""
    K = plan.K
    D = plan.U * plan.s[:K][None, :]
    Dn = D / np.linalg.norm(D, axis=1, keepdims=True)
    out = {k: [] for k in ("doa", "score", "margin", "yhat", "power")}
    B = plan.N // 2 + 1
    for a in range(0, X.shape[0], chunk):
        x = apply_mask(phat_vector(X[a:a + chunk]), None if mask is None else mask[a:a + chunk], B)
        Z = x @ plan.Vh.T                              # [F, K] = (V^H X)^T
        zn = np.linalg.norm(Z, axis=1)
        Zh = Z / np.where(zn > 0, zn, 1.0)[:, None]
        # squared distance between D^_q and the conjugate of Z^ (the row Z^^H)
        d2 = np.stack([np.sum(np.abs(Dn - np.conj(z)[None, :]) ** 2, axis=1) for z in Zh])
        score = 1.0 - 0.5 * d2
        # Z = 0 (a silent or fully masked frame): Z^ is undefined and every
        # direction is equally near; they tie exactly (lowest index wins)
        score[zn == 0] = 0.5
        qbar, s1, m = argmax_with_margin(score, plan.rep)
        out["doa"].append(qbar)
        out["score"].append(s1)
        out["margin"].append(m)
        out["yhat"].append(zn * s1)
        out["power"].append(np.array([exact_power(plan.tau[q], plan.N, xv) for q, xv in zip(qbar, x)]))
    return {k: np.concatenate(v) for k, v in out.items()}
