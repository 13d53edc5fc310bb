"""FP64 oracle of the STFT front end.  Test infrastructure only: see the
package docstring.

Section 2 of the paper analyses each microphone signal with a short-time
Fourier transform over frames of N samples with a sine window.  The reading
adopted (the paper gives no formula): frame f of microphone m covers samples
f hop .. f hop + N - 1, w[n] = sin(pi n / N) (periodic), and
X_m[f, k] = sum_{n=0}^{N-1} w[n] x_m[f hop + n] exp(-2 pi i k n / N) for
k = 0 .. N/2.  This module writes that sum out as a product with the
explicit (N/2 + 1) x N DFT matrix; no FFT is used."""
from __future__ import annotations

import numpy as np


def stft_frames(T: int, N: int, hop: int) -> int:
    """Number of whole frames in T samples: 1 + (T - N) // hop, 0 if T < N."""
    return 0 if T < N else 1 + (T - N) // hop


def sine_window(N: int) -> np.ndarray:
    """w[n] = sin(pi n / N), n = 0 .. N-1."""
    return np.sin(np.pi * np.arange(N) / N)


def dft_matrix(N: int) -> np.ndarray:
    """D[k, n] = exp(-2 pi i k n / N) for k = 0 .. N/2, n = 0 .. N-1 (the
    exponent's k n is reduced mod N in integers first, so every entry is a
    root of unity to full FP64 accuracy)."""
    k = np.arange(N // 2 + 1)[:, None]
    n = np.arange(N)[None, :]
    return np.exp(-2j * np.pi * ((k * n) % N) / N)


def stft(pcm: np.ndarray, N: int, hop: int) -> np.ndarray:
    """pcm [M, T] (real) -> X [F, M, N/2+1] complex128, by the definition
    above: window each frame, then multiply by the DFT matrix."""
    pcm = np.asarray(pcm, dtype=np.float64)
    M, T = pcm.shape
    F = stft_frames(T, N, hop)
    D = dft_matrix(N)
    w = sine_window(N)
    X = np.zeros((F, M, N // 2 + 1), dtype=np.complex128)
    for f in range(F):
        seg = pcm[:, f * hop:f * hop + N] * w[None, :]   # M x N
        X[f] = seg @ D.T
    return X
