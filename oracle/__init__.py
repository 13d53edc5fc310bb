"""FP64 CPU oracle for SVD-PHAT (Grondin & Glass, arXiv 1811.11785).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct statement of what the GPU library computes, used to check it.  Only
the tests, the smoke check and the benchmark's CPU-baseline leg may import
it; the library never does, and this package imports nothing from the
library.  It is written from the paper's equations with numpy complex128 and
LAPACK (scipy) and shares no code with the GPU path.

Section references are to the paper: Section 2 (SRP-PHAT, eqs. 1-6),
Section 3 (SVD-PHAT, eqs. 7-15 and Algorithm 1), Section 4 (Results,
Tables 1-2, eqs. 16-20).

Readings of the text that the paper leaves open (each one pinned by a test):

* Eq. (14) writes Re{D_q . Z^H}; it is read as the plain (unconjugated)
  product Re(sum_k D_qk Z_k), the only reading under which it equals row q of
  eq. (9) at full rank.
* Eq. (11) chooses the smallest K with sum_{k<=K} s_k^2 >= (1-delta) ||W||_F^2
  (inclusive).  Where the cut falls inside a cluster of (numerically) equal
  singular values the truncated factorisation is not unique; K is then
  extended over the whole cluster (s_{K+1} >= (1-1e-9) s_K).  The upper bound
  K_max is min(Q, P(N/2+1)) (the rank bound).
* Division by zero in eq. (3) (a silent bin) gives X_ij[k] = 0.
* Directions with identical delay rows give identical rows of W and so
  identical powers: they form one class, reported by its lowest index.
"""
from .svdphat import (  # noqa: F401
    mic_pairs, tdoa_farfield, steering_matrix, phat_vector, srp_phat_power,
    truncated_svd, choose_rank, svd_phat_power, direction_classes,
    argmax_with_margin, exact_power, OraclePlan, make_plan, locate,
    srp_locate, dirichlet_power, stacked_projection, normalized_locate, apply_mask,
)
from .stft import stft, stft_frames, sine_window, dft_matrix  # noqa: F401
from .rmse import doa_map, rmse_alpha  # noqa: F401
from .peaks import peaks, valid_peaks  # noqa: F401
from .mlp import (  # noqa: F401
    gelu, gelu_grad, mlp_forward, mlp_backward, softmax_xent, adam_step,
    coarse_cells, proposal_features,
)
