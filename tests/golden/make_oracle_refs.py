"""Writes the FP64 oracle's answers for the first frames of the full-size
workloads, and the oracle's powers of every direction for a few sampled
frames.  Calls only the input generators and the oracle.

For each, the same frames are also searched with the normalised form of
eq. (15) (nn_* fields).

Workloads:
  planar_q10242  planar 7-mic array of Table 2, icosphere level 5 (10242
                 directions), N = 512, delta = 1e-5, one source per segment;
  cube_q10242    3-D 7-mic array of Table 2, level 5, two simultaneous sources;
  cube_q40962    3-D array, level 6 (40962 directions), two sources.

Usage: python tests/golden/make_oracle_refs.py [name ...]"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# frames answered in full, and frames whose every power is stored: the first
# frames, 64-frame tile edges, 100-frame segment edges and the last frame
SPEC = {
    "planar_q10242": dict(frames=2000, y_rows=[0, 1, 2, 63, 64, 65, 99, 100, 127, 128, 511, 1023, 1024,
                                               1500, 1998, 1999]),
    "cube_q10242": dict(frames=2000, y_rows=[0, 1, 63, 64, 99, 100, 1000, 1999]),
    "cube_q40962": dict(frames=400, y_rows=[0, 1, 63, 64, 99, 100, 257, 399]),
}


def make(name: str):
    spec = SPEC[name]
    frames, rows = spec["frames"], np.asarray(spec["y_rows"], dtype=np.int64)
    w = synth.workload(name, frames=frames)
    plan = oracle.make_plan(w["mics"], w["grid"], w["fs"], w["c"], w["N"], w["delta"])
    X = w["X"][:frames]
    r = oracle.locate(plan, X)
    s = oracle.srp_locate(plan, X)
    nn = oracle.normalized_locate(plan, X)
    np.savez_compressed(
        os.path.join(HERE, f"{name}_oracle.npz"),
        frames=np.int64(frames), K=np.int64(plan.K), K_paper=np.int64(plan.K_paper),
        residual=np.float64(plan.residual), n_classes=np.int64(len(np.unique(plan.rep))),
        sigma=plan.s[:plan.K + 8], doa=r["doa"].astype(np.int32),
        margin=r["margin"].astype(np.float64), power=r["power"], yhat=r["yhat"],
        srp_doa=s["doa"].astype(np.int32), srp_margin=s["margin"], srp_power=s["power"],
        y_rows=rows, y=r["y"][rows].astype(np.float32), srp_y=s["y"][rows].astype(np.float32),
        nn_doa=nn["doa"].astype(np.int32), nn_margin=nn["margin"], nn_yhat=nn["yhat"], nn_power=nn["power"])
    print(name, "K", plan.K, "residual", plan.residual, flush=True)


def main(names):
    for name in names or list(SPEC):
        make(name)


if __name__ == "__main__":
    main(sys.argv[1:])
