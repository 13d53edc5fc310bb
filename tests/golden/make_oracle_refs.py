"""Writes the FP64 oracle's answers for the first frames of the full-size
planar workload (7-mic planar array of Table 2, icosphere level 5 = 10242
directions, N = 512, delta = 1e-5).  Calls only the input generators and the
oracle.  Usage: python tests/golden/make_oracle_refs.py"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main(frames: int = 2000):
    for name in ("planar_q10242",):
        w = synth.workload(name)
        plan = oracle.make_plan(w["mics"], w["grid"], w["fs"], w["c"], w["N"], w["delta"])
        X = w["X"][:frames]
        r = oracle.locate(plan, X)
        s = oracle.srp_locate(plan, X)
        np.savez_compressed(
            os.path.join(HERE, f"{name}_oracle.npz"),
            frames=np.int64(frames), K=np.int64(plan.K), K_paper=np.int64(plan.K_paper),
            residual=np.float64(plan.residual), n_classes=np.int64(len(np.unique(plan.rep))),
            sigma=plan.s[:plan.K + 8], doa=r["doa"].astype(np.int32),
            margin=r["margin"].astype(np.float64), power=r["power"], yhat=r["yhat"],
            srp_doa=s["doa"].astype(np.int32), srp_margin=s["margin"], srp_power=s["power"])
        print(name, "K", plan.K, "residual", plan.residual)


if __name__ == "__main__":
    main()
