"""Benchmark: frames/s of SVD-PHAT on one MI355X on the planar 7-mic array
(Table 2) with Q = 10242 directions (icosphere level 5), N = 512, hop 256,
delta = 1e-5, 20000 seeded synthetic frames (plane-wave white-noise source,
random direction and SNR U[0, 20] dB per 100-frame segment).

One step = one call of the whole hot path over the 20000-frame batch already
resident in HBM: PHAT, Z = S V^H X, Y = Re(U Z), argmax with FP32 rescoring
(and hi/lo recomputation where the margin is small), power of the chosen
direction.  The headline form is FP16 MFMA with FP32 accumulation; plain
FP32 SRP-PHAT (eq. (9)) on the same batch is timed beside it.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes of one launch of the streamed FP16 GEMM1 over the 20000-frame
# planar workload: rocprofv3 FETCH_SIZE and WRITE_SIZE of that launch, each
# scaled by what the counter reads for a plain 256 MiB device copy in the same
# process (factors 2.0 and 1.0).  They hold only for the kernel sources they
# were measured on, identified by the SHA-256 of those files.
GEMM1_TRAFFIC = {
    "sources": ["paper_1811_11785_amd/csrc/gemm1.hip", "paper_1811_11785_amd/csrc/device.h"],
    "sha256": "aab0897f026f1d583b0149b6e99bc50e7d9e5711b44ca5bbb1730d3eff9d1d44 "
              "c09dbf5ca8c0a66b1e97d4c9b3af4a0cb1a154cdb1de4a0a12789e61b229d75a",
    "frames": 20000,
    "bytes": 416.0e6 + 13.8e6,
}


def _gemm1_traffic(frames):
    """Counter-measured HBM bytes per GEMM1 launch, or None once the kernel
    sources differ from the measured ones or the batch differs."""
    import hashlib
    if frames != GEMM1_TRAFFIC["frames"]:
        return None
    try:
        h = " ".join(hashlib.sha256(open(os.path.join(ROOT, f), "rb").read()).hexdigest()
                     for f in GEMM1_TRAFFIC["sources"])
    except OSError:
        return None
    return GEMM1_TRAFFIC["bytes"] if h == GEMM1_TRAFFIC["sha256"] else None
MFMA_FP16_PEAK_TFLOPS = 2500.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timed(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, budget_s: float):
    """The FP64 oracle timed on the host's cores on a bounded sample of the
    same frames (its offline SVD is built first and timed separately): with
    every core the BLAS uses, then on one core, and the plain SRP-PHAT oracle
    on a few frames.  Returns (baseline dict, plan seconds, doa, margin) with
    the oracle's answers for the frames it covered."""
    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    t0 = time.perf_counter()
    log("oracle plan (FP64 SVD of W) ...")
    plan = oracle.make_plan(w["mics"], w["grid"], w["fs"], w["c"], w["N"], w["delta"])
    plan_s = time.perf_counter() - t0
    log(f"oracle plan {plan_s:.1f} s; timing oracle.locate for up to {budget_s:.0f} s")
    X = w["X"]
    done, chunk = 0, 256
    t0 = time.perf_counter()
    doas, margins = [], []
    while time.perf_counter() - t0 < budget_s and done < X.shape[0]:
        r = oracle.locate(plan, X[done:done + chunk])
        doas.append(r["doa"])
        margins.append(r["margin"])
        done += r["doa"].shape[0]
    dt = time.perf_counter() - t0
    n1 = 256
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        oracle.locate(plan, X[:n1])
        one_core = n1 / (time.perf_counter() - t1)
    ns = 64
    t1 = time.perf_counter()
    oracle.srp_locate(plan, X[:ns])
    srp_fps = ns / (time.perf_counter() - t1)
    base = dict(value=done / dt, unit="frames/s", cores=int(cores), kind="oracle",
                sample=f"first {done} of the {X.shape[0]} frames, FP64 numpy/LAPACK oracle.locate "
                       f"(PHAT, Z = S V^H X, Y = Re(U Z), argmax, row power); offline SVD "
                       f"{plan_s:.1f} s excluded",
                one_core_fps=one_core, one_core_sample=f"first {n1} frames, BLAS limited to 1 thread",
                srp_oracle_fps=srp_fps, srp_oracle_sample=f"first {ns} frames, oracle.srp_locate (eq. (9)), "
                                                          f"{cores} threads",
                cpu_model=_cpu_model(), os_cpu_count=os.cpu_count())
    return base, plan_s, np.concatenate(doas), np.concatenate(margins)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames", type=int, default=20000)
    ap.add_argument("--srp-steps", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--workload", default="planar_q10242",
                    help="planar_q10242 (default, the headline line), cube_q10242, cube_q40962, ragged256 "
                         "or proposal_q40962")
    ap.add_argument("--batches", default="1,256,4096", help="batch sizes of the cube workloads")
    ap.add_argument("--train-frames", type=int, default=2_000_000, help="training pairs of the proposal")
    ap.add_argument("--train-epochs", type=int, default=20, help="passes over the proposal's training pairs")
    ap.add_argument("--arrays", type=int, default=256, help="arrays of the ragged workload")
    ap.add_argument("--single-frames", type=int, default=2048,
                    help="single-frame calls timed at batch 1 (3-D workloads)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one plain device copy of this many MB (a known-size reference "
                         "for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the frames of a batch are "
              f"independent, so N GPUs would each run this benchmark on their own frames.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1811_11785_amd as amd
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    amd.lib()
    if args.workload == "ragged256":
        return bench_ragged(args, torch, amd, synth)
    # a plain device copy of known size, to scale the traffic counters
    if args.calib_copy_mb:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "proposal_q40962":
        return bench_proposal(args, torch, amd, synth)
    if args.workload in ("cube_q10242", "cube_q40962"):
        return bench_cube(args, torch, amd, synth)
    w = synth.workload("planar_q10242", frames=args.frames)
    F = w["X"].shape[0]
    t0 = time.perf_counter()
    plan = amd.Plan(w["mics"], w["grid"], w["fs"], w["c"], w["N"], w["delta"], keep_w=True)
    plan_s = time.perf_counter() - t0
    info = plan.info
    log(f"plan built in {plan_s:.1f} s: K={info['K']} classes={info['n_classes']}")
    X = torch.from_numpy(w["X"]).cuda()
    dev = X.device
    doa = torch.empty(F, dtype=torch.int32, device=dev)
    power = torch.empty(F, dtype=torch.float32, device=dev)
    yhat = torch.empty(F, dtype=torch.float32, device=dev)
    margin = torch.empty(F, dtype=torch.float32, device=dev)
    h = plan.handle

    def svd_step(prec, mode):
        return lambda: amd.svdphat_locate(h, X, prec, mode, doa, power, yhat, margin)

    forms = {
        "fp16": (amd.FP16, amd.RESCORE | amd.HILO),
        "bf16": (amd.BF16, amd.RESCORE | amd.HILO),
        "fp32": (amd.FP32, amd.RESCORE),
    }
    results = {}
    for name, (prec, mode) in forms.items():
        step = svd_step(prec, mode)
        nw = args.warmup if name == "fp16" else 2
        ns = args.steps if name == "fp16" else max(3, args.steps // 5)
        _timed(step, nw, torch)
        dt = _timed(step, ns, torch)
        results[name] = dict(fps=F * ns / dt, ms_per_step=1e3 * dt / ns, steps=ns)
        d = doa.cpu().numpy()
        results[name]["doa"] = d
        log(f"{name}: {results[name]['fps']:.4g} frames/s ({results[name]['ms_per_step']:.3f} ms/step)")
    # the normalised search of eq. (15), and a binary time-frequency mask
    # (each bin of each frame kept with probability 0.7), both in the FP16
    # form with rescoring and hi/lo
    prec, mode = forms["fp16"]
    extra = {}
    g = torch.Generator(device=dev)
    g.manual_seed(11785)
    tfmask = (torch.rand((F, info["B"]), generator=g, device=dev) < 0.7).to(torch.uint8)
    masked = lambda: amd._check(amd.lib().svdphat_locate_masked(
        h, amd._ptr(X), F, amd._ptr(tfmask), prec, mode, amd._ptr(doa), amd._ptr(power), amd._ptr(yhat),
        amd._ptr(margin), None, amd._stream(None)))
    for name, step in (("fp16_eq15", svd_step(prec, mode | amd.NORMALIZED)), ("fp16_masked", masked)):
        ns = max(3, args.steps // 5)
        _timed(step, 2, torch)
        dt = _timed(step, ns, torch)
        extra[name] = dict(fps=F * ns / dt, ms_per_step=1e3 * dt / ns)
        if name == "fp16_eq15":
            extra[name]["same_direction_as_eq14"] = float(np.mean(doa.cpu().numpy() == results["fp16"]["doa"]))
        log(f"{name}: {extra[name]['fps']:.4g} frames/s ({extra[name]['ms_per_step']:.3f} ms/step)")
    del tfmask
    # plain FP32 SRP-PHAT on the same batch
    srp = lambda: amd.svdphat_srp_locate(h, X, doa, power)
    _timed(srp, 1, torch)
    dt = _timed(srp, args.srp_steps, torch)
    srp_fps = F * args.srp_steps / dt
    srp_doa = doa.cpu().numpy()
    log(f"plain fp32 srp: {srp_fps:.4g} frames/s")

    # STFT front end on the same number of frames of microphone samples
    # (HIP events on the launch stream, which is torch's current stream), and
    # the whole path from samples: STFT, then the FP16 search
    pcm = torch.from_numpy(synth.workload_pcm("planar_q10242", F)).cuda()
    Tm = pcm.shape[1]
    Xs = torch.empty((F, info["M"], info["B"]), dtype=torch.complex64, device=dev)
    st = lambda: amd.svdphat_stft(pcm, info["N"], info["N"] // 2, Xs)
    _timed(st, 2, torch)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        st()
    e1.record()
    torch.cuda.synchronize()
    stft_us = 1e3 * e0.elapsed_time(e1) / args.steps
    prec16, mode16 = forms["fp16"]
    e2e = lambda: (st(), amd.svdphat_locate(h, Xs, prec16, mode16, doa, power, yhat, margin))
    _timed(e2e, 2, torch)
    dt = _timed(e2e, args.steps, torch)
    stft_bytes = info["M"] * Tm * 4 + F * info["M"] * info["B"] * 8
    stft = dict(kernel="k_stft", us_per_launch=stft_us, frames_per_s=F / (stft_us * 1e-6),
                algorithmic_bytes=stft_bytes, achieved_GBps=stft_bytes / (stft_us * 1e-6) / 1e9,
                peak_GBps=HBM_PEAK_GBS, frac=stft_bytes / (stft_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                end_to_end_fps=F * args.steps / dt, end_to_end_ms_per_step=1e3 * dt / args.steps,
                samples_per_mic=Tm)
    log(f"stft: {stft_us:.1f} us per {F} frames; samples -> directions {stft['end_to_end_fps']:.4g} frames/s")
    del pcm, Xs

    # per-kernel durations with HIP events on the launch stream (same work)
    amd.svdphat_timing_reset()
    amd.svdphat_timing_enable(True)
    prec, mode = forms["fp16"]
    for _ in range(args.steps):
        amd.svdphat_locate(h, X, prec, mode, doa, power, yhat, margin)
    amd.svdphat_timing_enable(False)
    kt = amd.svdphat_timing_read()
    amd.svdphat_timing_reset()
    # event counts in a pass of their own (their atomics would skew the timing)
    amd.svdphat_timing_enable(False, counts=True)
    amd.svdphat_locate(h, X, prec, mode, doa, power, yhat, margin)
    amd.svdphat_timing_enable(False)
    kc = amd.svdphat_timing_read()
    amd.svdphat_timing_reset()
    amd.svdphat_timing_enable(True)
    for _ in range(args.srp_steps):
        amd.svdphat_srp_locate(h, X, doa, power)
    amd.svdphat_timing_enable(False)
    kt_srp = amd.svdphat_timing_read()
    torch.cuda.synchronize()
    counts = {k[6:]: v[0] / max(v[1], 1) for k, v in kc.items() if k.startswith("count:")}
    kernels = {k: dict(avg_us=1e3 * v[0] / v[1], launches=v[1]) for k, v in kt.items()}
    kernels_srp = {k: dict(avg_us=1e3 * v[0] / v[1], launches=v[1]) for k, v in kt_srp.items()}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])

    # roofline of the dominant kernel: algorithmic bytes / flops per launch
    M, B, K2, ncls = info["M"], info["B"], 2 * info["K"], info["n_classes"]
    L = info["L"]
    x_bytes = F * M * B * 8
    a_bytes = K2 * 2 * L * 2
    if dom == "gemm1":
        algo = x_bytes + a_bytes + F * K2 * 4
        dur = kernels[dom]["avg_us"] * 1e-6
        roof = dict(bound="hbm", achieved=algo / dur / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                    traffic=_gemm1_traffic(F), algorithmic_bytes=algo)
    elif dom == "gemm2":
        flops = 2.0 * ncls * K2 * F
        dur = kernels[dom]["avg_us"] * 1e-6
        roof = dict(bound="mfma", achieved=flops / dur / 1e12, peak=MFMA_FP16_PEAK_TFLOPS, unit="TFLOP/s",
                    traffic=None)
    else:
        algo = x_bytes
        dur = kernels[dom]["avg_us"] * 1e-6
        roof = dict(bound="hbm", achieved=algo / dur / 1e9, peak=HBM_PEAK_GBS, unit="GB/s", traffic=None)
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = dom
    # both GEMMs against the dense FP16 MFMA peak (algorithmic flops:
    # 2 x 2K x 2L per frame for GEMM1, 2 x classes x 2K for GEMM2)
    mfma_fracs = {}
    for k, fl in (("gemm1", 2.0 * K2 * 2 * L * F), ("gemm2", 2.0 * ncls * K2 * F)):
        if k in kernels:
            tf = fl / (kernels[k]["avg_us"] * 1e-6) / 1e12
            mfma_fracs[k] = dict(tflops=tf, peak=MFMA_FP16_PEAK_TFLOPS, frac=tf / MFMA_FP16_PEAK_TFLOPS)

    # reduced powers of every direction for the stored oracle rows, per form
    # (the whole batch in one call, y_opt out)
    gold = dict(np.load(os.path.join(ROOT, "tests", "golden", "planar_q10242_oracle.npz")))
    rows = torch.from_numpy(gold["y_rows"]).to(dev)
    yref = gold["y"].astype(np.float64)
    yerr = {}
    yopt = torch.empty((F, info["Q"]), dtype=torch.float32, device=dev)
    for name, (prec, mode) in forms.items():
        amd.svdphat_locate(h, X, prec, mode, doa, power, yhat, margin, yopt)
        yv = yopt.index_select(0, rows).cpu().numpy().astype(np.float64)
        e = np.max(np.abs(yv - yref), axis=1) / np.max(np.abs(yref), axis=1)
        yerr[name] = dict(max=float(e.max()), mean=float(e.mean()), frames=int(len(e)))
    del yopt
    torch.cuda.synchronize()

    # accuracy against the stored FP64 oracle answers (first frames)
    n = min(int(gold["frames"]), F)
    judged = gold["margin"][:n] > 1e-5
    acc = {}
    for name in forms:
        d = results[name]["doa"][:n]
        acc[name] = dict(match_all=float(np.mean(d == gold["doa"][:n])),
                         match_judged=float(np.mean(d[judged] == gold["doa"][:n][judged])),
                         match_vs_fp64_srp=float(np.mean(d == gold["srp_doa"][:n])))
    acc["srp_fp32"] = dict(match_vs_fp64_srp=float(np.mean(srp_doa[:n] == gold["srp_doa"][:n])),
                           match_vs_fp64_svd=float(np.mean(srp_doa[:n] == gold["doa"][:n])))

    cpu = None
    if not args.no_cpu:
        cpu, oracle_plan_s, odoa, omargin = cpu_baseline(w, args.cpu_budget)
        # every frame the oracle covered (all of them within the budget)
        m = len(odoa)
        jm = omargin > 1e-5
        for name in forms:
            d = results[name]["doa"][:m]
            acc[name]["oracle_frames"] = m
            acc[name]["match_all_frames"] = float(np.mean(d == odoa))
            acc[name]["match_judged_all_frames"] = float(np.mean(d[jm] == odoa[jm]))
            acc[name]["judged_share"] = float(np.mean(jm))

    head = results["fp16"]
    out = {
        "metric": "frames/s at Q=10242, 7 mics: mixed SVD-PHAT vs plain FP32; argmax match %",
        "value": head["fps"],
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16",
        "data": "synthetic",
        "config": {"workload": "planar_q10242", "array": "planar 7-mic (Table 2)", "Q": info["Q"],
                   "K": info["K"], "n_classes": ncls, "N": info["N"], "frames_per_step": F,
                   "delta": w["delta"], "form": "FP16 MFMA, FP32 accumulate, FP32 rescoring, hi/lo fallback"},
        "roofline": roof,
        "mfma_fracs": mfma_fracs,
        "cpu_baseline": cpu,
        "plain_fp32_srp_fps": srp_fps,
        "speedup_vs_plain_fp32": head["fps"] / srp_fps,
        "forms_fps": {k: v["fps"] for k, v in results.items()},
        "eq15_and_mask": extra,
        "argmax_match": acc,
        "y_error": yerr,
        "kernels_us": kernels,
        "kernels_srp_us": kernels_srp,
        "per_frame_counts": counts,
        "stft_front_end": stft,
        "plan_build_s": plan_s,
    }
    if cpu is not None:
        out["oracle_plan_s"] = oracle_plan_s
    print(json.dumps(out))


def bench_cube(args, torch, amd, synth):
    """The 3-D 7-microphone array of Table 2 (two simultaneous white-noise
    sources per 100-frame segment) at Q = 10242 or 40962, BF16 with FP32
    rescoring, at several batch sizes.  Batch 1 is the streaming use: one
    svdphat_locate call per frame, timed as a host loop of calls and as the
    same calls captured once into a HIP graph and replayed (the launch
    overhead of the host loop removed).  Accuracy against the stored FP64
    oracle answers of the first frames."""
    name = args.workload
    frames = 40960
    w = synth.workload(name, frames=frames)
    t0 = time.perf_counter()
    plan = amd.Plan(w["mics"], w["grid"], w["fs"], w["c"], w["N"], w["delta"])
    plan_s = time.perf_counter() - t0
    info = plan.info
    log(f"{name}: plan {plan_s:.1f} s, K={info['K']}, classes={info['n_classes']}")
    X = torch.from_numpy(w["X"]).cuda()
    F = X.shape[0]
    dev = X.device
    doa = torch.empty(F, dtype=torch.int32, device=dev)
    power = torch.empty(F, dtype=torch.float32, device=dev)
    yhat = torch.empty(F, dtype=torch.float32, device=dev)
    margin = torch.empty(F, dtype=torch.float32, device=dev)
    h = plan.handle
    prec, mode = amd.BF16, amd.RESCORE
    gold = dict(np.load(os.path.join(ROOT, "tests", "golden", f"{name}_oracle.npz")))
    ng = int(gold["frames"])
    K2, L, ncls = 2 * info["K"], info["L"], info["n_classes"]
    out = {"metric": f"frames/s, 3-D array, Q={info['Q']}, BF16 + FP32 rescoring", "unit": "frames/s",
           "n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic",
           "config": {"workload": name, "array": "3-D 7-mic (Table 2)", "Q": info["Q"], "K": info["K"],
                      "n_classes": ncls, "N": info["N"], "frames": F, "sources": 2},
           "plan_build_s": plan_s, "batches": {}}
    for B in [int(b) for b in args.batches.split(",")]:
        if B == 1:
            n1 = args.single_frames
            sl = [X[f:f + 1] for f in range(n1)]
            outs = [(doa[f:f + 1], power[f:f + 1], yhat[f:f + 1], margin[f:f + 1]) for f in range(n1)]

            def loop():
                for f in range(n1):
                    amd.svdphat_locate(h, sl[f], prec, mode, *outs[f])
            _timed(loop, 1, torch)
            dt = _timed(loop, 2, torch) / 2
            host_fps = n1 / dt
            # the same n1 calls captured once into a graph on a side stream
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                for f in range(n1):
                    amd.svdphat_locate(h, sl[f], prec, mode, *outs[f], stream=s)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                for f in range(n1):
                    amd.svdphat_locate(h, sl[f], prec, mode, *outs[f], stream=s)
            g.replay()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 5
            e0.record()
            for _ in range(reps):
                g.replay()
            e1.record()
            torch.cuda.synchronize()
            us = 1e3 * e0.elapsed_time(e1) / (reps * n1)
            del g
            # per-kernel durations (HIP events around each launch)
            amd.svdphat_timing_reset()
            amd.svdphat_timing_enable(True)
            for f in range(min(256, n1)):
                amd.svdphat_locate(h, sl[f], prec, mode, *outs[f])
            amd.svdphat_timing_enable(False)
            kt = amd.svdphat_timing_read()
            amd.svdphat_timing_reset()
            kern = {k: dict(avg_us=1e3 * v[0] / v[1], launches=v[1]) for k, v in kt.items()}
            # bytes a frame reads if the FP32 operands are not cached: A (2K x 2L)
            # and U (classes x 2K), and the frame
            op_bytes = K2 * 2 * L * 4 + ncls * K2 * 4 + info["M"] * info["B"] * 8
            r = dict(form="GEMV form, FP32 projections, exact FP32 argmax", frames=n1,
                     host_loop_fps=host_fps, graph_fps=1e6 / us, graph_us_per_frame=us, kernels_us=kern,
                     operand_bytes_per_frame=op_bytes,
                     operand_GBps_graph=op_bytes / (us * 1e-6) / 1e9, hbm_peak_GBps=HBM_PEAK_GBS)
            d = doa[:n1].cpu().numpy()
            m = min(n1, ng)
        else:
            nb = F // B
            def step():
                for i in range(nb):
                    amd.svdphat_locate(h, X[i * B:(i + 1) * B], prec, mode, doa[i * B:(i + 1) * B],
                                       power[i * B:(i + 1) * B], yhat[i * B:(i + 1) * B],
                                       margin[i * B:(i + 1) * B])
            _timed(step, 1, torch)
            ns = max(2, args.steps // 10)
            dt = _timed(step, ns, torch)
            fps = nb * B * ns / dt
            amd.svdphat_timing_reset()
            amd.svdphat_timing_enable(True)
            step()
            amd.svdphat_timing_enable(False)
            kt = amd.svdphat_timing_read()
            amd.svdphat_timing_reset()
            kern = {k: dict(avg_us=1e3 * v[0] / v[1], launches=v[1]) for k, v in kt.items()}
            flops = 2.0 * K2 * 2 * L + 2.0 * ncls * K2
            g1 = kern.get("gemm1", {}).get("avg_us")
            g2 = kern.get("gemm2", {}).get("avg_us")
            r = dict(form="BF16 MFMA, FP32 accumulate, FP32 rescoring", fps=fps, ms_per_batch=1e3 * dt / (ns * nb),
                     kernels_us=kern,
                     gemm1_mfma_frac=(2.0 * K2 * 2 * L * B / (g1 * 1e-6) / 1e12 / MFMA_FP16_PEAK_TFLOPS) if g1 else None,
                     gemm2_mfma_frac=(2.0 * ncls * K2 * B / (g2 * 1e-6) / 1e12 / MFMA_FP16_PEAK_TFLOPS) if g2 else None,
                     mflop_per_frame=flops / 1e6)
            d = doa[:nb * B].cpu().numpy()
            m = min(nb * B, ng)
        judged = gold["margin"][:m] > 1e-5
        r["match_all"] = float(np.mean(d[:m] == gold["doa"][:m]))
        r["match_judged"] = float(np.mean(d[:m][judged] == gold["doa"][:m][judged]))
        r["oracle_frames"] = m
        out["batches"][str(B)] = r
        log(f"batch {B}: {json.dumps(r)[:300]}")
    head = out["batches"].get("4096") or next(iter(out["batches"].values()))
    out["value"] = head.get("fps", head.get("graph_fps"))
    out["steps"] = args.steps
    out["warmup"] = args.warmup
    print(json.dumps(out))


def bench_ragged(args, torch, amd, synth):
    """Many arrays with their own plans in one graph launch (FP16 + FP32
    rescoring) against one svdphat_locate call per array."""
    arrs = synth.ragged_workload(args.arrays)
    grids = {lv: synth.icosphere(lv) for lv in sorted({a["level"] for a in arrs})}
    t0 = time.perf_counter()
    plans = []
    for i, a in enumerate(arrs):
        plans.append(amd.Plan(a["mics"], grids[a["level"]], 16000.0, 343.0, 512, a["delta"]))
        if i % 32 == 31:
            log(f"plans {i + 1}/{len(arrs)} ({time.perf_counter() - t0:.1f} s)")
    plan_s = time.perf_counter() - t0
    Xs = [torch.from_numpy(a["X"]).cuda() for a in arrs]
    Ftot = sum(x.shape[0] for x in Xs)
    t0 = time.perf_counter()
    # tuning results cached across runs of this process's machine (tmp dir)
    cache = os.path.join(tempfile.gettempdir(), "svdphat_ragged_tune.jsonl")
    rg = amd.Ragged(plans, [x.shape[0] for x in Xs], tune=True, tune_cache=cache)
    tune_s = time.perf_counter() - t0
    tuned, cached = rg.info()
    log(f"{len(arrs)} arrays, {Ftot} frames; plans {plan_s:.1f} s, ragged build+tune {tune_s:.1f} s")
    doas = [torch.empty(x.shape[0], dtype=torch.int32, device="cuda") for x in Xs]
    pows = [torch.empty(x.shape[0], dtype=torch.float32, device="cuda") for x in Xs]
    step = lambda: amd.svdphat_ragged_locate(rg._h, Xs, doas, pows)
    _timed(step, args.warmup, torch)
    dt = _timed(step, args.steps, torch)
    fps = Ftot * args.steps / dt
    rdoa = [d.cpu().numpy().copy() for d in doas]
    # one call per array on the same stream
    def singles():
        for p, x, d, pw in zip(plans, Xs, doas, pows):
            amd.svdphat_locate(p.handle, x, amd.FP16, amd.RESCORE, d, pw)
    _timed(singles, 1, torch)
    ns = max(1, args.steps // 5)
    dts = _timed(singles, ns, torch)
    single_fps = Ftot * ns / dts
    agree = float(np.mean(np.concatenate([a == d.cpu().numpy() for a, d in zip(rdoa, doas)])))
    Ks = [p.info["K"] for p in plans]
    # roofline of the whole step: every array's STFT frames read once against
    # HBM, and the two products' arithmetic (GEMM1: 2 Rp 2L per frame, GEMM2:
    # 2 classes Rp per frame, Rp = 2K padded to 32) against FP16 MFMA
    step_s = dt / args.steps
    in_bytes = sum(x.numel() * x.element_size() for x in Xs)
    flops = 0.0
    for p, x in zip(plans, Xs):
        rp = -(-2 * p.info["K"] // 32) * 32
        flops += x.shape[0] * (2.0 * rp * 2 * p.info["L"] + 2.0 * p.info["n_classes"] * rp)
    roof = {"bound": "hbm", "achieved": in_bytes / step_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": in_bytes / step_s / 1e9 / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": in_bytes,
            "kernel": "whole step (graph of grouped stages)"}
    mfma = {"tflops": flops / step_s / 1e12, "peak": 2500.0, "frac": flops / step_s / 1e12 / 2500.0,
            "flops_per_step": flops}
    out = {
        "metric": "frames/s, ragged batch of arrays in one graph launch",
        "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp16", "data": "synthetic",
        "config": {"workload": "ragged256", "arrays": len(arrs), "frames_per_step": Ftot,
                   "M_range": [min(len(a["mics"]) for a in arrs), max(len(a["mics"]) for a in arrs)],
                   "K_range": [min(Ks), max(Ks)], "Q_levels": sorted(grids)},
        "single_call_fps": single_fps, "speedup_vs_single_calls": fps / single_fps,
        "doa_agreement_with_single_calls": agree, "tuned_shapes": tuned, "cached_shapes": cached,
        "plan_build_s": plan_s, "ragged_build_s": tune_s, "roofline": roof, "mfma": mfma,
    }
    print(json.dumps(out))


def bench_proposal(args, torch, amd, synth):
    """Learned proposal on the planar array at Q = 40962 (icosphere level 6)
    with 642 coarse cells (level 3): trained on the method's own labels, then
    timed against the full search on fresh frames."""
    mics = synth.geometry("2d")
    fine, coarse = synth.icosphere(6), synth.icosphere(3)
    t0 = time.perf_counter()
    plan = amd.Plan(mics, fine, 16000.0, 343.0, 512, 1e-5)
    plan_s = time.perf_counter() - t0
    prop = amd.Proposal(plan, coarse, hidden=256, seed=1)
    log(f"plan {plan_s:.1f} s, K={plan.info['K']}, classes={plan.info['n_classes']}")
    batch = 8192
    nsteps = max(1, args.train_frames // batch)
    total = nsteps * max(1, args.train_epochs)
    t0 = time.perf_counter()
    losses = []
    for step in range(total):
        # the same nsteps batches (train_frames pairs) in every epoch
        X = synth.plane_wave_fd_torch(mics, batch // 64, 64, 512, 16000.0, 343.0, seed=5_000_000 + step % nsteps)
        lr = 2e-3 if step < int(0.7 * total) else 5e-4
        losses.append(prop.train_step(X, lr=lr))
        if step % 100 == 0:
            log(f"train step {step}/{total} loss {losses[-1]:.3f}")
    train_s = time.perf_counter() - t0
    # evaluation: 20000 fresh frames, SNR U[-5, 20] dB, 100-frame segments
    X = synth.plane_wave_fd_torch(mics, 200, 100, 512, 16000.0, 343.0, seed=9_999_999)
    F = X.shape[0]
    dev = X.device
    doa = torch.empty(F, dtype=torch.int32, device=dev)
    power = torch.empty(F, dtype=torch.float32, device=dev)
    fell = torch.empty(F, dtype=torch.uint8, device=dev)
    yhat = torch.empty(F, dtype=torch.float32, device=dev)
    margin = torch.empty(F, dtype=torch.float32, device=dev)
    fdoa = torch.empty(F, dtype=torch.int32, device=dev)
    h = plan.handle
    prop_step = lambda: amd.lib().svdphat_proposal_locate(prop._h, amd._ptr(X), F, 8, 0.5, amd._ptr(doa),
                                                          amd._ptr(power), amd._ptr(fell), amd._stream(None))
    full_step = lambda: amd.svdphat_locate(h, X, amd.FP16, amd.RESCORE | amd.HILO, fdoa, power, yhat, margin)
    _timed(prop_step, args.warmup, torch)
    dtp = _timed(prop_step, args.steps, torch)
    pdoa, pfell = doa.cpu().numpy(), fell.cpu().numpy().astype(bool)
    _timed(full_step, args.warmup, torch)
    dtf = _timed(full_step, args.steps, torch)
    full = fdoa.cpu().numpy()
    # per-kernel durations of the proposal path (HIP events on its stream)
    amd.svdphat_timing_reset()
    amd.svdphat_timing_enable(True)
    for _ in range(args.steps):
        prop_step()
    amd.svdphat_timing_enable(False)
    kt = amd.svdphat_timing_read()
    amd.svdphat_timing_reset()
    kernels = {k: dict(avg_us=1e3 * v[0] / v[1], launches=v[1]) for k, v in kt.items()}
    # rows rescored per confident frame (the kernel's own count) against the
    # full search, which scores every direction class and rescores tiles
    amd.svdphat_timing_enable(False, counts=True)
    prop_step()
    full_step()
    torch.cuda.synchronize()
    amd.svdphat_timing_enable(False)
    cnt = amd.svdphat_timing_read()
    amd.svdphat_timing_reset()
    rows, conf_frames = cnt.get("count:proposal_rows_rescored", (0.0, 0))
    tiles, _ = cnt.get("count:final_tiles_rescored", (0.0, 0))
    work = {"rows_rescored_per_confident_frame": rows / max(conf_frames, 1),
            "full_search_classes_scored_per_frame": plan.info["n_classes"],
            "full_search_fp32_rows_rescored_per_frame": 64.0 * tiles / F}
    out = {
        "metric": "frames/s, learned proposal vs full search (planar, Q=40962)",
        "value": F * args.steps / dtp, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dtp / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp16", "data": "synthetic",
        "config": {"workload": "proposal_q40962", "Q": 40962, "cells": 642, "hidden": 256,
                   "K": plan.info["K"], "frames_per_step": F, "train_pairs": nsteps * batch,
                   "train_epochs": max(1, args.train_epochs),
                   "topk": 8, "conf_min": 0.5},
        "full_search_fps": F * args.steps / dtf, "speedup_vs_full_search": dtf / dtp,
        "miss_rate_vs_full_search": float(np.mean(pdoa != full)),
        "fallback_rate": float(pfell.mean()),
        "miss_rate_confident_frames": float(np.mean(pdoa[~pfell] != full[~pfell])) if (~pfell).any() else 0.0,
        "final_loss": float(np.mean(losses[-10:])), "train_s": train_s, "plan_build_s": plan_s,
        "kernels_us": kernels, "work": work,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
