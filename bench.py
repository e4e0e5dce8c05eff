#!/usr/bin/env python3
"""Benchmark of the online IS-NMF hot path on one MI355X.

Workload: one pass of online IS-NMF (Algorithm 1 with mini-batches, fresh
restarts) over N = 1,000,000 synthetic Gamma/Exponential power-spectrogram
frames, F = 513, K = 50, minibatch b = 128, I = 20 multiplicative updates of
h per frame, FP32 fused MFMA path.  A "step" is one isnmf_online_step: the
inner fit of the minibatch, the fold into A and B, W = sqrt(A/B) and the
column rescaling.  V is resident in HBM before the timed region starts.

Printed: one JSON line with the whole-job frames/s, the fit kernel's
roofline position (HIP events around every fit launch), the plain FP32
comparison path, and the FP64 CPU oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "online IS-NMF frames/s at F=513,K=50 vs plain FP32; p99 chunk latency"
F, K, B, ITERS = 513, 50, 128, 20
PEAK_FP32_MFMA = 157.3e12        # MI355X dense FP32 matrix peak, FLOP/s


def flops_per_frame(F: int, K: int, iters: int) -> float:
    """Algorithmic flops of one frame: I+1 model products W h, I pairs
    W^T r2, W^T r1, and the rank-1 increments of A and B: (3I + 3) F K MACs."""
    return 2.0 * (3 * iters + 3) * F * K


# HBM traffic of the fit kernel measured with rocprofv3 --pmc (FETCH_SIZE,
# WRITE_SIZE), keyed by the sha1 of the kernel source it was measured on.
# A changed kernel has no entry, and its traffic is reported as null.
TRAFFIC = {
    # FETCH_SIZE 707.9 KiB x 2.0 + WRITE_SIZE 547.0 KiB x 1.0 per b=128 launch
    # (profiles/fused_fit_F513_K50_b128_pmc.md)
    "69c549109c00391bd413404f3696582ba3f5306d": 1962.8 * 1024,
}


def _src_hash() -> str:
    p = os.path.join(ROOT, "paper_1106_4198_amd", "csrc", "fused.hip")
    return hashlib.sha1(open(p, "rb").read()).hexdigest()


def cpu_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(V, W0, target_s: float):
    """The FP64 oracle on the host cores over a bounded prefix of the stream."""
    import numpy as np
    import oracle

    nt = cpu_threads()
    oracle.set_threads(nt)
    st = oracle.OnlineState(W0.astype(np.float64))
    t0 = time.perf_counter()
    st.step(V[:, :B].astype(np.float64), iters=ITERS)
    one = time.perf_counter() - t0
    steps = max(2, min(256, int(target_s / max(one, 1e-3))))
    Vs = V[:, :steps * B].astype(np.float64)
    st = oracle.OnlineState(W0.astype(np.float64))
    t0 = time.perf_counter()
    for s in range(steps):
        st.step(Vs[:, s * B:(s + 1) * B], iters=ITERS)
    dt = time.perf_counter() - t0
    oracle.set_threads(1)
    return {"value": steps * B / dt, "unit": "frames/s", "cores": nt, "kind": "oracle",
            "sample": f"first {steps} minibatches ({steps * B} frames) of the same stream, "
                      f"F={F} K={K} b={B} I={ITERS}, FP64, {dt:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="minibatch steps to time (default: the whole pass, 7813)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--frames", type=int, default=1_000_000)
    ap.add_argument("--plain-steps", type=int, default=100)
    ap.add_argument("--form-steps", type=int, default=2000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--seed", type=int, default=2011)
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic, to scale rocprofv3 FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU design is described in DESIGN.md and not measured", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1106_4198_amd import binding as bd
    from paper_1106_4198_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    if args.copy_calib_mib > 0:
        src = torch.ones(args.copy_calib_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    N = args.frames
    steps_full = (N + B - 1) // B
    steps = steps_full if args.steps is None else max(1, min(args.steps, steps_full))
    nframes = min(N, steps * B)

    t0 = time.perf_counter()
    V = synth.frames(F, K, N, args.seed, threads=cpu_threads())
    W0 = synth.initial_dictionary(F, K, args.seed)
    gen_s = time.perf_counter() - t0
    Vt = torch.from_numpy(np.ascontiguousarray(V.T)).to(dev)     # (N, F): frame-contiguous
    Wt = torch.from_numpy(np.ascontiguousarray(W0.T)).to(dev)
    torch.cuda.synchronize()
    print(f"[bench] data ready: N={N} F={F} ({Vt.numel() * 4 / 2**30:.2f} GiB) in {gen_s:.1f} s",
          file=sys.stderr, flush=True)

    # warm-up on a scratch stream state
    g = bd.OnlineISNMF(Wt, B, inner_iters=ITERS)
    assert g.kernel_used == "fused"
    if args.warmup > 0:
        g.run_pass(Vt[:min(N, args.warmup * B)], B)
    torch.cuda.synchronize()
    g.close()

    # timed region: `steps` minibatch steps from frame 0 of a fresh state
    g = bd.OnlineISNMF(Wt, B, inner_iters=ITERS)
    loss = torch.zeros((), dtype=torch.float64, device=dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    g.run_pass(Vt[:nframes], B, loss_sum=loss)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    fps = nframes / (ms / 1e3)
    assert g.status() == 0
    online_loss = loss.item() / nframes / F
    g.close()
    print(f"[bench] fused FP32: {steps} steps, {ms:.1f} ms, {fps:.4g} frames/s", file=sys.stderr,
          flush=True)

    # roofline of the fit kernel: HIP events around every fit launch of the same pass
    g = bd.OnlineISNMF(Wt, B, inner_iters=ITERS)
    g.set_timing(True, steps)
    g.run_pass(Vt[:nframes], B)
    launches, fit_ms = g.timing()
    g.close()
    fit_flops = flops_per_frame(F, K, ITERS) * nframes
    achieved = fit_flops / (fit_ms / 1e3)
    traffic = TRAFFIC.get(_src_hash())
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA, "traffic": traffic,
                "kernel": "fused_fit_kernel<8,1,52>", "launches": launches,
                "avg_launch_us": fit_ms * 1e3 / max(launches, 1),
                "flops_per_launch": flops_per_frame(F, K, ITERS) * B}

    # precision forms: BF16 / FP16 products, same stream prefix
    def time_form(precision, nsteps):
        gw = bd.OnlineISNMF(Wt, B, inner_iters=ITERS, precision=precision)
        gw.run_pass(Vt[:B * 4], B)
        gw.close()
        gf = bd.OnlineISNMF(Wt, B, inner_iters=ITERS, precision=precision)
        torch.cuda.synchronize()
        e0.record()
        gf.run_pass(Vt[:nsteps * B], B)
        e1.record()
        torch.cuda.synchronize()
        v = nsteps * B / (e0.elapsed_time(e1) / 1e3)
        gf.close()
        return v

    f_steps = max(1, min(args.form_steps, steps))
    forms = {p: {"value": time_form(p, f_steps), "unit": "frames/s", "steps": f_steps}
             for p in ("bf16", "fp16")}

    # the plain FP32 path (one op per launch) over a prefix, same shapes
    p_steps = max(1, min(args.plain_steps, steps))
    gp = bd.OnlineISNMF(Wt, B, inner_iters=ITERS, kernel="plain")
    gp.run_pass(Vt[:B], B)
    torch.cuda.synchronize()
    gp.close()
    gp = bd.OnlineISNMF(Wt, B, inner_iters=ITERS, kernel="plain")
    e0.record()
    gp.run_pass(Vt[:p_steps * B], B)
    e1.record()
    torch.cuda.synchronize()
    plain_fps = p_steps * B / (e0.elapsed_time(e1) / 1e3)
    gp.close()

    out = {
        "metric": METRIC,
        "value": fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"online IS-NMF one pass, fresh restarts: F={F} K={K} "
                               f"N={nframes} frames b={B} I={ITERS}, fused FP32 MFMA",
                   "F": F, "K": K, "b": B, "inner_iters": ITERS, "frames": nframes,
                   "generator": "V=(W_true H_true)*E, W_true~Gamma(0.5), H_true~Gamma(0.3), "
                                "E~Exp(1), seeded PCG64"},
        "roofline": roofline,
        "plain_fp32": {"value": plain_fps, "unit": "frames/s", "steps": p_steps,
                       "speedup_fused": fps / plain_fps},
        "online_loss_per_entry": online_loss,
        "forms": forms,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(V, W0, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
