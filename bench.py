#!/usr/bin/env python3
"""Benchmark of the online IS-NMF hot path on one MI355X.

Workload: one pass of online IS-NMF (Algorithm 1 with mini-batches, fresh
restarts) over N = 1,000,000 synthetic Gamma/Exponential power-spectrogram
frames, F = 513, K = 50, minibatch b = 128, I = 20 multiplicative updates of
h per frame, FP32 fused path (the fit variant, MFMA tile or VALU, chosen by
the library's autotuner before timing).  A "step" is one isnmf_online_step: the
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
PEAK_FP32_VECTOR = 157.3e12      # MI355X FP32 vector peak (packed FMA), FLOP/s
# FP32 FMA without packed math: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
PEAK_FP32_VALU_UNPACKED = 256 * 4 * 16 * 2 * 2.4e9


def flops_per_frame(F: int, K: int, iters: int) -> float:
    """Algorithmic flops of one frame's whole step: I+1 model products W h,
    I pairs W^T r2, W^T r1, and the rank-1 increments of A and B:
    (3I + 3) F K multiply-adds."""
    return 2.0 * (3 * iters + 3) * F * K


def fit_flops_per_frame(F: int, K: int, iters: int) -> float:
    """Flops of one frame inside the fit kernel alone: I+1 model products and
    I pairs of transposed products, (3I + 1) F K multiply-adds."""
    return 2.0 * (3 * iters + 1) * F * K


# HBM traffic of the fit kernel measured with rocprofv3 --pmc (FETCH_SIZE,
# WRITE_SIZE), keyed by (kernel, sha1 of the sources it was built from).  A
# changed kernel has no entry and its traffic is reported as null.
FIT_SOURCES = {
    "valu": ("fit_valu.h", "fit_valu.hip"),
    "mfma": ("fit_body.h", "fit_launch.h", "fit_f32.hip"),
}
TRAFFIC = {
    # FETCH_SIZE 716.0 KiB x 2.0 + WRITE_SIZE 558.5 KiB x 1.0 per b=128 launch
    # (profiles/fit_valu_F513_K50_b128_pmc.md)
    ("fit_valu_kernel<7,9,false,8>", "95871bd11515f8a347fbf5913caec1f1600f0aa3"): (716.0 * 2.0 + 558.5) * 1024,
}


def _src_hash(kind: str) -> str:
    h = hashlib.sha1()
    for name in FIT_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_1106_4198_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def fit_kernel_name(nw: int, cpw: int, kmax: int, wg: int) -> tuple:
    """(kind, kernel symbol) of the tuned FP32 fit variant for (F, K)."""
    if cpw == 0:
        return "valu", f"fit_valu_kernel<{(K + 7) // 8},{(F + 8 * nw - 1) // (8 * nw)},false,{nw}>"
    return "mfma", f"fit_single_kernel<{nw},{cpw},{kmax},0,{bool(wg)}>"


def cpu_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


# minibatch steps at which the forms' errors are reported; 7813 is the end of
# the pass over 10^6 frames (7812 full minibatches and one of 64 frames)
CHECKPOINTS = (1, 10, 100, 1000, 7813)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(V, W0, target_s: float, snaps=None, accuracy_steps: int = 0):
    """The FP64 oracle on the host cores over a bounded prefix of the stream
    (the timed sample).  With snaps (a dict), the same oracle run continues,
    untimed, to accuracy_steps minibatches, and snaps receives its (W, A, B,
    loss sum) after each step count in CHECKPOINTS it reaches."""
    import numpy as np
    import oracle

    nt = cpu_threads()
    oracle.set_threads(nt)
    st = oracle.OnlineState(W0.astype(np.float64))
    t0 = time.perf_counter()
    st.step(V[:, :B].astype(np.float64), iters=ITERS)
    one = time.perf_counter() - t0
    steps = max(2, min(2048, int(target_s / max(one, 1e-3))))
    Vs = V[:, :steps * B].astype(np.float64)
    st = oracle.OnlineState(W0.astype(np.float64))

    def snap(s):
        if snaps is not None and s in CHECKPOINTS:
            snaps[s] = (st.W.copy(), st.A.copy(), st.B.copy(), st.loss_sum)

    t0 = time.perf_counter()
    for s in range(steps):
        st.step(Vs[:, s * B:(s + 1) * B], iters=ITERS)
        snap(s + 1)
    dt = time.perf_counter() - t0
    del Vs
    if snaps is not None:
        last = min(accuracy_steps, (V.shape[1] + B - 1) // B)
        t1 = time.perf_counter()
        for s in range(steps, last):
            st.step(V[:, s * B:(s + 1) * B].astype(np.float64), iters=ITERS)
            snap(s + 1)
        if last > steps:
            print(f"[bench] oracle continued to minibatch {last} for the accuracy checkpoints "
                  f"({time.perf_counter() - t1:.1f} s, untimed)", file=sys.stderr, flush=True)
    oracle.set_threads(1)
    return {"value": steps * B / dt, "unit": "frames/s", "cores": nt, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"first {steps} minibatches ({steps * B} frames) of the same stream, "
                      f"F={F} K={K} b={B} I={ITERS}, FP64, {dt:.1f} s"}


PEAK_BF16_MFMA = 2500e12        # MI355X dense BF16 matrix peak, FLOP/s


def form_accuracy(bd, torch, np, Vt, Wt, snaps, fp32_variant, form_variants=None):
    """Relative error (Frobenius) of W, A, B and of the online loss sum against
    the FP64 oracle's snapshots, per form, at the checkpoints the oracle
    reached: each form runs the same stream prefix from W(0).  The FP32 fused
    form runs fp32_variant (nw, cpw, wg), the fit variant of the timed pass,
    and the 16-bit forms the variants they were timed on (form_variants)."""
    cps = sorted(snaps)
    out = {"checkpoints": cps, "reference": "FP64 oracle, same stream prefix from W(0)",
           "measure": "||x - x_oracle||_F / ||x_oracle||_F; loss: |sum - sum_oracle| / sum_oracle"}
    if not cps:
        return out

    def rel(x, y):
        return float(np.linalg.norm(x - y) / np.linalg.norm(y))

    bd.tune_set(F, K, "fp32", *fp32_variant)
    for p, v in (form_variants or {}).items():
        bd.tune_set(F, K, p, *v)
    for name, kw in (("fp32", {}), ("bf16", {"precision": "bf16"}), ("fp16", {"precision": "fp16"}),
                     ("fp32_plain", {"kernel": "plain"})):
        g = bd.OnlineISNMF(Wt, B, inner_iters=ITERS, **kw)
        loss = torch.zeros((), dtype=torch.float64, device=Vt.device)
        rec = {"W": [], "A": [], "B": [], "loss": []}
        done = 0
        for c in cps:
            g.run_pass(Vt[done * B:c * B], B, loss_sum=loss)
            done = c
            _, A, Bm, _ = g.get()
            W64 = g.get_w64()
            Wr, Ar, Br, lr = snaps[c]
            rec["W"].append(rel(W64.cpu().double().numpy().T, Wr))
            rec["A"].append(rel(A.cpu().numpy().T, Ar))
            rec["B"].append(rel(Bm.cpu().numpy().T, Br))
            rec["loss"].append(abs(loss.item() - lr) / lr)
        assert g.status() == 0
        g.close()
        out[name] = rec
    return out


def gen_streams(synth, shapes, seed0, threads):
    """Per-stream seeded frames: shapes = [(F, K, frames)] -> [(V F x N, W0)]."""
    from concurrent.futures import ThreadPoolExecutor

    def one(i):
        F, K, N = shapes[i]
        return synth.frames(F, K, N, seed0 + i), synth.initial_dictionary(F, K, seed0 + i)

    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, range(len(shapes))))


def bench_batched(bd, synth, torch, np, dev, S, steps, threads, mixed, seed0, precision="bf16"):
    """S streams advanced together, one replayed hipGraph per step; BF16
    products, or FP32 (the metric's own arithmetic)."""
    rng = np.random.default_rng(seed0)
    if mixed:
        Fs = rng.choice([257, 513, 1025], size=S)
        Ks = rng.integers(16, 129, size=S)
        bs = rng.choice([32, 64, 128, 256], size=S)
    else:
        Fs, Ks, bs = np.full(S, F), np.full(S, K), np.full(S, B)
    warm = 1
    shapes = [(int(Fs[i]), int(Ks[i]), int(bs[i]) * (steps + warm)) for i in range(S)]
    t0 = time.perf_counter()
    data = gen_streams(synth, shapes, seed0, threads)
    gen_s = time.perf_counter() - t0
    Vs = [torch.from_numpy(np.ascontiguousarray(V.T)).to(dev) for V, _ in data]
    shape_set = sorted(set((int(a), int(b)) for a, b in zip(Fs, Ks)))

    def tune(floor):
        # kernel variant per distinct shape, timed at the frames of every
        # stream of that shape and at least `floor`
        chosen = {}
        for (Fi, Ki) in shape_set:
            nb = int(sum(int(bb) for a, b2, bb in zip(Fs, Ks, bs) if int(a) == Fi and int(b2) == Ki))
            bd.autotune(Fi, Ki, max(nb, floor), precision=precision, trials=2)
            chosen[(Fi, Ki)] = bd.tune_get(Fi, Ki, precision)
        return chosen

    def make():
        hs = [bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(W0.T)).to(dev), int(b),
                             precision=precision) for (_, W0), b in zip(data, bs)]
        return hs, bd.MultiISNMF(hs, Vs, [int(x) for x in bs], loss=True)

    # Step-level choice of the tuning: a floor of 8192 frames tunes each shape
    # for throughput (right when a shape's launch is full), 1024 leans to
    # latency (right when a shape has few frames and one slow workgroup would
    # hold the whole step).  With several shapes, tunings at 8192 (twice: the
    # per-shape choices are timed alone and vary from one tuning to the next),
    # at 1024, and a table by rule (the 16-frame tile variants wherever they
    # fit) are each timed on the captured step itself (one warm-up and three
    # timed replays), and the table of the fastest is restored for the timed
    # run, so that the run measures the configuration that was chosen.
    def by_rule(base):
        # the 16-frame tile variant wherever it fits, else its streamed form:
        # the throughput variants, chosen without per-shape timings
        chosen = {}
        bd.tune_clear()
        for (Fi, Ki), v in base.items():
            for cand in ((8, -1, 0), (8, -2, 0), v):
                try:
                    bd.tune_set(Fi, Ki, precision, *cand)
                except bd.IsnmfError:
                    continue
                chosen[(Fi, Ki)] = cand
                break
        return chosen

    floors = [8192, 8192, 1024, "rule"] if len(shape_set) > 1 else [8192]
    trial, tables = [], []
    for fl in floors:
        bd.tune_clear()
        tables.append((fl, by_rule(tables[0][1]) if fl == "rule" else tune(fl)))
        if len(floors) > 1:
            hs, m = make()
            m.run(1, graph=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m.run(3, graph=True)
            torch.cuda.synchronize()
            trial.append((time.perf_counter() - t0) / 3 * 1e3)
            m.close()
            for h in hs:
                h.close()
    best = min(range(len(trial)), key=trial.__getitem__) if trial else 0
    floor, variants = tables[best]
    bd.tune_clear()
    for (Fi, Ki), v in variants.items():
        bd.tune_set(Fi, Ki, precision, *v)
    tuned = len(shape_set)
    hs, m = make()
    m.run(warm, graph=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    m.run(steps, graph=True)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    frames = int(sum(int(b) * steps for b in bs))
    flops = float(sum(flops_per_frame(int(Fi), int(Ki), ITERS) * int(b) * steps
                      for Fi, Ki, b in zip(Fs, Ks, bs)))
    fit_launches, fold_launches, rescale_launches = m.launches()
    m.close()
    for h in hs:
        h.close()
    peak = PEAK_BF16_MFMA if precision == "bf16" else PEAK_FP32_MFMA
    out = {"value": frames / (ms / 1e3), "unit": "frames/s", "streams": S, "steps": steps,
           "ms_per_step": ms / steps, "precision": precision, "graph": True,
           "achieved_tflops": flops / (ms / 1e3) / 1e12,
           f"frac_{precision}_peak": flops / (ms / 1e3) / peak,
           "gen_s": round(gen_s, 1),
           "launches_per_step": {"fit": fit_launches, "fold": fold_launches,
                                 "rescale": rescale_launches}}
    n_tile = sum(1 for v in variants.values() if v[1] == -1)
    n_stile = sum(1 for v in variants.values() if v[1] == -2)
    n_t32 = sum(1 for v in variants.values() if v[1] == -3)
    out["variants"] = {"shapes": tuned, "tile16x16x32": n_tile, "tile16x16x32_streamed": n_stile,
                       "tile16x16x4_fp32": n_t32,
                       "tune_floor_frames": floor,
                       "trial_ms_per_step": [[fl, round(v, 3)] for (fl, _), v in zip(tables, trial)]}
    if mixed:
        out["workload"] = ("F in {257,513,1025}, K ~ U[16,128], b in {32,64,128,256}, "
                           f"{steps} timed minibatches per stream; {tuned} shapes autotuned")
    else:
        out["workload"] = f"{S} streams of F={F} K={K} b={B}, {steps} timed minibatches each"
        out["variant"] = list(variants[(F, K)])
    bd.tune_clear()
    return out


def bench_batch_mu(bd, torch, np, Vt, Wt, N, cycles):
    """Batch MU (section 2.1) over the first N frames from W(0), H = 1, with the
    objective of eq. (1) after every cycle.  Algorithmic work per cycle: the
    H update (W H and the pair W^T r2, W^T r1), the statistics of eq. (3) at
    the new H (W H again and the rank-N products) and the objective's W H:
    7 F K N multiply-adds.  The fit runs the variant the autotuner picks for
    one update of N frames; the shape's tuning entry is restored afterwards."""
    V = Vt[:N]
    saved = bd.tune_get(F, K, "fp32")
    bd.autotune(F, K, N, precision="fp32", inner_iters=1, trials=3)
    variant = bd.tune_get(F, K, "fp32")
    try:
        return _time_batch_mu(bd, torch, np, V, Wt, N, cycles, variant)
    finally:
        bd.tune_set(F, K, "fp32", *saved)


def _time_batch_mu(bd, torch, np, V, Wt, N, cycles, variant):

    def fresh():
        return Wt.clone(), torch.ones((N, K), dtype=torch.float32, device=V.device)

    W, H = fresh()
    bd.batch_mu(V, W, H, 1)                         # warm-up (and workspace allocation)
    torch.cuda.synchronize()
    W, H = fresh()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    tr = bd.batch_mu(V, W, H, cycles)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    tr = tr.cpu().numpy()
    flops = 2.0 * 7 * F * K * N * cycles
    return {"value": cycles / (ms / 1e3), "unit": "cycles/s", "frames": N, "cycles": cycles,
            "ms_per_cycle": ms / cycles, "frame_cycles_per_s": N * cycles / (ms / 1e3),
            "achieved_tflops": flops / (ms / 1e3) / 1e12,
            "frac_fp32_peak": flops / (ms / 1e3) / PEAK_FP32_MFMA,
            "objective_per_entry": [float(tr[0]) / F, float(tr[-1]) / F],
            "monotone": bool(np.all(np.diff(tr) <= 1e-6 * tr[:-1])), "fit_variant": list(variant)}


def bench_multipass(bd, torch, np, Vt, Wt, N, passes, seed):
    """Warm-restart passes over a finite set of N frames (section 2.3): H of
    all N frames resident, each pass in its own seeded random order, FP32
    fused path.  frames/s counts visits (passes x N)."""
    rng = np.random.default_rng(seed)
    perm = torch.from_numpy(np.stack([rng.permutation(N) for _ in range(passes)])
                            .astype(np.int32)).to(Vt.device)
    V = Vt[:N]
    g = bd.OnlineISNMF(Wt, B, inner_iters=ITERS, warm=True)
    H = torch.ones((N, K), dtype=torch.float32, device=Vt.device)
    nw = min(N, 4 * B)                                  # warm-up: one pass over a prefix
    pw = torch.arange(nw, dtype=torch.int32, device=Vt.device).view(1, nw)
    g.run_passes(V[:nw], pw, B, H[:nw])
    g.close()
    g = bd.OnlineISNMF(Wt, B, inner_iters=ITERS, warm=True)
    H = torch.ones((N, K), dtype=torch.float32, device=Vt.device)
    loss = torch.zeros((), dtype=torch.float64, device=Vt.device)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    g.run_passes(V, perm, B, H, loss)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert g.status() == 0
    g.close()
    return {"value": passes * N / (ms / 1e3), "unit": "frames/s (visits)", "frames": N,
            "passes": passes, "b": B, "ms": ms,
            "loss_per_entry": loss.item() / (passes * N * F)}


def bench_heldout(bd, synth, torch, np, g, Wt, dev, seed, start, n_test=8192):
    """The paper's criterion (section 3): unseen frames of the same stream (the
    n_test frames after the pass), their h fitted at a frozen dictionary, then
    eq. (1) per matrix entry; at the learned W (handle g) and at W(0)."""
    Vte = synth.frames(F, K, n_test, seed, start=start)
    Vt = torch.from_numpy(np.ascontiguousarray(Vte.T)).to(dev)
    # at the generator's true factors the expected divergence per entry is Euler's
    # gamma (E[e - log e - 1] for e ~ Exp(1)): the floor a dictionary can reach
    out = {"frames": n_test, "first_frame": start, "floor_per_entry": 0.5772156649015329}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for name in ("W", "W0"):
        h = g if name == "W" else bd.OnlineISNMF(Wt, B, inner_iters=ITERS)
        H = torch.empty((n_test, K), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        e0.record()
        for s0 in range(0, n_test, B):
            h.fit(Vt[s0:s0 + B], H[s0:s0 + B])
        e1.record()
        torch.cuda.synchronize()
        W = h.get()[0]
        out[f"objective_{name}_per_entry"] = bd.objective(Vt, W, H).item() / F
        if name == "W":
            out["fit_frames_per_s"] = n_test / (e0.elapsed_time(e1) / 1e3)
        else:
            h.close()
    return out


def study_forgetting(bd, synth, torch, np, dev, seed, n_train=10_000, n_test=2_000,
                     Fs=257, Ks=10, betas=(1, 10, 100, 1000), rs=(0.5, 0.7, 0.9, 1.0),
                     checkpoints=(1, 2, 5, 10, 20), long_checkpoints=(1, 2, 5, 10, 20, 50, 100),
                     long_beta=100, batch_cycles=(1, 2, 5, 10, 20, 50, 100, 200)):
    """The paper's small/medium-set protocol (section 3) on the synthetic
    stand-in: online IS-NMF with warm restarts and one update of h per sample,
    passes over a finite train set in a new order each pass, for a grid of
    minibatch sizes beta and forgetting factors r (rho = r^(beta/N), section
    2.3), against batch MU from the same W(0) (K random train frames, as the
    paper initialises W).  The criterion is the paper's: eq. (1) per matrix
    entry on held-out frames of the same stream, their h fitted (100 updates)
    at the learned W, against the GPU time spent learning.  A run whose W or h
    leaves the positive numbers (a guard flag) is marked unstable.  Minibatches
    of at least long_beta frames take the longer pass schedule (their passes
    are short on the GPU)."""
    V = synth.frames(Fs, Ks, n_train + n_test, seed)
    rng = np.random.default_rng(seed)
    cols = rng.choice(n_train, size=Ks, replace=False)
    W0 = np.ascontiguousarray(V[:, cols].T)                       # (K, F): K train frames
    Vtr = torch.from_numpy(np.ascontiguousarray(V[:, :n_train].T)).to(dev)
    Vte = torch.from_numpy(np.ascontiguousarray(V[:, n_train:].T)).to(dev)
    W0t = torch.from_numpy(W0).to(dev)
    P = max(max(checkpoints), max(long_checkpoints))
    perm = torch.from_numpy(np.stack([rng.permutation(n_train) for _ in range(P)])
                            .astype(np.int32)).to(dev)

    def heldout(W):
        g = bd.OnlineISNMF(W.contiguous(), n_test, inner_iters=100)
        H = torch.empty((n_test, Ks), dtype=torch.float32, device=dev)
        g.fit(Vte, H)
        val = bd.objective(Vte, g.get()[0], H).item() / Fs
        g.close()
        return val

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    out = {"study": "forgetting factor and minibatch size (section 3 protocol, synthetic)",
           "F": Fs, "K": Ks, "train_frames": n_train, "test_frames": n_test,
           "inner_iters": 1, "restarts": "warm", "init": "K random train frames",
           "heldout_W0_per_entry": heldout(W0t), "floor_per_entry": 0.5772156649015329,
           "online": {}, "batch": []}
    for beta in betas:
        for r in rs:
            rho = bd.forgetting_rho(r, beta, n_train)
            g = bd.OnlineISNMF(W0t, beta, inner_iters=1, warm=True, rho=rho)
            H = torch.ones((n_train, Ks), dtype=torch.float32, device=dev)
            pts, done, ms = [], 0, 0.0
            for c in (long_checkpoints if beta >= long_beta else checkpoints):
                torch.cuda.synchronize()
                e0.record()
                g.run_passes(Vtr, perm[done:c].contiguous(), beta, H)
                e1.record()
                torch.cuda.synchronize()
                ms += e0.elapsed_time(e1)
                done = c
                if g.status() != 0:
                    pts.append([c, round(ms, 2), None])
                    break
                pts.append([c, round(ms, 2), heldout(g.get()[0])])
            out["online"][f"beta={beta},r={r}"] = {"rho": rho, "stable": g.status() == 0,
                                                   "passes_ms_heldout": pts}
            g.close()
    W = W0t.clone()
    H = torch.ones((n_train, Ks), dtype=torch.float32, device=dev)
    done, ms = 0, 0.0
    for c in batch_cycles:
        torch.cuda.synchronize()
        e0.record()
        bd.batch_mu(Vtr, W, H, c - done, trace=False)
        e1.record()
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        done = c
        out["batch"].append([c, round(ms, 2), heldout(W)])
    return out


def bench_served(bd, synth, torch, np, dev, S, n_chunks, duration_s, threads, seed0,
                 tune="latency"):
    """Continuous batching: S sessions (F in {257,513}, K in {32,64}, BF16
    products), chunks of U[1,512] frames.  Capacity with every chunk queued at
    once, then Poisson arrivals at 50% and 90% of it: p50/p99 chunk latency.
    tune: kernel variants timed at four mean chunks, a lightly loaded step
    ("latency"), or at a whole served step ("throughput", capacity only)."""
    rng = np.random.default_rng(seed0)
    Fs = rng.choice([257, 513], size=S)
    Ks = rng.choice([32, 64], size=S)
    pool_n = 16384
    pools = {}
    for Fi in (257, 513):
        V = synth.frames(Fi, 50, pool_n, seed0 + Fi, threads=threads)
        pools[Fi] = torch.from_numpy(np.ascontiguousarray(V.T)).to(dev)
    # kernel variant per shape, timed at four mean chunks (latency: one chunk
    # alone would pick the one-frame-per-workgroup VALU variant, which halves
    # the capacity) or at a served step's size: all sessions of a shape with a
    # mean chunk each
    variants = {}
    for Fi in (257, 513):
        for Ki in (32, 64):
            nb = 1024 if tune == "latency" else int(np.sum((Fs == Fi) & (Ks == Ki))) * 256
            bd.autotune(Fi, Ki, max(nb, 256), precision="bf16", trials=2)
            variants[f"{Fi}x{Ki}"] = list(bd.tune_get(Fi, Ki, "bf16"))
    hs = [bd.OnlineISNMF(torch.from_numpy(np.ascontiguousarray(
        synth.initial_dictionary(int(Fs[i]), int(Ks[i]), seed0 + i).T)).to(dev), 512,
        precision="bf16") for i in range(S)]

    def chunk(i, L):
        o = int(rng.integers(0, pool_n - L))
        return pools[int(Fs[i])][o:o + L]

    def run(arrivals, sess, lens):
        srv = bd.Server(max_sessions=S, max_per_step=S, max_frames=1 << 16, inflight=2)
        ids = [srv.open(h) for h in hs]
        loss = torch.zeros(S, dtype=torch.float64, device=dev)   # each session's running loss
        for i, sid in enumerate(ids):
            srv.set_loss(sid, loss[i:i + 1])
        chunks = [chunk(int(sx), int(L)) for sx, L in zip(sess, lens)]
        t0 = bd.Server.clock()
        k = 0
        n = len(arrivals)
        while k < n:
            now = bd.Server.clock() - t0
            while k < n and arrivals[k] <= now:
                srv.submit(ids[int(sess[k])], chunks[k], t0 + arrivals[k])
                k += 1
            srv.pump()
        srv.drain()
        r = srv.results(1 << 20)
        lat = (r["done"] - r["arrival"]) * 1e3
        span = r["done"].max() - (t0 + arrivals[0])
        steps, frames = srv.stats()
        srv.close()
        return {"frames_per_s": frames / span, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "chunks": int(n), "steps": steps}

    lens = rng.integers(1, 513, size=n_chunks)
    sess = rng.integers(0, S, size=n_chunks)
    cap = run(np.zeros(n_chunks), sess, lens)
    out = {"sessions": S, "precision": "bf16", "chunk_frames": "U[1,512]", "tuned_for": tune,
           "variants": variants, "capacity": cap}
    for load in ((0.5, 0.9) if tune == "latency" else ()):
        rate = load * cap["frames_per_s"] / lens.mean()          # chunks per second
        n = max(64, int(rate * duration_s))
        l2 = rng.integers(1, 513, size=n)
        s2 = rng.integers(0, S, size=n)
        arr = np.cumsum(rng.exponential(1.0 / rate, size=n))
        arr -= arr[0]
        out[f"load_{int(load * 100)}"] = run(arr, s2, l2)
    for h in hs:
        h.close()
    bd.tune_clear()
    return out


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
    ap.add_argument("--accuracy-steps", type=int, default=CHECKPOINTS[-1],
                    help="minibatches the oracle runs for the accuracy checkpoints "
                         "(default: the whole pass; the oracle part is untimed)")
    ap.add_argument("--batch-mu-frames", type=int, default=100_000)
    ap.add_argument("--batch-mu-cycles", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--seed", type=int, default=2011)
    ap.add_argument("--batch-streams", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=8)
    ap.add_argument("--serve-sessions", type=int, default=1024)
    ap.add_argument("--serve-chunks", type=int, default=4096)
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--no-forms", action="store_true", help="skip the batched and served forms")
    ap.add_argument("--only", default="",
                    help="comma-separated forms to run besides the timed pass (bf16, fp16, plain, "
                         "batch_mu, multipass, batched_uniform, batched_uniform_fp32, "
                         "batched_mixed, served, served_throughput); default all")
    ap.add_argument("--study", default="", choices=["", "forgetting"],
                    help="run a study instead of the benchmark: 'forgetting' is the paper's "
                         "(beta, r) protocol of section 3 on synthetic frames (one JSON line)")
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
    if args.study == "forgetting":
        print(json.dumps(study_forgetting(bd, synth, torch, np, dev, args.seed)), flush=True)
        return 0
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

    # pick the FP32 fit variant for this shape (MFMA tile or VALU), then warm up
    tuned_v, tuned_us = bd.autotune(F, K, B, precision="fp32", inner_iters=ITERS, trials=20)
    nw, cpw, wg = bd.tune_get(F, K, "fp32")
    kind, kname = fit_kernel_name(nw, cpw, 52, wg)
    print(f"[bench] autotuned FP32 fit: {kname} ({tuned_us:.1f} us per launch)", file=sys.stderr,
          flush=True)
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
    print(f"[bench] fused FP32: {steps} steps, {ms:.1f} ms, {fps:.4g} frames/s", file=sys.stderr,
          flush=True)
    heldout = bench_heldout(bd, synth, torch, np, g, Wt, dev, args.seed, N)
    g.close()
    print(f"[bench] held-out: {heldout}", file=sys.stderr, flush=True)

    # roofline of the fit kernel: HIP events around every fit launch of the same pass
    g = bd.OnlineISNMF(Wt, B, inner_iters=ITERS)
    g.set_timing(True, steps)
    g.run_pass(Vt[:nframes], B)
    launches, fit_ms = g.timing()
    g.close()
    fit_flops = fit_flops_per_frame(F, K, ITERS) * nframes
    achieved = fit_flops / (fit_ms / 1e3)
    traffic = TRAFFIC.get((kname, _src_hash(kind)))
    peak = PEAK_FP32_VECTOR if kind == "valu" else PEAK_FP32_MFMA
    roofline = {"bound": "alu" if kind == "valu" else "mfma", "achieved": achieved / 1e12,
                "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic, "kernel": kname, "launches": launches,
                "avg_launch_us": fit_ms * 1e3 / max(launches, 1),
                "flops_per_launch": fit_flops_per_frame(F, K, ITERS) * B}
    if kind == "valu":
        # one frame per workgroup: b = 128 workgroups on 128 of the 256 CUs
        roofline["peak_unpacked_fp32"] = PEAK_FP32_VALU_UNPACKED / 1e12
        roofline["cus_used"] = min(B, 256)

    # precision forms: BF16 / FP16 products, same stream prefix, each on the fit
    # variant the autotuner picks for one minibatch
    form_variants = {}

    def time_form(precision, nsteps):
        bd.autotune(F, K, B, precision=precision, inner_iters=ITERS, trials=10)
        form_variants[precision] = bd.tune_get(F, K, precision)
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

    only = set(x for x in args.only.split(",") if x)

    def want(name):
        return not only or name in only

    f_steps = max(1, min(args.form_steps, steps))
    forms = {p: {"value": time_form(p, f_steps), "unit": "frames/s", "steps": f_steps}
             for p in ("bf16", "fp16") if want(p)}
    for p in forms:
        forms[p]["variant"] = list(form_variants[p])

    # the plain FP32 path (one op per launch) over a prefix, same shapes
    plain_fps = None
    p_steps = max(1, min(args.plain_steps, steps))
    if want("plain"):
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

    if want("batch_mu"):
        forms["batch_mu"] = bench_batch_mu(bd, torch, np, Vt, Wt, min(N, args.batch_mu_frames),
                                           args.batch_mu_cycles)
        print(f"[bench] batch MU: {forms['batch_mu']}", file=sys.stderr, flush=True)
    if want("multipass"):
        forms["multipass"] = bench_multipass(bd, torch, np, Vt, Wt, min(N, 65536), 3,
                                             args.seed + 7)
        print(f"[bench] multipass: {forms['multipass']['value']:.4g} frames/s", file=sys.stderr,
              flush=True)

    if not args.no_forms:
        thr = cpu_threads()
        if want("batched_uniform"):
            forms["batched_uniform"] = bench_batched(bd, synth, torch, np, dev, args.batch_streams,
                                                     args.batch_steps, thr, False, 70000)
            print(f"[bench] batched uniform: {forms['batched_uniform']['value']:.4g} frames/s",
                  file=sys.stderr, flush=True)
        if want("batched_uniform_fp32"):
            # the roofline run in the metric's own arithmetic: FP32 products
            forms["batched_uniform_fp32"] = bench_batched(bd, synth, torch, np, dev,
                                                          args.batch_streams, args.batch_steps,
                                                          thr, False, 70000, precision="fp32")
            print(f"[bench] batched uniform FP32: {forms['batched_uniform_fp32']}",
                  file=sys.stderr, flush=True)
        if want("batched_mixed"):
            forms["batched_mixed"] = bench_batched(bd, synth, torch, np, dev, args.batch_streams,
                                                   max(2, args.batch_steps // 2), thr, True, 80000)
            print(f"[bench] batched mixed: {forms['batched_mixed']['value']:.4g} frames/s",
                  file=sys.stderr, flush=True)
        if want("served"):
            forms["served"] = bench_served(bd, synth, torch, np, dev, args.serve_sessions,
                                           args.serve_chunks, args.serve_seconds, thr, 90000)
            print(f"[bench] served: {forms['served']}", file=sys.stderr, flush=True)
        if want("served_throughput"):
            forms["served_throughput"] = bench_served(bd, synth, torch, np, dev,
                                                      args.serve_sessions, args.serve_chunks,
                                                      args.serve_seconds, thr, 90000,
                                                      tune="throughput")
            print(f"[bench] served (throughput variants): {forms['served_throughput']}",
                  file=sys.stderr, flush=True)

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
                               f"N={nframes} frames b={B} I={ITERS}, fused FP32 ({kname})",
                   "F": F, "K": K, "b": B, "inner_iters": ITERS, "frames": nframes,
                   "fit_variant": kname,
                   "generator": "V=(W_true H_true)*E, W_true~Gamma(0.5), H_true~Gamma(0.3), "
                                "E~Exp(1), seeded PCG64"},
        "roofline": roofline,
        "plain_fp32": {"value": plain_fps, "unit": "frames/s", "steps": p_steps,
                       "speedup_fused": fps / plain_fps if plain_fps else None},
        "online_loss_per_entry": online_loss,
        "heldout": heldout,
        "forms": forms,
    }
    if not args.no_cpu:
        snaps = {}
        out["cpu_baseline"] = cpu_baseline(V, W0, args.cpu_seconds, snaps, args.accuracy_steps)
        out["accuracy"] = form_accuracy(bd, torch, np, Vt, Wt, snaps, (nw, cpw, wg),
                                       form_variants)
        print(f"[bench] accuracy vs the FP64 oracle: {out['accuracy']}", file=sys.stderr,
              flush=True)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
