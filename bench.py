#!/usr/bin/env python3
"""Benchmark of the factored extrinsic likelihood on one MI355X.

Default workload (the headline configuration): 3 detectors, 21 modes (l <= 4),
Q pregridded at 32768 Hz over +-0.1 s (6554 samples per mode and detector),
network SNR 600, 1e6 prior extrinsic samples.  One step = the whole path over
the batch: every sample's lnL (written out) and the log-sum-exp into ln Z and
n_eff.  `value` is the FP64 path's lnL evaluations per second (every lnL
within 1e-9 relative of the FP64 oracle); the mixed path is reported beside it
with its error statement.

    python bench.py [--steps K] [--warmup W] [--extras] [--no-cpu]

Prints ONE JSON line.  --gpus N > 1 exits: this library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "extrinsic lnL evals/sec (+ grad evals/sec) at |ΔlnL|≤1e-3 vs FP64 oracle"
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector (256 CUs x 2.4 GHz x 128 flop/clk)
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector, packed (dual-issue) instructions
# The build keeps packed FP32 instructions out of its code, so the FP32 pass's
# attainable vector peak is the unpacked rate, the same as FP64's.
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def survey_flops_per_sample(K, M):
    """Algorithmic flops of one lnL evaluation, counted on the method's own
    Hermitian/symmetric-reduced forms (P = M(M+1)/2 mode pairs):
    40 (sky frame) + 57 K (antenna, delay, stencil weights) + 10 M (harmonics)
    + 6 K M (coefficients x F Y) + 20 K M (Lagrange read and data term)
    + 8 K P (the two quadratic forms) + P.  Transcendentals not counted."""
    P = M * (M + 1) // 2
    return 40 + 57 * K + 10 * M + 6 * K * M + 20 * K * M + 8 * K * P + P


def lclass(lmax):
    return 2 if lmax <= 2 else (3 if lmax <= 3 else (4 if lmax <= 4 else 8))


def basis_count(L):
    NI = 2 * L
    return (NI + 1) + L * 2 * (NI + 1) + L * 2 * NI


def flops_per_sample(K, M, lmax):
    """Flops of one lnL evaluation as this library computes it (FMA = 2; the
    model-norm term as the harmonic-basis contraction), transcendentals (5
    sincos) not included.  Reported beside the algorithmic count."""
    L = lclass(lmax)
    NI = 2 * L
    B = basis_count(L)
    sky = 58
    per_det = 49 + 3 + 11               # antenna, delay + stencil; data combine; norm weights
    harm = 6 * NI + 12 * L + M * (2 * L + 4)
    data = 24 * M * K
    quad = B * (6 * K + 2)
    return sky + per_det * K + harm + data + quad + 5


def bytes_per_sample(weighted=False, write_lnL=True):
    return 56 + (8 if weighted else 0) + (8 if write_lnL else 0)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_tiles_fp64_3det_21modes_1e6_hbm_traffic.txt")
# The likelihood kernel's device code and build flags: a committed counter
# summary stays valid while these are unchanged (host-side launch logic lives
# in rift_ile.hip, and the profiling command fixes the launch shape).
KERNEL_SOURCES = ["paper_2609_37393_amd/csrc/ile_device.h", "paper_2609_37393_amd/csrc/ile_kernels.h",
                  "paper_2609_37393_amd/csrc/ile_grad.h", "paper_2609_37393_amd/csrc/inst.hip",
                  "paper_2609_37393_amd/build.py"]


def kernel_sources_sha256():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def bench_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, each calibrated on a plain copy of
    known size), or None when the kernel sources changed since it was taken."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith(" "):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_sources_sha256") != kernel_sources_sha256():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


WARM_S = 0.3


def warm_up(fn, warmup, torch, min_s=0.3):
    """W untimed steps, then more of the same until at least `min_s` seconds of
    GPU work have run: the clocks settle only after ~0.1 s of sustained load,
    so a short warm-up would time the kernels below their steady state."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < min_s:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()


def c2_inputs(synth, n):
    pt = synth.make_point(3, 21, 6554, 32768.0, 600.0, 2)
    th = synth.prior_samples(n, 2)
    return pt, th


def run_path(ile, torch, pt, tht, precision, steps, warmup, tune, variants=True, config=None):
    n = tht.shape[1]
    plan = ile.Plan([pt], [n], precision=precision)
    if config is not None:
        plan.config = config
    elif tune:
        plan.tune(tht)
    lnl = torch.empty(n, dtype=torch.float64, device="cuda")
    z = torch.empty(1, dtype=torch.float64, device="cuda")
    ne = torch.empty(1, dtype=torch.float64, device="cuda")
    err = torch.empty(1, dtype=torch.float64, device="cuda")

    def step():
        plan.lnZ(tht, lnZ_out=z, neff_out=ne, lnL_out=lnl, err_out=err)

    # the tuned shape with and without arrival-time binning (context only)
    variants_out = {}
    base = plan.config
    for srt in ((0, 1) if variants else ()):
        cfg = dict(base)
        cfg["sort"] = srt
        plan.config = cfg
        sec_v, _ = time_steps(step, max(3, steps // 5), 2, torch)
        plan.profile(True)
        step()
        kms_v, nl = plan.profile_read()
        plan.profile(False)
        variants_out[f"sort{srt}"] = {"ms_per_step": 1e3 * sec_v / max(3, steps // 5), "kernel_ms": kms_v / max(1, nl)}
    plan.config = base
    warm_up(step, warmup, torch, WARM_S)
    plan.profile(True)
    secs, wall = time_steps(step, steps, 0, torch)
    kms, launches = plan.profile_read()
    plan.profile(False)
    out = {
        "secs": secs,
        "wall": wall,
        "kernel_ms_avg": kms / max(1, launches),
        "launches": launches,
        "lnZ": z.item(),
        "neff": ne.item(),
        "lnZ_err_bound": err.item(),
        "config": plan.config,
        "refined": plan.refined() if precision == "mixed" else 0,
        "variants": variants_out,
        "lnL": lnl,
    }
    plan.close()
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pt, th, gpu_lnL, budget_s=12.0):
    """The FP64 oracle as it stands, on this host, for about `budget_s` seconds:
    consecutive chunks of the same samples, wrapping round to the start if the
    whole workload finishes early.  Parity is taken on the first pass."""
    import oracle

    oracle.build(force=False)
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = th.shape[1]
    done = 0
    first = []
    chunk = 50000
    t0 = time.perf_counter()
    pos = 0
    while time.perf_counter() - t0 < budget_s:
        c = min(chunk, n - pos)
        out = oracle.lnL(pt, th[:, pos:pos + c], nthreads=nthreads)
        if done < n:
            first.append(out)
        done += c
        pos = (pos + c) % n
    el = time.perf_counter() - t0
    # one thread, on a shorter prefix of the same samples
    t1 = time.perf_counter()
    done1, pos1 = 0, 0
    while time.perf_counter() - t1 < budget_s / 4:
        c = min(5000, n - pos1)
        oracle.lnL(pt, th[:, pos1:pos1 + c], nthreads=1)
        done1 += c
        pos1 = (pos1 + c) % n
    el1 = time.perf_counter() - t1
    l_or = np.concatenate(first)[:n]
    m = l_or.size
    d = np.abs(gpu_lnL[:m] - l_or)
    passes = done / n
    return {
        "value": done / el,
        "unit": "lnL evals/s",
        "cores": nthreads,
        "kind": "oracle",
        "sample": f"{done} evaluations ({passes:.2f} passes over the {n} samples of the same workload) in {el:.1f} s",
        "single_thread": {"value": done1 / el1, "sample": f"{done1} evaluations in {el1:.1f} s, 1 thread"},
        "cpu_model": _cpu_model(),
    }, {
        "samples": int(m),
        "max_abs_dlnL": float(d.max()),
        "max_rel_dlnL": float((d / np.maximum(1.0, np.abs(l_or))).max()),
    }


# ---------------------------------------------------------------------------
# Extra configurations
# ---------------------------------------------------------------------------
def _c1_run(ile, synth, torch, steps, n):
    pt = synth.make_point(2, 2, 410, 4096.0, 20.0, 1)
    th = torch.as_tensor(synth.prior_samples(n, 1), device="cuda").contiguous()
    r = run_path(ile, torch, pt, th, "fp64", steps, 3, tune=False, variants=False)
    ks = r["kernel_ms_avg"] / 1e3
    # against its own roofline: 64 algorithmic HBM bytes per sample (theta in,
    # lnL out) and the FP64 vector peak
    res = {"n": n, "lnL_evals_per_s": n * steps / r["secs"], "ms_per_step": 1e3 * r["secs"] / steps,
           "kernel_ms": r["kernel_ms_avg"],
           "hbm_frac": 64.0 * n / ks / (PEAK_HBM_GBS * 1e9),
           "alu_frac": survey_flops_per_sample(2, 2) * n / ks / (PEAK_FP64_TFLOPS * 1e12)}
    # the same step captured into a HIP graph and replayed (launch overhead)
    plan = ile.Plan([pt], [n])
    z = torch.empty(1, dtype=torch.float64, device="cuda")
    lnl = torch.empty(n, dtype=torch.float64, device="cuda")
    plan.lnZ(th, lnZ_out=z, lnL_out=lnl)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(16):
            plan.lnZ(th, lnZ_out=z, lnL_out=lnl)
    secs, _ = time_steps(g.replay, max(3, steps // 4), 2, torch)
    res["graph16"] = {"lnL_evals_per_s": 16 * n * max(3, steps // 4) / secs,
                      "ms_per_step": 1e3 * secs / (16 * max(3, steps // 4))}
    plan.close()
    return res


def extra_c1(ile, synth, torch, steps, cpu=True):
    """2 detectors, (2,+-2), 410 samples at 4096 Hz, SNR 20, 1e4 prior samples
    (launch-bound at this size; also reported as 16 steps in one graph)."""
    return _c1_run(ile, synth, torch, steps, 10_000)


def extra_c1_big(ile, synth, torch, steps, cpu=True):
    """The C1 point at 1e7 samples (steady state for its roofline)."""
    return _c1_run(ile, synth, torch, steps, 10_000_000)


def extra_c3(ile, synth, torch, steps, n_points=512, per_point=200_000, cpu=True):
    """512 points, M ~ U{2,4,9,16,21}, n_t ~ U[400, 6554] at 32768 Hz, K = 3,
    SNR log-U[20, 1000], 2e5 samples each; one graph-captured launch set."""
    rng = np.random.default_rng(3)
    net = synth.network(3, 3)
    base = {M: synth.make_point(3, M, 6554, 32768.0, 100.0, 300 + M, net=net) for M in (2, 4, 9, 16, 21)}
    pts, counts = [], []
    for p in range(n_points):
        M = int(rng.choice([2, 4, 9, 16, 21]))
        n_t = int(rng.integers(400, 6555))
        snr = 20.0 * 50.0 ** rng.uniform()
        b = base[M]
        c0 = (6554 - n_t) // 2
        pt = dict(b)
        pt["Q"] = b["Q"][:, :, c0:c0 + n_t] * (snr / 100.0)
        pt["U"] = b["U"] * (snr / 100.0) ** 2
        pt["V"] = b["V"] * (snr / 100.0) ** 2
        pt["t0"] = b["t0"] + c0 * b["dt"]
        pts.append(pt)
        counts.append(per_point)
    N = n_points * per_point
    log(f"c3: {n_points} points, {N} samples")
    th = torch.empty((7, N), dtype=torch.float64, device="cuda")
    chunk = 4_000_000
    for s in range(0, N, chunk):
        c = min(chunk, N - s)
        th[:, s:s + c] = torch.as_tensor(synth.prior_samples(c, 1000 + s // chunk), device="cuda")
    res = {}
    M_of = [int(p["lm"].shape[0]) for p in pts]
    flops = sum(survey_flops_per_sample(3, M) * c for M, c in zip(M_of, counts))
    for prec in ("fp64", "mixed"):
        plan = ile.Plan(pts, counts, precision=prec)
        choice = plan.tune(th)
        z = torch.empty(n_points, dtype=torch.float64, device="cuda")
        ne = torch.empty(n_points, dtype=torch.float64, device="cuda")
        plan.lnZ(th, lnZ_out=z, neff_out=ne)
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            plan.lnZ(th, lnZ_out=z, neff_out=ne)
        secs, _ = time_steps(g.replay, steps, 1, torch)
        res[prec] = {"lnL_evals_per_s": N * steps / secs, "ms_per_step": 1e3 * secs / steps,
                     "tuned_config": plan.config, "tuner_choice": choice,
                     "alu_frac": flops * steps / secs / (1e12 * (PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_UNPACKED_TFLOPS))}
        if prec == "mixed":
            res[prec]["refined"] = plan.refined()
        plan.close()
    return res


def seed_near_peak(ile, torch, synth, pt, sig, n=200_000, rounds=(100.0, 30.0, 10.0, 3.0, 1.0)):
    """Seeding of the chains (not timed): the best of n prior draws, then the
    best of n draws around the current best at shrinking widths (rounds x
    sig), every lnL from the library itself."""
    th = synth.prior_samples(n, 4)
    best = th[:, int(torch.argmax(ile.lnL(pt, th)).item())]
    for r, w in enumerate(rounds):
        th = synth.perturbed_samples(best, np.asarray(sig) * w, n, 40 + r)
        th = np.concatenate([best[:, None], th], axis=1)
        best = th[:, int(torch.argmax(ile.lnL(pt, th)).item())]
    return best


def extra_c4(ile, synth, torch, steps, chains=4096, nsteps=64, cpu=True):
    """4096 chains x 64 leapfrog-style gradient evaluations (K = 3, 9 modes,
    SNR 600), the 64 steps captured into one graph."""
    pt = synth.make_point(3, 9, 6554, 32768.0, 600.0, 4)
    sig = np.array([1e-3, 1e-3, 5e-3, 5e-3, 5e-3, 3e-6, 5e-3])
    th0 = seed_near_peak(ile, torch, synth, pt, sig)
    start = synth.perturbed_samples(th0, sig, chains, 5)
    plan = ile.Plan([pt], [chains])
    q = torch.as_tensor(start, device="cuda").contiguous()
    c = q.clone()
    c[3] = torch.cos(q[3])
    c[6] = torch.log(q[6])
    cq = c.clone()
    p = torch.zeros_like(c)
    eps = 0.1
    step_q = eps * sig * sig  # eps sigma^2 per parameter (mass diag(sigma^-2))
    g = torch.empty_like(q)

    # the chain moves in (.., cos incl, .., .., ln dist), the coordinates of
    # the gradient, and hands them to the library as they are; per leapfrog
    # step one launch per momentum half-step and one drift launch (with the
    # reflecting boundary of cos incl)
    def run():
        plan.grad(0, cq, grad_out=g, coords="sampler")
        for _ in range(nsteps - 1):
            p.add_(g, alpha=0.5 * eps)
            ile.leapfrog_drift(cq, p, step_q)
            plan.grad(0, cq, grad_out=g, coords="sampler")
            p.add_(g, alpha=0.5 * eps)

    run()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        run()
    secs, _ = time_steps(graph.replay, steps, 1, torch)
    # kernel-only rate from a separate eager pass with events
    plan.profile(True)
    run()
    kms, launches = plan.profile_read()
    plan.profile(False)
    finite = float(torch.isfinite(g).all(dim=0).double().mean().item())
    plan.close()
    evals = chains * nsteps
    res = {"grad_evals_per_s": evals * steps / secs, "ms_per_graph": 1e3 * secs / steps,
           "kernel_ms_avg": kms / max(1, launches), "chains": chains, "steps_per_chain": nsteps,
           "finite_fraction_after_64_steps": finite,
           "workload": "3 detectors, 9 modes (l<=3), Q 6554 samples at 32768 Hz, SNR 600; "
                       "4096 chains x 64 gradient evaluations in one graph"}
    if cpu:
        import oracle

        t0 = time.perf_counter()
        done = 0
        while time.perf_counter() - t0 < 3.0:
            oracle.grad(pt, start[:, :1024])
            done += 1024
        res["cpu_oracle_grad_evals_per_s"] = done / (time.perf_counter() - t0)
    return res


def extra_c5(ile, synth, torch, steps, cpu=True):
    """K = 5 (two 40-km-class), 21 modes, 13108 samples at 32768 Hz, SNR 1000:
    1e7 prior samples in 10 chunks of 1e6 (ln Z merged), FP64 and mixed
    precision, with the merged ln Z of both against the FP64 oracle's over the
    same 1e7 samples."""
    net = synth.network(5, 5)
    pt = synth.make_point(5, 21, 13108, 32768.0, 1000.0, 5, net=net)
    n = 10_000_000
    ths = [synth.prior_samples(2_000_000, 500 + j) for j in range(5)]
    th = torch.empty((7, n), dtype=torch.float64, device="cuda")
    for j in range(5):
        th[:, j * 2_000_000:(j + 1) * 2_000_000] = torch.as_tensor(ths[j], device="cuda")
    res = {"workload": "5 detectors, 21 modes (l<=4), Q 13108 samples at 32768 Hz, SNR 1000, "
                       "1e7 prior samples in 10 chunks of 1e6"}
    chunks = [1_000_000] * 10
    fps = survey_flops_per_sample(5, 21)
    zs = {}
    for prec in ("fp64", "mixed"):
        # ten chunks as ten "points" sharing the tables: one launch, then an LSE merge
        plan = ile.Plan([pt] * 10, chunks, precision=prec)
        plan.tune(th)
        z = torch.empty(10, dtype=torch.float64, device="cuda")
        err = torch.empty(10, dtype=torch.float64, device="cuda")
        plan.lnZ(th, lnZ_out=z, err_out=err)
        secs, _ = time_steps(lambda: plan.lnZ(th, lnZ_out=z, err_out=err), steps, 1, torch)
        plan.profile(True)
        plan.lnZ(th, lnZ_out=z, err_out=err)
        kms, nl = plan.profile_read()
        plan.profile(False)
        zz = z.cpu().numpy()
        m = zz.max()
        zs[prec] = float(m + math.log(np.mean(np.exp(zz - m))))
        peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_UNPACKED_TFLOPS
        res[prec] = {"lnL_evals_per_s": n * steps / secs, "ms_per_step": 1e3 * secs / steps,
                     "kernel_ms": kms / max(1, nl), "lnZ": zs[prec], "tuned_config": plan.config,
                     "alu_frac": fps * n / (kms / max(1, nl) / 1e3) / (1e12 * peak)}
        if prec == "mixed":
            res[prec]["refined"] = plan.refined()
            res[prec]["lnZ_err_bound"] = float(err.max().item())
        plan.close()
    res["speedup_mixed_vs_fp64"] = res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"]
    res["dlnZ_mixed_vs_fp64"] = abs(zs["mixed"] - zs["fp64"])
    if cpu:
        import oracle

        t0 = time.perf_counter()
        l_or = np.concatenate([oracle.lnL(pt, t) for t in ths])
        zc = [oracle.lnZ(l_or[j * 1_000_000:(j + 1) * 1_000_000])[0] for j in range(10)]
        m = max(zc)
        z_or = m + math.log(np.mean(np.exp(np.array(zc) - m)))
        res["oracle_lnZ"] = z_or
        res["dlnZ_fp64_vs_oracle"] = abs(zs["fp64"] - z_or)
        res["dlnZ_mixed_vs_oracle"] = abs(zs["mixed"] - z_or)
        res["oracle_s"] = time.perf_counter() - t0
    del th
    return res


def extra_c5_batch(ile, synth, torch, steps, n_batch=64, per_point=200_000, cpu=True):
    """64 intrinsic points of the 5-detector network (16 points at 4 SNR
    scalings, 400 to 1000), 2e5 samples each, with the mixed-precision ln Z
    difference from the FP64 path and the largest reported bound."""
    net = synth.network(5, 5)
    fps = survey_flops_per_sample(5, 21)
    base = [synth.make_point(5, 21, 13108, 32768.0, 1000.0, 900 + b, net=net) for b in range(n_batch // 4)]
    pts = []
    for b in base:
        for scale in (1.0, 0.8, 0.6, 0.4):
            q = dict(b)
            q["Q"] = b["Q"] * scale
            q["U"] = b["U"] * scale * scale
            q["V"] = b["V"] * scale * scale
            pts.append(q)
    counts = [per_point] * len(pts)
    N = per_point * len(pts)
    thb = torch.empty((7, N), dtype=torch.float64, device="cuda")
    for i in range(len(pts)):
        thb[:, i * per_point:(i + 1) * per_point] = torch.as_tensor(synth.prior_samples(per_point, 2000 + i),
                                                                    device="cuda")
    zb = {}
    batch = {}
    for prec in ("fp64", "mixed"):
        plan = ile.Plan(pts, counts, precision=prec)
        plan.tune(thb)
        z = torch.empty(len(pts), dtype=torch.float64, device="cuda")
        err = torch.empty(len(pts), dtype=torch.float64, device="cuda")
        plan.lnZ(thb, lnZ_out=z, err_out=err)
        secs, _ = time_steps(lambda: plan.lnZ(thb, lnZ_out=z, err_out=err), steps, 1, torch)
        zb[prec] = z.cpu().numpy()
        peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_UNPACKED_TFLOPS
        batch[prec] = {"lnL_evals_per_s": N * steps / secs, "ms_per_step": 1e3 * secs / steps,
                       "tuned_config": plan.config, "alu_frac": fps * N * steps / secs / (1e12 * peak)}
        if prec == "mixed":
            batch[prec]["max_lnZ_err_bound"] = float(err.max().item())
            batch[prec]["refined"] = plan.refined()
        plan.close()
    batch["max_abs_dlnZ_mixed_vs_fp64"] = float(np.abs(zb["mixed"] - zb["fp64"]).max())
    batch["points"] = len(pts)
    batch["samples_per_point"] = per_point
    return batch


def wide_flops_per_sample(K, M, n_a, response):
    """Algorithmic flops of one composite-index lnL evaluation: the static
    count with the mode index widened to A = n_a M (P_A = A(A+1)/2 pairs),
    plus the composite coefficients (rotation: F at five hour angles, ~40
    flops each, the 5x5 complex transform and the phases; arms: the arm
    projections and n_a powers)."""
    A = n_a * M
    P = A * (A + 1) // 2
    if response in ("rotation", "rotation_delay"):
        # with the delay drift: its three harmonics (~20 flops) and, per
        # order-p coefficient, one complex product per drift harmonic (8 flops)
        coef = 5 * 40 + 200 + 40 + (0 if n_a == 5 else 20 + 8 * 3 * 7 + (0 if n_a == 12 else 8 * (9 + 5 * 9)))
    else:
        coef = 40 + 12 * n_a
    return 40 + 57 * K + 10 * M + K * coef + 6 * K * A + 20 * K * A + 8 * K * P + P


def extra_wide(ile, synth, torch, steps, cpu=True):
    """The generalised response (composite index A = (a, lm)): Earth rotation
    (5 sidereal terms) at widths 20 and 105, rotation with the delay drift to
    orders 1 and 2 (12 and 21 terms) at 4 modes, finite arms (p_max = 3) at
    width 16; 3 detectors, Q 6554 samples at 32768 Hz, SNR 600.  Each call is
    timed whole (the description's upload and the synchronisation
    included)."""
    res = {}
    for name, resp, M, n_a, n in (("rotation_w20", "rotation", 4, 5, 1_000_000),
                                  ("rotation_w105", "rotation", 21, 5, 200_000),
                                  ("rotation_delay_w48", "rotation_delay", 4, 12, 1_000_000),
                                  ("rotation_delay_w84", "rotation_delay", 4, 21, 200_000),
                                  ("arms_w16", "arms", 4, 4, 1_000_000)):
        pt = synth.make_point_wide(3, M, n_a, 6554, 32768.0, 600.0, 60 + M, response=resp)
        dp = ile.DeviceWidePoint.from_dict(pt)
        th = torch.as_tensor(synth.prior_samples(n, 61), device="cuda").contiguous()
        ile.wide_lnZ(dp, th)
        torch.cuda.synchronize()
        reps = max(3, steps // 2)
        t0 = time.perf_counter()
        for _ in range(reps):
            z, _ = ile.wide_lnZ(dp, th)
        torch.cuda.synchronize()
        secs = (time.perf_counter() - t0) / reps
        fl = wide_flops_per_sample(3, M, n_a, resp)
        r = {"response": resp, "modes": M, "terms": n_a, "width": M * n_a, "n_samples": n,
             "lnL_evals_per_s": n / secs, "ms_per_call": 1e3 * secs, "flops_per_sample": fl,
             "alu_frac_of_call": fl * n / secs / (PEAK_FP64_TFLOPS * 1e12), "lnZ": z.item()}
        if cpu:
            import oracle

            k = min(n, 20_000)
            t0 = time.perf_counter()
            oracle.lnL_wide(pt, th[:, :k].cpu().numpy())
            r["cpu_oracle_lnL_evals_per_s"] = k / (time.perf_counter() - t0)
        res[name] = r
        del th, dp
    return res


def extra_dmarg(ile, synth, torch, steps, cpu=True):
    """The headline point (3 detectors, 21 modes, SNR 600, 1e6 prior
    samples) with the likelihood marginalised over distance in the kernel:
    prior p(D) ~ D^2 on [10, 1000] Mpc, a 20-node adaptive Gauss-Hermite rule
    per sample (Eq. (ap:dgh)), then ln Z_d; against the FP64 oracle's ln Z_d
    over the same samples."""
    pt, th = c2_inputs(synth, 1_000_000)
    n = th.shape[1]
    tht = torch.as_tensor(th, device="cuda").contiguous()
    plan = ile.Plan([pt], [n])
    plan.tune(tht)
    z = torch.empty(1, dtype=torch.float64, device="cuda")
    ne = torch.empty(1, dtype=torch.float64, device="cuda")
    ll = torch.empty(n, dtype=torch.float64, device="cuda")

    def step():
        plan.lnZ_dmarg(tht, 10.0, 1000.0, 20, lnZ_out=z, neff_out=ne, lnL_out=ll)

    warm_up(step, 3, torch, WARM_S)
    secs, _ = time_steps(step, steps, 0, torch)
    plan.profile(True)
    step()
    kms, nl = plan.profile_read()
    plan.profile(False)
    fps = survey_flops_per_sample(3, 21) + 20 * 8
    res = {"workload": "3 detectors, 21 modes (l<=4), Q 6554 samples at 32768 Hz, SNR 600, 1e6 prior samples; "
                       "lnL marginalised over distance (p(D) ~ D^2 on [10, 1000] Mpc, 20 Gauss-Hermite nodes)",
           "lnLd_evals_per_s": n * steps / secs, "ms_per_step": 1e3 * secs / steps, "kernel_ms": kms / max(1, nl),
           "flops_per_sample": fps, "alu_frac": fps * n / (kms / max(1, nl) / 1e3) / (PEAK_FP64_TFLOPS * 1e12),
           "lnZd": z.item(), "neff": ne.item(), "launch": plan.config}
    plan.close()
    if cpu:
        import oracle

        t0 = time.perf_counter()
        want = oracle.lnL_dmarg(pt, th, 10.0, 1000.0, 20)
        res["cpu_oracle_lnLd_evals_per_s"] = n / (time.perf_counter() - t0)
        z_or, _ = oracle.lnZ(want)
        res["dlnZd_vs_oracle"] = abs(res["lnZd"] - z_or)
    return res


def extra_pregrid(ile, synth, torch, steps, cpu=True):
    """The Fourier refinement x8 of the native 4096 Hz correlation tables
    (Eq. (q-time-pregrid)) of the headline point (3 detectors x 21 modes, 820
    native samples) and the five-detector point (5 x 21, 1639 samples): time per
    table set, and the oracle's FFT implementation on the host beside it."""
    res = {}
    for name, K, n in (("c2_table", 3, 820), ("c5_table", 5, 1639)):
        pt = synth.make_point(K, 21, n, 4096.0, 600.0, 7 + K)
        q = torch.as_tensor(pt["Q"], device="cuda").contiguous()
        nf = (n - 1) * 8 + 1
        out = torch.empty((K, 21, nf), dtype=torch.complex128, device="cuda")
        step = lambda: ile.pregrid(q, 8, out=out)
        step()
        secs, _ = time_steps(step, steps, 2, torch)
        S = K * 21
        flops = 4.0 * S * nf * n  # a real kernel value times a complex sample: 2 FMAs per (series, fine, native)
        r = {"series": S, "native": n, "refined": nf, "ms_per_call": 1e3 * secs / steps,
             "flops_per_call": flops, "alu_frac": flops / (secs / steps) / (PEAK_FP64_TFLOPS * 1e12)}
        if cpu:
            import oracle

            t0 = time.perf_counter()
            want = oracle.pregrid(pt["Q"], 8)
            r["cpu_oracle_ms"] = 1e3 * (time.perf_counter() - t0)
            r["max_abs_diff_vs_oracle"] = float(np.abs(out.cpu().numpy() - want).max())
            r["max_abs_q"] = float(np.abs(pt["Q"]).max())
        res[name] = r
    return res


def extra_tmarg(ile, synth, torch, steps, cpu=True):
    """The headline point (3 detectors, 21 modes, SNR 600) marginalised over
    geocentric time by the fixed-spacing Simpson rule at the table's rate
    (Eq. (ap:tfixed)): 657 times over the prior's 20 ms, 1e5 samples of the
    other six parameters; against the FP64 oracle on a sample of them."""
    pt = synth.make_point(3, 21, 6554, 32768.0, 600.0, 2)
    n, n_t = 100_000, 657
    h = 0.02 / (n_t - 1)
    th = synth.prior_samples(n, 2)
    tht = torch.as_tensor(th, device="cuda").contiguous()
    plan = ile.Plan([pt], [n])
    z = torch.empty(1, dtype=torch.float64, device="cuda")
    ll = torch.empty(n, dtype=torch.float64, device="cuda")

    def step():
        plan.lnZ_tmarg(tht, -0.01, h, n_t, lnZ_out=z, lnL_out=ll)

    step()
    secs, _ = time_steps(step, max(2, steps // 3), 1, torch)
    per = secs / max(2, steps // 3)
    plan.profile(True)
    step()
    kms, nl = plan.profile_read()
    plan.profile(False)
    plan.close()
    # the model-norm term once, the data term (antenna, stencils, gather, interpolation, coefficients) per time
    fps = survey_flops_per_sample(3, 21) + (n_t - 1) * 3 * (57 + 26 * 21)
    res = {"workload": "3 detectors, 21 modes (l<=4), Q 6554 samples at 32768 Hz, SNR 600; 1e5 samples of the other "
                       "parameters, Simpson rule on 657 times (32768 Hz) over 20 ms",
           "lnLt_evals_per_s": n / per, "data_terms_per_s": n * n_t / per, "ms_per_call": 1e3 * per,
           "kernel_ms": kms / max(1, nl), "flops_per_sample": fps,
           "alu_frac": fps * n / (kms / max(1, nl) / 1e3) / (PEAK_FP64_TFLOPS * 1e12), "lnZt": z.item()}
    if cpu:
        import oracle

        idx = np.random.default_rng(1).choice(n, 300, replace=False)
        t0 = time.perf_counter()
        want = oracle.lnL_tmarg(pt, th[:, idx], -0.01, h, n_t)
        res["cpu_oracle_lnLt_evals_per_s"] = idx.size / (time.perf_counter() - t0)
        res["max_abs_dlnLt_vs_oracle_sampled"] = float(np.nanmax(np.abs(ll.cpu().numpy()[idx] - want)))
    return res


def extra_tband(ile, synth, torch, steps, cpu=True):
    """The headline point (3 detectors, 21 modes, SNR 600) marginalised over
    geocentric time by the band-limited full-window rule (Eq. (ap:tband)):
    64 nodes at 4096 Hz (above the 3400 Hz Nyquist rate of the 1700 Hz band)
    over 15.4 ms, 16 or 64 fine intervals each (1009 or 4033 fine times, 65536
    or 262144 Hz), 1e5 samples of the other six parameters; against the FP64
    oracle on a sample."""
    pt = synth.make_point(3, 21, 6554, 32768.0, 600.0, 2)
    n = 100_000
    th = synth.prior_samples(n, 2)
    tht = torch.as_tensor(th, device="cuda").contiguous()
    plan = ile.Plan([pt], [n])
    z = torch.empty(1, dtype=torch.float64, device="cuda")
    ll = torch.empty(n, dtype=torch.float64, device="cuda")
    res = {"workload": "3 detectors, 21 modes (l<=4), Q 6554 samples at 32768 Hz, SNR 600; 1e5 samples of the other "
                       "parameters, band-limited rule on 64 nodes at 4096 Hz"}
    for M in (16, 64):
        rule = (-0.0077, 1.0 / 4096, 64, M)

        def step():
            plan.lnZ_tband(tht, *rule, lnZ_out=z, lnL_out=ll)

        step()
        k = max(2, steps // 3)
        secs, _ = time_steps(step, k, 1, torch)
        per = secs / k
        plan.profile(True)
        step()
        kms, nl = plan.profile_read()
        plan.profile(False)
        fine = 63 * M + 1
        rest = 1e3 * per - kms / max(1, nl)
        r = {"lnLt_evals_per_s": n / per, "data_terms_per_s": n * 64 / per, "ms_per_call": 1e3 * per,
             "data_pass_kernel_ms": kms / max(1, nl), "reconstruction_and_reduction_ms": rest, "fine_times": fine,
             "reconstruction_flops_per_sample": 2 * fine * 64,
             "reconstruction_tflops": 2 * fine * 64 * n / (rest / 1e3) / 1e12, "lnZt": z.item()}
        if cpu:
            import oracle

            idx = np.random.default_rng(1).choice(n, 200, replace=False)
            t0 = time.perf_counter()
            want = oracle.lnL_tband(pt, th[:, idx], *rule)
            r["cpu_oracle_lnLt_evals_per_s"] = idx.size / (time.perf_counter() - t0)
            r["max_abs_dlnLt_vs_oracle_sampled"] = float(np.nanmax(np.abs(ll.cpu().numpy()[idx] - want)))
        res[f"fine{M}"] = r
    plan.close()
    return res


def extra_erai(ile, synth, torch, steps, cpu=True):
    """The headline point (3 detectors, 21 modes, SNR 600, 1e6 prior samples)
    marginalised jointly over phiref and psi by exact reconstruction
    (Eqs. (ap:angleharm), (ap:nyquist)): 9 data-term and 17 model-norm phases
    per sample, then the exponential on a 32 x 16 and a 64 x 32 grid; against
    the FP64 oracle on a sample."""
    pt, th = c2_inputs(synth, 1_000_000)
    n = th.shape[1]
    tht = torch.as_tensor(th, device="cuda").contiguous()
    plan = ile.Plan([pt], [n])
    z = torch.empty(1, dtype=torch.float64, device="cuda")
    ll = torch.empty(n, dtype=torch.float64, device="cuda")
    res = {"workload": "3 detectors, 21 modes (l<=4), Q 6554 samples at 32768 Hz, SNR 600, 1e6 prior samples; "
                       "lnL marginalised over phiref and psi (9 + 17 sampling phases)"}
    for n_phi, n_psi in ((32, 16), (64, 32)):
        def step():
            plan.lnZ_erai(tht, n_phi, n_psi, lnZ_out=z, lnL_out=ll)

        step()
        k = max(2, steps // 3)
        secs, _ = time_steps(step, k, 1, torch)
        per = secs / k
        plan.profile(True)
        step()
        kms, nl = plan.profile_read()
        plan.profile(False)
        r = {"lnL_evals_per_s": n / per, "ms_per_call": 1e3 * per, "data_pass_kernel_ms": kms / max(1, nl),
             "grid_and_reduction_ms": 1e3 * per - kms / max(1, nl), "exp_per_sample": n_phi * n_psi,
             "lnZ": z.item()}
        if cpu:
            import oracle

            idx = np.random.default_rng(3).choice(n, 200, replace=False)
            t0 = time.perf_counter()
            want = oracle.lnL_erai(pt, th[:, idx], n_phi, n_psi)
            r["cpu_oracle_evals_per_s"] = idx.size / (time.perf_counter() - t0)
            r["max_abs_dlnL_vs_oracle_sampled"] = float(np.nanmax(np.abs(ll.cpu().numpy()[idx] - want)))
        res[f"grid{n_phi}x{n_psi}"] = r
    plan.close()
    return res


def extra_pmarg(ile, synth, torch, steps, cpu=True):
    """The headline point (3 detectors, 21 modes, SNR 600, 1e6 prior
    samples) marginalised over polarisation in the kernel: the periodic
    trapezoid rule on 64 points of q(u) (Eq. (ap:psiexp)), Laplace's method
    (Eq. (ap:psilaplace)) and the stationary-point cells (Eq. (ap:psicells));
    each against the FP64 oracle on a sample."""
    pt, th = c2_inputs(synth, 1_000_000)
    n = th.shape[1]
    tht = torch.as_tensor(th, device="cuda").contiguous()
    plan = ile.Plan([pt], [n])
    z = torch.empty(1, dtype=torch.float64, device="cuda")
    ll = torch.empty(n, dtype=torch.float64, device="cuda")
    res = {"workload": "3 detectors, 21 modes (l<=4), Q 6554 samples at 32768 Hz, SNR 600, 1e6 prior samples; "
                       "lnL marginalised over polarisation"}
    idx = np.random.default_rng(3).choice(n, 300, replace=False)
    for method, npts in (("trapezoid", 64), ("laplace", 0), ("cells", 0)):
        def step():
            plan.lnZ_pmarg(tht, method, npts, lnZ_out=z, lnL_out=ll)

        step()
        secs, _ = time_steps(step, max(3, steps // 2), 1, torch)
        per = secs / max(3, steps // 2)
        plan.profile(True)
        step()
        kms, nl = plan.profile_read()
        plan.profile(False)
        r = {"lnLp_evals_per_s": n / per, "ms_per_step": 1e3 * per, "kernel_ms": kms / max(1, nl), "lnZp": z.item()}
        if cpu:
            import oracle

            t0 = time.perf_counter()
            want = oracle.lnL_pmarg(pt, th[:, idx], method, npts)
            r["cpu_oracle_lnLp_evals_per_s"] = idx.size / (time.perf_counter() - t0)
            r["max_abs_dlnLp_vs_oracle_sampled"] = float(np.nanmax(np.abs(ll.cpu().numpy()[idx] - want)))
        res[method if method != "trapezoid" else f"trapezoid{npts}"] = r
    plan.close()
    return res


def extra_hmc(ile, synth, torch, steps, chains=16384, n_leapfrog=8, cpu=True):
    """Metropolis-adjusted HMC transitions of 16384 chains, 8 leapfrog steps
    each, on the gradient (3 detectors, 9 modes, SNR 100), every transition
    one library call with its random numbers drawn beforehand (not timed)."""
    pt = synth.make_point(3, 9, 6554, 32768.0, 100.0, 44)
    sig = np.array([1e-3, 1e-3, 5e-3, 5e-3, 5e-3, 3e-6, 5e-3])
    box = (-0.01, 0.01, 10.0, 1000.0)
    eps = 0.3
    th0 = seed_near_peak(ile, torch, synth, pt, sig)
    start = synth.perturbed_samples(th0, sig, chains, 6)
    start[3] = np.cos(start[3])
    start[6] = np.log(start[6])
    plan = ile.Plan([pt], [chains])
    c = torch.as_tensor(start, device="cuda").contiguous()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    burn, k = 6, max(10, steps)
    Z = torch.randn((burn + k, 7, chains), dtype=torch.float64, device="cuda", generator=gen)
    U = torch.rand((burn + k, chains), dtype=torch.float64, device="cuda", generator=gen)
    ll = torch.empty(chains, dtype=torch.float64, device="cuda")
    acc = torch.empty(chains, dtype=torch.int32, device="cuda")
    acc_sum = torch.zeros(chains, dtype=torch.int32, device="cuda")
    it = iter(range(burn + k))

    def step():
        i = next(it)
        plan.hmc(0, c, Z[i], U[i], sig, eps, n_leapfrog, box, lnL_out=ll, accepted_out=acc)
        acc_sum.add_(acc)

    for _ in range(burn):  # also warms every launch of the timed step
        step()
    acc_sum.zero_()
    secs, _ = time_steps(step, k, 0, torch)
    plan.profile(True)
    plan.hmc(0, c, Z[0], U[0], sig, eps, n_leapfrog, box, lnL_out=ll, accepted_out=acc)
    kms, nl = plan.profile_read()
    plan.profile(False)
    per = secs / k
    res = {"transitions_per_s": chains / per, "grad_evals_per_s": chains * (n_leapfrog + 1) / per,
           "ms_per_transition": 1e3 * per, "grad_kernel_ms_avg": kms / max(1, nl),
           "acceptance": float(acc_sum.double().mean().item() / k), "chains": chains, "n_leapfrog": n_leapfrog,
           "eps": eps, "mean_lnL": float(ll.mean().item()),
           "workload": "3 detectors, 9 modes (l<=3), Q 6554 samples at 32768 Hz, SNR 100; 16384 chains, "
                       "one Metropolis-adjusted HMC transition (8 leapfrog steps) per call",
           "note": "rate excludes drawing the random numbers; per transition 9 gradient launches and 9 "
                   "elementwise launches (each the kicks and drift between two gradients)"}
    if cpu:
        import oracle

        cs = c[:, :256].cpu().numpy()
        z = Z[0, :, :256].cpu().numpy()
        u = U[0, :256].cpu().numpy()
        t0 = time.perf_counter()
        done = 0
        while time.perf_counter() - t0 < 3.0:
            oracle.hmc_step(pt, cs, z, u, sig, eps, n_leapfrog, *box)
            done += 256
        res["cpu_oracle_transitions_per_s"] = done / (time.perf_counter() - t0)
    # the same chains on the likelihood marginalised over distance (20-node
    # rule): two gradient evaluations and a combine per leapfrog point
    dm = (10.0, 1000.0, 20)
    it2 = iter(range(burn + k))

    def step_dm():
        i = next(it2)
        plan.hmc(0, c, Z[i], U[i], sig, eps, n_leapfrog, box, lnL_out=ll, accepted_out=acc, dmarg=dm)
        acc_sum.add_(acc)

    for _ in range(burn):
        step_dm()
    acc_sum.zero_()
    secs_dm, _ = time_steps(step_dm, k, 0, torch)
    res["distance_marginalised"] = {"transitions_per_s": chains * k / secs_dm, "ms_per_transition": 1e3 * secs_dm / k,
                                    "acceptance": float(acc_sum.double().mean().item() / k),
                                    "mean_lnLd": float(ll.mean().item())}
    plan.close()
    return res


def extra_nuts(ile, synth, torch, steps, chains=16384, max_depth=6, cpu=True):
    """No-U-Turn transitions of 16384 chains (3 detectors, 9 modes, SNR 100),
    at most 6 doublings, the chains in lockstep with one gradient launch per
    leapfrog step for the batch; random numbers drawn beforehand (not
    timed)."""
    pt = synth.make_point(3, 9, 6554, 32768.0, 100.0, 44)
    sig = np.array([1e-3, 1e-3, 5e-3, 5e-3, 5e-3, 3e-6, 5e-3])
    box = (-0.01, 0.01, 10.0, 1000.0)
    eps, D = 0.3, max_depth
    th0 = seed_near_peak(ile, torch, synth, pt, sig)
    start = synth.perturbed_samples(th0, sig, chains, 6)
    start[3] = np.cos(start[3])
    start[6] = np.log(start[6])
    plan = ile.Plan([pt], [chains])
    c = torch.as_tensor(start, device="cuda").contiguous()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(9)
    burn, k = 3, max(4, steps // 2)
    tot = burn + k
    Z = torch.randn((tot, 7, chains), dtype=torch.float64, device="cuda", generator=gen)
    DI = torch.rand((tot, D, chains), dtype=torch.float64, device="cuda", generator=gen)
    ME = torch.rand((tot, D, chains), dtype=torch.float64, device="cuda", generator=gen)
    LE = torch.rand((tot, 2 ** D - 1, chains), dtype=torch.float64, device="cuda", generator=gen)
    ll = torch.empty(chains, dtype=torch.float64, device="cuda")
    info = torch.empty((3, chains), dtype=torch.int32, device="cuda")
    it = iter(range(tot))
    stats = []

    def step():
        i = next(it)
        plan.nuts(0, c, Z[i], DI[i], ME[i], LE[i], sig, eps, D, box, lnL_out=ll, info_out=info)

    for _ in range(burn):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps_total = 0
    depth_total = 0.0
    for _ in range(k):
        step()
        inf = info.cpu().numpy()
        steps_total += int(inf[1].sum())
        depth_total += float(inf[0].mean())
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    per = secs / k
    plan.close()
    return {"workload": "3 detectors, 9 modes (l<=3), Q 6554 samples at 32768 Hz, SNR 100; 16384 chains, one "
                        "No-U-Turn transition (at most 6 doublings, step 0.3) per call",
            "transitions_per_s": chains / per, "ms_per_transition": 1e3 * per,
            "leapfrog_steps_per_s": steps_total / secs, "mean_steps": steps_total / (k * chains),
            "mean_depth": depth_total / k, "mean_lnL": float(ll.mean().item()),
            "note": "wall time per call, including the per-step launches and the early-stop checks (the chains "
                    "advance in lockstep, so a call lasts as long as its longest tree)"}


def extra_smc(ile, synth, torch, steps, particles=65536, cpu=True):
    """An adaptive SMC ladder (Eqs. (sampler-menu:tempered-target),
    (sampler-menu:smc-update)) from the prior to the posterior of a 3-detector,
    9-mode point at SNR 5: 65536 particles; per rung the library's reweight
    (rung chosen at a conditional effective-size fraction of 0.5),
    systematic resampling, and two tempered HMC moves (4 leapfrog steps of
    0.25, proposal widths 0.2 x the cloud's spread).  The caller's logic
    (widths, random numbers, the loop) is host code; every per-particle step
    is a library kernel."""
    pt = synth.make_point(3, 9, 6554, 32768.0, 5.0, 44)
    n = particles
    box = (-0.01, 0.01, 10.0, 1000.0)
    th = synth.prior_samples(n, 5)
    th[3] = np.cos(th[3])
    th[6] = np.log(th[6])
    plan = ile.Plan([pt], [n])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)

    def ladder():
        c = torch.as_tensor(th, device="cuda").contiguous()
        c2 = torch.empty_like(c)
        lnL = torch.empty(n, dtype=torch.float64, device="cuda")
        g = torch.empty((7, n), dtype=torch.float64, device="cuda")
        plan.grad(0, c, lnL_out=lnL, grad_out=g, coords="sampler")
        lnW = torch.zeros(n, dtype=torch.float64, device="cuda")
        out = torch.empty(2, dtype=torch.float64, device="cuda")
        beta, lnZ, rungs, acc_sum = 0.0, 0.0, 0, 0.0
        while beta < 1.0 and rungs < 200:
            ile.smc_reweight(lnL, lnW, beta, 0.5, out=out)
            o = out.cpu().numpy()
            beta, lnZ, rungs = float(o[0]), lnZ + float(o[1]), rungs + 1
            u = float(torch.rand(1, generator=gen, device="cuda").item())
            anc = torch.empty(n, dtype=torch.int64, device="cuda")
            ile.smc_resample(lnW, u, c, c2, anc)
            c, c2 = c2, c
            lnW.zero_()  # the moves below return lnL at the moved particles
            sig = np.maximum(0.2 * c.std(dim=1).cpu().numpy(), 1e-12)
            for _ in range(2):
                z = torch.randn((7, n), dtype=torch.float64, device="cuda", generator=gen)
                uu = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
                _, acc = plan.hmc(0, c, z, uu, sig, 0.25, 4, box, lnL_out=lnL, beta=beta)
                acc_sum += float(acc.double().mean().item())
        return beta, lnZ, rungs, acc_sum / max(1, 2 * rungs)

    def ladder_rwm(moves=4):
        """The same ladder with the paper's moves: after resampling, random-walk
        Metropolis with the proposal covariance (2.38^2 / 7) C of the cloud,
        C from the device moments."""
        c = torch.as_tensor(th, device="cuda").contiguous()
        c2 = torch.empty_like(c)
        lnL = torch.empty(n, dtype=torch.float64, device="cuda")
        g = torch.empty((7, n), dtype=torch.float64, device="cuda")
        plan.grad(0, c, lnL_out=lnL, grad_out=g, coords="sampler")
        l2 = torch.empty_like(lnL)
        lnW = torch.zeros(n, dtype=torch.float64, device="cuda")
        out = torch.empty(2, dtype=torch.float64, device="cuda")
        beta, lnZ, rungs, acc_sum = 0.0, 0.0, 0, 0.0
        while beta < 1.0 and rungs < 200:
            ile.smc_reweight(lnL, lnW, beta, 0.5, out=out)
            o = out.cpu().numpy()
            beta, lnZ, rungs = float(o[0]), lnZ + float(o[1]), rungs + 1
            u = float(torch.rand(1, generator=gen, device="cuda").item())
            anc = torch.empty(n, dtype=torch.int64, device="cuda")
            ile.smc_resample(lnW, u, c, c2, anc)
            torch.index_select(lnL, 0, anc, out=l2)
            c, c2, lnL, l2 = c2, c, l2, lnL
            lnW.zero_()
            _, cov = ile.moments(c)
            for _ in range(moves):
                z = torch.randn((7, n), dtype=torch.float64, device="cuda", generator=gen)
                uu = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
                acc, _ = plan.rwm(0, c, z, uu, cov, 2.38 ** 2 / 7, box, lnL, beta=beta)
                acc_sum += float(acc.double().mean().item())
        return beta, lnZ, rungs, acc_sum / max(1, moves * rungs)

    ladder()  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    beta, lnZ, rungs, acc = ladder()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ladder_rwm()  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    beta_r, lnZ_r, rungs_r, acc_r = ladder_rwm()
    torch.cuda.synchronize()
    wall_r = time.perf_counter() - t0
    # the same normalisation by brute-force prior Monte Carlo: 4e9 prior draws
    # (rift_ile_mixture_is with alpha = 1) in chunks of 4e6
    Nc = 4_000_000
    gref = torch.Generator(device="cuda")
    gref.manual_seed(3)
    zeros = torch.zeros(Nc, dtype=torch.float64, device="cuda")
    m_run, s_run, s2_run = -np.inf, 0.0, 0.0
    torch.cuda.synchronize()
    t_ref = time.perf_counter()
    for _ in range(1000):
        vv = torch.rand((7, Nc), dtype=torch.float64, device="cuda", generator=gref)
        thr, _, _, _ = ile.mixture_is(1.0, [], None, None, 1.0, box, vv, vv, zeros)
        _, _, llr = ile.lnZ([pt], thr, want_lnL=True)
        lm = float(llr.max())
        w = torch.exp(llr - lm)
        s1, s2 = float(w.sum()), float((w * w).sum())
        m = max(m_run, lm)
        s_run = s_run * np.exp(m_run - m) + s1 * np.exp(lm - m)
        s2_run = s2_run * np.exp(2 * (m_run - m)) + s2 * np.exp(2 * (lm - m))
        m_run = m
    torch.cuda.synchronize()
    ref_s = time.perf_counter() - t_ref
    del vv, thr, llr, w, zeros
    # the reweight alone at this size
    lnLt = torch.as_tensor(-0.5 * 40.0 * np.random.default_rng(1).chisquare(3, n), device="cuda")
    lnWt = torch.zeros(n, dtype=torch.float64, device="cuda")
    secs, _ = time_steps(lambda: ile.smc_reweight(lnLt, lnWt.zero_(), 0.0, 0.5), 10, 2, torch)
    plan.close()
    dm12 = _smc_dmarg_snr12(ile, synth, torch, box)
    return {"workload": "3 detectors, 9 modes (l<=3), Q 6554 samples at 32768 Hz, SNR 5; 65536 particles from the "
                        "prior; adaptive SMC ladder (target fraction 0.5), 2 tempered HMC moves per rung",
            "rungs": rungs, "ladder_ms": 1e3 * wall, "ms_per_rung": 1e3 * wall / max(1, rungs),
            "final_beta": beta, "lnZ_smc": lnZ, "lnZ_prior_mc_4e9": float(m_run + np.log(s_run / (1000 * Nc))),
            "kish_prior_mc_4e9": s_run ** 2 / s2_run, "prior_mc_4e9_s": ref_s,
            "move_acceptance": acc, "reweight_ms": 1e3 * secs / 10,
            "rwm_moves": {"moves_per_rung": 4, "rungs": rungs_r, "ladder_ms": 1e3 * wall_r,
                          "ms_per_rung": 1e3 * wall_r / max(1, rungs_r), "final_beta": beta_r, "lnZ_smc": lnZ_r,
                          "move_acceptance": acc_r},
            "distance_marginalised_snr12": dm12}


def _smc_dmarg_snr12(ile, synth, torch, box, n=262144):
    """The SMC ladder on the likelihood marginalised over distance against the
    same ladder on all seven rows, for a 3-detector, 9-mode point at SNR 12:
    262144 particles from the prior, rungs at a conditional effective-size
    fraction of 0.9, 8 tempered HMC moves per rung of 4 leapfrog steps of
    0.15 (widths 0.2 x the cloud's spread); on the marginal the moves are
    rift_ile_plan_hmc_dmarg's (the distance row carries no momentum).  The
    reference is brute-force prior Monte Carlo of the marginal likelihood,
    1e9 prior draws (rift_ile_mixture_is with alpha = 1) through
    rift_ile_plan_lnZ_dmarg; both ladders estimate the same ln Z."""
    pt = synth.make_point(3, 9, 6554, 32768.0, 12.0, 61)
    dm = (10.0, 1000.0, 20)
    th = synth.prior_samples(n, 5)
    th[3] = np.cos(th[3])
    th[6] = np.log(th[6])
    plan = ile.Plan([pt], [n])

    def ladder(marg, seed):
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        c = torch.as_tensor(th, device="cuda").contiguous()
        c2 = torch.empty_like(c)
        lnL = torch.empty(n, dtype=torch.float64, device="cuda")
        g = torch.empty((7, n), dtype=torch.float64, device="cuda")
        if marg:
            plan.grad_dmarg(0, c, *dm, lnLd_out=lnL, grad_out=g)
        else:
            plan.grad(0, c, lnL_out=lnL, grad_out=g, coords="sampler")
        lnW = torch.zeros(n, dtype=torch.float64, device="cuda")
        out = torch.empty(2, dtype=torch.float64, device="cuda")
        beta, lnZ, rungs, acc_sum = 0.0, 0.0, 0, 0.0
        while beta < 1.0 and rungs < 200:
            ile.smc_reweight(lnL, lnW, beta, 0.9, out=out)
            o = out.cpu().numpy()
            beta, lnZ, rungs = float(o[0]), lnZ + float(o[1]), rungs + 1
            u = float(torch.rand(1, generator=gen, device="cuda").item())
            anc = torch.empty(n, dtype=torch.int64, device="cuda")
            ile.smc_resample(lnW, u, c, c2, anc)
            c, c2 = c2, c
            lnW.zero_()
            sig = np.maximum(0.2 * c.std(dim=1).cpu().numpy(), 1e-12)
            for _ in range(8):
                z = torch.randn((7, n), dtype=torch.float64, device="cuda", generator=gen)
                uu = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
                _, acc = plan.hmc(0, c, z, uu, sig, 0.15, 4, box, lnL_out=lnL, beta=beta,
                                  dmarg=dm if marg else None)
                acc_sum += float(acc.double().mean().item())
        return lnZ, rungs, acc_sum / max(1, 8 * rungs)

    ladder(True, 1)  # warm
    res = {}
    for marg, key in ((True, "marginal"), (False, "all_rows")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runs = [ladder(marg, 11 + 100 * s) for s in range(3)]
        torch.cuda.synchronize()
        z = [r[0] for r in runs]
        res[key] = {"lnZ_smc_seeds": z, "lnZ_smc_mean": float(np.mean(z)), "lnZ_smc_sd": float(np.std(z, ddof=1)),
                    "rungs": float(np.mean([r[1] for r in runs])),
                    "move_acceptance": float(np.mean([r[2] for r in runs])),
                    "ladder_ms": 1e3 * (time.perf_counter() - t0) / 3}
    plan.close()
    Nc, chunks = 4_000_000, 250
    plan_ref = ile.Plan([pt], [Nc])
    gref = torch.Generator(device="cuda")
    gref.manual_seed(3)
    zeros = torch.zeros(Nc, dtype=torch.float64, device="cuda")
    ll = torch.empty(Nc, dtype=torch.float64, device="cuda")
    m_run, s_run, s2_run = -np.inf, 0.0, 0.0
    torch.cuda.synchronize()
    t_ref = time.perf_counter()
    for _ in range(chunks):
        vv = torch.rand((7, Nc), dtype=torch.float64, device="cuda", generator=gref)
        thr, _, _, _ = ile.mixture_is(1.0, [], None, None, 1.0, box, vv, vv, zeros)
        plan_ref.lnZ_dmarg(thr, *dm, lnL_out=ll)
        lm = float(ll.max())
        w = torch.exp(ll - lm)
        s1, s2 = float(w.sum()), float((w * w).sum())
        m = max(m_run, lm)
        s_run = s_run * np.exp(m_run - m) + s1 * np.exp(lm - m)
        s2_run = s2_run * np.exp(2 * (m_run - m)) + s2 * np.exp(2 * (lm - m))
        m_run = m
    torch.cuda.synchronize()
    ref_s = time.perf_counter() - t_ref
    plan_ref.close()
    res.update({"workload": "3 detectors, 9 modes, SNR 12; 262144 particles; ladder at fraction 0.9, 8 HMC moves "
                            "per rung (4 leapfrog steps of 0.15); 3 seeds each, on L marginalised over distance "
                            "(20 nodes) and on all 7 rows",
                "lnZ_prior_mc_1e9": float(m_run + np.log(s_run / (chunks * Nc))),
                "kish_prior_mc_1e9": s_run ** 2 / s2_run, "prior_mc_1e9_s": ref_s})
    return res


def extra_is(ile, synth, torch, steps, draws=1_000_000, cpu=True):
    """The importance-sampling normalisation with a defensive Gaussian-mixture
    proposal (Eq. (sampler-menu:is)) for a 3-detector, 9-mode point at SNR 4,
    where one Gaussian covers the posterior (above that the sky is multimodal
    and the proposal needs a component per recovered mode): a pilot of 1e6
    prior draws, one component fitted by the device moments of its 4000 best
    draws weighted by their likelihood (covariance widened by s = 1.5, prior
    share alpha = 0.3), then 1e6 draws from the mixture with their weights and
    ln Z through the likelihood kernel.  Reported beside the prior Monte-Carlo
    ln Z of 4e6 prior draws, each with its Kish effective size."""
    pt = synth.make_point(3, 9, 6554, 32768.0, 4.0, 61)
    box = (-0.01, 0.01, 10.0, 1000.0)
    thp = synth.prior_samples(1_000_000, 62)
    lp = ile.lnL(pt, thp).cpu().numpy()
    best = np.argsort(lp)[-4000:]
    c = thp[:, best].copy()
    c[3] = np.cos(c[3])
    c[6] = np.log(c[6])
    ct = torch.as_tensor(c, device="cuda").contiguous()
    lwt = torch.as_tensor(lp[best] - lp[best].max(), device="cuda").contiguous()
    mean, cov = ile.moments(ct, lwt)
    cov_h = cov.cpu().numpy()
    scale, alpha = 1.5, 0.3
    f = np.ones(7)
    for j, P in ((0, 2 * np.pi), (2, np.pi), (4, 2 * np.pi)):
        f[j] = min(1.0, 0.45 * P / np.sqrt(scale * cov_h[j, j]))
    covt = torch.as_tensor((f[:, None] * cov_h * f[None, :])[None], device="cuda").contiguous()
    meant = mean[None].contiguous()
    n = draws
    gen = torch.Generator(device="cuda")
    gen.manual_seed(64)
    z = torch.randn((7, n), dtype=torch.float64, device="cuda", generator=gen)
    v = torch.rand((7, n), dtype=torch.float64, device="cuda", generator=gen)
    u = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
    th = torch.empty((7, n), dtype=torch.float64, device="cuda")
    lnw = torch.empty(n, dtype=torch.float64, device="cuda")
    comp = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    draw = (lambda: ile.mixture_is(alpha, [1.0], meant, covt, scale, box, z, v, u, th, lnw, comp, st))
    secs_draw, _ = time_steps(draw, steps, 2, torch)
    big = torch.as_tensor(thp, device="cuda").contiguous()
    big[3] = torch.cos(big[3])
    big[6] = torch.log(big[6])
    lwb = torch.as_tensor(lp - lp.max(), device="cuda").contiguous()
    secs_mom, _ = time_steps(lambda: ile.moments(big, lwb), steps, 2, torch)
    zi, _, li = ile.lnZ([pt], th, lnw=lnw, want_lnL=True)
    secs_z, _ = time_steps(lambda: ile.lnZ([pt], th, lnw=lnw), steps, 2, torch)
    thq = synth.prior_samples(4_000_000, 65)
    zp, _, lq = ile.lnZ([pt], thq, want_lnL=True)

    def kish(t):
        w = torch.exp(t - t.max())
        return float((w.sum() ** 2 / (w * w).sum()).cpu())
    out = {"workload": "3 detectors, 9 modes (l<=3), Q 6554 samples at 32768 Hz, SNR 4; a component fitted to "
                       "the best 4000 of 1e6 prior draws; 1e6 draws from 0.3 prior + 0.7 N(mu, 1.5 C)",
           "status": int(st.cpu()[0]), "mixture_is_ms": 1e3 * secs_draw / steps,
           "mixture_draws_per_s": n * steps / secs_draw, "moments_1e6_ms": 1e3 * secs_mom / steps,
           "lnZ_ms": 1e3 * secs_z / steps, "lnZ_is": float(zi.cpu()[0]), "kish_is": kish(li + lnw),
           "lnZ_prior_mc_4e6": float(zp.cpu()[0]), "kish_prior_mc_4e6": kish(lq)}
    del z, v, u, th, lnw, comp, big, li, lq
    torch.cuda.empty_cache()
    out["distance_marginalised_snr12"] = _is_dmarg_multimode(ile, synth, torch, steps)
    return out


def _kmeans(X, k, iters=50, seed=0):
    rng = np.random.default_rng(seed)
    C = X[rng.choice(len(X), k, replace=False)]
    for _ in range(iters):
        lab = ((X[:, None, :] - C[None]) ** 2).sum(-1).argmin(1)
        for j in range(k):
            if np.any(lab == j):
                C[j] = X[lab == j].mean(0)
    return lab


def _is_dmarg_multimode(ile, synth, torch, steps):
    """SNR 12 with the likelihood marginalised over distance in the kernel:
    one component per k-means cluster (4) of the best 8000 of 2e6 pilot draws,
    each fitted by the device moments over the six sampled rows; 2e6 draws
    from 0.1 prior + 0.9 sum_m a_m N(mu_m, 2 C_m) weighted over those rows,
    ln Z through rift_ile_plan_lnZ_dmarg; against brute-force prior Monte
    Carlo of 1e8 draws (drawn by rift_ile_mixture_is with alpha = 1)."""
    box = (-0.01, 0.01, 10.0, 1000.0)
    per = ((0, 2 * np.pi), (2, np.pi), (4, 2 * np.pi))
    pt = synth.make_point(3, 9, 6554, 32768.0, 12.0, 61)
    N = 2_000_000
    plan = ile.Plan([pt], [N])
    ll = torch.empty(N, dtype=torch.float64, device="cuda")
    zeros = torch.zeros(N, dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    m_run, s_run, s2_run, pilot = -np.inf, 0.0, 0.0, None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(50):
        v = torch.rand((7, N), dtype=torch.float64, device="cuda", generator=gen)
        th, _, _, _ = ile.mixture_is(1.0, [], None, None, 1.0, box, v, v, zeros)
        plan.lnZ_dmarg(th, box[2], box[3], 20, lnL_out=ll)
        lm = float(ll.max())
        w = torch.exp(ll - lm)
        s1, s2 = float(w.sum()), float((w * w).sum())
        m = max(m_run, lm)
        s_run = s_run * np.exp(m_run - m) + s1 * np.exp(lm - m)
        s2_run = s2_run * np.exp(2 * (m_run - m)) + s2 * np.exp(2 * (lm - m))
        m_run = m
        if pilot is None:
            pilot = (th.cpu().numpy(), ll.cpu().numpy())
    torch.cuda.synchronize()
    prior_s = time.perf_counter() - t0
    thp, lp = pilot
    best = np.argsort(lp)[-8000:]
    c = thp[:, best].copy()
    c[3] = np.cos(c[3])
    c[6] = np.log(c[6])
    lb = lp[best]
    feats = np.stack([np.cos(c[0]) * np.cos(c[1]), np.sin(c[0]) * np.cos(c[1]), np.sin(c[1]), np.cos(c[4]),
                      np.sin(c[4]), np.cos(2 * c[2]), np.sin(2 * c[2]), c[3]], 1)
    lab = _kmeans(feats, 4)
    means, covs, a = [], [], []
    for j in range(4):
        sel = lab == j
        cj = c[:, sel].copy()
        for r, P in per:
            mu = np.arctan2(np.sin(2 * np.pi * cj[r] / P).mean(), np.cos(2 * np.pi * cj[r] / P).mean()) * P / (2 * np.pi)
            cj[r] = mu + ((cj[r] - mu + P / 2) % P) - P / 2
        mm, C = ile.moments(torch.as_tensor(cj, device="cuda").contiguous(),
                            torch.as_tensor(0.5 * (lb[sel] - lb[sel].max()), device="cuda").contiguous())
        C = C.cpu().numpy()
        f = np.ones(7)
        for r, P in per:
            f[r] = min(1.0, 0.45 * P / np.sqrt(2.0 * C[r, r]))
        means.append(mm.cpu().numpy())
        covs.append(f[:, None] * C * f[None, :])
        a.append(np.exp(lb[sel] - lb.max()).sum())
    a = np.array(a) / np.sum(a)
    mt = torch.as_tensor(np.array(means), device="cuda").contiguous()
    ct = torch.as_tensor(np.array(covs), device="cuda").contiguous()
    gen.manual_seed(7)
    z = torch.randn((7, N), dtype=torch.float64, device="cuda", generator=gen)
    v = torch.rand((7, N), dtype=torch.float64, device="cuda", generator=gen)
    u = torch.rand(N, dtype=torch.float64, device="cuda", generator=gen)
    th = torch.empty((7, N), dtype=torch.float64, device="cuda")
    lnw = torch.empty(N, dtype=torch.float64, device="cuda")
    comp = torch.empty(N, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    draw = (lambda: ile.mixture_is(0.1, a, mt, ct, 2.0, box, z, v, u, th, lnw, comp, st, rows=0b0111111))
    secs_draw, _ = time_steps(draw, steps, 2, torch)
    zi, _ = plan.lnZ_dmarg(th, box[2], box[3], 20, lnw=lnw, lnL_out=ll)
    t = ll + lnw
    t = t[torch.isfinite(t)]
    w = torch.exp(t - t.max())
    plan.close()
    return {"workload": "3 detectors, 9 modes, SNR 12, distance marginalised in the kernel (20-node Gauss-Hermite); "
                        "4 components from k-means clusters of the best 8000 of 2e6 pilot draws; 2e6 IS draws over "
                        "the other six rows",
            "status": int(st.cpu()[0]), "mixture_is_ms_2e6": 1e3 * secs_draw / steps,
            "lnZ_is": float(zi.cpu()[0]), "kish_is_2e6": float((w.sum() ** 2 / (w * w).sum()).cpu()),
            "lnZ_prior_mc_1e8": float(m_run + np.log(s_run / (50 * N))), "kish_prior_mc_1e8": s_run ** 2 / s2_run,
            "prior_mc_1e8_s": prior_s}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--samples", type=int, default=1_000_000)
    ap.add_argument("--workloads", default="c1,c4,c5,wide,dmarg,pregrid,tmarg,tband,pmarg,erai,hmc,nuts,smc,is",
                    help="workloads timed beside the headline one (comma list of c1, c4, c5, wide, dmarg, pregrid, "
                         "tmarg, tband, pmarg, erai, hmc, nuts, smc, is, "
                         "c3, c1big; "
                         "'none' for the headline alone)")
    ap.add_argument("--extras", nargs="?", const="c3,c1big,c5batch", default="",
                    help="add the longer workloads (the 512-point batch c3, C1 at 1e7 samples c1big, "
                         "the 64-point 5-detector batch c5batch)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--warm-s", type=float, default=0.3,
                    help="minimum seconds of warm-up work before each timed region (counter runs use 0)")
    ap.add_argument("--no-variants", action="store_true",
                    help="time only the chosen launch shape (for profiler runs)")
    ap.add_argument("--config", default=None,
                    help="fixed launch shape block,tile_blocks,blocks_per_cu,sort for both paths (no tuning)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with a plain 256-MiB elementwise copy kernel (counter calibration)")
    args = ap.parse_args()
    global WARM_S
    WARM_S = max(0.0, args.warm_s)
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "design only)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2609_37393_amd import ile, synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    ile.load()
    t_start = time.perf_counter()
    n = args.samples
    log(f"building inputs (n = {n})")
    pt, th = c2_inputs(synth, n)
    tht = torch.as_tensor(th, device="cuda").contiguous()
    K, M = pt["Q"].shape[0], pt["Q"].shape[1]
    lmax = int(pt["lm"][:, 0].max())

    log("fp64 path")
    fixed = None
    if args.config:
        b, tb, bpc, srt = (int(x) for x in args.config.split(","))
        fixed = {"block": b, "tile_blocks": tb, "blocks_per_cu": bpc, "sort": srt}
    r64 = run_path(ile, torch, pt, tht, "fp64", args.steps, args.warmup, tune=not args.no_tune,
                   variants=not args.no_variants, config=fixed)
    log("mixed path")
    r32 = run_path(ile, torch, pt, tht, "mixed", args.steps, args.warmup, tune=not args.no_tune,
                   variants=not args.no_variants, config=fixed)

    fps = survey_flops_per_sample(K, M)
    fps_own = flops_per_sample(K, M, lmax)
    value = n * args.steps / r64["secs"]
    kern_s = r64["kernel_ms_avg"] / 1e3
    achieved = fps * n / kern_s / 1e12
    kern32_s = r32["kernel_ms_avg"] / 1e3
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "lnL evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r64["secs"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "3 detectors, 21 modes (l<=4), Q 6554 samples/mode/detector at 32768 Hz, "
                        "network SNR 600, 1e6 prior extrinsic samples; lnL per sample + ln Z",
            "n_samples": n,
            "launch": r64["config"],
            "launch_variants": r64["variants"],
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": bench_traffic(),
            "kernel": "k_tiles<double,3,4,MODE_LSE64>",
            "kernel_ms_avg": r64["kernel_ms_avg"],
            "flops_per_sample": fps,
            "flops_per_sample_formulation": fps_own,
            "frac_formulation": fps_own * n / kern_s / 1e12 / PEAK_FP64_TFLOPS,
            "hbm_bytes_per_sample": bytes_per_sample(),
        },
        "mixed": {
            "lnL_evals_per_s": n * args.steps / r32["secs"],
            "ms_per_step": 1e3 * r32["secs"] / args.steps,
            "speedup_vs_fp64": r64["secs"] / r32["secs"],
            "kernel": "k_tiles<float,3,4,MODE_PASS32>",
            "kernel_ms_avg": r32["kernel_ms_avg"],
            "alu_frac_fp32_pass": fps * n / kern32_s / 1e12 / PEAK_FP32_UNPACKED_TFLOPS,
            "alu_peak_fp32_pass": PEAK_FP32_UNPACKED_TFLOPS,
            "refined_samples": r32["refined"],
            "dlnZ_vs_fp64": abs(r32["lnZ"] - r64["lnZ"]),
            "lnZ_err_bound": r32["lnZ_err_bound"],
            "launch": r32["config"],
            "launch_variants": r32["variants"],
        },
        "lnZ": r64["lnZ"],
        "neff": r64["neff"],
    }
    gpu_lnL = r64["lnL"].cpu().numpy()
    l32 = r32["lnL"].cpu().numpy()
    top = gpu_lnL >= gpu_lnL.max() - 20.0
    out["mixed"]["max_dlnL_posterior_set_vs_fp64"] = float(np.abs(l32[top] - gpu_lnL[top]).max())
    del r64, r32
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cb, par = cpu_baseline(pt, th, gpu_lnL)
        out["cpu_baseline"] = cb
        out["parity"] = par
    del tht
    torch.cuda.empty_cache()
    wanted = [x.strip() for x in args.workloads.split(",") if x.strip() and x.strip() != "none"]
    wanted += [x.strip() for x in args.extras.split(",") if x.strip()]
    fns = {"c1": extra_c1, "c4": extra_c4, "c5": extra_c5, "c3": extra_c3, "c1big": extra_c1_big,
           "c5batch": extra_c5_batch, "wide": extra_wide, "dmarg": extra_dmarg, "pregrid": extra_pregrid,
           "tmarg": extra_tmarg, "tband": extra_tband, "pmarg": extra_pmarg, "erai": extra_erai,
           "hmc": extra_hmc, "nuts": extra_nuts, "smc": extra_smc, "is": extra_is}
    for name in wanted:
        log(f"workload {name}")
        try:
            out[name] = fns[name](ile, synth, torch, max(3, args.steps // 10), cpu=not args.no_cpu)
        except Exception as e:  # report, keep the headline line
            out[name] = {"error": repr(e)}
        torch.cuda.empty_cache()
    if args.calib_copy:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.add(a, 0.0, out=b)  # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
    out["bench_wall_s"] = time.perf_counter() - t_start
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
