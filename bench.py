#!/usr/bin/env python3
"""Benchmark: pair evaluations per second of one dense RGB-D-frame registration on MI355X.

Headline workload (one step = one full registration, inputs resident in HBM):
  two synthetic 640x480 RGB-D frames of a piecewise-planar room, a seeded
  random subset of 300,000 valid pixels per frame (the dense frame), 5 label
  channels, ground-truth motion <= 5 deg / 0.05 m; kernel cutoff 3 ell with
  the voxel-grid neighbour search; 100 gradient-flow iterations with ell
  annealed geometrically 0.2 -> 0.05 m over 4 stages; FP32 pair terms,
  compensated FP32 partials, FP64 reduction, step and pose.
value = pairs inside the cutoff evaluated over the timed registrations / wall time.

Also reported: the pair kernel against the FP32 vector roofline (event-timed
on the launch stream), per-registration latency p50/p99, the all-FP64 path
on the same registration, teacher-forced parity and the CPU oracle timed on
a bounded sample of the same registration (its own trajectory's poses), the
30k semi-dense RGB-D pair (fixed, conjugate-direction and quartic step
rules, and all pairs without the cutoff), a batched run through the
continuous-batching scheduler (regs/s, per-request latency), Poisson
serving at 200-2000 requests/s, and the remaining workloads.  --legs picks
which of those legs run after the headline (default: all); --no-extra runs
the headline and its CPU baseline only.
"""
import argparse
import hashlib
import json
import os
import sys
import time

from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 26          # d:3, r^2:5, exponent scale:1, label product (5 ch):9, weight:1, W:1, D:6
# quartic pass: d:3, r^2:5, scale:1, labels:9, weight:1, beta:5, gamma/delta/eps:18, beta^2:1,
# g2:2, g3:4, g4:8, four sums:8
QUARTIC_FLOPS_PER_PAIR = 65
PEAK_TFLOPS = 157.3          # MI355X published FP32 vector peak (counts packed FP32, two FMAs per lane per cycle)
# the FP32 issue ceiling without packed FP32 (which this library's kernels do
# not use): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
PEAK_UNPACKED_TFLOPS = 78.6
METRIC = "pair-evals/s per registration + batched regs/s, p50/p99 latency @1e-5 rel"
KERNEL_SRC = os.path.join(ROOT, "paper_1904_02266_amd", "csrc", "cvo_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pairs_dense300k_traffic.md")
# the legs after the headline registration, in the order they run
LEGS = ("rgbd30k", "batched", "serving", "bruteforce", "frontend", "planes", "odometry")
GOLDEN = os.path.join(ROOT, "tests", "golden", "dense300k_trajectory.json")
SAMPLE_ITERS = (0, 25, 50, 99)   # one iteration of each length-scale stage (oracle sample, parity)


def progress(msg):
    """One line per finished leg on stderr (the JSON line stays alone on stdout)."""
    print(f"bench: {msg} ({time.strftime('%H:%M:%S')})", file=sys.stderr, flush=True)


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per pair-kernel launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy), or None when
    the kernel source has changed since the counters were taken."""
    try:
        with open(KERNEL_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        fields = {}
        with open(path) as f:
            for line in f:
                if ":" in line and line.startswith("- "):
                    key, val = line[2:].split(":", 1)
                    fields[key.strip()] = val.strip().strip("`")
        if fields.get("kernel_source_sha256") != sha:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _gen_request(args):
    seed, ns, nt = args
    from paper_1904_02266_amd import synth
    p = synth.rgbd_pair(ns, nt, seed=seed)
    return p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat


def gen_batch(nreq):
    """The batched run's inputs, drawn in worker processes.  Called before this
    process touches the GPU (the workers are forked)."""
    if nreq <= 0:
        return []
    from paper_1904_02266_amd import synth
    with ProcessPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
        return list(ex.map(_gen_request, synth.batched_sizes(nreq)))


def _gen_pool_pair(seed):
    from paper_1904_02266_amd import synth
    p = synth.rgbd_pair(300000, 300000, seed=seed, select="random")
    rng = np.random.default_rng(seed + 17)
    a, b = rng.permutation(len(p.src_xyz)), rng.permutation(len(p.tgt_xyz))
    return p.src_xyz[a], p.src_feat[a], p.tgt_xyz[b], p.tgt_feat[b]


def _gen_dense(seed):
    from paper_1904_02266_amd import synth
    p = synth.rgbd_pair(300000, 300000, seed=seed, select="random")
    return (p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat), p.T_true


def dense_bruteforce(cloud, golden, iters=(0, 1, 5, 10, 25, 50, 99)):
    """The dense-300k frame pair (a seeded random subset of 300,000 valid
    pixels per frame) evaluated without a cutoff: all 9.0e10 pairs of one
    gradient evaluation, at the poses and length-scales of the stored oracle
    trajectory's iterations `iters`, the pair kernel event-timed (the
    kernel's measurement point at full occupancy, no pairs wasted outside a
    cutoff), and the same evaluations with every pair term in FP64."""
    import torch
    from paper_1904_02266_amd import Context, Params
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(a).to(dev) for a in cloud]
    torch.cuda.synchronize()
    tr = np.array(golden["trace"])
    ctx = Context(0)

    def one(T, ell, precision):
        prm = Params(stage_ell=(ell,), cutoff_mult=0.0, max_iters=1, precision=precision)
        ctx.kernel_stats(reset=True)
        ctx.set_profiling(True)
        out = ctx.register(*t, prm, T0=T)
        ctx.set_profiling(False)
        return out, ctx.kernel_stats(reset=True)

    one(np.eye(4), float(tr[0, 8]), "fp32")  # warm-up
    poses, ms, pairs, ms64, worst = [], 0.0, 0, 0.0, 0.0
    for k in iters:
        T = np.eye(4) if k == 0 else tr[k - 1, 10:26].reshape(4, 4)
        ell = float(tr[k, 8])
        out, ks = one(T, ell, "fp32")
        o64, k64 = one(T, ell, "fp64")
        g32 = np.array([out["F"], *out["omega"], *out["v"]])
        g64 = np.array([o64["F"], *o64["omega"], *o64["v"]])
        f_rel = float(abs(g32[0] - g64[0]) / g64[0])
        g_rel = float(np.linalg.norm(g32[1:] - g64[1:]) / max(np.linalg.norm(g64[1:]), 1e-300))
        worst = max(worst, f_rel)
        ms += ks["ms"]
        ms64 += k64["ms"]
        pairs += ks["pairs"]
        poses.append({"iter": k, "ell": ell, "pair_kernel_ms": ks["ms"],
                      "tflops": FLOPS_PER_PAIR * ks["pairs"] / (ks["ms"] * 1e-3) / 1e12,
                      "fp64_pair_kernel_ms": k64["ms"], "F": out["F"], "F_rel_diff_fp64": f_rel,
                      "grad_normwise_rel_diff_fp64": g_rel})
    ctx.close()
    ach = FLOPS_PER_PAIR * pairs / (ms * 1e-3) / 1e12
    return {"pairs": pairs // len(iters), "pair_kernel_ms": ms / len(iters), "achieved_tflops": ach,
            "frac": ach / PEAK_TFLOPS, "pair_evals_per_s": pairs / (ms * 1e-3),
            "kernel": "k_pairs<float,5,false,false>", "poses": poses,
            "note": "oracle trajectory poses of the listed iterations, each at its stage's length-scale",
            "fp64_path": {"pair_kernel_ms": ms64 / len(iters), "speedup_of_mixed": ms64 / ms,
                          "max_F_rel_diff": worst,
                          "note": "FP32-Kahan against FP64 at each pose: F relative, and (omega, v) "
                                  "normwise relative to |(omega, v)|, which shrinks toward convergence"}}


def frontend_vga(frame, k=30000, steps=20):
    """The device front end on one synthetic 640x480 RGB-D frame already in
    HBM (30,000 points kept): ms per frame and the algorithmic bytes (depth
    and colour read, points and labels written) per second."""
    import torch
    from paper_1904_02266_amd import Context
    dev = torch.device("cuda:0")
    d = torch.from_numpy(frame.depth).to(dev)
    c = torch.from_numpy(frame.rgb).to(dev)
    ctx = Context(0)
    ctx.frontend(d, c, k, frame.fx, frame.fy, frame.cx, frame.cy, frame.dmin, frame.dmax)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        xyz, feat = ctx.frontend(d, c, k, frame.fx, frame.fy, frame.cx, frame.cy, frame.dmin, frame.dmax)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    ctx.close()
    P = frame.depth.size
    algo = 16 * P + 32 * xyz.shape[0]
    return {"ms_per_frame": el * 1e3, "pixels": P, "points": int(xyz.shape[0]),
            "algorithmic_bytes": algo, "achieved_gb_per_s": algo / el / 1e9,
            "note": "synchronous call (host reads the selected count back); 14 short kernels per frame"}


def planes_c1(steps=10):
    """The 2,000-point three-plane registration (all pairs, 50 steps):
    launch-bound, reported as ms per registration."""
    import torch
    from paper_1904_02266_amd import Context, params_planes, synth
    p = synth.planes_pair(2000, seed=1)
    ctx = Context(0)
    ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, params_planes())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.register(p.src_xyz, p.src_feat, p.tgt_xyz, p.tgt_feat, params_planes())
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    ctx.close()
    E = out["T"][:3, :3] @ p.T_true[:3, :3].T
    return {"ms_per_registration": el * 1e3, "iterations": 50, "pairs_per_registration": out["pairs_within"],
            "rot_err_deg": float(np.degrees(np.arccos(np.clip((np.trace(E) - 1) / 2, -1, 1)))),
            "note": "host inputs (about 64 KB per cloud copied per call)"}


def gen_serving_pool(npairs):
    """Frame pairs the serving requests are cut from (random pixel subsets of
    300k points; a request of n points takes the first n).  Drawn in worker
    processes before this process touches the GPU."""
    if npairs <= 0:
        return []
    with ProcessPoolExecutor(max_workers=max(1, min(16, npairs))) as ex:
        return list(ex.map(_gen_pool_pair, [5100 + k for k in range(npairs)]))


def window_rates(arrivals, latencies_ms, ok, window_s):
    """Completions against arrivals over the second half of an arrival
    window: (completions per s there, completions / arrivals there, or None
    without arrivals).  arrivals in s from the window's start, latencies from
    submission to completion, ok the requests that succeeded."""
    h0, h1 = 0.5 * window_s, window_s
    half_arr = sum(1 for ts in arrivals if h0 <= ts < h1)
    half_done = sum(1 for ts, lat, good in zip(arrivals, latencies_ms, ok) if good and h0 <= ts + lat / 1e3 < h1)
    return half_done / (h1 - h0), (half_done / half_arr if half_arr else None)


def serving(pool, rates=(100, 150, 200, 500, 1000, 2000), window_s=10.0, table1_rates=(200,)):
    """Poisson arrivals at each rate over window_s seconds, cloud sizes
    lognormal (median 20k, shape 1.0, clamped to 1000..300000) cut from the
    pool, RGB-D schedule with the conjugate-direction quartic step, stop once
    the last stage's applied twist |tau d| < 1e-5, at most 200 iterations
    (and the Table 1 parameter set at table1_rates); each request is submitted
    at its arrival time and its latency is submission to completion (the
    library's wall clock).  A rate is served when, over the second half of
    the window (past the start-up, before the drain), requests complete at
    >= 95% of the rate they arrive at: the admitted requests share the GPU,
    so under overload every latency grows and only the completion rate
    shows the backlog.  throughput_per_s counts the completions over the
    span from the first arrival to the last completion, drain included."""
    import torch
    from paper_1904_02266_amd import Context, params_rgbd, params_table1, synth
    dev = torch.device("cuda:0")
    dpool = [[torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in c] for c in pool]
    torch.cuda.synchronize()
    runs = [("rgbd", params_rgbd(step_rule="conjugate", tol=1e-5, stage_tol=1e-4, max_iters=200), r) for r in rates]
    runs += [("table1", params_table1(), r) for r in table1_rates]
    out = []
    for pname, prm, rate in runs:
        stream = synth.serving_stream(rate, window_s=window_s)
        ctx = Context(0, max_slots=4096)
        t0 = time.perf_counter()
        subs = []
        for arr, seed, ns, nt in stream:
            c = dpool[seed % len(dpool)]
            now = time.perf_counter() - t0
            if arr > now:
                time.sleep(arr - now)
            ts = time.perf_counter() - t0
            tk, keep = ctx.submit(c[0][:ns], c[1][:ns], c[2][:nt], c[3][:nt], prm)
            subs.append((tk, keep, ts))
        res = [(ctx.poll(tk), ts) for tk, _, ts in subs]
        st = ctx.serving_stats()
        ctx.close()
        ok = [r for r, _ in res if r["rc"] == 0]
        fails = {}
        for r, _ in res:
            if r["rc"] != 0:
                fails[str(r["rc"])] = fails.get(str(r["rc"]), 0) + 1
        lat = np.array([r["wall_ms"] for r in ok])
        end = max(ts + r["wall_ms"] / 1e3 for r, ts in res)
        steady, steady_frac = window_rates([ts for _, ts in res], [r["wall_ms"] for r, _ in res],
                                           [r["rc"] == 0 for r, _ in res], window_s)
        progress(f"serving {pname} at {rate}/s: {len(ok)} of {len(res)} in {end:.1f} s")
        out.append({"params": pname, "rate": rate, "requests": len(res), "completed": len(ok),
                    "throughput_per_s": len(ok) / end, "span_s": end,
                    "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                    "steady_throughput_per_s": steady,
                    "steady_completed_per_arrived": steady_frac,
                    "mean_iters": float(np.mean([r["iters"] for r in ok])),
                    "converged": float(np.mean([r["converged"] for r in ok])), "failed_by_code": fails,
                    "hbm_peak_gb": st["hbm_peak"] / 1e9})
    sat = None
    for r in out:
        if r["params"] == "rgbd" and (r["steady_completed_per_arrived"] or 0.0) >= 0.95:
            sat = r["rate"] if sat is None else max(sat, r["rate"])
    top = max((r["steady_throughput_per_s"] for r in out if r["params"] == "rgbd"), default=None)
    return {"window_s": window_s, "sizes": "lognormal median 20k, shape 1.0, clamped 1000..300000",
            "params": {"rgbd": "RGB-D schedule (a stage also ends once |tau d| < 1e-4), conjugate-direction "
                               "quartic step, stop at |tau d| < 1e-5 in the last stage, cap 200 iterations",
                       "table1": "Table 1 set: quartic step, value floor 1e-3, thresholds 1e-5 / 5e-5, cap 200"},
            "saturation": {"highest_rate_served_per_s": sat, "max_throughput_per_s": top,
                           "criterion": "completions >= 0.95 x arrivals over the second half of the window; "
                                        "max_throughput_per_s is the completion rate over that half"},
            "rates": out}


def batched_both(clouds):
    """The batched run in the mixed-precision path and in the all-FP64 path
    (every pair term in FP64) on the same requests."""
    out = batched(clouds)
    f64 = batched(clouds, repeats=1, precision="fp64")
    out["fp64_path"] = {"regs_per_s": f64["regs_per_s"], "pair_evals_per_s": f64["pair_evals_per_s"],
                        "wall_s": f64["wall_s"], "latency_ms": f64["latency_ms"],
                        "speedup_of_mixed": out["regs_per_s"] / f64["regs_per_s"]}
    return out


def batched(clouds, repeats=2, precision="fp32"):
    """The registrations of `clouds` (the RGB-D generator, per-request seeds
    4000 + k, cloud sizes uniform in 5000..60000, 100 iterations each)
    submitted at once to the continuous-batching scheduler; inputs already on
    the device."""
    import torch
    from paper_1904_02266_amd import Context, params_rgbd
    nreq = len(clouds)
    dev = torch.device("cuda:0")
    dclouds = [[torch.from_numpy(a).to(dev) for a in c] for c in clouds]
    torch.cuda.synchronize()
    ctx = Context(0, max_slots=max(nreq, 1))
    prm = params_rgbd(precision=precision)

    def run():
        t0 = time.perf_counter()
        tks = [ctx.submit(*c, prm) for c in dclouds]
        outs = [ctx.poll(tk) for tk, _ in tks]
        return time.perf_counter() - t0, outs

    run()  # warm-up
    best = None
    for _ in range(repeats):
        el, outs = run()
        if any(o["rc"] != 0 for o in outs):
            raise RuntimeError("a batched registration failed: " + str([o["rc"] for o in outs]))
        if best is None or el < best[0]:
            best = (el, outs)
    el, outs = best
    ctx.close()
    lat = [o["wall_ms"] for o in outs]
    pairs = sum(o["pairs_within"] for o in outs)
    return {"requests": nreq, "sizes": "n_src, n_tgt uniform in 5000..60000 (seeds 4000+k)", "iterations": 100,
            "wall_s": el, "regs_per_s": nreq / el, "pair_evals_per_s": pairs / el,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "note": "all requests submitted at once; latency = submission to completion"}


def rot_err_deg(T, T_true):
    E = T[:3, :3] @ T_true[:3, :3].T
    return float(np.degrees(np.arccos(np.clip((np.trace(E) - 1) / 2, -1, 1))))


def trans_err_m(T, T_true):
    E = T[:3, :3] @ T_true[:3, :3].T
    return float(np.linalg.norm(T[:3, 3] - E @ T_true[:3, 3]))


def time_registrations(ctx, t, prm, steps, warmup):
    """Wall time of `steps` registrations after `warmup` untimed ones, then the
    same registrations with HIP events around every launch (pair kernel
    average).  Inputs are device tensors."""
    import torch
    for _ in range(warmup):
        ctx.register(*t, prm)
    torch.cuda.synchronize()
    lat, pairs, examined = [], 0, 0
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        out = ctx.register(*t, prm)
        lat.append((time.perf_counter() - s0) * 1e3)
        pairs += out["pairs_within"]
        examined += out["pairs_examined"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.kernel_stats(reset=True)
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    te0 = time.perf_counter()
    for _ in range(steps):
        ctx.register(*t, prm)
    torch.cuda.synchronize()
    elapsed_ev = time.perf_counter() - te0
    ctx.set_profiling(False)
    ks = ctx.kernel_stats(reset=True)
    return {"out": out, "elapsed": elapsed, "lat": lat, "pairs": pairs, "examined": examined, "ks": ks,
            "elapsed_ev": elapsed_ev}


def roofline_of(ks, traffic):
    achieved = FLOPS_PER_PAIR * ks["pairs"] / (ks["ms"] * 1e-3) / 1e12 if ks["ms"] > 0 else 0.0
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS, "traffic": traffic,
            "kernel": "k_pairs<float,5,true,false>", "kernel_ms_avg": ks["ms"] / max(1, ks["launches"]),
            "launches": ks["launches"], "flops_per_pair": FLOPS_PER_PAIR,
            "pairs_per_launch": ks["pairs"] / max(1, ks["launches"]),
            "peak_unpacked": PEAK_UNPACKED_TFLOPS, "frac_of_unpacked": achieved / PEAK_UNPACKED_TFLOPS,
            "peak_note": "peak = published FP32 vector rate (packed FP32); peak_unpacked = the issue ceiling "
                         "without packed FP32 (256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz), which the "
                         "kernels do not use",
            "prepare_kernel_ms_avg": ks["prepare_ms"] / max(1, ks["launches"])}


def oracle_sample(pair, golden, ctx, t, iters=SAMPLE_ITERS):
    """The FP64 oracle (grid enumeration, all host threads) at the oracle
    trajectory's poses of `iters`: the CPU baseline's timing, and the GPU's
    F, omega, v at the same poses against it (teacher-forced parity).  Also a
    one-thread rate and the brute-force enumeration's rate, each on a sample
    of targets."""
    import oracle
    from paper_1904_02266_amd import Params
    tr = np.array(golden["trace"])
    a2 = golden["a2"]
    nth = oracle.default_threads()
    t_cpu, p_cpu, worst = 0.0, 0, 0.0
    for k in iters:
        Tk = np.eye(4) if k == 0 else tr[k - 1, 10:26].reshape(4, 4)
        ell = tr[k, 8]
        c0 = time.perf_counter()
        r = oracle.eval(pair.src_xyz, pair.src_feat, pair.tgt_xyz, pair.tgt_feat, Tk, ell=ell, kappa=3.0, a2=a2,
                        nthreads=nth, grid=True)
        t_cpu += time.perf_counter() - c0
        p_cpu += r["within"]
        g = ctx.eval(*t, Tk, Params(stage_ell=(ell,), cutoff_mult=3.0, a2=a2))
        err = max([abs(g[0] - r["g"][0]) / r["g"][0]] + [abs(g[q] - r["g"][q]) / r["abs"][q] for q in range(1, 7)])
        worst = max(worst, err)
    # one thread, every 16th target at the last iteration's pose
    k = iters[-1]
    Tk = tr[k - 1, 10:26].reshape(4, 4)
    sel = np.arange(0, pair.tgt_xyz.shape[0], 16, dtype=np.int32)
    c0 = time.perf_counter()
    r1 = oracle.eval(pair.src_xyz, pair.src_feat, pair.tgt_xyz, pair.tgt_feat, Tk, ell=tr[k, 8], kappa=3.0, a2=a2,
                     nthreads=1, grid=True, sel=sel)
    t1 = time.perf_counter() - c0
    # brute force (every pair tested), all threads, every 256th target
    selb = np.arange(0, pair.tgt_xyz.shape[0], 256, dtype=np.int32)
    c0 = time.perf_counter()
    rb = oracle.eval(pair.src_xyz, pair.src_feat, pair.tgt_xyz, pair.tgt_feat, Tk, ell=tr[k, 8], kappa=3.0, a2=a2,
                     nthreads=nth, sel=selb)
    tb = time.perf_counter() - c0
    cpu = {"value": p_cpu / t_cpu, "unit": "pair-evals/s", "cores": nth, "kind": "oracle",
           "sample": f"{len(iters)} of the 100 FP64 evaluations of the registration (oracle grid enumeration of "
                     f"the cutoff pairs) at the oracle trajectory's poses of iterations {list(iters)}, "
                     f"{p_cpu:.3g} pairs in {t_cpu:.1f} s",
           "nproc": os.cpu_count(),
           "one_core": {"value": r1["within"] / t1, "unit": "pair-evals/s", "cores": 1,
                        "sample": f"iteration {k}, every 16th target ({sel.size}), {t1:.1f} s"},
           "brute_force": {"value": rb["within"] / tb, "examined_per_s": rb["examined"] / tb, "unit": "pair-evals/s",
                           "cores": nth, "sample": f"iteration {k}, every 256th target ({selb.size}), every pair "
                                                   f"tested, {tb:.1f} s"}}
    parity = {"max_rel_err": worst, "criterion": "F rel; omega,v abs / oracle sum|terms| (teacher-forced at the "
                                                 "oracle's poses)", "iters": list(iters)}
    return cpu, parity


def rgbd30k(ctx, pair, steps, quartic_steps):
    """The 30k semi-dense RGB-D pair: fixed-step registration (kernel and
    pose error), the same registration over all pairs (no cutoff), and the
    conjugate-direction and quartic step rules (pose error, iterations)."""
    import torch
    from paper_1904_02266_amd import params_rgbd
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(a).to(dev) for a in (pair.src_xyz, pair.src_feat, pair.tgt_xyz, pair.tgt_feat)]
    torch.cuda.synchronize()
    r = time_registrations(ctx, t, params_rgbd(), steps, 2)
    out = r["out"]
    res = {"workload": "640x480 synthetic RGB-D frame pair, 30,000 semi-dense points (highest intensity gradient) "
                       "per frame, cutoff 3 ell, ell 0.2->0.05 m over 4x25 iterations",
           "ms_per_registration": r["elapsed"] * 1e3 / steps,
           "pair_evals_per_s": r["pairs"] / r["elapsed"],
           "pairs_per_registration": r["pairs"] / steps, "pairs_examined_per_registration": r["examined"] / steps,
           "roofline": roofline_of(r["ks"], measured_traffic(os.path.join(ROOT, "profiles",
                                                                          "k_pairs_rgbd30k_traffic.md"))),
           "pose_error_fixed": {"rot_deg": rot_err_deg(out["T"], pair.T_true),
                                "trans_m": trans_err_m(out["T"], pair.T_true)}}
    # all pairs, no cutoff (the pruning's reference)
    rb = time_registrations(ctx, t, params_rgbd(cutoff_mult=0.0), max(2, steps // 4), 1)
    res["bruteforce_no_cutoff"] = {"ms_per_registration": rb["elapsed"] * 1e3 / max(2, steps // 4),
                                   "pairs_per_registration": rb["pairs"] / max(2, steps // 4),
                                   "pair_evals_per_s": rb["pairs"] / rb["elapsed"],
                                   "speedup_of_cutoff": rb["elapsed"] / max(2, steps // 4) /
                                   (r["elapsed"] / steps)}
    for rule in ("conjugate", "quartic"):
        if quartic_steps <= 0:
            break
        prm = params_rgbd(step_rule=rule)
        ctx.register(*t, prm)
        torch.cuda.synchronize()
        q0 = time.perf_counter()
        for _ in range(quartic_steps):
            oq = ctx.register(*t, prm)
        torch.cuda.synchronize()
        q_el = (time.perf_counter() - q0) / quartic_steps
        ctx.kernel_stats(reset=True)
        ctx.set_profiling(True)
        ctx.register(*t, prm)
        ctx.set_profiling(False)
        kq = ctx.kernel_stats(reset=True)
        q_ach = QUARTIC_FLOPS_PER_PAIR * kq["pairs"] / (kq["quartic_ms"] * 1e-3) / 1e12 if kq["quartic_ms"] else 0
        conv = ctx.register(*t, params_rgbd(step_rule=rule, tol=1e-5, max_iters=200))
        res[rule + "_rule"] = {
            "ms_per_registration": q_el * 1e3, "iterations": 100,
            "pose_error": {"rot_deg": rot_err_deg(oq["T"], pair.T_true), "trans_m": trans_err_m(oq["T"], pair.T_true)},
            "quartic_kernel_ms_avg": kq["quartic_ms"] / max(1, kq["launches"]),
            "quartic_pass_roofline": {"achieved": q_ach, "peak": PEAK_TFLOPS, "unit": "TFLOP/s",
                                      "frac": q_ach / PEAK_TFLOPS, "flops_per_pair": QUARTIC_FLOPS_PER_PAIR,
                                      "kernel": "k_pairs<float,5,true,true>"},
            "with_tol_1e-5": {"iters": conv["iters"], "converged": bool(conv["converged"]),
                              "rot_deg": rot_err_deg(conv["T"], pair.T_true),
                              "trans_m": trans_err_m(conv["T"], pair.T_true)}}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-oracle", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--batch", type=int, default=256, help="requests in the batched run (0: skip)")
    ap.add_argument("--quartic-steps", type=int, default=3,
                    help="timed 30k registrations with the conjugate and quartic step rules (0: skip)")
    ap.add_argument("--odometry-frames", type=int, default=8,
                    help="frames of the synthetic odometry sequence (0: skip)")
    ap.add_argument("--serving-window", type=float, default=10.0,
                    help="seconds of Poisson arrivals per serving rate (0: skip)")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline registration, its roofline and the CPU baseline")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated extra legs to run after the headline (default: all of "
                         + ", ".join(LEGS) + ")")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the measurement, copy a MIB-MiB device buffer once (reference dispatch "
                         "of known size for hardware-counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    extra = not args.no_extra
    legs = set(x.strip() for x in args.legs.split(",") if x.strip()) if extra else set()
    unknown = legs - set(LEGS)
    if unknown:
        print(f"bench.py: unknown legs {sorted(unknown)}; choose from {', '.join(LEGS)}", file=sys.stderr)
        sys.exit(2)
    batch_clouds = gen_batch(args.batch if "batched" in legs else 0)
    progress(f"batched inputs drawn ({len(batch_clouds)})")
    serve_pool = gen_serving_pool(6 if (args.serving_window > 0 and "serving" in legs) else 0)
    with ProcessPoolExecutor(max_workers=1) as ex:
        dense_cloud, G = ex.submit(_gen_dense, 3).result()
    odo_frames = None
    if args.odometry_frames > 1 and ("odometry" in legs or "frontend" in legs):
        from paper_1904_02266_amd import synth as _synth
        odo_frames = _synth.rgbd_sequence(args.odometry_frames, seed=9)
    with open(GOLDEN) as f:
        golden = json.load(f)

    import torch
    from paper_1904_02266_amd import Context, params_rgbd, synth

    dev = torch.device("cuda:0")
    pair = synth.CloudPair(*dense_cloud, T_true=G)
    t = [torch.from_numpy(a).to(dev) for a in dense_cloud]
    torch.cuda.synchronize()
    ctx = Context(0)
    prm = params_rgbd()

    # headline: the dense registration, timed region = the registrations alone
    progress("inputs ready")
    r = time_registrations(ctx, t, prm, args.steps, args.warmup)
    out, elapsed, lat, ks = r["out"], r["elapsed"], r["lat"], r["ks"]
    progress(f"headline: {elapsed * 1e3 / args.steps:.1f} ms per registration")

    cpu = parity = None
    if not args.no_oracle:
        cpu, parity = oracle_sample(pair, golden, ctx, t)
        progress(f"oracle sample: {cpu['value']:.3g} pair-evals/s on {cpu['cores']} threads")

    # the same registration with every pair term in FP64
    prm64 = params_rgbd(precision="fp64")
    ctx.register(*t, prm64)
    torch.cuda.synchronize()
    f0 = time.perf_counter()
    n64 = 2
    for _ in range(n64):
        o64 = ctx.register(*t, prm64)
    torch.cuda.synchronize()
    f_el = (time.perf_counter() - f0) / n64
    fp64_path = {"ms_per_registration": f_el * 1e3, "pair_evals_per_s": o64["pairs_within"] / f_el,
                 "speedup_of_mixed": f_el / (elapsed / args.steps),
                 "pose_diff_vs_mixed": {"rot_deg": rot_err_deg(o64["T"], out["T"]),
                                        "trans_m": float(np.linalg.norm(o64["T"][:3, 3] - out["T"][:3, 3]))}}
    To = np.array(golden["trace"])[99, 10:26].reshape(4, 4)
    vs_oracle = {"rot_deg": rot_err_deg(out["T"], To), "trans_m": float(np.linalg.norm(out["T"][:3, 3] - To[:3, 3])),
                 "fp64_rot_deg": rot_err_deg(o64["T"], To),
                 "fp64_trans_m": float(np.linalg.norm(o64["T"][:3, 3] - To[:3, 3]))}

    c2 = batch = serve = dense = fe = c1 = odo = None
    progress("fp64 path done")
    if "rgbd30k" in legs:
        c2 = rgbd30k(ctx, synth.rgbd_pair(30000, 30000, seed=2), max(4, args.steps), args.quartic_steps)
        progress("rgbd 30k done")
    if batch_clouds:
        batch = batched_both(batch_clouds)
        progress("batched done")
    if serve_pool:
        serve = serving(serve_pool, window_s=args.serving_window)
        progress("serving done")
    if "bruteforce" in legs:
        dense = dense_bruteforce(dense_cloud, golden)
        progress("dense brute force done")
    if "frontend" in legs and odo_frames:
        fe = frontend_vga(odo_frames[0])
    if "planes" in legs:
        c1 = planes_c1()
    if "odometry" in legs and odo_frames:
        from paper_1904_02266_amd import odometry, params_table1
        odometry.run_on_device(ctx, odo_frames[:2], params_table1())  # warm-up
        torch.cuda.synchronize()
        o0 = time.perf_counter()
        res = odometry.run_on_device(ctx, odo_frames, params_table1())
        torch.cuda.synchronize()
        o_el = time.perf_counter() - o0
        odo = {"frames": len(odo_frames), "frames_per_s": (len(odo_frames) - 1) / o_el,
               "ms_per_frame": o_el * 1e3 / (len(odo_frames) - 1),
               "params": "Table 1 (quartic step, value floor 1e-3, ell 0.15/0.10/0.06/0.03, thresholds 1e-5/5e-5)",
               "per_frame": "device front end of the new frame (30,000 points) + registration; frames uploaded "
                            "from host memory each step (the images' PCIe copy is inside the timing)",
               "iterations": res.iterations, "relative_error_cdf": res.cdf(),
               "sequence": "synthetic, 640x480, 1 deg / 2 cm per frame, 1% depth noise, seed 9"}

    line = {
        "metric": METRIC,
        "value": r["pairs"] / elapsed,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "dense-300k: 640x480 synthetic RGB-D frame pair, a seeded random subset of 300,000 "
                               "valid pixels per frame, 5 label channels, cutoff 3 ell with voxel grid, "
                               "ell 0.2->0.05 m over 4x25 iterations, fixed step",
                   "points_src": int(dense_cloud[0].shape[0]), "points_tgt": int(dense_cloud[2].shape[0]),
                   "iterations": 100, "precision": "fp32 pair terms, kahan fp32 partials, fp64 reduce+step"},
        "roofline": roofline_of(ks, measured_traffic()),
        "cpu_baseline": cpu,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "pairs_per_registration": r["pairs"] / args.steps,
        "pairs_examined_per_registration": r["examined"] / args.steps,
        "within_cutoff_fraction_of_examined": r["pairs"] / max(1, r["examined"]),
        "instrumented_ms_per_step": r["elapsed_ev"] * 1e3 / args.steps,
        "pose_error": {"rot_deg": rot_err_deg(out["T"], G), "trans_m": trans_err_m(out["T"], G)},
        "final_pose_vs_oracle": vs_oracle,
        "parity": parity,
        "fp64_path": fp64_path,
        "rgbd_30k": c2,
        "batched": batch,
        "serving": serve,
        "dense_300k_bruteforce_eval": dense,
        "frontend_vga": fe,
        "planes_2k": c1,
        "odometry": odo,
    }
    print(json.dumps(line), flush=True)
    ctx.close()
    if args.copy_calibration > 0:
        a = torch.ones(args.copy_calibration * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
        bb = torch.empty_like(a)
        torch.cuda.synchronize()
        bb.copy_(a)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
