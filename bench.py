"""Benchmark of the recombination solver on one MI355X.

One "step" is one whole run of the method on the pulsed-beam chamber
(256 x 256 x 200 nodes, spacing 5e-4 cm, gap 0.1 cm at 200 V, one
instantaneous pulse of 400 parallel Gaussian tracks): time step selection,
track deposition, explicit stepping with per-step tallies until every ion is
collected (or recombined), and the result f.  Inputs are synthetic and
seeded; the track list and the workspace are resident before timing.

Printed: one JSON line with voxel-steps/s (one voxel-step = both ion species
updated at one interior node for one time step), the roofline of the
stepping kernel (algorithmic bytes per launch over its average launch time,
measured here with HIP events on the stream the kernel runs on) and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-steps/s + % HBM peak; k_s evals/s surrogate vs solver at 0.1% err"
PEAK_HBM_GBS = 8000.0
BYTES_PER_VOXEL_STEP = 32.0  # read + write of two FP64 species per node and step


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kernel", choices=("auto", "plain", "blocked"), default="auto")
    ap.add_argument("--T", type=int, default=0, help="steps per pass of the blocked kernel")
    ap.add_argument("--tile-y", type=int, default=0, help="tile rows (0 = default)")
    ap.add_argument("--tile-x", type=int, default=0,
                    help="tile columns of the one-step kernel: 32, 64 or 128 (column pairs); 0 = default")
    ap.add_argument("--z-chunk", type=int, default=0, help="planes per tile of the one-step kernel (0 = default)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--kernel-steps", type=int, default=200,
                    help="launches in the stepping-kernel timing")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only run the stepping kernel on the workload grid (for counter runs)")
    ap.add_argument("--variant", choices=("none", "space-charge", "free-electrons"), default="none",
                    help="with --kernel-only: the space-charge stepping instance, or a free-electron run "
                         "(uniform dose, electron phase then ions) on the workload grid")
    ap.add_argument("--no-sweep", action="store_true", help="skip the batched 96-chamber sweep")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate experiment")
    ap.add_argument("--surrogate-train", type=int, default=32768, help="surrogate training samples")
    ap.add_argument("--surrogate-steps", type=int, default=600000, help="surrogate training steps")
    ap.add_argument("--continuous-ms", type=float, default=0.4,
                    help="beam-on time of the continuous-beam run (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy two fields of the workload grid with a plain device copy "
                         "(reference for the HBM byte counters)")
    return ap.parse_args()


def kernel_source_hash(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1610_06749_amd", "csrc", n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_name, workload, src_hash, shape):
    """HBM bytes per launch from the committed counter summary, or None when
    no summary exists, it was taken with another launch shape, or the kernel
    source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_name}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != src_hash or not vals.get("launch_shape", "").startswith(shape):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(ch, tr):
    """The CPU oracle (single-threaded plain C) on a bounded sample of the
    same workload: deposition of 16 of the 400 tracks and 40 steps of the
    full grid, scaled to one whole run."""
    import numpy as np

    import oracle
    dt = oracle.dt(ch)
    nint = (ch["nz"] - 1) * ch["nx"] * ch["ny"]
    t0 = time.perf_counter()
    pos, neg, _ = oracle.deposit(ch, tr[:16], 0, dt)
    t_dep = (time.perf_counter() - t0) / 16.0
    nsteps = 40
    t0 = time.perf_counter()
    oracle.advance(ch, dt, pos, neg, nsteps)
    t_step = (time.perf_counter() - t0) / nsteps
    return t_dep, t_step, nint, np


def continuous_run(it, W, beam_s):
    """The continuous beam (512 x 512 x 256 nodes, tilted tracks arriving as
    a Poisson process, 4 of them at t = 0) with the beam on for beam_s, then
    off until every ion is collected: f and the collected current
    I_l = q (C+_l + C-_l) / (2 dt) (both electrodes, both species)."""
    import numpy as np
    import torch
    ch, tr = W.continuous_beam(duration_s=beam_s)
    ws = it.workspace(ch, tr.shape[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = it.it_solve(ch, tr, ws=ws, trace=True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    trc = r["trace"]
    dt = r["dt"]
    q = 1.602176634e-19
    cur = q * (trc[:, 1] + trc[:, 2] + trc[:, 3] + trc[:, 4]) / (2.0 * dt)
    on = int(min(len(cur), math.ceil(beam_s / dt)))
    nint = ch["nx"] * ch["ny"] * (ch["nz"] - 1)
    return {"workload": f"continuous beam 512x512x256, beam on {beam_s * 1e3:g} ms then off to collection",
            "tracks": int(tr.shape[0]), "steps": r["steps"], "dt": dt, "f": r["f"], "ks": r["ks"],
            "flags": r["flags"], "seconds": sec, "voxel_steps_per_s": r["steps"] * nint / sec,
            "current_mean_beam_on_A": float(cur[:on].mean()) if on else 0.0,
            "current_peak_A": float(cur.max()), "charge_collected_C": float(cur.sum() * dt),
            "current_trace_points": int(len(cur))}


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(msg, file=sys.stderr, flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1610_06749_amd as it
    import workloads as W

    torch.cuda.set_device(0)
    ch, tr = W.pulsed_beam()
    if a.copy_calibration:
        shape = (ch["nz"] + 1, ch["ny"], ch["nx"])
        src = torch.ones((2,) + shape, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8}))
        return
    kernel = {"auto": it.IT_KERNEL_AUTO, "plain": it.IT_KERNEL_PLAIN, "blocked": it.IT_KERNEL_BLOCKED}[a.kernel]
    ex = {"kernel": kernel, "steps_per_pass": a.T, "tile_y": a.tile_y, "tile_x": a.tile_x, "z_chunk": a.z_chunk}
    ws = it.workspace(ch, tr.shape[0])
    nint = (ch["nz"] - 1) * ch["nx"] * ch["ny"]
    stream = torch.cuda.current_stream()

    if a.kernel_only and a.variant == "free-electrons":
        che = dict(ch, uniform_n0=3e9, attach_coeff=5.0, mu_e=1500.0, D_e=1500.0 * 0.02526,
                   max_steps=max(a.kernel_steps, 1))
        r = it.it_solve(che, W.no_tracks())
        torch.cuda.synchronize()
        print(json.dumps({"free_electron_run": {k: r[k] for k in ("e_steps", "steps", "flags", "f")}}))
        return
    if a.kernel_only and a.variant == "space-charge":
        ch = dict(ch, space_charge=1)
    if a.kernel_only:
        dt = it.it_dt(ch, tr)
        pos0, neg0 = W.perturbed_field((ch["nz"] + 1, ch["ny"], ch["nx"]), seed=5, scale=1e9)
        gp, gn = torch.tensor(pos0, device="cuda"), torch.tensor(neg0, device="cuda")
        chk = dict(ch, max_steps=max(a.kernel_steps, 1))
        it.it_advance(chk, dt, gp, gn, a.kernel_steps, exec=ex, ws=it.workspace(chk, 0))
        torch.cuda.synchronize()
        print(json.dumps({"kernel_only_steps": a.kernel_steps, "nodes": nint}))
        return
    for _ in range(a.warmup):
        it.it_solve(ch, tr, exec=ex, ws=ws)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        results.append(it.it_solve(ch, tr, exec=ex, ws=ws))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    voxel_steps = sum(r["steps"] for r in results) * nint
    r0 = results[0]
    value = voxel_steps / elapsed
    progress(f"pulsed beam: {a.steps} timed runs of {r0['steps']} steps, {elapsed / a.steps * 1e3:.1f} ms each")

    # Stepping kernel alone: K launches minus 1 launch of it_advance on the
    # same grid, bracketed by HIP events on the stream the kernel runs on.
    dt = r0["dt"]
    pos0, neg0 = W.perturbed_field((ch["nz"] + 1, ch["ny"], ch["nx"]), seed=5, scale=1e9)
    gp = torch.tensor(pos0, device="cuda")
    gn = torch.tensor(neg0, device="cuda")
    chk = dict(ch, max_steps=max(a.kernel_steps, 1))
    wsk = it.workspace(chk, 0)

    T_pass = 1 if kernel == it.IT_KERNEL_PLAIN or a.T <= 1 else a.T
    launches = max(a.kernel_steps // T_pass, 2)
    kname = "step_plain" if T_pass == 1 else f"step_blocked_T{T_pass}"
    src = ["kernels_plain.hip", "stencil_plain.h", "reduce.h", "internal.h"] if T_pass == 1 else \
        ["kernels_blocked.hip", "reduce.h", "internal.h"]

    def timed_advance(n, timer=None):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        exn = dict(ex, timing_events=timer) if timer is not None else ex
        e0.record(stream)
        it.it_advance(chk, dt, gp, gn, n, exec=exn, ws=wsk, stream=stream)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3

    # one pass = the stepping kernel plus its tally reduction.  The library
    # records HIP events on the run's stream: one before the first and one
    # after the last stepping launch (the timed region), and, separately, a
    # pair around every launch (each pair adds its own overhead)
    timed_advance(launches * T_pass)
    t_pass = min(timed_advance(launches * T_pass) for _ in range(3)) / launches
    span = it.KernelTimer(span=True)
    timed_advance(launches * T_pass, span)
    per_launch = float(span.durations()[0]) / launches
    timer = it.KernelTimer(launches)
    timed_advance(launches * T_pass, timer)
    d = timer.durations()[1:]  # the first launch pays the cold start
    bytes_per_launch = BYTES_PER_VOXEL_STEP * nint * T_pass  # compulsory traffic of one pass
    achieved = bytes_per_launch / per_launch / 1e9
    workload_name = "pulsed_256x256x200"
    shape = f"tile_x {a.tile_x} tile_y {16 if a.tile_y == 16 else 8} z_chunk {a.z_chunk}" if T_pass == 1 else \
        f"T {T_pass}"
    traffic = read_traffic(kname, workload_name, kernel_source_hash(src), shape)
    progress(f"{kname}: {per_launch * 1e6:.1f} us per launch")

    cpu = None
    if not a.no_cpu:
        t_dep, t_step, nint_c, _ = cpu_baseline(ch, tr)
        steps_full = r0["steps"]
        t_run = t_dep * tr.shape[0] + t_step * steps_full
        cpu = {"value": nint_c * steps_full / t_run, "unit": "voxel-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"single-threaded C oracle: deposit of 16 of the 400 tracks "
                         f"({t_dep * 16:.1f} s) and 40 steps of the full 256x256x200 grid "
                         f"({t_step * 40:.1f} s), scaled to one whole run of {steps_full} steps"}
        progress("cpu baseline done")

    sweep = None
    if not a.no_sweep:
        chs, trs = W.batched_sweep()
        it.it_solve_batch(chs[:4], trs[:4])  # warm-up (graph instantiation path)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = it.it_solve_batch(chs, trs)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        vs = sum(r["steps"] * c["nx"] * c["ny"] * (c["nz"] - 1) for r, c in zip(res, chs))
        sweep = {"workload": "96 chambers, transverse 64-256, gap 50-250 intervals, 50-400 V, "
                             "LET 1-500 keV/um, 1-500 tracks and 0.01-1 mGy per pulse",
                 "seconds": sec, "voxel_steps": vs, "voxel_steps_per_s": vs / sec,
                 "ks_evals_per_s": len(chs) / sec, "max_steps": max(r["steps"] for r in res),
                 "flags": sorted({r["flags"] for r in res})}
        progress(f"sweep: {sec:.1f} s")

    cont = None
    if a.continuous_ms > 0:
        cont = continuous_run(it, W, a.continuous_ms * 1e-3)
        progress(f"continuous beam: {cont['seconds']:.1f} s")

    sur = None
    if not a.no_surrogate:
        from paper_1610_06749_amd import surrogate
        sur = surrogate.evaluate(n_train=a.surrogate_train, steps=a.surrogate_steps, log=progress)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "pulsed beam: 256x256x200 nodes, 400 parallel tracks, one pulse, "
                               "run to full collection",
                   "time_steps_per_run": r0["steps"], "f": r0["f"], "ks": r0["ks"],
                   "kernel": kname},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": kname, "launch_ms": per_launch * 1e3, "launches_timed": launches,
                     "launch_ms_event_pairs": float(d.mean()) * 1e3,
                     "pass_ms_with_tally_reduction": t_pass * 1e3,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "cpu_baseline": cpu,
        "sweep": sweep,
        "continuous": cont,
        "surrogate": sur,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
