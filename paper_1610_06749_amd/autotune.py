"""Launch-shape autotuner for the stepping kernels.

Times every candidate execution choice on the caller's grid and keeps the
fastest per voxel-step:

* single chambers (``tune``): the plain kernel with 64 x 8, 64 x 16 or
  32 x 16 tiles, or 128 x 8 tiles of column pairs (even nx), and the
  temporally blocked kernel at each depth T, each timed
  over whole passes
  (the stepping kernel plus its tally reduction) on a perturbed field of the
  chamber's shape;
* batched sweeps (``tune_batch``): the tile shape and planes per tile of the
  batched kernel and the passes per captured graph, each timed on the batch
  itself with the step count capped.

Results are cached per (grid, device) in memory and, when a path is given,
in a JSON file, so one tuning serves every later run of that shape.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import binding as B

PLAIN = [dict(kernel=B.IT_KERNEL_PLAIN, tile_y=8), dict(kernel=B.IT_KERNEL_PLAIN, tile_y=16),
         dict(kernel=B.IT_KERNEL_PLAIN, tile_x=32)]
PAIR = [dict(kernel=B.IT_KERNEL_PLAIN, tile_x=128)]  # tiles of column pairs: grids with an even nx
# the temporally blocked kernel at each depth with its default rows per
# thread, and the next larger tile that still fits the registers
BLOCKED = [dict(kernel=B.IT_KERNEL_BLOCKED, steps_per_pass=T) for T in (2, 3, 4)] + \
    [dict(kernel=B.IT_KERNEL_BLOCKED, steps_per_pass=2, tile_y=40),
     dict(kernel=B.IT_KERNEL_BLOCKED, steps_per_pass=3, tile_y=24)]

_memo: dict = {}


def _device_name():
    import torch
    return torch.cuda.get_device_name(0)


def _load(path):
    if path and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def _store(path, table):
    if path:
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)


def _perturbed(shape, seed=5, scale=1e9):
    # a smooth positive field with a ripple: the timing does not depend on
    # the values, only on finite, non-trivial data
    rng = np.random.default_rng(seed)
    f = scale * (1.0 + 0.1 * rng.standard_normal(shape))
    f[0] = 0.0
    f[-1] = 0.0
    return f


def time_exec(ch, ex, steps=64, reps=3, dt=None):
    """Seconds per voxel-step of one execution choice on the chamber's grid
    (best of ``reps`` runs of ``steps`` steps through it_advance)."""
    import torch
    shape = (ch["nz"] + 1, ch["ny"], ch["nx"])
    if dt is None:
        dt = B.it_dt(ch, None)
    chk = dict(ch, max_steps=max(steps, 1))
    pos = torch.tensor(_perturbed(shape, 5), device="cuda")
    neg = torch.tensor(_perturbed(shape, 6), device="cuda")
    ws = B.workspace(chk, 0)
    stream = torch.cuda.current_stream()
    B.it_advance(chk, dt, pos, neg, steps, exec=ex, ws=ws, stream=stream)  # warm-up
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        B.it_advance(chk, dt, pos, neg, steps, exec=ex, ws=ws, stream=stream)
        e1.record(stream)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    nint = ch["nx"] * ch["ny"] * (ch["nz"] - 1)
    return best / (steps * nint)


def _kernel_options(ch):
    """The chamber options that select another kernel instance: absorbing
    sides ("a") and the space-charge term ("s")."""
    return ("a" if ch.get("lateral_bc", 0) else "") + ("s" if ch.get("space_charge", 0) else "")


def _batch_options(ch):
    """The kernel options plus a pulse train's pulse count and period, which
    decide the passes a batch can take (a blocked pass holds at most one
    pulse)."""
    opts = _kernel_options(ch)
    if ch.get("n_pulses", 0) >= 2:
        opts += f"p{int(ch['n_pulses'])}/{float(ch['pulse_period_s']):.9g}"
    return opts


def tune(ch, candidates=None, steps=64, cache=None, verbose=False):
    """Best execution choice (an ``exec`` dict for it_solve / it_advance) for
    the chamber's grid.  ``cache``: optional JSON path."""
    key = f"{ch['nx']}x{ch['ny']}x{ch['nz']}{_kernel_options(ch)}@{_device_name()}"
    if key in _memo:
        return dict(_memo[key])
    table = _load(cache)
    if key in table:
        _memo[key] = table[key]["exec"]
        return dict(_memo[key])
    cands = candidates if candidates is not None else PLAIN + (PAIR if ch["nx"] % 2 == 0 else []) + BLOCKED
    timings = []
    for ex in cands:
        try:
            t = time_exec(ch, ex, steps=steps)
        except B.ItError as e:
            if e.code != B.IT_ENOTSUP:  # a depth the grid does not support is skipped
                raise
            continue
        timings.append((t, ex))
        if verbose:
            print(f"autotune {key}: {ex} -> {1.0 / t:.4g} voxel-steps/s", flush=True)
    if not timings:
        raise RuntimeError(f"no candidate execution ran on {key}")
    t_best, ex_best = min(timings, key=lambda p: p[0])
    _memo[key] = dict(ex_best)
    table[key] = {"exec": dict(ex_best), "voxel_steps_per_s": 1.0 / t_best,
                  "all": [[dict(ex), 1.0 / t] for t, ex in timings]}
    _store(cache, table)
    return dict(ex_best)


def batch_candidates(rows=(8,), graph_passes=(32,), z_chunks=(16,), narrow=False,
                     blocked_T=(2, 3), blocked_z=(0, 32), blocked_graph=(32,)):
    """Execution choices tried for a batch: the one-step batched kernel with
    64-column tiles of each of ``rows`` (and 32 x 16 when ``narrow``), each
    planes-per-tile and passes-per-graph choice; and the temporally blocked
    batched kernel at each depth, chunk length (0: the library's choice, no
    cap) and passes per graph."""
    shapes = [dict(tile_y=r, tile_x=64) for r in rows] + ([dict(tile_y=16, tile_x=32)] if narrow else [])
    out = [dict(kernel=B.IT_KERNEL_PLAIN, check_every=g, z_chunk=z, **sh)
           for sh in shapes for g in graph_passes for z in z_chunks]
    out += [dict(kernel=B.IT_KERNEL_BLOCKED, steps_per_pass=T, check_every=g, z_chunk=z)
            for T in blocked_T for g in blocked_graph for z in blocked_z]
    return out


def tune_batch(chs, trs, steps=96, candidates=None, cache=None, verbose=False, **kw):
    """Best ``exec`` for it_solve_batch on these chambers among
    ``candidates`` (default: batch_candidates(**kw)), each timed on the batch
    with every instance's step count capped at ``steps``; a choice the
    batch does not support (IT_ENOTSUP, e.g. blocked passes for a train
    whose period is shorter than a pass) is skipped.  Cached per grids and
    options of the instances."""
    import torch
    sig = "|".join(f"{c['nx']}x{c['ny']}x{c['nz']}{_batch_options(c)}" for c in chs)
    key = f"batch:{len(chs)}:{hashlib.sha256(sig.encode()).hexdigest()[:12]}@{_device_name()}"
    if key in _memo:
        return dict(_memo[key])
    table = _load(cache)
    if key in table:
        _memo[key] = table[key]["exec"]
        return dict(_memo[key])
    capped = [dict(c, max_steps=steps) for c in chs]
    vs = sum(c["nx"] * c["ny"] * (c["nz"] - 1) for c in chs) * steps
    timings = []
    cands = candidates if candidates is not None else batch_candidates(**kw)
    for ex in cands:
        try:
            B.it_solve_batch(capped, trs, exec=ex)  # warm-up
        except B.ItError as e:
            if e.code != B.IT_ENOTSUP:
                raise
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.it_solve_batch(capped, trs, exec=ex)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / vs
        timings.append((t, ex))
        if verbose:
            print(f"autotune {key}: {ex} -> {1.0 / t:.4g} voxel-steps/s", flush=True)
    if not timings:
        raise RuntimeError(f"no candidate execution ran on {key}")
    t_best, ex_best = min(timings, key=lambda p: p[0])
    _memo[key] = dict(ex_best)
    table[key] = {"exec": dict(ex_best), "voxel_steps_per_s": 1.0 / t_best,
                  "all": [[dict(ex), 1.0 / t] for t, ex in timings]}
    _store(cache, table)
    return dict(ex_best)
