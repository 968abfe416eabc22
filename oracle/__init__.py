"""CPU oracle for the recombination solver -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The product path (the GPU
library and its Python binding) never imports, links or runs it.

* ``oracle.c`` (built to ``liboracle.so`` with plain gcc, no fast-math) holds
  the solver itself, in FP64, written as plain loops from the paper.
* ``closed_forms.py`` holds the paper's analytic theories (Jaffe, Boag) used to
  pin the solver.
* ``mlp.py`` holds the FP64 reference network for the surrogate kernels.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# Timing build of the same source: the plane loops shared among OpenMP
# threads.  Every grid sum goes through per-plane partial sums added in plane
# order, so it returns the same bits as the single-threaded build (a CPU test
# checks this).
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared"]

P_KEYS = ("dx", "dy", "gap", "voltage", "mu_pos", "mu_neg", "D_pos", "D_neg",
          "alpha", "W_eV", "dt_safety", "stop_tol", "uniform_n0", "space_charge", "reaction_limit",
          "attach_coeff", "mu_e", "D_e", "lateral_bc", "n_pulses", "pulse_period_s")
_OPTIONAL = ("space_charge", "reaction_limit", "attach_coeff", "mu_e", "D_e", "lateral_bc", "n_pulses",
             "pulse_period_s")
E_KEYS = ("e_released", "e_collected_anode", "e_collected_cathode", "e_recombined", "e_steps", "e_dt",
          "e_left", "released_neg_charge")
E_TRACE_KEYS = ("recombined_pn", "recombined_pe", "pos_anode", "pos_cathode", "neg_anode", "neg_cathode",
                "e_anode", "e_cathode", "pos_inflight", "neg_inflight", "e_inflight", "pos_abs", "neg_abs",
                "e_abs")
R_KEYS = ("f", "ks", "f_R", "n_released", "n_recombined", "n_inflight_pos",
          "n_inflight_neg", "col_pos_anode", "col_pos_cathode", "col_neg_anode",
          "col_neg_cathode", "dt", "steps", "flags", "max_beta_n", "n_space_charge_pos",
          "n_space_charge_neg", "n_released_neg", "n_escaped_pos", "n_escaped_neg", "pulses",
          "period_released", "period_collected", "period_recombined")
TRACE_KEYS = ("recombined", "pos_anode", "pos_cathode", "neg_anode", "neg_cathode",
              "pos_inflight", "neg_inflight", "pos_abs", "neg_abs", "released", "pos_space_charge",
              "neg_space_charge", "released_neg", "pos_escaped", "neg_escaped")
NT = len(TRACE_KEYS)

FLAG_MAX_STEPS, FLAG_NONFINITE, FLAG_REACTION, FLAG_EMPTY = 1, 2, 4, 8


def _stale(path):
    return not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE arithmetic, no FMA):
    the single-threaded build and the OpenMP timing build."""
    for path, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or _stale(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", *_CFLAGS, *extra, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIB


_libs = {}
_threaded = False


def use_threads(flag: bool) -> None:
    """Route every following call to the OpenMP build (True) or to the
    single-threaded build (False, the default).  Both give the same bits."""
    global _threaded
    _threaded = bool(flag)


def threads() -> int:
    """Threads the current build's plane loops use."""
    return int(lib().orc_threads())


def lib():
    key = "omp" if _threaded else "plain"
    if key not in _libs:
        build()
        L = ctypes.CDLL(_LIB_OMP if _threaded else _LIB)
        L.orc_threads.argtypes = []
        L.orc_threads.restype = ctypes.c_int
        L.orc_electron_dt.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int64]
        L.orc_electron_dt.restype = ctypes.c_double
        L.orc_step3.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                ctypes.c_double] + [ctypes.POINTER(ctypes.c_double)] * 7
        L.orc_step3.restype = None
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.orc_dt.argtypes = [dp, i64, i64, i64, dp, i64, dp]
        L.orc_reference_density.argtypes = [dp, i64, i64, dp, i64]
        L.orc_reference_density.restype = ctypes.c_double
        L.orc_dt.restype = ctypes.c_int
        L.orc_weights.argtypes = [dp, i64, ctypes.c_double, ctypes.c_int, dp]
        L.orc_weights.restype = None
        L.orc_deposit.argtypes = [dp, i64, i64, i64, dp, i64, i64, ctypes.c_double, dp, dp, dp]
        L.orc_deposit.restype = None
        L.orc_uniform.argtypes = [dp, i64, i64, i64, ctypes.c_double, dp, dp]
        L.orc_uniform.restype = ctypes.c_double
        L.orc_step.argtypes = [dp, i64, i64, i64, ctypes.c_double, dp, dp, dp, dp, dp]
        L.orc_step.restype = None
        L.orc_solve.argtypes = [dp, i64, i64, i64, dp, i64, i64, dp, dp, dp, dp]
        L.orc_solve.restype = ctypes.c_int
        L.orc_advance.argtypes = [dp, i64, i64, i64, ctypes.c_double, i64, dp, dp, dp]
        L.orc_advance.restype = ctypes.c_int
        L.orc_solve_free_electrons.argtypes = [dp, i64, i64, i64, dp, i64, i64, dp, dp, dp, dp, dp, dp]
        L.orc_solve_free_electrons.restype = ctypes.c_int
        L.orc_free_fraction.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_free_fraction.restype = ctypes.c_double
        _libs[key] = L
    return _libs[key]


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _params(ch):
    return np.array([float(ch.get(k, 0.0)) if k in _OPTIONAL else float(ch[k]) for k in P_KEYS],
                    dtype=np.float64)


def _shape(ch):
    return (ch["nz"] + 1, ch["ny"], ch["nx"])


TRACK_COLS = 8  # let, b, x, y, theta, phi, t, b_neg (0: the negative ions share b)


def _trk(tracks):
    """Track rows as the C code reads them: 8 columns (7-column rows get
    b_neg = 0)."""
    if tracks is None:
        return np.zeros((0, TRACK_COLS))
    a = np.asarray(tracks, dtype=np.float64)
    a = a.reshape(-1, a.shape[-1] if a.ndim > 1 else 7)
    if a.shape[1] == 7:
        a = np.concatenate([a, np.zeros((a.shape[0], 1))], axis=1)
    return np.ascontiguousarray(a)


def reference_density(ch, tracks) -> float:
    tr = _trk(tracks)
    return lib().orc_reference_density(_ptr(_params(ch)), ch["nx"], ch["ny"], _ptr(tr), tr.shape[0])


def dt(ch, tracks=None) -> float:
    """Time step for this chamber and track list (the track list only
    matters through the recombination bound)."""
    out = np.zeros(1)
    tr = _trk(tracks)
    rc = lib().orc_dt(_ptr(_params(ch)), ch["nx"], ch["ny"], ch["nz"], _ptr(tr), tr.shape[0], _ptr(out))
    if rc:
        raise ValueError("no stable time step: neither drift nor diffusion constrains dt")
    return float(out[0])


def free_fraction(a, d) -> float:
    """p of eq. free_elec."""
    return lib().orc_free_fraction(float(a), float(d))


def electron_dt(ch) -> float:
    """Largest electron step of eq. vNeum (mu_e, D_e), without kappa."""
    return float(lib().orc_electron_dt(_ptr(_params(ch)), ch["nz"]))


def step3(ch, dt_, pos, neg, ele):
    """One electron-phase step of the three carriers; returns (new_pos,
    new_neg, new_ele, tally dict with keys E_TRACE_KEYS)."""
    pos, neg, ele = (np.ascontiguousarray(a, dtype=np.float64) for a in (pos, neg, ele))
    outs = [np.zeros_like(pos) for _ in range(3)]
    tally = np.zeros(len(E_TRACE_KEYS))
    lib().orc_step3(_ptr(_params(ch)), ch["nx"], ch["ny"], ch["nz"], dt_, _ptr(pos), _ptr(neg), _ptr(ele),
                    _ptr(outs[0]), _ptr(outs[1]), _ptr(outs[2]), _ptr(tally))
    return outs[0], outs[1], outs[2], dict(zip(E_TRACE_KEYS, tally))


def weights(ch, dt_, species: int):
    """(c, sx, sy, sz) of the Appendix for species 0 (positive) or 1 (negative)."""
    out = np.zeros(4)
    lib().orc_weights(_ptr(_params(ch)), ch["nz"], dt_, species, _ptr(out))
    return tuple(out)


def deposit(ch, tracks, step: int, dt_, pos=None, neg=None):
    """Deposit the tracks due at ``step`` into (pos, neg); returns (pos, neg, released)."""
    shape = _shape(ch)
    pos = np.zeros(shape) if pos is None else pos
    neg = np.zeros(shape) if neg is None else neg
    tr = _trk(tracks)
    rel = np.zeros(2)
    lib().orc_deposit(_ptr(_params(ch)), ch["nx"], ch["ny"], ch["nz"], _ptr(tr),
                      tr.shape[0], int(step), dt_, _ptr(pos), _ptr(neg), _ptr(rel))
    return pos, neg, (float(rel[0]) if rel[0] == rel[1] else (float(rel[0]), float(rel[1])))


def uniform(ch, n0, pos=None, neg=None):
    shape = _shape(ch)
    pos = np.zeros(shape) if pos is None else pos
    neg = np.zeros(shape) if neg is None else neg
    rel = lib().orc_uniform(_ptr(_params(ch)), ch["nx"], ch["ny"], ch["nz"], float(n0),
                            _ptr(pos), _ptr(neg))
    return pos, neg, rel


def step(ch, dt_, pos, neg):
    """One step; returns (new_pos, new_neg, tally dict)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    neg = np.ascontiguousarray(neg, dtype=np.float64)
    npos, nneg = np.zeros_like(pos), np.zeros_like(neg)
    tally = np.zeros(NT)
    lib().orc_step(_ptr(_params(ch)), ch["nx"], ch["ny"], ch["nz"], dt_, _ptr(pos), _ptr(neg),
                   _ptr(npos), _ptr(nneg), _ptr(tally))
    return npos, nneg, dict(zip(TRACE_KEYS, tally))


def advance(ch, dt_, pos, neg, nsteps: int, with_trace: bool = False):
    """Advance copies of (pos, neg) by nsteps without deposits."""
    pos = np.array(pos, dtype=np.float64, order="C", copy=True)
    neg = np.array(neg, dtype=np.float64, order="C", copy=True)
    trace = np.zeros((nsteps, NT)) if with_trace else None
    rc = lib().orc_advance(_ptr(_params(ch)), ch["nx"], ch["ny"], ch["nz"], dt_, int(nsteps),
                           _ptr(pos), _ptr(neg), _ptr(trace))
    if rc:
        raise MemoryError("oracle advance failed")
    return (pos, neg, trace) if with_trace else (pos, neg)


def solve(ch, tracks, with_trace: bool = False, with_fields: bool = True):
    """Full run; returns a dict of the result, plus 'trace' [steps, NT] and
    the final fields 'pos', 'neg' of shape (nz+1, ny, nx).  Trace columns are
    ``TRACE_KEYS``."""
    tr = _trk(tracks)
    shape = _shape(ch)
    pos, neg = np.zeros(shape), np.zeros(shape)
    ms = int(ch["max_steps"])
    trace = np.zeros((ms, NT)) if with_trace else None
    res = np.zeros(len(R_KEYS))
    fe = float(ch.get("mu_e", 0.0)) > 0.0
    if fe:  # free-electron component: electron phase, then the ions
        res_e = np.zeros(len(E_KEYS))
        trace_e = np.zeros((ms, len(E_TRACE_KEYS))) if with_trace else None
        rc = lib().orc_solve_free_electrons(_ptr(_params(ch)), ch["nx"], ch["ny"], ch["nz"], _ptr(tr),
                                            tr.shape[0], ms, _ptr(pos), _ptr(neg), _ptr(trace), _ptr(res),
                                            _ptr(res_e), _ptr(trace_e))
    else:
        rc = lib().orc_solve(_ptr(_params(ch)), ch["nx"], ch["ny"], ch["nz"], _ptr(tr), tr.shape[0],
                             ms, _ptr(pos), _ptr(neg), _ptr(trace), _ptr(res))
    if rc == -2:
        raise ValueError("no stable time step")
    if rc == -3:
        raise ValueError("free electrons need an instantaneous pulse, no space charge, periodic lateral "
                         "boundaries and no pulse train; a pulse train needs every track at t = 0")
    if rc == -1 and not fe:
        raise ValueError("invalid pulse train: the period must be positive and at least one step")
    if rc:
        raise MemoryError("oracle solve failed")
    out = dict(zip(R_KEYS, res.tolist()))
    if fe:
        out.update(zip(E_KEYS, res_e.tolist()))
        out["e_steps"] = int(out["e_steps"])
        if with_trace:
            out["trace_e"] = trace_e[: out["e_steps"]].copy()
    out["steps"] = int(out["steps"])
    out["flags"] = int(out["flags"])
    out["pulses"] = int(out["pulses"])
    if with_trace:
        out["trace"] = trace[: out["steps"]].copy()
    if with_fields:
        out["pos"], out["neg"] = pos, neg
    return out
