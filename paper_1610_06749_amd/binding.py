"""Thin ctypes binding of ``libiontracks.so`` (the C ABI of include/iontracks.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides device memory (workspace and field tensors) and the HIP
stream.  The functions carry the C names; chambers are the dictionaries of
``workloads`` and track lists are float64 arrays of shape (n, 7) or (n, 8) whose rows
have the layout of ``it_track``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libiontracks.so")

IT_OK, IT_EINVAL, IT_ENODT, IT_EWORKSPACE, IT_EHIP, IT_ENOTSUP = 0, -1, -2, -3, -4, -5
IT_FLAG_MAX_STEPS, IT_FLAG_NONFINITE, IT_FLAG_REACTION, IT_FLAG_EMPTY = 1, 2, 4, 8
IT_TRACE_COLS = 15
IT_KERNEL_AUTO, IT_KERNEL_PLAIN, IT_KERNEL_BLOCKED = 0, 1, 2
TRACE_KEYS = ("recombined", "pos_anode", "pos_cathode", "neg_anode", "neg_cathode",
              "pos_inflight", "neg_inflight", "pos_abs", "neg_abs", "released", "pos_space_charge",
              "neg_space_charge", "released_neg", "pos_escaped", "neg_escaped")


class ItError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {it_strerror(code)} (status {code})")


class it_chamber(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("space_charge", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("gap", ctypes.c_double),
                ("voltage", ctypes.c_double), ("mu_pos", ctypes.c_double), ("mu_neg", ctypes.c_double),
                ("D_pos", ctypes.c_double), ("D_neg", ctypes.c_double), ("alpha", ctypes.c_double),
                ("W_eV", ctypes.c_double), ("dt_safety", ctypes.c_double), ("stop_tol", ctypes.c_double),
                ("uniform_n0", ctypes.c_double), ("reaction_limit", ctypes.c_double),
                ("attach_coeff", ctypes.c_double), ("mu_e", ctypes.c_double), ("D_e", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("lateral_bc", ctypes.c_int32), ("n_pulses", ctypes.c_int32),
                ("pulse_period_s", ctypes.c_double)]


class it_result(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in (
        "f", "ks", "f_R", "n_released", "n_recombined", "n_inflight_pos", "n_inflight_neg",
        "col_pos_anode", "col_pos_cathode", "col_neg_anode", "col_neg_cathode", "dt", "max_beta_n",
        "n_space_charge_pos", "n_space_charge_neg", "n_released_neg", "e_released", "e_collected_anode",
        "e_collected_cathode", "e_recombined", "e_left", "e_dt", "released_neg_charge", "n_escaped_pos",
        "n_escaped_neg")] + \
        [("e_steps", ctypes.c_int64), ("steps", ctypes.c_int64), ("flags", ctypes.c_int32),
         ("passes", ctypes.c_int32), ("pulses", ctypes.c_int32), ("reserved", ctypes.c_int32),
         ("period_released", ctypes.c_double), ("period_collected", ctypes.c_double),
         ("period_recombined", ctypes.c_double)]


class it_exec(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("steps_per_pass", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("timing_events", ctypes.POINTER(ctypes.c_void_p)), ("n_timing_events", ctypes.c_int32),
                ("z_chunk", ctypes.c_int32), ("timing_span", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("host_buffer", ctypes.c_void_p), ("host_buffer_bytes", ctypes.c_size_t)]


_lib = None


def lib():
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        chp = ctypes.POINTER(it_chamber)
        L.it_strerror.argtypes = [ctypes.c_int]
        L.it_strerror.restype = ctypes.c_char_p
        L.it_dt.argtypes = [chp, vp, i64, dp]
        L.it_validate.argtypes = [chp, vp, i64]
        L.it_workspace_size.argtypes = [chp, i64, ctypes.POINTER(ctypes.c_size_t)]
        L.it_host_buffer_size.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.it_solve.argtypes = [chp, vp, i64, ctypes.POINTER(it_exec), vp, ctypes.c_size_t, vp, vp, vp, vp,
                               ctypes.POINTER(it_result)]
        L.it_advance.argtypes = [chp, ctypes.c_double, i64, ctypes.POINTER(it_exec), vp, vp, vp,
                                 ctypes.c_size_t, vp, vp]
        L.it_workspace_size_batch.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(it_exec),
                                              ctypes.POINTER(ctypes.c_size_t)]
        L.it_solve_batch.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.POINTER(it_exec), vp, ctypes.c_size_t,
                                     vp, vp]
        szp = ctypes.POINTER(ctypes.c_size_t)
        L.it_mlp_model_bytes.argtypes = [ctypes.c_int32, szp]
        L.it_mlp_init.argtypes = [vp, ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp]
        L.it_mlp_baseline.argtypes = [vp, vp, i64, vp, vp]
        L.it_mlp_train_ws_bytes.argtypes = [ctypes.c_int32, i64, szp]
        L.it_mlp_grad.argtypes = [vp, ctypes.c_int32, vp, vp, i64, vp, vp, vp, ctypes.c_size_t, vp]
        L.it_mlp_train.argtypes = [vp, ctypes.c_int32, vp, vp, i64, i64, ctypes.c_int32, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_int32, vp, vp, ctypes.c_size_t, vp]
        L.it_mlp_query_ws_bytes.argtypes = [i64, szp]
        L.it_mlp_query.argtypes = [vp, vp, i64, ctypes.c_float, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.it_mlp_query_static.argtypes = [vp, vp, i64, ctypes.c_float, vp, vp, vp, vp, vp, vp]
        for name in ("it_dt", "it_validate", "it_workspace_size", "it_host_buffer_size", "it_solve", "it_advance",
                     "it_workspace_size_batch", "it_solve_batch", "it_mlp_model_bytes", "it_mlp_init",
                     "it_mlp_train_ws_bytes", "it_mlp_grad", "it_mlp_train", "it_mlp_query_ws_bytes",
                     "it_mlp_query", "it_mlp_query_static", "it_mlp_baseline"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def it_strerror(code: int) -> str:
    return lib().it_strerror(int(code)).decode()


def _chamber(ch) -> it_chamber:
    c = it_chamber()
    for k in ("nx", "ny", "nz", "max_steps"):
        setattr(c, k, int(ch[k]))
    for k in ("dx", "dy", "gap", "voltage", "mu_pos", "mu_neg", "D_pos", "D_neg", "alpha", "W_eV",
              "dt_safety", "stop_tol", "uniform_n0"):
        setattr(c, k, float(ch[k]))
    for k in ("reaction_limit", "attach_coeff", "mu_e", "D_e"):  # optional keys
        setattr(c, k, float(ch.get(k, 0.0)))
    c.space_charge = int(ch.get("space_charge", 0))
    c.lateral_bc = int(ch.get("lateral_bc", 0))
    c.n_pulses = int(ch.get("n_pulses", 0))
    c.pulse_period_s = float(ch.get("pulse_period_s", 0.0))
    return c


TRACK_COLS = 8  # it_track: let, b, x, y, theta, phi, t, b_neg (0: the negative ions share b)


def _track_rows(tracks):
    """Track rows as the C ABI's it_track: 8 doubles (7-column rows get
    b_neg = 0)."""
    a = np.asarray(tracks, dtype=np.float64)
    a = a.reshape(-1, a.shape[-1] if a.ndim > 1 else 7)
    if a.shape[1] == 7:
        a = np.concatenate([a, np.zeros((a.shape[0], 1))], axis=1)
    if a.shape[1] != TRACK_COLS:
        raise ValueError("track rows need 7 or 8 columns")
    return np.ascontiguousarray(a)


def _tracks(tracks):
    tr = _track_rows(tracks)
    return tr, (tr.ctypes.data if tr.shape[0] else None)


def it_host_buffer_size(ninst: int = 1) -> int:
    out = ctypes.c_size_t()
    _check(lib().it_host_buffer_size(int(ninst), ctypes.byref(out)), "it_host_buffer_size")
    return out.value


_host_buffers = {}


def host_buffer(ninst: int = 1):
    """A page-locked host tensor of it_host_buffer_size(ninst) bytes (the
    caller-owned read-back buffer of it_exec), kept for reuse by calls of the
    same size that do not overlap."""
    import torch
    need = it_host_buffer_size(ninst)
    buf = _host_buffers.get(need)
    if buf is None:
        buf = torch.empty(need, dtype=torch.uint8, pin_memory=True)
        _host_buffers[need] = buf
    return buf


def _exec(ex, ninst: int = 1, host: bool = True):
    """it_exec for the call: the caller's options (dict or None) plus, when
    ``host``, a page-locked read-back buffer (``host_buffer``: a pinned
    tensor, False for none, or absent for the binding's own)."""
    e = it_exec()
    ex = ex or {}
    for k in ("kernel", "steps_per_pass", "tile_y", "check_every", "z_chunk", "tile_x"):
        setattr(e, k, int(ex.get(k, 0)))
    tev = ex.get("timing_events")
    if tev is not None:  # a KernelTimer
        e.timing_events = tev.handles
        e.n_timing_events = len(tev.handles)
        e.timing_span = 1 if tev.span else 0
    hb = ex.get("host_buffer") if host else False
    if hb is None:
        hb = host_buffer(ninst)
    if hb is not False:
        e.host_buffer = ctypes.c_void_p(hb.data_ptr())
        e.host_buffer_bytes = hb.numel() * hb.element_size()
    return ctypes.byref(e)


def _check(rc, where):
    if rc != IT_OK:
        raise ItError(rc, where)


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def it_dt(ch, tracks=None) -> float:
    tr, ptr = _tracks(np.zeros((0, 7)) if tracks is None else tracks)
    out = ctypes.c_double()
    _check(lib().it_dt(ctypes.byref(_chamber(ch)), ptr, tr.shape[0], ctypes.byref(out)), "it_dt")
    return out.value


def it_validate(ch, tracks) -> None:
    tr, ptr = _tracks(tracks)
    _check(lib().it_validate(ctypes.byref(_chamber(ch)), ptr, tr.shape[0]), "it_validate")


def it_workspace_size(ch, ntracks: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().it_workspace_size(ctypes.byref(_chamber(ch)), int(ntracks), ctypes.byref(out)),
           "it_workspace_size")
    return out.value


class KernelTimer:
    """Timing events for the stepping kernel: pass as ``exec["timing_events"]``
    to it_solve / it_advance; the library records a pair around each of the
    first ``launches`` stepping-kernel launches of the call, or, with
    ``span=True``, a pair around each of the first ``launches`` runs of
    consecutive stepping launches (a deposit ends a run).  ``durations()``
    returns the measured times in seconds (after the call returned): one per
    launch, or one per run."""

    def __init__(self, launches=1, span=False):
        self.span = bool(span)
        L = lib()
        self._L = L
        L.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        L.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        L.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        L.hipEventDestroy.argtypes = [ctypes.c_void_p]
        L.hipGetLastError.argtypes = []
        self.handles = (ctypes.c_void_p * (2 * int(launches)))()
        for k in range(2 * int(launches)):
            h = ctypes.c_void_p()
            if L.hipEventCreateWithFlags(ctypes.byref(h), 0) != 0:
                raise RuntimeError("hipEventCreateWithFlags failed")
            self.handles[k] = h

    def durations(self):
        out = []
        ms = ctypes.c_float()
        for k in range(0, len(self.handles), 2):
            if self._L.hipEventSynchronize(self.handles[k + 1]) != 0:
                raise RuntimeError("hipEventSynchronize failed")
            if self._L.hipEventElapsedTime(ctypes.byref(ms), self.handles[k], self.handles[k + 1]) != 0:
                # launches beyond the ones the call issued were not recorded;
                # clear the error the query left in the runtime's state
                self._L.hipGetLastError()
                break
            out.append(ms.value * 1e-3)
        return np.array(out)

    def __del__(self):
        for h in getattr(self, "handles", []):
            if h:
                self._L.hipEventDestroy(h)


def workspace(ch, ntracks: int, device="cuda"):
    import torch
    return torch.empty(it_workspace_size(ch, ntracks), dtype=torch.uint8, device=device)


def _result(r: it_result) -> dict:
    out = {k: getattr(r, k) for k, _ in it_result._fields_}
    out["steps"] = int(out["steps"])
    out["e_steps"] = int(out["e_steps"])
    out["flags"] = int(out["flags"])
    out["passes"] = int(out["passes"])
    out["pulses"] = int(out["pulses"])
    del out["reserved"]
    return out


def it_solve(ch, tracks, exec=None, ws=None, stream=None, trace=False, fields=False) -> dict:
    """Runs the solver; returns the result dict (keys of ``it_result``),
    plus 'trace' (numpy [steps, 10]) and 'pos'/'neg' (device tensors of shape
    (nz+1, ny, nx)) on request."""
    import torch
    c = _chamber(ch)
    tr, ptr = _tracks(tracks)
    if ws is None:
        ws = workspace(ch, tr.shape[0])
    htrace = np.zeros((int(ch["max_steps"]), IT_TRACE_COLS)) if trace else None
    shape = (ch["nz"] + 1, ch["ny"], ch["nx"])
    pos = torch.empty(shape, dtype=torch.float64, device=ws.device) if fields else None
    neg = torch.empty(shape, dtype=torch.float64, device=ws.device) if fields else None
    res = it_result()
    rc = lib().it_solve(ctypes.byref(c), ptr, tr.shape[0], _exec(exec), ctypes.c_void_p(ws.data_ptr()),
                        ws.numel(), _stream(stream),
                        htrace.ctypes.data if trace else None,
                        ctypes.c_void_p(pos.data_ptr()) if fields else None,
                        ctypes.c_void_p(neg.data_ptr()) if fields else None, ctypes.byref(res))
    _check(rc, "it_solve")
    out = _result(res)
    if trace:
        out["trace"] = htrace[: out["steps"]].copy()
    if fields:
        out["pos"], out["neg"] = pos, neg
    return out


def it_advance(ch, dt, pos, neg, nsteps, exec=None, ws=None, stream=None, trace=False):
    """Advances device tensors pos/neg (float64, (nz+1, ny, nx), contiguous)
    in place by nsteps steps; returns the trace (numpy) when asked."""
    import torch
    c = _chamber(ch)
    shape = (ch["nz"] + 1, ch["ny"], ch["nx"])
    for t in (pos, neg):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and tuple(t.shape) == shape and t.is_contiguous()):
            raise ValueError(f"fields must be contiguous float64 CUDA tensors of shape {shape}")
    if ws is None:
        ws = workspace(ch, 0, device=pos.device)
    htrace = np.zeros((int(nsteps), IT_TRACE_COLS)) if trace else None
    rc = lib().it_advance(ctypes.byref(c), float(dt), int(nsteps), _exec(exec),
                          ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(neg.data_ptr()),
                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream),
                          htrace.ctypes.data if trace else None)
    _check(rc, "it_advance")
    return htrace


def _batch_args(chambers, track_lists):
    n = len(chambers)
    chs = (it_chamber * n)(*[_chamber(c) for c in chambers])
    lists = [_track_rows(t) for t in track_lists]
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([t.shape[0] for t in lists])
    tracks = np.ascontiguousarray(np.concatenate(lists) if offsets[-1] else np.zeros((1, TRACK_COLS)))
    return n, chs, offsets, tracks


def it_workspace_size_batch(chambers, track_lists, exec=None) -> int:
    n, chs, offsets, _ = _batch_args(chambers, track_lists)
    out = ctypes.c_size_t()
    _check(lib().it_workspace_size_batch(ctypes.addressof(chs), offsets.ctypes.data, n, _exec(exec, host=False),
                                         ctypes.byref(out)), "it_workspace_size_batch")
    return out.value


def it_solve_batch(chambers, track_lists, exec=None, ws=None, stream=None) -> list:
    """Runs a sweep of chambers (list of dicts, list of (n_q, 7 or 8) track arrays)
    to completion in batched launches; returns one result dict per chamber."""
    import torch
    n, chs, offsets, tracks = _batch_args(chambers, track_lists)
    if ws is None:
        ws = torch.empty(it_workspace_size_batch(chambers, track_lists, exec), dtype=torch.uint8,
                         device="cuda")
    res = (it_result * n)()
    rc = lib().it_solve_batch(ctypes.addressof(chs), offsets.ctypes.data, tracks.ctypes.data, n, _exec(exec, n),
                              ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream), ctypes.addressof(res))
    _check(rc, "it_solve_batch")
    return [_result(r) for r in res]


# --------------------------------------------------------------------------
# Surrogate network
# --------------------------------------------------------------------------
IT_MLP_PARAMS = 34049
IT_MLP_BF16, IT_MLP_FP32 = 0, 1


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def it_mlp_model_bytes(members: int) -> int:
    out = ctypes.c_size_t()
    _check(lib().it_mlp_model_bytes(int(members), ctypes.byref(out)), "it_mlp_model_bytes")
    return out.value


def it_mlp_init(model, members, params, norm, phys=None, stream=None, precision=None):
    """model: device uint8 tensor of it_mlp_model_bytes; params float32
    [members, IT_MLP_PARAMS]; norm float32 [26]; phys None or 6 floats (the
    analytic-baseline constants); precision IT_MLP_BF16 (default) or
    IT_MLP_FP32."""
    p = np.ascontiguousarray(params, dtype=np.float32).reshape(members, IT_MLP_PARAMS)
    nm = np.ascontiguousarray(norm, dtype=np.float32).reshape(26)
    ph = None if phys is None else np.ascontiguousarray(phys, dtype=np.float64).reshape(6)
    prec = IT_MLP_BF16 if precision is None else int(precision)
    _check(lib().it_mlp_init(_dptr(model), int(members), p.ctypes.data, nm.ctypes.data,
                             None if ph is None else ph.ctypes.data, prec, _stream(stream)), "it_mlp_init")


def it_mlp_baseline(model, X, stream=None):
    import torch
    out = torch.empty(X.shape[0], dtype=torch.float64, device=X.device)
    _check(lib().it_mlp_baseline(_dptr(model), _dptr(X), int(X.shape[0]), _dptr(out), _stream(stream)),
           "it_mlp_baseline")
    return out


def _train_ws(members, n, device):
    import torch
    out = ctypes.c_size_t()
    _check(lib().it_mlp_train_ws_bytes(int(members), int(n), ctypes.byref(out)), "it_mlp_train_ws_bytes")
    return torch.empty(out.value, dtype=torch.uint8, device=device)


def it_mlp_grad(model, members, X, t, stream=None):
    """Gradient [members, IT_MLP_PARAMS] (device tensor) and losses (numpy)."""
    import torch
    n = X.shape[0]
    ws = _train_ws(members, n, X.device)
    grad = torch.empty((members, IT_MLP_PARAMS), dtype=torch.float32, device=X.device)
    loss = np.zeros(members, dtype=np.float32)
    _check(lib().it_mlp_grad(_dptr(model), int(members), _dptr(X), _dptr(t), int(n), _dptr(grad),
                             loss.ctypes.data, _dptr(ws), ws.numel(), _stream(stream)), "it_mlp_grad")
    return grad, loss


def it_mlp_train(model, members, X, t, steps, lr, log_every=0, stream=None, batch=0, lr_final=None):
    """Adam steps on device data (X [n, 6], t [n]); minibatches of ``batch``
    rows (0 = full batch), learning rate decaying from lr to lr_final (a
    half cosine; None = constant).  Returns the logged losses."""
    n = X.shape[0]
    ws = _train_ws(members, batch or n, X.device)
    nlog = (steps + log_every - 1) // log_every if log_every > 0 else 0
    loss = np.zeros((max(nlog, 1), members), dtype=np.float32)
    _check(lib().it_mlp_train(_dptr(model), int(members), _dptr(X), _dptr(t), int(n), int(batch), int(steps),
                              float(lr), float(lr if lr_final is None else lr_final), int(log_every),
                              loss.ctypes.data if nlog else None, _dptr(ws), ws.numel(), _stream(stream)),
           "it_mlp_train")
    return loss[:nlog]


def it_mlp_query(model, X, spread_tol, stream=None, ws=None, out=None):
    """Returns (mean, spread, fallback mask, fallback indices, count) with
    the first four as device tensors."""
    import torch
    nq = X.shape[0]
    dev = X.device
    if ws is None:
        need = ctypes.c_size_t()
        _check(lib().it_mlp_query_ws_bytes(int(nq), ctypes.byref(need)), "it_mlp_query_ws_bytes")
        ws = torch.empty(need.value, dtype=torch.uint8, device=dev)
    if out is None:
        out = (torch.empty(nq, dtype=torch.float32, device=dev), torch.empty(nq, dtype=torch.float32, device=dev),
               torch.empty(nq, dtype=torch.uint8, device=dev), torch.empty(nq, dtype=torch.int64, device=dev))
    mean, spread, fb, idx = out
    cnt = ctypes.c_int64()
    _check(lib().it_mlp_query(_dptr(model), _dptr(X), int(nq), float(spread_tol), _dptr(mean), _dptr(spread),
                              _dptr(fb), _dptr(idx), ctypes.byref(cnt), _dptr(ws), ws.numel(), _stream(stream)),
           "it_mlp_query")
    return mean, spread, fb, idx[: cnt.value], cnt.value


IT_MLP_QUERY_STATIC_MAX = 1 << 23


def it_mlp_query_static(model, X, spread_tol, out, stream=None):
    """The allocation-free query: results into ``out`` = (mean, spread,
    fallback mask, fallback indices), device tensors the caller made, with
    the library's own scratch; returns the fallback count."""
    mean, spread, fb, idx = out
    cnt = ctypes.c_int64()
    _check(lib().it_mlp_query_static(_dptr(model), _dptr(X), int(X.shape[0]), float(spread_tol), _dptr(mean),
                                     _dptr(spread), _dptr(fb), _dptr(idx), ctypes.byref(cnt), _stream(stream)),
           "it_mlp_query_static")
    return cnt.value
