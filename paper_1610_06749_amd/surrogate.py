"""Learned surrogate for ln k_s with the solver as its reference and fallback.

Pipeline (every numerical step runs in the library's kernels):

1. Training data: each sample (LET, b, V, gap, dose per pulse, pulse rate)
   becomes a chamber (one centred track parallel to the field plus the
   dose as uniform pre-ionisation, a train of such pulses when the rate
   makes them overlap, see ``workloads.surrogate_chamber``) at the two gap
   resolutions around its real plane count, and its reference ln k_s is
   their weighted blend (``workloads.surrogate_resolutions``), so that the
   target is continuous in the inputs; both come from the batched solver
   (``it_solve_batch``).  Runs are grouped by their expected number of time
   steps so that the chambers of one batched run finish together.
2. Training: an ensemble of MLPs learns the residual of ln k_s over the
   analytic baseline -ln f_Jaffe - ln f_Boag (``it_mlp_train``).
3. Queries (``it_mlp_query``): ensemble mean; a query whose inputs leave the
   training box, or whose ensemble spread exceeds the tolerance, is flagged
   and answered by the solver instead (``Surrogate.answer``; ``evaluate``
   times both parts together).
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import binding as B

try:
    import workloads as W
except ImportError:  # pragma: no cover - the package is used from the repository root
    W = None


def phys_constants():
    """Constants of the analytic baseline: averaged D and mu, alpha, W,
    mu+ + mu-, ion pairs per cm^3 and mGy (air, as the workloads use)."""
    a = W.AIR
    return np.array([0.5 * (a["D_pos"] + a["D_neg"]), 0.5 * (a["mu_pos"] + a["mu_neg"]), a["alpha"],
                     a["W_eV"], a["mu_pos"] + a["mu_neg"], W.ion_pairs_per_mGy(a["W_eV"])])


def expected_steps(ch, tr):
    """Rough step count of a run (transit of the slower ion over the gap,
    with margin for the diffusion tail; a pulse train's periods): used only
    to group chambers."""
    dt = B.it_dt(ch, tr)
    if ch.get("n_pulses", 0) >= 2:
        return ch["n_pulses"] * ch["pulse_period_s"] / dt
    E = ch["voltage"] / ch["gap"]
    return 1.5 * ch["gap"] / (min(ch["mu_pos"], ch["mu_neg"]) * E) / dt + 50


def solver_lnks(X, group=512, stream=None, log=None):
    """Reference ln k_s of every input row from the batched solver (the
    blend of the two gap resolutions); returns (lnks, total voxel-steps,
    seconds).  A row whose run ends non-finite (the explicit scheme's
    recombination term can blow up in the corner of the input box where
    fast trains stack dense tracks) gets NaN.  ``log``: None or a callable
    taking a progress message."""
    import torch
    chs, trs, est, owner, weight = [], [], [], [], []
    for q, x in enumerate(X):
        for nz, w in W.surrogate_resolutions(x):
            ch, tr = W.surrogate_chamber(x, nz=nz)
            chs.append(ch)
            trs.append(tr)
            est.append(expected_steps(ch, tr))
            owner.append(q)
            weight.append(w)
    order = np.argsort(est, kind="stable")
    out = np.zeros(len(X))
    vs = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g0 in range(0, len(chs), group):
        if log and g0 and g0 % (8 * group) == 0:
            log(f"solver runs: {g0} of {len(chs)}")
        idx = order[g0:g0 + group]
        res = B.it_solve_batch([chs[i] for i in idx], [trs[i] for i in idx], stream=stream)
        for i, r in zip(idx, res):
            if r["flags"] & B.IT_FLAG_MAX_STEPS:
                raise RuntimeError(f"solver run {i} stopped at max_steps (flags {r['flags']})")
            if r["flags"] & B.IT_FLAG_NONFINITE:
                out[owner[i]] = math.nan
                continue
            out[owner[i]] += weight[i] * math.log(r["ks"])
            vs += r["steps"] * chs[i]["nx"] * chs[i]["ny"] * (chs[i]["nz"] - 1)
    torch.cuda.synchronize()
    return out, vs, time.perf_counter() - t0


def minibatch_order(n, batch, seed):
    """Row order and minibatch size for training on n rows: one shuffle of
    the rows, continued from its start up to the next multiple of ``batch``
    (the library's minibatches tile the data it is given), so that every
    row is used and fewer than ``batch`` of them twice per pass; a full
    batch (0) when ``batch`` is not positive or not below n."""
    perm = np.random.default_rng(seed).permutation(n)
    if batch <= 0 or batch >= n:
        return perm, 0
    pad = -n % batch
    return np.concatenate([perm, perm[:pad]]), batch


class Surrogate:
    def __init__(self, members=4, seed=W.SEED_BASE + 5 if W else 0, precision=B.IT_MLP_FP32):
        self.members = members
        self.seed = seed
        self.precision = precision
        self.model = None

    def fit(self, X, lnks, steps=150000, lr=2e-3, lr_final=1e-5, batch=2048, log_every=1000, margin=1e-3):
        """Standardisation from the training inputs (log space), training box
        with a small margin, targets standardised around the residual; then
        ``steps`` Adam steps on minibatches of ``batch`` rows of the data
        shuffled once (``minibatch_order``), the rate decaying from lr to
        lr_final (half cosine)."""
        import torch
        X = np.asarray(X, dtype=np.float64)
        lnks = np.asarray(lnks, dtype=np.float64)
        L = np.log(X)
        mu, sd = L.mean(axis=0), L.std(axis=0)
        sd = np.where(sd > 0, sd, 1.0)
        Z = (L - mu) / sd
        # residual statistics need the baseline: evaluate it on the device
        self.model = torch.empty(B.it_mlp_model_bytes(self.members), dtype=torch.uint8, device="cuda")
        norm0 = np.concatenate([mu, sd, Z.min(0) - margin, Z.max(0) + margin, [0.0, 1.0]])
        params = W.mlp_init(self.seed, self.members)
        B.it_mlp_init(self.model, self.members, params, norm0, phys_constants(), precision=self.precision)
        Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
        base = B.it_mlp_baseline(self.model, Xd).cpu().numpy()
        resid = lnks - base
        norm = np.concatenate([mu, sd, Z.min(0) - margin, Z.max(0) + margin, [resid.mean(), resid.std()]])
        B.it_mlp_init(self.model, self.members, params, norm, phys_constants(), precision=self.precision)
        perm, batch = minibatch_order(len(X), batch, self.seed + 1)
        Xd = torch.tensor(X[perm], dtype=torch.float32, device="cuda")
        td = torch.tensor(lnks[perm], dtype=torch.float32, device="cuda")
        t0 = time.perf_counter()
        self.loss_log = B.it_mlp_train(self.model, self.members, Xd, td, steps, lr, log_every, batch=batch,
                                       lr_final=lr_final)
        self.train_seconds = time.perf_counter() - t0
        self.train_steps = steps
        self.batch = batch or len(X)
        return self

    def query(self, Xq, spread_tol):
        import torch
        Xd = Xq if isinstance(Xq, torch.Tensor) else torch.tensor(np.asarray(Xq), dtype=torch.float32,
                                                                 device="cuda")
        return B.it_mlp_query(self.model, Xd, spread_tol)

    def answer(self, Xq, spread_tol, Xq_host=None, out=None):
        """ln k_s for every query: the ensemble mean where it is trusted, the
        solver elsewhere (NaN where the solver's run ends non-finite).
        Xq_host: the queries in float64 on the host (default: read back from
        Xq); out: the query's output buffers (see ``binding.it_mlp_query``).
        Returns (lnks, fallback mask)."""
        import torch
        Xd = Xq if isinstance(Xq, torch.Tensor) else torch.tensor(np.asarray(Xq), dtype=torch.float32,
                                                                 device="cuda")
        mean, spread, fb, idx, n = B.it_mlp_query(self.model, Xd, spread_tol, out=out)
        lnks = mean.double().cpu().numpy()
        mask = fb.cpu().numpy().astype(bool)
        if n:
            if Xq_host is None:
                Xq_host = np.asarray(Xq.cpu().numpy() if hasattr(Xq, "cpu") else Xq, dtype=np.float64)
            sel = idx[:n].cpu().numpy()
            lnks[sel] = solver_lnks(Xq_host[sel])[0]
        return lnks, mask


def solver_data(n_train=32768, n_hold=1024, seed=None, log=None, n_overlap=0, min_overlap=3.0):
    """Training and held-out data from the solver: a dict of the inputs,
    ln k_s, voxel-steps and seconds of each set.  ``n_overlap`` more
    training rows come from the deep pulse-train part of the box (rate x
    twice the slower ion's transit at least ``min_overlap``,
    ``workloads.surrogate_inputs_overlapping``); the held-out rows stay
    uniform.  Rows the solver could not compute (non-finite) are left out
    and counted (``*_nonfinite``)."""
    base_seed = W.SEED_BASE + 5 if seed is None else seed
    Xtr = W.surrogate_inputs(base_seed, n_train)
    if n_overlap:
        Xtr = np.concatenate([Xtr, W.surrogate_inputs_overlapping(base_seed + 3, n_overlap, min_overlap)])
    ytr, vs_tr, sec_tr = solver_lnks(Xtr, log=log)
    Xh = W.surrogate_inputs(base_seed + 1, n_hold)
    yh, vs_h, sec_h = solver_lnks(Xh, log=log)
    ktr, kh = np.isfinite(ytr), np.isfinite(yh)
    return dict(seed=base_seed, Xtr=Xtr[ktr], ytr=ytr[ktr], vs_tr=vs_tr, sec_tr=sec_tr, Xh=Xh[kh], yh=yh[kh],
                vs_h=vs_h, sec_h=sec_h, train_nonfinite=int(np.sum(~ktr)), holdout_nonfinite=int(np.sum(~kh)))


def evaluate(n_train=32768, n_hold=1024, n_query=65536, spread_tol=1e-3, members=4, steps=600000, seed=None,
             precision=B.IT_MLP_FP32, data=None, extra_tols=(5e-4,), log=None, time_extra=False, n_overlap=0):
    """The surrogate experiment: train on n_train solver runs (plus
    ``n_overlap`` from the deep pulse-train part of the box, see
    ``solver_data``), check on n_hold held-out solver runs, time n_query
    uniform queries (``data`` from
    ``solver_data`` reuses solver runs).  The figures are taken at the
    spread tolerance ``spread_tol``, where the queries are also answered end
    to end (the query plus the solver on the queries it flags, timed
    together); ``at_spread_tol`` repeats the accuracy, query throughput and
    fallback figures at each of ``extra_tols`` (the end-to-end answer is
    timed there only with ``time_extra``).  ``log``: None or a callable
    taking a progress message.  Returns a dict."""
    import torch
    say = log or (lambda msg: None)
    d = data if data is not None else solver_data(n_train, n_hold, seed, log=log, n_overlap=n_overlap)
    base_seed = d["seed"]
    Xtr, ytr, vs_tr, sec_tr = d["Xtr"], d["ytr"], d["vs_tr"], d["sec_tr"]
    Xh, yh, sec_h = d["Xh"], d["yh"], d["sec_h"]
    n_train, n_hold = len(Xtr), len(Xh)
    say(f"surrogate: {n_train} training and {n_hold} held-out samples from the solver in {sec_tr + sec_h:.0f} s")
    s = Surrogate(members=members, seed=base_seed + 100, precision=precision)
    s.fit(Xtr, ytr, steps=steps)
    say(f"surrogate: {steps} training steps in {s.train_seconds:.0f} s")
    Xhd = torch.tensor(Xh, dtype=torch.float32, device="cuda")
    base = B.it_mlp_baseline(s.model, Xhd).cpu().numpy()
    rel_base = np.abs(np.expm1(base - yh))
    Xq_h = W.surrogate_inputs(base_seed + 2, n_query)
    Xq = torch.tensor(Xq_h, dtype=torch.float32, device="cuda")
    out = (torch.empty(n_query, dtype=torch.float32, device="cuda"),
           torch.empty(n_query, dtype=torch.float32, device="cuda"),
           torch.empty(n_query, dtype=torch.uint8, device="cuda"),
           torch.empty(n_query, dtype=torch.int64, device="cuda"))
    solver_rate = n_hold / sec_h  # reference k_s evaluations per second by the batched solver

    def at_tol(tol, timed):
        mean, spread, fb, idx, n_fb = s.query(Xh, tol)
        m = mean.double().cpu().numpy()
        mask = fb.cpu().numpy().astype(bool)
        rel = np.abs(np.expm1(m - yh))  # relative error of k_s
        acc = ~mask
        # query throughput at the full batch (inputs resident, fallback excluded)
        B.it_mlp_query(s.model, Xq, tol, out=out)
        torch.cuda.synchronize()
        reps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            _, _, _, _, nq_fb = B.it_mlp_query(s.model, Xq, tol, out=out)
        e1.record()
        e1.synchronize()
        q_sec = e0.elapsed_time(e1) * 1e-3 / reps
        fb_frac_q = nq_fb / n_query
        fig = {
            "spread_tol_ln": tol,
            "holdout_accepted_fraction": float(acc.mean()),
            "holdout_rel_err_accepted_max": float(rel[acc].max()) if acc.any() else None,
            "holdout_rel_err_accepted_p99": float(np.quantile(rel[acc], 0.99)) if acc.any() else None,
            "holdout_accepted_beyond_0.1pct": int(np.sum(rel[acc] > 1e-3)),
            "query_seconds": q_sec, "query_rate": n_query / q_sec,
            "query_fallback_fraction": fb_frac_q, "query_fallbacks": int(nq_fb),
            "surrogate_over_solver": (n_query / q_sec) / solver_rate,
        }
        if timed:
            # surrogate plus solver fallback, timed end to end: the query, its
            # answers read back, and the batched solver on the queries it
            # flagged (the solver's accuracy on that part)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lnks, _ = s.answer(Xq, tol, Xq_host=Xq_h, out=out)
            torch.cuda.synchronize()
            combined_sec = time.perf_counter() - t0
            say(f"surrogate: {n_query} queries with {nq_fb} solver fallbacks in {combined_sec:.2f} s")
            fig.update({
                "with_fallback_seconds": combined_sec, "with_fallback_rate": n_query / combined_sec,
                "fallback_nonfinite": int(np.sum(~np.isfinite(lnks))),
                "surrogate_with_fallback_over_solver": (n_query / combined_sec) / solver_rate,
            })
        return rel, acc, fig

    rel, acc, main = at_tol(spread_tol, True)
    res = {
        # training rows holding three or more pulses in flight (deep trains)
        "n_train": n_train, "n_train_overlap": int(np.sum([W.surrogate_overlap(x) >= 3.0 for x in Xtr])),
        "n_holdout": n_hold, "n_query": n_query, "members": members,
        "train_nonfinite": d.get("train_nonfinite", 0), "holdout_nonfinite": d.get("holdout_nonfinite", 0),
        "precision": "fp32" if precision == B.IT_MLP_FP32 else "bf16",
        "train_data_seconds": sec_tr, "train_data_voxel_steps": vs_tr, "train_seconds": s.train_seconds,
        "train_steps": s.train_steps, "train_batch": s.batch,
        "final_loss": float(s.loss_log[-1].max()) if s.loss_log is not None and len(s.loss_log) else None,
        "holdout_frac_within_0.1pct_all": float(np.mean(rel < 1e-3)),
        "holdout_rel_err_all_median": float(np.median(rel)),
        "holdout_rel_err_all_p90": float(np.quantile(rel, 0.9)),
        "baseline_rel_err_median": float(np.median(rel_base)),
        "baseline_rel_err_p90": float(np.quantile(rel_base, 0.9)),
        "solver_ks_rate": solver_rate,
    }
    res.update(main)
    res["at_spread_tol"] = [at_tol(t, time_extra)[2] for t in extra_tols]
    say("surrogate: queries timed")
    return res
