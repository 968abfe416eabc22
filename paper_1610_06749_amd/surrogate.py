"""Learned surrogate for ln k_s with the solver as its judge and fallback.

Pipeline (every numerical step runs in the library's kernels):

1. Training data: each sample (LET, b, V, gap, dose per pulse, pulse rate)
   becomes one chamber (one centred track parallel to the field plus the
   dose as uniform pre-ionisation, see ``workloads.surrogate_chamber``) and
   ln k_s comes from the batched solver (``it_solve_batch``).  Samples are
   grouped by their expected number of time steps so that the chambers of
   one batched run finish together.
2. Training: an ensemble of MLPs learns the residual of ln k_s over the
   analytic baseline -ln f_Jaffe - ln f_Boag (``it_mlp_train``).
3. Queries (``it_mlp_query``): ensemble mean; a query whose inputs leave the
   training box, or whose ensemble spread exceeds the tolerance, is flagged
   and answered by the solver instead.
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
    with margin for the diffusion tail): used only to group chambers."""
    dt = B.it_dt(ch, tr)
    E = ch["voltage"] / ch["gap"]
    return 1.5 * ch["gap"] / (min(ch["mu_pos"], ch["mu_neg"]) * E) / dt + 50


def solver_lnks(X, group=512, stream=None):
    """ln k_s of every input row from the batched solver; returns (lnks,
    total voxel-steps, seconds)."""
    import torch
    chs, trs, est = [], [], []
    for x in X:
        ch, tr = W.surrogate_chamber(x)
        chs.append(ch)
        trs.append(tr)
        est.append(expected_steps(ch, tr))
    order = np.argsort(est)
    out = np.empty(len(X))
    vs = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g0 in range(0, len(X), group):
        idx = order[g0:g0 + group]
        res = B.it_solve_batch([chs[i] for i in idx], [trs[i] for i in idx], stream=stream)
        for i, r in zip(idx, res):
            if r["flags"] & (B.IT_FLAG_NONFINITE | B.IT_FLAG_MAX_STEPS):
                raise RuntimeError(f"solver run {i} did not finish cleanly (flags {r['flags']})")
            out[i] = math.log(r["ks"])
            vs += r["steps"] * chs[i]["nx"] * chs[i]["ny"] * (chs[i]["nz"] - 1)
    torch.cuda.synchronize()
    return out, vs, time.perf_counter() - t0


class Surrogate:
    def __init__(self, members=4, seed=W.SEED_BASE + 5 if W else 0):
        self.members = members
        self.seed = seed
        self.model = None

    def fit(self, X, lnks, steps=150000, lr=2e-3, lr_final=1e-5, batch=2048, log_every=1000, margin=1e-3):
        """Standardisation from the training inputs (log space), training box
        with a small margin, targets standardised around the residual; then
        ``steps`` Adam steps on minibatches of ``batch`` rows of the data
        shuffled once, the rate decaying from lr to lr_final (half cosine)."""
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
        B.it_mlp_init(self.model, self.members, params, norm0, phys_constants())
        Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
        base = B.it_mlp_baseline(self.model, Xd).cpu().numpy()
        resid = lnks - base
        norm = np.concatenate([mu, sd, Z.min(0) - margin, Z.max(0) + margin, [resid.mean(), resid.std()]])
        B.it_mlp_init(self.model, self.members, params, norm, phys_constants())
        n = len(X)
        if batch <= 0 or batch >= n or n % batch:
            batch = 0  # full batch
        perm = np.random.default_rng(self.seed + 1).permutation(n)
        Xd = torch.tensor(X[perm], dtype=torch.float32, device="cuda")
        td = torch.tensor(lnks[perm], dtype=torch.float32, device="cuda")
        t0 = time.perf_counter()
        self.loss_log = B.it_mlp_train(self.model, self.members, Xd, td, steps, lr, log_every, batch=batch,
                                       lr_final=lr_final)
        self.train_seconds = time.perf_counter() - t0
        self.train_steps = steps
        self.batch = batch or n
        return self

    def query(self, Xq, spread_tol):
        import torch
        Xd = Xq if isinstance(Xq, torch.Tensor) else torch.tensor(np.asarray(Xq), dtype=torch.float32,
                                                                 device="cuda")
        return B.it_mlp_query(self.model, Xd, spread_tol)

    def answer(self, Xq, spread_tol):
        """ln k_s for every query: the ensemble mean where it is trusted, the
        solver elsewhere.  Returns (lnks, fallback mask)."""
        mean, spread, fb, idx, n = self.query(Xq, spread_tol)
        out = mean.double().cpu().numpy()
        mask = fb.cpu().numpy().astype(bool)
        if n:
            Xh = np.asarray(Xq.cpu().numpy() if hasattr(Xq, "cpu") else Xq, dtype=np.float64)
            sel = idx.cpu().numpy()
            out[sel] = solver_lnks(Xh[sel])[0]
        return out, mask


def evaluate(n_train=8192, n_hold=512, n_query=65536, spread_tol=1e-3, members=4, steps=150000, seed=None):
    """The surrogate experiment: train on n_train solver runs, judge on
    n_hold held-out solver runs, time n_query queries.  Returns a dict."""
    import torch
    base_seed = W.SEED_BASE + 5 if seed is None else seed
    Xtr = W.surrogate_inputs(base_seed, n_train)
    ytr, vs_tr, sec_tr = solver_lnks(Xtr)
    s = Surrogate(members=members, seed=base_seed + 100)
    s.fit(Xtr, ytr, steps=steps)
    Xh = W.surrogate_inputs(base_seed + 1, n_hold)
    yh, vs_h, sec_h = solver_lnks(Xh)
    mean, spread, fb, idx, n_fb = s.query(Xh, spread_tol)
    m = mean.double().cpu().numpy()
    mask = fb.cpu().numpy().astype(bool)
    rel = np.abs(np.expm1(m - yh))  # relative error of k_s
    Xhd = torch.tensor(Xh, dtype=torch.float32, device="cuda")
    base = B.it_mlp_baseline(s.model, Xhd).cpu().numpy()
    rel_base = np.abs(np.expm1(base - yh))
    acc = ~mask
    # query throughput at the full batch (inputs resident, fallback excluded)
    Xq = torch.tensor(W.surrogate_inputs(base_seed + 2, n_query), dtype=torch.float32, device="cuda")
    out = (torch.empty(n_query, dtype=torch.float32, device="cuda"),
           torch.empty(n_query, dtype=torch.float32, device="cuda"),
           torch.empty(n_query, dtype=torch.uint8, device="cuda"),
           torch.empty(n_query, dtype=torch.int64, device="cuda"))
    B.it_mlp_query(s.model, Xq, spread_tol, out=out)
    torch.cuda.synchronize()
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        _, _, _, _, nq_fb = B.it_mlp_query(s.model, Xq, spread_tol, out=out)
    e1.record()
    e1.synchronize()
    q_sec = e0.elapsed_time(e1) * 1e-3 / reps
    solver_rate = n_hold / sec_h  # k_s evaluations per second by the batched solver
    fb_frac_q = nq_fb / n_query
    # surrogate plus solver fallback at equal (solver) accuracy on the flagged part
    combined = 1.0 / (q_sec / n_query + fb_frac_q / solver_rate)
    return {
        "n_train": n_train, "n_holdout": n_hold, "n_query": n_query, "members": members,
        "spread_tol_ln": spread_tol,
        "train_data_seconds": sec_tr, "train_data_voxel_steps": vs_tr, "train_seconds": s.train_seconds,
        "train_steps": s.train_steps, "train_batch": s.batch,
        "final_loss": float(s.loss_log[-1].max()) if s.loss_log is not None and len(s.loss_log) else None,
        "holdout_accepted_fraction": float(acc.mean()),
        "holdout_rel_err_accepted_max": float(rel[acc].max()) if acc.any() else None,
        "holdout_rel_err_accepted_p99": float(np.quantile(rel[acc], 0.99)) if acc.any() else None,
        "holdout_frac_within_0.1pct_all": float(np.mean(rel < 1e-3)),
        "holdout_rel_err_all_median": float(np.median(rel)),
        "holdout_rel_err_all_p90": float(np.quantile(rel, 0.9)),
        "baseline_rel_err_median": float(np.median(rel_base)),
        "baseline_rel_err_p90": float(np.quantile(rel_base, 0.9)),
        "query_seconds": q_sec, "query_rate": n_query / q_sec,
        "query_fallback_fraction": fb_frac_q,
        "solver_ks_rate": solver_rate,
        "surrogate_over_solver": (n_query / q_sec) / solver_rate,
        "surrogate_with_fallback_over_solver": combined / solver_rate,
    }
