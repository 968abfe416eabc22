"""Seeded synthetic inputs for the recombination solver.

This module only *describes* chambers and draws track lists.  It holds none of
the method's arithmetic (no time step, no deposition, no transport), so the
CPU oracle and the GPU library can both take their inputs from here without
sharing any code of the method.

A chamber is a plain ``dict`` whose keys mirror the C struct ``it_chamber``:

    nx, ny      transverse node counts
    nz          number of gap intervals; planes k=0 (anode) and k=nz (cathode)
                are the electrodes, interior planes are 1..nz-1
    dx, dy      transverse node spacing [cm]; the gap spacing is gap/nz
    gap         electrode distance d [cm]
    voltage     polarisation voltage V [V]; the field E = V/d points from the
                anode (z=0) to the cathode (z=d)
    mu_pos, mu_neg   ion mobilities [cm^2/(V s)]
    D_pos, D_neg     ion diffusion constants [cm^2/s]
    alpha       recombination constant [cm^3/s]
    W_eV        mean energy per ion pair [eV]
    dt_safety   factor kappa in (0,1] applied to the largest stable time step
    stop_tol    stop once both in-flight counts are <= stop_tol * released
    max_steps   hard limit on the number of time steps
    uniform_n0  uniform ion-pair density added to both species at t=0 [cm^-3]
    space_charge  1 adds the space-charge screening term, 0 leaves it out
    lateral_bc  0 periodic lateral boundaries, 1 absorbing ones
    reaction_limit  rho >= 0: the time step is also bounded by
                alpha dt n_ref <= rho, n_ref the reference peak density of
                the inputs (0 leaves only the transport bound)

A track list is a float64 array of shape (n, 7) with columns
``[let_keV_um, b_cm, x_cm, y_cm, theta, phi, t_s]``: linear energy transfer,
Gaussian track radius, the point where the axis crosses mid-gap, the polar
angle to the field, the azimuth, and the arrival time.

The transport constants of dry air used by every workload here are the ones
the workloads are specified with (mobilities 1.73/1.87, D = 0.045, alpha
1.6e-6, W = 34 eV).  The paper's own Table II values are in ``TABLE_II``.
"""
from __future__ import annotations

import math

import numpy as np

TRACK_COLUMNS = ("let_keV_um", "b_cm", "x_cm", "y_cm", "theta", "phi", "t_s")

AIR = dict(mu_pos=1.73, mu_neg=1.87, D_pos=0.045, D_neg=0.045, alpha=1.60e-6, W_eV=34.0)

# Table II of the paper (ion transport constants and recombination constant).
TABLE_II = dict(D_pos=2.82e-2, D_neg=4.35e-2, mu_pos=1.36, mu_neg=2.10, alpha=1.60e-6)

# Table I of the paper: (LET in air [keV/um], Gaussian track radius [um]).
TABLE_I = {
    "Fe40": (1.02, 50.0),
    "Ne60": (0.115, 20.0),
    "C90": (3.03e-2, 10.5),
    "p100": (7.76e-4, 10.0),
}

# Ion pairs per cm^3 released in air by 1 mGy: dose * rho_air / (W q).
RHO_AIR_G_CM3 = 1.205e-3
Q_E = 1.602176634e-19
SEED_BASE = 1610067490


def ion_pairs_per_mGy(W_eV: float = 34.0) -> float:
    """Uniform ion-pair density [cm^-3] that 1 mGy releases in air."""
    energy_j_per_cm3 = 1e-3 * RHO_AIR_G_CM3 * 1e-3  # J/kg * kg/cm^3
    return energy_j_per_cm3 / (W_eV * Q_E)


REACTION_LIMIT = 0.5


def chamber(nx, ny, nz, dx, gap, voltage, dy=None, *, dt_safety=1.0, stop_tol=1e-12,
            max_steps=1_000_000, uniform_n0=0.0, space_charge=0, reaction_limit=REACTION_LIMIT,
            lateral_bc=0, **consts) -> dict:
    """A chamber dict with air's constants (AIR), any of which ``consts``
    may replace; other keywords are refused rather than dropped (options
    such as a pulse train's n_pulses go into the dict afterwards)."""
    unknown = set(consts) - set(AIR)
    if unknown:
        raise TypeError(f"chamber(): unknown keywords {sorted(unknown)}")
    c = dict(AIR)
    c.update(consts)
    return dict(nx=int(nx), ny=int(ny), nz=int(nz), dx=float(dx),
                dy=float(dx if dy is None else dy), gap=float(gap), voltage=float(voltage),
                mu_pos=float(c["mu_pos"]), mu_neg=float(c["mu_neg"]),
                D_pos=float(c["D_pos"]), D_neg=float(c["D_neg"]),
                alpha=float(c["alpha"]), W_eV=float(c["W_eV"]),
                dt_safety=float(dt_safety), stop_tol=float(stop_tol),
                max_steps=int(max_steps), uniform_n0=float(uniform_n0),
                space_charge=int(space_charge), reaction_limit=float(reaction_limit),
                lateral_bc=int(lateral_bc))


def tracks(rows) -> np.ndarray:
    a = np.asarray(rows, dtype=np.float64).reshape(-1, 7)
    return np.ascontiguousarray(a)


def no_tracks() -> np.ndarray:
    return np.zeros((0, 7), dtype=np.float64)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def single_track(**over):
    """One Gaussian track parallel to the field in a 64x64x100 grid.

    Gap 0.02 cm at 30 V, spacing 2e-4 cm, LET 100 keV/um, b = 1e-3 cm,
    axis through the node (32, 32)."""
    ch = chamber(64, 64, 100, 2e-4, 0.02, 30.0)
    ch.update(over)
    tr = tracks([[100.0, 1e-3, 32 * ch["dx"], 32 * ch["dy"], 0.0, 0.0, 0.0]])
    return ch, tr


def pulsed_beam(seed: int = SEED_BASE + 2, ntracks: int = 400, **over):
    """One instantaneous pulse of 400 parallel tracks in a 256x256x200 grid.

    Gap 0.1 cm at 200 V, spacing 5e-4 cm.  Track positions uniform over the
    periodic cell, ln LET ~ N(ln 50, 0.5^2), b ~ U[5e-4, 2e-3] cm."""
    ch = chamber(256, 256, 200, 5e-4, 0.1, 200.0)
    ch.update(over)
    rng = np.random.default_rng(seed)
    lx, ly = ch["nx"] * ch["dx"], ch["ny"] * ch["dy"]
    x = rng.uniform(0.0, lx, ntracks)
    y = rng.uniform(0.0, ly, ntracks)
    let = np.exp(rng.normal(math.log(50.0), 0.5, ntracks))
    b = rng.uniform(5e-4, 2e-3, ntracks)
    z = np.zeros(ntracks)
    return ch, tracks(np.stack([let, b, x, y, z, z, z], axis=1))


def continuous_beam(seed: int = SEED_BASE + 3, duration_s: float = 0.0, forced: int = 4,
                    fluence_rate=2e5, grid=(512, 512, 256), **over):
    """Continuous beam on a 512x512x256 grid (spacing 4e-4 cm, gap 0.1 cm, 300 V).

    Arrival times form a Poisson process of rate ``fluence_rate`` x (cell
    area) per second over ``[0, duration_s)``; ``forced`` extra tracks arrive
    at t = 0 so that a short window already carries a non-trivial field.
    Tilt theta ~ U[0, 30 deg], azimuth phi ~ U[0, 2 pi), LET log-uniform on
    [1, 300] keV/um, b ~ U[5e-4, 2e-3] cm, positions uniform over the cell.
    """
    nx, ny, nz = grid
    ch = chamber(nx, ny, nz, 4e-4, 0.1, 300.0)
    ch.update(over)
    rng = np.random.default_rng(seed)
    lx, ly = ch["nx"] * ch["dx"], ch["ny"] * ch["dy"]
    rate = fluence_rate * lx * ly
    times = [0.0] * forced
    t = 0.0
    while duration_s > 0.0:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            break
        times.append(t)
    n = len(times)
    x = rng.uniform(0.0, lx, n)
    y = rng.uniform(0.0, ly, n)
    theta = rng.uniform(0.0, math.radians(30.0), n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    let = np.exp(rng.uniform(math.log(1.0), math.log(300.0), n))
    b = rng.uniform(5e-4, 2e-3, n)
    return ch, tracks(np.stack([let, b, x, y, theta, phi, np.asarray(times)], axis=1))


# Arrival times [s] of the continuous-beam window's tracks: four at t = 0
# and one at each of four later instants inside the window.
WINDOW_TIMES = (0.0, 0.0, 0.0, 0.0, 8.0e-6, 2.0e-5, 3.4e-5, 4.6e-5)
WINDOW_STEPS = 2000


def continuous_window(steps: int = WINDOW_STEPS):
    """A fixed window of the continuous beam on its 512x512x256 grid: the
    first eight tracks the continuous-beam generator draws (tilted 0-30 deg,
    LET log-uniform on [1, 300] keV/um), four arriving at t = 0 and one at
    each of 8, 20, 34 and 46 us, stepped for exactly ``steps`` time steps
    (stop_tol = 0).  The densest track bounds the time step (reaction
    limit), and at that step the four later arrivals fall inside a
    2000-step window, so the window holds five deposit events."""
    ch, tr = continuous_beam(duration_s=0.0, forced=len(WINDOW_TIMES))
    tr[:, 6] = WINDOW_TIMES
    ch.update(max_steps=int(steps), stop_tol=0.0)
    return ch, tr


def shaped_pulse(ch, seed: int, fluence_cm2: float, shape, t_end: float, shape_max: float, let=50.0,
                 b=1e-3, theta=0.0, region: str = "cell", r_min: float | None = None) -> np.ndarray:
    """Tracks of a pulse of finite length (section "Distribution of ion
    tracks"): arrival times form a Poisson process of rate
    fluence_cm2 * area * shape(t) on [0, t_end), where shape(t) [1/s] is the
    pulse shape g(t) normalised to unit integral and shape_max bounds it
    (sampled by thinning a homogeneous process of rate fluence * area *
    shape_max).  Positions are uniform over the transverse cell
    (region="cell") or over a centred disc of radius r_min (region="disc",
    area pi r_min^2).  let, b: scalars or callables of the generator (one
    value per track); theta: tilt to the field, azimuths uniform."""
    rng = np.random.default_rng(seed)
    lx, ly = ch["nx"] * ch["dx"], ch["ny"] * ch["dy"]
    if region == "cell":
        area = lx * ly
    elif region == "disc":
        area = math.pi * r_min * r_min
    else:
        raise ValueError("region is 'cell' or 'disc'")
    rate_max = fluence_cm2 * area * shape_max
    times = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate_max)
        if t >= t_end:
            break
        if rng.uniform() * shape_max < shape(t):
            times.append(t)
    n = len(times)
    if region == "cell":
        x = rng.uniform(0.0, lx, n)
        y = rng.uniform(0.0, ly, n)
    else:
        rad = r_min * np.sqrt(rng.uniform(0.0, 1.0, n))
        ang = rng.uniform(0.0, 2.0 * math.pi, n)
        x = 0.5 * lx + rad * np.cos(ang)
        y = 0.5 * ly + rad * np.sin(ang)
    lets = let(rng, n) if callable(let) else np.full(n, float(let))
    bs = b(rng, n) if callable(b) else np.full(n, float(b))
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    return tracks(np.stack([lets, bs, x, y, np.full(n, float(theta)), phi, np.asarray(times, dtype=float)],
                           axis=1))


def batched_sweep(seed: int = SEED_BASE + 4, ninst: int = 96, max_tracks: int = 500,
                  transverse=(64, 256), gap_voxels=(50, 250), spacing=5e-4):
    """A sweep of ``ninst`` chambers of uneven grids (one pulse each).

    Per instance: nx = ny ~ U{64..256}, nz ~ U{50..250} at spacing 5e-4 cm
    (gap = nz * spacing); voltages log-spaced over 50..400 V across the
    instances; one LET per instance, log-uniform on [1, 500] keV/um; b ~
    U[5e-4, 2e-3] cm; 1..500 parallel tracks at t = 0 uniform over the cell;
    dose per pulse log-uniform on [0.01, 1] mGy, realised as a uniform
    pre-ionisation of both species.
    Returns (list of chambers, list of track arrays)."""
    rng = np.random.default_rng(seed)
    volts = np.geomspace(50.0, 400.0, ninst)
    chs, trs = [], []
    per_mgy = ion_pairs_per_mGy(AIR["W_eV"])
    for i in range(ninst):
        n_t = int(rng.integers(transverse[0], transverse[1] + 1))
        nz = int(rng.integers(gap_voxels[0], gap_voxels[1] + 1))
        dose = math.exp(rng.uniform(math.log(0.01), math.log(1.0)))
        ch = chamber(n_t, n_t, nz, spacing, nz * spacing, float(volts[i]),
                     uniform_n0=dose * per_mgy)
        let = math.exp(rng.uniform(math.log(1.0), math.log(500.0)))
        b = rng.uniform(5e-4, 2e-3)
        k = int(rng.integers(1, max_tracks + 1))
        lx = n_t * spacing
        x = rng.uniform(0.0, lx, k)
        y = rng.uniform(0.0, lx, k)
        z = np.zeros(k)
        trs.append(tracks(np.stack([np.full(k, let), np.full(k, b), x, y, z, z, z], axis=1)))
        chs.append(ch)
    return chs, trs


def perturbed_field(shape, seed: int, scale: float = 1e9):
    """Smooth positive random density fields (for stepping tests that start
    from a given state rather than from deposited tracks).  Returns two
    arrays of shape (nz+1, ny, nx) with zero electrode planes."""
    nzp1, ny, nx = shape
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(2):
        f = rng.uniform(0.0, scale, size=shape)
        f[0] = 0.0
        f[-1] = 0.0
        out.append(np.ascontiguousarray(f))
    return out[0], out[1]


# --------------------------------------------------------------------------
# Surrogate inputs
# --------------------------------------------------------------------------
# Ranges of the six surrogate inputs: LET [keV/um], b [cm], V [V], gap [cm],
# dose per pulse [mGy], pulse repetition rate [Hz].  Where the pulse period
# is shorter than the ions' collection (up to ~0.2 ms at 50 V over
# 0.125 cm; rates above ~2.8 kHz there) the sample is a pulse train
# (surrogate_train), so the rate moves k_s.
SURROGATE_RANGES = ((1.0, 500.0), (5e-4, 2e-3), (50.0, 400.0), (0.025, 0.125), (0.01, 1.0), (10.0, 1.0e5))
SURROGATE_LOG = (True, False, True, False, True, True)
MLP_PARAMS = 34049
MLP_HIDDEN = 128


def surrogate_inputs(seed: int, n: int) -> np.ndarray:
    """n input rows [LET, b, V, gap, dose, rate] (float64), log-uniform or
    uniform over SURROGATE_RANGES."""
    rng = np.random.default_rng(seed)
    cols = []
    for (lo, hi), lg in zip(SURROGATE_RANGES, SURROGATE_LOG):
        if lg:
            cols.append(np.exp(rng.uniform(math.log(lo), math.log(hi), n)))
        else:
            cols.append(rng.uniform(lo, hi, n))
    return np.stack(cols, axis=1)


def surrogate_overlap(x) -> float:
    """How many pulse periods the ions of one pulse stay in flight for a
    surrogate sample: rate x T with T = 2 d^2 / (min(mu+, mu-) V) as in
    surrogate_train (below 1 the sample is a single pulse)."""
    V, d, rate = float(x[2]), float(x[3]), float(x[5])
    return rate * 2.0 * d * d / (min(AIR["mu_pos"], AIR["mu_neg"]) * V)


def surrogate_inputs_overlapping(seed: int, n: int, min_overlap: float = 3.0) -> np.ndarray:
    """n input rows drawn as surrogate_inputs draws them, kept only where
    surrogate_overlap is at least min_overlap (deep pulse trains), by
    rejection in the order drawn."""
    rng_seed, out, have = seed, [], 0
    while have < n:
        X = surrogate_inputs(rng_seed, max(4 * n, 4096))
        keep = X[np.array([surrogate_overlap(x) >= min_overlap for x in X])]
        out.append(keep)
        have += len(keep)
        rng_seed += 7919
    return np.concatenate(out)[:n]


def surrogate_train(x):
    """Pulse train of a surrogate sample, (n_pulses, period): with the
    pulse period P = 1 / rate at least T = 2 d^2 / (min(mu+, mu-) V), twice
    the slower ion's transit of the whole gap, a pulse is collected before
    the next arrives and the sample is one pulse, (0, 0.0); otherwise
    N = ceil(T / P) + 1 pulses, so that the last period still holds every
    earlier pulse whose ions are in flight."""
    V, d, rate = float(x[2]), float(x[3]), float(x[5])
    T = 2.0 * d * d / (min(AIR["mu_pos"], AIR["mu_neg"]) * V)
    P = 1.0 / rate
    if P >= T:
        return 0, 0.0
    return int(math.ceil(T / P)) + 1, P


def surrogate_chamber(x, cells: int = 24, b_over_dx: float = 2.5, dz_over_dx: float = 1.25, nz=None):
    """Chamber and track of one surrogate sample: one Gaussian track parallel
    to the field through the centre of a periodic cell of cells x cells nodes
    at spacing b / b_over_dx, gap intervals of about dz_over_dx times that
    spacing (coarser gap intervals let Lax-Wendroff ripples at the ion
    column fronts drive the recombination sink unstable: at 1.5 a few
    fast pulse trains of dense tracks, whose ripples pile up pulse after
    pulse, end non-finite) or exactly nz of them, the dose as uniform pre-ionisation, everything at t = 0 (one
    pulse), repeated as the pulse train of surrogate_train when the rate
    makes pulses overlap."""
    let, b, V, d, dose, _rate = (float(v) for v in x)
    dx = b / b_over_dx
    if nz is None:
        nz = max(8, int(math.ceil(d / (dz_over_dx * dx))))
    ch = chamber(cells, cells, int(nz), dx, d, V, uniform_n0=dose * ion_pairs_per_mGy(AIR["W_eV"]))
    n, P = surrogate_train(x)
    if n:
        ch.update(n_pulses=n, pulse_period_s=P)
    tr = tracks([[let, b, (cells // 2) * dx, (cells // 2) * dx, 0.0, 0.0, 0.0]])
    return ch, tr


def surrogate_resolutions(x, b_over_dx: float = 2.5, dz_over_dx: float = 1.25):
    """The two gap resolutions whose results define a surrogate sample's
    reference ln k_s, with their weights: nz0 = floor(nu) and nz0 + 1 around
    the real plane count nu = d / (dz_over_dx b / b_over_dx), weights
    1 - (nu - nz0) and nu - nz0.  A run at one integer plane count jumps by a
    few 1e-4 in k_s where the count steps; the blend is continuous in the
    inputs."""
    b, d = float(x[1]), float(x[3])
    nu = max(8.0, d / (dz_over_dx * b / b_over_dx))
    n0 = int(math.floor(nu))
    w = nu - n0
    return [(n0, 1.0 - w), (n0 + 1, w)]


def mlp_init(seed: int, members: int) -> np.ndarray:
    """Initial weights [members, MLP_PARAMS] (float32): He-style uniform
    weights, zero biases, in the flat layout W1, b1, W2, b2, W3, b3, w4, b4."""
    rng = np.random.default_rng(seed)
    shapes = ((MLP_HIDDEN, 6), (MLP_HIDDEN,), (MLP_HIDDEN, MLP_HIDDEN), (MLP_HIDDEN,),
              (MLP_HIDDEN, MLP_HIDDEN), (MLP_HIDDEN,), (MLP_HIDDEN,), (1,))
    out = []
    for _ in range(members):
        parts = []
        for k, shape in enumerate(shapes):
            if k % 2 == 1:
                parts.append(np.zeros(shape))
            else:
                fan_in = shape[1] if len(shape) == 2 else shape[0]
                lim = math.sqrt(6.0 / fan_in)
                parts.append(rng.uniform(-lim, lim, shape))
        out.append(np.concatenate([p.ravel() for p in parts]))
    return np.stack(out).astype(np.float32)
