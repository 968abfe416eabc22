"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each checks it against
a closed form, an exact invariant of the discrete scheme, an independent
(dense-matrix) formulation, or a library routine.  They run on the CPU only.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as cf

AIR_MU = 0.5 * (1.73 + 1.87)


# ---------------------------------------------------------------------------
# time step: eq. vNeum
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ch", [
    W.single_track()[0],
    W.pulsed_beam()[0],
    W.chamber(10, 12, 30, 3e-4, 0.03, 100.0, dy=7e-4, D_pos=0.02, D_neg=0.07),
    W.chamber(4, 4, 8, 1e-3, 0.08, 0.0),                       # no field: diffusion only
    W.chamber(4, 4, 8, 1e-3, 0.08, 50.0, D_pos=0.0, D_neg=0.0),  # no diffusion: drift only
])
def test_dt_is_largest_step_satisfying_von_neumann(orc, ch):
    dt = orc.dt(ch)
    lhs = []
    for s in (0, 1):
        c, sx, sy, sz = orc.weights(ch, dt, s)
        # eq. vNeum with c_x = c_y = 0: both inequalities, written out
        assert 0.0 <= 8 * sx * sy * sz + 1e-300
        lhs.append(2 * (sx + sy + sz) + c * c)
    assert max(lhs) <= 1.0 + 1e-14
    assert max(lhs) == pytest.approx(1.0, abs=1e-13)   # largest: the bound is tight
    # 0.1% more would violate the bound for the limiting species
    for s in (0, 1):
        c, sx, sy, sz = orc.weights(ch, dt * 1.001, s)
        lhs[s] = 2 * (sx + sy + sz) + c * c
    assert max(lhs) > 1.0


def test_dt_single_track_value(orc):
    # E = 1500 V/cm, dz = 2e-4 cm: the negative ions (faster) limit dt.
    ch, _ = W.single_track()
    dt = orc.dt(ch)
    A = 2 * 0.045 * 3 / (2e-4) ** 2
    B = (1.87 * 1500 / 2e-4) ** 2
    assert dt == pytest.approx((-A + math.sqrt(A * A + 4 * B)) / (2 * B), rel=1e-14)


def test_dt_safety_factor_scales(orc):
    ch = W.single_track()[0]
    dt1 = orc.dt(ch)
    ch["dt_safety"] = 0.5
    assert orc.dt(ch) == pytest.approx(0.5 * dt1, rel=1e-15)


def test_dt_no_transport_is_an_error(orc):
    ch = W.chamber(4, 4, 8, 1e-3, 0.08, 0.0, D_pos=0.0, D_neg=0.0)
    with pytest.raises(ValueError):
        orc.dt(ch)


def test_reaction_limit_single_track(orc):
    """With the recombination bound active and binding, alpha dt n_ref = rho
    where n_ref is the track's peak density N0/(pi b^2) (eq. Gaussian)."""
    ch, tr = W.single_track(reaction_limit=0.5)
    peak = 100.0 * 1e7 / 34.0 / (math.pi * 1e-6)
    assert orc.reference_density(ch, tr) == pytest.approx(peak, rel=1e-14)
    assert orc.dt(ch, tr) == pytest.approx(0.5 / (1.6e-6 * peak), rel=1e-14)
    assert orc.dt(ch, tr) < orc.dt(ch)
    ch["reaction_limit"] = 0.0
    assert orc.dt(ch, tr) == orc.dt(ch)


def test_reference_density_sums_simultaneous_tracks(orc):
    ch = W.chamber(64, 64, 10, 2e-4, 10 * 2e-4, 20.0, uniform_n0=3e9)
    b1, b2, d = 8e-4, 6e-4, 5e-4
    tr = W.tracks([[40.0, b1, 6e-3, 6e-3, 0.0, 0.0, 0.0],
                   [30.0, b2, 6e-3 + d, 6e-3, 0.0, 0.0, 0.0],
                   [90.0, 6e-4, 6e-3, 6e-3, 0.0, 0.0, 1e-6]])     # later: does not add
    p1 = 40e7 / 34 / (math.pi * b1 * b1)
    p2 = 30e7 / 34 / (math.pi * b2 * b2)
    p3 = 90e7 / 34 / (math.pi * 6e-4 ** 2)
    at1 = p1 + p2 * math.exp(-d * d / (b2 * b2))
    at2 = p2 + p1 * math.exp(-d * d / (b1 * b1))
    expect = 3e9 + max(at1, at2, p3)
    assert orc.reference_density(ch, tr) == pytest.approx(expect, rel=1e-13)


def test_reaction_limit_keeps_dense_pulse_finite(orc):
    """A dense track core (alpha dt n ~ 4 at the transport bound) diverges
    with the transport bound alone and stays finite and conservative with
    the recombination bound."""
    ch = W.chamber(24, 24, 30, 5e-4, 30 * 5e-4, 30.0, reaction_limit=0.0)
    tr = W.tracks([[60.0, 5e-4, 6e-3, 6e-3, 0.0, 0.0, 0.0]])
    r = orc.solve(ch, tr, with_fields=False)
    assert r["flags"] & 2 and r["max_beta_n"] > 1.0
    ch["reaction_limit"] = 0.5
    r = orc.solve(ch, tr, with_trace=True, with_fields=False)
    assert r["flags"] == 0 and r["max_beta_n"] <= 0.5 * (1 + 1e-12)
    _check_conservation(r)
    assert 0.0 < r["f"] < 1.0


def _checkerboard(ch, amp=1.0):
    shape = (ch["nz"] + 1, ch["ny"], ch["nx"])
    k, j, i = np.indices(shape)
    f = amp * (1.0 + 0.5 * (-1.0) ** (i + j + k))
    f[0] = 0.0
    f[-1] = 0.0
    return np.ascontiguousarray(f)


@pytest.mark.parametrize("ch", [
    # diffusion-limited: no field, the checkerboard stays in the grid
    W.chamber(8, 8, 40, 2e-4, 40 * 2e-4, 0.0, alpha=0.0),
    # drift-limited: small diffusion, long gap so the mode stays in flight
    W.chamber(4, 4, 600, 2e-4, 600 * 2e-4, 30.0, alpha=0.0, D_pos=1e-4, D_neg=1e-4),
])
def test_stable_at_kappa_one_unstable_beyond(orc, ch):
    """The paper's bound is the edge of stability: the most oscillatory mode
    does not grow at kappa = 1 and blows up with a 5% larger step."""
    f = _checkerboard(ch)
    dt = orc.dt(ch)
    p, n = orc.advance(ch, dt, f, f, 250)
    # Lax-Wendroff is not monotone, so allow a small overshoot, not growth
    assert max(np.max(np.abs(p)), np.max(np.abs(n))) <= 2.0
    p, n = orc.advance(ch, dt * 1.05, f, f, 250)
    assert max(np.max(np.abs(p)), np.max(np.abs(n))) > 1e3


# ---------------------------------------------------------------------------
# one step against an independent dense-matrix formulation (Appendix)
# ---------------------------------------------------------------------------

def _dense_step(ch, dt, pos, neg):
    """n^{l+1} = n^l + dt [ D (Dxx + Dyy + Dzz) n - v Dz n ] - alpha dt n+ n-,
    with the Appendix's derivative matrices assembled on the full node grid
    (electrode planes included), then the electrode planes read out as the
    collected amounts and reset to zero."""
    nx, ny, nz = ch["nx"], ch["ny"], ch["nz"]
    dx, dy, dz = ch["dx"], ch["dy"], ch["gap"] / nz
    E = ch["voltage"] / ch["gap"]
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz + 1)

    def periodic_second(m, h):
        M = -2 * np.eye(m)
        for a in range(m):
            M[a, (a + 1) % m] += 1
            M[a, (a - 1) % m] += 1
        return M / h ** 2

    def open_shift(m, off):
        return np.eye(m, k=off)  # (S n)_a = n_{a+off}, zero outside

    Dxx = np.kron(np.kron(Iz, Iy), periodic_second(nx, dx))
    Dyy = np.kron(np.kron(Iz, periodic_second(ny, dy)), Ix)
    up, down = open_shift(nz + 1, 1), open_shift(nz + 1, -1)
    Dzz1 = (up - 2 * Iz + down) / dz ** 2
    Dzz = np.kron(np.kron(Dzz1, Iy), Ix)
    backward = (Iz - down) / dz          # (n_k - n_{k-1})/dz
    central = (up - down) / (2 * dz)     # (n_{k+1} - n_{k-1})/(2 dz)
    out, col = [], []
    for s, (mu, D, sign) in enumerate([(ch["mu_pos"], ch["D_pos"], 1.0), (ch["mu_neg"], ch["D_neg"], -1.0)]):
        v = sign * mu * E
        c = v * dt / dz
        Dz1 = c * backward + (1 - c) * central
        Dz = np.kron(np.kron(Dz1, Iy), Ix)
        M = np.eye((nz + 1) * ny * nx) + dt * (D * (Dxx + Dyy + Dzz) - v * Dz)
        n_old = (pos, neg)[s].ravel()
        n_new = M @ n_old - ch["alpha"] * dt * pos.ravel() * neg.ravel()
        n_new = n_new.reshape(nz + 1, ny, nx)
        dV = dx * dy * dz
        col.append((n_new[0].sum() * dV, n_new[nz].sum() * dV))
        n_new[0] = 0.0
        n_new[nz] = 0.0
        out.append(n_new)
    return out[0], out[1], col


@pytest.mark.parametrize("geom", [(4, 4, 5), (3, 5, 2), (1, 1, 7)])
def test_one_step_matches_dense_matrix_scheme(orc, geom):
    nx, ny, nz = geom
    ch = W.chamber(nx, ny, nz, 3e-4, nz * 2.5e-4, 40.0, dy=4e-4, D_pos=0.03, D_neg=0.05,
                   alpha=1.6e-6)
    dt = orc.dt(ch)
    pos, neg = W.perturbed_field((nz + 1, ny, nx), seed=7, scale=3e11)
    p1, n1, tally = orc.step(ch, dt, pos, neg)
    p2, n2, col = _dense_step(ch, dt, pos, neg)
    scale = max(np.abs(pos).max(), np.abs(neg).max())
    assert np.max(np.abs(p1 - p2)) <= 1e-14 * scale
    assert np.max(np.abs(n1 - n2)) <= 1e-14 * scale
    dV = ch["dx"] * ch["dy"] * ch["gap"] / nz
    tot = (pos.sum() + neg.sum()) * dV
    assert tally["pos_anode"] == pytest.approx(col[0][0], abs=1e-13 * tot)
    assert tally["pos_cathode"] == pytest.approx(col[0][1], abs=1e-13 * tot)
    assert tally["neg_anode"] == pytest.approx(col[1][0], abs=1e-13 * tot)
    assert tally["neg_cathode"] == pytest.approx(col[1][1], abs=1e-13 * tot)
    rec = ch["alpha"] * dt * np.sum(pos[1:nz] * neg[1:nz]) * dV
    assert tally["recombined"] == pytest.approx(rec, rel=1e-13)
    assert tally["pos_inflight"] == pytest.approx(p2.sum() * dV, rel=1e-13)
    assert tally["neg_abs"] == pytest.approx(np.abs(n2).sum() * dV, rel=1e-13)


# ---------------------------------------------------------------------------
# exact discrete invariants: moments of the scheme (P3, P3c)
# ---------------------------------------------------------------------------

def _blob(ch, centre, sigma):
    shape = (ch["nz"] + 1, ch["ny"], ch["nx"])
    k, j, i = np.indices(shape).astype(float)
    r2 = ((i - centre[0]) ** 2 + (j - centre[1]) ** 2 + (k - centre[2]) ** 2)
    f = 1e10 * np.exp(-r2 / (2 * sigma ** 2))
    f[0] = 0.0
    f[-1] = 0.0
    return np.ascontiguousarray(f)


def _moments(f, axis_len, axis, h):
    coords = np.arange(axis_len) * h
    m0 = f.sum()
    proj = f.sum(axis=tuple(a for a in range(3) if a != axis))
    m1 = (proj * coords).sum() / m0
    var = (proj * (coords - m1) ** 2).sum() / m0
    return m0, m1, var


def test_pure_diffusion_moments_exact(orc):
    """E = 0, alpha = 0: mass and mean are constant and every axis' variance
    grows by exactly 2 D dt per step (explicit 3-point diffusion)."""
    ch = W.chamber(48, 40, 44, 2e-4, 44 * 2.5e-4, 0.0, dy=3e-4, alpha=0.0, D_pos=0.03, D_neg=0.05)
    dt = orc.dt(ch)
    f = _blob(ch, (24, 20, 22), 1.6)
    steps = 12
    p, n = orc.advance(ch, dt, f, f, steps)
    for field, D in ((p, 0.03), (n, 0.05)):
        for axis, L, h in ((2, 48, 2e-4), (1, 40, 3e-4), (0, 45, 2.5e-4)):
            m0a, m1a, va = _moments(f, L, axis, h)
            m0b, m1b, vb = _moments(field, L, axis, h)
            assert m0b == pytest.approx(m0a, rel=1e-13)
            assert m1b == pytest.approx(m1a, rel=1e-13)
            assert vb - va == pytest.approx(2 * D * dt * steps, rel=1e-10)


def test_drift_diffusion_moments_exact(orc):
    """alpha = 0, E > 0: the z-mean moves by exactly v dt per step (v = +mu+ E
    for positive, -mu- E for negative ions) and the z-variance still grows by
    exactly 2 D dt per step (Lax-Wendroff adds no variance)."""
    ch = W.chamber(8, 8, 160, 2e-4, 160 * 2e-4, 40.0, alpha=0.0, D_pos=0.02, D_neg=0.04)
    dt = orc.dt(ch)
    E = ch["voltage"] / ch["gap"]
    f = _blob(ch, (4, 4, 80), 3.0)
    steps = 10
    p, n = orc.advance(ch, dt, f, f, steps)
    dz = ch["gap"] / ch["nz"]
    for field, v, D in ((p, 1.73 * E, 0.02), (n, -1.87 * E, 0.04)):
        m0a, m1a, va = _moments(f, 161, 0, dz)
        m0b, m1b, vb = _moments(field, 161, 0, dz)
        assert m0b == pytest.approx(m0a, rel=1e-13)
        assert m1b - m1a == pytest.approx(v * dt * steps, rel=1e-10)
        assert vb - va == pytest.approx(2 * D * dt * steps, rel=1e-9)


def _spread_track_error(orc, refine):
    """Max-norm error, relative to the peak, of the mid-gap profile of a
    track column after pure diffusion to b^2 + 4 D t = 2 b^2, against the
    spread Gaussian N0/(pi (b^2 + 4 D t)) exp(-r^2/(b^2 + 4 D t)) (eq.
    Gaussian with the radius of a diffusing column), for both species."""
    b = 1e-3
    h = b / (4 * refine)
    n = 40 * refine
    D = {"pos": 0.03, "neg": 0.05}
    ch = W.chamber(n, n, n, h, n * 2 * h, 0.0, alpha=0.0, D_pos=D["pos"], D_neg=D["neg"],
                   dt_safety=0.5, stop_tol=0.0)
    tr = W.tracks([[10.0, b, (n // 2) * h, (n // 2) * h, 0.0, 0.0, 0.0]])
    dt = orc.dt(ch)
    steps = 36 * refine * refine        # t = b^2/(4 D_neg) at both resolutions
    ch["max_steps"] = steps
    r = orc.solve(ch, tr)
    t = steps * dt
    j, i = np.indices((n, n))
    r2 = ((i - n // 2) * h) ** 2 + ((j - n // 2) * h) ** 2
    N0 = 10.0 * 1e7 / 34.0
    err = {}
    for s in ("pos", "neg"):
        w2 = b * b + 4 * D[s] * t
        exact = N0 / (math.pi * w2) * np.exp(-r2 / w2)
        err[s] = np.max(np.abs(r[s][n // 2] - exact)) / exact.max()
    return err, dt


def test_gaussian_track_spreading_converges_at_second_order(orc):
    """P3b: a Gaussian column under pure diffusion stays Gaussian with
    b^2 -> b^2 + 4 D t.  The explicit scheme reaches that profile with an
    O(dx^2) + O(dt) error, so halving every spacing (dt / 4, four times the
    steps) divides the error by about 4."""
    e1, dt1 = _spread_track_error(orc, 1)
    e2, dt2 = _spread_track_error(orc, 2)
    assert dt2 == pytest.approx(dt1 / 4, rel=1e-14)
    for s in ("pos", "neg"):
        assert e1[s] < 2e-2
        assert 3.6 < e1[s] / e2[s] < 4.4, (s, e1[s], e2[s])


# ---------------------------------------------------------------------------
# deposition: eqs. linear_density, Gaussian, created; requirement (i)
# ---------------------------------------------------------------------------

def _lattice_sum(b, h, x0):
    """h/(b sqrt(pi)) sum_m exp(-(m h - x0)^2 / b^2) by Poisson summation:
    1 + 2 sum_k exp(-pi^2 k^2 b^2/h^2) cos(2 pi k x0/h)."""
    return 1.0 + 2.0 * sum(math.exp(-(math.pi * k * b / h) ** 2) * math.cos(2 * math.pi * k * x0 / h)
                           for k in range(1, 8))


@pytest.mark.parametrize("b_over_h,frac", [(1.0, 0.0), (1.0, 0.37), (0.8, 0.5), (1.5, 0.21), (5.0, 0.0)])
def test_released_count_matches_poisson_summation(orc, b_over_h, frac):
    """I0 = dx dy sum n0 = N0 * Sx * Sy exactly, where S is the Gaussian's
    lattice sum; a coarse grid makes S measurably differ from 1."""
    h = 2e-4
    b = b_over_h * h
    n_cells = int(math.ceil(24 * b / h)) + 2
    ch = W.chamber(n_cells, n_cells, 6, h, 6 * 2e-4, 10.0)
    x0 = (n_cells // 2 + frac) * h
    y0 = (n_cells // 2 + 0.5 * frac) * h
    let = 7.5
    tr = W.tracks([[let, b, x0, y0, 0.0, 0.0, 0.0]])
    dt = orc.dt(ch)
    _, _, rel = orc.deposit(ch, tr, 0, dt)
    N0 = let * 1e7 / 34.0
    expect = N0 * (ch["nz"] - 1) * (ch["gap"] / ch["nz"]) * _lattice_sum(b, h, frac * h) * \
        _lattice_sum(b, h, 0.5 * frac * h)
    assert rel == pytest.approx(expect, rel=1e-13)


@pytest.mark.parametrize("theta,phi", [(math.radians(20), 0.3), (math.radians(30), 2.2), (math.radians(55), 4.0)])
def test_tilted_track_line_density(orc, theta, phi):
    """A track at angle theta crosses every plane z = const with N0/cos(theta)
    ion pairs per unit height (eq. created with l = d/cos theta)."""
    h = 2e-4
    b = 5 * h
    ch = W.chamber(96, 96, 20, h, 20 * 2e-4, 10.0)
    tr = W.tracks([[2.0, b, 48 * h + 1e-5, 47 * h, theta, phi, 0.0]])
    _, _, rel = orc.deposit(ch, tr, 0, orc.dt(ch))
    N0 = 2.0 * 1e7 / 34.0
    assert rel == pytest.approx(N0 * (ch["nz"] - 1) * (ch["gap"] / ch["nz"]) / math.cos(theta), rel=1e-12)


def test_deposit_profile_is_gaussian_in_perpendicular_distance(orc):
    ch = W.chamber(32, 32, 10, 2e-4, 10 * 2e-4, 10.0)
    th, ph = 0.4, 1.1
    x0, y0 = 16 * 2e-4 + 3e-5, 15 * 2e-4
    b = 1.2e-3
    tr = W.tracks([[3.0, b, x0, y0, th, ph, 0.0]])
    pos, neg, _ = orc.deposit(ch, tr, 0, orc.dt(ch))
    u = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    N0 = 3.0 * 1e7 / 34.0
    for (k, j, i) in [(5, 16, 16), (3, 14, 19), (8, 20, 12), (1, 16, 16), (9, 10, 22)]:
        p = np.array([i * 2e-4 - x0, j * 2e-4 - y0, k * 2e-4 - 1e-3])
        r2 = float(p @ p - (p @ u) ** 2)
        val = N0 / (math.pi * b * b) * math.exp(-r2 / b ** 2) if r2 <= 64 * b * b else 0.0
        assert pos[k, j, i] == pytest.approx(val, rel=1e-12, abs=1e-300)
        assert neg[k, j, i] == pos[k, j, i]
    assert np.all(pos[0] == 0) and np.all(pos[-1] == 0)


def test_track_deposited_at_floor_of_time_over_dt(orc):
    ch, _ = W.single_track(max_steps=6, stop_tol=0.0)
    dt = orc.dt(ch, W.tracks([[1.0, 1e-3, 32 * 2e-4, 32 * 2e-4, 0.0, 0.0, 0.0]]))
    tr = W.tracks([[1.0, 1e-3, 32 * 2e-4, 32 * 2e-4, 0.0, 0.0, 2.999 * dt],
                   [1.0, 1e-3, 32 * 2e-4, 32 * 2e-4, 0.0, 0.0, 40 * dt]])   # beyond max_steps
    r = orc.solve(ch, tr, with_trace=True, with_fields=False)
    tr_ = r["trace"]
    assert np.all(tr_[:2, 5] == 0.0) and tr_[2, 5] > 0.0
    one = orc.deposit(ch, tr[:1], 2, dt)[2]
    assert r["n_released"] == pytest.approx(one, rel=1e-15)


# ---------------------------------------------------------------------------
# conservation (P1), alpha -> 0 (P2)
# ---------------------------------------------------------------------------

def _check_conservation(r, tol=1e-12):
    """released = collected + recombined + in flight - space-charge change,
    step by step and species by species (the released column holds what was
    deposited before each step)."""
    tr = r["trace"]
    N = r["n_released"]
    assert tr[:, 9].sum() == pytest.approx(N, rel=1e-14)
    assert tr[:, 12].sum() == pytest.approx(r["n_released_neg"], rel=1e-14)
    for s, (a, c, S, Q, rel, X) in enumerate(((1, 2, 5, 10, 9, 13), (3, 4, 6, 11, 12, 14))):
        prev = np.concatenate([[0.0], tr[:-1, S]]) + tr[:, rel]
        err = prev - tr[:, a] - tr[:, c] - tr[:, 0] + tr[:, Q] - tr[:, X] - tr[:, S]
        assert np.max(np.abs(err)) <= tol * N


def test_conservation_single_track(orc):
    ch, tr = W.single_track()
    r = orc.solve(ch, tr, with_trace=True, with_fields=False)
    _check_conservation(r)
    assert r["flags"] == 0
    assert r["f"] == pytest.approx(r["f_R"], abs=2e-12)


def test_conservation_tilted_tracks_and_uniform(orc):
    ch = W.chamber(24, 20, 30, 3e-4, 30 * 3e-4, 20.0, uniform_n0=3e9)
    tr = W.tracks([[20.0, 8e-4, 1e-3, 2e-3, 0.4, 1.0, 0.0],
                   [5.0, 6e-4, 5e-3, 1e-3, 0.2, 4.0, 1e-7]])
    r = orc.solve(ch, tr, with_trace=True, with_fields=False)
    _check_conservation(r)


def test_conservation_with_space_charge(orc):
    ch = W.chamber(24, 20, 30, 3e-4, 30 * 3e-4, 20.0, uniform_n0=3e9, space_charge=1)
    tr = W.tracks([[60.0, 8e-4, 1e-3, 2e-3, 0.4, 1.0, 0.0],
                   [25.0, 6e-4, 5e-3, 1e-3, 0.0, 0.0, 1e-7]])
    r = orc.solve(ch, tr, with_trace=True, with_fields=False)
    _check_conservation(r)
    assert r["flags"] == 0
    # the screening term removes ions of the charge in excess: n+ where the
    # positive ions have drifted ahead, n- where the negative ones have
    assert r["n_space_charge_pos"] < 0.0 and r["n_space_charge_neg"] < 0.0
    assert r["n_space_charge_pos"] == pytest.approx(r["trace"][:, 10].sum(), rel=1e-12)


# ---------------------------------------------------------------------------
# separate track radii of the two species (b- > b+, "The charge carrier
# distribution in the track")
# ---------------------------------------------------------------------------

def _with_bneg(tr, factor):
    out = np.concatenate([tr, np.zeros((tr.shape[0], 1))], axis=1)
    out[:, 7] = factor * tr[:, 1]
    return out


def test_equal_radii_reproduce_the_shared_radius(orc):
    ch, tr = W.single_track(max_steps=40, stop_tol=0.0)
    tr[0, 0] = 20.0
    a = orc.solve(ch, tr)
    b = orc.solve(ch, _with_bneg(tr, 1.0))
    assert a["f"] == b["f"] and np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["neg"], b["neg"])


def test_separate_radii_conservation_and_released(orc):
    ch, tr = W.single_track()
    tr[0, 0] = 20.0
    r = orc.solve(ch, _with_bneg(tr, 1.5), with_trace=True, with_fields=False)
    _check_conservation(r)
    # both species carry N0 per unit length (Poisson summation of the
    # columns); the wider one loses the Gaussian's mass beyond the minimum
    # image, half a cell = 4.3 b- away: e^{-4.3^2} ~ 1e-8
    N0l = 20.0 * 1e7 / ch["W_eV"] * ch["gap"] * (ch["nz"] - 1) / ch["nz"]
    assert r["n_released"] == pytest.approx(N0l, rel=1e-9)
    assert r["n_released_neg"] == pytest.approx(N0l, rel=1e-7)
    assert r["f"] == pytest.approx((r["col_pos_anode"] + r["col_pos_cathode"] + r["col_neg_anode"]
                                    + r["col_neg_cathode"]) / (r["n_released"] + r["n_released_neg"]), rel=1e-14)


def test_wider_negative_track_recombines_less(orc):
    """A wider negative-ion column overlaps the positive one less densely:
    f rises from (b, b) to (b, 1.5 b), and stays below (1.5 b, 1.5 b)."""
    ch, tr = W.single_track()
    tr[0, 0] = 20.0
    f_bb = orc.solve(ch, tr, with_fields=False)["f"]
    f_bw = orc.solve(ch, _with_bneg(tr, 1.5), with_fields=False)["f"]
    wide = tr.copy()
    wide[0, 1] *= 1.5
    f_ww = orc.solve(ch, wide, with_fields=False)["f"]
    assert f_bb < f_bw < f_ww


def test_separate_radii_swap_mirror_symmetry(orc):
    """Exchanging the species (mobilities, diffusion constants and radii)
    and mirroring z maps the run onto itself."""
    base = dict(mu_pos=1.73, mu_neg=1.87, D_pos=0.045, D_neg=0.06)
    swap = dict(mu_pos=1.87, mu_neg=1.73, D_pos=0.06, D_neg=0.045)
    ch1, tr = W.single_track(**base)
    ch2, _ = W.single_track(**swap)
    tr[0, 0] = 20.0
    t1 = _with_bneg(tr, 1.4)
    t2 = t1.copy()
    t2[0, 1], t2[0, 7] = t1[0, 7], t1[0, 1]
    ch1["max_steps"] = ch2["max_steps"] = 60
    ch1["stop_tol"] = ch2["stop_tol"] = 0.0
    r1 = orc.solve(ch1, t1)
    r2 = orc.solve(ch2, t2)
    assert r2["f"] == pytest.approx(r1["f"], rel=1e-12)
    scale = max(r1["neg"].max(), r1["pos"].max())
    assert np.max(np.abs(r2["pos"] - r1["neg"][::-1])) <= 1e-12 * scale
    assert np.max(np.abs(r2["neg"] - r1["pos"][::-1])) <= 1e-12 * scale


# ---------------------------------------------------------------------------
# space-charge screening (eq. theEquation's n div E, div E by Maxwell-Gauss)
# ---------------------------------------------------------------------------

Q_OVER_EPS0 = 1.602176634e-19 / 8.8541878128e-14   # V cm


def _pointwise_case(space_charge=1, **consts):
    # no field, no diffusion: every node evolves on its own
    return W.chamber(3, 2, 6, 1e-3, 6e-3, 0.0, D_pos=0.0, D_neg=0.0, space_charge=space_charge, **consts)


def test_space_charge_pointwise_map(orc):
    """With no field and no diffusion the update at each node is the map
    n+' = n+ - b n+ n- - m+ dt (q/eps0) n+ (n+ - n-) and
    n-' = n- - b n+ n- + m- dt (q/eps0) n- (n+ - n-), written out here."""
    ch = _pointwise_case()
    rng = np.random.default_rng(3)
    shape = (7, 2, 3)
    p0 = rng.uniform(1e10, 5e11, shape)
    n0 = rng.uniform(1e10, 5e11, shape)
    p0[0] = p0[-1] = n0[0] = n0[-1] = 0.0
    dt = 2e-8
    op, on = orc.advance(ch, dt, p0, n0, 5)
    P, N = p0.copy(), n0.copy()
    b = ch["alpha"] * dt
    for _ in range(5):
        net = P - N
        P, N = (P - b * P * N - ch["mu_pos"] * dt * Q_OVER_EPS0 * P * net,
                N - b * P * N + ch["mu_neg"] * dt * Q_OVER_EPS0 * N * net)
        P[0] = P[-1] = N[0] = N[-1] = 0.0
    assert np.max(np.abs(op - P)) <= 1e-13 * P.max()
    assert np.max(np.abs(on - N)) <= 1e-13 * N.max()


def test_space_charge_single_species_decay(orc):
    """One species alone, no field, no diffusion, no recombination: the
    screening term gives dn/dt = -mu q n^2/eps0, whose solution is
    n0 / (1 + mu q n0 t / eps0); the explicit update converges to it at
    first order in dt."""
    ch = _pointwise_case(alpha=0.0)
    n0 = 2e11
    shape = (7, 2, 3)
    P0 = np.zeros(shape)
    P0[1:-1] = n0
    T = 4e-6
    exact = n0 / (1.0 + ch["mu_pos"] * Q_OVER_EPS0 * n0 * T)
    errs = []
    for steps in (50, 100, 200):
        op, _ = orc.advance(ch, T / steps, P0, np.zeros(shape), steps)
        errs.append(abs(op[3, 1, 1] - exact) / exact)
    assert errs[-1] < 1e-2
    for a, b_ in zip(errs[:-1], errs[1:]):
        assert 0.45 < b_ / a < 0.55


def test_space_charge_vanishes_for_neutral_plasma(orc):
    """Equal densities of both species carry no net charge: the runs with and
    without the term are identical."""
    ch0 = W.chamber(20, 18, 24, 3e-4, 24 * 3e-4, 20.0, uniform_n0=5e9, max_steps=30, stop_tol=0.0)
    ch1 = dict(ch0, space_charge=1)
    d0 = orc.dt(ch0)
    p, n, _ = orc.uniform(ch0, 5e9)
    a = orc.step(ch0, d0, p, n)
    b = orc.step(ch1, d0, p, n)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert b[2]["pos_space_charge"] == 0.0 and b[2]["neg_space_charge"] == 0.0


def test_space_charge_dt_bound(orc):
    """With the term on, the reaction bound uses k = alpha + max(mu) q/eps0."""
    ch, tr = W.single_track(space_charge=1)
    nref = orc.reference_density(ch, tr)
    k = ch["alpha"] + max(ch["mu_pos"], ch["mu_neg"]) * Q_OVER_EPS0
    expect = min(orc.dt(dict(ch, reaction_limit=0.0)), ch["reaction_limit"] / (k * nref))
    assert orc.dt(ch, tr) == pytest.approx(expect, rel=1e-14)
    assert orc.dt(ch, tr) < orc.dt(dict(ch, space_charge=0), tr)


def test_space_charge_swap_mirror_symmetry(orc):
    """The term keeps the species-swap symmetry: -mu+ n+ (n+ - n-) for n+ and
    +mu- n- (n+ - n-) for n- exchange roles when the species do."""
    base = dict(mu_pos=1.73, mu_neg=1.87, D_pos=0.045, D_neg=0.06, space_charge=1)
    swap = dict(mu_pos=1.87, mu_neg=1.73, D_pos=0.06, D_neg=0.045, space_charge=1)
    ch1, tr = W.single_track(**base)
    ch2, _ = W.single_track(**swap)
    tr[0, 0] = 20.0
    ch1["max_steps"] = ch2["max_steps"] = 60
    ch1["stop_tol"] = ch2["stop_tol"] = 0.0
    r1 = orc.solve(ch1, tr)
    r2 = orc.solve(ch2, tr)
    assert r1["n_space_charge_pos"] != 0.0
    assert r2["f"] == pytest.approx(r1["f"], rel=1e-12)
    assert r2["n_space_charge_pos"] == pytest.approx(r1["n_space_charge_neg"], rel=1e-10)
    scale = max(r1["neg"].max(), r1["pos"].max())
    assert np.max(np.abs(r2["pos"] - r1["neg"][::-1])) <= 1e-12 * scale


def test_no_recombination_collects_everything(orc):
    ch, tr = W.single_track(alpha=0.0)
    r = orc.solve(ch, tr, with_fields=False)
    assert abs(1.0 - r["f"]) <= 2e-12
    assert r["n_recombined"] == 0.0


# ---------------------------------------------------------------------------
# exact symmetries and linearity (P6-P8)
# ---------------------------------------------------------------------------

def test_species_swap_mirror_symmetry(orc):
    base = dict(mu_pos=1.73, mu_neg=1.87, D_pos=0.045, D_neg=0.06)
    swap = dict(mu_pos=1.87, mu_neg=1.73, D_pos=0.06, D_neg=0.045)
    ch1, tr = W.single_track(**base)
    ch2, _ = W.single_track(**swap)
    tr[0, 0] = 20.0
    ch1["max_steps"] = ch2["max_steps"] = 60        # both species still in flight
    ch1["stop_tol"] = ch2["stop_tol"] = 0.0
    r1 = orc.solve(ch1, tr)
    r2 = orc.solve(ch2, tr)
    assert r2["f"] == pytest.approx(r1["f"], rel=1e-12)
    assert r2["col_pos_anode"] == pytest.approx(r1["col_neg_cathode"], rel=1e-10)
    assert r2["col_pos_cathode"] == pytest.approx(r1["col_neg_anode"], rel=1e-10)
    scale = max(r1["neg"].max(), r1["pos"].max())
    assert np.max(np.abs(r2["pos"] - r1["neg"][::-1])) <= 1e-12 * scale
    assert np.max(np.abs(r2["neg"] - r1["pos"][::-1])) <= 1e-12 * scale


def test_periodic_translation_invariance(orc):
    ch, tr = W.single_track(max_steps=60, stop_tol=0.0)
    tr[0, 0] = 30.0
    tr[0, 2] += 0.3e-4
    r1 = orc.solve(ch, tr)
    tr2 = tr.copy()
    tr2[0, 2] += 7 * ch["dx"]
    tr2[0, 3] -= 11 * ch["dy"]
    r2 = orc.solve(ch, tr2)
    assert r2["f"] == pytest.approx(r1["f"], rel=1e-12)
    shifted = np.roll(np.roll(r1["pos"], 7, axis=2), -11, axis=1)
    assert np.max(np.abs(r2["pos"] - shifted)) <= 1e-10 * r1["pos"].max()


def test_linear_superposition_without_recombination(orc):
    ch = W.chamber(20, 18, 24, 3e-4, 24 * 3e-4, 20.0, alpha=0.0, max_steps=25, stop_tol=0.0)
    A = W.tracks([[5.0, 9e-4, 2e-3, 3e-3, 0.3, 0.5, 0.0]])
    B = W.tracks([[9.0, 6e-4, 4e-3, 1e-3, 0.0, 0.0, 0.0]])
    ra, rb = orc.solve(ch, A), orc.solve(ch, B)
    rab = orc.solve(ch, np.concatenate([A, B]))
    scale = rab["pos"].max()
    assert np.max(np.abs(rab["pos"] - ra["pos"] - rb["pos"])) <= 1e-13 * scale
    assert np.max(np.abs(rab["neg"] - ra["neg"] - rb["neg"])) <= 1e-13 * scale


# ---------------------------------------------------------------------------
# physics: Boag (pulsed general recombination) and Jaffe (initial recombination)
# ---------------------------------------------------------------------------

def _boag_run(orc, u, nz, D):
    V, d = 200.0, 0.1
    n0 = u * (1.73 + 1.87) * V / (1.6e-6 * d * d)
    ch = W.chamber(1, 1, nz, 1e-3, d, V, uniform_n0=n0, D_pos=D, D_neg=D)
    r = orc.solve(ch, W.no_tracks(), with_fields=False)
    return r["f"], cf.boag(cf.boag_u(n0, d, V, 1.73, 1.87, 1.6e-6))


@pytest.mark.parametrize("u", [0.1, 1.0, 10.0])
def test_boag_pulsed_general_recombination(orc, u):
    """Uniform pre-ionisation between the plates, no diffusion to speak of:
    the solver converges to f = ln(1+u)/u at first order in dz."""
    errs = []
    for nz in (400, 800, 1600):
        f, fb = _boag_run(orc, u, nz, 1e-4)
        errs.append((f - fb) / fb)
    assert abs(errs[-1]) < 2.5e-3 * max(u, 0.1) ** 0.5 + 1e-5
    for a, b in zip(errs[:-1], errs[1:]):
        assert 0.4 < b / a < 0.6          # first-order convergence toward Boag


def test_boag_with_air_diffusion_two_percent(orc):
    for u in (0.1, 1.0, 10.0):
        f, fb = _boag_run(orc, u, 200, 0.045)
        assert abs(f - fb) / fb < 0.02


@pytest.mark.parametrize("let", [0.1, 0.3, 1.0])
def test_jaffe_parallel_track(orc, let):
    """A single track parallel to the field in the weak-recombination regime
    Jaffe's theory describes: the recombined fraction agrees within 5%."""
    ch, tr = W.single_track()
    tr[0, 0] = let
    r = orc.solve(ch, tr, with_fields=False)
    fj = cf.jaffe_parallel(let, 1e-3, ch["voltage"] / ch["gap"], ch["gap"], 0.045, AIR_MU, 1.6e-6)
    assert abs((1 - r["f"]) / (1 - fj) - 1) < 0.05


def _tilted_single_track(orc, let, deg):
    ch, tr = W.single_track()
    tr[0, 0] = let
    tr[0, 4] = math.radians(deg)
    return orc.solve(ch, tr, with_fields=False), ch


@pytest.mark.parametrize("deg", [30, 45, 60, 90])
def test_jaffe_angular_formula_for_tilted_tracks(orc, deg):
    """A single track at angle theta to the field (eq. angle) in the regime
    the paper compares, theta in [pi/6, pi/2]: the recombined fraction agrees
    with Jaffe's angular formula within 15%."""
    r, ch = _tilted_single_track(orc, 1.0, deg)
    fj = cf.jaffe_angle(1.0, 1e-3, ch["voltage"] / ch["gap"], math.radians(deg), 0.045, AIR_MU, 1.6e-6)
    assert r["flags"] == 0
    assert abs((1 - r["f"]) / (1 - fj) - 1) < 0.15


def test_tilting_a_track_reduces_recombination(orc):
    """Columnar recombination falls as the track turns away from the field:
    f grows monotonically from the parallel track (eq. Jaffe_noangle) to the
    track parallel to the electrodes, as both of Jaffe's formulas order it."""
    fs = [_tilted_single_track(orc, 3.0, deg)[0]["f"] for deg in (0, 15, 30, 45, 60, 90)]
    assert all(b > a for a, b in zip(fs[:-1], fs[1:]))
    ch, _ = W.single_track()
    E = ch["voltage"] / ch["gap"]
    assert fs[0] < cf.jaffe_angle(3.0, 1e-3, E, math.radians(30), 0.045, AIR_MU, 1.6e-6) < fs[-1] + 0.01


# ---------------------------------------------------------------------------
# degenerate inputs
# ---------------------------------------------------------------------------

def test_empty_track_list(orc):
    ch = W.chamber(4, 4, 6, 1e-3, 6e-3, 10.0)
    r = orc.solve(ch, W.no_tracks(), with_fields=False)
    assert r["f"] == 1.0 and r["flags"] & 8 and r["steps"] == 1


def test_single_interior_plane(orc):
    ch = W.chamber(6, 6, 2, 2e-4, 4e-4, 5.0)
    tr = W.tracks([[10.0, 4e-4, 6e-4, 6e-4, 0.0, 0.0, 0.0]])
    r = orc.solve(ch, tr, with_trace=True, with_fields=False)
    _check_conservation(r)
    assert 0.0 < r["f"] <= 1.0


def test_stop_rule_first_step_below_tolerance_after_the_last_deposit(orc):
    """R8 read off the per-step records: the run ends at the first step at
    or after its last deposit whose sums of |n| dV are within stop_tol of
    each species' release.  Here the chamber already falls below the
    tolerance before a late track arrives (the rule waits for it), and the
    signed in-flight sums fall below it a few steps before the absolute
    ones (the rule uses the absolute sums)."""
    ch = W.chamber(12, 10, 16, 3e-4, 16 * 3e-4, 20.0, stop_tol=1e-3)
    tr = W.tracks([[20.0, 8e-4, 1.8e-3, 1.5e-3, 0.0, 0.0, 0.0],
                   [10.0, 6e-4, 1e-3, 1e-3, 0.3, 1.0, 3e-6]])
    r = orc.solve(ch, tr, with_trace=True, with_fields=False)
    assert r["flags"] == 0
    t = r["trace"]
    tol = ch["stop_tol"]
    last = int(np.flatnonzero(t[:, 9])[-1])
    assert last == int(math.floor(3e-6 / r["dt"]))
    below = (t[:, 7] <= tol * r["n_released"]) & (t[:, 8] <= tol * r["n_released_neg"])
    assert below[-1] and not below[last:-1].any()
    assert below[:last].any()
    signed = (t[:, 5] <= tol * r["n_released"]) & (t[:, 6] <= tol * r["n_released_neg"])
    assert signed[last:-1].any()


def test_max_steps_flag(orc):
    ch, tr = W.single_track(max_steps=10)
    r = orc.solve(ch, tr, with_fields=False)
    assert r["steps"] == 10 and r["flags"] & 1


# ---------------------------------------------------------------------------
# free-electron component (eqs. free_elec, ion_elec_distribution, model1-3)
# ---------------------------------------------------------------------------

def _attach_for(p_target, d):
    lo, hi = 1e-9, 1e7
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if cf.free_electron_fraction(mid, d) > p_target:
            lo = mid
        else:
            hi = mid
    return mid


def _fe_chamber(p_target, V, n0=3e9, d=0.1, nz=100, mu_e=1500.0):
    ch = W.chamber(2, 2, nz, 1e-3, d, V, uniform_n0=n0)
    ch.update(attach_coeff=_attach_for(p_target, d), mu_e=mu_e, D_e=mu_e * 0.02526)
    return ch


def test_free_electron_initial_split(orc):
    """The negative charge of the pulse splits into electrons, p of it
    (eq. free_elec), and negative ions n+ (1 - e^{-a z}) (eq.
    ion_elec_distribution): for a uniform dose both sums have closed forms."""
    ch = _fe_chamber(0.3, 200.0)
    r = orc.solve(dict(ch, max_steps=1), W.no_tracks(), with_fields=False)
    a, d, nz = ch["attach_coeff"], ch["gap"], ch["nz"]
    p = cf.free_electron_fraction(a, d)
    assert orc.free_fraction(a, d) == pytest.approx(p, rel=1e-15)
    Q = r["released_neg_charge"]
    assert Q == pytest.approx(r["n_released"], rel=1e-15)
    assert r["e_released"] == pytest.approx(p * Q, rel=1e-13)
    dz = d / nz
    k = np.arange(1, nz)
    col = ch["uniform_n0"] * ch["dx"] * ch["dy"] * dz * ch["nx"] * ch["ny"]
    assert r["n_released_neg"] == pytest.approx(col * np.sum(-np.expm1(-a * k * dz)), rel=1e-13)


def test_free_electron_split_field_node_by_node(orc):
    """Before any step (max_steps = 0) the fields hold the split itself: a
    uniform dose gives positive ions n0 at every interior node and negative
    ions n0 (1 - e^{-a z}) with z the node's distance from the anode, the
    plane k = 0 that collects the negative carriers (eq.
    ion_elec_distribution), so they grow towards the cathode."""
    ch = _fe_chamber(0.3, 200.0)
    r = orc.solve(dict(ch, max_steps=0), W.no_tracks(), with_fields=True)
    assert r["steps"] == 0
    n0, a, nz = ch["uniform_n0"], ch["attach_coeff"], ch["nz"]
    z = np.arange(1, nz) * ch["gap"] / nz
    expect = n0 * -np.expm1(-a * z)
    assert np.allclose(r["neg"][1:nz], expect[:, None, None], rtol=1e-13, atol=0.0)
    assert np.all(r["pos"][1:nz] == n0)
    assert r["neg"][1, 0, 0] < r["neg"][nz - 1, 0, 0]


def test_free_electron_phase_conservation(orc):
    """Phase 1 keeps every carrier's books step by step: in flight before =
    collected + recombined + in flight after (positive ions recombine with
    both negative carriers)."""
    ch = _fe_chamber(0.5, 100.0)
    r = orc.solve(ch, W.no_tracks(), with_trace=True, with_fields=False)
    t = r["trace_e"]
    N = r["n_released"]
    prev = lambda col, first: np.concatenate([[first], t[:-1, col]])
    err_p = prev(8, r["n_released"]) - t[:, 2] - t[:, 3] - t[:, 0] - t[:, 1] - t[:, 8]
    err_n = prev(9, r["n_released_neg"]) - t[:, 4] - t[:, 5] - t[:, 0] - t[:, 9]
    err_e = prev(10, r["e_released"]) - t[:, 6] - t[:, 7] - t[:, 1] - t[:, 10]
    for e in (err_p, err_n, err_e):
        assert np.max(np.abs(e)) <= 1e-12 * N
    # the electrons leave within the phase; the ions have hardly moved
    assert r["e_left"] <= 1e-9 * N and r["e_steps"] > 10


@pytest.mark.parametrize("p", [0.1, 0.5])
def test_free_electron_boag_models(orc, p):
    """Boag's free-electron models (eqs. model1-3) against the solver for a
    uniform instantaneous dose: within 2.5 % at 100 V and 1 % at 300 V, all
    three converging as the field grows (the paper's comparison); at p = 0.1
    model 1 is the closest, as the paper found."""
    dev = {}
    for V in (100.0, 300.0):
        ch = _fe_chamber(p, V)
        r = orc.solve(ch, W.no_tracks(), with_fields=False)
        assert r["flags"] == 0
        u = cf.boag_u(ch["uniform_n0"], ch["gap"], V, ch["mu_pos"], ch["mu_neg"], ch["alpha"])
        pp = cf.free_electron_fraction(ch["attach_coeff"], ch["gap"])
        dev[V] = [abs(m(u, pp) / r["f"] - 1) for m in (cf.boag_model1, cf.boag_model2, cf.boag_model3)]
        assert max(dev[V]) < (0.025 if V == 100.0 else 0.01)
        # free electrons escape recombination: f above the ions-only result
        assert r["f"] > orc.solve(dict(ch, mu_e=0.0), W.no_tracks(), with_fields=False)["f"]
        # electron-ion recombination is tiny next to the ionic one
        assert r["e_recombined"] < 1e-2 * r["n_recombined"]
    assert all(b < a for a, b in zip(dev[100.0], dev[300.0]))
    if p == 0.1:
        assert dev[100.0][0] == min(dev[100.0])


def test_all_electrons_free_collects_almost_everything(orc):
    """p -> 1: no negative ions form, the electrons leave before they can
    recombine, and f -> 1 as every model gives."""
    ch = _fe_chamber(0.9999, 100.0)
    r = orc.solve(ch, W.no_tracks(), with_fields=False)
    assert r["f"] > 0.999


# ---------------------------------------------------------------------------
# absorbing lateral boundaries (the option to the periodic reading): the
# nodes just outside the cell hold zero and what they would receive is
# tallied as escaped
# ---------------------------------------------------------------------------

def _dense_step_absorbing(ch, dt, pos, neg):
    """One step as a dense matrix on the grid padded by one ghost node on
    every lateral side (ghosts start at zero and have no wrap), so the
    ghosts' new values are what left through the lateral boundaries."""
    nx, ny, nz = ch["nx"], ch["ny"], ch["nz"]
    dx, dy, dz = ch["dx"], ch["dy"], ch["gap"] / nz
    E = ch["voltage"] / ch["gap"]
    X, Y = nx + 2, ny + 2
    Ix, Iy, Iz = np.eye(X), np.eye(Y), np.eye(nz + 1)

    def open_second(m, h):
        return (np.eye(m, k=1) - 2 * np.eye(m) + np.eye(m, k=-1)) / h ** 2

    def pad(f):
        g = np.zeros((nz + 1, Y, X))
        g[:, 1:-1, 1:-1] = f
        return g

    Dxx = np.kron(np.kron(Iz, Iy), open_second(X, dx))
    Dyy = np.kron(np.kron(Iz, open_second(Y, dy)), Ix)
    up, down = np.eye(nz + 1, k=1), np.eye(nz + 1, k=-1)
    Dzz = np.kron(np.kron((up - 2 * Iz + down) / dz ** 2, Iy), Ix)
    backward = (Iz - down) / dz
    central = (up - down) / (2 * dz)
    P, N = pad(pos), pad(neg)
    out, esc, sc = [], [], []
    for s, (mu, D, sign) in enumerate([(ch["mu_pos"], ch["D_pos"], 1.0), (ch["mu_neg"], ch["D_neg"], -1.0)]):
        v = sign * mu * E
        c = v * dt / dz
        Dz = np.kron(np.kron(c * backward + (1 - c) * central, Iy), Ix)
        M = np.eye((nz + 1) * Y * X) + dt * (D * (Dxx + Dyy + Dzz) - v * Dz)
        n_new = (M @ (P, N)[s].ravel() - ch["alpha"] * dt * P.ravel() * N.ravel()).reshape(nz + 1, Y, X)
        if ch.get("space_charge", 0):
            # the local screening term of each species, -+ mu dt (q/eps0) n (n+ - n-),
            # zero on the ghosts, so it changes no escape
            sc_term = -sign * mu * dt * Q_OVER_EPS0 * (P, N)[s] * (P - N)
            n_new += sc_term
            sc.append(sc_term[1:nz, 1:-1, 1:-1].sum() * dx * dy * dz)
        ghost = n_new[1:nz].sum() - n_new[1:nz, 1:-1, 1:-1].sum()
        esc.append(ghost * dx * dy * dz)
        out.append(n_new[:, 1:-1, 1:-1].copy())
        out[-1][0] = 0.0
        out[-1][nz] = 0.0
    return out[0], out[1], esc, sc


@pytest.mark.parametrize("geom", [(4, 4, 5), (3, 5, 2), (1, 1, 7), (6, 2, 4)])
def test_absorbing_step_matches_dense_matrix_scheme(orc, geom):
    nx, ny, nz = geom
    ch = W.chamber(nx, ny, nz, 3e-4, nz * 2.5e-4, 40.0, dy=4e-4, D_pos=0.03, D_neg=0.05,
                   alpha=1.6e-6, lateral_bc=1)
    dt = orc.dt(ch)
    pos, neg = W.perturbed_field((nz + 1, ny, nx), seed=8, scale=3e11)
    p1, n1, tally = orc.step(ch, dt, pos, neg)
    p2, n2, esc, _ = _dense_step_absorbing(ch, dt, pos, neg)
    scale = max(np.abs(pos).max(), np.abs(neg).max())
    assert np.max(np.abs(p1 - p2)) <= 1e-14 * scale
    assert np.max(np.abs(n1 - n2)) <= 1e-14 * scale
    tot = (pos.sum() + neg.sum()) * ch["dx"] * ch["dy"] * ch["gap"] / nz
    assert esc[0] > 0 and esc[1] > 0
    assert tally["pos_escaped"] == pytest.approx(esc[0], abs=1e-13 * tot)
    assert tally["neg_escaped"] == pytest.approx(esc[1], abs=1e-13 * tot)


@pytest.mark.parametrize("geom", [(4, 4, 5), (3, 5, 2), (6, 2, 4)])
def test_absorbing_step_with_space_charge_matches_dense_matrix_scheme(orc, geom):
    """Both options at once: the absorbing transport of the dense ghost-node
    scheme plus the local screening term of each species; escape and
    space-charge tallies from the same sums."""
    nx, ny, nz = geom
    ch = W.chamber(nx, ny, nz, 3e-4, nz * 2.5e-4, 40.0, dy=4e-4, D_pos=0.03, D_neg=0.05,
                   alpha=1.6e-6, lateral_bc=1, space_charge=1)
    dt = orc.dt(ch)
    pos, neg = W.perturbed_field((nz + 1, ny, nx), seed=9, scale=3e11)
    p1, n1, tally = orc.step(ch, dt, pos, neg)
    p2, n2, esc, sc = _dense_step_absorbing(ch, dt, pos, neg)
    p0, n0, _, _ = _dense_step_absorbing(dict(ch, space_charge=0), dt, pos, neg)
    scale = max(np.abs(pos).max(), np.abs(neg).max())
    assert np.max(np.abs(p2 - p0)) > 1e-4 * scale  # the screening term matters here
    assert np.max(np.abs(p1 - p2)) <= 1e-14 * scale
    assert np.max(np.abs(n1 - n2)) <= 1e-14 * scale
    tot = (pos.sum() + neg.sum()) * ch["dx"] * ch["dy"] * ch["gap"] / nz
    assert tally["pos_escaped"] == pytest.approx(esc[0], abs=1e-13 * tot)
    assert tally["neg_escaped"] == pytest.approx(esc[1], abs=1e-13 * tot)
    assert tally["pos_space_charge"] == pytest.approx(sc[0], abs=1e-13 * tot)
    assert tally["neg_space_charge"] == pytest.approx(sc[1], abs=1e-13 * tot)


def test_absorbing_pure_diffusion_eigenmode(orc):
    """E = 0, alpha = 0: a product of sines vanishing on the ghost nodes and
    on the electrodes is an eigenvector of the explicit scheme, so after m
    steps the field is lambda^m times the initial one, and the escaped
    tally follows the boundary nodes of that closed form."""
    nx, ny, nz = 9, 6, 8
    dx, dy, dz = 3e-4, 4e-4, 2.5e-4
    D = 0.04
    ch = W.chamber(nx, ny, nz, dx, nz * dz, 0.0, dy=dy, alpha=0.0, D_pos=D, D_neg=D, lateral_bc=1)
    dt = orc.dt(ch)
    a, b, c = 2, 1, 3
    i = np.arange(nx)
    j = np.arange(ny)
    k = np.arange(nz + 1)
    f0 = 1e10 * (np.sin(np.pi * c * k / nz)[:, None, None] * np.sin(np.pi * b * (j + 1) / (ny + 1))[None, :, None]
                 * np.sin(np.pi * a * (i + 1) / (nx + 1))[None, None, :])
    f0[0] = 0.0
    f0[nz] = 0.0
    sx, sy, sz = D * dt / dx ** 2, D * dt / dy ** 2, D * dt / dz ** 2
    lam = (1 - 4 * sx * np.sin(np.pi * a / (2 * (nx + 1))) ** 2 - 4 * sy * np.sin(np.pi * b / (2 * (ny + 1))) ** 2
           - 4 * sz * np.sin(np.pi * c / (2 * nz)) ** 2)
    m = 7
    p, n, tr = orc.advance(ch, dt, f0, f0, m, with_trace=True)
    assert np.max(np.abs(p - lam ** m * f0)) <= 1e-12 * np.abs(f0).max()
    dV = dx * dy * dz
    edge = sx * (f0[:, :, 0].sum() + f0[:, :, -1].sum()) + sy * (f0[:, 0, :].sum() + f0[:, -1, :].sum())
    expect = np.array([lam ** l * edge * dV for l in range(m)])
    got = tr[:, 13]
    assert np.max(np.abs(got - expect)) <= 1e-12 * np.abs(f0).sum() * dV


def test_absorbing_equals_antisymmetric_periodic_extension(orc):
    """Without recombination the scheme is linear and symmetric in x and y,
    so the absorbing cell evolves as the odd extension of its field on a
    periodic cell of 2(nx+1) by 2(ny+1) nodes, whose nodes at the mirror
    lines stay zero."""
    nx, ny, nz = 7, 5, 9
    ch_a = W.chamber(nx, ny, nz, 3e-4, nz * 2.5e-4, 30.0, dy=4e-4, alpha=0.0, D_pos=0.03, D_neg=0.05,
                     lateral_bc=1)
    X, Y = 2 * (nx + 1), 2 * (ny + 1)
    ch_p = dict(ch_a, nx=X, ny=Y, lateral_bc=0)
    dt = orc.dt(ch_a)
    assert dt == orc.dt(ch_p)
    p0, n0 = W.perturbed_field((nz + 1, ny, nx), seed=12, scale=1e10)

    def odd(f):
        g = np.zeros((nz + 1, Y, X))
        g[:, 1:ny + 1, 1:nx + 1] = f
        g[:, 1:ny + 1, nx + 2:] = -f[:, :, ::-1]
        g[:, ny + 2:, :] = -g[:, 1:ny + 1, :][:, ::-1, :]
        return g

    steps = 11
    pa, na = orc.advance(ch_a, dt, p0, n0, steps)
    pp, nn = orc.advance(ch_p, dt, odd(p0), odd(n0), steps)
    scale = np.abs(p0).max()
    assert np.max(np.abs(pp[:, 1:ny + 1, 1:nx + 1] - pa)) <= 1e-13 * scale
    assert np.max(np.abs(nn[:, 1:ny + 1, 1:nx + 1] - na)) <= 1e-13 * scale
    assert np.max(np.abs(pp[:, 0, :])) <= 1e-13 * scale and np.max(np.abs(pp[:, :, nx + 1])) <= 1e-13 * scale


def test_absorbing_deposit_is_the_unwrapped_profile(orc):
    """A track inside the cell deposits, on an absorbing cell, what it
    deposits on the first nx x ny nodes of a periodic cell twice as wide in
    both directions: there no node of the original cell is closer to a
    periodic image of the axis than to the axis itself."""
    nx, ny, nz = 20, 16, 10
    ch_a = W.chamber(nx, ny, nz, 3e-4, nz * 3e-4, 20.0, lateral_bc=1)
    ch_p = dict(ch_a, nx=2 * nx, ny=2 * ny, lateral_bc=0)
    tr = W.tracks([[30.0, 1.5e-3, 0.4e-3, 4.4e-3, 0.5, 0.7, 0.0]])  # near the x = 0 edge
    dt = orc.dt(ch_a, tr)
    pa, na, rel_a = orc.deposit(ch_a, tr, 0, dt)
    pp, npp, rel_p = orc.deposit(ch_p, tr, 0, dt)
    assert np.array_equal(pa, pp[:, :ny, :nx]) and np.array_equal(na, npp[:, :ny, :nx])
    # and the periodic deposit on the original cell differs (it wraps)
    pw, _, rel_w = orc.deposit(dict(ch_a, lateral_bc=0), tr, 0, dt)
    assert rel_w > rel_a * (1 + 1e-3)


def test_absorbing_far_from_the_edges_equals_periodic(orc):
    """While the densities stay away from the lateral edges the two
    boundary options step identically and nothing escapes."""
    ch_a = W.chamber(40, 40, 12, 2e-4, 12 * 2.5e-4, 10.0, lateral_bc=1)
    ch_p = dict(ch_a, lateral_bc=0)
    dt = orc.dt(ch_a)
    f = _blob(ch_a, (20, 20, 6), 1.2)
    pa, na, ta = orc.advance(ch_a, dt, f, 0.7 * f, 6, with_trace=True)
    pp, npp, tp = orc.advance(ch_p, dt, f, 0.7 * f, 6, with_trace=True)
    assert np.max(np.abs(pa - pp)) <= 1e-15 * f.max()
    assert np.max(np.abs(ta[:, 13:15])) <= 1e-14 * f.sum() * 2e-4 * 2e-4 * 2.5e-4


def test_absorbing_conservation_and_escape(orc):
    """A track at the corner of an absorbing cell: every species balances
    with the escaped column, charge escapes, and f falls below the
    recombination-only efficiency f_R."""
    ch = W.chamber(24, 20, 16, 3e-4, 16 * 3e-4, 15.0, lateral_bc=1)
    tr = W.tracks([[20.0, 8e-4, 0.2e-3, 0.3e-3, 0.0, 0.0, 0.0],
                   [10.0, 6e-4, 3.6e-3, 3.0e-3, 0.4, 2.0, 0.0]])
    r = orc.solve(ch, tr, with_trace=True, with_fields=False)
    assert r["flags"] == 0
    _check_conservation(r)
    assert r["n_escaped_pos"] > 1e-3 * r["n_released"] and r["n_escaped_neg"] > 1e-3 * r["n_released"]
    assert r["n_escaped_pos"] == pytest.approx(r["trace"][:, 13].sum(), rel=1e-12)
    col = r["col_pos_anode"] + r["col_pos_cathode"] + r["col_neg_anode"] + r["col_neg_cathode"]
    assert col + r["n_escaped_pos"] + r["n_escaped_neg"] + 2 * r["n_recombined"] == \
        pytest.approx(2 * r["n_released"], rel=1e-10)
    assert r["f"] < r["f_R"] - 1e-3


def test_absorbing_rejects_free_electrons(orc):
    ch = dict(W.chamber(8, 8, 6, 3e-4, 6 * 3e-4, 15.0, lateral_bc=1, uniform_n0=1e9), mu_e=1000.0, D_e=25.0)
    with pytest.raises(ValueError):
        orc.solve(ch, W.no_tracks())
