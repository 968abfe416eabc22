"""Pins of the oracle's electron phase (sections "The free-electron
component" and "Implementation of the free-electron models"): the
three-carrier step against an independent dense-matrix formulation, and the
electron time step against eq. vNeum's closed forms and its stability edge.
CPU only.
"""
import math

import numpy as np
import pytest

import workloads as W


def _carrier_matrix(ch, dt, v, D):
    """I + dt [D (Dxx + Dyy + Dzz) - v Dz] on the full node grid (electrode
    planes included, periodic x and y), with the Appendix's blended drift
    derivative Dz = c backward + (1 - c) central, c = v dt/dz."""
    nx, ny, nz = ch["nx"], ch["ny"], ch["nz"]
    dx, dy, dz = ch["dx"], ch["dy"], ch["gap"] / nz
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz + 1)

    def periodic_second(m, h):
        M = -2 * np.eye(m)
        for a in range(m):
            M[a, (a + 1) % m] += 1
            M[a, (a - 1) % m] += 1
        return M / h ** 2

    up, down = np.eye(nz + 1, k=1), np.eye(nz + 1, k=-1)
    lap = (np.kron(np.kron(Iz, Iy), periodic_second(nx, dx)) +
           np.kron(np.kron(Iz, periodic_second(ny, dy)), Ix) +
           np.kron(np.kron((up - 2 * Iz + down) / dz ** 2, Iy), Ix))
    c = v * dt / dz
    Dz1 = c * (Iz - down) / dz + (1 - c) * (up - down) / (2 * dz)
    Dz = np.kron(np.kron(Dz1, Iy), Ix)
    return np.eye((nz + 1) * ny * nx) + dt * (D * lap - v * Dz)


def _fe(nx, ny, nz, V=60.0, mu_e=900.0, D_e=20.0, alpha=1.6e-6):
    ch = W.chamber(nx, ny, nz, 3e-4, nz * 2.5e-4, V, dy=4e-4, D_pos=0.03, D_neg=0.05, alpha=alpha)
    ch.update(mu_e=mu_e, D_e=D_e, attach_coeff=3.0)
    return ch


@pytest.mark.parametrize("geom", [(4, 4, 5), (3, 5, 2), (1, 1, 7)])
def test_electron_step_matches_dense_matrix_scheme(orc, geom):
    """n' = M_s n - sink_s per carrier, with M_s assembled from the
    Appendix's difference operators for the carrier's own signed velocity
    (+mu+ E, -mu- E, -mu_e E) and diffusion constant; the sinks are
    beta n+ (n- + n_e), beta n+ n-, beta n+ n_e; what lands on the electrode
    planes is the carrier's collected amount."""
    nx, ny, nz = geom
    ch = _fe(nx, ny, nz)
    dt = min(orc.dt(ch), orc.electron_dt(ch))
    pos, neg = W.perturbed_field((nz + 1, ny, nx), seed=17, scale=3e11)
    ele, _ = W.perturbed_field((nz + 1, ny, nx), seed=18, scale=2e11)
    p1, n1, e1, tally = orc.step3(ch, dt, pos, neg, ele)
    E = ch["voltage"] / ch["gap"]
    beta = ch["alpha"] * dt
    sink_n = beta * pos.ravel() * neg.ravel()
    sink_e = beta * pos.ravel() * ele.ravel()
    carriers = [(pos, ch["mu_pos"] * E, ch["D_pos"], sink_n + sink_e),
                (neg, -ch["mu_neg"] * E, ch["D_neg"], sink_n),
                (ele, -ch["mu_e"] * E, ch["D_e"], sink_e)]
    dV = ch["dx"] * ch["dy"] * ch["gap"] / nz
    scale = max(np.abs(a).max() for a in (pos, neg, ele))
    tot = (pos.sum() + neg.sum() + ele.sum()) * dV
    names = ("pos", "neg", "e")
    for (n_old, v, D, sink), got, name in zip(carriers, (p1, n1, e1), names):
        new = (_carrier_matrix(ch, dt, v, D) @ n_old.ravel() - sink).reshape(nz + 1, ny, nx)
        anode, cathode = new[0].sum() * dV, new[nz].sum() * dV
        new[0] = 0.0
        new[nz] = 0.0
        assert np.max(np.abs(got - new)) <= 1e-14 * scale
        assert tally[f"{name}_anode"] == pytest.approx(anode, abs=1e-13 * tot)
        assert tally[f"{name}_cathode"] == pytest.approx(cathode, abs=1e-13 * tot)
        assert tally[f"{name}_inflight"] == pytest.approx(new.sum() * dV, rel=1e-13, abs=1e-13 * tot)
        assert tally[f"{name}_abs"] == pytest.approx(np.abs(new).sum() * dV, rel=1e-13)
    interior = (slice(1, nz), slice(None), slice(None))
    assert tally["recombined_pn"] == pytest.approx(beta * np.sum(pos[interior] * neg[interior]) * dV, rel=1e-13)
    assert tally["recombined_pe"] == pytest.approx(beta * np.sum(pos[interior] * ele[interior]) * dV, rel=1e-13)


def test_electron_dt_pure_drift_is_one_cell_per_step(orc):
    """D_e = 0: eq. vNeum reduces to (mu_e E dt/dz)^2 <= 1, so the largest
    step moves the electrons exactly one gap interval (Courant number 1)."""
    ch = _fe(6, 6, 40, V=80.0, mu_e=1200.0, D_e=0.0)
    dz = ch["gap"] / ch["nz"]
    E = ch["voltage"] / ch["gap"]
    assert orc.electron_dt(ch) == pytest.approx(dz / (ch["mu_e"] * E), rel=1e-15)


def test_electron_dt_pure_diffusion_closed_form(orc):
    """E = 0: eq. vNeum reduces to 2 D_e dt (1/dx^2 + 1/dy^2 + 1/dz^2) <= 1."""
    ch = _fe(6, 6, 40, V=0.0, mu_e=1200.0, D_e=25.0)
    dz = ch["gap"] / ch["nz"]
    h = 1 / ch["dx"] ** 2 + 1 / ch["dy"] ** 2 + 1 / dz ** 2
    assert orc.electron_dt(ch) == pytest.approx(1.0 / (2 * ch["D_e"] * h), rel=1e-15)


@pytest.mark.parametrize("mu_e,D_e", [(1500.0, 37.9), (300.0, 400.0), (5000.0, 1.0)])
def test_electron_dt_is_the_tight_von_neumann_bound(orc, mu_e, D_e):
    """General case: at the returned step the electrons' eq. vNeum holds with
    equality (2 s_sum + c^2 = 1, with s and c formed here from the chamber),
    and it is the smaller of the two regimes' limits' combination: below
    both the pure-drift and the pure-diffusion limits."""
    ch = _fe(6, 6, 40, V=120.0, mu_e=mu_e, D_e=D_e)
    dt = orc.electron_dt(ch)
    dz = ch["gap"] / ch["nz"]
    E = ch["voltage"] / ch["gap"]
    s = D_e * dt * (1 / ch["dx"] ** 2 + 1 / ch["dy"] ** 2 + 1 / dz ** 2)
    c = mu_e * E * dt / dz
    assert 2 * s + c * c == pytest.approx(1.0, abs=1e-14)
    assert dt < dz / (mu_e * E)
    assert dt < 1.0 / (2 * D_e * (1 / ch["dx"] ** 2 + 1 / ch["dy"] ** 2 + 1 / dz ** 2))


def test_electron_phase_step_capped_by_the_ion_step(orc):
    """The electron phase runs at min(kappa * electron step, ion step): fast
    electrons set it, electrons slower than the ions leave the ion step."""
    n0 = 3e9
    fast = _fe(4, 4, 40, V=100.0, mu_e=1500.0, D_e=37.9, alpha=1.6e-6)
    fast.update(uniform_n0=n0, dt_safety=0.8, max_steps=3)
    r = orc.solve(fast, W.no_tracks(), with_fields=False)
    assert r["e_dt"] == pytest.approx(0.8 * orc.electron_dt(fast), rel=1e-15)
    assert r["e_dt"] < r["dt"]
    slow = dict(fast, mu_e=0.5, D_e=0.01)
    r = orc.solve(slow, W.no_tracks(), with_fields=False)
    assert 0.8 * orc.electron_dt(slow) > r["dt"]
    assert r["e_dt"] == r["dt"]


def _checkerboard(ch, amp=1.0):
    k, j, i = np.indices((ch["nz"] + 1, ch["ny"], ch["nx"]))
    f = amp * (1.0 + 0.5 * (-1.0) ** (i + j + k))
    f[0] = 0.0
    f[-1] = 0.0
    return np.ascontiguousarray(f)


@pytest.mark.parametrize("mu_e,D_e,nz", [(0.0, 30.0, 40),      # diffusion-limited
                                         (1200.0, 0.05, 600)])  # drift-limited, long gap
def test_electron_step_stable_at_kappa_one_unstable_beyond(orc, mu_e, D_e, nz):
    """The electron step is the edge of stability of the three-carrier
    scheme: the most oscillatory electron mode does not grow at the bound
    and blows up with a 5 % larger step (von Neumann)."""
    ch = _fe(8 if nz == 40 else 4, 8 if nz == 40 else 4, nz, V=30.0 if mu_e else 0.0, mu_e=mu_e, D_e=D_e,
             alpha=0.0)
    ch["gap"] = nz * 2e-4
    zero = np.zeros((nz + 1, ch["ny"], ch["nx"]))
    dt = orc.electron_dt(ch)
    for factor, bounded in ((1.0, True), (1.05, False)):
        e = _checkerboard(ch)
        for _ in range(250):
            _, _, e, _ = orc.step3(ch, dt * factor, zero, zero, e)
        peak = np.max(np.abs(e))
        assert (peak <= 2.0) if bounded else (peak > 1e3), (factor, peak)
