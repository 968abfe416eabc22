"""Batched sweeps on the GPU against the CPU oracle, instance by instance."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_06749_amd as it
    it.lib()
    return it


def small_sweep(n=7, seed=5):
    """Uneven small chambers: transverse 20..90 nodes (ragged tiles), 6..40
    gap intervals, voltages 10..80 V, doses and 1..12 tracks of modest LET,
    one with no tracks and one with no pre-ionisation."""
    rng = np.random.default_rng(seed)
    chs, trs = [], []
    for q in range(n):
        nx = int(rng.integers(20, 91))
        ny = int(rng.integers(12, 70))
        nz = int(rng.integers(6, 41))
        ch = W.chamber(nx, ny, nz, 3e-4, nz * 3e-4, float(rng.uniform(10, 80)),
                       uniform_n0=0.0 if q == 1 else float(rng.uniform(1e8, 5e9)))
        k = 0 if q == 2 else int(rng.integers(1, 13))
        lx, ly = nx * 3e-4, ny * 3e-4
        tr = np.stack([rng.uniform(1, 20, k), rng.uniform(6e-4, 1.5e-3, k), rng.uniform(0, lx, k),
                       rng.uniform(0, ly, k), np.zeros(k), np.zeros(k), np.zeros(k)], axis=1)
        chs.append(ch)
        trs.append(W.tracks(tr))
    return chs, trs


@pytest.mark.parametrize("shape", [dict(tile_y=8), dict(tile_y=16), dict(tile_x=32)], ids=["64x8", "64x16", "32x16"])
def test_batch_matches_oracle_per_instance(gpu, orc, shape):
    chs, trs = small_sweep()
    res = gpu.it_solve_batch(chs, trs, exec=dict(shape, check_every=6))
    for ch, tr, g in zip(chs, trs, res):
        o = orc.solve(ch, tr, with_fields=False)
        assert g["steps"] == o["steps"] and g["flags"] == o["flags"]
        assert g["f"] == pytest.approx(o["f"], rel=1e-9)
        N = max(o["n_released"], 1.0)
        for k in ("n_released", "n_recombined", "col_pos_anode", "col_pos_cathode", "col_neg_anode",
                  "col_neg_cathode"):
            assert abs(g[k] - o[k]) <= 1e-9 * N, k


def test_batch_with_space_charge_on_some_instances(gpu, orc):
    """Instances with and without the screening term in one batch (the
    batch then runs the kernel instance with the term, at zero coefficients
    for the others)."""
    chs, trs = small_sweep(n=4, seed=12)
    for q in (0, 1, 3):
        chs[q]["space_charge"] = 1
    res = gpu.it_solve_batch(chs, trs, exec=dict(check_every=4))
    for ch, tr, g in zip(chs, trs, res):
        o = orc.solve(ch, tr, with_fields=False)
        assert g["steps"] == o["steps"] and g["flags"] == o["flags"]
        assert g["f"] == pytest.approx(o["f"], rel=1e-9)
        N = max(o["n_released"], 1.0)
        for k in ("n_recombined", "n_space_charge_pos", "n_space_charge_neg"):
            assert abs(g[k] - o[k]) <= 1e-9 * N, k
        assert (o["n_space_charge_pos"] != 0.0) == bool(ch["space_charge"])


def test_batch_with_separate_radii(gpu, orc):
    chs, trs = small_sweep(n=3, seed=14)
    t = trs[0]
    trs[0] = np.concatenate([t, 1.4 * t[:, 1:2]], axis=1)  # b- = 1.4 b
    res = gpu.it_solve_batch(chs, trs)
    for ch, tr, g in zip(chs, trs, res):
        o = orc.solve(ch, tr, with_fields=False)
        assert g["steps"] == o["steps"] and g["flags"] == o["flags"]
        assert g["f"] == pytest.approx(o["f"], rel=1e-9)
        assert g["n_released_neg"] == pytest.approx(o["n_released_neg"], rel=1e-9)


def test_batch_equals_single_runs(gpu):
    chs, trs = small_sweep(n=4, seed=9)
    res = gpu.it_solve_batch(chs, trs)
    for ch, tr, g in zip(chs, trs, res):
        s = gpu.it_solve(ch, tr, exec=dict(kernel=1))
        assert g["steps"] == s["steps"]
        assert g["f"] == pytest.approx(s["f"], rel=1e-12)


def test_batch_step_limit(gpu, orc):
    chs, trs = small_sweep(n=3, seed=2)
    for ch in chs:
        ch["max_steps"] = 25
    res = gpu.it_solve_batch(chs, trs, exec=dict(check_every=8))
    for ch, tr, g in zip(chs, trs, res):
        o = orc.solve(ch, tr, with_fields=False)
        assert g["steps"] == o["steps"] == 25 and g["flags"] == o["flags"]
        assert g["f"] == pytest.approx(o["f"], rel=1e-9)


def test_batch_rejects_later_tracks(gpu):
    chs, trs = small_sweep(n=2, seed=3)
    trs[1] = trs[1].copy()
    trs[1][0, 6] = 1e-3
    with pytest.raises(gpu.ItError) as e:
        gpu.it_solve_batch(chs, trs)
    assert e.value.code == gpu.IT_ENOTSUP


@pytest.mark.parametrize("ex", [dict(check_every=4), dict(kernel=1, check_every=4),
                                dict(kernel=2, steps_per_pass=2, check_every=4)],
                         ids=["default", "plain", "blocked2"])
def test_batch_with_absorbing_boundaries_on_some_instances(gpu, orc, ex):
    """Absorbing and periodic lateral boundaries in one batch (one-step and
    blocked passes); tracks placed near the edges so that charge escapes."""
    chs, trs = small_sweep(n=5, seed=21)
    for q in (0, 2, 3):
        chs[q]["lateral_bc"] = 1
        trs[q][:, 2] = np.minimum(trs[q][:, 2], 6e-4)  # next to the x = 0 edge
    res = gpu.it_solve_batch(chs, trs, exec=ex)
    for ch, tr, g in zip(chs, trs, res):
        o = orc.solve(ch, tr, with_fields=False)
        assert g["steps"] == o["steps"] and g["flags"] == o["flags"]
        assert g["f"] == pytest.approx(o["f"], rel=1e-9)
        N = max(o["n_released"], 1.0)
        for k in ("n_recombined", "col_pos_anode", "col_neg_cathode", "n_escaped_pos", "n_escaped_neg"):
            assert abs(g[k] - o[k]) <= 1e-9 * N, k
        assert (o["n_escaped_pos"] > 0.0) == bool(ch["lateral_bc"])  # every instance releases charge


@pytest.mark.parametrize("T", [2, 3])
def test_batch_blocked_rebuilds_match_oracle(gpu, orc, T):
    """Blocked passes with two passes per graph: the table is rebuilt as
    soon as a quarter of the instances stop, so the pass before each rebuild
    is recorded by the first pass after it, with the tile count the run
    state carries; every instance still matches the oracle.  (These small
    chambers never fill the machine, so the chunks are short from the start;
    the 96-chamber sweep against its stored results covers chunks that
    change at rebuilds.)"""
    chs, trs = small_sweep(n=9, seed=33)
    res = gpu.it_solve_batch(chs, trs, exec=dict(kernel=2, steps_per_pass=T, check_every=2, z_chunk=40))
    for ch, tr, g in zip(chs, trs, res):
        o = orc.solve(ch, tr, with_fields=False)
        assert g["steps"] == o["steps"] and g["flags"] == o["flags"]
        assert g["f"] == pytest.approx(o["f"], rel=1e-9)
        N = max(o["n_released"], 1.0)
        for k in ("n_released", "n_recombined", "col_pos_anode", "col_pos_cathode", "col_neg_anode",
                  "col_neg_cathode", "n_inflight_pos", "n_inflight_neg"):
            assert abs(g[k] - o[k]) <= 1e-9 * N, k
    assert len({r["steps"] for r in res}) > 3  # the instances stop at different steps
