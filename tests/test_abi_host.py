"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function the header declares, and its host-only entry points agree
with the oracle's time step and reject bad input."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(it_\w+)\s*\(", src, flags=re.M))
    return names


@pytest.fixture(scope="module")
def lib():
    import paper_1610_06749_amd as it
    return it


def test_header_declares_the_abi():
    names = _declared()
    assert {"it_dt", "it_validate", "it_workspace_size", "it_solve", "it_advance", "it_strerror"} <= names


def test_library_exports_every_declared_symbol(lib):
    L = ctypes.CDLL(lib.binding.LIB_PATH)
    for name in sorted(_declared()):
        assert hasattr(L, name), name


def test_host_dt_matches_oracle(lib, orc):
    for ch in (W.single_track()[0], W.pulsed_beam()[0], W.continuous_beam()[0],
               W.chamber(5, 7, 9, 3e-4, 0.01, 0.0), W.chamber(5, 7, 9, 3e-4, 0.01, 80.0, D_pos=0.0, D_neg=0.0)):
        assert lib.it_dt(ch) == pytest.approx(orc.dt(ch), rel=1e-15)
    for ch, tr in (W.single_track(), W.pulsed_beam(), W.continuous_beam(duration_s=2e-3),
                   W.single_track(space_charge=1), W.pulsed_beam(space_charge=1)):
        assert lib.it_dt(ch, tr) == pytest.approx(orc.dt(ch, tr), rel=1e-14)


def test_validate_rejects_bad_input(lib):
    ch, tr = W.single_track()
    lib.it_validate(ch, tr)
    for key, val in (("nz", 1), ("nx", 0), ("dx", -1.0), ("dt_safety", 1.5), ("alpha", -1.0),
                     ("max_steps", 0), ("W_eV", 0.0), ("D_pos", float("nan"))):
        with pytest.raises(lib.ItError) as e:
            lib.it_validate(dict(ch, **{key: val}), tr)
        assert e.value.code == lib.IT_EINVAL
    for col, val in ((1, 0.0), (0, -1.0), (6, -1e-9), (2, float("inf"))):
        bad = tr.copy()
        bad[0, col] = val
        with pytest.raises(lib.ItError):
            lib.it_validate(ch, bad)
    with pytest.raises(lib.ItError) as e:
        lib.it_validate(W.chamber(4, 4, 8, 1e-3, 0.08, 0.0, D_pos=0.0, D_neg=0.0, reaction_limit=0.0), tr)
    assert e.value.code == lib.IT_ENODT


def test_workspace_size_covers_fields_and_trace(lib):
    ch, _ = W.pulsed_beam()
    n = lib.it_workspace_size(ch, 400)
    field = (ch["nz"] + 1) * ch["ny"] * ch["nx"] * 8
    assert n >= 4 * field + ch["max_steps"] * 10 * 8
    assert lib.it_workspace_size(dict(ch, max_steps=10), 400) < n


def test_separate_radius_checks_and_dt(lib, orc):
    ch, tr = W.single_track()
    t8 = np.concatenate([tr, 0.5 * tr[:, 1:2]], axis=1)  # a narrower negative column: higher peak
    assert lib.it_dt(ch, t8) == pytest.approx(orc.dt(ch, t8), rel=1e-14)
    assert lib.it_dt(ch, t8) < lib.it_dt(ch, tr)
    bad = t8.copy()
    bad[0, 7] = -1e-3
    with pytest.raises(lib.ItError) as e:
        lib.it_validate(ch, bad)
    assert e.value.code == lib.IT_EINVAL


def test_space_charge_flag_values(lib):
    ch, tr = W.single_track(space_charge=1)
    lib.it_validate(ch, tr)
    with pytest.raises(lib.ItError) as e:
        lib.it_validate(dict(ch, space_charge=2), tr)
    assert e.value.code == lib.IT_EINVAL


def test_launch_shape_checks(lib):
    chs, trs = W.batched_sweep(ninst=3)
    base = lib.it_workspace_size_batch(chs, trs, dict(kernel=1))  # one-step passes, 16-plane chunks
    assert lib.it_workspace_size_batch(chs, trs, dict(kernel=1, z_chunk=4)) > base  # more tiles, more partials
    for z in (1, 3, 513, -2):
        with pytest.raises(lib.ItError) as e:
            lib.it_workspace_size_batch(chs, trs, dict(z_chunk=z))
        assert e.value.code == lib.IT_EINVAL
    # tile shapes: 64 or 32 columns; 32-column tiles have 16 rows
    assert lib.it_workspace_size_batch(chs, trs, dict(tile_x=32)) > 0
    for bad in (dict(tile_x=48), dict(tile_x=16), dict(tile_x=32, tile_y=8)):
        with pytest.raises(lib.ItError) as e:
            lib.it_workspace_size_batch(chs, trs, bad)
        assert e.value.code == lib.IT_EINVAL
    # tiles of column pairs are for single chambers
    with pytest.raises(lib.ItError) as e:
        lib.it_workspace_size_batch(chs, trs, dict(tile_x=128))
    assert e.value.code == lib.IT_ENOTSUP
    # in-plane offsets are 32-bit byte offsets: planes above 2^28 nodes are refused
    with pytest.raises(lib.ItError) as e:
        lib.it_validate(W.chamber(1 << 15, 1 << 14, 2, 1e-4, 2e-4, 10.0), np.zeros((0, 7)))
    assert e.value.code == lib.IT_EINVAL


def _solve_status(lib, ch, tr, ex):
    """it_solve's status for a call that must be refused before any device
    work (no workspace, no stream)."""
    B = lib.binding
    c = B._chamber(ch)
    rows, ptr = B._tracks(tr)
    res = B.it_result()
    return B.lib().it_solve(ctypes.byref(c), ptr, rows.shape[0], B._exec(ex, host=False), None, 0, None, None, None, None,
                            ctypes.byref(res))


def test_lateral_boundary_option_checks(lib, orc):
    ch, tr = W.single_track()
    lib.it_validate(dict(ch, lateral_bc=1), tr)
    for bad in (2, -1):
        with pytest.raises(lib.ItError) as e:
            lib.it_validate(dict(ch, lateral_bc=bad), tr)
        assert e.value.code == lib.IT_EINVAL
    ab = dict(ch, lateral_bc=1)
    # absorbing boundaries: the one-step and the blocked kernel, no free electrons
    assert _solve_status(lib, ab, tr, dict(kernel=2, steps_per_pass=4)) == lib.IT_EWORKSPACE
    assert _solve_status(lib, dict(ab, mu_e=1000.0, D_e=25.0), tr, None) == lib.IT_ENOTSUP
    assert _solve_status(lib, ab, tr, dict(kernel=1)) == lib.IT_EWORKSPACE  # accepted up to the workspace
    assert _solve_status(lib, ch, tr, dict(kernel=2, steps_per_pass=4)) == lib.IT_EWORKSPACE
    # the blocked kernel: 2..4 steps per pass, extended tiles of 24..48 rows
    for T, ty in ((2, 24), (3, 32), (4, 40), (2, 48)):
        assert _solve_status(lib, ch, tr, dict(kernel=2, steps_per_pass=T, tile_y=ty)) == lib.IT_EWORKSPACE
    assert _solve_status(lib, ch, tr, dict(kernel=2, steps_per_pass=5)) == lib.IT_ENOTSUP
    for ty in (8, 16, 20, 56):
        assert _solve_status(lib, ch, tr, dict(kernel=2, steps_per_pass=3, tile_y=ty)) == lib.IT_EINVAL
    # 32-column tiles belong to the one-step kernels
    assert _solve_status(lib, ch, tr, dict(kernel=1, tile_x=32)) == lib.IT_EWORKSPACE
    assert _solve_status(lib, ch, tr, dict(kernel=2, steps_per_pass=4, tile_x=32)) == lib.IT_EINVAL
    # so do tiles of column pairs, which need an even nx
    assert ch["nx"] % 2 == 0
    for ty in (0, 8, 16):
        assert _solve_status(lib, ch, tr, dict(kernel=1, tile_x=128, tile_y=ty)) == lib.IT_EWORKSPACE
    assert _solve_status(lib, ch, tr, dict(kernel=2, steps_per_pass=4, tile_x=128)) == lib.IT_EINVAL
    assert _solve_status(lib, dict(ch, nx=ch["nx"] - 1), tr, dict(kernel=1, tile_x=128)) == lib.IT_EINVAL
    # the recombination bound sums the tracks' profiles without periodic
    # images: two dense tracks at opposite x edges overlap only through the wrap
    ch2 = W.chamber(40, 40, 10, 2e-4, 10 * 2e-4, 20.0)
    tr2 = W.tracks([[200.0, 6e-4, 1e-4, 4e-3, 0.0, 0.0, 0.0], [200.0, 6e-4, 40 * 2e-4 - 1e-4, 4e-3, 0.0, 0.0, 0.0]])
    for bc in (0, 1):
        c = dict(ch2, lateral_bc=bc)
        assert lib.it_dt(c, tr2) == pytest.approx(orc.dt(c, tr2), rel=1e-14)
    assert lib.it_dt(dict(ch2, lateral_bc=1), tr2) > lib.it_dt(ch2, tr2) * 1.01


def test_host_buffer_size(lib):
    """The caller's read-back buffer: slots for a single run, two per
    chamber of a batch; refused for no chambers."""
    one = lib.binding.it_host_buffer_size(1)
    assert one > 0 and one % 8 == 0
    assert lib.binding.it_host_buffer_size(96) == 2 * 96 * one // 4
    assert lib.binding.it_host_buffer_size(2) == one  # at least the single-run slots
    with pytest.raises(lib.ItError) as e:
        lib.binding.it_host_buffer_size(0)
    assert e.value.code == lib.IT_EINVAL


def test_strerror_names_codes(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.it_strerror(code) and lib.it_strerror(code) != "unknown status code"
    assert lib.it_strerror(-99) == "unknown status code"


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1610_06749_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", src, flags=re.M), fn
                assert "liboracle" not in src and "oracle.c" not in src, fn


def test_struct_layouts_match_the_header(lib, tmp_path):
    """The binding's ctypes structures have the C header's field offsets and
    sizes (a C program built against the header prints them)."""
    import subprocess
    B = lib.binding
    structs = {"it_chamber": B.it_chamber, "it_result": B.it_result, "it_exec": B.it_exec}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "iontracks.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for name, cls in structs.items():
        assert got[(name, "sizeof")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)


def test_pulse_train_checks_and_step(lib, orc):
    """n_pulses >= 2 needs a finite positive period; it_dt then gives the
    shortened step P / ceil(P / dt1), the oracle's."""
    ch, tr = W.single_track()
    dt1 = lib.it_dt(ch, tr)
    for P in (7.3 * dt1, dt1, 0.4 * dt1):
        c = dict(ch, n_pulses=3, pulse_period_s=P)
        assert lib.it_dt(c, tr) == P / math.ceil(P / dt1)
        o = orc.solve(dict(c, max_steps=1), tr, with_fields=False)
        assert lib.it_dt(c, tr) == o["dt"]
    assert lib.it_dt(dict(ch, n_pulses=1, pulse_period_s=-1.0), tr) == dt1  # a single pulse ignores the period
    for bad in (dict(n_pulses=-1), dict(n_pulses=3, pulse_period_s=0.0), dict(n_pulses=3, pulse_period_s=-1e-6),
                dict(n_pulses=3, pulse_period_s=float("nan")), dict(n_pulses=2, pulse_period_s=1e30),
                dict(n_pulses=(1 << 20) + 1, pulse_period_s=1e-6)):
        with pytest.raises(lib.ItError) as e:
            lib.it_validate(dict(ch, **bad), tr)
        assert e.value.code == lib.IT_EINVAL, bad
