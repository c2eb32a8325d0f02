"""The C boundary on the CPU: the library loads, exports every symbol that
include/rod.h declares, and rejects invalid descriptors before touching the
device (host-side validation only: no kernel runs here)."""
import os
import re

import numpy as np
import pytest

from paper_2605_13766_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(rod_\w+)\s*\(", txt, flags=re.M))
    return names


def test_header_declares_the_boundary():
    names = declared_symbols()
    for f in ("rod_batch_create", "rod_step", "rod_energy", "rod_get_state", "rod_set_state",
              "rod_get_flags", "rod_batch_destroy", "rod_last_error", "rod_batch_info"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2605_13766_amd import rod
    L = rod.lib()
    for name in sorted(declared_symbols()):
        assert hasattr(L, name), name


def _create(inp, **kw):
    from paper_2605_13766_amd import rod
    return rod.RodBatch(inp, **kw)


def _expect(code, inp, **kw):
    from paper_2605_13766_amd import rod
    with pytest.raises(rod.RodError) as ei:
        _create(inp, **kw)
    assert ei.value.code == code, str(ei.value)
    return str(ei.value)


def test_invalid_descriptors_rejected():
    from paper_2605_13766_amd import rod
    base = W.ragged_batch(n_rods=3, n_min=16, n_max=20, seed=41)
    bad = base.copy(); bad.n_elems = bad.n_elems.copy(); bad.n_elems[0] = 0
    bad.position = bad.position[:-1]
    _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.dt = 0.0
    assert "dt" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.youngs[1] = -1.0
    _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.damping[0] = -0.1
    _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.director[5, 0, 0] += 1e-6
    assert "SO(3)" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.director[2] = -bad.director[2]          # det = -1
    assert "SO(3)" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.position[3] = bad.position[2]            # zero-length element
    assert "zero length" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.rest_length = np.full(base.n_elements, 0.01); bad.rest_length[4] = 0.0
    _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.couple_amp = np.ones((3, 3))              # no frequency / phase
    _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.bc_start = np.array([0, 2, 0], np.int32)
    _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.velocity[0, 0] = np.nan
    _expect(rod.ROD_EINVAL, bad)
    _expect(rod.ROD_EINVAL, base, tile_waves=3)
    _expect(rod.ROD_EINVAL, base, substeps=-1)
    assert "autotune" in _expect(rod.ROD_EINVAL, base, autotune=2)
    long_rod = W.ragged_batch(n_rods=1, n_min=600, n_max=600, seed=43)
    assert "outside" in _expect(rod.ROD_EINVAL, long_rod)


def test_tile_too_small_unsupported():
    from paper_2605_13766_amd import rod
    inp = W.ragged_batch(n_rods=2, n_min=100, n_max=120, seed=45)
    _expect(rod.ROD_EUNSUPPORTED, inp, tile_waves=1)


def test_null_handle_calls():
    from paper_2605_13766_amd import rod
    L = rod.lib()
    assert L.rod_step(None, 10, None) == rod.ROD_EINVAL
    assert L.rod_batch_info(None, None) == rod.ROD_EINVAL
    assert L.rod_contact_stats(None, None, None) == rod.ROD_EINVAL
    L.rod_batch_destroy(None)


def test_descriptor_layouts_match_the_headers(tmp_path):
    """Every struct of the boundary has the same size and member offsets in the
    C headers (compiled here with gcc) as in the Python binding's ctypes."""
    import ctypes
    import subprocess
    from paper_2605_13766_amd import rod
    pairs = [("rod_batch_desc", rod.RodBatchDesc), ("rod_tune_trial", rod.TuneTrial),
             ("rod_surrogate_desc", rod.SurrogateDesc), ("rod_train_desc", rod.TrainDesc),
             ("rod_judge_desc", rod.JudgeDesc), ("rod_surrogate_stats", rod.SurrogateStats)]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "rod_surrogate.h"', "int main(void) {"]
    want = []
    for cname, py in pairs:
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(py))
        for f in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f[0]}));')
            want.append(getattr(py, f[0]).offset)
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == want


def test_magnetic_descriptor_rejected_when_not_finite():
    from paper_2605_13766_amd import rod
    base = W.magnetic_carpet(grid=2, n=8)
    bad = base.copy(); bad.field = base.field.copy(); bad.field[4] = np.inf
    assert "field" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.field_freq = np.nan
    assert "field_freq" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.magnetization = base.magnetization.copy(); bad.magnetization[3, 1] = np.nan
    assert "magnetization" in _expect(rod.ROD_EINVAL, bad)


def test_muscle_descriptor_rejected_when_incomplete_or_not_finite():
    from paper_2605_13766_amd import rod
    base = W.active_filaments(n_rods=3, n=8)
    bad = base.copy(); bad.muscle_phase = None
    assert "muscle_amp needs" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.muscle_amp = base.muscle_amp.copy(); bad.muscle_amp[2] = np.nan
    assert "muscle" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.gravity = np.array([0.0, np.inf, 0.0])
    assert "gravity" in _expect(rod.ROD_EINVAL, bad)


def test_connection_descriptor_rejected_when_invalid():
    from paper_2605_13766_amd import rod
    base = W.millipede_swarm(n_bots=1)
    bad = base.copy(); bad.conn_rod = base.conn_rod.copy(); bad.conn_rod[3, 1] = base.n_rods
    assert "rod outside" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.conn_node = base.conn_node.copy(); bad.conn_node[0, 0] = 999
    assert "node outside" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.conn_rod = base.conn_rod.copy(); bad.conn_node = base.conn_node.copy()
    bad.conn_rod[0] = [0, 0]; bad.conn_node[0] = [2, 2]
    assert "itself" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.conn_k = base.conn_k.copy(); bad.conn_k[1] = -1.0
    assert ">= 0" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.conn_rest = None
    assert "conn_rest" in _expect(rod.ROD_EINVAL, bad)


def test_wall_descriptor_rejected_when_invalid():
    from paper_2605_13766_amd import rod
    base = W.active_filaments(n_rods=3, n=8, box=True)
    bad = base.copy(); bad.walls = base.walls.copy(); bad.walls[0, :3] = [0.0, 0.0, 2.0]
    assert "unit vector" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.walls = np.tile(base.walls, (2, 1))
    assert "n_walls" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.wall_mu = -0.1
    assert ">= 0" in _expect(rod.ROD_EINVAL, bad)
    bad = base.copy(); bad.wall_vslip = 0.0
    assert "wall_vslip" in _expect(rod.ROD_EINVAL, bad)


def test_rod_contact_descriptor_rejected_when_invalid():
    from paper_2605_13766_amd import rod
    base = W.fibre_pile(n_rods=4, n=8, L=0.08, per_row=1, rows=2)
    bad = base.copy(); bad.rod_contact = 3
    assert "rod_contact" in _expect(rod.ROD_EINVAL, bad)
    assert "substeps" in _expect(rod.ROD_EINVAL, base, substeps=2)
    assert "contact_skin" in _expect(rod.ROD_EINVAL, base, contact_skin=float("nan"))
    assert "contact_skin" in _expect(rod.ROD_EINVAL, base, contact_skin=float("inf"))
    bad = base.copy(); bad.walls = None; bad.wall_vslip = 0.0
    assert "wall_vslip" in _expect(rod.ROD_EINVAL, bad)


def test_empty_batch_rejected():
    """A batch with no rods is an error (ROD_EINVAL), not an empty launch."""
    from paper_2605_13766_amd import rod
    import dataclasses
    one = W.ragged_batch(n_rods=1, n_min=16, n_max=16, seed=41)
    empty = dataclasses.replace(
        one, n_elems=np.zeros(0, np.int32), position=np.zeros((0, 3)), velocity=np.zeros((0, 3)),
        director=np.zeros((0, 3, 3)), omega=np.zeros((0, 3)),
        **{k: np.zeros(0, np.int32 if k.startswith("bc_") else np.float64)
           for k in ("density", "youngs", "shear_modulus", "radius", "shear_coeff", "damping", "bc_start", "bc_end")})
    assert empty.n_rods == 0
    assert "n_rods" in _expect(rod.ROD_EINVAL, empty)
