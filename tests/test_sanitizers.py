"""AddressSanitizer and UBSan over the CPU code: the oracle (every workload kind
in both of its precisions) and the host runtime of the library (descriptor
validation, input gathering and checks, tile packing and the derivation of the
per-slot constants, which all run before the first device allocation; on a
machine without a GPU a valid batch then stops at that allocation with
ROD_EDEVICE).  Each runs in a child process with the sanitizer runtime
preloaded; any report aborts it."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow

_ORACLE_DRIVER = r"""
import numpy as np
from oracle import rodoracle as ro
from paper_2605_13766_amd import workloads as W
cases = [
    W.single_cantilever(n=20),
    W.ragged_batch(n_rods=4, n_min=2, n_max=40, seed=11),
    W.magnetic_carpet(grid=2, n=10),
    W.active_filaments(n_rods=3, n=12, box=True),
    W.millipede_swarm(n_bots=1),
    W.fibre_pile(n_rods=24, n=20, L=0.2, per_row=2, rows=4, noise=1e-2, seed=5),
]
for inp in cases:
    for cls in (ro.Oracle, ro.Oracle32):
        o = cls(inp)
        o.step(30)
        e = o.energy()
        assert np.all(np.isfinite(e)), inp.name
    o = ro.Oracle(inp)
    o.strains()
    o.accel()
print("oracle cases done", len(cases), flush=True)
"""

_HOST_DRIVER = r"""
import numpy as np
from paper_2605_13766_amd import rod, workloads as W
L = rod.lib()
def code(inp, **kw):
    try:
        rod.RodBatch(inp, **kw).close()
        return 0
    except rod.RodError as e:
        return e.code
base = W.ragged_batch(n_rods=3, n_min=16, n_max=20, seed=41)
bad = []
b = base.copy(); b.dt = 0.0; bad.append(b)
b = base.copy(); b.youngs = b.youngs.copy(); b.youngs[1] = -1.0; bad.append(b)
b = base.copy(); b.director = b.director.copy(); b.director[5, 0, 0] += 1e-6; bad.append(b)
b = base.copy(); b.position = b.position.copy(); b.position[3] = b.position[2]; bad.append(b)
b = base.copy(); b.velocity = b.velocity.copy(); b.velocity[0, 0] = np.nan; bad.append(b)
b = base.copy(); b.couple_amp = np.ones((3, 3)); bad.append(b)
for b in bad:
    assert code(b) == rod.ROD_EINVAL
assert code(base, tile_waves=3) == rod.ROD_EINVAL
assert code(W.ragged_batch(n_rods=1, n_min=600, n_max=600, seed=43)) == rod.ROD_EINVAL
assert code(W.ragged_batch(n_rods=2, n_min=100, n_max=120, seed=45), tile_waves=1) == rod.ROD_EUNSUPPORTED
valid = [
    (W.ragged_batch(n_rods=64, n_min=2, n_max=256, seed=12), {}),
    (W.ragged_batch(n_rods=64, n_min=2, n_max=256, seed=12), dict(precision="f32", tile_waves=8)),
    (W.magnetic_carpet(grid=4, n=50), dict(precision="f32")),
    (W.active_filaments(n_rods=8, n=50, box=True), {}),
    (W.millipede_swarm(n_bots=2), dict(precision="f32")),
    (W.fibre_pile(n_rods=24, n=20, L=0.2, per_row=2, rows=4, noise=1e-2, seed=5), {}),
]
for inp, kw in valid:
    c = code(inp, **kw)
    assert c in (rod.ROD_OK, rod.ROD_EDEVICE), (inp.name, c)
assert L.rod_step(None, 10, None) == rod.ROD_EINVAL
assert L.rod_energy_noalloc(None, None, None) == rod.ROD_EINVAL
L.rod_batch_destroy(None)
print("host cases done", len(bad) + 3 + len(valid), flush=True)
"""


def _run(driver, env_extra, timeout=600):
    env = dict(os.environ)
    env.update(env_extra)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    env["OMP_NUM_THREADS"] = "2"
    p = subprocess.run([sys.executable, "-c", driver], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=timeout)
    out = p.stdout + p.stderr
    print(out[-3000:])
    assert p.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out
    return out


def test_oracle_under_asan_and_ubsan(tmp_path):
    from oracle import rodoracle as ro
    d = ro.build_sanitized(str(tmp_path / "oracle"))
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    out = _run(_ORACLE_DRIVER, {"ROD_ORACLE_LIBDIR": d, "LD_PRELOAD": asan,
                                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
                                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    assert "oracle cases done 6" in out


def test_host_runtime_under_asan_and_ubsan(tmp_path):
    from paper_2605_13766_amd import build as B
    lib = B.build_sanitized(str(tmp_path / "lib"))
    out = _run(_HOST_DRIVER, {"ROD_LIBRARY": lib, "LD_PRELOAD": B.asan_runtime(),
                              "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
                              "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    assert "host cases done" in out


def test_the_harness_reports_a_planted_overflow(tmp_path):
    """The same flags and preload catch a one-past-the-end read (a planted
    mistake in a throwaway CPU library, not in the code under test)."""
    from oracle import rodoracle as ro
    src = tmp_path / "bad.c"
    src.write_text("double last(const double *a, int n) { double s = 0; for (int i = 0; i <= n; ++i) s += a[i];"
                   " return s; }\n#include <stdlib.h>\n"
                   "double run(void) { double *a = malloc(8 * sizeof(double)); for (int i = 0; i < 8; ++i) a[i] = i;"
                   " double s = last(a, 8); free(a); return s; }\n")
    so = tmp_path / "libbad.so"
    subprocess.check_call(["gcc", "-fPIC", "-shared", *ro._SAN_FLAGS, "-o", str(so), str(src)])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    p = subprocess.run([sys.executable, "-c", f"import ctypes; L = ctypes.CDLL({str(so)!r}); "
                        "L.run.restype = ctypes.c_double; print(L.run())"], env=env, capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0 and "heap-buffer-overflow" in p.stderr
