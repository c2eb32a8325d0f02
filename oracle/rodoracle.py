"""ctypes front end of the FP64 CPU oracle (``rod_oracle.c``) and of its FP32
mirror (the same source built in single precision).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never does.  It imports nothing from
the GPU package.  Inputs arrive as a ``RodInputs``-like object (any object with
the attributes of the boundary descriptor); loads may also be given in the
oracle's more general form (per-node forces, per-element couples) for the
closed-form checks.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rod_oracle.c")
_LIB = os.path.join(_HERE, "librod_oracle.so")
_LIB32 = os.path.join(_HERE, "librod_oracle32.so")

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int32)


def _orc_fields(rp):
    """Fields of the C struct orc_rods; `rp` is the pointer type of its `real`
    arrays (double in the oracle, float in the FP32 mirror)."""
    return [
        ("n_rods", C.c_int32),
        ("n_elems", _ip),
        ("density", rp), ("youngs", rp), ("shear_modulus", rp), ("radius", rp),
        ("shear_coeff", rp), ("damping", rp),
        ("bc_start", _ip), ("bc_end", _ip),
        ("rest_length", rp), ("rest_kappa", rp), ("node_force", rp), ("couple_amp", rp),
        ("couple_freq", _dp), ("couple_phase", _dp), ("pos0", _dp), ("dir0", rp),
        ("dt", C.c_double), ("t0", C.c_double), ("drop_term", C.c_int32),
        ("magnetization", rp), ("field", C.c_double * 9), ("field_freq", C.c_double),
        ("gravity", C.c_double * 3), ("muscle_amp", rp), ("muscle_axis", rp), ("muscle_freq", _dp),
        ("muscle_wavenumber", _dp), ("muscle_phase", _dp),
        ("n_conn", C.c_int32), ("conn_node", _ip), ("conn_k", _dp), ("conn_c", _dp), ("conn_rest", _dp),
        ("n_walls", C.c_int32), ("wall", _dp), ("wall_k", C.c_double), ("wall_c", C.c_double),
        ("wall_mu", C.c_double), ("wall_vslip", C.c_double),
        ("rod_contact", C.c_int32),
        ("origin", _dp),
    ]


class _OrcRods(C.Structure):
    _fields_ = _orc_fields(_dp)


class _OrcRods32(C.Structure):
    _fields_ = _orc_fields(_fp)


# names of the orc_rods arrays of type `real` (FP32 in the mirror)
_REAL_FIELDS = ("density", "youngs", "shear_modulus", "radius", "shear_coeff", "damping", "rest_length",
                "rest_kappa", "node_force", "couple_amp", "dir0", "magnetization", "muscle_amp", "muscle_axis")

_COMMON = ["-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-D_DEFAULT_SOURCE"]
# the FP32 mirror: the same source in single precision (literals included)
_F32_FLAGS = ["-DORC_F32", "-fsingle-precision-constant"]


def build(force: bool = False) -> str:
    """Compile the oracle and its FP32 mirror with gcc (-O2, OpenMP, no
    fast-math, no FMA contraction)."""
    for out, extra in ((_LIB, []), (_LIB32, _F32_FLAGS)):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            cmd = ["gcc", *_COMMON, *extra, "-o", out + ".tmp", _SRC, "-lm"]
            subprocess.check_call(cmd)
            os.replace(out + ".tmp", out)
    return _LIB


# AddressSanitizer and UBSan build (tests only): every error aborts the process
_SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build_sanitized(outdir: str) -> str:
    """Compile the oracle and its FP32 mirror with AddressSanitizer and UBSan
    into `outdir` (same file names).  Loaded by a process that has gcc's
    libasan preloaded and ROD_ORACLE_LIBDIR=outdir."""
    os.makedirs(outdir, exist_ok=True)
    for name, extra in (("librod_oracle.so", []), ("librod_oracle32.so", _F32_FLAGS)):
        out = os.path.join(outdir, name)
        subprocess.check_call(["gcc", *_COMMON, *extra, *_SAN_FLAGS, "-o", out, _SRC, "-lm"])
    return outdir


def _lib_paths():
    """The two libraries: those in ROD_ORACLE_LIBDIR when it is set (a
    sanitizer build), else the regular build (compiled when stale)."""
    d = os.environ.get("ROD_ORACLE_LIBDIR")
    if d:
        return os.path.join(d, "librod_oracle.so"), os.path.join(d, "librod_oracle32.so")
    build()
    return _LIB, _LIB32


_lib = None
_lib32 = None


def lib32():
    """The FP32 mirror's library (orc_step on float state arrays)."""
    global _lib32
    if _lib32 is None:
        L = C.CDLL(_lib_paths()[1])
        L.orc_step.argtypes = [C.POINTER(_OrcRods32), _fp, _fp, _fp, _fp, C.c_int64, C.c_int64, C.c_int]
        L.orc_step.restype = C.c_int
        _lib32 = L
    return _lib32


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(_lib_paths()[0])
        P = C.POINTER(_OrcRods)
        L.orc_step.argtypes = [P, _dp, _dp, _dp, _dp, C.c_int64, C.c_int64, C.c_int]
        L.orc_step.restype = C.c_int
        L.orc_strains.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        L.orc_strains.restype = C.c_int
        L.orc_accel.argtypes = [P, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp]
        L.orc_accel.restype = C.c_int
        L.orc_energy.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        L.orc_energy.restype = C.c_int
        L.orc_rodrigues.argtypes = [_dp, _dp]
        L.orc_segment_closest.argtypes = [_dp, _dp, _dp, _dp, _dp]
        L.orc_logmap.argtypes = [_dp, _dp]
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return C.cast(a.ctypes.data, t) if a is not None else t()


def rest_lengths_from(position, n_elems):
    """Chord lengths |r_{i+1} - r_i| of every element."""
    out = []
    off = 0
    for n in n_elems:
        seg = position[off:off + n + 1]
        out.append(np.linalg.norm(np.diff(seg, axis=0), axis=1))
        off += n + 1
    return np.concatenate(out)


class Oracle:
    """One batch of rods and its FP64 state, advanced by the C oracle.

    ``node_force`` [N_n,3] and ``elem_couple`` [N_e,3] override the boundary's
    per-rod ``end_force`` / ``couple_amp`` when given.
    """

    def __init__(self, inp, node_force=None, elem_couple=None, drop_term=0, t0=0.0):
        self.inp = inp
        n = np.ascontiguousarray(inp.n_elems, dtype=np.int32)
        R = n.shape[0]
        self.n_elems = n
        self.R = R
        Ne = int(n.sum())
        Nn = Ne + R
        self.pos = _d(inp.position).copy().reshape(Nn, 3)
        self.vel = _d(inp.velocity).copy().reshape(Nn, 3)
        self.dir = _d(inp.director).copy().reshape(Ne, 3, 3)
        self.omega = _d(inp.omega).copy().reshape(Ne, 3)
        self.pos0 = self.pos.copy()
        self.dir0 = self.dir.copy()
        self.rest_length = (_d(inp.rest_length) if inp.rest_length is not None
                            else rest_lengths_from(self.pos, n))
        self.rest_kappa = _d(inp.rest_kappa)
        if node_force is None and getattr(inp, "end_force", None) is not None:
            node_force = np.zeros((Nn, 3))
            node_off = np.concatenate([[0], np.cumsum(n + 1)[:-1]])
            node_force[node_off + n] = inp.end_force
        self.node_force = _d(node_force)
        if elem_couple is None and getattr(inp, "couple_amp", None) is not None:
            elem_couple = np.repeat(np.asarray(inp.couple_amp, float), n, axis=0)
        self.elem_couple = _d(elem_couple)
        cf = getattr(inp, "couple_freq", None)
        cp = getattr(inp, "couple_phase", None)
        self.couple_freq = _d(cf if cf is not None else np.zeros(R))
        self.couple_phase = _d(cp if cp is not None else np.full(R, np.pi / 2))
        mg = getattr(inp, "magnetization", None)
        self.magnetization = _d(np.asarray(mg, float).reshape(Ne, 3)) if mg is not None else None
        fl = getattr(inp, "field", None)
        self.field = np.zeros(9) if fl is None else np.asarray(fl, float).reshape(9).copy()
        self.field_freq = float(getattr(inp, "field_freq", 0.0) or 0.0)
        g = getattr(inp, "gravity", None)
        self.gravity = np.zeros(3) if g is None else np.asarray(g, float).reshape(3).copy()
        ma = getattr(inp, "muscle_amp", None)
        self.muscle = None
        if ma is not None:
            self.muscle = [_d(np.asarray(ma, float).reshape(-1))] + [
                _d(np.asarray(getattr(inp, k), float).reshape(-1))
                for k in ("muscle_axis", "muscle_freq", "muscle_wavenumber", "muscle_phase")]
        cr = getattr(inp, "conn_rod", None)
        self.conn = None
        if cr is not None and len(cr) > 0:
            no = np.concatenate([[0], np.cumsum(np.asarray(inp.n_elems) + 1)])
            nodes = no[np.asarray(cr, dtype=np.int64)] + np.asarray(inp.conn_node, dtype=np.int64)
            self.conn = (np.ascontiguousarray(nodes, dtype=np.int32),
                         _d(np.asarray(inp.conn_k, float)), _d(np.asarray(inp.conn_c, float)),
                         _d(np.asarray(inp.conn_rest, float)))
        wl = getattr(inp, "walls", None)
        self.walls = None if wl is None or len(wl) == 0 else _d(np.asarray(wl, float).reshape(-1, 4))
        self.wall_par = [float(getattr(inp, k, 0.0) or 0.0) for k in ("wall_k", "wall_c", "wall_mu", "wall_vslip")]
        self.rod_contact = int(getattr(inp, "rod_contact", 0) or 0)
        self.mat = {k: _d(getattr(inp, k)) for k in
                    ("density", "youngs", "shear_modulus", "radius", "shear_coeff", "damping")}
        self.bc_start = np.ascontiguousarray(inp.bc_start, dtype=np.int32)
        self.bc_end = np.ascontiguousarray(inp.bc_end, dtype=np.int32)
        self.dt = float(inp.dt)
        self.t0 = float(t0)
        self.step_index = 0
        self.drop_term = int(drop_term)
        self._mk()

    def _mk(self):
        s = _OrcRods()
        s.n_rods = self.R
        s.n_elems = _ptr(self.n_elems, _ip)
        for k, v in self.mat.items():
            setattr(s, k, _ptr(v))
        s.bc_start = _ptr(self.bc_start, _ip)
        s.bc_end = _ptr(self.bc_end, _ip)
        s.rest_length = _ptr(self.rest_length)
        s.rest_kappa = _ptr(self.rest_kappa)
        s.node_force = _ptr(self.node_force)
        s.couple_amp = _ptr(self.elem_couple)
        s.couple_freq = _ptr(self.couple_freq)
        s.couple_phase = _ptr(self.couple_phase)
        s.pos0 = _ptr(self.pos0)
        s.dir0 = _ptr(self.dir0)
        s.dt = self.dt
        s.t0 = self.t0
        s.drop_term = self.drop_term
        s.magnetization = _ptr(self.magnetization)
        s.field = (C.c_double * 9)(*[float(x) for x in self.field])
        s.field_freq = self.field_freq
        s.gravity = (C.c_double * 3)(*[float(x) for x in self.gravity])
        if self.muscle is not None:
            s.muscle_amp, s.muscle_axis, s.muscle_freq, s.muscle_wavenumber, s.muscle_phase = \
                [_ptr(a) for a in self.muscle]
        if self.walls is not None:
            s.n_walls = int(self.walls.shape[0])
            s.wall = _ptr(self.walls)
        if self.walls is not None or self.rod_contact:
            s.wall_k, s.wall_c, s.wall_mu, s.wall_vslip = self.wall_par
        s.rod_contact = self.rod_contact
        if self.conn is not None:
            s.n_conn = int(self.conn[0].shape[0])
            s.conn_node = self.conn[0].ctypes.data_as(_ip)
            s.conn_k, s.conn_c, s.conn_rest = [_ptr(a) for a in self.conn[1:]]
        self._s = s

    @property
    def time(self):
        return self.t0 + self.step_index * self.dt

    def step(self, n_steps=1, n_threads=0):
        rc = lib().orc_step(C.byref(self._s), _ptr(self.pos), _ptr(self.vel), _ptr(self.dir),
                            _ptr(self.omega), self.step_index, int(n_steps), int(n_threads))
        if rc != 0:
            raise MemoryError("oracle step failed")
        self.step_index += int(n_steps)

    def strains(self):
        Ne = self.dir.shape[0]
        sigma = np.empty((Ne, 3))
        kappa = np.empty((max(Ne - self.R, 0), 3))
        dil = np.empty(Ne)
        lib().orc_strains(C.byref(self._s), _ptr(self.pos), _ptr(self.dir), _ptr(sigma),
                          _ptr(kappa), _ptr(dil))
        return sigma, kappa, dil

    def accel(self, t=None):
        acc = np.empty_like(self.pos)
        alpha = np.empty_like(self.omega)
        t = self.time + 0.5 * self.dt if t is None else t
        lib().orc_accel(C.byref(self._s), _ptr(self.pos), _ptr(self.vel), _ptr(self.dir),
                        _ptr(self.omega), float(t), _ptr(acc), _ptr(alpha))
        return acc, alpha

    def energy(self):
        out = np.empty((self.R, 5))
        lib().orc_energy(C.byref(self._s), _ptr(self.pos), _ptr(self.vel), _ptr(self.dir),
                         _ptr(self.omega), _ptr(out))
        return out

    def state(self):
        return self.pos.copy(), self.vel.copy(), self.dir.copy(), self.omega.copy()


def rodrigues(u):
    E = np.empty(9)
    uu = _d(np.asarray(u, float).reshape(3))
    lib().orc_rodrigues(_ptr(uu), _ptr(E))
    return E.reshape(3, 3)


def logmap(R):
    u = np.empty(3)
    RR = _d(np.asarray(R, float).reshape(9))
    lib().orc_logmap(_ptr(RR), _ptr(u))
    return u


def segment_closest(p0, p1, q0, q1):
    """Parameters (s, t) of the closest points of two segments (the oracle's routine)."""
    out = np.zeros(2)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (p0, p1, q0, q1)]
    lib().orc_segment_closest(*[_ptr(x) for x in a], _ptr(out))
    return float(out[0]), float(out[1])


def max_threads():
    return int(lib().orc_max_threads())


def _f(a):
    """Round an FP64 array once to FP32 (round to nearest even)."""
    return None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


class Oracle32:
    """The FP32 mirror of the oracle: the same step carried out in single
    precision (see the header of rod_oracle.c), with positions held as an FP64
    origin per rod (its first node at creation) plus an FP32 anchor and FP32
    edge vectors.  Inputs are rounded once from FP64.

    ``state()`` returns FP64 arrays with node positions summed from origin,
    anchor and edges in FP64.  ``energy()`` evaluates the FP64 oracle's
    energies on that state with the rounded constants: the energies of the
    mirror's own state and model.
    """

    def __init__(self, inp, t0=0.0):
        o = Oracle(inp, t0=t0)
        self._o64 = o
        self.R = o.R
        self.n_elems = o.n_elems
        self.dt = o.dt
        self.t0 = o.t0
        self.step_index = 0
        no = np.concatenate([[0], np.cumsum(o.n_elems + 1)[:-1]]).astype(np.int64)
        self._no = no
        self.origin = np.ascontiguousarray(o.pos0[no])
        edges = np.diff(o.pos, axis=0)
        # row 0 of each rod: the anchor (node 0 relative to the origin, 0 at
        # creation); row j > 0: edge j - 1
        x = np.empty_like(o.pos)
        x[no] = 0.0
        rest = np.ones(len(o.pos), bool)
        rest[no] = False
        x[rest] = edges[np.nonzero(rest)[0] - 1]
        self.x = _f(x)
        self.vel = _f(o.vel)
        self.dir = _f(o.dir)
        self.omega = _f(o.omega)
        # the rounded constants, kept for the energies
        self._round = {k: _f(getattr(o, a)) for k, a in (
            ("rest_length", "rest_length"), ("rest_kappa", "rest_kappa"), ("node_force", "node_force"),
            ("couple_amp", "elem_couple"), ("dir0", "dir0"), ("magnetization", "magnetization"))}
        self._mat = {k: _f(v) for k, v in o.mat.items()}
        self._muscle = None if o.muscle is None else [_f(o.muscle[0]), _f(o.muscle[1])]
        s = _OrcRods32()
        for name, _ in _OrcRods32._fields_:
            if name in _REAL_FIELDS:
                continue
            setattr(s, name, getattr(o._s, name))
        for k, v in self._mat.items():
            setattr(s, k, _ptr(v, _fp))
        for k, v in self._round.items():
            setattr(s, k, _ptr(v, _fp))
        if self._muscle is not None:
            s.muscle_amp, s.muscle_axis = [_ptr(a, _fp) for a in self._muscle]
        s.origin = _ptr(self.origin)
        self._s = s

    @property
    def time(self):
        return self.t0 + self.step_index * self.dt

    def step(self, n_steps=1, n_threads=0):
        rc = lib32().orc_step(C.byref(self._s), _ptr(self.x, _fp), _ptr(self.vel, _fp), _ptr(self.dir, _fp),
                              _ptr(self.omega, _fp), self.step_index, int(n_steps), int(n_threads))
        if rc != 0:
            raise MemoryError("oracle step failed")
        self.step_index += int(n_steps)

    def positions(self):
        """Node positions in FP64: origin + anchor + the edges before each node."""
        x = self.x.astype(np.float64)
        pos = np.empty_like(x)
        for r, (a, n) in enumerate(zip(self._no, self.n_elems)):
            pos[a:a + n + 1] = self.origin[r] + np.cumsum(x[a:a + n + 1], axis=0)
        return pos

    def state(self):
        return (self.positions(), self.vel.astype(np.float64), self.dir.astype(np.float64),
                self.omega.astype(np.float64))

    def energy(self):
        e = self._o64
        saved = ({k: getattr(e, k) for k in ("rest_length", "rest_kappa", "node_force", "elem_couple")},
                 dict(e.mat), e.muscle)
        try:
            e.rest_length = self._round["rest_length"].astype(np.float64)
            for k, a in (("rest_kappa", "rest_kappa"), ("node_force", "node_force"), ("couple_amp", "elem_couple")):
                r = self._round[k]
                setattr(e, a, None if r is None else r.astype(np.float64))
            e.mat = {k: v.astype(np.float64) for k, v in self._mat.items()}
            e._mk()
            out = np.empty((self.R, 5))
            pos, vel, dr, om = self.state()
            lib().orc_energy(C.byref(e._s), _ptr(np.ascontiguousarray(pos)), _ptr(np.ascontiguousarray(vel)),
                             _ptr(np.ascontiguousarray(dr)), _ptr(np.ascontiguousarray(om)), _ptr(out))
        finally:
            for k, v in saved[0].items():
                setattr(e, k, v)
            e.mat = saved[1]
            e._mk()
        return out
