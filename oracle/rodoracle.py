"""ctypes front end of the FP64 CPU oracle (``rod_oracle.c``).

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

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class _OrcRods(C.Structure):
    _fields_ = [
        ("n_rods", C.c_int32),
        ("n_elems", _ip),
        ("density", _dp), ("youngs", _dp), ("shear_modulus", _dp), ("radius", _dp),
        ("shear_coeff", _dp), ("damping", _dp),
        ("bc_start", _ip), ("bc_end", _ip),
        ("rest_length", _dp), ("rest_kappa", _dp), ("node_force", _dp), ("couple_amp", _dp),
        ("couple_freq", _dp), ("couple_phase", _dp), ("pos0", _dp), ("dir0", _dp),
        ("dt", C.c_double), ("t0", C.c_double), ("drop_term", C.c_int32),
        ("magnetization", _dp), ("field", C.c_double * 9), ("field_freq", C.c_double),
        ("gravity", C.c_double * 3), ("muscle_amp", _dp), ("muscle_axis", _dp), ("muscle_freq", _dp),
        ("muscle_wavenumber", _dp), ("muscle_phase", _dp),
        ("n_conn", C.c_int32), ("conn_node", _ip), ("conn_k", _dp), ("conn_c", _dp), ("conn_rest", _dp),
        ("n_walls", C.c_int32), ("wall", _dp), ("wall_k", C.c_double), ("wall_c", C.c_double),
        ("wall_mu", C.c_double), ("wall_vslip", C.c_double),
        ("rod_contact", C.c_int32),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-D_DEFAULT_SOURCE", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
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


def max_threads():
    return int(lib().orc_max_threads())
