"""ctypes binding of librod.so (include/rod.h), argument marshalling only.

Every step of the rod path runs in the library's HIP kernels; this module
converts numpy arrays and torch streams to the boundary's plain pointers.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ROD_LIBRARY") or os.path.join(HERE, "librod.so")

ROD_OK, ROD_EINVAL, ROD_ENOMEM, ROD_EDEVICE, ROD_ENONFINITE, ROD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
ROD_F64, ROD_F32 = 0, 1
ROD_MAX_ELEMS = 512
ROD_FLAG_NONFINITE, ROD_FLAG_STRETCHED = 1, 2   # bits of flags()

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class RodBatchDesc(C.Structure):
    _fields_ = [
        ("n_rods", C.c_int32),
        ("n_elems", _ip),
        ("position", _dp), ("velocity", _dp), ("director", _dp), ("omega", _dp),
        ("rest_length", _dp), ("rest_kappa", _dp),
        ("density", _dp), ("youngs", _dp), ("shear_modulus", _dp), ("radius", _dp),
        ("shear_coeff", _dp), ("damping", _dp),
        ("bc_start", _ip), ("bc_end", _ip),
        ("end_force", _dp), ("couple_amp", _dp), ("couple_freq", _dp), ("couple_phase", _dp),
        ("dt", C.c_double), ("t0", C.c_double),
        ("precision", C.c_int32), ("substeps", C.c_int32), ("tile_waves", C.c_int32),
        ("inputs_on_device", C.c_int32), ("autotune", C.c_int32),
        ("magnetization", _dp), ("field", C.c_double * 9), ("field_freq", C.c_double),
        ("gravity", C.c_double * 3), ("muscle_amp", _dp), ("muscle_axis", _dp), ("muscle_freq", _dp),
        ("muscle_wavenumber", _dp), ("muscle_phase", _dp),
        ("n_connections", C.c_int32), ("conn_rod", _ip), ("conn_node", _ip), ("conn_k", _dp), ("conn_c", _dp),
        ("conn_rest", _dp),
        ("n_walls", C.c_int32), ("walls", _dp), ("wall_k", C.c_double), ("wall_c", C.c_double),
        ("wall_mu", C.c_double), ("wall_vslip", C.c_double),
        ("rod_contact", C.c_int32),
        ("contact_skin", C.c_double),
    ]


class TuneTrial(C.Structure):
    _fields_ = [("tile_waves", C.c_int32), ("substeps", C.c_int32), ("ns_per_element_step", C.c_double)]


class SurrogateDesc(C.Structure):
    _fields_ = [("k_substeps", C.c_int32), ("seed", C.c_uint64), ("max_rows", C.c_int32)]


SURROGATE_INPUTS, SURROGATE_OUTPUTS, SURROGATE_PARAMS = 96, 12, 159500


class TrainDesc(C.Structure):
    _fields_ = [("warmup_steps", C.c_int32), ("n_samples", C.c_int32), ("sample_stride", C.c_int32),
                ("epochs", C.c_int32), ("batch_rows", C.c_int32), ("lr", C.c_float), ("lr_min", C.c_float),
                ("val_fraction", C.c_float), ("seed", C.c_uint64), ("noise", C.c_float * 4)]


class JudgeDesc(C.Structure):
    _fields_ = [("judge_every", C.c_int32), ("judge_fraction", C.c_float), ("max_pos_error", C.c_float),
                ("max_orth_error", C.c_float), ("seed", C.c_uint64), ("max_energy_error", C.c_float)]


class SurrogateStats(C.Structure):
    _fields_ = [("coarse_steps", C.c_int64), ("judge_windows", C.c_int64), ("rods_judged", C.c_int64),
                ("rods_failed", C.c_int64), ("rods_plain", C.c_int64), ("max_pos_error", C.c_double),
                ("max_orth_error", C.c_double), ("max_energy_error", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RodError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rod error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load librod.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2605_13766_amd.build")
        # torch ships its own HIP runtime under the same soname as the system one the
        # library links; loading torch first makes both use torch's, whichever of
        # them the caller touches first.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.rod_batch_create.argtypes = [C.POINTER(RodBatchDesc), vp, C.POINTER(vp)]
        L.rod_step.argtypes = [vp, C.c_int64, vp]
        L.rod_energy.argtypes = [vp, _dp, vp]
        L.rod_energy_noalloc.argtypes = [vp, _dp, vp]
        L.rod_get_state.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, vp]
        L.rod_set_state.argtypes = [vp, _dp, _dp, _dp, _dp, C.c_double, vp]
        L.rod_get_flags.argtypes = [vp, _ip, vp]
        L.rod_batch_info.argtypes = [vp, C.POINTER(C.c_int64)]
        L.rod_contact_stats.argtypes = [vp, C.POINTER(C.c_int64), vp]
        L.rod_batch_destroy.argtypes = [vp]
        L.rod_batch_tuning.argtypes = [vp, C.POINTER(TuneTrial), C.c_int32, C.POINTER(C.c_int32)]
        L.rod_batch_tuning.restype = C.c_int
        L.rod_batch_destroy.restype = None
        L.rod_last_error.restype = C.c_char_p
        for f in ("rod_batch_create", "rod_step", "rod_energy", "rod_energy_noalloc", "rod_get_state", "rod_set_state",
                  "rod_get_flags", "rod_batch_info", "rod_contact_stats"):
            getattr(L, f).restype = C.c_int
        fp = C.POINTER(C.c_float)
        L.rod_surrogate_create.argtypes = [C.POINTER(SurrogateDesc), C.POINTER(vp)]
        L.rod_surrogate_destroy.argtypes = [vp]
        L.rod_surrogate_destroy.restype = None
        L.rod_surrogate_set_params.argtypes = [vp, fp]
        L.rod_surrogate_get_params.argtypes = [vp, fp]
        L.rod_surrogate_forward.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.rod_surrogate_gradients.argtypes = [vp, vp, vp, vp, C.c_int64, fp, fp, vp]
        L.rod_surrogate_train_step.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_float, fp, vp]
        L.rod_surrogate_features.argtypes = [vp, vp, vp, vp]
        L.rod_surrogate_collect.argtypes = [vp, vp, vp, vp, vp, vp]
        L.rod_surrogate_apply.argtypes = [vp, vp, vp, vp]
        L.rod_surrogate_set_normalization.argtypes = [vp, fp, fp, fp, fp]
        L.rod_surrogate_get_normalization.argtypes = [vp, fp, fp, fp, fp]
        L.rod_surrogate_train.argtypes = [vp, vp, C.POINTER(TrainDesc), fp, fp, vp]
        L.rod_surrogate_step.argtypes = [vp, vp, C.c_int64, C.POINTER(JudgeDesc), C.POINTER(SurrogateStats), vp]
        L.rod_surrogate_fallback_flags.argtypes = [vp, vp, _ip]
        L.rod_surrogate_reset_fallback.argtypes = [vp, vp]
        L.rod_surrogate_save.argtypes = [vp, C.c_char_p]
        L.rod_surrogate_perturb.argtypes = [vp, vp, fp, C.c_uint64, vp]
        L.rod_surrogate_collect_noisy.argtypes = [vp, vp, fp, C.c_uint64, vp, vp, vp, vp]
        L.rod_surrogate_load.argtypes = [vp, C.c_char_p]
        for f in ("rod_surrogate_create", "rod_surrogate_set_params", "rod_surrogate_get_params",
                  "rod_surrogate_forward", "rod_surrogate_gradients", "rod_surrogate_train_step",
                  "rod_surrogate_features", "rod_surrogate_collect", "rod_surrogate_apply",
                  "rod_surrogate_set_normalization", "rod_surrogate_get_normalization",
                  "rod_surrogate_train", "rod_surrogate_step", "rod_surrogate_fallback_flags",
                  "rod_surrogate_reset_fallback", "rod_surrogate_save", "rod_surrogate_load",
                  "rod_surrogate_perturb", "rod_surrogate_collect_noisy"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().rod_last_error().decode()


def _check(rc):
    if rc != ROD_OK:
        raise RodError(rc, last_error())


def _stream_ptr(stream) -> Optional[int]:
    """A torch.cuda.Stream, a raw integer handle or None (the null stream)."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _p(a, t=_dp):
    return C.cast(a.ctypes.data, t) if a is not None else t()


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class RodBatch:
    """A batch of rods resident on the GPU (owned by librod.so)."""

    def __init__(self, inp, precision: str = "f64", substeps: int = 0, tile_waves: int = 0,
                 t0: float = 0.0, stream=None, autotune: bool = False, device_inputs: bool = False,
                 contact_skin: float = 0.0):
        """device_inputs: hand the library device copies (torch tensors) of every
        input array instead of host arrays (inputs_on_device = 1).  contact_skin:
        the Verlet-list skin of node-sphere contact (m; 0: a fifth of the
        largest radius; negative: no lists)."""
        self._h = None
        prec = {"f64": ROD_F64, "f32": ROD_F32}[precision]
        keep = {}

        def arr(name, a, kind="d"):
            if a is None:
                return None
            v = np.ascontiguousarray(a, dtype=np.float64 if kind == "d" else np.int32)
            if device_inputs:
                import torch
                keep[name] = torch.from_numpy(v).to("cuda")
            else:
                keep[name] = v
            return v

        def ptr(name, t):
            if name not in keep:
                return None
            if device_inputs:
                return C.cast(C.c_void_p(keep[name].data_ptr()), t)
            return keep[name].ctypes.data_as(t)

        d = RodBatchDesc()
        n = arr("n", inp.n_elems, "i")
        d.n_rods = int(n.shape[0])
        d.n_elems = ptr("n", _ip)
        for name in ("position", "velocity", "director", "omega", "rest_length", "rest_kappa",
                     "density", "youngs", "shear_modulus", "radius", "shear_coeff", "damping",
                     "end_force", "couple_amp", "couple_freq", "couple_phase", "magnetization",
                     "muscle_amp", "muscle_axis", "muscle_freq", "muscle_wavenumber", "muscle_phase"):
            arr(name, getattr(inp, name, None))
            setattr(d, name, ptr(name, _dp))
        for name in ("bc_start", "bc_end", "conn_rod", "conn_node"):
            arr(name, getattr(inp, name, None), "i")
            setattr(d, name, ptr(name, _ip))
        for name in ("conn_k", "conn_c", "conn_rest"):
            arr(name, getattr(inp, name, None))
            setattr(d, name, ptr(name, _dp))
        cr = getattr(inp, "conn_rod", None)
        d.n_connections = 0 if cr is None else int(np.asarray(cr).shape[0])
        wl = getattr(inp, "walls", None)
        if wl is not None and len(wl) > 0:
            keep["walls"] = np.ascontiguousarray(np.asarray(wl, dtype=np.float64).reshape(-1, 4))   # host always
            d.n_walls = int(keep["walls"].shape[0])
            d.walls = keep["walls"].ctypes.data_as(_dp)
        d.rod_contact = int(getattr(inp, "rod_contact", 0) or 0)
        d.contact_skin = float(contact_skin)
        if d.n_walls > 0 or d.rod_contact:
            d.wall_k, d.wall_c = float(inp.wall_k), float(inp.wall_c)
            d.wall_mu, d.wall_vslip = float(inp.wall_mu), float(inp.wall_vslip)
        d.dt = float(inp.dt)
        d.t0 = float(t0)
        d.precision = prec
        d.substeps = int(substeps)
        d.tile_waves = int(tile_waves)
        d.inputs_on_device = 1 if device_inputs else 0
        d.autotune = int(autotune)
        if getattr(inp, "magnetization", None) is not None:
            fl = getattr(inp, "field", None)
            fl = np.zeros(9) if fl is None else np.asarray(fl, dtype=np.float64).reshape(9)
            d.field = (C.c_double * 9)(*[float(x) for x in fl])
            d.field_freq = float(getattr(inp, "field_freq", 0.0) or 0.0)
        g = getattr(inp, "gravity", None)
        if g is not None:
            d.gravity = (C.c_double * 3)(*[float(x) for x in np.asarray(g, dtype=np.float64).reshape(3)])
        if device_inputs:
            import torch
            torch.cuda.synchronize()
        h = C.c_void_p()
        _check(lib().rod_batch_create(C.byref(d), _stream_ptr(stream), C.byref(h)))
        self._h = h
        self.warning = last_error()
        self.precision = precision
        self.n_elems = n.copy()
        self.n_rods = d.n_rods
        self.n_elements = int(n.sum())
        self.n_nodes = self.n_elements + self.n_rods

    # ------------------------------------------------------------ calls
    def step(self, n_steps: int, stream=None):
        _check(lib().rod_step(self._h, int(n_steps), _stream_ptr(stream)))

    def energy(self, stream=None) -> np.ndarray:
        out = np.empty((self.n_rods, 5))
        _check(lib().rod_energy(self._h, _p(out), _stream_ptr(stream)))
        return out

    def energy_noalloc(self, stream=None) -> np.ndarray:
        """rod_energy_noalloc: the energies staged in the library's static buffer."""
        out = np.empty((self.n_rods, 5))
        _check(lib().rod_energy_noalloc(self._h, _p(out), _stream_ptr(stream)))
        return out

    def get_state(self, stream=None, check=True):
        """The state (host FP64 arrays) and time.  check=False returns it even
        when a rod has been flagged non-finite (the arrays are filled first)."""
        pos = np.empty((self.n_nodes, 3))
        vel = np.empty((self.n_nodes, 3))
        dr = np.empty((self.n_elements, 3, 3))
        om = np.empty((self.n_elements, 3))
        t = C.c_double()
        rc = lib().rod_get_state(self._h, _p(pos), _p(vel), _p(dr), _p(om), C.byref(t), _stream_ptr(stream))
        if check or rc != ROD_ENONFINITE:
            _check(rc)
        return pos, vel, dr, om, t.value

    def set_state(self, pos=None, vel=None, director=None, omega=None, t=0.0, stream=None):
        arrs = [_f64(pos), _f64(vel), _f64(director), _f64(omega)]
        _check(lib().rod_set_state(self._h, *[_p(a) for a in arrs], float(t), _stream_ptr(stream)))

    def tuning(self) -> list:
        """The autotuner's trials (empty unless created with autotune)."""
        buf = (TuneTrial * 12)()
        n = C.c_int32()
        _check(lib().rod_batch_tuning(self._h, buf, 12, C.byref(n)))
        return [{"tile_waves": t.tile_waves, "substeps": t.substeps, "ns_per_element_step": t.ns_per_element_step}
                for t in buf[:min(n.value, 12)]]

    def flags(self, stream=None) -> np.ndarray:
        out = np.empty(self.n_rods, dtype=np.int32)
        _check(lib().rod_get_flags(self._h, _p(out, _ip), _stream_ptr(stream)))
        return out

    def info(self) -> dict:
        a = (C.c_int64 * 8)()
        _check(lib().rod_batch_info(self._h, a))
        keys = ("n_rods", "n_elements", "n_tiles", "tile_waves", "substeps", "precision", "n_slots",
                "steps")
        return dict(zip(keys, [int(x) for x in a]))

    def contact_stats(self, stream=None) -> dict:
        """rod_contact_stats: the Verlet-list counters (zeros without lists)."""
        a = (C.c_int64 * 5)()
        _check(lib().rod_contact_stats(self._h, a, _stream_ptr(stream)))
        keys = ("passes", "builds", "fallbacks", "most_partners", "capacity")
        return dict(zip(keys, [int(x) for x in a]))

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.rod_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _dptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else C.c_void_p(int(t.data_ptr()))


class Surrogate:
    """The learned coarse step's network (owned by librod.so)."""

    def __init__(self, k_substeps: int = 32, seed: int = 0, max_rows: int = 0):
        d = SurrogateDesc(int(k_substeps), int(seed), int(max_rows))
        h = C.c_void_p()
        _check(lib().rod_surrogate_create(C.byref(d), C.byref(h)))
        self._h = h
        self.k = int(k_substeps)

    def set_params(self, flat):
        v = np.ascontiguousarray(flat, dtype=np.float32)
        assert v.size == SURROGATE_PARAMS
        _check(lib().rod_surrogate_set_params(self._h, v.ctypes.data_as(C.POINTER(C.c_float))))

    def get_params(self) -> np.ndarray:
        v = np.empty(SURROGATE_PARAMS, dtype=np.float32)
        _check(lib().rod_surrogate_get_params(self._h, v.ctypes.data_as(C.POINTER(C.c_float))))
        return v

    def forward(self, x_bf16, y_f32, stream=None):
        """x: torch bfloat16 [M, 96] on the GPU; y: torch float32 [M, 12] on the GPU."""
        _check(lib().rod_surrogate_forward(self._h, _dptr(x_bf16), int(x_bf16.shape[0]), _dptr(y_f32),
                                           _stream_ptr(stream)))

    def gradients(self, x_bf16, t_f32, mask_f32=None, stream=None):
        g = np.empty(SURROGATE_PARAMS, dtype=np.float32)
        loss = C.c_float()
        _check(lib().rod_surrogate_gradients(self._h, _dptr(x_bf16), _dptr(t_f32), _dptr(mask_f32),
                                             int(x_bf16.shape[0]), g.ctypes.data_as(C.POINTER(C.c_float)),
                                             C.byref(loss), _stream_ptr(stream)))
        return g, loss.value

    def train_step(self, x_bf16, t_f32, mask_f32=None, lr=1e-3, stream=None, return_loss=True):
        """One Adam step; returns the loss (synchronising) unless return_loss is False."""
        loss = C.c_float()
        _check(lib().rod_surrogate_train_step(self._h, _dptr(x_bf16), _dptr(t_f32), _dptr(mask_f32),
                                              int(x_bf16.shape[0]), float(lr),
                                              C.byref(loss) if return_loss else None, _stream_ptr(stream)))
        return loss.value if return_loss else None

    # ---------------------------------------------------------- data path
    @staticmethod
    def n_windows(batch) -> int:
        return int(batch.n_elements + batch.n_rods)

    def features(self, batch, out_f32, stream=None):
        _check(lib().rod_surrogate_features(self._h, batch._h, _dptr(out_f32), _stream_ptr(stream)))

    def collect(self, batch, feat, targ, mask, stream=None):
        _check(lib().rod_surrogate_collect(self._h, batch._h, _dptr(feat), _dptr(targ), _dptr(mask),
                                           _stream_ptr(stream)))

    def collect_noisy(self, batch, noise, seed, feat, targ, mask, stream=None):
        nz = np.ascontiguousarray(noise, dtype=np.float32)
        _check(lib().rod_surrogate_collect_noisy(self._h, batch._h, nz.ctypes.data_as(C.POINTER(C.c_float)), int(seed),
                                                 _dptr(feat), _dptr(targ), _dptr(mask), _stream_ptr(stream)))

    def perturb(self, batch, noise, seed, stream=None):
        nz = np.ascontiguousarray(noise, dtype=np.float32)
        _check(lib().rod_surrogate_perturb(self._h, batch._h, nz.ctypes.data_as(C.POINTER(C.c_float)), int(seed),
                                           _stream_ptr(stream)))

    def apply(self, batch, deltas, stream=None):
        _check(lib().rod_surrogate_apply(self._h, batch._h, _dptr(deltas), _stream_ptr(stream)))

    def set_normalization(self, mu_x, sd_x, mu_t, sd_t):
        a = [np.ascontiguousarray(v, dtype=np.float32) for v in (mu_x, sd_x, mu_t, sd_t)]
        _check(lib().rod_surrogate_set_normalization(self._h, *[x.ctypes.data_as(C.POINTER(C.c_float)) for x in a]))

    def get_normalization(self):
        a = [np.empty(n, dtype=np.float32) for n in (96, 96, 12, 12)]
        _check(lib().rod_surrogate_get_normalization(self._h, *[x.ctypes.data_as(C.POINTER(C.c_float)) for x in a]))
        return a

    def train(self, batch, warmup_steps=0, n_samples=2, sample_stride=None, epochs=2, batch_rows=4096,
              lr=1e-3, lr_min=1e-5, val_fraction=0.1, seed=0, noise=(0.0, 0.0, 0.0, 0.0), stream=None):
        d = TrainDesc(int(warmup_steps), int(n_samples), int(sample_stride or self.k), int(epochs),
                      int(batch_rows), float(lr), float(lr_min), float(val_fraction), int(seed),
                      (C.c_float * 4)(*[float(x) for x in noise]))
        ep = np.empty(int(epochs), dtype=np.float32)
        vl = C.c_float()
        _check(lib().rod_surrogate_train(self._h, batch._h, C.byref(d), ep.ctypes.data_as(C.POINTER(C.c_float)),
                                         C.byref(vl), _stream_ptr(stream)))
        return ep, vl.value

    def step(self, batch, n_coarse, judge_every=8, judge_fraction=0.01, max_pos_error=1e-3,
             max_orth_error=1e-5, seed=0, max_energy_error=5e-2, stream=None) -> dict:
        """n_coarse learned coarse steps (k plain steps each) with the plain
        integrator judging a sample of rods every judge_every steps."""
        j = JudgeDesc(int(judge_every), float(judge_fraction), float(max_pos_error), float(max_orth_error), int(seed),
                      float(max_energy_error))
        st = SurrogateStats()
        _check(lib().rod_surrogate_step(self._h, batch._h, int(n_coarse), C.byref(j), C.byref(st),
                                        _stream_ptr(stream)))
        return st.as_dict()

    def fallback_flags(self, batch) -> np.ndarray:
        f = np.empty(batch.n_rods, dtype=np.int32)
        _check(lib().rod_surrogate_fallback_flags(self._h, batch._h, _p(f, _ip)))
        return f

    def reset_fallback(self, batch):
        _check(lib().rod_surrogate_reset_fallback(self._h, batch._h))

    def save(self, path):
        _check(lib().rod_surrogate_save(self._h, os.fsencode(path)))

    def load(self, path):
        _check(lib().rod_surrogate_load(self._h, os.fsencode(path)))

    def close(self):
        if self._h is not None and _lib is not None:
            _lib.rod_surrogate_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
