"""ctypes binding of the C ABI in include/cl_lattice.h.

Argument marshalling only: every step of the lattice path runs in the HIP
library.  Importing this module without the built library raises
ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

# PyTorch ships its own HIP runtime under the same soname as the system one.
# Load it first so the library, torch streams and torch device memory share
# one runtime instance in this process.
try:
    import torch  # noqa: F401
except ImportError:  # the library also works without torch
    torch = None

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcl_lattice.so")

CL_OK, CL_EINVAL, CL_ENOMEM, CL_EDEVICE, CL_ESTATE, CL_EUNSTABLE, CL_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
CL_FP64, CL_FP32 = 0, 1
CL_STATIC, CL_SELF_CONSISTENT = 0, 1
CL_LEAPFROG, CL_VV4 = 0, 1

STATUS_NAMES = {0: "CL_OK", -1: "CL_EINVAL", -2: "CL_ENOMEM", -3: "CL_EDEVICE", -4: "CL_ESTATE",
                -5: "CL_EUNSTABLE", -6: "CL_EUNSUPPORTED"}


class cl_potential(C.Structure):
    _fields_ = [("m2", C.c_double * 2), ("lambda_", C.c_double * 2), ("g2", C.c_double), ("V0", C.c_double)]


class cl_scalars(C.Structure):
    _fields_ = [("a", C.c_double), ("b", C.c_double), ("eta", C.c_double), ("step", C.c_int64)]


class cl_observables(C.Structure):
    _fields_ = [("eta", C.c_double), ("a", C.c_double), ("H", C.c_double), ("EK", C.c_double * 2),
                ("EG", C.c_double * 2), ("EV", C.c_double), ("mean", C.c_double * 2), ("var", C.c_double * 2),
                ("hubble_residual", C.c_double), ("nonfinite", C.c_int32), ("reserved", C.c_int32)]


class cl_tile(C.Structure):
    _fields_ = [("tz", C.c_int), ("ty", C.c_int), ("cx", C.c_int), ("ry", C.c_int), ("pd", C.c_int)]


class cl_surrogate_cfg(C.Structure):
    _fields_ = [("n_fields", C.c_int), ("extra_inputs", C.c_int), ("hidden", C.c_int), ("layers", C.c_int),
                ("jump_steps", C.c_int), ("init_seed", C.c_uint64)]


class cl_train_cfg(C.Structure):
    _fields_ = [("epochs", C.c_int), ("lr", C.c_double), ("lr_final", C.c_double), ("shuffle_seed", C.c_uint64),
                ("holdout", C.c_int)]


class cl_train_report(C.Structure):
    _fields_ = [("steps", C.c_int), ("first_loss", C.c_double), ("last_epoch_loss", C.c_double),
                ("holdout_loss", C.c_double), ("holdout_zero", C.c_double), ("seconds", C.c_double)]


class cl_surrogate_norm(C.Structure):
    _fields_ = [("in_scale", C.c_double * 4), ("out_scale", C.c_double * 4), ("extra_mean", C.c_double * 4),
                ("extra_std", C.c_double * 4)]


class cl_surrogate_report(C.Structure):
    _fields_ = [("jumps", C.c_int), ("fallbacks", C.c_int), ("max_residual", C.c_double), ("seconds", C.c_double),
                ("net_seconds", C.c_double), ("fluct_rejects", C.c_int), ("reserved", C.c_int)]


OBS_DTYPE = np.dtype([("eta", "f8"), ("a", "f8"), ("H", "f8"), ("EK", "f8", 2), ("EG", "f8", 2), ("EV", "f8"),
                      ("mean", "f8", 2), ("var", "f8", 2), ("r", "f8"), ("nonfinite", "i4"),
                      ("reserved", "i4")])
assert OBS_DTYPE.itemsize == C.sizeof(cl_observables)

# Every symbol the header declares, with (restype, argtypes).
_P = C.c_void_p
_SIGS = {
    "cl_last_error": (C.c_char_p, [_P]),
    "cl_version": (C.c_char_p, []),
    "cl_power_spectrum": (C.c_int, [_P, C.c_int, C.c_int, C.c_double, C.c_int, _P, _P, _P]),
    "cl_create": (C.c_int, [C.c_int, C.c_double, C.c_int, C.c_int, C.POINTER(_P)]),
    "cl_create_dim": (C.c_int, [C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.POINTER(_P)]),
    "cl_destroy": (C.c_int, [_P]),
    "cl_set_stream": (C.c_int, [_P, _P]),
    "cl_attach_device_buffers": (C.c_int, [_P, _P, _P]),
    "cl_get_state_buffer": (C.c_int, [_P, C.POINTER(_P)]),
    "cl_set_background": (C.c_int, [_P, C.c_double, C.c_int, C.c_double, C.c_double]),
    "cl_set_potential": (C.c_int, [_P, C.POINTER(cl_potential)]),
    "cl_seed": (C.c_int, [_P, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double, C.c_double]),
    "cl_set_fields": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "cl_get_fields": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "cl_get_state": (C.c_int, [_P, C.POINTER(cl_scalars)]),
    "cl_set_state": (C.c_int, [_P, C.POINTER(cl_scalars)]),
    "cl_step": (C.c_int, [_P, C.c_int, C.c_double, C.c_int, _P]),
    "cl_step_noalloc": (C.c_int, [_P, C.c_int, C.c_double, C.c_int, _P]),
    "cl_gw_enable": (C.c_int, [_P, C.c_int]),
    "cl_gw_set": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "cl_gw_get": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "cl_gw_spectrum": (C.c_int, [_P, C.c_double, C.c_int, _P, _P, _P, C.POINTER(C.c_double)]),
    "cl_read_observables": (C.c_int, [_P, _P]),
    "cl_get_tile": (C.c_int, [_P, C.POINTER(cl_tile)]),
    "cl_set_tile": (C.c_int, [_P, C.POINTER(cl_tile)]),
    "cl_autotune": (C.c_int, [_P, C.c_int, C.c_char_p, C.c_size_t]),
    "cl_copy_bandwidth": (C.c_int, [C.c_size_t, C.c_int, C.POINTER(C.c_double)]),
    "cl_ensemble_create": (C.c_int, [C.c_int, C.POINTER(_P), C.POINTER(_P)]),
    "cl_ensemble_set_dt": (C.c_int, [_P, C.c_int, C.c_double]),
    "cl_ensemble_step": (C.c_int, [_P, C.c_int, C.c_int, _P]),
    "cl_ensemble_destroy": (C.c_int, [_P]),
    "cl_ensemble_get_tile": (C.c_int, [_P, C.c_int, C.POINTER(cl_tile)]),
    "cl_ensemble_autotune": (C.c_int, [_P, C.c_int, C.c_char_p, C.c_size_t]),
    "cl_surrogate_last_error": (C.c_char_p, []),
    "cl_surrogate_create": (C.c_int, [C.POINTER(cl_surrogate_cfg), C.POINTER(_P)]),
    "cl_surrogate_destroy": (C.c_int, [_P]),
    "cl_surrogate_num_params": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "cl_surrogate_get_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "cl_surrogate_set_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "cl_surrogate_forward": (C.c_int, [_P, C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "cl_surrogate_loss_grad": (C.c_int, [_P, C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                         C.POINTER(C.c_double), C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "cl_surrogate_apply_grad": (C.c_int, [_P, C.POINTER(C.c_float), C.c_double]),
    "cl_surrogate_get_normalisation": (C.c_int, [_P, C.POINTER(cl_surrogate_norm)]),
    "cl_surrogate_set_normalisation": (C.c_int, [_P, C.POINTER(cl_surrogate_norm)]),
    "cl_surrogate_dataset_reserve": (C.c_int, [_P, C.c_int, C.c_int]),
    "cl_surrogate_record_input": (C.c_int, [_P, _P]),
    "cl_surrogate_record_target": (C.c_int, [_P, _P]),
    "cl_surrogate_dataset_size": (C.c_int, [_P, C.POINTER(C.c_int)]),
    "cl_surrogate_train": (C.c_int, [_P, C.POINTER(cl_train_cfg), C.POINTER(cl_train_report)]),
    "cl_surrogate_save": (C.c_int, [_P, C.c_char_p]),
    "cl_surrogate_load": (C.c_int, [_P, C.c_char_p]),
    "cl_surrogate_set_gate": (C.c_int, [_P, C.c_double]),
    "cl_surrogate_set_jump": (C.c_int, [_P, C.c_int]),
    "cl_surrogate_advance": (C.c_int, [_P, _P, C.c_int, C.c_double, C.c_int, C.c_double, _P,
                                       C.POINTER(cl_surrogate_report)]),
}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library not built: {LIB_PATH} missing (run python -m paper_2607_24978_amd.build)")
lib = C.CDLL(LIB_PATH)
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class CLError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(st: int, handle=None):
    if st != CL_OK:
        msg = lib.cl_last_error(handle)
        raise CLError(st, msg.decode() if msg else "")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


PRECISIONS = {"fp64": CL_FP64, "fp32": CL_FP32}
INTEGRATORS = {"leapfrog": CL_LEAPFROG, "vv4": CL_VV4, "rk2": 2, "rk3": 3, "rk4": 4, "rk34": 5, "rk4_classic": 6}
EXPANSIONS = {"static": CL_STATIC, "self": CL_SELF_CONSISTENT}


class Lattice:
    """One lattice handle (cl_create / cl_create_dim ... cl_destroy); dim = 1
    or 2 gives a reduced lattice of N^dim sites."""

    def __init__(self, N: int, dx: float, n_fields: int = 1, precision: str = "fp64", dim: int = 3):
        h = _P()
        if dim == 3:
            _check(lib.cl_create(int(N), float(dx), int(n_fields), PRECISIONS[precision], C.byref(h)))
        else:
            _check(lib.cl_create_dim(int(dim), int(N), float(dx), int(n_fields), PRECISIONS[precision], C.byref(h)))
        self.h = h
        self.N, self.dx, self.n_fields, self.precision = int(N), float(dx), int(n_fields), precision
        self.dim = int(dim)

    def close(self):
        if self.h:
            lib.cl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_stream(self, stream_ptr: int):
        _check(lib.cl_set_stream(self.h, _P(stream_ptr)), self.h)

    def attach_device_buffers(self, state_ptr: int, state_pp_ptr: int):
        """Borrow caller device memory (e.g. two torch tensors' data_ptr()) in the
        library's row-interleaved layout; the caller keeps it alive."""
        _check(lib.cl_attach_device_buffers(self.h, _P(state_ptr), _P(state_pp_ptr)), self.h)

    def state_buffer(self) -> int:
        """Device address of the buffer holding the current state."""
        out = _P()
        _check(lib.cl_get_state_buffer(self.h, C.byref(out)), self.h)
        return out.value or 0

    def set_background(self, alpha=1.0, expansion="self", mp=1.0, a0=1.0):
        _check(lib.cl_set_background(self.h, float(alpha), EXPANSIONS[expansion], float(mp), float(a0)), self.h)

    def set_potential(self, m2=(0.0, 0.0), lam=(1.0, 0.0), g2=0.0, V0=0.0):
        pot = cl_potential((C.c_double * 2)(*m2), (C.c_double * 2)(*lam), float(g2), float(V0))
        _check(lib.cl_set_potential(self.h, C.byref(pot)), self.h)

    def seed(self, seed: int, fbar, pbar, cutoff: float = 0.0, amp: float = 1.0):
        fb = np.ascontiguousarray(list(fbar) + [0.0] * (2 - len(fbar)), dtype=np.float64)
        pb = np.ascontiguousarray(list(pbar) + [0.0] * (2 - len(pbar)), dtype=np.float64)
        _check(lib.cl_seed(self.h, C.c_uint64(seed), _dptr(fb), _dptr(pb), float(cutoff), float(amp)), self.h)

    def set_fields(self, f: np.ndarray, p: np.ndarray):
        shape = (self.n_fields,) + (self.N,) * self.dim
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(shape)
        p = np.ascontiguousarray(p, dtype=np.float64).reshape(shape)
        _check(lib.cl_set_fields(self.h, _dptr(f), _dptr(p)), self.h)

    def get_fields(self):
        shape = (self.n_fields,) + (self.N,) * self.dim
        f = np.empty(shape)
        p = np.empty(shape)
        _check(lib.cl_get_fields(self.h, _dptr(f), _dptr(p)), self.h)
        return f, p

    def get_state(self) -> dict:
        s = cl_scalars()
        _check(lib.cl_get_state(self.h, C.byref(s)), self.h)
        return dict(a=s.a, b=s.b, eta=s.eta, step=s.step)

    def set_state(self, a: float, b: float, eta: float, step: int = 0):
        s = cl_scalars(float(a), float(b), float(eta), int(step))
        _check(lib.cl_set_state(self.h, C.byref(s)), self.h)

    def step(self, integrator: str, dt: float, n: int, record: bool = True):
        out = np.zeros(max(n, 0), dtype=OBS_DTYPE) if record else None
        ptr = _P(out.ctypes.data) if record and n > 0 else None
        _check(lib.cl_step(self.h, INTEGRATORS[integrator], float(dt), int(n), ptr), self.h)
        return out

    def step_noalloc(self, integrator: str, dt: float, n: int, record: bool = True):
        out = np.zeros(max(n, 0), dtype=OBS_DTYPE) if record else None
        ptr = _P(out.ctypes.data) if record and n > 0 else None
        _check(lib.cl_step_noalloc(self.h, INTEGRATORS[integrator], float(dt), int(n), ptr), self.h)
        return out

    def get_tile(self) -> dict:
        t = cl_tile()
        _check(lib.cl_get_tile(self.h, C.byref(t)), self.h)
        return dict(tz=t.tz, ty=t.ty, cx=t.cx, ry=t.ry, pd=t.pd)

    def set_tile(self, tz: int, ty: int, cx: int, ry: int = 1, pd: int = 1):
        t = cl_tile(int(tz), int(ty), int(cx), int(ry), int(pd))
        _check(lib.cl_set_tile(self.h, C.byref(t)), self.h)

    def autotune(self, reps: int = 3) -> dict:
        import json
        buf = C.create_string_buffer(1 << 16)
        _check(lib.cl_autotune(self.h, int(reps), buf, len(buf)), self.h)
        return json.loads(buf.value.decode())

    def power_spectrum(self, field: int = 0, what: str = "f", width: float = 1.0, nbins: int | None = None):
        """(k, counts, sums, delta) of the binned power spectrum of f_field or pi_field."""
        if nbins is None:
            nbins = int(np.ceil(np.sqrt(3.0) * (self.N // 2) / width)) + 1
        counts = np.zeros(nbins, dtype=np.int64)
        sums = np.zeros(nbins, dtype=np.float64)
        delta = np.zeros(nbins, dtype=np.float64)
        _check(lib.cl_power_spectrum(self.h, int(field), 0 if what == "f" else 1, float(width), int(nbins),
                                     _P(counts.ctypes.data), _P(sums.ctypes.data), _P(delta.ctypes.data)), self.h)
        k = 2.0 * np.pi / (self.N * self.dx) * width * np.arange(nbins)
        return k, counts, sums, delta

    def gw_enable(self, on: bool = True):
        """Carry (or drop) the five traceless tensor components of the
        gravitational waves in the state (cl_gw_enable)."""
        _check(lib.cl_gw_enable(self.h, 1 if on else 0), self.h)

    def gw_set(self, v: np.ndarray, u: np.ndarray):
        shape = (5, self.N, self.N, self.N)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(shape)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(shape)
        _check(lib.cl_gw_set(self.h, _dptr(v), _dptr(u)), self.h)

    def gw_get(self):
        shape = (5, self.N, self.N, self.N)
        v = np.empty(shape)
        u = np.empty(shape)
        _check(lib.cl_gw_get(self.h, _dptr(v), _dptr(u)), self.h)
        return v, u

    def gw_spectrum(self, width: float = 1.0, nbins: int | None = None):
        """(counts, rho_l, omega_l, rho_GW) of the gravitational waves (cl_gw_spectrum)."""
        if nbins is None:
            nbins = int(np.ceil(np.sqrt(3.0) * (self.N // 2) / width)) + 1
        counts = np.zeros(nbins, dtype=np.int64)
        rho = np.zeros(nbins, dtype=np.float64)
        omega = np.zeros(nbins, dtype=np.float64)
        tot = C.c_double()
        _check(lib.cl_gw_spectrum(self.h, float(width), int(nbins), _P(counts.ctypes.data), _P(rho.ctypes.data),
                                  _P(omega.ctypes.data), C.byref(tot)), self.h)
        return counts, rho, omega, tot.value

    def read_observables(self):
        out = np.zeros(1, dtype=OBS_DTYPE)
        _check(lib.cl_read_observables(self.h, _P(out.ctypes.data)), self.h)
        return out[0]


def copy_bandwidth(nbytes: int, reps: int = 10) -> float:
    """Streaming-copy bandwidth of the current device in GB/s (cl_copy_bandwidth)."""
    g = C.c_double()
    _check(lib.cl_copy_bandwidth(C.c_size_t(nbytes), int(reps), C.byref(g)))
    return g.value


def _scheck(st: int):
    if st != CL_OK:
        msg = lib.cl_surrogate_last_error()
        raise CLError(st, msg.decode() if msg else "")


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Surrogate:
    """The learned surrogate (cl_surrogate_*)."""

    def __init__(self, n_fields=2, extra_inputs=2, hidden=32, layers=5, jump_steps=16, init_seed=0):
        cfg = cl_surrogate_cfg(n_fields, extra_inputs, hidden, layers, jump_steps, init_seed)
        h = _P()
        _scheck(lib.cl_surrogate_create(C.byref(cfg), C.byref(h)))
        self.s = h
        self.n_fields, self.extra_inputs, self.layers, self.jump_steps = n_fields, extra_inputs, layers, jump_steps
        self.cin = 2 * n_fields + extra_inputs
        self.cout = 2 * n_fields

    def close(self):
        if getattr(self, "s", None):
            lib.cl_surrogate_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_params(self) -> int:
        n = C.c_int64()
        _scheck(lib.cl_surrogate_num_params(self.s, C.byref(n)))
        return n.value

    def get_params(self) -> np.ndarray:
        out = np.empty(self.num_params(), dtype=np.float32)
        _scheck(lib.cl_surrogate_get_params(self.s, _fptr(out)))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        _scheck(lib.cl_surrogate_set_params(self.s, _fptr(theta)))

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        N = x.shape[-1]
        y = np.empty((self.cout, N, N, N), dtype=np.float32)
        _scheck(lib.cl_surrogate_forward(self.s, N, _fptr(x), _fptr(y)))
        return y

    def loss_grad(self, x, t, input_grad: bool = False):
        """(loss, parameter gradient) -- and the input gradient with input_grad."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        loss = C.c_double()
        g = np.empty(self.num_params(), dtype=np.float32)
        gx = np.empty_like(x) if input_grad else None
        _scheck(lib.cl_surrogate_loss_grad(self.s, x.shape[-1], _fptr(x), _fptr(t), C.byref(loss), _fptr(g),
                                           _fptr(gx) if input_grad else None))
        return (loss.value, g, gx) if input_grad else (loss.value, g)

    def apply_grad(self, grad, lr: float):
        grad = np.ascontiguousarray(grad, dtype=np.float32)
        _scheck(lib.cl_surrogate_apply_grad(self.s, _fptr(grad), float(lr)))

    def get_normalisation(self) -> dict:
        n = cl_surrogate_norm()
        _scheck(lib.cl_surrogate_get_normalisation(self.s, C.byref(n)))
        return {k: list(getattr(n, k)) for k, _ in cl_surrogate_norm._fields_}

    def set_normalisation(self, in_scale, out_scale, extra_mean=(0.0,) * 4, extra_std=(1.0,) * 4):
        n = cl_surrogate_norm()
        for k, v in (("in_scale", in_scale), ("out_scale", out_scale), ("extra_mean", extra_mean),
                     ("extra_std", extra_std)):
            vals = list(v) + [1.0 if k != "extra_mean" else 0.0] * (4 - len(v))
            setattr(n, k, (C.c_double * 4)(*vals))
        _scheck(lib.cl_surrogate_set_normalisation(self.s, C.byref(n)))

    def dataset_reserve(self, N: int, max_pairs: int):
        _scheck(lib.cl_surrogate_dataset_reserve(self.s, int(N), int(max_pairs)))

    def record_input(self, lat: "Lattice"):
        _scheck(lib.cl_surrogate_record_input(self.s, lat.h))

    def record_target(self, lat: "Lattice"):
        _scheck(lib.cl_surrogate_record_target(self.s, lat.h))

    def dataset_size(self) -> int:
        n = C.c_int()
        _scheck(lib.cl_surrogate_dataset_size(self.s, C.byref(n)))
        return n.value

    def train(self, epochs=1, lr=1e-3, lr_final=1e-5, shuffle_seed=0, holdout=0) -> dict:
        cfg = cl_train_cfg(int(epochs), float(lr), float(lr_final), int(shuffle_seed), int(holdout))
        rep = cl_train_report()
        _scheck(lib.cl_surrogate_train(self.s, C.byref(cfg), C.byref(rep)))
        return {k: getattr(rep, k) for k, _ in cl_train_report._fields_}

    def save(self, path: str):
        _scheck(lib.cl_surrogate_save(self.s, path.encode()))

    def load(self, path: str):
        _scheck(lib.cl_surrogate_load(self.s, path.encode()))

    JUMP_MODES = {"network": 0, "linear": 1}

    def set_jump(self, mode: str):
        """cl_surrogate_set_jump: "network" (the learned increment) or
        "linear" (the fluctuations' modes advanced by the linearised
        equations through the device FFT)."""
        _scheck(lib.cl_surrogate_set_jump(self.s, self.JUMP_MODES[mode]))

    def set_gate(self, fluct_tol: float):
        """Tolerance of the second (fluctuation) gate of advance(); <= 0 switches it off."""
        _scheck(lib.cl_surrogate_set_gate(self.s, float(fluct_tol)))

    def advance(self, lat: "Lattice", fallback: str, dt: float, n_jumps: int, threshold: float = 1e-3):
        out = np.zeros(max(n_jumps, 0), dtype=OBS_DTYPE)
        rep = cl_surrogate_report()
        ptr = _P(out.ctypes.data) if n_jumps > 0 else None
        _scheck(lib.cl_surrogate_advance(lat.h, self.s, INTEGRATORS[fallback], float(dt), int(n_jumps),
                                         float(threshold), ptr, C.byref(rep)))
        return out, {k: getattr(rep, k) for k, _ in cl_surrogate_report._fields_}


class Ensemble:
    """Several lattices advanced together (cl_ensemble_*)."""

    def __init__(self, members):
        self.members = list(members)
        arr = (_P * len(self.members))(*[m.h for m in self.members])
        e = _P()
        _check(lib.cl_ensemble_create(len(self.members), arr, C.byref(e)))
        self.e = e

    def set_dt(self, i: int, dt: float):
        _check(lib.cl_ensemble_set_dt(self.e, int(i), float(dt)))

    def step(self, integrator: str, n: int, record: bool = True):
        out = np.zeros((max(n, 0), len(self.members)), dtype=OBS_DTYPE) if record else None
        ptr = _P(out.ctypes.data) if record and n > 0 else None
        _check(lib.cl_ensemble_step(self.e, INTEGRATORS[integrator], int(n), ptr))
        return out

    def get_tile(self, i: int) -> dict:
        t = cl_tile()
        _check(lib.cl_ensemble_get_tile(self.e, int(i), C.byref(t)))
        return dict(tz=t.tz, ty=t.ty, cx=t.cx, ry=t.ry, pd=t.pd)

    def autotune(self, reps: int = 3) -> dict:
        """Time every distinct work decomposition on the current states (left
        unchanged) and keep the fastest; returns the library's JSON report."""
        buf = C.create_string_buffer(16384)
        _check(lib.cl_ensemble_autotune(self.e, int(reps), buf, len(buf)))
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "e", None):
            lib.cl_ensemble_destroy(self.e)
            self.e = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
