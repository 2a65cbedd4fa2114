"""Python binding of libnbody (include/nbody.h): argument marshalling only.

Device memory and streams come from PyTorch (ROCm build); every step of the computation runs in
the library's HIP kernels.  The functions and methods carry the C ABI's names.  If the shared
library has not been built this module raises on first use: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib", "libnbody.so")

NB_OK, NB_EINVAL, NB_EDEVICE, NB_ENOMEM, NB_ESTATE, NB_ENONFINITE, NB_EDTMIN = 0, -1, -2, -3, -4, -5, -6
PRECISIONS = {"fp32": 0, "ds": 1, "fp64": 2, "fp32all": 3, "fp32fixed": 4}
_STATUS_NAMES = {0: "NB_OK", -1: "NB_EINVAL", -2: "NB_EDEVICE", -3: "NB_ENOMEM", -4: "NB_ESTATE",
                 -5: "NB_ENONFINITE", -6: "NB_EDTMIN"}


class NBodyError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class nb_state(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("v", ctypes.c_void_p), ("a", ctypes.c_void_p),
                ("k", ctypes.c_void_p), ("m", ctypes.c_void_p), ("pot", ctypes.c_void_p),
                ("tick", ctypes.c_void_p), ("level", ctypes.c_void_p)]


class nb_control(ctypes.Structure):
    _fields_ = [("t_cur", ctypes.c_int64), ("t_next", ctypes.c_int64), ("t_end", ctypes.c_int64),
                ("n_steps", ctypes.c_int64), ("n_active_sum", ctypes.c_int64),
                ("n_act", ctypes.c_int32), ("flags", ctypes.c_int32)]


def _variant_dict(v):
    return dict(ipl=v.ipl, unroll=v.unroll, target=v.target, kmax=v.kmax,
                scalar_tiles=v.scalar_tiles)


class nb_variant(ctypes.Structure):
    _fields_ = [("ipl", ctypes.c_int32), ("unroll", ctypes.c_int32), ("target", ctypes.c_int32),
                ("kmax", ctypes.c_int32), ("scalar_tiles", ctypes.c_int32)]


EXPORTS = ["nb_create", "nb_destroy", "nb_set_stream", "nb_bind", "nb_init",
           "nb_schedule_block", "nb_active", "nb_predict", "nb_force", "nb_correct", "nb_step",
           "nb_run", "nb_energy", "nb_read_control", "nb_get_variant", "nb_set_variant",
           "nb_tune", "nb_profile", "nb_profile_read", "nb_sync", "nb_last_error", "nb_version",
           "nb_ens_create", "nb_ens_destroy", "nb_ens_set_stream", "nb_ens_bind",
           "nb_ens_set_layout", "nb_ens_init", "nb_ens_run", "nb_ens_control", "nb_ens_energy",
           "nb_ens_last_error", "nb_shared_step", "nb_force_vjp", "nb_step_vjp",
           "nb_scratch_bytes", "nb_bind_scratch", "nb_ens_scratch_bytes", "nb_ens_bind_scratch",
           "nb_ens_set_local", "nb_fma_rate", "nb_force_noalloc",
           "nb_set_resident", "nb_ens_set_split", "nb_ens_set_lanes"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libnbody.so and declare its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first "
                           "(python -m paper_astro_ph_0702058_amd.build)")
    # torch brings its own HIP runtime (same soname); loading it first makes the library bind
    # to that one, so that one runtime owns every device pointer in the process.
    _torch()
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "nb_create": [ctypes.POINTER(P), I32, D, I32, I32, I32],
        "nb_destroy": [P],
        "nb_set_stream": [P, P],
        "nb_bind": [P, ctypes.POINTER(nb_state)],
        "nb_init": [P, D],
        "nb_schedule_block": [P, D],
        "nb_active": [P, ctypes.POINTER(P), ctypes.POINTER(P)],
        "nb_predict": [P, P],
        "nb_force": [P, P, P, I32, P, P, P],
        "nb_correct": [P, P, P, P],
        "nb_step": [P, D, I32, I32],
        "nb_run": [P, D, I64, I64, I32, I32],
        "nb_energy": [P, ctypes.POINTER(D), ctypes.POINTER(D)],
        "nb_read_control": [P, ctypes.POINTER(nb_control)],
        "nb_get_variant": [P, I32, ctypes.POINTER(nb_variant)],
        "nb_set_variant": [P, I32, ctypes.POINTER(nb_variant)],
        "nb_tune": [P, I32, I32, I32, ctypes.POINTER(nb_variant), ctypes.POINTER(D)],
        "nb_profile": [P, I32],
        "nb_profile_read": [P, I32, ctypes.POINTER(D), ctypes.POINTER(I64)],
        "nb_sync": [P],
        "nb_shared_step": [P, D, I32],
        "nb_force_vjp": [P, P, P, P, P, P],
        "nb_step_vjp": [P, D, P, P, P, P, P],
        "nb_ens_create": [ctypes.POINTER(P), I32, P, P, I32, I32, I32],
        "nb_ens_destroy": [P],
        "nb_ens_set_stream": [P, P],
        "nb_ens_bind": [P, ctypes.POINTER(nb_state)],
        "nb_ens_set_layout": [P, P, I32, I32],
        "nb_ens_init": [P, D],
        "nb_ens_run": [P, D, I64, I32, I64, I32],
        "nb_ens_control": [P, ctypes.POINTER(nb_control)],
        "nb_ens_energy": [P, P, P],
        "nb_bind_scratch": [P, P, ctypes.c_size_t],
        "nb_ens_bind_scratch": [P, P, ctypes.c_size_t],
        "nb_ens_set_local": [P, I64, I32, I64],
        "nb_ens_set_split": [P, I32],
        "nb_ens_set_lanes": [P, I32, P],
        "nb_fma_rate": [P, ctypes.POINTER(D)],
        "nb_force_noalloc": [P, P, P, I32, P, P, P],
        "nb_set_resident": [P, I32],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.nb_last_error.argtypes = [P]
    lib.nb_last_error.restype = ctypes.c_char_p
    lib.nb_ens_last_error.argtypes = [P]
    lib.nb_ens_last_error.restype = ctypes.c_char_p
    lib.nb_version.argtypes = []
    lib.nb_version.restype = ctypes.c_char_p
    lib.nb_scratch_bytes.argtypes = [I32, I32]
    lib.nb_scratch_bytes.restype = ctypes.c_size_t
    lib.nb_ens_scratch_bytes.argtypes = [I32, P, I32]
    lib.nb_ens_scratch_bytes.restype = ctypes.c_size_t
    if path == LIB_PATH:
        _lib = lib
    return lib


def _torch():
    import torch
    return torch


def read_device_int32(addr: int, count: int) -> np.ndarray:
    """Copy `count` int32 values at device address `addr` to a new host array (synchronising),
    with the HIP runtime the library is bound to."""
    lib = load_library()
    out = np.empty(int(count), np.int32)
    if count > 0:
        _torch().cuda.synchronize()
        f = lib.hipMemcpy
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        f.restype = ctypes.c_int
        rc = f(out.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(addr), 4 * int(count), 2)
        if rc != 0:
            raise NBodyError(NB_EDEVICE, f"hipMemcpy failed ({rc})")
    return out


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _device_tensor(t, name, dtype, shape=None):
    """Raise unless t is a contiguous GPU tensor of this dtype (and shape): the library reads
    and writes through raw device pointers, so a host tensor or another element type would be
    misread on the device."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype must be {dtype} (got {t.dtype})")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a GPU tensor (got device {t.device})")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape must be {tuple(shape)} (got {tuple(t.shape)})")


def check_force_args(n, acc, jerk, pot, i_idx, n_i, n_i_max):
    """Validate nb_force arguments on the host before anything is enqueued.  acc, jerk:
    (3, n_i_max) float64 GPU tensors; pot: (n_i_max,).  i_idx: None (rows 0 .. n_i - 1), a
    device address (int, not checkable here), or an int32 GPU tensor of at least n_i_max
    entries (checked to lie in [0, n) when it is a tensor and no device count is given).  n_i:
    None, a device address, or an int32 GPU tensor of one or more entries."""
    torch = _torch()
    if not 0 <= n_i_max <= n:
        raise ValueError(f"n_i_max {n_i_max} outside [0, {n}]")
    _device_tensor(acc, "acc", torch.float64, (3, n_i_max))
    _device_tensor(jerk, "jerk", torch.float64, (3, n_i_max))
    _device_tensor(pot, "pot", torch.float64, (n_i_max,))
    if n_i is not None and not isinstance(n_i, int):
        _device_tensor(n_i, "n_i", torch.int32)
        if n_i.numel() < 1:
            raise ValueError("n_i: needs one entry")
    if i_idx is not None and not isinstance(i_idx, int):
        _device_tensor(i_idx, "i_idx", torch.int32)
        if i_idx.dim() != 1 or i_idx.numel() < (n_i_max if n_i is None else 1):
            raise ValueError(f"i_idx: a 1-D list of at least {n_i_max} entries is required")
        if n_i is None and n_i_max > 0:
            lo, hi = int(i_idx[:n_i_max].min()), int(i_idx[:n_i_max].max())
            if lo < 0 or hi >= n:
                raise ValueError(f"i_idx: indices must lie in [0, {n}) (got {lo} .. {hi})")


class DeviceState:
    """FP64 master state on the GPU as torch tensors, structure-of-arrays:
    x, v, a, k: (3, n) float64 (the planes of one (4, 3, n) buffer, xvak); m, pot: (n,)
    float64; tick: (n,) int64; level: (n,) int32."""

    def __init__(self, x, v, m, device="cuda"):
        torch = _torch()
        x = np.asarray(x, np.float64).reshape(-1, 3)
        v = np.asarray(v, np.float64).reshape(-1, 3)
        self.n = x.shape[0]
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        # x, v, a, k are the four (3, n) planes of one buffer, so that the whole dynamical
        # state is saved or restored by one device copy (xvak)
        self.xvak = torch.zeros((4, 3, self.n), **f64)
        self.x, self.v, self.a, self.k = self.xvak.unbind(0)
        self.x.copy_(torch.from_numpy(np.ascontiguousarray(x.T)))
        self.v.copy_(torch.from_numpy(np.ascontiguousarray(v.T)))
        self.m = torch.tensor(np.asarray(m, np.float64), **f64)
        self.pot = torch.zeros(self.n, **f64)
        self.tick = torch.zeros(self.n, dtype=torch.int64, device=dev)
        self.level = torch.zeros(self.n, dtype=torch.int32, device=dev)

    def as_struct(self):
        return nb_state(*(t.data_ptr() for t in
                          (self.x, self.v, self.a, self.k, self.m, self.pot, self.tick, self.level)))

    def numpy(self):
        """(x, v, a, k) as (n, 3) numpy arrays plus m, pot, tick, level."""
        g = lambda t: t.detach().cpu().numpy()
        return dict(x=g(self.x).T.copy(), v=g(self.v).T.copy(), a=g(self.a).T.copy(),
                    k=g(self.k).T.copy(), m=g(self.m), pot=g(self.pot), tick=g(self.tick),
                    level=g(self.level))


@dataclass
class Control:
    t_cur: int
    t_next: int
    t_end: int
    n_steps: int
    n_active_sum: int
    n_act: int
    flags: int


class Context:
    """One libnbody context: n particles, softening eps, steps in [2^-lmax, 2^-lmin]."""

    def __init__(self, n, eps, lmin=3, lmax=26, precision="fp32", stream=None, allow_dtmin=False):
        """allow_dtmin: do not raise NB_EDTMIN (a step request below 2^-lmax, clamped; the call
        itself completed); `dtmin_clamped` records that it was seen."""
        self.allow_dtmin = bool(allow_dtmin)
        self.dtmin_clamped = False
        self.lib = load_library()
        self.n = int(n)
        self.eps = float(eps)
        self.lmin, self.lmax = int(lmin), int(lmax)
        self.precision = precision
        h = ctypes.c_void_p()
        self._check(self.lib.nb_create(ctypes.byref(h), self.n, self.eps, self.lmin, self.lmax,
                                       PRECISIONS[precision]), ctx=None)
        self.h = h
        self.state = None
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream()
        self.nb_set_stream(s)
        # the library's work buffers live in one torch-owned device tensor
        nbytes = int(self.lib.nb_scratch_bytes(self.n, PRECISIONS[precision]))
        if nbytes == 0:
            raise NBodyError(NB_EINVAL, "nb_scratch_bytes: invalid arguments")
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.nb_bind_scratch(self.scratch)

    def nb_bind_scratch(self, scratch):
        """Bind a uint8 GPU tensor of at least nb_scratch_bytes() bytes as the workspace."""
        _device_tensor(scratch, "scratch", _torch().uint8)
        self._check(self.lib.nb_bind_scratch(self.h, _ptr(scratch), scratch.numel()))

    # -- plumbing
    def _check(self, status, ctx="self"):
        if status == NB_EDTMIN and self.allow_dtmin:
            self.dtmin_clamped = True
            return
        if status != NB_OK:
            msg = ""
            if ctx is not None and getattr(self, "h", None):
                msg = self.lib.nb_last_error(self.h).decode()
            raise NBodyError(status, msg)

    def close(self):
        if getattr(self, "h", None):
            self.lib.nb_destroy(self.h)
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

    # -- C ABI
    def nb_set_stream(self, stream):
        self.stream = stream
        self._check(self.lib.nb_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)))

    def nb_bind(self, state: DeviceState):
        assert state.n == self.n
        self.state = state
        self._struct = state.as_struct()
        self._check(self.lib.nb_bind(self.h, ctypes.byref(self._struct)))

    def nb_init(self, eta):
        self._check(self.lib.nb_init(self.h, float(eta)))

    def nb_schedule_block(self, eta):
        self._check(self.lib.nb_schedule_block(self.h, float(eta)))

    def nb_active(self):
        """(device address of the int32 block list, device address of its int32 count)."""
        idx, cnt = ctypes.c_void_p(), ctypes.c_void_p()
        self._check(self.lib.nb_active(self.h, ctypes.byref(idx), ctypes.byref(cnt)))
        return idx.value, cnt.value

    def nb_predict(self, t=None):
        """Predict all particles to the device int64 tensor t (ticks), or to the block time."""
        if t is not None:
            _device_tensor(t, "t", _torch().int64)
        self._check(self.lib.nb_predict(self.h, _ptr(t)))

    def nb_force(self, acc, jerk, pot, i_idx=None, n_i=None, n_i_max=None):
        """acc, jerk: (3, n_i_max) float64 tensors; pot: (n_i_max,).  i_idx: int32 tensor or a
        device address; n_i: int32 device tensor/address (or None = n_i_max)."""
        n_i_max = acc.shape[1] if n_i_max is None else int(n_i_max)
        check_force_args(self.n, acc, jerk, pot, i_idx, n_i, n_i_max)
        ii = ctypes.c_void_p(i_idx) if isinstance(i_idx, int) else _ptr(i_idx)
        nn = ctypes.c_void_p(n_i) if isinstance(n_i, int) else _ptr(n_i)
        self._check(self.lib.nb_force(self.h, ii, nn, n_i_max, _ptr(acc), _ptr(jerk), _ptr(pot)))

    def nb_force_noalloc(self, acc, jerk, pot, i_idx=None, n_i=None, n_i_max=None):
        """nb_force whose j-split partial sums live in the library's static device array
        (allocates nothing); same arguments and results."""
        n_i_max = acc.shape[1] if n_i_max is None else int(n_i_max)
        check_force_args(self.n, acc, jerk, pot, i_idx, n_i, n_i_max)
        ii = ctypes.c_void_p(i_idx) if isinstance(i_idx, int) else _ptr(i_idx)
        nn = ctypes.c_void_p(n_i) if isinstance(n_i, int) else _ptr(n_i)
        self._check(self.lib.nb_force_noalloc(self.h, ii, nn, n_i_max, _ptr(acc), _ptr(jerk),
                                              _ptr(pot)))

    def nb_correct(self, acc, jerk, pot):
        """acc, jerk: (3, n) float64 GPU tensors (the block's rows first), pot: (n,)."""
        torch = _torch()
        _device_tensor(acc, "acc", torch.float64, (3, self.n))
        _device_tensor(jerk, "jerk", torch.float64, (3, self.n))
        _device_tensor(pot, "pot", torch.float64, (self.n,))
        self._check(self.lib.nb_correct(self.h, _ptr(acc), _ptr(jerk), _ptr(pot)))

    def nb_step(self, eta, nsteps=1, use_graph=True):
        self._check(self.lib.nb_step(self.h, float(eta), int(nsteps), int(bool(use_graph))))

    def nb_run(self, eta, t_end, max_steps=0, chunk=64, use_graph=True):
        """Advance to time t_end (time units, converted to ticks)."""
        t_ticks = int(round(float(t_end) * 2.0 ** self.lmax))
        self._check(self.lib.nb_run(self.h, float(eta), t_ticks, int(max_steps), int(chunk),
                                    int(bool(use_graph))))

    def nb_set_resident(self, max_n):
        """nb_run on contexts of at most max_n particles uses one resident workgroup (0: never)."""
        self._check(self.lib.nb_set_resident(self.h, int(max_n)))

    def nb_energy(self):
        ek, ep = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.nb_energy(self.h, ctypes.byref(ek), ctypes.byref(ep)))
        return ek.value, ep.value

    def nb_read_control(self, check: bool = True) -> Control:
        """The scheduler record.  check=False: return it even when a latched device flag
        (NB_EDTMIN or NB_ENONFINITE) makes the call report an error; `flags` then says which."""
        c = nb_control()
        st = self.lib.nb_read_control(self.h, ctypes.byref(c))
        if check or st not in (NB_OK, NB_EDTMIN, NB_ENONFINITE):
            self._check(st)
        return Control(c.t_cur, c.t_next, c.t_end, c.n_steps, c.n_active_sum, c.n_act, c.flags)

    def nb_get_variant(self, which):
        v = nb_variant()
        self._check(self.lib.nb_get_variant(self.h, int(which), ctypes.byref(v)))
        return _variant_dict(v)

    def nb_set_variant(self, which, variant):
        """`variant`: ipl, unroll, target, kmax and optionally scalar_tiles (absent or 0: the
        context's current value)."""
        v = nb_variant(int(variant["ipl"]), int(variant["unroll"]), int(variant["target"]),
                       int(variant["kmax"]), int(variant.get("scalar_tiles", 0)))
        self._check(self.lib.nb_set_variant(self.h, int(which), ctypes.byref(v)))

    def nb_tune(self, which, n_i, reps=2):
        """Time every force-kernel variant and keep the fastest for `which` (0: full-force
        calls, 1: block-step calls).  Returns (variant dict, mean milliseconds)."""
        v, ms = nb_variant(), ctypes.c_double()
        self._check(self.lib.nb_tune(self.h, int(which), int(n_i), int(reps), ctypes.byref(v),
                                     ctypes.byref(ms)))
        return _variant_dict(v), ms.value

    def nb_shared_step(self, dt, nsteps=1):
        self._check(self.lib.nb_shared_step(self.h, float(dt), int(nsteps)))

    def nb_force_vjp(self, abar, kbar, xbar, vbar, mbar):
        """Adds the force VJP at the predicted stream to xbar, vbar (3, n) and mbar (n,)."""
        torch = _torch()
        for t, name in ((abar, "abar"), (kbar, "kbar"), (xbar, "xbar"), (vbar, "vbar")):
            _device_tensor(t, name, torch.float64, (3, self.n))
        _device_tensor(mbar, "mbar", torch.float64, (self.n,))
        self._check(self.lib.nb_force_vjp(self.h, _ptr(abar), _ptr(kbar), _ptr(xbar), _ptr(vbar),
                                          _ptr(mbar)))

    def nb_step_vjp(self, dt, xbar, vbar, abar, kbar, mbar):
        """In place: output adjoints of one shared step from the bound state -> input adjoints."""
        torch = _torch()
        for t, name in ((xbar, "xbar"), (vbar, "vbar"), (abar, "abar"), (kbar, "kbar")):
            _device_tensor(t, name, torch.float64, (3, self.n))
        _device_tensor(mbar, "mbar", torch.float64, (self.n,))
        self._check(self.lib.nb_step_vjp(self.h, float(dt), _ptr(xbar), _ptr(vbar), _ptr(abar),
                                         _ptr(kbar), _ptr(mbar)))

    def nb_profile(self, enable=True):
        self._check(self.lib.nb_profile(self.h, int(bool(enable))))

    def nb_profile_read(self, which=-1):
        """(total force-kernel milliseconds, number of timed launches) of one launch class
        (0: full force, 1: block steps and small lists, -1: all)."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(self.lib.nb_profile_read(self.h, int(which), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def nb_fma_rate(self):
        """Measured FP32 FMA rate of the device, TFLOP/s (calibration kernel)."""
        t = ctypes.c_double()
        self._check(self.lib.nb_fma_rate(self.h, ctypes.byref(t)))
        return t.value

    def nb_sync(self):
        self._check(self.lib.nb_sync(self.h))


def force_on_state(x, v, m, eps, precision="fp32", idx=None, device="cuda"):
    """Acceleration, jerk and potential of particles ``idx`` (all if None) of the state
    (x, v, m) at its own time, through nb_predict (zero time offset) and nb_force.
    Returns numpy (acc (n_i,3), jerk (n_i,3), pot (n_i,))."""
    torch = _torch()
    st = DeviceState(x, v, m, device=device)
    with Context(st.n, eps, precision=precision) as ctx:
        ctx.nb_bind(st)
        t0 = torch.zeros(1, dtype=torch.int64, device=device)
        ctx.nb_predict(t0)
        if idx is None:
            n_i = st.n
            ii = None
        else:
            ii = torch.as_tensor(np.asarray(idx, np.int32), device=device)
            n_i = ii.numel()
        acc = torch.zeros((3, n_i), dtype=torch.float64, device=device)
        jerk = torch.zeros_like(acc)
        pot = torch.zeros(n_i, dtype=torch.float64, device=device)
        if n_i > 0:
            ctx.nb_force(acc, jerk, pot, i_idx=ii)
        ctx.nb_sync()
        return acc.cpu().numpy().T.copy(), jerk.cpu().numpy().T.copy(), pot.cpu().numpy()


class Ensemble:
    """Many independent clusters stepped together (nb_ens_*).  `sizes`: particles per
    cluster; `eps`: softening per cluster; the state is one DeviceState over all particles,
    clusters contiguous in the given order."""

    def __init__(self, sizes, eps, lmin=3, lmax=26, precision="fp32", stream=None):
        self.lib = load_library()
        sizes = np.asarray(sizes, np.int64)
        self.C = int(sizes.size)
        self.offsets = np.zeros(self.C + 1, np.int32)
        self.offsets[1:] = np.cumsum(sizes)
        self.eps = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, np.float64), (self.C,)))
        self.lmin, self.lmax, self.precision = int(lmin), int(lmax), precision
        h = ctypes.c_void_p()
        st = self.lib.nb_ens_create(ctypes.byref(h), self.C,
                                    self.offsets.ctypes.data_as(ctypes.c_void_p),
                                    self.eps.ctypes.data_as(ctypes.c_void_p), self.lmin, self.lmax,
                                    PRECISIONS[precision])
        if st != NB_OK:
            raise NBodyError(st, "nb_ens_create failed")
        self.h = h
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream()
        self._check(self.lib.nb_ens_set_stream(self.h, ctypes.c_void_p(s.cuda_stream)))
        nbytes = int(self.lib.nb_ens_scratch_bytes(self.C, self.offsets.ctypes.data_as(ctypes.c_void_p),
                                                   PRECISIONS[precision]))
        if nbytes == 0:
            raise NBodyError(NB_EINVAL, "nb_ens_scratch_bytes: invalid arguments")
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self._check(self.lib.nb_ens_bind_scratch(self.h, _ptr(self.scratch), nbytes))

    def _check(self, status):
        if status != NB_OK:
            raise NBodyError(status, self.lib.nb_ens_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.nb_ens_destroy(self.h)
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

    def nb_ens_bind(self, state: DeviceState):
        assert state.n == int(self.offsets[-1])
        self.state = state
        self._struct = state.as_struct()
        self._check(self.lib.nb_ens_bind(self.h, ctypes.byref(self._struct)))

    def nb_ens_set_layout(self, tiles_per_item=None, ipl=1, unroll=2):
        arr = None
        if tiles_per_item is not None:
            self._tpi = np.ascontiguousarray(np.broadcast_to(np.asarray(tiles_per_item, np.int32),
                                                             (self.C,)))
            arr = self._tpi.ctypes.data_as(ctypes.c_void_p)
        self._check(self.lib.nb_ens_set_layout(self.h, arr, int(ipl), int(unroll)))

    def nb_ens_set_local(self, local_limit, local_steps=64, local_work=1 << 21):
        """Blocks of at most local_limit interactions (n_act * N_c, and n_act <= 1024) are
        advanced by the cluster's own workgroup, up to local_steps block steps and local_work
        interactions per cluster per global step (local_limit = 0: never)."""
        self._check(self.lib.nb_ens_set_local(self.h, int(local_limit), int(local_steps),
                                              int(local_work)))

    def nb_ens_set_split(self, smin):
        """Every block particle of a force item shared by at least smin lanes (power of 2)."""
        self._check(self.lib.nb_ens_set_split(self.h, int(smin)))

    def nb_ens_set_lanes(self, lane_of=None):
        """Independent lanes: lane_of[c] in [0, lanes) for every cluster (None: one lane)."""
        if lane_of is None:
            self._check(self.lib.nb_ens_set_lanes(self.h, 1, None))
            return
        lane_of = np.ascontiguousarray(lane_of, dtype=np.int32)
        if lane_of.shape != (self.C,):
            raise ValueError(f"lane_of: one lane per cluster ({self.C}) expected")
        lanes = int(lane_of.max()) + 1 if lane_of.size else 1
        self._check(self.lib.nb_ens_set_lanes(self.h, lanes, lane_of.ctypes.data_as(ctypes.c_void_p)))

    def nb_ens_init(self, eta):
        self._check(self.lib.nb_ens_init(self.h, float(eta)))

    def nb_ens_run(self, eta, t_end, steps_per_launch=128, max_steps=0, use_graph=True):
        t_ticks = int(round(float(t_end) * 2.0 ** self.lmax))
        self._check(self.lib.nb_ens_run(self.h, float(eta), t_ticks, int(steps_per_launch),
                                        int(max_steps), int(bool(use_graph))))

    def nb_ens_control(self):
        arr = (nb_control * self.C)()
        self._check(self.lib.nb_ens_control(self.h, arr))
        return [Control(c.t_cur, c.t_next, c.t_end, c.n_steps, c.n_active_sum, c.n_act, c.flags)
                for c in arr]

    def nb_ens_energy(self):
        ek = np.zeros(self.C); ep = np.zeros(self.C)
        self._check(self.lib.nb_ens_energy(self.h, ek.ctypes.data_as(ctypes.c_void_p),
                                           ep.ctypes.data_as(ctypes.c_void_p)))
        return ek, ep
