"""ctypes binding of liblb (include/lb.h): same names, argument marshalling only.

Every step of the lattice-Boltzmann update runs in the HIP kernels of
liblb.so; this module only converts arguments (NumPy arrays or torch tensors
to pointers, torch's current stream to a hipStream_t) and turns status codes
into ``LBError``.  It raises ``LBLibraryMissing`` if the library has not been
built -- there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblb.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_ESTATE, LB_ENONFINITE = 0, -1, -2, -3, -4, -5
LB_F64, LB_F32, LB_F16_SHIFTED = 0, 1, 2
LB_KERNEL_AUTO, LB_KERNEL_FUSED, LB_KERNEL_TWO_PASS, LB_KERNEL_FUSED_STAGED = 0, 1, 2, 3
KERNELS = {"auto": LB_KERNEL_AUTO, "fused": LB_KERNEL_FUSED, "two_pass": LB_KERNEL_TWO_PASS,
           "fused_staged": LB_KERNEL_FUSED_STAGED}
STORAGE = {"f64": LB_F64, "f32": LB_F32, "f16s": LB_F16_SHIFTED}
LB_MODEL_SHAN_CHEN, LB_MODEL_COLOUR_GRADIENT = 0, 1
MODELS = {"shan_chen": LB_MODEL_SHAN_CHEN, "colour_gradient": LB_MODEL_COLOUR_GRADIENT}
Q = 19


class LBLibraryMissing(RuntimeError):
    pass


class LBError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {lb_strerror(status)} (status {status})")


class lb_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("tau", ctypes.c_double * 2),
        ("G", ctypes.c_double),
        ("psi_ref", ctypes.c_double),
        ("rho0", ctypes.c_double * 2),
        ("storage", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


_lib = None

# (name, restype, argtypes) of every symbol include/lb.h declares
_P = ctypes.c_void_p
_SIGNATURES = [
    ("lb_params_default", None, [ctypes.POINTER(lb_params)]),
    ("lb_create", ctypes.c_int, [ctypes.POINTER(lb_params), ctypes.POINTER(_P)]),
    ("lb_destroy", ctypes.c_int, [_P]),
    ("lb_set_stream", ctypes.c_int, [_P, _P]),
    ("lb_set_fields", ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int]),
    ("lb_step", ctypes.c_int, [_P, ctypes.c_int32]),
    ("lb_moments", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int]),
    ("lb_get_populations", ctypes.c_int, [_P, _P, ctypes.c_int]),
    ("lb_set_populations", ctypes.c_int, [_P, _P, ctypes.c_int]),
    ("lb_totals", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
    ("lb_timing", ctypes.c_int, [_P, ctypes.c_int]),
    ("lb_timing_read", ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]),
    ("lb_timing_slots", ctypes.c_int32, []),
    ("lb_timing_name", ctypes.c_char_p, [ctypes.c_int32]),
    ("lb_set_kernel", ctypes.c_int, [_P, ctypes.c_int32]),
    ("lb_set_coupling", ctypes.c_int, [_P, ctypes.c_double]),
    ("lb_set_model", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double]),
    ("lb_state_bytes", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    ("lb_save_state", ctypes.c_int, [_P, _P, ctypes.c_int]),
    ("lb_restore_state", ctypes.c_int, [_P, _P, ctypes.c_int]),
    ("lb_step_between", ctypes.c_int, [_P, _P, _P]),
    ("lb_adjoint_begin", ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    ("lb_adjoint_step", ctypes.c_int, [_P, _P]),
    ("lb_adjoint_result", ctypes.c_int, [_P, _P, _P, ctypes.POINTER(ctypes.c_double), ctypes.c_int]),
    ("lb_adjoint_lambda", ctypes.c_int, [_P, _P, ctypes.c_int]),
    ("lb_record_bytes", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    ("lb_step_record", ctypes.c_int, [_P, _P]),
    ("lb_adjoint_step_record", ctypes.c_int, [_P, _P]),
    ("lb_device_bytes", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    ("lb1_create", ctypes.c_int, [ctypes.POINTER(lb_params), ctypes.POINTER(_P)]),
    ("lb1_destroy", ctypes.c_int, [_P]),
    ("lb1_set_stream", ctypes.c_int, [_P, _P]),
    ("lb1_set_fields", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int]),
    ("lb1_step", ctypes.c_int, [_P, ctypes.c_int32]),
    ("lb1_moments", ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    ("lb1_get_populations", ctypes.c_int, [_P, _P, ctypes.c_int]),
    ("lb1_totals", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
    ("lb1_set_particles", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _P, _P, _P]),
    ("lb1_get_particles", ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    ("lb_set_particles", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _P, _P, _P]),
    ("lb_get_particles", ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    ("lb_snapshot_totals", ctypes.c_int, [ctypes.POINTER(lb_params), _P, _P, _P, ctypes.c_int32]),
    ("lb_strerror", ctypes.c_char_p, [ctypes.c_int]),
    ("lb_abi_version", ctypes.c_int32, []),
]
SYMBOLS = [s[0] for s in _SIGNATURES]


def library():
    """Load liblb.so once; raise LBLibraryMissing if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LBLibraryMissing(
                f"{LIB_PATH} is not built; run `python -m paper_2112_08264_amd.build` (hipcc, gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status: int, where: str) -> int:
    if status != LB_OK:
        raise LBError(status, where)
    return status


def lb_strerror(status: int) -> str:
    return library().lb_strerror(int(status)).decode()


def lb_abi_version() -> int:
    return int(library().lb_abi_version())


def _current_stream(device: int):
    try:
        import torch
    except ImportError:  # pragma: no cover - torch is part of the image
        return None
    if not torch.cuda.is_available():
        return None
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(a, dtype_name: str, count: int, what: str):
    """(pointer, on_device) of a contiguous NumPy array or torch tensor, or (None, 0)."""
    if a is None:
        return None, 0
    mod = type(a).__module__
    if mod.startswith("torch"):
        if not a.is_contiguous():
            raise ValueError(f"{what}: tensor must be contiguous")
        if str(a.dtype) != f"torch.{dtype_name}":
            raise TypeError(f"{what}: expected torch.{dtype_name}, got {a.dtype}")
        if a.numel() != count:
            raise ValueError(f"{what}: expected {count} elements, got {a.numel()}")
        return ctypes.c_void_p(a.data_ptr()), int(a.is_cuda)
    import numpy as np
    if not isinstance(a, np.ndarray):
        raise TypeError(f"{what}: expected a NumPy array or a torch tensor")
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError(f"{what}: array must be C-contiguous")
    if a.dtype != np.dtype(dtype_name):
        raise TypeError(f"{what}: expected {dtype_name}, got {a.dtype}")
    if a.size != count:
        raise ValueError(f"{what}: expected {count} elements, got {a.size}")
    return ctypes.c_void_p(a.ctypes.data), 0


def _same_side(*flags):
    s = {f for f in flags if f is not None}
    if len(s) > 1:
        raise ValueError("all arrays of one call must be either host or device")
    return s.pop() if s else 0


# ---------------------------------------------------------------------------
# Thin wrappers, one per C entry point
# ---------------------------------------------------------------------------
def lb_params_default() -> lb_params:
    p = lb_params()
    library().lb_params_default(ctypes.byref(p))
    return p


def lb_create(params: lb_params) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(library().lb_create(ctypes.byref(params), ctypes.byref(ctx)), "lb_create")
    return ctx


def lb_destroy(ctx) -> None:
    _check(library().lb_destroy(ctx), "lb_destroy")


def lb_set_stream(ctx, stream) -> None:
    _check(library().lb_set_stream(ctx, stream), "lb_set_stream")


def lb_set_fields(ctx, n: int, rho_a, rho_b, u=None, solid=None) -> None:
    pa, da = _ptr(rho_a, "float64", n, "rho_a")
    pb, db = _ptr(rho_b, "float64", n, "rho_b")
    pu, du = _ptr(u, "float64", 3 * n, "u")
    ps, ds = _ptr(solid, "uint8", n, "solid")
    on_dev = _same_side(da, db, du if u is not None else None, ds if solid is not None else None)
    _check(library().lb_set_fields(ctx, pa, pb, pu, ps, on_dev), "lb_set_fields")


def lb_step(ctx, nsteps: int) -> None:
    _check(library().lb_step(ctx, int(nsteps)), "lb_step")


def lb_moments(ctx, n: int, rho_a=None, rho_b=None, u=None) -> None:
    pa, da = _ptr(rho_a, "float64", n, "rho_a")
    pb, db = _ptr(rho_b, "float64", n, "rho_b")
    pu, du = _ptr(u, "float64", 3 * n, "u")
    on_dev = _same_side(da if rho_a is not None else None, db if rho_b is not None else None,
                        du if u is not None else None)
    _check(library().lb_moments(ctx, pa, pb, pu, on_dev), "lb_moments")


def lb_get_populations(ctx, n: int, f) -> None:
    pf, df = _ptr(f, "float64", 2 * Q * n, "f")
    _check(library().lb_get_populations(ctx, pf, df), "lb_get_populations")


def lb_set_populations(ctx, n: int, f) -> None:
    pf, df = _ptr(f, "float64", 2 * Q * n, "f")
    _check(library().lb_set_populations(ctx, pf, df), "lb_set_populations")


def lb_totals(ctx) -> Tuple[Tuple[float, ...], bool]:
    out = (ctypes.c_double * 5)()
    nf = ctypes.c_int(0)
    st = library().lb_totals(ctx, out, ctypes.byref(nf))
    if st not in (LB_OK, LB_ENONFINITE):
        _check(st, "lb_totals")
    return tuple(out), bool(nf.value)


def lb_timing(ctx, enable: bool) -> None:
    _check(library().lb_timing(ctx, int(bool(enable))), "lb_timing")


def lb_timing_read(ctx, slot: int) -> Tuple[float, int]:
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(library().lb_timing_read(ctx, int(slot), ctypes.byref(ms), ctypes.byref(n)), "lb_timing_read")
    return ms.value, n.value


def lb_timing_slots() -> int:
    return int(library().lb_timing_slots())


def lb_timing_name(slot: int) -> Optional[str]:
    r = library().lb_timing_name(int(slot))
    return r.decode() if r is not None else None


def lb_set_kernel(ctx, kernel) -> None:
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    _check(library().lb_set_kernel(ctx, k), "lb_set_kernel")


def lb_set_coupling(ctx, G: float) -> None:
    _check(library().lb_set_coupling(ctx, float(G)), "lb_set_coupling")


def lb_set_model(ctx, model, sigma: float = 0.0, beta: float = 0.0) -> None:
    m = MODELS[model] if isinstance(model, str) else int(model)
    _check(library().lb_set_model(ctx, m, float(sigma), float(beta)), "lb_set_model")


def lb_state_bytes(ctx) -> int:
    b = ctypes.c_int64(0)
    _check(library().lb_state_bytes(ctx, ctypes.byref(b)), "lb_state_bytes")
    return b.value


def _raw(buf, nbytes: int, what: str):
    """(pointer, on_device) of a contiguous byte buffer (uint8 tensor or NumPy array) of nbytes."""
    mod = type(buf).__module__
    if mod.startswith("torch"):
        if not buf.is_contiguous() or buf.numel() * buf.element_size() != nbytes:
            raise ValueError(f"{what}: need a contiguous buffer of {nbytes} bytes")
        return ctypes.c_void_p(buf.data_ptr()), int(buf.is_cuda)
    import numpy as np
    if not isinstance(buf, np.ndarray) or not buf.flags["C_CONTIGUOUS"] or buf.nbytes != nbytes:
        raise ValueError(f"{what}: need a contiguous buffer of {nbytes} bytes")
    return ctypes.c_void_p(buf.ctypes.data), 0


def lb_save_state(ctx, dst) -> None:
    p, d = _raw(dst, lb_state_bytes(ctx), "dst")
    _check(library().lb_save_state(ctx, p, d), "lb_save_state")


def lb_restore_state(ctx, src) -> None:
    p, d = _raw(src, lb_state_bytes(ctx), "src")
    _check(library().lb_restore_state(ctx, p, d), "lb_restore_state")


def lb_step_between(ctx, fin, fout) -> None:
    nb = lb_state_bytes(ctx)
    pi, di = _raw(fin, nb, "fin")
    po, do = _raw(fout, nb, "fout")
    if not (di and do):
        raise ValueError("lb_step_between needs device buffers")
    _check(library().lb_step_between(ctx, pi, po), "lb_step_between")


def lb_adjoint_begin(ctx, n: int, dJ_drho_a=None, dJ_drho_b=None) -> None:
    pa, da = _ptr(dJ_drho_a, "float64", n, "dJ_drho_a")
    pb, db = _ptr(dJ_drho_b, "float64", n, "dJ_drho_b")
    on_dev = _same_side(da if dJ_drho_a is not None else None, db if dJ_drho_b is not None else None)
    _check(library().lb_adjoint_begin(ctx, pa, pb, on_dev), "lb_adjoint_begin")


def lb_adjoint_step(ctx, state) -> None:
    p, d = _raw(state, lb_state_bytes(ctx), "state")
    if not d:
        raise ValueError("lb_adjoint_step needs a device snapshot")
    _check(library().lb_adjoint_step(ctx, p), "lb_adjoint_step")


def lb_adjoint_result(ctx, n: int, dJ_drho_a0=None, dJ_drho_b0=None) -> float:
    pa, da = _ptr(dJ_drho_a0, "float64", n, "dJ_drho_a0")
    pb, db = _ptr(dJ_drho_b0, "float64", n, "dJ_drho_b0")
    on_dev = _same_side(da if dJ_drho_a0 is not None else None, db if dJ_drho_b0 is not None else None)
    g = ctypes.c_double(0.0)
    _check(library().lb_adjoint_result(ctx, pa, pb, ctypes.byref(g), on_dev), "lb_adjoint_result")
    return g.value


def lb_adjoint_lambda(ctx, n: int, lam) -> None:
    p, d = _ptr(lam, "float64", 2 * Q * n, "lam")
    _check(library().lb_adjoint_lambda(ctx, p, d), "lb_adjoint_lambda")


def lb_record_bytes(ctx) -> int:
    b = ctypes.c_int64(0)
    _check(library().lb_record_bytes(ctx, ctypes.byref(b)), "lb_record_bytes")
    return b.value


def lb_step_record(ctx, record) -> None:
    p, d = _raw(record, lb_record_bytes(ctx), "record")
    if not d:
        raise ValueError("lb_step_record needs a device buffer")
    _check(library().lb_step_record(ctx, p), "lb_step_record")


def lb_adjoint_step_record(ctx, record) -> None:
    p, d = _raw(record, lb_record_bytes(ctx), "record")
    if not d:
        raise ValueError("lb_adjoint_step_record needs a device buffer")
    _check(library().lb_adjoint_step_record(ctx, p), "lb_adjoint_step_record")


def lb_device_bytes(ctx) -> int:
    b = ctypes.c_int64(0)
    _check(library().lb_device_bytes(ctx, ctypes.byref(b)), "lb_device_bytes")
    return b.value


def lb_snapshot_totals(params: lb_params, snapshot, out, solid=None) -> int:
    """Totals of a device snapshot into ``out`` (6 float64: host or device);
    returns the status (LB_OK, or LB_ENONFINITE for a host ``out``)."""
    nbytes = snapshot.numel() * snapshot.element_size() if type(snapshot).__module__.startswith("torch") else -1
    ps, ds = _raw(snapshot, nbytes, "snapshot")
    if not ds:
        raise ValueError("lb_snapshot_totals needs a device snapshot")
    n = int(params.nx) * int(params.ny) * int(params.nz)
    pm, dm = _ptr(solid, "uint8", n, "solid")
    if solid is not None and not dm:
        raise ValueError("lb_snapshot_totals needs a device solid mask")
    po, do = _ptr(out, "float64", 6, "out")
    st = library().lb_snapshot_totals(ctypes.byref(params), ps, pm, po, do)
    if st not in (LB_OK, LB_ENONFINITE):
        _check(st, "lb_snapshot_totals")
    return st


# ---------------------------------------------------------------------------
# Convenience object over one context
# ---------------------------------------------------------------------------
# ---- single-fluid step (the paper's case 1) ---------------------------------
def lb1_create(params: lb_params) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(library().lb1_create(ctypes.byref(params), ctypes.byref(ctx)), "lb1_create")
    return ctx


def lb1_destroy(ctx) -> None:
    _check(library().lb1_destroy(ctx), "lb1_destroy")


def lb1_set_stream(ctx, stream) -> None:
    _check(library().lb1_set_stream(ctx, stream), "lb1_set_stream")


def lb1_set_fields(ctx, n: int, rho, u=None, solid=None) -> None:
    pr, dr = _ptr(rho, "float64", n, "rho")
    pu, du = _ptr(u, "float64", 3 * n, "u")
    ps, ds = _ptr(solid, "uint8", n, "solid")
    on_dev = _same_side(dr, du if u is not None else None, ds if solid is not None else None)
    _check(library().lb1_set_fields(ctx, pr, pu, ps, on_dev), "lb1_set_fields")


def lb1_step(ctx, nsteps: int) -> None:
    _check(library().lb1_step(ctx, int(nsteps)), "lb1_step")


def lb1_moments(ctx, n: int, rho=None, u=None) -> None:
    pr, dr = _ptr(rho, "float64", n, "rho")
    pu, du = _ptr(u, "float64", 3 * n, "u")
    on_dev = _same_side(dr if rho is not None else None, du if u is not None else None)
    _check(library().lb1_moments(ctx, pr, pu, on_dev), "lb1_moments")


def lb1_get_populations(ctx, n: int, f) -> None:
    pf, df = _ptr(f, "float64", Q * n, "f")
    _check(library().lb1_get_populations(ctx, pf, df), "lb1_get_populations")


def lb1_totals(ctx) -> Tuple[Tuple[float, ...], bool]:
    out = (ctypes.c_double * 4)()
    nf = ctypes.c_int(0)
    st = library().lb1_totals(ctx, out, ctypes.byref(nf))
    if st not in (LB_OK, LB_ENONFINITE):
        _check(st, "lb1_totals")
    return tuple(out), bool(nf.value)


def _host3(a, count: int, what: str):
    """Host float64 [count][3] array (copied to C order) or None."""
    import numpy as np

    if a is None:
        return None
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if arr.size != 3 * count:
        raise ValueError(f"{what}: expected {count} x 3 values, got {arr.size}")
    return arr


def _set_particles(name: str, ctx, pos, radius: float, mass: float, vel=None, omega=None) -> None:
    import numpy as np

    fn = getattr(library(), name)
    if pos is None or np.size(pos) == 0:
        _check(fn(ctx, 0, float(radius), float(mass), None, None, None), name)
        return
    count = np.size(pos) // 3
    arrs = [_host3(a, count, w) for a, w in ((pos, "pos"), (vel, "vel"), (omega, "omega"))]
    ptrs = [None if a is None else ctypes.c_void_p(a.ctypes.data) for a in arrs]
    _check(fn(ctx, count, float(radius), float(mass), *ptrs), name)


def _get_particles(name: str, ctx, count: int):
    import numpy as np

    outs = [np.empty((count, 3)) for _ in range(5)]
    _check(getattr(library(), name)(ctx, *[ctypes.c_void_p(o.ctypes.data) for o in outs]), name)
    return tuple(outs)


def lb1_set_particles(ctx, pos, radius: float, mass: float, vel=None, omega=None) -> None:
    """Place rigid spheres (host arrays [P][3]); pos=None or empty removes them."""
    _set_particles("lb1_set_particles", ctx, pos, radius, mass, vel, omega)


def lb1_get_particles(ctx, count: int):
    """(pos, vel, omega, force, torque), each a host float64 array [count][3]."""
    return _get_particles("lb1_get_particles", ctx, count)


def lb_set_particles(ctx, pos, radius: float, mass: float, vel=None, omega=None) -> None:
    """Place rigid spheres in a colour-gradient context (host arrays [P][3]);
    pos=None or empty removes them."""
    _set_particles("lb_set_particles", ctx, pos, radius, mass, vel, omega)


def lb_get_particles(ctx, count: int):
    """(pos, vel, omega, force, torque) of a two-component context's particles."""
    return _get_particles("lb_get_particles", ctx, count)


class SingleFluid:
    """A single-fluid lattice (the paper's case 1) on one GPU: owns an
    lb1_ctx.  ``shape`` is (nz, ny, nx); arrays as for ``Lattice``."""

    def __init__(self, shape, tau=1.0, storage="f64", rho0=1.0, device: int = 0, stream=None):
        nz, ny, nx = (int(s) for s in shape)
        p = lb_params_default()
        p.nx, p.ny, p.nz = nx, ny, nz
        p.tau[0] = float(tau)
        p.rho0[0] = float(rho0)
        p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        p.device = int(device)
        p.stream = stream if stream is not None else _current_stream(device)
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        self.nparticles = 0
        self.ctx = lb1_create(p)

    def close(self):
        if self.ctx is not None and self.ctx.value is not None:
            lb1_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_fields(self, rho, u=None, solid=None):
        lb1_set_fields(self.ctx, self.n, rho, u, solid)
        self.nparticles = 0  # new fields drop the particles

    def step(self, nsteps: int = 1):
        lb1_step(self.ctx, nsteps)

    def moments(self, rho=None, u=None):
        lb1_moments(self.ctx, self.n, rho, u)

    def get_populations(self, f):
        lb1_get_populations(self.ctx, self.n, f)

    def totals(self):
        return lb1_totals(self.ctx)

    def set_particles(self, pos, radius: float, mass: float, vel=None, omega=None):
        import numpy as np

        lb1_set_particles(self.ctx, pos, radius, mass, vel, omega)
        self.nparticles = 0 if pos is None else int(np.size(pos) // 3)

    def particles(self):
        """(pos, vel, omega, force, torque) of the particles, host [P][3] each."""
        return lb1_get_particles(self.ctx, self.nparticles)


class Lattice:
    """One lattice on one GPU: owns an lb_ctx and forwards to the C entry points.

    ``shape`` is (nz, ny, nx).  Arrays passed in and out are NumPy (host) or
    torch tensors (host or device), float64, C order [z][y][x].
    """

    def __init__(self, shape, tau=(1.0, 1.0), G=0.0, psi_ref=1.0, storage="f64", rho0=(1.0, 1.0),
                 device: int = 0, stream=None, kernel="auto", model="shan_chen", sigma=0.0, beta=0.0):
        nz, ny, nx = (int(s) for s in shape)
        p = lb_params_default()
        p.nx, p.ny, p.nz = nx, ny, nz
        p.tau[0], p.tau[1] = float(tau[0]), float(tau[1])
        p.G = float(G)
        p.psi_ref = float(psi_ref)
        p.rho0[0], p.rho0[1] = float(rho0[0]), float(rho0[1])
        p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        p.device = int(device)
        p.stream = stream if stream is not None else _current_stream(device)
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        self.params = p
        self.nparticles = 0
        self.ctx = lb_create(p)
        try:
            lb_set_kernel(self.ctx, kernel)
            lb_set_model(self.ctx, model, sigma, beta)
        except Exception:
            self.close()
            raise

    def close(self):
        if self.ctx is not None and self.ctx.value is not None:
            lb_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_fields(self, rho_a, rho_b, u=None, solid=None):
        lb_set_fields(self.ctx, self.n, rho_a, rho_b, u, solid)
        self.nparticles = 0  # new fields drop the particles

    def step(self, nsteps: int = 1):
        lb_step(self.ctx, nsteps)

    def moments(self, rho_a=None, rho_b=None, u=None):
        lb_moments(self.ctx, self.n, rho_a, rho_b, u)

    def get_populations(self, f):
        lb_get_populations(self.ctx, self.n, f)

    def set_populations(self, f):
        lb_set_populations(self.ctx, self.n, f)

    def totals(self):
        return lb_totals(self.ctx)

    def set_particles(self, pos, radius: float, mass: float, vel=None, omega=None):
        """Rigid spheres in the colour-gradient fluid (host arrays [P][3]);
        pos=None removes them."""
        import numpy as np

        lb_set_particles(self.ctx, pos, radius, mass, vel, omega)
        self.nparticles = 0 if pos is None else int(np.size(pos) // 3)

    def particles(self):
        """(pos, vel, omega, force, torque) of the particles, host [P][3] each."""
        return lb_get_particles(self.ctx, self.nparticles)
