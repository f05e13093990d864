"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad parameters before touching a device."""

import ctypes
import os
import re

import pytest

import paper_2112_08264_amd as P
from paper_2112_08264_amd import lb as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lb.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb1?_[a-z_0-9]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = P.library()
    names = declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    # the binding wraps exactly the declared entry points
    assert sorted(L.SYMBOLS) == names


def test_abi_version_and_params_layout():
    assert P.lb_abi_version() == 1
    # lb_params as C lays it out: 3 int32, pad, 2 double, 2 double, 2 double, 2 int32, pointer
    assert ctypes.sizeof(P.lb_params) == 4 * 3 + 4 + 8 * 2 + 8 + 8 + 8 * 2 + 4 * 2 + 8
    p = P.lb_params_default()
    assert (p.nx, p.ny, p.nz) == (1, 1, 1)
    assert tuple(p.tau) == (1.0, 1.0) and p.psi_ref == 1.0 and p.storage == P.LB_F64


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("ny", -3), ("nz", 0),
    ("tau", (0.5, 1.0)), ("tau", (1.0, 0.2)), ("tau", (float("nan"), 1.0)),
    ("psi_ref", 0.0), ("psi_ref", float("inf")), ("G", float("nan")), ("storage", 7),
])
def test_create_rejects_bad_parameters_without_a_device(field, value):
    p = P.lb_params_default()
    if field == "tau":
        p.tau[0], p.tau[1] = value
    else:
        setattr(p, field, value)
    with pytest.raises(P.LBError) as e:
        P.lb_create(p)
    assert e.value.status == P.LB_EINVAL


def test_create_rejects_oversized_lattice():
    p = P.lb_params_default()
    p.nx, p.ny, p.nz = 2048, 2048, 1024  # 2^32 nodes: beyond the 32-bit node index
    with pytest.raises(P.LBError) as e:
        P.lb_create(p)
    assert e.value.status == P.LB_EINVAL


def test_null_arguments_are_rejected():
    lib = P.library()
    assert lib.lb_create(None, None) == P.LB_EINVAL
    out = ctypes.c_void_p()
    assert lib.lb_create(None, ctypes.byref(out)) == P.LB_EINVAL
    assert out.value is None
    assert lib.lb_step(None, 1) == P.LB_EINVAL
    assert lib.lb_set_fields(None, None, None, None, None, 0) == P.LB_EINVAL
    assert lib.lb_moments(None, None, None, None, 0) == P.LB_EINVAL
    assert lib.lb_totals(None, None, None) == P.LB_EINVAL
    assert lib.lb_get_populations(None, None, 0) == P.LB_EINVAL
    assert lib.lb_set_populations(None, None, 0) == P.LB_EINVAL
    assert lib.lb_set_model(None, P.LB_MODEL_COLOUR_GRADIENT, 0.01, 0.7) == P.LB_EINVAL
    assert lib.lb_destroy(None) == P.LB_OK


def test_strerror_covers_every_status():
    for s in (P.LB_OK, P.LB_EINVAL, P.LB_ENOMEM, P.LB_EDEVICE, P.LB_ESTATE, P.LB_ENONFINITE):
        assert P.lb_strerror(s) and P.lb_strerror(s) != "unknown status"
    assert P.lb_strerror(42) == "unknown status"


def test_timing_slot_names():
    names = [P.lb_timing_name(i) for i in range(P.lb_timing_slots())]
    assert all(names) and len(set(names)) == len(names)
    assert P.lb_timing_name(P.lb_timing_slots()) is None


@pytest.mark.parametrize("field,value", [("nx", 0), ("nz", -1), ("storage", 9)])
def test_single_fluid_create_rejects_bad_parameters_without_a_device(field, value):
    p = P.lb_params_default()
    setattr(p, field, value)
    ctx = ctypes.c_void_p()
    assert P.library().lb1_create(ctypes.byref(p), ctypes.byref(ctx)) == P.LB_EINVAL
    assert ctx.value is None


def test_single_fluid_create_rejects_tau_at_or_below_one_half():
    p = P.lb_params_default()
    p.tau[0] = 0.5
    ctx = ctypes.c_void_p()
    assert P.library().lb1_create(ctypes.byref(p), ctypes.byref(ctx)) == P.LB_EINVAL


def test_single_fluid_calls_reject_null_context():
    lib = P.library()
    assert lib.lb1_step(None, 1) == P.LB_EINVAL
    assert lib.lb1_set_particles(None, 1, 2.0, 10.0, None, None, None) == P.LB_EINVAL
    assert lib.lb1_get_particles(None, None, None, None, None, None) == P.LB_EINVAL
    assert lib.lb1_destroy(None) == P.LB_OK



def test_snapshot_totals_rejects_bad_arguments_without_a_device():
    lib = P.library()
    buf = (ctypes.c_double * 8)()
    p = P.lb_params_default()
    out = (ctypes.c_double * 6)()
    assert lib.lb_snapshot_totals(None, buf, None, out, 0) == P.LB_EINVAL
    assert lib.lb_snapshot_totals(ctypes.byref(p), None, None, out, 0) == P.LB_EINVAL
    assert lib.lb_snapshot_totals(ctypes.byref(p), buf, None, None, 0) == P.LB_EINVAL
    for field, value in (("nx", 0), ("nz", -1), ("storage", 9)):
        q = P.lb_params_default()
        setattr(q, field, value)
        assert lib.lb_snapshot_totals(ctypes.byref(q), buf, None, out, 0) == P.LB_EINVAL, field
    q = P.lb_params_default()
    q.nx, q.ny, q.nz = 2048, 2048, 1024  # beyond the 32-bit node index
    assert lib.lb_snapshot_totals(ctypes.byref(q), buf, None, out, 0) == P.LB_EINVAL
    q = P.lb_params_default()
    q.storage = P.LB_F16_SHIFTED
    q.rho0[0] = float("nan")
    assert lib.lb_snapshot_totals(ctypes.byref(q), buf, None, out, 0) == P.LB_EINVAL
