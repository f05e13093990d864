"""lb_snapshot_totals, the entry point that allocates nothing, against lb_totals.

Both run the same reduction kernels in the same order, so the totals of a
device snapshot must equal the context's totals of the same state bit for
bit.  The entry point keeps its partial sums in a fixed device array shared
by every call on the GPU: two calls in a row, the second on a smaller
lattice (fewer partials than the first left behind), must both be right.
"""

import sys

import numpy as np
import pytest

import paper_2112_08264_amd as P
import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _state(shape, storage, with_solid, seed, steps=5):
    """A context stepped a few times, its device snapshot and its device mask (or None)."""
    torch = _torch()
    a, b = synth.fluid_fields(shape, 0.05, seed)
    solid = None
    if with_solid:
        nz, ny, nx = shape
        centre = np.array([[nx / 2 + 0.3, ny / 2 - 0.2, nz / 2 + 0.1]])
        solid = synth.solid_mask(shape, centre, min(shape) / 4 + 0.5).astype(np.uint8)
    lat = P.Lattice(shape, tau=(0.8, 1.0), G=3.5, storage=storage)
    lat.set_fields(a.reshape(-1).copy(), b.reshape(-1).copy(), None,
                   None if solid is None else solid.reshape(-1).copy())
    lat.step(steps)
    snap = torch.empty(P.lb_state_bytes(lat.ctx), dtype=torch.uint8, device="cuda")
    P.lb_save_state(lat.ctx, snap)
    mask = None if solid is None else torch.from_numpy(solid.reshape(-1).copy()).cuda()
    torch.cuda.synchronize()
    return lat, snap, mask


def _check_against_context(lat, snap, mask):
    torch = _torch()
    ref, nonfinite = lat.totals()
    assert not nonfinite
    host = np.full(6, np.nan)
    st = P.lb_snapshot_totals(lat.params, snap, host, mask)
    assert st == P.LB_OK
    assert tuple(host[:5]) == tuple(ref), (host[:5], ref)
    assert host[5] == 0.0
    dev = torch.full((6,), float("nan"), dtype=torch.float64, device="cuda")
    assert P.lb_snapshot_totals(lat.params, snap, dev, mask) == P.LB_OK
    torch.cuda.synchronize()
    got = dev.cpu().numpy()
    assert tuple(got[:5]) == tuple(ref) and got[5] == 0.0


def test_snapshot_totals_equal_context_totals_on_two_calls_second_smaller():
    # first call: 16 x 20 x 64 float64 (the step keeps a tile-major state;
    # the device snapshot is in the structure of arrays), 1 workgroup per
    # 256 nodes -> 80 partials
    _say("case no-alloc totals: 16x20x64 f64, then 5x7x9 f16s with a sphere")
    lat, snap, mask = _state((16, 20, 64), "f64", False, 31)
    try:
        _check_against_context(lat, snap, mask)
    finally:
        lat.close()
    # second call, smaller: 315 nodes -> 2 partials; the array still holds
    # the first call's 80
    lat, snap, mask = _state((5, 7, 9), "f16s", True, 32)
    try:
        _check_against_context(lat, snap, mask)
    finally:
        lat.close()


def test_snapshot_totals_flag_a_non_finite_population():
    torch = _torch()
    _say("case no-alloc totals: non-finite population, 6x8x10 f32")
    lat, snap, mask = _state((6, 8, 10), "f32", False, 33)
    try:
        npad = (6 * 8 * 10 + 127) // 128 * 128
        snap.view(torch.float32)[3 * npad + 5] = float("inf")  # population plane 3, node 5
        host = np.zeros(6)
        assert P.lb_snapshot_totals(lat.params, snap, host, mask) == P.LB_ENONFINITE
        assert host[5] == 1.0
        P.lb_restore_state(lat.ctx, snap)
        _, nonfinite = lat.totals()
        assert nonfinite
    finally:
        lat.close()


def test_snapshot_totals_reject_an_oversized_lattice():
    torch = _torch()
    p = P.lb_params_default()
    p.nx, p.ny, p.nz = 2048, 2048, 1024  # 2^32 nodes
    snap = torch.zeros(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.LBError) as e:
        P.lb_snapshot_totals(p, snap, np.zeros(6))
    assert e.value.status == P.LB_EINVAL
