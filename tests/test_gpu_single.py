"""Parity of the single-fluid HIP step (lb1_* through the C ABI) with the FP64
single-fluid oracle (the paper's case 1).

float64 follows the oracle's operation order and is held to bit equality;
float32 and float16-shifted storage to bounds from their precision.
"""

import sys

import numpy as np
import pytest

import paper_2112_08264_amd as P
from oracle import lb_oracle as O
from oracle import lb_single as S
import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _init(shape, seed, amp=0.05, vel=0.05):
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-amp, amp, shape)
    u = tuple(rng.uniform(-vel, vel, shape) for _ in range(3))
    return rho, u


def run_gpu(shape, tau, rho, u, steps, solid=None, storage="f64"):
    torch = _torch()
    n = int(np.prod(shape))
    with P.SingleFluid(shape, tau=tau, storage=storage) as lat:
        uu = None if u is None else np.ascontiguousarray(np.stack(u).reshape(-1))
        lat.set_fields(np.ascontiguousarray(rho.reshape(-1)), uu,
                       None if solid is None else np.ascontiguousarray(solid.reshape(-1).astype(np.uint8)))
        lat.step(steps)
        f = torch.empty(19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(f)
        torch.cuda.synchronize()
        return f.cpu().numpy().reshape((19,) + tuple(shape))


@pytest.mark.parametrize("shape", [(4, 4, 4), (5, 6, 7), (3, 1, 9), (1, 1, 1), (9, 17, 64), (2, 9, 300)])
def test_f64_single_fluid_bitwise_equal_to_oracle(shape):
    _say(f"case single f64 bitwise shape={shape}")
    rho, u = _init(shape, 31)
    ref = S.step(S.init_equilibrium(rho, u), 0.7, n=5)
    got = run_gpu(shape, 0.7, rho, u, 5)
    assert np.array_equal(got, ref)


def test_f64_single_fluid_with_solids_bitwise():
    shape = (12, 14, 40)
    _say(f"case single f64 solids shape={shape}")
    centres = synth.sphere_centres(shape, 4, 2.5, 35)
    solid = synth.solid_mask(shape, centres, 2.5)
    rho, u = _init(shape, 36)
    ref = S.step(S.init_equilibrium(rho, u, solid), 0.9, solid, n=30)
    got = run_gpu(shape, 0.9, rho, u, 30, solid=solid)
    assert np.array_equal(got, ref)
    assert np.all(got[:, solid.astype(bool)] == 0.0)


def test_single_fluid_moments_and_totals():
    torch = _torch()
    shape = (6, 7, 8)
    n = int(np.prod(shape))
    _say(f"case single moments/totals shape={shape}")
    rho, u = _init(shape, 37)
    f = S.step(S.init_equilibrium(rho, u), 0.8, n=7)
    want_rho, want_u = S.moments(f)
    (wM, *wP), _ = S.totals(f)
    with P.SingleFluid(shape, tau=0.8) as lat:
        lat.set_fields(rho.ravel().copy(), np.stack(u).reshape(-1).copy())
        lat.step(7)
        r, uu = np.empty(n), np.empty(3 * n)
        lat.moments(r, uu)
        np.testing.assert_array_equal(r, want_rho.ravel())
        np.testing.assert_array_equal(uu.reshape(3, -1), np.stack(want_u).reshape(3, -1))
        dr = torch.empty(n, dtype=torch.float64, device="cuda")
        lat.moments(rho=dr)
        assert np.array_equal(dr.cpu().numpy(), r)
        (M, *Pm), nonfinite = lat.totals()
        assert not nonfinite
        assert abs(M - wM) <= 1e-14 * wM
        for a in range(3):
            assert abs(Pm[a] - wP[a]) <= 1e-14 * wM


# bounds: float32 rounds each stored population to 2^-24 relative, a few
# ulps of a density near 1 per step, over 100 steps at most ~3e-5; float16
# keeps 11 bits of |f - w_i rho0| (about 0.1 w_i here), the bound used for
# the two-component form
@pytest.mark.parametrize("storage,bound", [("f32", 3e-5), ("f16s", 2e-3)])
def test_single_fluid_reduced_storage_error_against_oracle(storage, bound):
    torch = _torch()
    shape = (32, 32, 32)
    n = int(np.prod(shape))
    _say(f"case single {storage} vs oracle, 100 steps")
    rho, u = _init(shape, 38, amp=0.02, vel=0.03)
    ref = S.step(S.init_equilibrium(rho, u), 0.9, n=100)
    want_rho, _ = S.moments(ref)
    with P.SingleFluid(shape, tau=0.9, storage=storage) as lat:
        lat.set_fields(rho.ravel().copy(), np.stack(u).reshape(-1).copy())
        lat.step(100)
        r = torch.empty(n, dtype=torch.float64, device="cuda")
        lat.moments(rho=r)
        err = float(np.max(np.abs(r.cpu().numpy() - want_rho.ravel())))
    _say(f"  max |drho| {err:.2e} (bound {bound:.0e})")
    assert err <= bound


def test_single_fluid_error_paths():
    with P.SingleFluid((4, 4, 4)) as lat:
        with pytest.raises(P.LBError) as e:
            lat.step(1)
        assert e.value.status == P.LB_ESTATE
        bad = np.ones(64)
        bad[5] = np.nan
        with pytest.raises(P.LBError) as e:
            lat.set_fields(bad)
        assert e.value.status == P.LB_EINVAL
        lat.set_fields(np.ones(64))
        with pytest.raises(P.LBError):
            lat.step(-1)


def test_full_size_single_fluid_sampled_one_step():
    """The single-fluid benchmark lattice (256^3, float32, in the launch
    configuration the benchmark times): after 20 GPU steps, one more GPU step
    at sampled nodes against the float64 oracle stepped on a 5^3 block of the
    exported state (one step at the centre needs nodes within distance 1).
    Bound: float32 arithmetic and storage rounding, 1e-5 w_i."""
    torch = _torch()
    w = synth.WORKLOADS["case1_256_f32"]
    shape, n = w.shape, w.nodes
    _say(f"case {w.name} sampled one-step parity")
    rho, _ = synth.fluid_fields(shape, w.amp, w.seed)
    sites = [tuple(int(v) for v in s) for s in synth.sample_sites(shape, 16, 81)]
    with P.SingleFluid(shape, tau=w.tau[0], storage=w.storage) as lat:
        lat.set_fields(rho.ravel().copy())
        lat.step(20)
        f = torch.empty(19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(f)
        f4 = f.view(19, *shape)
        blocks = []
        for (x, y, z) in sites:
            zi = torch.tensor([(z + d) % shape[0] for d in range(-2, 3)], device="cuda")
            yi = torch.tensor([(y + d) % shape[1] for d in range(-2, 3)], device="cuda")
            xi = torch.tensor([(x + d) % shape[2] for d in range(-2, 3)], device="cuda")
            blocks.append(f4.index_select(1, zi).index_select(2, yi).index_select(3, xi).cpu().numpy())
        lat.step(1)
        lat.get_populations(f)
        got = [f4[:, z, y, x].cpu().numpy() for (x, y, z) in sites]
    for (x, y, z), blk, g in zip(sites, blocks, got):
        want = S.step(blk, w.tau[0])[:, 2, 2, 2]
        assert np.max(np.abs(g - want) / (1e-5 * O.W)) <= 1.0, (x, y, z)
