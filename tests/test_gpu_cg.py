"""Parity of the colour-gradient HIP step (lb_set_model with
LB_MODEL_COLOUR_GRADIENT, through the C ABI) with the FP64 colour-gradient
oracle (the paper's two-component model, Appendix; case 2 of Sec. 5).

float64 follows the oracle's operation order and is held to bit equality;
float32 to bounds from its precision.
"""

import sys

import numpy as np
import pytest

import paper_2112_08264_amd as P
from oracle import lb_cg as CG
import synth

pytestmark = pytest.mark.gpu

PAR = CG.Params((0.8, 1.1), 0.02, 0.7)


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mixed(shape, seed, amp=0.3, vel=0.03):
    rng = np.random.default_rng(seed)
    r1 = 0.5 + rng.uniform(-amp, amp, shape)
    u = [rng.uniform(-vel, vel, shape) for _ in range(3)]
    return r1, 1.0 - r1, u


def _lattice(shape, p, storage="f64", kernel="auto"):
    return P.Lattice(shape, tau=p.tau, storage=storage, kernel=kernel, model="colour_gradient", sigma=p.sigma,
                     beta=p.beta)


def run_gpu(shape, p, r1, r2, steps, u=None, storage="f64", kernel="auto"):
    torch = _torch()
    n = int(np.prod(shape))
    with _lattice(shape, p, storage, kernel) as lat:
        uu = None if u is None else np.ascontiguousarray(np.stack(u).reshape(-1))
        lat.set_fields(np.ascontiguousarray(r1.reshape(-1)), np.ascontiguousarray(r2.reshape(-1)), uu)
        lat.step(steps)
        f = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(f)
        torch.cuda.synchronize()
        return f.cpu().numpy().reshape((2, 19) + tuple(shape))


# (9, 17, 64): staged 64 x 4 tiles; (5, 8, 64) and (3, 12, 128): the same on the
# tile-major layout (ny a multiple of 4); (8, 12, 32): staged 32 x 8; the others
# unstaged, with ragged tiles
@pytest.mark.parametrize("kernel", ["fused", "fused_staged"])
@pytest.mark.parametrize("shape", [(4, 4, 4), (5, 6, 7), (3, 1, 9), (1, 1, 1), (9, 17, 64), (5, 8, 64), (3, 12, 128),
                                   (8, 12, 32), (2, 9, 300)])
def test_f64_colour_gradient_bitwise_equal_to_oracle(shape, kernel):
    _say(f"case cg f64 bitwise shape={shape} kernel={kernel}")
    r1, r2, u = _mixed(shape, 41)
    ref = CG.step(CG.init_equilibrium(r1, r2, u), PAR, n=5)
    got = run_gpu(shape, PAR, r1, r2, 5, u=u, kernel=kernel)
    assert np.array_equal(got, ref)


def test_f64_case2_pure_nodes_bitwise_over_z_chunks():
    """The paper's case-2 start (every node pure red or pure blue, so rho_k = 0
    at half the nodes) on 64^3, where z is split into chunks of 4 planes."""
    shape = (64, 64, 64)
    _say(f"case cg f64 case-2 start shape={shape}")
    r1, r2 = synth.colour_fields(shape, 42)
    ref = CG.step(CG.init_equilibrium(r1, r2), PAR, n=3)
    got = run_gpu(shape, PAR, r1, r2, 3)
    assert np.array_equal(got, ref)


def test_f64_case2_32_workload_200_steps_bitwise():
    w = synth.WORKLOADS["case2_32_f64"]
    _say(f"case {w.name}")
    p = CG.Params(w.tau, w.sigma, w.beta)
    r1, r2 = synth.colour_fields(w.shape, w.seed)
    ref = CG.step(CG.init_equilibrium(r1, r2), p, n=w.steps)
    got = run_gpu(w.shape, p, r1, r2, w.steps)
    _say(f"  bit-identical fraction {np.mean(got == ref):.6f}")
    assert np.array_equal(got, ref)


def test_colour_gradient_moments_and_totals():
    torch = _torch()
    shape = (6, 7, 8)
    n = int(np.prod(shape))
    _say(f"case cg moments/totals shape={shape}")
    r1, r2, u = _mixed(shape, 43)
    f0 = CG.init_equilibrium(r1, r2, u)
    f = CG.step(f0, PAR, n=7)
    w1, w2, wu = CG.moments(f)
    (M1, M2, *_), _ = CG.totals(f0)
    with _lattice(shape, PAR) as lat:
        lat.set_fields(r1.ravel().copy(), r2.ravel().copy(), np.stack(u).reshape(-1).copy())
        lat.step(7)
        a, b, uu = np.empty(n), np.empty(n), np.empty(3 * n)
        lat.moments(a, b, uu)
        np.testing.assert_array_equal(a, w1.ravel())
        np.testing.assert_array_equal(b, w2.ravel())
        np.testing.assert_array_equal(uu.reshape(3, -1), np.stack(wu).reshape(3, -1))
        (N1, N2, *_), nonfinite = lat.totals()
        assert not nonfinite
        assert abs(N1 - M1) <= 1e-13 * M1 and abs(N2 - M2) <= 1e-13 * M2


# (24, 24, 32): structure of arrays; (6, 12, 64): the tile-major layout
@pytest.mark.parametrize("shape", [(24, 24, 32), (6, 12, 64)])
def test_f32_one_step_from_an_oracle_state(shape):
    """One float32 step from a state the float64 oracle has demixed for 40 steps
    (loaded by lb_set_populations, one rounding to float32): every population
    within 2e-6 of the oracle's next step.  Bound: float32 rounds each value to
    2^-24 relative; one step chains about twenty roundings of values below 0.5
    plus the rounding of the loaded state, and the interface terms of nodes
    near |grad Theta| = 0 carry the same relative error."""
    torch = _torch()
    n = int(np.prod(shape))
    _say(f"case cg f32 one step shape={shape}")
    f = CG.step(CG.init_equilibrium(*synth.colour_fields(shape, 44)), PAR, n=40)
    want = CG.step(f, PAR)
    with _lattice(shape, PAR, storage="f32") as lat:
        lat.set_fields(np.ones(n), np.ones(n))
        lat.set_populations(np.ascontiguousarray(f.reshape(-1)))
        lat.step(1)
        g = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(g)
        got = g.cpu().numpy().reshape(f.shape)
    err = float(np.max(np.abs(got - want)))
    _say(f"  max |df| {err:.2e}")
    assert err <= 2e-6


def test_f32_trajectory_error_against_oracle():
    """float32 over 50 steps from a smoothly mixed state: the density error
    stays at the float32 rounding level amplified by the flow, <= 1e-4."""
    torch = _torch()
    shape = (32, 32, 32)
    n = int(np.prod(shape))
    _say(f"case cg f32 vs oracle, 50 steps")
    r1, r2, u = _mixed(shape, 45, amp=0.3, vel=0.02)
    ref = CG.step(CG.init_equilibrium(r1, r2, u), PAR, n=50)
    w1, w2, _ = CG.moments(ref)
    with _lattice(shape, PAR, storage="f32") as lat:
        lat.set_fields(r1.ravel().copy(), r2.ravel().copy(), np.stack(u).reshape(-1).copy())
        lat.step(50)
        a = torch.empty(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        lat.moments(a, b)
        err = max(float(np.max(np.abs(a.cpu().numpy() - w1.ravel()))),
                  float(np.max(np.abs(b.cpu().numpy() - w2.ravel()))))
    _say(f"  max |drho| {err:.2e}")
    assert err <= 1e-4


def test_colour_gradient_error_paths():
    n = 64
    with pytest.raises(P.LBError) as e:
        P.Lattice((4, 4, 4), storage="f16s", model="colour_gradient", sigma=0.01, beta=0.7)
    assert e.value.status == P.LB_EINVAL
    for sigma, beta in ((-0.1, 0.7), (0.01, -1.0), (float("nan"), 0.7), (0.01, float("inf"))):
        with pytest.raises(P.LBError):
            P.Lattice((4, 4, 4), model="colour_gradient", sigma=sigma, beta=beta)
    with _lattice((4, 4, 4), PAR) as lat:
        with pytest.raises(P.LBError) as e:
            P.lb_set_model(lat.ctx, 7)
        assert e.value.status == P.LB_EINVAL
        # solids are not part of this model
        with pytest.raises(P.LBError) as e:
            lat.set_fields(np.ones(n), np.ones(n), None, np.zeros(n, dtype=np.uint8))
        assert e.value.status == P.LB_EINVAL
        # the phase field needs rho_A + rho_B > 0 everywhere
        a, b = np.ones(n), np.ones(n)
        a[5] = b[5] = 0.0
        with pytest.raises(P.LBError) as e:
            lat.set_fields(a, b)
        assert e.value.status == P.LB_EINVAL
        lat.set_fields(np.full(n, 0.7), np.full(n, 0.3))
        # the adjoint and the two-pass step are Shan-Chen only
        with pytest.raises(P.LBError) as e:
            P.lb_adjoint_begin(lat.ctx, n)
        assert e.value.status == P.LB_EINVAL
        P.lb_set_kernel(lat.ctx, "two_pass")
        with pytest.raises(P.LBError) as e:
            lat.step(1)
        assert e.value.status == P.LB_EINVAL
        P.lb_set_kernel(lat.ctx, "auto")
        lat.step(1)


def test_model_switch_back_to_shan_chen_runs_the_shan_chen_step():
    from oracle import lb_oracle as O
    torch = _torch()
    shape = (5, 6, 7)
    n = int(np.prod(shape))
    a, b = synth.fluid_fields(shape, 0.1, 46)
    p = O.Params((0.8, 1.1), 3.5)
    ref = O.step(O.init_equilibrium(a, b), p, n=3)
    with P.Lattice(shape, tau=p.tau, G=p.G, model="colour_gradient", sigma=0.02, beta=0.7) as lat:
        P.lb_set_model(lat.ctx, "shan_chen")
        lat.set_fields(a.ravel().copy(), b.ravel().copy())
        lat.step(3)
        f = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(f)
        got = f.cpu().numpy().reshape(ref.shape)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("name", ["case2_256_f32", "case2_256_f64"])
def test_full_size_case2_sampled_one_step(name):
    """The case-2 benchmark lattice (256^3, in the launch configuration the
    benchmark times): after 20 GPU steps, one more GPU step at sampled nodes
    against the float64 oracle stepped on a 5^3 block of the exported state
    (one step at the centre needs the phase field within distance 2).
    float64: bit equality; float32: 2e-6 (as the one-step bound above)."""
    torch = _torch()
    w = synth.WORKLOADS[name]
    shape, n = w.shape, w.nodes
    p = CG.Params(w.tau, w.sigma, w.beta)
    _say(f"case {w.name} sampled one-step parity")
    r1, r2 = synth.colour_fields(shape, w.seed)
    sites = [tuple(int(v) for v in s) for s in synth.sample_sites(shape, 16, 82)]
    with _lattice(shape, p, storage=w.storage) as lat:
        lat.set_fields(r1.ravel().copy(), r2.ravel().copy())
        lat.step(20)
        f = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(f)
        f5 = f.view(2, 19, *shape)
        blocks = []
        for (x, y, z) in sites:
            zi = torch.tensor([(z + d) % shape[0] for d in range(-2, 3)], device="cuda")
            yi = torch.tensor([(y + d) % shape[1] for d in range(-2, 3)], device="cuda")
            xi = torch.tensor([(x + d) % shape[2] for d in range(-2, 3)], device="cuda")
            blocks.append(f5.index_select(2, zi).index_select(3, yi).index_select(4, xi).cpu().numpy())
        lat.step(1)
        lat.get_populations(f)
        got = [f5[:, :, z, y, x].cpu().numpy() for (x, y, z) in sites]
    for (x, y, z), blk, g in zip(sites, blocks, got):
        want = CG.step(blk, p)[:, :, 2, 2, 2]
        if w.storage == "f64":
            assert np.array_equal(g, want), (x, y, z)
        else:
            assert np.max(np.abs(g - want)) <= 2e-6, (x, y, z)
