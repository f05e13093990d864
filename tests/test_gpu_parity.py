"""Parity of the HIP step (through the C ABI) with the FP64 CPU oracle.

The float64 path is designed to perform the oracle's IEEE operations in the
oracle's order, so it is held to bit equality on short runs and to the
1e-12 relative-per-population bar (oracle.population_error) on the 200-step
32^3 workload.  float32 and float16-shifted storage are held to error bounds
derived from their precision.
"""

import os
import sys

import numpy as np
import pytest

import paper_2112_08264_amd as P
from oracle import lb_oracle as O
from oracle import naive as N
import synth

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-12


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


KERNELS = ["fused", "two_pass", "fused_staged"]


def run_gpu(shape, tau, G, rho_a, rho_b, steps, u=None, solid=None, storage="f64", kernel="fused"):
    """Run ``steps`` steps through the C ABI and return the float64 populations [2][19][z][y][x]."""
    torch = _torch()
    n = int(np.prod(shape))
    with P.Lattice(shape, tau=tau, G=G, storage=storage, kernel=kernel) as lat:
        uu = None if u is None else np.ascontiguousarray(np.stack(u).reshape(-1))
        lat.set_fields(np.ascontiguousarray(rho_a.reshape(-1)), np.ascontiguousarray(rho_b.reshape(-1)), uu,
                       None if solid is None else np.ascontiguousarray(solid.reshape(-1).astype(np.uint8)))
        lat.step(steps)
        f = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(f)
        torch.cuda.synchronize()
        return f.cpu().numpy().reshape((2, 19) + tuple(shape))


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("shape", [(4, 4, 4), (5, 6, 7), (3, 1, 9), (1, 1, 1), (11, 19, 45), (9, 17, 64)])
def test_f64_bitwise_equal_to_oracle_on_small_and_ragged_boxes(shape, kernel):
    _say(f"case f64 bitwise shape={shape} kernel={kernel}")
    a, b = synth.fluid_fields(shape, 0.2, 21)
    rng = np.random.default_rng(22)
    u = [rng.uniform(-0.05, 0.05, shape) for _ in range(3)]
    p = O.Params((0.8, 1.3), 3.5)
    ref = O.step(O.init_equilibrium(a, b, u), p, n=5)
    got = run_gpu(shape, p.tau, p.G, a, b, 5, u=u, kernel=kernel)
    assert O.population_error(got, ref) <= TOL_F64
    assert np.array_equal(got, ref), "float64 path is meant to reproduce the oracle bit for bit"


@pytest.mark.parametrize("kernel", KERNELS)
def test_f64_mix32_200_steps_within_1e12(kernel):
    w = synth.WORKLOADS["mix32_f64"]
    _say(f"case {w.name} kernel={kernel}")
    a, b = synth.fluid_fields(w.shape, w.amp, w.seed)
    p = O.Params(w.tau, w.G)
    ref = O.step(O.init_equilibrium(a, b), p, n=w.steps)
    got = run_gpu(w.shape, w.tau, w.G, a, b, w.steps, kernel=kernel)
    err = O.population_error(got, ref)
    _say(f"  population error {err:.3e}, bit-identical fraction {np.mean(got == ref):.6f}")
    assert err <= TOL_F64
    # the run has demixed, so the comparison is not of a near-uniform field
    assert np.ptp(O.density(ref[0])) > 0.5


@pytest.mark.parametrize("kernel", KERNELS)
def test_f64_solids_match_oracle(kernel):
    shape = (12, 14, 40)
    _say(f"case f64 solids shape={shape} kernel={kernel}")
    centres = synth.sphere_centres(shape, 4, 2.5, 31)
    solid = synth.solid_mask(shape, centres, 2.5)
    assert 0 < solid.sum() < solid.size
    a, b = synth.fluid_fields(shape, 0.02, 32)
    p = O.Params((1.0, 0.9), 3.5)
    ref = O.step(O.init_equilibrium(a, b, solid=solid), p, solid, n=40)
    got = run_gpu(shape, p.tau, p.G, a, b, 40, solid=solid, kernel=kernel)
    assert O.population_error(got, ref) <= TOL_F64
    assert np.array_equal(got, ref)
    assert np.all(got[:, :, solid.astype(bool)] == 0.0)


# The staged kernel runs when nx is a multiple of 32, on 64 x 4 tiles when nx
# is a multiple of 64 (other shapes fall back to the plain fused kernel):
# rows past a short y extent, a single plane, several tiles along x, chunks
# of one plane, for both tile shapes.
@pytest.mark.parametrize("shape", [(4, 4, 32), (3, 5, 32), (1, 1, 32), (2, 9, 96), (69, 3, 32),
                                   (5, 8, 64), (3, 3, 64), (1, 1, 64), (2, 9, 192), (69, 5, 64)])
def test_f64_staged_kernel_bitwise_equal_to_oracle(shape):
    _say(f"case f64 staged bitwise shape={shape}")
    a, b = synth.fluid_fields(shape, 0.2, 23)
    rng = np.random.default_rng(24)
    u = [rng.uniform(-0.05, 0.05, shape) for _ in range(3)]
    p = O.Params((0.8, 1.3), 3.5)
    ref = O.step(O.init_equilibrium(a, b, u), p, n=4)
    got = run_gpu(shape, p.tau, p.G, a, b, 4, u=u, kernel="fused_staged")
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("shape", [(128, 2048, 32), (128, 1024, 64)])
def test_f64_tiling_with_several_rounds_of_workgroups_bitwise(shape):
    """A lattice with as many 32 x 8 (or 64 x 4) columns as the GPU has
    compute units (256): the columns are cut into 64-plane chunks and
    numbered round by round; every node must still be stepped exactly once."""
    _say(f"case f64 several rounds of workgroups shape={shape}")
    a, b = synth.fluid_fields(shape, 0.05, 25)
    p = O.Params((0.9, 1.1), 3.5)
    ref = O.step(O.init_equilibrium(a, b), p, n=2)
    got = run_gpu(shape, p.tau, p.G, a, b, 2)
    assert np.array_equal(got, ref)


def test_f64_staged_selection_with_solids_matches_oracle():
    """With solid nodes the staged selection runs the unstaged kernel."""
    shape = (12, 14, 32)
    _say(f"case f64 staged solids shape={shape}")
    centres = synth.sphere_centres(shape, 4, 2.5, 33)
    solid = synth.solid_mask(shape, centres, 2.5)
    assert 0 < solid.sum() < solid.size
    a, b = synth.fluid_fields(shape, 0.02, 34)
    p = O.Params((1.0, 0.9), 3.5)
    ref = O.step(O.init_equilibrium(a, b, solid=solid), p, solid, n=30)
    got = run_gpu(shape, p.tau, p.G, a, b, 30, solid=solid, kernel="fused_staged")
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("with_solid", [False, True])
def test_f64_staged_kernel_moment_record_equals_plain_kernel(with_solid):
    """lb_step_record through the staged kernel writes the same record and
    state as through the plain fused kernel."""
    torch = _torch()
    shape = (9, 10, 64)
    n = int(np.prod(shape))
    _say(f"case staged record solid={with_solid}")
    a, b = synth.fluid_fields(shape, 0.05, 35)
    solid = synth.solid_mask(shape, np.array([[30.0, 5.0, 4.0]]), 2.5).ravel().copy() if with_solid else None
    out = []
    for kernel in ("fused", "fused_staged"):
        with P.Lattice(shape, tau=(0.9, 1.1), G=3.5, kernel=kernel) as lat:
            lat.set_fields(a.ravel().copy(), b.ravel().copy(), None, solid)
            recs = []
            for _ in range(3):
                r = torch.empty(P.lb_record_bytes(lat.ctx), dtype=torch.uint8, device="cuda")
                P.lb_step_record(lat.ctx, r)
                recs.append(r)
            f = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
            lat.get_populations(f)
            torch.cuda.synchronize()
            out.append(([r.cpu() for r in recs], f.cpu()))
    for r0, r1 in zip(out[0][0], out[1][0]):
        assert torch.equal(r0, r1)
    assert torch.equal(out[0][1], out[1][1])


def test_population_roundtrip_and_moments_and_totals():
    torch = _torch()
    shape = (6, 7, 8)
    n = int(np.prod(shape))
    _say(f"case roundtrip/moments/totals shape={shape}")
    a, b = synth.fluid_fields(shape, 0.3, 41)
    f0 = O.step(O.init_equilibrium(a, b), O.Params((0.9, 0.9), 3.5), n=30)
    p = O.Params((0.9, 0.9), 3.5)
    with P.Lattice(shape, tau=p.tau, G=p.G) as lat:
        lat.set_populations(np.ascontiguousarray(f0.reshape(-1)))
        back = np.empty(2 * 19 * n)
        lat.get_populations(back)
        assert np.array_equal(back.reshape(f0.shape), f0)
        ra, rb, u = np.empty(n), np.empty(n), np.empty(3 * n)
        lat.moments(ra, rb, u)
        wa, wb, wu = O.moments(f0, p)
        np.testing.assert_allclose(ra, wa.ravel(), rtol=1e-15)
        np.testing.assert_allclose(rb, wb.ravel(), rtol=1e-15)
        np.testing.assert_allclose(u.reshape(3, -1), np.stack(wu).reshape(3, -1), rtol=1e-13, atol=1e-16)
        # device-side outputs give the same numbers
        dra = torch.empty(n, dtype=torch.float64, device="cuda")
        lat.moments(rho_a=dra)
        assert np.array_equal(dra.cpu().numpy(), ra)
        tot, nonfinite = lat.totals()
        want, wnf = O.totals(f0)
        assert not nonfinite and not wnf
        np.testing.assert_allclose(tot[:2], want[:2], rtol=1e-14)
        np.testing.assert_allclose(tot[2:], want[2:], atol=1e-12)
        # bitwise repeatable reduction
        assert lat.totals()[0] == tot


def test_conservation_on_gpu_over_many_steps():
    shape = (24, 24, 24)
    _say(f"case conservation shape={shape}")
    a, b = synth.fluid_fields(shape, 0.02, 51)
    with P.Lattice(shape, tau=(0.8, 0.8), G=3.5) as lat:
        lat.set_fields(a.ravel().copy(), b.ravel().copy())
        t0, _ = lat.totals()
        lat.step(500)
        t1, nf = lat.totals()
    assert not nf
    assert abs(t1[0] - t0[0]) / t0[0] < 1e-12
    assert abs(t1[1] - t0[1]) / t0[1] < 1e-12
    assert max(abs(v) for v in t1[2:]) / (t0[0] + t0[1]) < 1e-12


# The density target of the reduced storages is max |drho| <= 1e-3 against
# the float64 oracle.  On the 32^3 demixing workload float32 meets it with a
# wide margin after 100 steps; float16-shifted meets it after 10 steps and
# not after 100 (the quench amplifies its per-step storage error of a few
# 1e-6 past the target), so the 100-step row holds float16-shifted to the
# looser bound 2e-3 and says so: that row is not the target.
@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("storage,steps,tol_rho", [("f32", 100, 1e-4), ("f16s", 10, 1e-3), ("f16s", 100, 2e-3)])
def test_reduced_storage_error_against_oracle(storage, steps, tol_rho, kernel):
    w = synth.WORKLOADS["mix32_f64"]
    _say(f"case {storage} vs oracle on {w.name} ({steps} steps) kernel={kernel}")
    a, b = synth.fluid_fields(w.shape, w.amp, w.seed)
    p = O.Params(w.tau, w.G)
    ref = O.step(O.init_equilibrium(a, b), p, n=steps)
    got = run_gpu(w.shape, w.tau, w.G, a, b, steps, storage=storage, kernel=kernel)
    drho = max(np.max(np.abs(O.density(got[k]) - O.density(ref[k]))) for k in range(2))
    _say(f"  max |drho| = {drho:.3e} (bound {tol_rho:.0e})")
    assert drho <= tol_rho


def test_error_paths_on_device():
    torch = _torch()
    shape = (4, 4, 4)
    n = 64
    with P.Lattice(shape, tau=(1.0, 1.0), G=3.5) as lat:
        with pytest.raises(P.LBError) as e:
            lat.step(1)
        assert e.value.status == P.LB_ESTATE
        with pytest.raises(P.LBError) as e:
            P.lb_moments(lat.ctx, n, np.empty(n))
        assert e.value.status == P.LB_ESTATE
        bad = np.ones(n)
        bad[5] = np.nan
        with pytest.raises(P.LBError) as e:
            lat.set_fields(bad, np.ones(n))
        assert e.value.status == P.LB_EINVAL
        neg = np.ones(n)
        neg[3] = -0.5
        with pytest.raises(P.LBError) as e:
            lat.set_fields(np.ones(n), neg)
        assert e.value.status == P.LB_EINVAL
        fbad = np.ones(2 * 19 * n)
        fbad[100] = np.inf
        with pytest.raises(P.LBError) as e:
            lat.set_populations(fbad)
        assert e.value.status == P.LB_EINVAL
        with pytest.raises(P.LBError) as e:
            lat.step(-1)
        assert e.value.status == P.LB_EINVAL
        # a finite state whose momentum is absurd overflows within a step
        # (the velocity squared exceeds the float64 range); totals flag it
        fa = np.ones((2, 19, n))
        fa[0, 1] = 1e200
        fa[0, 2] = -1e200
        lat.set_populations(fa.ravel())
        lat.step(2)
        _, nonfinite = lat.totals()
        assert nonfinite
        # recovers after a valid reset
        lat.set_fields(np.ones(n), np.ones(n))
        lat.step(1)
        assert not lat.totals()[1]


@pytest.mark.slow
def test_full_size_spinodal256_sampled_one_step_parity():
    """At the benchmark size: run on the GPU, then check one more GPU step at
    sampled nodes against the per-node oracle twin computed from the GPU state."""
    torch = _torch()
    w = synth.WORKLOADS["spinodal256_f64"]
    shape = w.shape
    n = w.nodes
    _say(f"case {w.name} sampled one-step parity")
    a, b = synth.fluid_fields(shape, w.amp, w.seed)
    with P.Lattice(shape, tau=w.tau, G=w.G) as lat:
        lat.set_fields(a.ravel().copy(), b.ravel().copy())
        t0, _ = lat.totals()
        lat.step(50)
        f = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(f)
        f_host = f.cpu().numpy().reshape((2, 19) + shape)
        lat.step(1)
        lat.get_populations(f)
        t1, nf = lat.totals()
    assert not nf
    assert abs(t1[0] - t0[0]) / t0[0] < 1e-12 and abs(t1[1] - t0[1]) / t0[1] < 1e-12
    f1 = f.view(2, 19, *shape)
    sites = synth.sample_sites(shape, 24, 61)
    want = N.step_at(f_host, sites, w.tau, w.G)
    for s, (x, y, z) in enumerate(sites):
        got = f1[:, :, z, y, x].cpu().numpy()
        err = np.max(np.abs(got - want[s]) / np.maximum(np.abs(want[s]), 1e-3 * O.W[None, :]))
        assert err <= 1e-13, (x, y, z, err)


def _gather_block(torch, f5, solid3, site, r=2):
    """Populations (2, 19, 2r+1, 2r+1, 2r+1) and solid flags around ``site``
    (periodic), copied to the host.  One step at the block's centre depends
    only on nodes within distance 2, so the per-node twin can step the block
    as if it were a periodic box of its own."""
    nz, ny, nx = f5.shape[2:]
    x, y, z = (int(v) for v in site)
    dev = f5.device
    zi = torch.tensor([(z + d) % nz for d in range(-r, r + 1)], device=dev)
    yi = torch.tensor([(y + d) % ny for d in range(-r, r + 1)], device=dev)
    xi = torch.tensor([(x + d) % nx for d in range(-r, r + 1)], device=dev)
    blk = f5.index_select(2, zi).index_select(3, yi).index_select(4, xi).cpu().numpy()
    sol = None
    if solid3 is not None:
        sol = solid3.index_select(0, zi).index_select(1, yi).index_select(2, xi).cpu().numpy()
    return blk, sol


@pytest.mark.parametrize("wname", ["spinodal256_f32", "spinodal256_f16s", "spheres512_f32"])
def test_full_size_reduced_storage_sampled_one_step(wname):
    """The float32 and float16-shifted forms at their benchmark sizes (256^3,
    and 512^3 with 2000 spheres), in the launch configuration the benchmark
    times: after 20 GPU steps, one more GPU step at sampled nodes against the
    float64 per-node twin stepped from the exported GPU state.  The bound is
    the storage's rounding of the result -- half an ulp of float16 at
    |f - w_i rho0| for the shifted form -- plus float32 arithmetic (1e-5 w_i)."""
    torch = _torch()
    w = synth.WORKLOADS[wname]
    shape, n = w.shape, w.nodes
    _say(f"case {wname} full-size sampled one-step parity")
    a, b = synth.fluid_fields(shape, w.amp, w.seed)
    solid = None
    sites = [tuple(int(v) for v in s) for s in synth.sample_sites(shape, 12, 71)]
    if w.spheres:
        centres = synth.sphere_centres(shape, w.spheres, w.radius, w.sphere_seed)
        solid = synth.solid_mask(shape, centres, w.radius)
        sites = [s for s in sites if not solid[s[2], s[1], s[0]]]
        # fluid nodes next to a sphere, to exercise bounce-back
        nz, ny, nx = shape
        for cx, cy, cz in centres[:60]:
            x, y, z = (int(round(cx)) + 6) % nx, int(round(cy)) % ny, int(round(cz)) % nz
            if solid[z, y, x]:
                continue
            near = any(solid[(z + dz) % nz, (y + dy) % ny, (x + dx) % nx]
                       for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1))
            if near:
                sites.append((x, y, z))
            if len(sites) >= 24:
                break
        assert len(sites) >= 18
    with P.Lattice(shape, tau=w.tau, G=w.G, storage=w.storage) as lat:
        lat.set_fields(a.ravel().copy(), b.ravel().copy(), None,
                       None if solid is None else solid.reshape(-1).astype(np.uint8).copy())
        lat.step(20)
        f = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(f)
        f5 = f.view(2, 19, *shape)
        s3 = None if solid is None else torch.tensor(solid.astype(np.uint8), device="cuda")
        blocks = [_gather_block(torch, f5, s3, s) for s in sites]
        lat.step(1)
        lat.get_populations(f)
        got = [f5[:, :, z, y, x].cpu().numpy() for (x, y, z) in sites]
        _, nonfinite = lat.totals()
    assert not nonfinite
    shift = (O.W[None, :] * np.asarray(w.rho0)[:, None]) if w.storage == "f16s" else 0.0
    worst = 0.0
    for (x, y, z), (blk, sol), g in zip(sites, blocks, got):
        want = N.step_at(blk, [(2, 2, 2)], w.tau, w.G, solid=sol)[0]
        bound = 1e-5 * O.W[None, :]
        if w.storage == "f16s":
            bound = bound + 2.0 ** -11 * 1.01 * np.abs(want - shift)
        ratio = np.max(np.abs(g - want) / bound)
        worst = max(worst, ratio)
        assert ratio <= 1.0, (x, y, z, ratio)
    _say(f"  worst error / bound {worst:.3f} over {len(sites)} sites")



@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_float_tall_tiles_equal_the_64x4_tiles_bitwise(storage):
    """Float storage without solids runs 64 x 8 tiles where their columns keep
    chunks of at least 64 planes; the node arithmetic does not depend on the
    tile, so the result equals, bit for bit, that of the 64 x 4 kernel with
    solid handling (run here through an all-fluid solid mask).  128 x 1020 x
    64: 256 columns of 64 x 8 with a ragged last tile row, one 64-plane chunk
    each."""
    torch = _torch()
    shape = (64, 1020, 128)
    n = int(np.prod(shape))
    _say(f"case {storage} tall tiles vs 64x4 shape={shape}")
    a, b = synth.fluid_fields(shape, 0.02, 23)
    out = []
    for solid in (None, np.zeros(n, dtype=np.uint8)):
        with P.Lattice(shape, tau=(0.8, 0.9), G=3.5, storage=storage) as lat:
            lat.set_fields(a.reshape(-1).copy(), b.reshape(-1).copy(), None, solid)
            lat.step(3)
            f = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
            lat.get_populations(f)
            torch.cuda.synchronize()
            out.append(f)
    assert torch.isfinite(out[0]).all()
    assert torch.equal(out[0], out[1])


@pytest.mark.parametrize("shape", [(1, 4, 64), (5, 8, 64), (3, 12, 128), (6, 4, 192)])
def test_f64_tile_major_step_bitwise_equal_to_oracle(shape):
    """The staged float64 step on 64 x 4 tiles runs on the tile-major layout
    (nx a multiple of 64, ny of 4); every other call first puts the state back
    in the structure-of-arrays layout.  Steps interleaved with totals,
    population reads and a snapshot round trip stay bitwise equal to the
    oracle."""
    torch = _torch()
    _say(f"case f64 tile-major shape={shape}")
    n = int(np.prod(shape))
    a, b = synth.fluid_fields(shape, 0.2, 24)
    rng = np.random.default_rng(25)
    u = [rng.uniform(-0.05, 0.05, shape) for _ in range(3)]
    p = O.Params((0.8, 1.3), 3.5)
    f0 = O.init_equilibrium(a, b, u)
    f = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
    with P.Lattice(shape, tau=p.tau, G=p.G, kernel="fused_staged") as lat:
        lat.set_fields(a.reshape(-1).copy(), b.reshape(-1).copy(), np.stack(u).reshape(-1).copy())
        lat.step(2)
        (_, _, _, _, _), nonfinite = lat.totals()
        assert not nonfinite
        lat.step(1)
        lat.get_populations(f)
        torch.cuda.synchronize()
        assert np.array_equal(f.cpu().numpy().reshape((2, 19) + tuple(shape)), O.step(f0, p, n=3))
        snap = torch.empty(int(P.lb_state_bytes(lat.ctx)) // 8, dtype=torch.float64, device="cuda")
        lat.step(1)
        P.lb_save_state(lat.ctx, snap)
        lat.step(2)
        P.lb_restore_state(lat.ctx, snap)
        lat.step(2)
        lat.get_populations(f)
        torch.cuda.synchronize()
        assert np.array_equal(f.cpu().numpy().reshape((2, 19) + tuple(shape)), O.step(f0, p, n=6))
        # a host snapshot taken from the tile-major state (converted in place)
        host = np.empty(int(P.lb_state_bytes(lat.ctx)) // 8)
        P.lb_save_state(lat.ctx, host)
        lat.step(3)
        P.lb_restore_state(lat.ctx, host)
        lat.step(1)
        lat.get_populations(f)
        torch.cuda.synchronize()
    assert np.array_equal(f.cpu().numpy().reshape((2, 19) + tuple(shape)), O.step(f0, p, n=7))


@pytest.mark.parametrize("storage", ["f32", "f16s"])
@pytest.mark.parametrize("shape,with_solid", [((5, 8, 64), False), ((3, 12, 128), False), ((70, 4, 64), False),
                                              ((6, 8, 64), True), ((40, 16, 192), False), ((9, 8, 64), False),
                                              ((70, 24, 128), False)])
def test_float_tile_major_step_equals_the_structure_of_arrays_step(shape, with_solid, storage):
    """Float storage runs on the tile-major layout where nx is a multiple of 64
    and ny of 4.  lb_step_between steps snapshots, which are in the
    structure-of-arrays layout, with the structure-of-arrays kernel; the node
    arithmetic does not depend on the layout, so three steps each way give
    the same populations bit for bit (with totals and a population read
    between the tile-major steps).  Shapes: one tile (x and y wrap onto the
    tile itself), three tiles in x, 64 x 8 tiles in several z-chunks with a
    ragged last chunk."""
    torch = _torch()
    n = int(np.prod(shape))
    _say(f"case {storage} tile-major vs structure of arrays shape={shape} solid={with_solid}")
    a, b = synth.fluid_fields(shape, 0.05, 26)
    solid = synth.solid_mask(shape, np.array([[30.0, 4.0, 3.0]]), 2.2).reshape(-1) if with_solid else None
    with P.Lattice(shape, tau=(0.8, 1.1), G=3.5, storage=storage) as lat:
        lat.set_fields(a.reshape(-1).copy(), b.reshape(-1).copy(), None, solid)
        nb = P.lb_state_bytes(lat.ctx)
        snaps = [torch.empty(nb, dtype=torch.uint8, device="cuda") for _ in range(4)]
        P.lb_save_state(lat.ctx, snaps[0])
        for t in range(3):
            P.lb_step_between(lat.ctx, snaps[t], snaps[t + 1])
        lat.step(2)
        (_, _, _, _, _), nonfinite = lat.totals()
        assert not nonfinite
        f = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(f)
        lat.step(1)
        lat.get_populations(f)
        P.lb_restore_state(lat.ctx, snaps[3])
        g = torch.empty_like(f)
        lat.get_populations(g)
        torch.cuda.synchronize()
    assert torch.equal(f, g)


def test_f64_kernel_switches_between_layouts_bitwise():
    """Switching between the staged step (tile-major layout) and the two-pass
    step (structure of arrays) in the middle of a run reorders the state at
    each switch; 2 + 2 + 1 steps stay bitwise equal to the oracle."""
    torch = _torch()
    shape = (5, 8, 64)
    n = int(np.prod(shape))
    _say(f"case f64 kernel switches shape={shape}")
    a, b = synth.fluid_fields(shape, 0.2, 27)
    p = O.Params((0.8, 1.3), 3.5)
    f = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")
    with P.Lattice(shape, tau=p.tau, G=p.G, kernel="fused_staged") as lat:
        lat.set_fields(a.reshape(-1).copy(), b.reshape(-1).copy())
        lat.step(2)
        P.lb_set_kernel(lat.ctx, "two_pass")
        lat.step(2)
        P.lb_set_kernel(lat.ctx, "fused_staged")
        lat.step(1)
        lat.get_populations(f)
        torch.cuda.synchronize()
    assert np.array_equal(f.cpu().numpy().reshape((2, 19) + tuple(shape)), O.step(O.init_equilibrium(a, b), p, n=5))


@pytest.mark.parametrize("storage", ["f16s", "f32"])
def test_full_size_tile_major_step_equals_the_structure_of_arrays_step(storage):
    """The 256^3 spinodal workload as the benchmark launches it (float16-shifted:
    64 x 8 tiles in 128-plane chunks; float32: 64 x 4 tiles, loads two planes
    ahead) against the structure-of-arrays kernel, two steps each way from
    the same state: the same populations bit for bit."""
    torch = _torch()
    w = synth.WORKLOADS["spinodal256_f64"]
    _say(f"case {storage} full size tile-major vs structure of arrays shape={w.shape}")
    a, b = synth.fluid_fields(w.shape, w.amp, w.seed)
    with P.Lattice(w.shape, tau=w.tau, G=w.G, storage=storage) as lat:
        lat.set_fields(a.reshape(-1).copy(), b.reshape(-1).copy())
        nb = P.lb_state_bytes(lat.ctx)
        snaps = [torch.empty(nb, dtype=torch.uint8, device="cuda") for _ in range(2)]
        P.lb_save_state(lat.ctx, snaps[0])
        P.lb_step_between(lat.ctx, snaps[0], snaps[1])
        P.lb_step_between(lat.ctx, snaps[1], snaps[0])
        lat.step(2)
        mine = torch.empty(nb, dtype=torch.uint8, device="cuda")
        P.lb_save_state(lat.ctx, mine)
        torch.cuda.synchronize()
        assert torch.equal(mine, snaps[0])
        (_, _, _, _, _), nonfinite = lat.totals()
        assert not nonfinite


@pytest.mark.parametrize("storage,shape", [("f64", (5, 8, 64)), ("f64", (3, 12, 128)), ("f32", (6, 12, 64)),
                                           ("f16s", (7, 8, 128))])
def test_reads_of_the_tile_major_state_in_place(storage, shape):
    """lb_moments, lb_totals and lb_get_populations read the state in the
    order the steps left it (tile-major here), without reordering it: their
    results equal, bit for bit, those read after a host snapshot has put the
    state back in the structure of arrays, and steps taken after such reads
    continue the same trajectory (float64: bitwise the oracle's)."""
    torch = _torch()
    n = int(np.prod(shape))
    _say(f"case {storage} moments/totals on the tile-major state shape={shape}")
    a, b = synth.fluid_fields(shape, 0.2, 28)
    p = O.Params((0.8, 1.1), 3.5)
    f = torch.empty(2 * 19 * n, dtype=torch.float64, device="cuda")

    def read(lat):
        ra, rb, u = (torch.empty(k * n, dtype=torch.float64, device="cuda") for k in (1, 1, 3))
        lat.moments(ra, rb, u)
        tot, nonfinite = lat.totals()
        assert not nonfinite
        return torch.cat([ra, rb, u]), tot

    with P.Lattice(shape, tau=p.tau, G=p.G, storage=storage) as lat:
        lat.set_fields(a.reshape(-1).copy(), b.reshape(-1).copy())
        lat.step(3)
        m_tiled, t_tiled = read(lat)
        lat.step(1)
        m_tiled2, t_tiled2 = read(lat)
        g_tiled = torch.empty_like(f)
        lat.get_populations(g_tiled)
        host = np.empty(int(P.lb_state_bytes(lat.ctx)), dtype=np.uint8)
        P.lb_save_state(lat.ctx, host)  # a host snapshot: the structure-of-arrays order from here on
        m_soa, t_soa = read(lat)
        lat.get_populations(f)
        torch.cuda.synchronize()
        assert torch.equal(m_tiled2, m_soa)
        assert t_tiled2 == t_soa
        assert torch.equal(g_tiled, f)
        assert not torch.equal(m_tiled, m_tiled2)
        lat.step(1)
        lat.get_populations(f)
        torch.cuda.synchronize()
    if storage == "f64":
        assert np.array_equal(f.cpu().numpy().reshape((2, 19) + tuple(shape)),
                              O.step(O.init_equilibrium(a, b), p, n=5))
