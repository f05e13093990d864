"""Parity of the moving-particle step (lb1_set_particles / lb1_step through
the C ABI) with the FP64 particle oracle (the paper's particle solver on the
single-fluid step).

The oracle sums each particle's force, torque and covering momentum exactly
and rounds once (math.fsum); the GPU sums the same float64 terms in its own
order.  After one step from a shared state the two forces and torques may
differ by at most the summation bound of the terms (``PT.sum_bound``), and
every population the sums do not reach is bitwise equal.  Over 15 steps the
rounding differences of the sums propagate: states are held to the 1e-12
relative-per-population bar and particle state to 1e-12 absolute (two
summation orders of the oracle itself differ by about 1e-15 there).
float32 is held to bounds from its precision.
"""

import math
import sys

import numpy as np
import pytest

import paper_2112_08264_amd as P
from oracle import lb_oracle as O
from oracle import lb_particles as PT
from oracle import lb_single as S
import synth

import particle_window as PW

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _fluid(shape, seed, amp=0.01, vel=0.01):
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-amp, amp, shape)
    u = [rng.uniform(-vel, vel, shape) for _ in range(3)]
    return rho, u


def run_gpu(shape, tau, rho, u, part, steps, storage="f64"):
    torch = _torch()
    n = int(np.prod(shape))
    with P.SingleFluid(shape, tau=tau, storage=storage) as lat:
        lat.set_fields(np.ascontiguousarray(rho.reshape(-1)), np.ascontiguousarray(np.stack(u).reshape(-1)))
        lat.set_particles(part.pos, part.radius, part.mass, part.vel, part.omg)
        lat.step(steps)
        f = torch.empty(19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(f)
        torch.cuda.synchronize()
        return f.cpu().numpy().reshape((19,) + tuple(shape)), lat.particles()


CASES = {
    # two particles crossing nodes
    "two": ((20, 18, 22), PT.Particles(3.2, 400.0, [[6.3, 5.2, 7.1], [15.4, 12.6, 13.2]],
                                       [[0.08, -0.05, 0.06], [-0.07, 0.06, -0.05]],
                                       [[0.0, 0.0, 0.02], [0.02, -0.01, 0.0]])),
    # three particles, two of them across the periodic boundaries (masses about three times the fluid they
    # displace: much lighter spheres make the explicit coupling oscillate)
    "wrap": ((19, 21, 24), PT.Particles(2.7, 250.0, [[0.4, 10.2, 18.7], [22.9, 20.6, 3.3], [12.0, 5.5, 9.9]],
                                        [[-0.12, 0.03, 0.09], [0.1, 0.11, -0.04], [0.0, 0.1, 0.0]],
                                        [[0.01, 0.02, -0.01], [0.0, 0.0, 0.0], [-0.02, 0.0, 0.03]])),
    # two spheres under one node apart: fluid nodes between them have links into both
    "close": ((16, 18, 28), PT.Particles(3.3, 400.0, [[8.2, 9.1, 8.4], [15.6, 9.4, 8.0]],
                                         [[0.03, 0.0, 0.01], [-0.03, 0.01, 0.0]],
                                         [[0.0, 0.01, 0.0], [0.01, 0.0, -0.01]])),
    # two overlapping spheres: nodes inside both belong to the lower index
    "overlap": ((18, 18, 22), PT.Particles(3.1, 400.0, [[9.3, 8.8, 9.1], [13.4, 9.6, 9.0]],
                                           [[0.02, 0.0, 0.0], [0.02, 0.01, 0.0]], None)),
}


U = 2.0 ** -53


@pytest.mark.parametrize("name", sorted(CASES))
def test_f64_particles_match_oracle_over_15_steps(name):
    shape, part = CASES[name]
    _say(f"case particles f64 15 steps {name} shape={shape}")
    rho, u = _fluid(shape, 51)
    f, owner = PT.init(rho, part, u)
    ref, q, owner_end = PT.step(f, 0.8, part.copy(), owner, n=15)
    assert np.all(np.isfinite(ref))
    got, (pos, vel, omg, force, torque) = run_gpu(shape, 0.8, rho, u, part, 15)
    assert np.sum(owner_end != owner) > 0
    perr = O.population_error(got[None], ref[None])
    serr = max(float(np.max(np.abs(a - b))) for a, b in ((pos, q.pos), (vel, q.vel), (omg, q.omg),
                                                          (force, q.force), (torque, q.torque)))
    _say(f"  population error {perr:.1e}, particle state {serr:.1e}")
    assert perr <= 1e-12
    assert serr <= 1e-12


@pytest.mark.parametrize("name", sorted(CASES))
def test_f64_particles_first_step_within_the_summation_bound(name):
    """One step from the shared initial state.  The fluid step before the sums
    is bitwise equal, so the GPU's force and torque must lie within the
    summation bound of the oracle's own link terms, the velocities within
    that bound over m (and I) plus the roundings of the two updates, and every
    population not at a node uncovered in the step bitwise equal."""
    shape, part = CASES[name]
    _say(f"case particles f64 first step {name} shape={shape}")
    rho, u = _fluid(shape, 51)
    f, owner = PT.init(rho, part, u)
    fnew, rho_t = PT.fluid_step(f, 0.8, part, owner)
    nP = part.pos.shape[0]
    bF = np.array([PT.sum_bound(PT.link_terms(fnew, rho_t, part, owner, p)) for p in range(nP)])
    F, T = PT.link_forces(fnew, rho_t, part, owner)
    q = PT.move(part, F, T, shape)
    owner1 = PT.owner_map(shape, q)
    bC = np.array([PT.sum_bound(PT.remap_terms(fnew.copy(), q, owner, owner1, 1.0, p)) for p in range(nP)])
    ref = PT.remap(fnew, q, owner, owner1, 1.0)
    got, (pos, vel, omg, force, torque) = run_gpu(shape, 0.8, rho, u, part, 1)
    assert np.all(np.abs(force - F) <= bF[:, :3])
    assert np.all(np.abs(torque - T) <= bF[:, 3:])
    m, inertia = part.mass, part.inertia
    tol_v = (bF[:, :3] + bC[:, :3]) / m + 8 * U * (np.abs(q.vel) + np.abs(F) / m + np.abs(part.vel))
    tol_w = (bF[:, 3:] + bC[:, 3:]) / inertia + 8 * U * (np.abs(q.omg) + np.abs(T) / inertia + np.abs(part.omg))
    assert np.all(np.abs(vel - q.vel) <= tol_v)
    assert np.all(np.abs(omg - q.omg) <= tol_w)
    assert np.all(np.abs(pos - q.pos) <= bF[:, :3] / m + 8 * U * (np.abs(q.pos) + 1.0))
    uncovered = (owner != PT.FLUID) & (owner1 == PT.FLUID)
    keep = ~uncovered
    assert np.array_equal(got[:, keep], ref[:, keep])
    if np.any(uncovered):
        assert O.population_error(got[None][:, :, uncovered], ref[None][:, :, uncovered]) <= 1e-13


def test_f64_resting_particle_is_the_fixed_solid_step():
    shape = (14, 15, 16)
    _say(f"case particles f64 resting shape={shape}")
    rho, u = _fluid(shape, 52)
    part = PT.Particles(3.5, math.inf, [[7.0, 6.5, 8.2]], None, None)
    f, owner = PT.init(rho, part, u)
    ref = S.step(f, 0.8, (owner != PT.FLUID).astype(np.uint8), n=6)
    got, (pos, *_rest) = run_gpu(shape, 0.8, rho, u, part, 6)
    assert np.array_equal(got, ref)
    assert np.array_equal(pos, part.pos)


def test_f64_total_momentum_conserved_with_many_particles():
    torch = _torch()
    shape = (48, 48, 48)
    n = int(np.prod(shape))
    _say(f"case particles f64 momentum shape={shape}")
    rng = np.random.default_rng(53)
    centres = synth.sphere_centres(shape, 20, 3.5, 54, min_sep=9.0)
    vel = rng.uniform(-0.05, 0.05, (20, 3))
    omg = rng.uniform(-0.01, 0.01, (20, 3))
    rho, u = _fluid(shape, 55)
    mass = synth.particle_mass(3.5)
    with P.SingleFluid(shape, tau=0.9) as lat:
        lat.set_fields(rho.ravel().copy(), np.stack(u).reshape(-1).copy())
        lat.set_particles(centres, 3.5, mass, vel, omg)

        def total():
            (M, px, py, pz), nonfinite = lat.totals()
            assert not nonfinite
            _, v, *_ = lat.particles()
            return M, np.array([px, py, pz]) + mass * v.sum(axis=0)

        M0, P0 = total()
        lat.step(100)
        M1, P1 = total()
    _say(f"  |dP| {np.max(np.abs(P1 - P0)):.2e}, dM/M {abs(M1 - M0) / M0:.2e}")
    assert np.max(np.abs(P1 - P0)) <= 1e-12 * M0
    assert abs(M1 - M0) <= 1e-3 * M0  # uncovered nodes start at rho0: mass is not conserved exactly


def test_f32_particles_against_the_oracle():
    """float32 fluid with float64 particle arithmetic, 15 steps: particle
    positions within 1e-6 and populations within 1e-5 of the float64 oracle
    (float32 rounds each population to 2^-24 relative; forces sum a few
    hundred links of such values)."""
    shape, part = CASES["two"]
    _say(f"case particles f32 shape={shape}")
    rho, u = _fluid(shape, 56)
    f, owner = PT.init(rho, part, u)
    ref, q, _ = PT.step(f, 0.8, part.copy(), owner, n=15)
    got, (pos, vel, *_rest) = run_gpu(shape, 0.8, rho, u, part, 15, storage="f32")
    perr = float(np.max(np.abs(pos - q.pos)))
    ferr = float(np.max(np.abs(got - ref)))
    _say(f"  max |dpos| {perr:.2e}, max |df| {ferr:.2e}")
    assert perr <= 1e-6
    assert ferr <= 1e-5


def test_particle_error_paths():
    n = 16 ** 3
    good = np.array([[8.0, 8.0, 8.0]])
    with P.SingleFluid((16, 16, 16)) as lat:
        with pytest.raises(P.LBError) as e:
            lat.set_particles(good, 2.0, 10.0)
        assert e.value.status == P.LB_ESTATE
        lat.set_fields(np.ones(n))
        for args in ((good, 6.5, 10.0),               # box 17 > 16
                     (good, -1.0, 10.0), (good, 2.0, 0.0), (good, 2.0, float("nan")),
                     (np.array([[16.0, 8.0, 8.0]]), 2.0, 10.0)):
            with pytest.raises(P.LBError) as e:
                lat.set_particles(*args)
            assert e.value.status == P.LB_EINVAL
        with pytest.raises(P.LBError) as e:
            lat.set_particles(good, 2.0, 10.0, vel=np.array([[0.5, 0.0, 0.0]]))
        assert e.value.status == P.LB_EINVAL
        with pytest.raises(P.LBError) as e:
            lat.particles()
        assert e.value.status == P.LB_ESTATE
        lat.set_particles(good, 2.0, math.inf)
        lat.step(2)
        pos, *_ = lat.particles()
        assert np.array_equal(pos, good)
        lat.set_particles(None, 2.0, 1.0)  # removes them
        lat.step(1)
    with P.SingleFluid((16, 16, 16)) as lat:
        lat.set_fields(np.ones(n), None, np.zeros(n, dtype=np.uint8))
        with pytest.raises(P.LBError) as e:
            lat.set_particles(good, 2.0, 10.0)
        assert e.value.status == P.LB_EINVAL
    with P.SingleFluid((16, 16, 16), storage="f16s") as lat:
        lat.set_fields(np.ones(n))
        with pytest.raises(P.LBError) as e:
            lat.set_particles(good, 2.0, 10.0)
        assert e.value.status == P.LB_EINVAL


@pytest.mark.parametrize("name", ["case3c_256_f32", "case3c_256_f64"])
def test_full_size_case3c_conserves_momentum(name):
    """The 10% moving-sphere workload (2407 spheres of radius 5.5 in 256^3), in
    the launch configuration the benchmark times, set moving: 20 steps keep the
    total momentum (fluid plus particles) to rounding, every particle inside
    the box and the state finite."""
    w = synth.WORKLOADS[name]
    _say(f"case {w.name} momentum")
    rho, _ = synth.fluid_fields(w.shape, w.amp, w.seed)
    centres = synth.sphere_centres(w.shape, w.spheres, w.radius, w.sphere_seed)
    rng = np.random.default_rng(57)
    vel = rng.uniform(-0.02, 0.02, (w.spheres, 3))
    mass = synth.particle_mass(w.radius)
    with P.SingleFluid(w.shape, tau=w.tau[0], storage=w.storage) as lat:
        lat.set_fields(rho.ravel().copy())
        lat.set_particles(centres, w.radius, mass, vel)

        def total():
            (M, px, py, pz), nonfinite = lat.totals()
            assert not nonfinite
            pos, v, *_ = lat.particles()
            return M, np.array([px, py, pz]) + mass * v.sum(axis=0), pos

        M0, P0, _ = total()
        lat.step(20)
        M1, P1, pos = total()
    # each step rounds every stored population once (about 0.4 at most): a random walk of
    # 20 x 19 x N roundings, allowed ten standard deviations
    u = 2.0 ** -53 if w.storage == "f64" else 2.0 ** -24
    tol = 10.0 * math.sqrt(20 * 19 * w.nodes) * u * 0.4
    _say(f"  |dP| {np.max(np.abs(P1 - P0)):.2e} (bound {tol:.1e})")
    assert np.max(np.abs(P1 - P0)) <= tol
    assert np.all(pos >= 0.0) and np.all(pos < 256.0)



@pytest.mark.parametrize("name", ["case3c_256_f64", "case3c_256_f32"])
def test_full_size_case3c_sampled_one_step(name):
    """The 10% moving-sphere workload (2407 spheres, 256^3) as the benchmark
    launches it, one step, checked sphere by sphere: 8 sampled spheres
    against the oracle stepped on a 32^3 window around each (the window
    reduction and its exactness are described in ``particle_window``).
    float64 force and torque are held to the summation bound of the
    sphere's link terms, velocities and position to that bound propagated
    through the leap-frog and the covering sums, and the populations within
    R + 3 of the centre bit for bit (nodes the step uncovers, whose
    populations carry the new velocity, to 1e-13).  Spheres across the
    periodic ends are covered by the small-box tests, against the
    whole-lattice oracle."""
    torch = _torch()
    w = synth.WORKLOADS[name]
    _say(f"case {w.name} sampled one step")
    shape = w.shape
    n = w.nodes
    rho, _ = synth.fluid_fields(shape, w.amp, w.seed)
    centres = synth.sphere_centres(shape, w.spheres, w.radius, w.sphere_seed)
    rng = np.random.default_rng(58)
    vel = rng.uniform(-0.03, 0.03, (w.spheres, 3))
    omg = rng.uniform(-0.003, 0.003, (w.spheres, 3))
    mass = synth.particle_mass(w.radius)
    sample = PW.isolated(centres, w.radius, shape, 8, 59)
    assert sample.size == 8
    with P.SingleFluid(shape, tau=w.tau[0], storage=w.storage) as lat:
        lat.set_fields(rho.ravel().copy())
        lat.set_particles(centres, w.radius, mass, vel, omg)
        lat.step(1)
        f = torch.empty(19 * n, dtype=torch.float64, device="cuda")
        lat.get_populations(f)
        pos, v1, w1, force, torque = lat.particles()
        torch.cuda.synchronize()
    f = f.view(19, n)
    errs = []
    for p in sample:
        F, T, r1, vr, wr, ref, idx, bd = PW.step_window(rho, w.tau[0], w.radius, mass, centres[p], vel[p], omg[p],
                                                        shape)
        got = f[:, torch.from_numpy(idx).to("cuda")].cpu().numpy()
        if w.storage == "f64":
            u53 = 2.0 ** -53
            bF, bC = bd["link"], bd["cover"]
            inertia = 0.4 * mass * w.radius * w.radius
            assert np.all(np.abs(force[p] - F) <= bF[:3]), p
            assert np.all(np.abs(torque[p] - T) <= bF[3:]), p
            assert np.all(np.abs(v1[p] - vr) <= (bF[:3] + bC[:3]) / mass
                          + 8 * u53 * (np.abs(vr) + np.abs(F) / mass + np.abs(vel[p]))), p
            assert np.all(np.abs(w1[p] - wr) <= (bF[3:] + bC[3:]) / inertia
                          + 8 * u53 * (np.abs(wr) + np.abs(T) / inertia + np.abs(omg[p]))), p
            assert np.all(np.abs(pos[p] - r1) <= bF[:3] / mass + 8 * u53 * (np.abs(r1) + 1.0)), p
            keep = ~bd["uncovered"]
            assert np.array_equal(got[:, keep], ref[:, keep]), p
            if np.any(bd["uncovered"]):
                assert O.population_error(got[None][:, :, ~keep], ref[None][:, :, ~keep]) <= 1e-13, p
        else:
            # A sphere of radius 5.5 has about 2200 links.  Each adds 2 g, g a float32 population near 1/18
            # carrying a few float32 roundings (about 1e-8 each).  A random walk over them gives about 1e-6, and
            # the 18 links of one fluid node share that node's collision, so their errors need not cancel: the
            # bounds allow 20 times the walk.  Torque arms reach R + 1; v and omega divide by m and I.
            errs.append([np.max(np.abs(force[p] - F)), np.max(np.abs(torque[p] - T)), np.max(np.abs(pos[p] - r1)),
                         np.max(np.abs(v1[p] - vr)), np.max(np.abs(w1[p] - wr)), np.max(np.abs(got - ref))])
    if errs:
        e = np.max(np.array(errs), axis=0)
        _say("  max |dF| {:.1e} |dT| {:.1e} |dpos| {:.1e} |dv| {:.1e} |domega| {:.1e} |df| {:.1e}".format(*e))
        assert e[0] <= 2e-5 and e[1] <= 2e-4
        assert e[2] <= 1e-7 and e[3] <= 1e-7 and e[4] <= 1e-7
        assert e[5] <= 1e-6
    _say(f"  {sample.size} particles checked")
