"""Pins of the colour-gradient-with-particles oracle (the paper's case 3:
Sec. 5 particle table; Sec. 2 particle paragraph; Appendix, colour-gradient
model and Eqs. UPI, LADDFLBE, FORCEPP, FORCEPARTEQ, TORQUEPARTEQ) against what
the model and its special cases fix (no GPU)."""

import math

import numpy as np

from oracle import lb_cg as CG
from oracle import lb_cg_particles as CP
from oracle import lb_oracle as O
from oracle import lb_particles as PT
from oracle import lb_single as S
import synth


def _colours(shape, seed):
    r1, r2 = synth.colour_fields(shape, seed)
    return r1.reshape(shape), r2.reshape(shape)


def _mixture(shape, seed, amp=0.05):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, shape)
    rho = 1.0 + rng.uniform(-amp, amp, shape)
    return rho * c, rho * (1.0 - c)


def test_without_solids_it_is_the_colour_gradient_step():
    shape = (6, 7, 8)
    r1, r2 = _mixture(shape, 1)
    p = CP.Params((0.9, 1.1), 0.01, 0.7)
    f = CG.init_equilibrium(r1, r2)
    got = CP.step_solid(f, p, np.zeros(shape, dtype=bool), n=3)
    assert np.array_equal(got, CG.step(f, p.cg, n=3))


def test_fixed_solids_conserve_each_component_and_stay_empty():
    shape = (14, 14, 14)
    solid = synth.solid_mask(shape, np.array([[4.2, 5.1, 6.3], [10.4, 9.2, 8.8]]), 2.6).astype(bool)
    r1, r2 = _mixture(shape, 2)
    f = O.init_equilibrium(r1, r2, solid=solid)
    p = CP.Params((1.0, 0.8), 0.01, 0.7)
    (m1, m2, *_), _ = O.totals(f)
    f = CP.step_solid(f, p, solid, n=60)
    (n1, n2, *_), nonfinite = O.totals(f)
    assert not nonfinite
    assert np.ptp(O.density(f[0])[~solid]) > 0.5  # it has demixed
    assert abs(n1 - m1) / m1 < 1e-13 and abs(n2 - m2) / m2 < 1e-13
    assert np.all(f[:, :, solid] == 0.0)


def test_without_surface_tension_the_sum_of_the_components_is_the_single_fluid_step():
    """sigma = beta = 0 and equal tau: no perturbation, no recolouring force,
    omega = 1/tau, so f^1 + f^2 follows the single-fluid BGK step with the same
    bounce-back (within rounding: the two sum in different orders)."""
    shape = (10, 11, 12)
    solid = synth.solid_mask(shape, np.array([[5.3, 4.8, 6.1]]), 2.9).astype(bool)
    r1, r2 = _mixture(shape, 3)
    f = O.init_equilibrium(r1, r2, solid=solid)
    got = CP.step_solid(f, CP.Params((0.8, 0.8), 0.0, 0.0), solid, n=8)
    want = S.step(f[0] + f[1], 0.8, solid.astype(np.uint8), n=8)
    assert np.max(np.abs((got[0] + got[1]) - want)) < 1e-14


def test_a_wall_is_neutral_a_pure_phase_at_rest_beside_it_stays_at_rest():
    """Neutral wetting (CP1): a solid neighbour adds no phase gradient, so a
    pure phase at rest beside a particle sees grad Theta = 0 and neither the
    perturbation nor the recolouring acts: the state is a fixed point."""
    shape = (12, 12, 12)
    solid = synth.solid_mask(shape, np.array([[6.2, 5.7, 6.4]]), 3.3).astype(bool)
    for r1v, r2v in ((1.0, 0.0), (0.0, 0.9)):
        f = O.init_equilibrium(np.full(shape, r1v), np.full(shape, r2v), solid=solid)
        g = CP.step_solid(f, CP.Params((1.0, 1.0), 0.02, 0.7), solid, n=10)
        assert np.max(np.abs(g - f)) < 1e-15


def test_an_interface_meets_a_wall_at_right_angles():
    """The paper's 90 degree contact angle: two flat interfaces normal to x in
    a 2-D box whose row y = 0 is solid stay flat and in place; the
    zero-crossing of Theta is at x = 7.5 in every fluid row."""
    nx, ny = 32, 12
    shape = (1, ny, nx)
    solid = np.zeros(shape, dtype=bool)
    solid[0, 0, :] = True
    x = np.arange(nx)
    inner = ((x >= nx // 4) & (x < 3 * nx // 4)).astype(np.float64)
    r1 = np.broadcast_to(inner, shape).copy()
    r2 = 1.0 - r1
    f = O.init_equilibrium(r1, r2, solid=solid)
    f = CP.step_solid(f, CP.Params((1.0, 1.0), 0.01, 0.7), solid, n=400)
    a, b = O.density(f[0])[0], O.density(f[1])[0]
    for y in range(1, ny):
        th = (a[y] - b[y]) / (a[y] + b[y])
        k = int(np.nonzero((th[:-1] < 0) & (th[1:] >= 0))[0][0])
        assert abs(k + (-th[k]) / (th[k + 1] - th[k]) - 7.5) < 1e-6, y


def test_resting_heavy_particle_is_the_fixed_solid_step():
    shape = (13, 14, 15)
    r1, r2 = _mixture(shape, 4)
    part = PT.Particles(3.4, math.inf, [[7.1, 6.6, 7.9]], None, None)
    f, owner = CP.init(r1, r2, part)
    p = CP.Params((1.0, 0.9), 0.01, 0.7)
    g, q, _ = CP.step(f.copy(), p, part, owner, n=4)
    h = CP.step_solid(f.copy(), p, owner != PT.FLUID, n=4)
    assert np.array_equal(g, h)
    assert np.array_equal(q.pos, part.pos)


def test_total_momentum_is_conserved_while_particles_move_in_a_demixing_mixture():
    shape = (18, 16, 20)
    r1, r2 = _colours(shape, 5)
    part = PT.Particles(3.1, 300.0, [[5.8, 5.1, 6.6], [14.3, 11.2, 12.4]],
                        [[0.07, -0.05, 0.06], [-0.06, 0.05, -0.04]], [[0.0, 0.0, 0.02], [0.02, -0.01, 0.0]])
    f, owner = CP.init(r1, r2, part)
    p = CP.Params((1.0, 1.0), 0.01, 0.7, (0.5, 0.5))
    P0 = CP.total_momentum(f, part)
    changes = 0
    for _ in range(20):
        f, part, owner_new = CP.step(f, p, part, owner)
        changes += int(np.sum(owner_new != owner))
        owner = owner_new
    P1 = CP.total_momentum(f, part)
    assert changes > 20
    assert np.max(np.abs(P1 - P0)) < 1e-13 * np.sum(r1 + r2)
    assert np.all(f[:, :, owner != PT.FLUID] == 0.0)


def test_first_step_force_in_a_uniform_mixture_is_the_link_sum_closed_form():
    """A uniform mixture at rest (Theta constant, no perturbation, no
    recolouring flux): f^k* = w_i rho^k and each component of each link hands
    the particle c_i (2 w_i rho^k - 6 w_i rho^k c_i.U), so
    F = -6 (rho^1 + rho^2) sum_links w_i c_i (c_i . U) and T = 0."""
    shape = (20, 20, 20)
    U = np.array([0.01, -0.02, 0.005])
    part = PT.Particles(4.3, math.inf, [[10.0, 10.0, 10.0]], [U], None)
    f, owner = CP.init(np.full(shape, 0.7), np.full(shape, 0.45), part)
    _, q, _ = CP.step(f, CP.Params((0.9, 0.9), 0.01, 0.7), part, owner)
    M = np.zeros((3, 3))
    nz, ny, nx = shape
    for z, y, x in zip(*np.nonzero(owner == 0)):
        for i in range(1, O.Q):
            if owner[(z - O.C[i, 2]) % nz, (y - O.C[i, 1]) % ny, (x - O.C[i, 0]) % nx] == PT.FLUID:
                M += O.W[i] * np.outer(O.C[i], O.C[i])
    want = -6.0 * (0.7 + 0.45) * M @ U
    assert np.max(np.abs(q.force[0] - want)) < 1e-13 * np.max(np.abs(want))
    assert np.max(np.abs(q.torque[0])) < 1e-12 * np.max(np.abs(want))


def test_uncovered_nodes_take_the_stated_densities_and_the_surface_velocity():
    """A translating particle of infinite mass in a uniform mixture moving with
    it (rho^k = rho0^k, u = U everywhere): the moving-wall bounce-back returns
    f^eq_ibar exactly and uncovered nodes start at f^eq(rho0^k, U), so the
    state stays uniform while the particle crosses nodes."""
    shape = (14, 14, 16)
    U = np.array([0.06, 0.0, 0.0])
    rho0 = (0.55, 0.45)
    part = PT.Particles(3.2, math.inf, [[7.2, 6.9, 7.1]], [U], None)
    ones = np.ones(shape)
    f, owner = CP.init(rho0[0] * ones, rho0[1] * ones, part, [U[0] * ones, 0 * ones, 0 * ones])
    owner0 = owner.copy()
    p = CP.Params((1.0, 1.0), 0.01, 0.7, rho0)
    feq = [O.equilibrium(np.float64(rho0[k]), np.float64(U[0]), np.float64(0.0), np.float64(0.0)) for k in range(2)]
    for _ in range(20):
        f, part, owner = CP.step(f, p, part, owner)
        assert np.max(np.abs(part.force[0])) < 1e-13
    fl = owner == PT.FLUID
    for k in range(2):
        assert np.max(np.abs(f[k][:, fl] - feq[k][:, None])) < 1e-14
    assert np.sum(owner != owner0) > 10


def test_window_step_equals_the_whole_lattice_step():
    """Locality and exact translation of the case-3 step: for spheres far from
    every other sphere and from the lattice's ends, one oracle step of a 32^3
    window around the sphere (``particle_window.step_window_cg``) gives the
    whole-lattice step's force, torque, position, velocities and both
    components' nearby populations bit for bit (the full-size GPU check relies
    on this).  96^3, pure colours at random, 30 moving spheres of radius 5.5."""
    import particle_window as PW
    L = 96
    shape = (L, L, L)
    R = 5.5
    centres = synth.sphere_centres(shape, 30, R, 4)
    rng = np.random.default_rng(59)
    vel = rng.uniform(-0.03, 0.03, (30, 3))
    omg = rng.uniform(-0.003, 0.003, (30, 3))
    mass = synth.particle_mass(R)
    r1, r2 = synth.colour_fields(shape, 12)
    p = CP.Params((1.0, 1.0), 0.01, 0.7, (0.5, 0.5))
    part = PT.Particles(R, mass, centres, vel, omg)
    f, owner = CP.init(r1, r2, part)
    f1, q, _ = CP.step(f, p, part.copy(), owner, n=1)
    f1 = f1.reshape(2, 19, -1)
    sample = PW.isolated(centres, R, shape, 3, 0, margin=7.0)
    assert sample.size == 3
    for k in sample:
        F, T, rr, vr, wr, fw, idx, _ = PW.step_window_cg(r1, r2, p, R, mass, centres[k], vel[k], omg[k], shape)
        assert np.array_equal(F, q.force[k]) and np.array_equal(T, q.torque[k]), k
        assert np.array_equal(rr, q.pos[k]) and np.array_equal(vr, q.vel[k]) and np.array_equal(wr, q.omg[k]), k
        assert np.array_equal(fw, f1[:, :, idx]), k
