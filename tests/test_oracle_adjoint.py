"""Pins of the oracle's discrete adjoint against central finite differences of
the oracle's own forward step (no GPU).  The adjoint is derived by hand, the
forward step is the pinned oracle, so agreement ties the two together."""

import numpy as np
import pytest

from oracle import lb_adjoint as A
from oracle import lb_oracle as O
import synth


def _state(shape, seed, amp=0.3, solid=None):
    rng = np.random.default_rng(seed)
    a, b = synth.fluid_fields(shape, amp, seed)
    u = [rng.uniform(-0.04, 0.04, shape) for _ in range(3)]
    f = O.init_equilibrium(a, b, u, solid=solid)
    f = f * (1.0 + rng.uniform(-0.05, 0.05, f.shape))
    if solid is not None:
        f[:, :, solid.astype(bool)] = 0.0
    return f


def _solid(shape):
    s = np.zeros(shape, np.uint8)
    s[1, 2, 3] = s[2, 2, 3] = s[3, 4, 1] = 1
    return s


@pytest.mark.parametrize("with_solid", [False, True])
def test_one_step_adjoint_matches_finite_differences(with_solid):
    shape = (4, 5, 6)
    solid = _solid(shape) if with_solid else None
    p = O.Params((0.8, 1.3), 3.5)
    f = _state(shape, 1, solid=solid)
    rng = np.random.default_rng(2)
    lam_next = rng.standard_normal(f.shape)
    if solid is not None:
        lam_next[:, :, solid.astype(bool)] = 0.0
    lam, _ = A.adjoint_step(f, lam_next, p, solid)
    for trial in range(3):
        d = rng.standard_normal(f.shape)
        if solid is not None:
            d[:, :, solid.astype(bool)] = 0.0
        h = 1e-6
        Lp = np.sum(lam_next * O.step(f + h * d, p, solid))
        Lm = np.sum(lam_next * O.step(f - h * d, p, solid))
        fd = (Lp - Lm) / (2 * h)
        an = np.sum(lam * d)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (trial, fd, an)


def test_one_step_coupling_derivative():
    shape = (4, 4, 5)
    f = _state(shape, 3)
    rng = np.random.default_rng(4)
    lam_next = rng.standard_normal(f.shape)
    G, h = 3.5, 1e-6
    _, dG = A.adjoint_step(f, lam_next, O.Params((0.9, 1.1), G))
    Lp = np.sum(lam_next * O.step(f, O.Params((0.9, 1.1), G + h)))
    Lm = np.sum(lam_next * O.step(f, O.Params((0.9, 1.1), G - h)))
    fd = (Lp - Lm) / (2 * h)
    assert abs(fd - dG) <= 1e-7 * max(1.0, abs(dG))


def test_adjoint_is_linear_and_zero_for_zero_seed():
    shape = (3, 4, 4)
    f = _state(shape, 5)
    p = O.Params((1.0, 1.0), 3.5)
    rng = np.random.default_rng(6)
    l1, l2 = rng.standard_normal(f.shape), rng.standard_normal(f.shape)
    a1, g1 = A.adjoint_step(f, l1, p)
    a2, g2 = A.adjoint_step(f, l2, p)
    a3, g3 = A.adjoint_step(f, 2.0 * l1 - l2, p)
    np.testing.assert_allclose(a3, 2.0 * a1 - a2, atol=1e-12)
    assert abs(g3 - (2.0 * g1 - g2)) < 1e-10
    z, gz = A.adjoint_step(f, np.zeros_like(l1), p)
    assert np.all(z == 0.0) and gz == 0.0


@pytest.mark.parametrize("with_solid", [False, True])
def test_full_horizon_gradient_matches_central_differences(with_solid):
    shape = (5, 5, 6)
    steps = 15
    solid = _solid((5, 5, 6)) if with_solid else None
    p = O.Params((1.0, 1.0), 3.5)
    a, b = synth.fluid_fields(shape, 0.02, 7)
    target = synth.smooth_target(shape, 8)
    J, ga, gb, dG = A.gradient(a, b, target, p, steps, solid)

    def J_of(ra, G=p.G):
        f = O.init_equilibrium(ra, b, solid=solid)
        f = O.step(f, O.Params(p.tau, G), solid, n=steps)
        return A.objective(f, target, solid)

    sites = synth.sample_sites(shape, 6, 9, exclude=solid)
    for (x, y, z) in sites:
        errs = []
        for h in (1e-5, 5e-6):
            ap, am = a.copy(), a.copy()
            ap[z, y, x] += h
            am[z, y, x] -= h
            errs.append((J_of(ap) - J_of(am)) / (2 * h))
        fd = errs[1]
        # Richardson agreement of the two step sizes bounds the FD error itself
        assert abs(errs[0] - errs[1]) <= 1e-7 * max(1e-3, abs(fd))
        assert abs(fd - ga[z, y, x]) <= 1e-6 * max(1e-3, abs(fd)), ((x, y, z), fd, ga[z, y, x])
    h = 1e-6
    fdG = (J_of(a, p.G + h) - J_of(a, p.G - h)) / (2 * h)
    assert abs(fdG - dG) <= 1e-6 * max(1e-3, abs(fdG))
    if solid is not None:
        assert np.all(ga[solid.astype(bool)] == 0.0)
