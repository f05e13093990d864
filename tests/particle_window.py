"""One particle step of the oracle on a periodic window around one sphere.

For a sphere with no other centre within 2R + 5 and every coordinate in
[16, L - 16], the result
near the sphere (its force, torque, position, velocities and the populations
within R + 3 of its centre) does not depend on anything the window leaves
out: the links, the covering and those populations involve only nodes within
R + 3 + sqrt 2 of the centre, none of them across the lattice's periodic
ends (where the lattice frame rounds wrapped coordinates differently).  The
window puts the centre in [16, 17), the binade of the lattice coordinate or a
finer one, so the shift is exact, and so is every coordinate difference in
both frames.  The move is taken in the
lattice's own frame, where the position's rounding lives.
"""

import numpy as np

from oracle import lb_particles as PT

WINDOW = 32


def isolated(centres, radius, shape, count, seed, margin=5.0):
    """Up to ``count`` sphere indices (seeded choice) with no other centre
    within 2R + margin (minimum image) and every coordinate in [16, L - 16]."""
    nz, ny, nx = shape
    box = np.array([nx, ny, nz], dtype=np.float64)
    d = centres[:, None, :] - centres[None, :, :]
    d -= box * np.round(d / box)
    d2 = np.einsum("ijk,ijk->ij", d, d)
    np.fill_diagonal(d2, np.inf)
    reach = 2.0 * radius + margin
    inner = np.all((centres >= 16.0) & (centres <= box - 16.0), axis=1)
    iso = np.nonzero((d2.min(axis=1) > reach * reach) & inner)[0]
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(iso, size=min(count, iso.size), replace=False))


def step_window(rho, tau, radius, mass, r, v, w, shape):
    """One oracle step of sphere (r, v, w) in a WINDOW^3 box cut from the
    lattice's initial density ``rho`` (fluid at rest).  Returns
    (force, torque, pos, vel, omega, populations, node indices, bounds) with
    the populations [19][k] at the window nodes within R + 3 of the centre,
    their flat lattice indices [k], and ``bounds`` a dict: the summation
    bounds "link" and "cover" [6] of the sphere's link and covering sums
    (``PT.sum_bound``) and "uncovered" [k], the compared nodes the step
    uncovers."""
    nz, ny, nx = shape
    j = np.arange(WINDOW)
    o = np.floor(r).astype(np.int64) - WINDOW // 2
    zi, yi, xi = np.meshgrid((o[2] + j) % nz, (o[1] + j) % ny, (o[0] + j) % nx, indexing="ij")
    here = PT.Particles(radius, mass, [r - o], [v], [w])
    f0, own0 = PT.init(rho[zi, yi, xi], here)
    f1, rho_t = PT.fluid_step(f0, tau, here, own0)
    b_link = PT.sum_bound(PT.link_terms(f1, rho_t, here, own0, 0))
    F, T = PT.link_forces(f1, rho_t, here, own0)
    moved = PT.move(PT.Particles(radius, mass, [r], [v], [w]), F, T, shape)
    there = PT.Particles(radius, mass, [moved.pos[0] - o], moved.vel, moved.omg)
    own1 = PT.owner_map((WINDOW,) * 3, there)
    b_cover = PT.sum_bound(PT.remap_terms(f1.copy(), there, own0, own1, 1.0, 0))
    f1 = PT.remap(f1, there, own0, own1, 1.0)
    zw, yw, xw = np.meshgrid(j, j, j, indexing="ij")
    c = r - o
    near = ((xw - c[0]) ** 2 + (yw - c[1]) ** 2) + (zw - c[2]) ** 2 <= (radius + 3.0) ** 2
    bz, by, bx = zw[near], yw[near], xw[near]
    idx = (((bz + o[2]) % nz * ny + (by + o[1]) % ny) * nx + (bx + o[0]) % nx).ravel()
    unc = ((own0 != PT.FLUID) & (own1 == PT.FLUID))[bz, by, bx]
    bounds = {"link": b_link, "cover": b_cover, "uncovered": unc}
    return F[0], T[0], moved.pos[0], there.vel[0], there.omg[0], f1[:, bz, by, bx], idx, bounds


def step_window_cg(r1, r2, p, radius, mass, r, v, w, shape):
    """The same for the colour-gradient fluid with particles (the paper's
    case 3): one step of ``oracle.lb_cg_particles`` with parameters ``p`` in a
    WINDOW^3 box cut from the lattice's initial densities (r1, r2) at rest.
    The phase-field stencil (and the wetting test of its neighbours) reaches
    one node further than the single fluid's collision, so the compared
    populations (within R + 3) depend on nodes within R + 4 + sqrt 2 of the
    centre, still inside the window; the sampled spheres need no other centre
    within 2R + 7 (``isolated(..., margin=7)``), so that no other sphere's
    node lies that close.  Returns
    (force, torque, pos, vel, omega, populations [2][19][k], node indices,
    bounds) as ``step_window``."""
    from oracle import lb_cg_particles as CP

    nz, ny, nx = shape
    j = np.arange(WINDOW)
    o = np.floor(r).astype(np.int64) - WINDOW // 2
    zi, yi, xi = np.meshgrid((o[2] + j) % nz, (o[1] + j) % ny, (o[0] + j) % nx, indexing="ij")
    here = PT.Particles(radius, mass, [r - o], [v], [w])
    f0, own0 = CP.init(r1[zi, yi, xi], r2[zi, yi, xi], here)
    f1, rho_t = CP.fluid_step(f0, p, here, own0)
    b_link = PT.sum_bound(CP.link_terms(f1, rho_t, here, own0, 0))
    F, T = CP.link_forces(f1, rho_t, here, own0)
    moved = PT.move(PT.Particles(radius, mass, [r], [v], [w]), F, T, shape)
    there = PT.Particles(radius, mass, [moved.pos[0] - o], moved.vel, moved.omg)
    own1 = PT.owner_map((WINDOW,) * 3, there)
    b_cover = PT.sum_bound(CP.remap_terms(f1.copy(), there, own0, own1, p.rho0, 0))
    f1 = CP.remap(f1, there, own0, own1, p.rho0)
    zw, yw, xw = np.meshgrid(j, j, j, indexing="ij")
    c = r - o
    near = ((xw - c[0]) ** 2 + (yw - c[1]) ** 2) + (zw - c[2]) ** 2 <= (radius + 3.0) ** 2
    bz, by, bx = zw[near], yw[near], xw[near]
    idx = (((bz + o[2]) % nz * ny + (by + o[1]) % ny) * nx + (bx + o[0]) % nx).ravel()
    unc = ((own0 != PT.FLUID) & (own1 == PT.FLUID))[bz, by, bx]
    bounds = {"link": b_link, "cover": b_cover, "uncovered": unc}
    return F[0], T[0], moved.pos[0], there.vel[0], there.omg[0], f1[:, :, bz, by, bx], idx, bounds
