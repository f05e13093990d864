"""FP64 CPU oracle for the colour-gradient two-component step with moving
rigid spheres: the paper's case 3 (two immiscible fluids with colloidal
particles, Sec. 5, particle table).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this module; the GPU library never
does, and this module imports nothing from it.

What it follows:

* The colour-gradient collision of ``lb_cg`` (Appendix: BGK with the mean
  viscosity's omega, perturbation, recolouring) at every fluid node.
* The particle solver of ``lb_particles`` (Sec. 2 and Eq. PARDYN; the step
  order of Sec. 3; Appendix Eqs. UPI, LADDFLBE, FORCEPP, FORCEPARTEQ,
  TORQUEPARTEQ): particle nodes are solid, links from fluid nodes bounce
  back with the moving-wall term, the particles receive the momentum the
  links exchange, leap-frog, then covering and uncovering.  Particle
  arithmetic is float64 and each particle's sums are correctly rounded.

Readings for two components (the paper defers them to LBsoft):

* CP1, wetting.  The paper sets the particles' wettability to a 90 degree
  contact angle (Sec. 5).  Neutral wetting is read as a wall across which
  the phase field has no gradient: in the stencil
  grad Theta(x) = 3 sum_i w_i Theta(x + c_i) c_i of a fluid node x, a
  neighbour x + c_i inside a particle contributes the node's own Theta(x).
  A flat interface meeting a flat wall at right angles is then at rest
  (pinned).  Solid nodes do not collide and hold zero populations.
* CP2, the moving-wall term per component.  Each component bounces back
  with its own density: for the link from fluid node x into particle node
  x + c_i, f^k_ibar(x, t+1) = f^k*_i(x) - W^k_i with
  W^k_i = 2 rho^k(x) w_i (u_b . c_i) / c_s^2, so that the two components
  together carry the single-fluid term of the mixture density (Eq. LADDFLBE
  with rho = rho^1 + rho^2).  The particle receives
  c_i (f^k*_i(x) + f^k_ibar(x, t+1)) = c_i (2 f^k_ibar + W^k_i) from each
  component of each link (Eq. FORCEPP without its interior-fluid term).
* CP3, uncovering.  A node the move uncovers starts at
  f^k_i = f^eq_i(rho0^k, u_b) for each component, rho0 from the parameters,
  and takes that momentum from the particle (the single-fluid reading, per
  component).  The case-3 workloads use rho0 = (1/2, 1/2): a node of the
  fluids' total density and neutral colour, which the recolouring then
  sorts.  A covered node hands the momentum of both components to the
  particle.  Masses are therefore not conserved exactly while particles
  move.

Operation order of the float64 terms: as ``lb_cg`` for the collision (with
the wetting stencil above, neighbour terms in index order) and as
``lb_particles`` for the wall term, the link force and torque, per
component.
"""

from __future__ import annotations

import dataclasses
from typing import Tuple

import numpy as np

from . import lb_cg as CG
from . import lb_oracle as O
from . import lb_particles as PT

Q = O.Q
C = O.C
W = O.W
OPP = O.OPP
FLUID = PT.FLUID


@dataclasses.dataclass(frozen=True)
class Params:
    """Colour-gradient parameters and the component densities rho0 of
    uncovered nodes."""

    tau: Tuple[float, float] = (1.0, 1.0)
    sigma: float = 0.0
    beta: float = 0.0
    rho0: Tuple[float, float] = (0.5, 0.5)

    @property
    def cg(self) -> CG.Params:
        return CG.Params(self.tau, self.sigma, self.beta)


def gradient_wetting(theta: np.ndarray, solid: np.ndarray):
    """grad Theta = 3 sum_{i=1..18} w_i Theta'(x + c_i) c_i with Theta' = Theta(x)
    where x + c_i is solid (CP1), neighbour terms in index order."""
    S = [np.zeros_like(theta) for _ in range(3)]
    for i in range(1, Q):
        nb = O._neighbour(theta, C[i])
        nb_solid = O._neighbour(solid, C[i])
        t = W[i] * np.where(nb_solid, theta, nb)
        for a in range(3):
            S[a] = S[a] + C[i, a] * t
    return tuple(3.0 * S[a] for a in range(3))


def collide(f: np.ndarray, p: Params, solid: np.ndarray) -> np.ndarray:
    """Colour-gradient collision at the fluid nodes, the wetting stencil of
    CP1 for the phase-field gradient; zero at solid nodes."""
    solid = np.asarray(solid, dtype=bool)
    rho1 = O.density(f[0])
    rho2 = O.density(f[1])
    rho = rho1 + rho2
    safe = np.where(solid, 1.0, rho)
    m1 = O.momentum(f[0])
    m2 = O.momentum(f[1])
    u = tuple((m1[a] + m2[a]) / safe for a in range(3))
    theta = np.where(solid, 0.0, (rho1 - rho2) / safe)
    n, gn = CG.unit_normal(gradient_wetting(theta, solid))
    r1 = np.where(solid, 0.5, rho1)  # keeps the arithmetic finite at solid nodes, whose result is discarded
    r2 = np.where(solid, 0.5, rho2)
    omega = CG.effective_omega(r1, r2, p.cg)
    A = (2.25 * p.sigma) * omega
    pert, cn = CG.perturbation(n, gn, A)
    feq = [O.equilibrium(rho1, *u), O.equilibrium(rho2, *u)]
    fstar = np.empty_like(f[0])
    for i in range(Q):
        fa = (f[0, i] + omega * (feq[0][i] - f[0, i])) + pert[i]
        fb = (f[1, i] + omega * (feq[1][i] - f[1, i])) + pert[i]
        fstar[i] = fa + fb
    out = CG.recolour(fstar, r1, r2, cn, p.beta)
    out[:, :, solid] = 0.0
    return out


def step_solid(f: np.ndarray, p: Params, solid: np.ndarray, n: int = 1) -> np.ndarray:
    """The colour-gradient step with fixed solid nodes: the collision above
    and streaming with halfway bounce-back at rest (``lb_oracle.stream``)."""
    for _ in range(int(n)):
        f = O.stream(collide(f, p, solid), solid)
    return f


def fluid_step(f: np.ndarray, p: Params, part: PT.Particles, owner: np.ndarray):
    """Collision, moving-wall bounce-back per component (CP2) and streaming.
    Returns (f(t+1), (rho^1(t), rho^2(t)))."""
    shape = f.shape[-3:]
    solid = owner != FLUID
    rho = [np.where(solid, 0.0, O.density(f[k])) for k in range(2)]
    fs = collide(f, p, solid)
    x, y, z = PT._coords(shape)
    out = np.zeros_like(f)
    for j in range(Q):
        i = OPP[j]
        src_owner = O._shift(owner, C[j])  # owner of x - c_j = x + c_i
        src_solid = src_owner != FLUID
        bounce = (~solid) & src_solid
        pidx = np.where(bounce, src_owner, 0)
        for k in range(2):
            res = np.where(src_solid, 0.0, O._shift(fs[k, j], C[j]))
            if np.any(bounce):
                Wi, _ = PT._wall(i, x, y, z, rho[k], pidx, part, shape)
                res = np.where(bounce, fs[k, i] - Wi, res)
            res[solid] = 0.0
            out[k, j] = res
    return out, rho


def link_terms(fnew: np.ndarray, rho, part: PT.Particles, owner: np.ndarray, p: int) -> np.ndarray:
    """The float64 terms [links x 2][6] of particle p: per link and component,
    (F^k_i, r_b x F^k_i) with F^k_i = c_i ((g + g) + W^k_i), g = f^k_ibar(x, t+1)."""
    shape = fnew.shape[-3:]
    nz, ny, nx = shape
    (cx, cy, cz), (zw, yw, xw) = PT._box_nodes(part, p, shape)
    mine = owner[zw, yw, xw] == p
    zw, yw, xw = zw[mine], yw[mine], xw[mine]
    out = []
    for i in range(1, Q):
        xf = (xw - C[i, 0]) % nx
        yf = (yw - C[i, 1]) % ny
        zf = (zw - C[i, 2]) % nz
        link = owner[zf, yf, xf] == FLUID
        if not np.any(link):
            continue
        xf, yf, zf = xf[link], yf[link], zf[link]
        for k in range(2):
            g = fnew[k, OPP[i], zf, yf, xf]
            Wi, rb = PT._wall(i, xf.astype(np.float64), yf.astype(np.float64), zf.astype(np.float64),
                              rho[k][zf, yf, xf], np.full(xf.shape, p), part, shape)
            t = (g + g) + Wi
            Fi = [C[i, a] * t for a in range(3)]
            Ti = [rb[1] * Fi[2] - rb[2] * Fi[1], rb[2] * Fi[0] - rb[0] * Fi[2], rb[0] * Fi[1] - rb[1] * Fi[0]]
            out.append(np.stack(Fi + Ti, axis=-1))
    return np.concatenate(out) if out else np.zeros((0, 6))


def link_forces(fnew: np.ndarray, rho, part: PT.Particles, owner: np.ndarray):
    """Force and torque on each particle: the correctly rounded sums of its terms."""
    P = part.pos.shape[0]
    F = np.zeros((P, 3))
    T = np.zeros((P, 3))
    for q in range(P):
        s = PT.exact_sums(link_terms(fnew, rho, part, owner, q))
        F[q] = s[:3]
        T[q] = s[3:]
    return F, T


def remap_terms(f: np.ndarray, part: PT.Particles, owner_old: np.ndarray, owner_new: np.ndarray, rho0, p: int):
    """Covering and uncovering of particle p for both components (CP3):
    updates f in place at the nodes p covers or uncovers and returns the
    momentum and moment terms [nodes x 2][6] the particle receives."""
    (cx, cy, cz), (zw, yw, xw) = PT._box_nodes(part, p, f.shape[-3:])
    covered = (owner_new[zw, yw, xw] == p) & (owner_old[zw, yw, xw] == FLUID)
    uncovered = (owner_old[zw, yw, xw] == p) & (owner_new[zw, yw, xw] == FLUID)
    d = [cx - part.pos[p, 0], cy - part.pos[p, 1], cz - part.pos[p, 2]]
    terms = []
    for b in np.nonzero(covered | uncovered)[0]:
        z, y, x = zw[b], yw[b], xw[b]
        db = [d[0][b], d[1][b], d[2][b]]
        for k in range(2):
            if covered[b]:
                vals = f[k, :, z, y, x].copy()
                f[k, :, z, y, x] = 0.0
                sign = 1.0
            else:
                v, w = part.vel[p], part.omg[p]
                ub = [v[0] + (w[1] * db[2] - w[2] * db[1]),
                      v[1] + (w[2] * db[0] - w[0] * db[2]),
                      v[2] + (w[0] * db[1] - w[1] * db[0])]
                vals = O.equilibrium(np.float64(rho0[k]), np.float64(ub[0]), np.float64(ub[1]), np.float64(ub[2]))
                f[k, :, z, y, x] = vals
                sign = -1.0
            mom = O.momentum(vals.reshape(Q, 1))
            mv = [sign * float(mom[a][0]) for a in range(3)]
            terms.append(mv + [db[1] * mv[2] - db[2] * mv[1], db[2] * mv[0] - db[0] * mv[2],
                               db[0] * mv[1] - db[1] * mv[0]])
    return np.array(terms, dtype=np.float64).reshape(-1, 6)


def remap(f: np.ndarray, part: PT.Particles, owner_old: np.ndarray, owner_new: np.ndarray, rho0):
    """Covering and uncovering after the move; corrects the particle
    velocities by the correctly rounded sums of the terms."""
    I = part.inertia
    for q in range(part.pos.shape[0]):
        s = PT.exact_sums(remap_terms(f, part, owner_old, owner_new, rho0, q))
        part.vel[q] = part.vel[q] + s[:3] / part.mass
        part.omg[q] = part.omg[q] + s[3:] / I
    return f


def init(rho1: np.ndarray, rho2: np.ndarray, part: PT.Particles, u=None):
    """Both fluids at f^eq(rho^k, u) outside the particles, zero inside; returns (f, owner)."""
    owner = PT.owner_map(rho1.shape, part)
    f = O.init_equilibrium(rho1, rho2, u, owner != FLUID)
    return f, owner


def step(f: np.ndarray, p: Params, part: PT.Particles, owner: np.ndarray, n: int = 1):
    """Advance fluids and particles by ``n`` steps; returns (f, part, owner)."""
    for _ in range(int(n)):
        fnew, rho = fluid_step(f, p, part, owner)
        F, T = link_forces(fnew, rho, part, owner)
        part = PT.move(part, F, T, f.shape[-3:])
        owner_new = PT.owner_map(f.shape[-3:], part)
        fnew = remap(fnew, part, owner, owner_new, p.rho0)
        f, owner = fnew, owner_new
    return f, part, owner


def total_momentum(f: np.ndarray, part: PT.Particles):
    """Fluid momentum of both components (correctly rounded) plus sum_p m v_p."""
    import math

    m = [O.momentum(f[k]) for k in range(2)]
    return np.array([math.fsum(np.concatenate([m[0][a].ravel(), m[1][a].ravel()])) +
                     math.fsum(part.mass * part.vel[:, a]) for a in range(3)])
