"""FP64 CPU oracle for the single-fluid D3Q19 step with moving rigid spheres:
the paper's particle solver.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this module; the GPU library never
does, and this module imports nothing from it.

What it follows:

* Particles are rigid spheres.  Only the exterior holds fluid; nodes inside a
  particle are solid (Sec. 2, after Jansen and Harting).
* Their motion obeys Newton's equations for position, velocity and angular
  velocity (Sec. 2, Eq. PARDYN), advanced by leap-frog.
* Per time step, in the paper's order (Sec. 3):
  1. collision at fluid nodes (BGK, Sec. 2 Eq. 1);
  2. bounce-back at particle surfaces with the moving-wall correction
     (Appendix, Eq. LADDFLBE), the surface velocity u_b = v_p + omega_p x r_b
     at the link midpoint r_b (Eq. UPI), and the force and torque on each
     particle summed over its links (Eqs. FORCEPP, FORCEPARTEQ, TORQUEPARTEQ),
     accumulated in float64;
  3. evolution of the particles;
  4. streaming.

Readings where the paper is silent, garbled, or defers to LBsoft:

* Node x belongs to particle p when (d_x d_x + d_y d_y) + d_z d_z <= R^2 with
  d = x - r_p.  A node inside two particles belongs to the lower index.  All
  particles have one radius R.
* Eq. UPI prints r_b x omega_p.  It is read as the rigid-body velocity
  omega_p x r_b; the printed order would turn the surface against the
  particle's own rotation.  r_b is the link midpoint x + c_i / 2 minus r_p,
  folded to the nearest periodic image.
* Only the exterior population is reflected (there is no interior fluid).
  For the link from fluid node x to solid node x + c_i:
  f_ibar(x, t+1) = f*_i(x) - W_i, with W_i = 2 rho(x) w_i (u_b . c_i) / c_s^2
  and rho(x) the fluid node's density.  The particle receives the momentum
  the link exchanges, F_i = c_i (f*_i(x) + f_ibar(x, t+1)) = c_i (2 f_ibar + W_i).
  This is Eq. FORCEPP without its interior-fluid term.  The torque is
  r_b x F_i.
* Leap-frog: velocities live at half steps.  Step t bounces with
  v(t - 1/2), omega(t - 1/2) and r(t).  Then v(t + 1/2) = v(t - 1/2) + F(t) / m,
  omega(t + 1/2) = omega(t - 1/2) + T(t) / I with I = (2/5) m R^2, and
  r(t + 1) = r(t) + v(t + 1/2), wrapped into the box.
* Covering and uncovering after the move (the paper defers to LBsoft).
  A node that turns solid drops its populations and hands their momentum
  sum_i c_i f_i (and its moment d x that, d = x - r_p) to the particle.  A
  node that turns fluid starts at f^eq(rho0, u_b(x)) and takes that
  population's momentum (and moment) from the particle.  The velocities are
  corrected by these totals over m and I.  A particle must move less than one
  node per step.
* Solid nodes hold zero populations.  The collision and the equilibrium are
  those of ``lb_single`` / ``lb_oracle``.

Particle sums.  The paper asks only that the force and torque on a particle
be accumulated in double precision, because the link terms largely cancel
(Sec. 5, particle paragraph).  This oracle takes the plain definition: each
component of a particle's force, torque and covering momentum is the exact
sum of its float64 terms, rounded once (math.fsum, correctly rounded).  Any
other summation of the same n terms differs from it by at most
(n - 1) u sum|t| + u |sum t|, u = 2^-53 (the bound ``sum_bound`` states).

Scalar arithmetic orders (the terms themselves):

* W_i = (6 w_i) (rho (c_i . u_b)), with
  u_b = v + (omega_y r_z - omega_z r_y, omega_z r_x - omega_x r_z, omega_x r_y - omega_y r_x).
* F_i = c_i ((g + g) + W_i) with g = f_ibar(x, t+1).
* T_i = (r_y F_z - r_z F_y, r_z F_x - r_x F_z, r_x F_y - r_y F_x).
* Distances: (d_x d_x + d_y d_y) + d_z d_z.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from . import lb_oracle as O

Q = O.Q
C = O.C
W = O.W
OPP = O.OPP
FLUID = np.iinfo(np.int32).max  # owner of a fluid node


@dataclasses.dataclass
class Particles:
    """Particle state (float64): positions at integer steps, velocities and
    angular velocities at half steps, and the force and torque of the last
    step; all [P][3]."""

    radius: float
    mass: float
    pos: np.ndarray
    vel: np.ndarray
    omg: np.ndarray
    force: Optional[np.ndarray] = None
    torque: Optional[np.ndarray] = None

    def __post_init__(self):
        self.pos = np.array(self.pos, dtype=np.float64).reshape(-1, 3)
        n = self.pos.shape[0]
        self.vel = np.zeros((n, 3)) if self.vel is None else np.array(self.vel, dtype=np.float64).reshape(n, 3)
        self.omg = np.zeros((n, 3)) if self.omg is None else np.array(self.omg, dtype=np.float64).reshape(n, 3)
        self.force = np.zeros((n, 3)) if self.force is None else np.array(self.force, dtype=np.float64)
        self.torque = np.zeros((n, 3)) if self.torque is None else np.array(self.torque, dtype=np.float64)

    @property
    def inertia(self) -> float:
        return 0.4 * self.mass * self.radius * self.radius

    def copy(self) -> "Particles":
        return Particles(self.radius, self.mass, self.pos.copy(), self.vel.copy(), self.omg.copy(),
                         self.force.copy(), self.torque.copy())


def box_size(radius: float) -> int:
    return int(math.floor(2.0 * radius)) + 4


def _box(r, radius):
    """Box origin lo (ints) and size S for a particle at r."""
    return [int(math.floor(r[a] - radius)) - 1 for a in range(3)], box_size(radius)


def owner_map(shape, part: Particles) -> np.ndarray:
    """owner[z][y][x] = lowest index of a particle containing the node, else FLUID."""
    nz, ny, nx = shape
    L = (nx, ny, nz)
    owner = np.full(shape, FLUID, dtype=np.int64)
    R2 = part.radius * part.radius
    for p in range(part.pos.shape[0]):
        lo, S = _box(part.pos[p], part.radius)
        j = np.arange(S)
        cz, cy, cx = np.meshgrid(lo[2] + j, lo[1] + j, lo[0] + j, indexing="ij")
        dx = cx - part.pos[p, 0]
        dy = cy - part.pos[p, 1]
        dz = cz - part.pos[p, 2]
        inside = (dx * dx + dy * dy) + dz * dz <= R2
        zw, yw, xw = cz[inside] % L[2], cy[inside] % L[1], cx[inside] % L[0]
        owner[zw, yw, xw] = np.minimum(owner[zw, yw, xw], p)
    return owner


def _fold(d, L):
    """Nearest periodic image of a coordinate difference."""
    d = np.where(d > 0.5 * L, d - L, d)
    return np.where(d < -0.5 * L, d + L, d)


def _coords(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def _wall(i, xf, yf, zf, rho, p_idx, part: Particles, shape):
    """W_i and r_b for links from fluid coordinates (xf, yf, zf) in direction i
    into particles p_idx (arrays of equal shape)."""
    nz, ny, nx = shape
    r = part.pos[p_idx]
    v = part.vel[p_idx]
    w = part.omg[p_idx]
    rb = [_fold((xf + 0.5 * C[i, 0]) - r[..., 0], nx),
          _fold((yf + 0.5 * C[i, 1]) - r[..., 1], ny),
          _fold((zf + 0.5 * C[i, 2]) - r[..., 2], nz)]
    ub = [v[..., 0] + (w[..., 1] * rb[2] - w[..., 2] * rb[1]),
          v[..., 1] + (w[..., 2] * rb[0] - w[..., 0] * rb[2]),
          v[..., 2] + (w[..., 0] * rb[1] - w[..., 1] * rb[0])]
    cub = (C[i, 0] * ub[0] + C[i, 1] * ub[1]) + C[i, 2] * ub[2]
    return (6.0 * W[i]) * (rho * cub), rb


def fluid_step(f: np.ndarray, tau: float, part: Particles, owner: np.ndarray):
    """Collision, moving-wall bounce-back and streaming.  Returns (f(t+1), rho(t))."""
    shape = f.shape[-3:]
    solid = owner != FLUID
    rho = O.density(f)
    m = O.momentum(f)
    den = np.where(solid, 1.0, rho)
    u = [m[a] / den for a in range(3)]
    om = 1.0 / tau
    feq = O.equilibrium(rho, u[0], u[1], u[2])
    fs = (1.0 - om) * f + om * feq
    fs[:, solid] = 0.0
    x, y, z = _coords(shape)
    out = np.zeros_like(f)
    for j in range(Q):
        i = OPP[j]
        # out_j(x) = fs_j(x - c_j) from a fluid source, or the bounce of direction i = opp(j)
        src_owner = O._shift(owner, C[j])  # owner of x - c_j = x + c_i
        pulled = O._shift(fs[j], C[j])
        src_solid = src_owner != FLUID
        bounce = solid == False  # noqa: E712
        bounce = bounce & src_solid
        res = np.where(src_solid, 0.0, pulled)
        if np.any(bounce):
            pidx = np.where(bounce, src_owner, 0)
            Wi, _ = _wall(i, x, y, z, rho, pidx, part, shape)
            res = np.where(bounce, fs[i] - Wi, res)
        res[solid] = 0.0
        out[j] = res
    return out, rho


def exact_sums(terms: np.ndarray) -> np.ndarray:
    """Correctly rounded sum of terms [n][6] per component (math.fsum)."""
    t = np.asarray(terms, dtype=np.float64).reshape(-1, 6)
    return np.array([math.fsum(t[:, d]) for d in range(6)])


def sum_bound(terms: np.ndarray) -> np.ndarray:
    """Per component, the largest difference between the correctly rounded sum
    of terms [n][6] and any sum of them evaluated by n - 1 float64 additions
    in any order: (n - 1) u sum|t| / (1 - (n - 1) u) + u |sum t|, u = 2^-53
    (the standard bound for recursive summation, plus the final rounding of
    the exact sum)."""
    t = np.asarray(terms, dtype=np.float64).reshape(-1, 6)
    u = 2.0 ** -53
    n = max(t.shape[0] - 1, 0)
    gamma = n * u / (1.0 - n * u)
    return np.array([gamma * math.fsum(np.abs(t[:, d])) + u * abs(math.fsum(t[:, d])) for d in range(6)])


def _box_nodes(part: Particles, p: int, shape):
    """Unwrapped coordinates (x, y, z float arrays in box order) and wrapped indices."""
    nz, ny, nx = shape
    lo, S = _box(part.pos[p], part.radius)
    j = np.arange(S)
    cz, cy, cx = np.meshgrid(lo[2] + j, lo[1] + j, lo[0] + j, indexing="ij")
    cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()
    return (cx, cy, cz), (cz % nz, cy % ny, cx % nx)


def link_terms(fnew: np.ndarray, rho: np.ndarray, part: Particles, owner: np.ndarray, p: int) -> np.ndarray:
    """The float64 terms (F_i, r_b x F_i) [links][6] of particle p's links in
    the step just made (fnew = f(t+1), rho = rho(t), positions and velocities
    of step t): every link from a fluid node into a node of the particle."""
    shape = fnew.shape[-3:]
    nz, ny, nx = shape
    (cx, cy, cz), (zw, yw, xw) = _box_nodes(part, p, shape)
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
        g = fnew[OPP[i], zf, yf, xf]
        Wi, rb = _wall(i, xf.astype(np.float64), yf.astype(np.float64), zf.astype(np.float64),
                       rho[zf, yf, xf], np.full(xf.shape, p), part, shape)
        t = (g + g) + Wi
        Fi = [C[i, a] * t for a in range(3)]
        Ti = [rb[1] * Fi[2] - rb[2] * Fi[1], rb[2] * Fi[0] - rb[0] * Fi[2], rb[0] * Fi[1] - rb[1] * Fi[0]]
        out.append(np.stack(Fi + Ti, axis=-1))
    return np.concatenate(out) if out else np.zeros((0, 6))


def link_forces(fnew: np.ndarray, rho: np.ndarray, part: Particles, owner: np.ndarray):
    """Force and torque on each particle: the correctly rounded sums of its link terms."""
    P = part.pos.shape[0]
    F = np.zeros((P, 3))
    T = np.zeros((P, 3))
    for p in range(P):
        s = exact_sums(link_terms(fnew, rho, part, owner, p))
        F[p] = s[:3]
        T[p] = s[3:]
    return F, T


def move(part: Particles, F: np.ndarray, T: np.ndarray, shape) -> Particles:
    """Leap-frog: v += F/m, omega += T/I, r += v (wrapped into the box)."""
    nz, ny, nx = shape
    L = np.array([nx, ny, nz], dtype=np.float64)
    q = part.copy()
    I = q.inertia
    q.vel = q.vel + F / q.mass
    q.omg = q.omg + T / I
    r = q.pos + q.vel
    r = np.where(r >= L, r - L, r)
    q.pos = np.where(r < 0.0, r + L, r)
    q.force = F.copy()
    q.torque = T.copy()
    return q


def remap_terms(f: np.ndarray, part: Particles, owner_old: np.ndarray, owner_new: np.ndarray, rho0: float, p: int):
    """Covering and uncovering of particle p (see the module docstring):
    updates f in place at the nodes p covers or uncovers and returns the
    momentum and moment terms [nodes][6] that the particle receives."""
    (cx, cy, cz), (zw, yw, xw) = _box_nodes(part, p, f.shape[-3:])
    covered = (owner_new[zw, yw, xw] == p) & (owner_old[zw, yw, xw] == FLUID)
    uncovered = (owner_old[zw, yw, xw] == p) & (owner_new[zw, yw, xw] == FLUID)
    d = [cx - part.pos[p, 0], cy - part.pos[p, 1], cz - part.pos[p, 2]]
    terms = []
    for b in np.nonzero(covered | uncovered)[0]:
        z, y, x = zw[b], yw[b], xw[b]
        db = [d[0][b], d[1][b], d[2][b]]
        if covered[b]:
            vals = f[:, z, y, x].copy()
            f[:, z, y, x] = 0.0
            sign = 1.0
        else:
            v, w = part.vel[p], part.omg[p]
            ub = [v[0] + (w[1] * db[2] - w[2] * db[1]),
                  v[1] + (w[2] * db[0] - w[0] * db[2]),
                  v[2] + (w[0] * db[1] - w[1] * db[0])]
            vals = O.equilibrium(np.float64(rho0), np.float64(ub[0]), np.float64(ub[1]), np.float64(ub[2]))
            f[:, z, y, x] = vals
            sign = -1.0
        mom = O.momentum(vals.reshape(Q, 1))
        mv = [sign * float(mom[a][0]) for a in range(3)]
        terms.append(mv + [db[1] * mv[2] - db[2] * mv[1], db[2] * mv[0] - db[0] * mv[2],
                           db[0] * mv[1] - db[1] * mv[0]])
    return np.array(terms, dtype=np.float64).reshape(-1, 6)


def remap(f: np.ndarray, part: Particles, owner_old: np.ndarray, owner_new: np.ndarray, rho0: float):
    """Covering and uncovering after the move (see the module docstring).
    Modifies f in place and corrects the particle velocities by the correctly
    rounded sums of the terms."""
    I = part.inertia
    for p in range(part.pos.shape[0]):
        s = exact_sums(remap_terms(f, part, owner_old, owner_new, rho0, p))
        part.vel[p] = part.vel[p] + s[:3] / part.mass
        part.omg[p] = part.omg[p] + s[3:] / I
    return f


def init(rho: np.ndarray, part: Particles, u=None):
    """Fluid at f^eq(rho, u) outside the particles, zero inside; returns (f, owner)."""
    from . import lb_single as S

    owner = owner_map(rho.shape, part)
    f = S.init_equilibrium(rho, u, owner != FLUID)
    return f, owner


def step(f: np.ndarray, tau: float, part: Particles, owner: np.ndarray, rho0: float = 1.0, n: int = 1):
    """Advance fluid and particles by ``n`` steps; returns (f, part, owner)."""
    for _ in range(int(n)):
        fnew, rho = fluid_step(f, tau, part, owner)
        F, T = link_forces(fnew, rho, part, owner)
        part = move(part, F, T, f.shape[-3:])
        owner_new = owner_map(f.shape[-3:], part)
        fnew = remap(fnew, part, owner, owner_new, rho0)
        f, owner = fnew, owner_new
    return f, part, owner


def total_momentum(f: np.ndarray, part: Particles):
    """Fluid momentum (correctly rounded sums) plus sum_p m v_p."""
    m = O.momentum(f)
    return np.array([math.fsum(m[a].ravel()) + math.fsum(part.mass * part.vel[:, a]) for a in range(3)])
