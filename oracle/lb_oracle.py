"""FP64 CPU oracle for the two-component D3Q19 Shan-Chen lattice-Boltzmann step.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark import this module; the GPU library never does, and this
module imports nothing from it.  It is plain vectorised NumPy in float64,
written for a reader to check against the paper by eye, not for speed.

What it follows
---------------
* D3Q19 velocity set (Sec. 2): the rest vector, the 6 nearest neighbours at
  distance 1 and the 12 next-nearest at distance sqrt(2); the 8 cube corners
  are left out.
* Weights w = 1/3, 1/18, 1/36 for |c|^2 = 0, 1, 2 (Appendix, D3Q19 table).
* Two population sets f_i^k, one per component k; rho^k = sum_i f_i^k and the
  mixture momentum sum_k sum_i f_i^k c_i (Appendix, two-component LBE and the
  moment definitions that follow it).
* Second-order equilibrium (Appendix, Eq. LEQ) with c_s^2 = 1/3, i.e.
  f_i^eq = w_i rho (1 + 3 c.v + 4.5 (c.v)^2 - 1.5 v.v).
* BGK relaxation f* = (1 - omega) f + omega f^eq with omega = 1/tau (Sec. 2,
  Eq. 1), so the kinematic viscosity is c_s^2 (tau - 1/2) (Sec. 2, Eq. 2).
* Streaming f_i(x + c_i, t + 1) = f*_i(x, t) (Eq. 1), periodic on all axes, as
  in the paper's test boxes (Sec. 5).
* Halfway bounce-back at solid nodes at rest (Appendix, Eq. LADDFLBE with the
  wall velocity set to zero): a population whose source node is solid is
  replaced by the node's own post-collision population of the opposite
  direction.

The paper's two-component model is colour-gradient; the inter-component force
used here is the Shan-Chen pseudopotential force, which the paper does not
describe.  Readings taken where the paper is silent:

* Pseudopotential psi_k = rho_0 (1 - exp(-rho_k / rho_0)), Shan and Chen's
  original form, with rho_0 = 1.  (With psi = rho the coupling G = 3.5 of the
  spinodal workloads blows up within a dozen steps; with this psi it demixes
  and stays bounded.)
* S_k(x) = sum_{i=1..18} w_i psi_kbar(x + c_i) c_i with the D3Q19 weights
  above; F_k = -G psi_k S_k (G > 0 demixes).  Solid nodes count as rho = 0,
  hence psi = 0, in this sum.
* Forcing by velocity shift: common velocity
  u' = (sum_k omega_k m_k) / (sum_k omega_k rho_k), m_k = sum_i f_i^k c_i, and
  each component relaxes towards f^eq(rho_k, v_k) with
  v_k = u' + tau_k F_k / rho_k = u' - (tau_k G)(psi_k / rho_k) S_k, where
  psi_k / rho_k takes its limit 1 at rho_k = 0.
* State = pre-collision populations f(t); one step = densities, force,
  collision, streaming.  Solid nodes do not collide; their populations are 0.
* Output velocity (moments): u = (sum_k m_k + (F_A + F_B) / 2) / (rho_A + rho_B).
* Densities may dip slightly below zero in a demixed state; nothing here
  forbids it.

Order of floating-point operations (fixed so that an independent
implementation performing the same IEEE operations in the same order agrees
bit for bit):

* rho = ((f_0 + f_1) + f_2) + ... + f_18, in index order.
* m_a = sum over i = 0..18 of c_ia f_i, accumulated in index order from 0
  (terms with c_ia = 0 add a signed zero and change nothing else).
* psi = rho_0 (1 - e) with e = exp_cw(-(rho / rho_0)) below (a fixed
  sequence of IEEE operations, so that it is reproducible bit for bit).
* S_a = sum over i = 1..18 of c_ia (w_i psi(x + c_i)), in index order from 0.
* den = omega_A rho_A + omega_B rho_B;
  u'_a = (omega_A m_Aa + omega_B m_Ba) / den.
* a_k = (tau_k G)(psi_k / rho_k), the product tau_k G formed first;
  v_ka = u'_a - a_k S_ka.
* v.v = (v_x v_x + v_y v_y) + v_z v_z;  c.v = (c_x v_x + c_y v_y) + c_z v_z;
  f^eq_i = (w_i rho) (((1 + 3 c.v) + (4.5 c.v) c.v) - 1.5 v.v).
* f* = (1 - omega) f + omega f^eq, with 1 - omega formed first.
* No fused multiply-add anywhere (NumPy evaluates each product and sum
  separately).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# D3Q19 lattice (Sec. 2; weights from the Appendix table).
# Index order: 0 rest; 1..6 the axis neighbours (+x, -x, +y, -y, +z, -z);
# 7..18 the face diagonals in opposite pairs.
# ---------------------------------------------------------------------------
C = np.array(
    [
        [0, 0, 0],
        [1, 0, 0], [-1, 0, 0],
        [0, 1, 0], [0, -1, 0],
        [0, 0, 1], [0, 0, -1],
        [1, 1, 0], [-1, -1, 0],
        [1, -1, 0], [-1, 1, 0],
        [1, 0, 1], [-1, 0, -1],
        [1, 0, -1], [-1, 0, 1],
        [0, 1, 1], [0, -1, -1],
        [0, 1, -1], [0, -1, 1],
    ],
    dtype=np.int64,
)
Q = 19
W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12, dtype=np.float64)
OPP = np.array([int(np.nonzero((C == -C[i]).all(axis=1))[0][0]) for i in range(Q)], dtype=np.int64)
CS2 = 1.0 / 3.0


@dataclasses.dataclass(frozen=True)
class Params:
    """Relaxation times per component (tau > 1/2), the coupling G and the
    reference density rho_0 of the pseudopotential psi = rho_0 (1 - exp(-rho / rho_0))."""

    tau: Tuple[float, float] = (1.0, 1.0)
    G: float = 0.0
    psi_ref: float = 1.0

    @property
    def omega(self) -> Tuple[float, float]:
        return (1.0 / self.tau[0], 1.0 / self.tau[1])


def _shift(a: np.ndarray, c) -> np.ndarray:
    """out[z, y, x] = a[z - c_z, y - c_y, x - c_x] with periodic wrap."""
    return np.roll(a, shift=(int(c[2]), int(c[1]), int(c[0])), axis=(-3, -2, -1))


def _neighbour(a: np.ndarray, c) -> np.ndarray:
    """out[x] = a[x + c] with periodic wrap."""
    return _shift(a, (-c[0], -c[1], -c[2]))


# ---------------------------------------------------------------------------
# Local quantities
# ---------------------------------------------------------------------------
def equilibrium(rho: np.ndarray, vx: np.ndarray, vy: np.ndarray, vz: np.ndarray) -> np.ndarray:
    """f_i^eq(rho, v) for i = 0..18 (Appendix, Eq. LEQ, c_s^2 = 1/3)."""
    vv = (vx * vx + vy * vy) + vz * vz
    out = np.empty((Q,) + np.shape(rho), dtype=np.float64)
    for i in range(Q):
        cu = (C[i, 0] * vx + C[i, 1] * vy) + C[i, 2] * vz
        out[i] = (W[i] * rho) * (((1.0 + 3.0 * cu) + 4.5 * cu * cu) - 1.5 * vv)
    return out


def density(fk: np.ndarray) -> np.ndarray:
    """rho^k = sum_i f_i^k, accumulated in index order."""
    rho = fk[0].copy()
    for i in range(1, Q):
        rho = rho + fk[i]
    return rho


def momentum(fk: np.ndarray):
    """m^k = sum_i f_i^k c_i, accumulated in index order."""
    out = []
    for a in range(3):
        m = np.zeros_like(fk[0])
        for i in range(Q):
            m = m + C[i, a] * fk[i]
        out.append(m)
    return tuple(out)


# e^x by Cody-Waite range reduction and a Taylor polynomial (Cody & Waite,
# "Software Manual for the Elementary Functions", 1980): n = rint(x / ln 2),
# r = (x - n ln2_hi) - n ln2_lo with |r| <= ln(2)/2, e^r = sum_{k<=13} r^k / k!
# by Horner's rule, e^x = 2^n e^r.  The degree-13 truncation error is below
# 1e-17 relative on |r| <= ln(2)/2.  ln2_hi keeps 32 significant bits so that
# n * ln2_hi is exact for |n| < 2^21.
LN2_HI = float.fromhex("0x1.62e42fee00000p-1")
LN2_LO = float.fromhex("0x1.a39ef35793c76p-33")
INV_LN2 = float.fromhex("0x1.71547652b82fep+0")
EXP_DEGREE = 13
EXP_COEF = [1.0 / math.factorial(k) for k in range(EXP_DEGREE + 1)]


def exp_cw(x: np.ndarray) -> np.ndarray:
    """e^x, evaluated as described above (accurate to a couple of ulp for |x| < 700)."""
    x = np.asarray(x, dtype=np.float64)
    n = np.rint(x * INV_LN2)
    r = (x - n * LN2_HI) - n * LN2_LO
    p = np.full_like(r, EXP_COEF[EXP_DEGREE])
    for k in range(EXP_DEGREE - 1, -1, -1):
        p = p * r + EXP_COEF[k]
    return np.ldexp(p, n.astype(np.int32))


def pseudopotential(rho: np.ndarray, psi_ref: float) -> np.ndarray:
    """psi = rho_0 (1 - exp(-rho / rho_0)) (Shan & Chen's original choice); psi(0) = 0."""
    return psi_ref * (1.0 - exp_cw(-(rho / psi_ref)))


def psi_over_rho(rho: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """psi / rho, with its limit 1 where rho == 0."""
    zero = rho == 0.0
    return np.where(zero, 1.0, psi / np.where(zero, 1.0, rho))


def sc_sum(psi_other: np.ndarray):
    """S(x) = sum_{i=1..18} w_i psi_other(x + c_i) c_i (periodic)."""
    S = [np.zeros_like(psi_other) for _ in range(3)]
    for i in range(1, Q):
        t = W[i] * _neighbour(psi_other, C[i])
        for a in range(3):
            S[a] = S[a] + C[i, a] * t
    return tuple(S)


# ---------------------------------------------------------------------------
# One step
# ---------------------------------------------------------------------------
def _fluid(shape, solid: Optional[np.ndarray]) -> Optional[np.ndarray]:
    if solid is None:
        return None
    s = np.asarray(solid).astype(bool)
    if s.shape != tuple(shape):
        raise ValueError(f"solid mask shape {s.shape} != lattice {tuple(shape)}")
    return s


def collide(f: np.ndarray, p: Params, solid: Optional[np.ndarray] = None):
    """Post-collision populations f* for both components.

    Returns (fs, aux) where aux holds rho, psi, m, S and u' used on the way;
    solid nodes are left at zero.
    """
    s = _fluid(f.shape[-3:], solid)
    om = p.omega
    rho = [density(f[k]) for k in range(2)]
    if s is not None:
        for k in range(2):
            rho[k] = np.where(s, 0.0, rho[k])
    psi = [pseudopotential(rho[k], p.psi_ref) for k in range(2)]
    m = [momentum(f[k]) for k in range(2)]
    S = [sc_sum(psi[1]), sc_sum(psi[0])]
    den = om[0] * rho[0] + om[1] * rho[1]
    if s is not None:
        den = np.where(s, 1.0, den)
    up = tuple((om[0] * m[0][a] + om[1] * m[1][a]) / den for a in range(3))
    fs = np.empty_like(f)
    for k in range(2):
        # v_k = u' + tau_k F_k / rho_k with F_k = -G psi_k S_k
        a_k = (p.tau[k] * p.G) * psi_over_rho(rho[k], psi[k])
        v = [up[a] - a_k * S[k][a] for a in range(3)]
        feq = equilibrium(rho[k], v[0], v[1], v[2])
        omc = 1.0 - om[k]
        fs[k] = omc * f[k] + om[k] * feq
    if s is not None:
        fs[:, :, s] = 0.0
    return fs, {"rho": rho, "psi": psi, "m": m, "S": S, "u_common": up}


def stream(fs: np.ndarray, solid: Optional[np.ndarray] = None) -> np.ndarray:
    """Pull streaming with halfway bounce-back at rest.

    f_i(x, t+1) = f*_i(x - c_i)      if x - c_i is fluid
                = f*_opp(i)(x)       if x - c_i is solid (x fluid)
    Solid nodes end with zero populations.
    """
    s = _fluid(fs.shape[-3:], solid)
    out = np.empty_like(fs)
    for i in range(Q):
        pulled = _shift(fs[:, i], C[i])
        if s is not None:
            src_solid = _shift(s, C[i])
            pulled = np.where(src_solid, fs[:, OPP[i]], pulled)
        out[:, i] = pulled
    if s is not None:
        out[:, :, s] = 0.0
    return out


def step(f: np.ndarray, p: Params, solid: Optional[np.ndarray] = None, n: int = 1) -> np.ndarray:
    """Advance the pre-collision state ``f`` [2][19][nz][ny][nx] by ``n`` steps."""
    for _ in range(int(n)):
        fs, _ = collide(f, p, solid)
        f = stream(fs, solid)
    return f


def init_equilibrium(rho_a: np.ndarray, rho_b: np.ndarray, u=None, solid: Optional[np.ndarray] = None) -> np.ndarray:
    """f_i^k(x, 0) = f_i^eq(rho_k(x), u(x)); zero at solid nodes.  u = (ux, uy, uz) or None for rest."""
    rho_a = np.asarray(rho_a, dtype=np.float64)
    rho_b = np.asarray(rho_b, dtype=np.float64)
    if u is None:
        z = np.zeros_like(rho_a)
        u = (z, z, z)
    f = np.empty((2, Q) + rho_a.shape, dtype=np.float64)
    f[0] = equilibrium(rho_a, *u)
    f[1] = equilibrium(rho_b, *u)
    s = _fluid(rho_a.shape, solid)
    if s is not None:
        f[:, :, s] = 0.0
    return f


def moments(f: np.ndarray, p: Params, solid: Optional[np.ndarray] = None):
    """(rho_A, rho_B, (ux, uy, uz)) of the pre-collision state.

    u = (m_A + m_B + (F_A + F_B) / 2) / (rho_A + rho_B) with F_k = -G psi_k S_k;
    zero at solid nodes.
    """
    s = _fluid(f.shape[-3:], solid)
    rho = [density(f[k]) for k in range(2)]
    if s is not None:
        for k in range(2):
            rho[k] = np.where(s, 0.0, rho[k])
    psi = [pseudopotential(rho[k], p.psi_ref) for k in range(2)]
    m = [momentum(f[k]) for k in range(2)]
    S = [sc_sum(psi[1]), sc_sum(psi[0])]
    tot = rho[0] + rho[1]
    if s is not None:
        tot = np.where(s, 1.0, tot)
    u = []
    for a in range(3):
        FA = (-p.G * psi[0]) * S[0][a]
        FB = (-p.G * psi[1]) * S[1][a]
        ua = ((m[0][a] + m[1][a]) + 0.5 * (FA + FB)) / tot
        if s is not None:
            ua = np.where(s, 0.0, ua)
        u.append(ua)
    return rho[0], rho[1], tuple(u)


def totals(f: np.ndarray):
    """Conserved totals (M_A, M_B, P_x, P_y, P_z) and a non-finite flag.

    Masses are sums of rho_k over all nodes; P = sum_x sum_k m_k.  Each total
    is a correctly rounded sum (math.fsum).
    """
    nonfinite = not bool(np.all(np.isfinite(f)))
    M = [math.fsum(density(f[k]).ravel()) for k in range(2)]
    P = []
    mA = momentum(f[0])
    mB = momentum(f[1])
    for a in range(3):
        P.append(math.fsum(np.concatenate([mA[a].ravel(), mB[a].ravel()])))
    return (M[0], M[1], P[0], P[1], P[2]), nonfinite


def population_error(f_test: np.ndarray, f_ref: np.ndarray) -> float:
    """max over k, i, x of |f_test - f_ref| / max(|f_ref|, 1e-3 w_i).

    The floor 1e-3 w_i keeps populations that pass near zero from inflating
    the relative error.
    """
    f_test = np.asarray(f_test, dtype=np.float64)
    f_ref = np.asarray(f_ref, dtype=np.float64)
    floor = (1e-3 * W).reshape((1, Q) + (1,) * (f_ref.ndim - 2))
    return float(np.max(np.abs(f_test - f_ref) / np.maximum(np.abs(f_ref), floor)))
