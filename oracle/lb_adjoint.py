"""FP64 discrete adjoint of the oracle step (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU baseline use this
module; it imports nothing from the GPU library.

For one step f(t) -> f(t+1) (see lb_oracle), given lam(t+1) = dJ/df(t+1) it
returns lam(t) = dJ/df(t) and the step's contribution to dJ/dG.  The
derivation follows the forward definitions term by term:

  streaming transpose   a_i(x) = lam_i(x + c_i)        if x + c_i is fluid
                               = lam_opp(i)(x)         if x + c_i is solid
  collision             f*_i = (1 - w) f_i + w feq_i(rho_k, v_k)
                        feq_i = w_i rho E_i,  E_i = 1 + 3 cu + 4.5 cu^2 - 1.5 vv
                        dfeq_i/drho = w_i E_i,  dfeq_i/dv = w_i rho (3 c_i + 9 cu c_i - 3 v)
  velocity shift        v_k = u' - a_k S_k,  a_k = tau_k G g(rho_k),  g = psi / rho
                        u' = (sum_k om_k m_k) / D,  D = sum_k om_k rho_k
  force stencil         S_k(x) = sum_j w_j psi_kbar(x + c_j) c_j,  psi = rho0 (1 - exp(-rho/rho0))

With A_k = sum_i a_i om_k w_i E_i, V_k = sum_i a_i om_k dfeq_i/dv (= dJ/dv_k),
U = V_A + V_B (= dJ/du'), W_k = a_k V_k (= -dJ/dS_k):

  lam_j^k(x) = (1 - om_k) a_j^k(x) + R_k(x) + c_j . (om_k U(x) / D(x))
  R_k(x)     = A_k - om_k (U . u') / D - (V_k . S_k) tau_k G g'(rho_k)
               - psi'(rho_k(x)) sum_j w_j c_j . W_kbar(x - c_j)
  dJ/dG     += sum_x sum_k -(V_k . S_k) tau_k g(rho_k)

Solid nodes carry no populations, so lam is zero there and psi = 0 is a
constant (no gradient flows into it).  The initial state f = w_i rho_k (fluid
at rest) gives dJ/drho_k(x, 0) = sum_i w_i lam_i^k(x, 0).
"""

from __future__ import annotations

from typing import Optional

import numpy as np

from . import lb_oracle as O


def _g(rho, ref):
    """g = psi / rho and g' = (psi' rho - psi) / rho^2, with their limits at rho = 0."""
    psi = ref * (1.0 - np.exp(-rho / ref))
    dpsi = np.exp(-rho / ref)
    zero = rho == 0.0
    r = np.where(zero, 1.0, rho)
    g = np.where(zero, 1.0, psi / r)
    dg = np.where(zero, -0.5 / ref, (dpsi * r - psi) / (r * r))
    return psi, dpsi, g, dg


def adjoint_step(f: np.ndarray, lam_next: np.ndarray, p: O.Params, solid: Optional[np.ndarray] = None):
    """(lam(t), dJ/dG contribution) from the pre-collision state f(t) and lam(t+1)."""
    s = None if solid is None else np.asarray(solid).astype(bool)
    om = p.omega
    C = O.C
    W = O.W
    # forward quantities at t
    rho = [O.density(f[k]) for k in range(2)]
    if s is not None:
        rho = [np.where(s, 0.0, r) for r in rho]
    m = [np.stack(O.momentum(f[k])) for k in range(2)]
    psi, dpsi, g, dg = [], [], [], []
    for k in range(2):
        a, b, c_, d = _g(rho[k], p.psi_ref)
        if s is not None:
            a = np.where(s, 0.0, a)
        psi.append(a)
        dpsi.append(b)
        g.append(c_)
        dg.append(d)
    S = [np.stack(O.sc_sum(psi[1])), np.stack(O.sc_sum(psi[0]))]
    D = om[0] * rho[0] + om[1] * rho[1]
    if s is not None:
        D = np.where(s, 1.0, D)
    up = (om[0] * m[0] + om[1] * m[1]) / D
    ak = [p.tau[k] * p.G * g[k] for k in range(2)]
    v = [up - ak[k] * S[k] for k in range(2)]

    # streaming transpose
    a = np.empty_like(lam_next)
    for i in range(O.Q):
        a[:, i] = O._neighbour(lam_next[:, i], C[i])
        if s is not None:
            dst_solid = O._neighbour(s, C[i])
            a[:, i] = np.where(dst_solid, lam_next[:, O.OPP[i]], a[:, i])

    A, V = [], []
    for k in range(2):
        vv = (v[k] * v[k]).sum(axis=0)
        Ak = np.zeros_like(rho[k])
        Vk = np.zeros_like(v[k])
        for i in range(O.Q):
            ci = C[i].astype(np.float64)[:, None, None, None]
            cu = (ci * v[k]).sum(axis=0)
            E = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * vv
            Ak = Ak + a[k, i] * om[k] * W[i] * E
            Vk = Vk + a[k, i] * om[k] * W[i] * rho[k] * (3.0 * ci + 9.0 * cu * ci - 3.0 * v[k])
        A.append(Ak)
        V.append(Vk)
    U = V[0] + V[1]
    dJdG = 0.0
    lam = np.empty_like(lam_next)
    Wk = [ak[k] * V[k] for k in range(2)]
    for k in range(2):
        kb = 1 - k
        VS = (V[k] * S[k]).sum(axis=0)
        # psi-stencil term: psi_k(x) enters S_kbar(x - c_j) with weight w_j c_j
        T = np.zeros_like(rho[k])
        for j in range(1, O.Q):
            cj = C[j].astype(np.float64)[:, None, None, None]
            T = T + W[j] * (cj * O._shift(Wk[kb], C[j])).sum(axis=0)
        R = A[k] - om[k] * (U * up).sum(axis=0) / D - VS * p.tau[k] * p.G * dg[k] - dpsi[k] * T
        Mk = om[k] * U / D
        for j in range(O.Q):
            cj = C[j].astype(np.float64)[:, None, None, None]
            lam[k, j] = (1.0 - om[k]) * a[k, j] + R + (cj * Mk).sum(axis=0)
        contrib = -VS * p.tau[k] * g[k]
        if s is not None:
            contrib = np.where(s, 0.0, contrib)
        dJdG += float(contrib.sum())
    if s is not None:
        lam[:, :, s] = 0.0
    return lam, dJdG


def density_gradient_seed(dJ_drho_a: np.ndarray, dJ_drho_b: np.ndarray, solid=None) -> np.ndarray:
    """lam(T) for an objective of the final densities: dJ/df_i^k = dJ/drho_k for every i."""
    lam = np.empty((2, O.Q) + dJ_drho_a.shape, dtype=np.float64)
    lam[0] = dJ_drho_a[None]
    lam[1] = dJ_drho_b[None]
    if solid is not None:
        lam[:, :, np.asarray(solid).astype(bool)] = 0.0
    return lam


def initial_density_gradient(lam0: np.ndarray):
    """dJ/drho_k(x, 0) = sum_i w_i lam_i^k(x, 0) for f(x, 0) = w_i rho_k(x)."""
    return tuple(np.tensordot(O.W, lam0[k], axes=(0, 0)) for k in range(2))


def objective(f_T: np.ndarray, target: np.ndarray, solid=None) -> float:
    """J = sum_x (rho_A(x, T) - target(x))^2 over fluid nodes."""
    r = O.density(f_T[0])
    d = r - target
    if solid is not None:
        d = np.where(np.asarray(solid).astype(bool), 0.0, d)
    return float(np.sum(d * d))


def gradient(rho_a0, rho_b0, target, p: O.Params, steps: int, solid=None):
    """(J, dJ/drho_A(0), dJ/drho_B(0), dJ/dG) for J = sum (rho_A(T) - target)^2."""
    f = O.init_equilibrium(rho_a0, rho_b0, solid=solid)
    states = [f]
    for _ in range(steps):
        f = O.step(f, p, solid)
        states.append(f)
    J = objective(f, target, solid)
    r = O.density(f[0])
    g_a = 2.0 * (r - target)
    if solid is not None:
        g_a = np.where(np.asarray(solid).astype(bool), 0.0, g_a)
    lam = density_gradient_seed(g_a, np.zeros_like(g_a), solid)
    dJdG = 0.0
    for t in range(steps - 1, -1, -1):
        lam, dg = adjoint_step(states[t], lam, p, solid)
        dJdG += dg
    ga, gb = initial_density_gradient(lam)
    return J, ga, gb, dJdG
