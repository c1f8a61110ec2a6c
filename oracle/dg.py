"""Weak-form nodal DGSEM residual of the 3D compressible Navier-Stokes equations.

Test infrastructure only (see ``oracle/__init__``).

What is computed, and where the paper defines it:

* conserved state q = (rho, rho u, rho v, rho w, rho e) at every DOF, Eq. (1);
* inviscid flux f^a and viscous flux f^nu with the Stokes stress tensor and a
  heat flux kappa grad T, App. A (the "rho u_3" entry of the first row of f^a is
  read as rho v_3);
* Roe's approximate Riemann solver for the advective interface flux and Bassi-
  Rebay 1 (BR1) for the viscous one, Sec. 3.1;
* Smagorinsky eddy viscosity as the optional LES closure, Sec. 3.1 / Table 1;
* the discrete operator p(q) of Eq. (1)/(3): the weak-form DGSEM on uniform,
  affine, periodic hexahedra with Gauss-Legendre nodes (Sec. 2.6);
* the Taylor-Green vortex initial condition, Eq. (11);
* the CFL time step of Eq. (7) (with the (P+1)^2 scaling that the printed time
  steps of Tables 1 and 2 follow);
* diagnostics: kinetic energy, the infinity-norm error of Eq. (9), totals.

Array layout.  A field is an array ``A[..., ez, ey, ex, k, j, i]``: three
element axes followed by three node axes (i along x).  The flat layout used at
the library boundary, ``q[v][e][n]`` with e = ex + N (ey + N ez) and
n = i + (P+1)(j + (P+1) k), is exactly this array reshaped.

Readings of points the paper leaves open:
gamma = 1.4, Pr = 0.72, mu = 1/Re constant, T == p/rho (so kappa = mu gamma /
((gamma-1) Pr)), Smagorinsky filter width h/(P+1) and Pr_t = 0.6, no entropy
fix in the Roe solver, BR1 common value = mean of the primitive variables
computed from each side's traced conserved state, viscous interface flux =
mean of the two one-sided viscous fluxes, and a constant reference pressure
p_ref subtracted from the momentum fluxes (a constant flux has zero weak
divergence, so p(q) changes only by rounding).
"""
from dataclasses import dataclass

import numpy as np

from .basis import Basis

NVAR = 5


@dataclass
class Params:
    """Physical and discretisation parameters of one TGV solve (Sec. 3.1)."""
    N: int                 # elements per direction
    P: int                 # polynomial order
    Re: float              # Reynolds number rho0 V0 L / mu
    Mach: float = 0.1      # M0 of Eq. (11)
    gamma: float = 1.4
    Pr: float = 0.72
    Cs: float = 0.0        # Smagorinsky constant; 0 switches the closure off
    Pr_t: float = 0.6      # turbulent Prandtl number of the closure
    L: float = 2.0 * np.pi  # box side; the TGV box is [0, 2 pi]^3
    viscous: bool = True   # False: Euler equations (no BR1 / viscous terms)
    p_ref: float = None    # subtracted from momentum fluxes; None -> p0

    def __post_init__(self):
        self.h = self.L / self.N
        self.s = 2.0 / self.h                     # d/dx = s d/dxi
        self.J = (self.h / 2.0) ** 3              # volume Jacobian
        self.mu = 1.0 / self.Re                   # rho0 = V0 = 1, unit length
        self.p0 = 1.0 / (self.gamma * self.Mach ** 2)
        if self.p_ref is None:
            self.p_ref = self.p0
        self.kappa = self.mu * self.gamma / ((self.gamma - 1.0) * self.Pr)
        self.delta = self.h / (self.P + 1)        # LES filter width


# ----------------------------------------------------------------- layout helpers

def node_axis(d):
    return -1 - d


def elem_axis(d):
    return -4 - d


def to_blocks(q_flat, N, P):
    """q[v][e][n] -> A[v, ez, ey, ex, k, j, i]."""
    n = P + 1
    return np.asarray(q_flat, dtype=np.float64).reshape(NVAR, N, N, N, n, n, n)


def to_flat(A):
    N = A.shape[-4]
    n = A.shape[-1]
    return A.reshape(A.shape[0], N ** 3, n ** 3)


def along(vec, d):
    """Shape ``vec`` so that it broadcasts along the node axis of direction d."""
    return np.asarray(vec).reshape((-1,) + (1,) * d)


def apply_line(A, M, d):
    """out[.., a, ..] = sum_m M[a, m] A[.., m, ..] along the node axis of d."""
    ax = node_axis(d)
    out = np.moveaxis(A, ax, -1) @ np.asarray(M).T
    return np.moveaxis(out, -1, ax)


def trace(A, b, d):
    """Value at a face of direction d: sum_m b_m A_m along the normal line
    (Gauss points have no end points); keeps a length-1 node axis."""
    return apply_line(A, np.asarray(b)[None, :], d)


def upper(F, d):
    """F of the neighbour at +1 in direction d (periodic)."""
    return np.roll(F, -1, axis=elem_axis(d))


def lower(F, d):
    """F of the neighbour at -1 in direction d (periodic)."""
    return np.roll(F, 1, axis=elem_axis(d))


# ------------------------------------------------------------ thermodynamics

def velocity(q):
    return q[1:4] / q[0]


def pressure(q, gamma):
    vel = velocity(q)
    return (gamma - 1.0) * (q[4] - 0.5 * q[0] * np.sum(vel * vel, axis=0))


def gradient_variables(q, gamma):
    """BR1 gradient variables w = (u, v, w, theta), theta = p / rho (= T, R = 1)."""
    vel = velocity(q)
    theta = pressure(q, gamma) / q[0]
    return np.concatenate([vel, theta[None]], axis=0)


# --------------------------------------------------------------------- fluxes

def inviscid_flux(q, d, prm):
    """Row d of f^a (App. A) with p_ref removed from the momentum rows."""
    vel = velocity(q)
    p = pressure(q, prm.gamma)
    vd = vel[d]
    F = np.empty_like(q)
    F[0] = q[1 + d]
    F[1:4] = q[1:4] * vd
    F[1 + d] = F[1 + d] + (p - prm.p_ref)
    F[4] = (q[4] + p) * vd
    return F


def roe_waves(qL, qR, d, gamma):
    """Roe-averaged eigen-decomposition of the jump qR - qL along direction d.

    Returns a list of (lambda_k, alpha_k * r_k) pairs: eigenvalue and wave.
    Roe (1981): rho~ = sqrt(rhoL rhoR), v~ and H~ are sqrt(rho)-weighted means,
    c~^2 = (gamma-1)(H~ - |v~|^2/2).  Waves: acoustic v~_d -/+ c~, entropy,
    and two shear waves, all moving at v~_d.
    """
    rL, rR = qL[0], qR[0]
    vL, vR = velocity(qL), velocity(qR)
    pL, pR = pressure(qL, gamma), pressure(qR, gamma)
    HL = (qL[4] + pL) / rL
    HR = (qR[4] + pR) / rR
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    rt = sL * sR
    vt = (sL * vL + sR * vR) / (sL + sR)
    Ht = (sL * HL + sR * HR) / (sL + sR)
    v2 = np.sum(vt * vt, axis=0)
    ct = np.sqrt((gamma - 1.0) * (Ht - 0.5 * v2))
    vn = vt[d]

    drho = rR - rL
    dv = vR - vL
    dp = pR - pL

    a_minus = (dp - rt * ct * dv[d]) / (2.0 * ct * ct)
    a_plus = (dp + rt * ct * dv[d]) / (2.0 * ct * ct)
    a_entropy = drho - dp / (ct * ct)

    def vec(rho_c, mom, ene):
        return np.concatenate([rho_c[None], mom, ene[None]], axis=0)

    one = np.ones_like(rt)
    ed = np.zeros((3,) + rt.shape)
    ed[d] = 1.0
    waves = [
        (vn - ct, a_minus * vec(one, vt - ct * ed, Ht - ct * vn)),
        (vn, a_entropy * vec(one, vt, 0.5 * v2)),
        (vn + ct, a_plus * vec(one, vt + ct * ed, Ht + ct * vn)),
    ]
    for t in range(3):
        if t == d:
            continue
        et = np.zeros((3,) + rt.shape)
        et[t] = 1.0
        waves.append((vn, (rt * dv[t]) * vec(np.zeros_like(rt), et, vt[t])))
    return waves


def roe_flux(qL, qR, d, prm):
    """Roe flux along +d, qL on the lower side: the central average minus half
    the |lambda|-weighted waves.  No entropy fix."""
    F = 0.5 * (inviscid_flux(qL, d, prm) + inviscid_flux(qR, d, prm))
    for lam, wave in roe_waves(qL, qR, d, prm.gamma):
        F = F - 0.5 * np.abs(lam) * wave
    return F


def smagorinsky_mu(rho, g, prm):
    """mu_t = rho (Cs Delta)^2 sqrt(2 S:S), S = (grad v + grad v^T) / 2.
    g[j, a] = d_j w_a with w = (u, v, w, theta)."""
    SS = np.zeros_like(rho)
    for a in range(3):
        for b in range(3):
            S_ab = 0.5 * (g[a, b] + g[b, a])
            SS = SS + S_ab * S_ab
    return rho * (prm.Cs * prm.delta) ** 2 * np.sqrt(2.0 * SS)


def viscous_flux(q, g, d, prm):
    """Row d of f^nu (App. A): (0, tau_{1d}, tau_{2d}, tau_{3d},
    sum_a v_a tau_{ad} + kappa dT/dx_d), tau = mu (grad v + grad v^T)
    - 2/3 mu (div v) I, with mu and kappa raised by the Smagorinsky closure."""
    vel = velocity(q)
    mu = prm.mu
    kappa = prm.kappa
    if prm.Cs > 0.0:
        mut = smagorinsky_mu(q[0], g, prm)
        mu = mu + mut
        kappa = kappa + mut * prm.gamma / ((prm.gamma - 1.0) * prm.Pr_t)
    div = g[0, 0] + g[1, 1] + g[2, 2]
    F = np.zeros_like(q)
    for a in range(3):
        tau_ad = mu * (g[a, d] + g[d, a])
        if a == d:
            tau_ad = tau_ad - (2.0 / 3.0) * mu * div
        F[1 + a] = tau_ad
        F[4] = F[4] + vel[a] * tau_ad
    F[4] = F[4] + kappa * g[d, 3]
    return F


# ------------------------------------------------------------------ operators

def weak_derivative(F, Fhat_p, Fhat_m, basis, d, s):
    """Weak-form derivative along d of a nodal field F with interface values
    Fhat_p (upper face) and Fhat_m (lower face): multiply by l_i, integrate by
    parts, Gauss quadrature, diagonal mass matrix:
        (s / w_i) [ b+_i Fhat+ - b-_i Fhat- - sum_m w_m l_i'(xi_m) F_m ]."""
    w = basis.weights
    M = (basis.D * w[:, None]).T          # M[i, m] = w_m D[m, i] = w_m l_i'(xi_m)
    vol = apply_line(F, M, d)
    return s * (along(basis.bp / w, d) * Fhat_p
                - along(basis.bm / w, d) * Fhat_m
                - vol / along(w, d))


def br1_gradient(q, prm, basis):
    """BR1 lifted gradient of w = (u, v, w, theta); result g[j, a] = d_j w_a."""
    W = gradient_variables(q, prm.gamma)
    g = []
    for d in range(3):
        w_in = gradient_variables(trace(q, basis.bp, d), prm.gamma)
        w_out = gradient_variables(upper(trace(q, basis.bm, d), d), prm.gamma)
        what_p = 0.5 * (w_in + w_out)
        what_m = lower(what_p, d)
        g.append(weak_derivative(W, what_p, what_m, basis, d, prm.s))
    return np.stack(g)


def residual(q, prm, basis=None, source=None):
    """The DG operator p(q) of Eq. (1)/(3) on the block array q[v, ez, ey, ex, k, j, i].

    R = - sum_d weak_derivative(f^a_d - f^nu_d; Roe - BR1 interface flux).
    ``source`` (same shape, optional) is added, e.g. a manufactured source."""
    if basis is None:
        basis = Basis(prm.P)
    g = br1_gradient(q, prm, basis) if prm.viscous else None
    R = np.zeros_like(q)
    for d in range(3):
        G = inviscid_flux(q, d, prm)
        qL = trace(q, basis.bp, d)
        qR = upper(trace(q, basis.bm, d), d)
        Fhat = roe_flux(qL, qR, d, prm)
        if prm.viscous:
            G = G - viscous_flux(q, g, d, prm)
            gL = trace(g, basis.bp, d)
            gR = upper(trace(g, basis.bm, d), d)
            Fhat = Fhat - 0.5 * (viscous_flux(qL, gL, d, prm) + viscous_flux(qR, gR, d, prm))
        R = R - weak_derivative(G, Fhat, lower(Fhat, d), basis, d, prm.s)
    if source is not None:
        R = R + source
    return R


# ------------------------------------------------------------- mesh and TGV

def node_coordinates(prm, basis=None):
    """Physical coordinates X, Y, Z with the block shape (ez, ey, ex, k, j, i)."""
    if basis is None:
        basis = Basis(prm.P)
    N, n, h = prm.N, basis.n, prm.h
    e = np.arange(N)
    x1 = (e[:, None] * h + (basis.nodes[None, :] + 1.0) * h / 2.0)   # [ex, i]
    X = x1[None, None, :, None, None, :]
    Y = x1[None, :, None, None, :, None]
    Z = x1[:, None, None, :, None, None]
    shape = (N, N, N, n, n, n)
    return (np.broadcast_to(X, shape), np.broadcast_to(Y, shape), np.broadcast_to(Z, shape))


def tgv_initial_condition(prm, basis=None):
    """Eq. (11): rho = rho0, v1 = V0 sin x cos y cos z, v2 = -V0 cos x sin y cos z,
    v3 = 0, p = rho0 V0^2/(gamma M0^2) + rho0 V0^2/16 (cos 2x + cos 2y)(cos 2z + 2)."""
    X, Y, Z = node_coordinates(prm, basis)
    rho = np.ones_like(X)
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(X)
    p = prm.p0 + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    E = p / (prm.gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E])


# ------------------------------------------------------------ time step, diagnostics

def max_wave_speed(q, prm):
    """max over nodes of |v| + c, c = sqrt(gamma p / rho)."""
    vel = velocity(q)
    c = np.sqrt(prm.gamma * pressure(q, prm.gamma) / q[0])
    return float(np.max(np.sqrt(np.sum(vel * vel, axis=0)) + c))


def stable_dt(q, prm, cfl=0.4):
    """Eq. (7) with the (P+1)^2 order scaling: dt_a = CFL h / ((P+1)^2 max(|v|+c)),
    dt_v = CFL h^2 / ((P+1)^4 max(nu, gamma nu / Pr)), nu = mu / min(rho);
    dt = min(dt_a, dt_v), taken once from the given state."""
    n = prm.P + 1
    dt_a = cfl * prm.h / (n * n * max_wave_speed(q, prm))
    nu = prm.mu / float(np.min(q[0]))
    diff = max(nu, prm.gamma * nu / prm.Pr)
    dt_v = cfl * prm.h ** 2 / (n ** 4 * diff)
    return min(dt_a, dt_v)


def steps_for(t_end, dt):
    """Number of steps n = ceil(t_end / dt) and the adjusted step t_end / n."""
    n = int(np.ceil(t_end / dt - 1e-12))
    return n, t_end / n


def quadrature_weights(basis):
    w = basis.weights
    return w[:, None, None] * w[None, :, None] * w[None, None, :]   # [k, j, i]


def kinetic_energy(q, prm, basis=None):
    """KE = (1 / |Omega|) integral of rho |v|^2 / 2, by the Gauss quadrature."""
    if basis is None:
        basis = Basis(prm.P)
    Wq = quadrature_weights(basis)
    ke = 0.5 * np.sum(q[1:4] ** 2, axis=0) / q[0]
    return float(np.sum(Wq * ke) * prm.J / prm.L ** 3)


def totals(q, prm, basis=None):
    """Integral of each conserved variable over the box."""
    if basis is None:
        basis = Basis(prm.P)
    Wq = quadrature_weights(basis)
    return np.array([np.sum(Wq * q[v]) * prm.J for v in range(NVAR)])


def error_inf(q_lo, q_ref):
    """Eq. (9): infinity norm of q_LO - Gq_HO for rho u, rho v, rho w."""
    return np.array([float(np.max(np.abs(q_lo[v] - q_ref[v]))) for v in (1, 2, 3)])
