"""Pins of the oracle's DG residual p(q) (Eq. (1)/(3), App. A, Sec. 3.1).

Each test pins the oracle to something other than itself: invariants the weak
form guarantees (free-stream preservation, discrete conservation, symmetry),
the defining property of Roe's linearisation, closed-form continuum residuals
that the discrete operator must approach spectrally, and exactness cases.
"""
import numpy as np
import pytest

import synthetic
from oracle import dg
from oracle.basis import Basis


def blocks(q, prm):
    return dg.to_blocks(q, prm.N, prm.P)


# ------------------------------------------------------------------ Roe flux

def _random_face_states(rng, n=200, mom=1.0):
    q = np.empty((5, n))
    q[0] = 1.0 + 0.3 * rng.uniform(-1, 1, n)
    q[1:4] = mom * rng.uniform(-1, 1, (3, n))
    q[4] = 20.0 + 5.0 * rng.uniform(-1, 1, n)
    return q


@pytest.mark.parametrize("d", [0, 1, 2])
def test_roe_consistency(d):
    prm = dg.Params(N=2, P=2, Re=100.0)
    q = _random_face_states(np.random.default_rng(1))
    F = dg.roe_flux(q, q, d, prm)
    Fa = dg.inviscid_flux(q, d, prm)
    assert np.max(np.abs(F - Fa)) < 1e-13 * np.max(np.abs(Fa))


@pytest.mark.parametrize("d", [0, 1, 2])
def test_roe_linearisation_property(d):
    """Roe's matrix satisfies A~ (qR - qL) = f(qR) - f(qL): the signed waves sum
    to the flux jump (Roe 1981)."""
    prm = dg.Params(N=2, P=2, Re=100.0, p_ref=0.0)
    rng = np.random.default_rng(2)
    qL, qR = _random_face_states(rng), _random_face_states(rng)
    jump = dg.inviscid_flux(qR, d, prm) - dg.inviscid_flux(qL, d, prm)
    total = sum(lam * wave for lam, wave in dg.roe_waves(qL, qR, d, prm.gamma))
    assert np.max(np.abs(total - jump)) < 1e-12 * np.max(np.abs(jump))
    # and the waves sum to the state jump itself
    waves = sum(wave for _, wave in dg.roe_waves(qL, qR, d, prm.gamma))
    assert np.max(np.abs(waves - (qR - qL))) < 1e-12 * np.max(np.abs(qR - qL))


def test_roe_supersonic_upwinding():
    """When every Roe wave speed is positive the flux is the left state's flux."""
    prm = dg.Params(N=2, P=2, Re=100.0)
    rng = np.random.default_rng(3)

    def state(n=100):
        rho = 1.0 + 0.2 * rng.uniform(-1, 1, n)
        vel = np.stack([30.0 + rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)])
        p = 1.0 + 0.2 * rng.uniform(-1, 1, n)
        E = p / (prm.gamma - 1) + 0.5 * rho * np.sum(vel * vel, axis=0)
        return np.concatenate([rho[None], rho * vel, E[None]])
    qL, qR = state(), state()
    lam_min = min(np.min(lam) for lam, _ in dg.roe_waves(qL, qR, 0, prm.gamma))
    assert lam_min > 0
    F = dg.roe_flux(qL, qR, 0, prm)
    FL = dg.inviscid_flux(qL, 0, prm)
    assert np.max(np.abs(F - FL)) < 1e-12 * np.max(np.abs(FL))


@pytest.mark.parametrize("d", [0, 1, 2])
def test_roe_mirror_symmetry(d):
    """Reflecting x_d -> -x_d swaps the sides and flips the normal momentum:
    F(M qR, M qL) = -M F(qL, qR) with M = diag(1, .., -1 at 1+d, .., 1)."""
    prm = dg.Params(N=2, P=2, Re=100.0)
    rng = np.random.default_rng(4)
    qL, qR = _random_face_states(rng), _random_face_states(rng)
    M = np.ones((5, 1))
    M[1 + d] = -1
    lhs = dg.roe_flux(M * qR, M * qL, d, prm)
    rhs = -M * dg.roe_flux(qL, qR, d, prm)
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * np.max(np.abs(rhs))


# --------------------------------------------------------- residual invariants

@pytest.mark.parametrize("Cs", [0.0, 0.1])
def test_free_stream_preservation(Cs):
    rng = np.random.default_rng(5)
    for trial in range(3):
        prm = dg.Params(N=3, P=3, Re=200.0, Cs=Cs)
        rho = 1.0 + 0.2 * rng.uniform(-1, 1)
        mom = rng.uniform(-1, 1, 3)
        q = blocks(synthetic.constant_state(3, 3, rho, mom, 180.0 + rng.uniform(-5, 5)), prm)
        R = dg.residual(q, prm)
        scale = (np.max(np.abs(dg.inviscid_flux(q, 0, prm))) + prm.p_ref) * prm.s
        assert np.max(np.abs(R)) < 1e-13 * scale


@pytest.mark.parametrize("Cs,viscous", [(0.0, False), (0.0, True), (0.1, True)])
def test_discrete_conservation(Cs, viscous):
    prm = dg.Params(N=3, P=3, Re=50.0, Cs=Cs, viscous=viscous)
    b = Basis(prm.P)
    q = blocks(synthetic.random_state(3, 3, seed=6), prm)
    R = dg.residual(q, prm, b)
    Wq = dg.quadrature_weights(b) * prm.J
    for v in range(5):
        tot = np.sum(Wq * R[v])
        mag = np.sum(Wq * np.abs(R[v]))
        assert abs(tot) < 1e-13 * mag, (v, tot, mag)


def test_translation_equivariance():
    prm = dg.Params(N=3, P=2, Re=100.0, Cs=0.1)
    q = blocks(synthetic.random_state(3, 2, seed=7), prm)
    R = dg.residual(q, prm)
    for d in range(3):
        qs = np.roll(q, 1, axis=dg.elem_axis(d))
        Rs = dg.residual(qs, prm)
        assert np.array_equal(Rs, np.roll(R, 1, axis=dg.elem_axis(d)))


def test_axis_permutation_equivariance():
    """Relabel the axes cyclically x->y->z->x (element and node axes together)
    and permute the momentum components alike; the residual permutes the same way."""
    prm = dg.Params(N=3, P=3, Re=80.0, Cs=0.1)
    q = blocks(synthetic.random_state(3, 3, seed=8), prm)
    R = dg.residual(q, prm)

    def cyc(A):
        # new field value at (x, y, z) = old value at (z, x, y):
        # new axes order (ez, ey, ex) <- old (ey, ex, ez), nodes likewise
        out = np.moveaxis(A, [-6, -5, -4, -3, -2, -1], [-4, -6, -5, -1, -3, -2])
        mom = out[1:4].copy()
        out = out.copy()
        out[1], out[2], out[3] = mom[2], mom[0], mom[1]
        return out

    Rc = dg.residual(cyc(q), prm)
    ref = cyc(R)
    for v in range(5):
        assert np.max(np.abs(Rc[v] - ref[v])) <= 1e-13 * np.max(np.abs(ref[v]))


def test_mirror_symmetry_of_tgv_preserved():
    """The TGV state is odd in u under x -> -x; the residual keeps that symmetry."""
    prm = dg.Params(N=4, P=3, Re=200.0)
    q = dg.tgv_initial_condition(prm)
    R = dg.residual(q, prm)

    def mirror_x(A):
        # x -> 2 pi - x: reverse element and node order along x
        return A[..., ::-1, :, :, ::-1]
    Rm = mirror_x(R)
    sign = np.array([1, -1, 1, 1, 1.0])[:, None, None, None, None, None, None]
    ref = sign * Rm
    for v in range(5):
        assert np.max(np.abs(R[v] - ref[v])) < 1e-12 * max(np.max(np.abs(R[v])), 1.0)


# --------------------------------------------------------- TGV initial state

@pytest.mark.parametrize("N,P", [(3, 3), (4, 3), (4, 8), (8, 3)])
def test_tgv_kinetic_energy_is_one_eighth(N, P):
    prm = dg.Params(N=N, P=P, Re=1600.0)
    q = dg.tgv_initial_condition(prm)
    assert abs(dg.kinetic_energy(q, prm) - 0.125) < 1e-14
    tot = dg.totals(q, prm)
    vol = prm.L ** 3
    assert abs(tot[0] / vol - 1.0) < 1e-14
    assert np.max(np.abs(tot[1:4])) < 1e-13


def test_tgv_mean_energy():
    prm = dg.Params(N=4, P=3, Re=1600.0)
    q = dg.tgv_initial_condition(prm)
    mean_E = dg.totals(q, prm)[4] / prm.L ** 3
    # <p> = p0 + (1/16)<(cos2x + cos2y)(cos2z + 2)> = p0; <rho|v|^2/2> = 1/8
    assert abs(mean_E - (prm.p0 / 0.4 + 0.125)) < 1e-12 * mean_E


# ------------------------------------------------- closed-form continuum residuals

def _sym_tgv_residual(Re, Mach, gamma=1.4, Pr=0.72):
    """Continuum right-hand side of App. A at the TGV initial state, with sympy."""
    import sympy as sp
    x, y, z = sp.symbols("x y z", real=True)
    X = (x, y, z)
    rho = sp.Integer(1)
    vel = [sp.sin(x) * sp.cos(y) * sp.cos(z), -sp.cos(x) * sp.sin(y) * sp.cos(z), sp.Integer(0)]
    p0 = 1 / (gamma * Mach ** 2)
    p = p0 + (sp.cos(2 * x) + sp.cos(2 * y)) * (sp.cos(2 * z) + 2) / 16
    mu = 1.0 / Re
    kappa = mu * gamma / ((gamma - 1) * Pr)
    E = p / (gamma - 1) + rho * sum(v * v for v in vel) / 2
    T = p / rho
    div = sum(sp.diff(vel[a], X[a]) for a in range(3))
    tau = [[mu * (sp.diff(vel[a], X[b]) + sp.diff(vel[b], X[a])) - (sp.Rational(2, 3) * mu * div if a == b else 0)
            for b in range(3)] for a in range(3)]
    r_rho = -sum(sp.diff(rho * vel[b], X[b]) for b in range(3))
    r_mom = [-sum(sp.diff(rho * vel[a] * vel[b] + (p if a == b else 0) - tau[a][b], X[b]) for b in range(3))
             for a in range(3)]
    r_E = -sum(sp.diff((E + p) * vel[b] - sum(vel[a] * tau[a][b] for a in range(3)) - kappa * sp.diff(T, X[b]), X[b])
               for b in range(3))
    return [sp.lambdify((x, y, z), e, "numpy") for e in [r_rho] + r_mom + [r_E]]


def test_tgv_momentum_closed_form():
    """An independent, incompressible closed form of d(rho u)/dt at t = 0:
    -1/8 sin 2x cos 2z - (3/Re) sin x cos y cos z (and its mirror for rho v)."""
    Re = 200.0
    errs = []
    for P in (3, 5, 7):
        prm = dg.Params(N=4, P=P, Re=Re)
        q = dg.tgv_initial_condition(prm)
        R = dg.residual(q, prm)
        X, Y, Z = dg.node_coordinates(prm)
        ru = -np.sin(2 * X) * np.cos(2 * Z) / 8 - 3 / Re * np.sin(X) * np.cos(Y) * np.cos(Z)
        rv = -np.sin(2 * Y) * np.cos(2 * Z) / 8 + 3 / Re * np.cos(X) * np.sin(Y) * np.cos(Z)
        rw = (np.cos(2 * X) + np.cos(2 * Y)) * np.sin(2 * Z) / 8
        errs.append(max(np.max(np.abs(R[1] - ru)), np.max(np.abs(R[2] - rv)), np.max(np.abs(R[3] - rw))))
    print("momentum closed-form errors", errs)
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 5
    assert errs[2] < 2e-4


def test_tgv_all_components_converge_to_continuum():
    Re, Mach = 100.0, 0.1
    funcs = _sym_tgv_residual(Re, Mach)
    errs = []
    for P in (3, 5, 7):
        prm = dg.Params(N=4, P=P, Re=Re, Mach=Mach)
        q = dg.tgv_initial_condition(prm)
        R = dg.residual(q, prm)
        X, Y, Z = dg.node_coordinates(prm)
        e = []
        for v in range(5):
            ex = np.broadcast_to(np.asarray(funcs[v](X, Y, Z), dtype=np.float64), X.shape)
            e.append(np.max(np.abs(R[v] - ex)))
        errs.append(e)
    errs = np.array(errs)
    for v in range(5):
        assert errs[2, v] < 3e-3 * max(1.0, errs[0, v]), (v, errs[:, v])
        assert errs[2, v] < errs[0, v] / 20, (v, errs[:, v])


def _analytic_state(prm, rho, u, v, w, p):
    X, Y, Z = dg.node_coordinates(prm)
    args = (X, Y, Z)
    r = np.broadcast_to(rho(*args), X.shape)
    vel = [np.broadcast_to(f(*args), X.shape) for f in (u, v, w)]
    pp = np.broadcast_to(p(*args), X.shape)
    E = pp / (prm.gamma - 1) + 0.5 * r * sum(c * c for c in vel)
    return np.stack([r, r * vel[0], r * vel[1], r * vel[2], E]), (X, Y, Z)


def test_pure_heat_conduction_closed_form():
    """Fluid at rest with uniform pressure and rho = 1/(1 + a sin x): only the heat
    flux acts, d(rho e)/dt = kappa d2T/dx2 with T = p/rho = p (1 + a sin x)."""
    a = 0.1
    errs = []
    for P in (3, 5, 7):
        prm = dg.Params(N=4, P=P, Re=10.0)
        p0 = prm.p0
        q, (X, Y, Z) = _analytic_state(prm, lambda x, y, z: 1.0 / (1.0 + a * np.sin(x)),
                                       lambda *c: 0.0 * c[0], lambda *c: 0.0 * c[0], lambda *c: 0.0 * c[0],
                                       lambda *c: p0 + 0.0 * c[0])
        R = dg.residual(q, prm)
        exact = prm.kappa * (-p0 * a * np.sin(X))
        assert np.max(np.abs(R[0:4])) < 1e-11 * p0
        errs.append(np.max(np.abs(R[4] - exact)) / np.max(np.abs(exact)))
    assert errs[2] < 1e-3 and errs[1] < errs[0] / 5 and errs[2] < errs[1] / 5, errs


def test_shear_layer_viscous_work_closed_form():
    """u = U sin y, rho = 1, uniform p: d(rho u)/dt = -mu U sin y and
    d(rho e)/dt = d/dy(u tau_xy) = mu U^2 cos 2y; mass and other momenta unchanged."""
    U = 0.5
    errs = []
    for P in (3, 5, 7):
        prm = dg.Params(N=4, P=P, Re=20.0)
        q, (X, Y, Z) = _analytic_state(prm, lambda *c: 1.0 + 0.0 * c[0], lambda x, y, z: U * np.sin(y),
                                       lambda *c: 0.0 * c[0], lambda *c: 0.0 * c[0], lambda *c: prm.p0 + 0.0 * c[0])
        R = dg.residual(q, prm)
        ru = -prm.mu * U * np.sin(Y)
        rE = prm.mu * U * U * np.cos(2 * Y)
        errs.append(max(np.max(np.abs(R[1] - ru)) / (prm.mu * U), np.max(np.abs(R[4] - rE)) / (prm.mu * U * U),
                        np.max(np.abs(R[[0, 2, 3]])) / (prm.mu * U)))
    assert errs[2] < 1e-3 and errs[1] < errs[0] / 5 and errs[2] < errs[1] / 5, errs


# ------------------------------------------------------------------ BR1 gradient

def test_br1_gradient_exact_for_continuous_piecewise_polynomials():
    """A periodic field that is continuous across faces and a polynomial of degree
    <= P in each variable inside each element has the elementwise derivative as
    its BR1 gradient: the weak form integrates it by parts exactly.  Here the
    velocities and theta are quadratic and rho e is quartic, so P = 4."""
    prm = dg.Params(N=4, P=4, Re=100.0)
    b = Basis(prm.P)
    X, Y, Z = dg.node_coordinates(prm, b)
    tri = lambda s: (s - np.pi) ** 2          # continuous, kink only at 0 == 2 pi
    dtri = lambda s: 2 * (s - np.pi)
    u, v, w = 0.1 * tri(X), 0.02 * tri(Z), 0.03 * tri(Y)
    rho = np.ones_like(X)
    theta = 70.0 + 0.05 * tri(Z)
    E = rho * theta / (prm.gamma - 1) + 0.5 * rho * (u * u + v * v + w * w)
    q = np.stack([rho, rho * u, rho * v, rho * w, E])
    g = dg.br1_gradient(q, prm, b)
    exact = np.zeros((3, 4) + X.shape)
    exact[0, 0] = 0.1 * dtri(X)
    exact[2, 1] = 0.02 * dtri(Z)
    exact[1, 2] = 0.03 * dtri(Y)
    exact[2, 3] = 0.05 * dtri(Z)
    for j in range(3):
        for a in range(4):
            assert np.max(np.abs(g[j, a] - exact[j, a])) < 1e-11, (j, a)


# ------------------------------------------------------------------ Smagorinsky

def test_smagorinsky_rigid_translation_and_shear():
    prm = dg.Params(N=2, P=2, Re=100.0, Cs=0.1)
    rho = np.array([1.0, 1.2])
    g = np.zeros((3, 4, 2))
    assert np.all(dg.smagorinsky_mu(rho, g, prm) == 0.0)
    shear = 3.0
    g[1, 0] = shear   # du/dy
    mut = dg.smagorinsky_mu(rho, g, prm)
    assert np.allclose(mut, rho * (prm.Cs * prm.delta) ** 2 * shear, rtol=1e-15, atol=0)


# ------------------------------------------------------------------ time step

def test_dt_follows_printed_time_steps():
    """Tables 1 and 2 print the time steps of P = 2..5 on the 8^3 mesh at
    M0 = 0.08 (golden file); the CFL-0.4 rule with (P+1)^2 reproduces them to
    within 15 % (Eq. (7), Sec. 2.3)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_time_steps.json")
    gold = json.load(open(path))
    for entry in gold["entries"]:
        P = entry["P"]
        prm = dg.Params(N=8, P=P, Re=1600.0, Mach=gold["Mach"])
        q = dg.tgv_initial_condition(prm)
        dt = dg.stable_dt(q, prm)
        assert abs(dt / entry["dt"] - 1.0) < 0.15, (P, dt, entry["dt"])


def test_dt_between_analytic_bounds():
    """Nodal max(|v|+c) lies below the continuum maximum, so dt is above the bound
    from max|v| + max c, and approaches it as P grows."""
    prm = dg.Params(N=4, P=3, Re=30.0)
    q = dg.tgv_initial_condition(prm)
    dt = dg.stable_dt(q, prm)
    c_max = np.sqrt(prm.gamma * (prm.p0 + 2.0 * 3.0 / 16.0))   # max p at rho = 1
    bound = 0.4 * prm.h / (16 * (1.0 + c_max))
    assert bound < dt < 1.01 * bound
    n, dt2 = dg.steps_for(1.0, dt)
    assert n * dt2 == pytest.approx(1.0, rel=1e-15) and dt2 <= dt
