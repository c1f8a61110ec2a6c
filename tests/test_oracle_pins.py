"""Pins of oracle functions that the closed forms and invariants of the other
oracle tests leave open, each with the planted mistakes it must catch.

* Eq. (9) error norm: constructed states whose density and energy differ far
  more than their momenta do.
* Per-variable rescaling statistics of the training pairs (Sec. 2.2): a
  constructed dataset with known mean and standard deviation per variable, and
  a constant variable that hits the floor.
* Smagorinsky closure inside the viscous flux (Sec. 3.1; Table 1 cases 3b/3c):
  the closure's contribution to the residual converges spectrally to its
  continuum closed form, derived symbolically, for two turbulent Prandtl
  numbers, on a state with a temperature gradient (so the eddy conductivity
  acts) and a strain rate bounded away from zero (so |S| is smooth).
* Viscous branch of the Eq. (7) time step: the closed form where it binds and
  its h^2, (P+1)^-4 and kinematic-viscosity scalings.
* Round-off floor: the FP64 residual of the 4^3, P = 3 Taylor-Green case
  against the same operator evaluated in 80-bit extended precision.

A planted mistake is a local change of the oracle (monkeypatched on the CPU
for the duration of one check); every pin below is shown to fail under the
mistakes named beside it.
"""
import copy

import numpy as np
import pytest

from oracle import dg, forcing
from oracle.basis import Basis


# ------------------------------------------------------------ Eq. (9) norm

def _error_inf_case():
    """Two states on a 2^3, P = 1 mesh: density and energy differ by 5 and 100
    everywhere; the momenta differ at single nodes by known amounts."""
    rng = np.random.default_rng(11)
    q_ref = rng.uniform(-1.0, 1.0, (5, 8, 8))
    q = q_ref.copy()
    q[0] += 5.0
    q[4] -= 100.0
    q[1, 3, 2] += 0.25
    q[2, 7, 0] -= 0.75
    q[3, 0, 5] += 0.125
    q[2, 1, 1] += 0.5           # smaller than the other rho v difference
    return q, q_ref, np.array([0.25, 0.75, 0.125])


def check_error_inf():
    q, q_ref, expect = _error_inf_case()
    got = dg.error_inf(q, q_ref)
    return got.shape == (3,) and np.max(np.abs(got - expect)) < 1e-15


def test_error_inf_constructed():
    assert check_error_inf()


def _mutant_error_inf_indices(q_lo, q_ref):
    return np.array([float(np.max(np.abs(q_lo[v] - q_ref[v]))) for v in (0, 1, 2)])


def _mutant_error_inf_signed(q_lo, q_ref):
    return np.array([float(np.max(q_lo[v] - q_ref[v])) for v in (1, 2, 3)])


@pytest.mark.parametrize("mutant", [_mutant_error_inf_indices, _mutant_error_inf_signed])
def test_error_inf_pin_catches_planted_mistakes(monkeypatch, mutant):
    monkeypatch.setattr(dg, "error_inf", mutant)
    assert not check_error_inf()


# ------------------------------------------------ per-variable rescaling stats

def _stats_case():
    """Rows [6][5 n_p] with n_p = 4.  Every variable's values are
    m_v + s_v z with the same sign pattern z: twelve +1 and twelve -1 over the
    6 x 4 block (mean 0, population standard deviation 1), unevenly spread
    over the columns so that column statistics differ from the variable's.
    x variable 4 and y variable 0 are constant (the floor)."""
    z = np.array([[1, -1, 1, -1],
                  [1, -1, -1, 1],
                  [1, -1, 1, -1],
                  [1, -1, -1, 1],
                  [1, -1, 1, -1],
                  [-1, 1, -1, 1]], dtype=np.float64)
    mx, sx = np.array([1.0, -0.5, 0.25, 2.0, 178.5]), np.array([0.01, 0.5, 2.0, 1.0, 0.0])
    my, sy = np.array([0.3, 1e-3, -2e-3, 0.0, 5.0]), np.array([0.0, 1e-4, 3e-4, 1e-3, 0.25])
    X = np.concatenate([mx[v] + sx[v] * z for v in range(5)], axis=1)
    Y = np.concatenate([my[v] + sy[v] * z for v in range(5)], axis=1)
    floor = lambda m: 1e-12 * max(1.0, abs(m))
    sx_exp = np.array([s if s > 0 else floor(m) for m, s in zip(mx, sx)])
    sy_exp = np.array([s if s > 0 else floor(m) for m, s in zip(my, sy)])
    return X, Y, (mx, sx_exp, my, sy_exp)


def check_normalisation():
    X, Y, expect = _stats_case()
    nrm = forcing.normalisation_from_pairs(X, Y)
    got = (nrm.mu_in, nrm.sigma_in, nrm.mu_out, nrm.sigma_out)
    return all(np.allclose(g, e, rtol=1e-12, atol=1e-15 * max(1.0, np.max(np.abs(e)))) for g, e in zip(got, expect))


def test_normalisation_constructed():
    assert check_normalisation()


def _mutant_stats_sample_std(X, Y, nv=5):
    n_p = X.shape[1] // nv

    def stats(A):
        A3 = A.reshape(A.shape[0], nv, n_p)
        mu = A3.mean(axis=(0, 2))
        sd = np.sqrt(((A3 - mu[None, :, None]) ** 2).sum(axis=(0, 2)) / (A3.shape[0] * n_p - 1))
        return mu, np.maximum(sd, 1e-12 * np.maximum(1.0, np.abs(mu)))
    mi, si = stats(np.asarray(X, dtype=np.float64))
    mo, so = stats(np.asarray(Y, dtype=np.float64))
    return forcing.Normalisation(mi, si, mo, so)


def _mutant_stats_mean_of_column_std(X, Y, nv=5):
    n_p = X.shape[1] // nv

    def stats(A):
        A3 = A.reshape(A.shape[0], nv, n_p)
        mu = A3.mean(axis=(0, 2))
        sd = A3.std(axis=0).mean(axis=1)
        return mu, np.maximum(sd, 1e-12 * np.maximum(1.0, np.abs(mu)))
    mi, si = stats(np.asarray(X, dtype=np.float64))
    mo, so = stats(np.asarray(Y, dtype=np.float64))
    return forcing.Normalisation(mi, si, mo, so)


def _mutant_stats_absolute_floor(X, Y, nv=5):
    n_p = X.shape[1] // nv

    def stats(A):
        A3 = A.reshape(A.shape[0], nv, n_p)
        return A3.mean(axis=(0, 2)), np.maximum(A3.std(axis=(0, 2)), 1e-12)
    mi, si = stats(np.asarray(X, dtype=np.float64))
    mo, so = stats(np.asarray(Y, dtype=np.float64))
    return forcing.Normalisation(mi, si, mo, so)


@pytest.mark.parametrize("mutant", [_mutant_stats_sample_std, _mutant_stats_mean_of_column_std,
                                    _mutant_stats_absolute_floor])
def test_normalisation_pin_catches_planted_mistakes(monkeypatch, mutant):
    monkeypatch.setattr(forcing, "normalisation_from_pairs", mutant)
    assert not check_normalisation()


# ------------------------------------------ Smagorinsky closure, closed form

LES_ELL = 0.05      # the closure's length C_s Delta, held fixed across meshes


def _les_fields():
    """A smooth state whose strain rate is bounded away from zero:
    u = a sin x, v = sqrt(2) a cos x, w = b sin y gives 2 S:S = 2 a^2 + b^2 cos^2 y;
    density and pressure vary, so T = p / rho has a gradient."""
    import sympy as sp
    x, y, z = sp.symbols("x y z", real=True)
    a, b = sp.Rational(1, 2), sp.Rational(1, 5)
    rho = 1 + sp.Rational(1, 10) * sp.sin(z) * sp.cos(x)
    vel = [a * sp.sin(x), sp.sqrt(2) * a * sp.cos(x), b * sp.sin(y)]
    return (x, y, z), rho, vel


def _les_closed_form(prm_like, Pr_t):
    """Continuum contribution of the closure to the right-hand side of App. A's
    equations: div of (0, tau_t, v . tau_t + kappa_t grad T), with
    mu_t = rho l^2 sqrt(2 S:S), kappa_t = mu_t gamma / ((gamma - 1) Pr_t)."""
    import sympy as sp
    X, rho, vel = _les_fields()
    g = prm_like.gamma
    p = prm_like.p0 + sp.Rational(1, 2) * sp.cos(X[0] + X[2])
    T = p / rho
    S = [[(sp.diff(vel[i], X[j]) + sp.diff(vel[j], X[i])) / 2 for j in range(3)] for i in range(3)]
    SS = sum(S[i][j] ** 2 for i in range(3) for j in range(3))
    mut = rho * LES_ELL ** 2 * sp.sqrt(2 * SS)
    kt = mut * g / ((g - 1) * Pr_t)
    div = sum(sp.diff(vel[i], X[i]) for i in range(3))
    tau = [[2 * mut * S[i][j] - (sp.Rational(2, 3) * mut * div if i == j else 0) for j in range(3)] for i in range(3)]
    out = [sp.Integer(0)]
    for i in range(3):
        out.append(sum(sp.diff(tau[i][j], X[j]) for j in range(3)))
    out.append(sum(sp.diff(sum(vel[i] * tau[i][j] for i in range(3)) + kt * sp.diff(T, X[j]), X[j])
                   for j in range(3)))
    fns = [sp.lambdify(X, e, "numpy") for e in out]
    return fns, sp.lambdify(X, [rho] + [rho * v for v in vel] + [p / (g - 1) + rho * sum(v * v for v in vel) / 2],
                            "numpy")


def _les_contribution_errors(Pr_t, orders=(3, 5, 7), N=4, Re=1000.0):
    """Max-norm error, per order, of R(C_s) - R(0) against the closed form
    (relative to the closed form's maximum, momentum and energy rows)."""
    errs = []
    fns = state = None
    for P in orders:
        h = 2.0 * np.pi / N
        Cs = LES_ELL * (P + 1) / h
        prm_les = dg.Params(N=N, P=P, Re=Re, Cs=Cs, Pr_t=Pr_t)
        prm_0 = dg.Params(N=N, P=P, Re=Re, Cs=0.0, Pr_t=Pr_t)
        if fns is None:
            fns, state = _les_closed_form(prm_les, Pr_t)
        X, Y, Z = dg.node_coordinates(prm_les)
        q = np.stack([np.broadcast_to(np.asarray(f, dtype=np.float64), X.shape) for f in state(X, Y, Z)])
        dR = dg.residual(q, prm_les) - dg.residual(q, prm_0)
        e = []
        for v in range(1, 5):
            ex = np.broadcast_to(np.asarray(fns[v](X, Y, Z), dtype=np.float64), X.shape)
            e.append(np.max(np.abs(dR[v] - ex)) / np.max(np.abs(ex)))
        e.append(np.max(np.abs(dR[0])))
        errs.append(e)
    return np.array(errs)


def check_les(Pr_t):
    errs = _les_contribution_errors(Pr_t)
    # spectral convergence in P at fixed mesh: P = 7 within 1e-4 of the
    # closed form and at least 20x below P = 3, mass row untouched
    return bool(np.all(errs[-1, :4] < 1e-4) and np.all(errs[-1, :4] < errs[0, :4] / 20) and errs[-1, 4] == 0.0), errs


@pytest.mark.parametrize("Pr_t", [0.6, 0.3])
def test_smagorinsky_closure_closed_form(Pr_t):
    ok, errs = check_les(Pr_t)
    print("LES contribution errors (rows P = 3, 5, 7; momenta, energy, mass):\n", errs)
    assert ok, errs


def _flux_with(**changes):
    """The oracle's viscous flux with some closure constants replaced (a
    planted mistake in how the closure's coefficients are formed)."""
    orig = dg.viscous_flux

    def mutant(q, g, d, prm):
        p2 = copy.copy(prm)
        for key, fn in changes.items():
            setattr(p2, key, fn(prm))
        return orig(q, g, d, p2)
    return mutant


@pytest.mark.parametrize("name,mutant", [
    ("Pr in place of Pr_t", _flux_with(Pr_t=lambda p: p.Pr)),
    ("eddy conductivity dropped", _flux_with(Pr_t=lambda p: np.inf)),
    ("filter width h / P", _flux_with(delta=lambda p: p.h / p.P)),
])
def test_smagorinsky_pin_catches_planted_mistakes(monkeypatch, name, mutant):
    monkeypatch.setattr(dg, "viscous_flux", mutant)
    ok, errs = check_les(0.6)
    assert not ok, (name, errs)


def test_smagorinsky_pin_catches_missing_factor_two(monkeypatch):
    orig = dg.smagorinsky_mu
    monkeypatch.setattr(dg, "smagorinsky_mu", lambda rho, g, prm: orig(rho, g, prm) / np.sqrt(2.0))
    ok, errs = check_les(0.6)
    assert not ok, errs


# ------------------------------------------------ Eq. (7), viscous branch

def check_dt_viscous():
    """Re = 1 on the 4^3 mesh: the viscous bound binds.  Its value is
    CFL h^2 / ((P+1)^4 max(nu, gamma nu / Pr)) with nu = mu / min rho, and it
    scales with h^2, (P+1)^-4, Re, and the minimum density."""
    res = []
    prm = dg.Params(N=4, P=3, Re=1.0)
    q = dg.tgv_initial_condition(prm)
    dt = dg.stable_dt(q, prm)
    closed = 0.4 * prm.h ** 2 / (4 ** 4 * (1.4 / 0.72))
    res.append(abs(dt / closed - 1.0) < 1e-14)
    # advective bound for comparison: the viscous one must bind
    res.append(dt < 0.4 * prm.h / (16 * dg.max_wave_speed(q, prm)))
    # scalings
    prm2 = dg.Params(N=8, P=3, Re=1.0)
    res.append(abs(dg.stable_dt(dg.tgv_initial_condition(prm2), prm2) / dt - 0.25) < 1e-14)
    prm3 = dg.Params(N=4, P=7, Re=1.0)
    res.append(abs(dg.stable_dt(dg.tgv_initial_condition(prm3), prm3) / dt - 1.0 / 16) < 1e-14)
    prm4 = dg.Params(N=4, P=3, Re=0.5)
    res.append(abs(dg.stable_dt(q, prm4) / dt - 0.5) < 1e-14)
    q2 = q.copy()
    q2[0, 0, 0, 0, 0, 0, 0] = 0.5          # one lighter node: nu doubles there
    q2[4, 0, 0, 0, 0, 0, 0] = q[4, 0, 0, 0, 0, 0, 0] - 0.25 * np.sum(q[1:4, 0, 0, 0, 0, 0, 0] ** 2)
    res.append(abs(dg.stable_dt(q2, prm) / dt - 0.5) < 1e-14)
    return all(res), res


def test_dt_viscous_branch():
    ok, res = check_dt_viscous()
    assert ok, res


def _mutant_dt(kind):
    def fn(q, prm, cfl=0.4):
        n = prm.P + 1
        dt_a = cfl * prm.h / (n * n * dg.max_wave_speed(q, prm))
        nu = prm.mu / float(np.min(q[0]))
        diff = {"no thermal diffusivity": nu}.get(kind, max(nu, prm.gamma * nu / prm.Pr))
        if kind == "dynamic viscosity":
            diff = max(prm.mu, prm.gamma * prm.mu / prm.Pr)
        p = 2 if kind == "(P+1)^2 scaling" else 4
        hh = prm.h if kind == "h scaling" else prm.h ** 2
        return min(dt_a, cfl * hh / (n ** p * diff))
    return fn


@pytest.mark.parametrize("kind", ["no thermal diffusivity", "dynamic viscosity", "(P+1)^2 scaling", "h scaling"])
def test_dt_viscous_pin_catches_planted_mistakes(monkeypatch, kind):
    monkeypatch.setattr(dg, "stable_dt", _mutant_dt(kind))
    ok, res = check_dt_viscous()
    assert not ok, (kind, res)


# ----------------------------------------------------------- round-off floor

def longdouble_params(prm):
    """The same Params with every derived constant formed in 80-bit extended
    precision from the float64 inputs."""
    p = copy.copy(prm)
    ld = np.longdouble
    p.h = ld(prm.L) / prm.N
    p.s = ld(2) / p.h
    p.J = (p.h / 2) ** 3
    p.mu = ld(1) / ld(prm.Re)
    p.p0 = ld(1) / (ld(prm.gamma) * ld(prm.Mach) ** 2)
    p.p_ref = p.p0
    p.kappa = p.mu * ld(prm.gamma) / ((ld(prm.gamma) - 1) * ld(prm.Pr))
    p.delta = p.h / (prm.P + 1)
    p.gamma = ld(prm.gamma)
    return p


def roundoff_floor(q, prm):
    """Per-variable relative L2 difference between the FP64 residual and the
    80-bit one on the same (float64) input state."""
    R64 = dg.residual(q, prm)
    Rld = dg.residual(q.astype(np.longdouble), longdouble_params(prm), Basis(prm.P, np.longdouble))
    den = np.sqrt(np.sum(Rld.reshape(5, -1) ** 2, axis=1))
    num = np.sqrt(np.sum((R64.astype(np.longdouble) - Rld).reshape(5, -1) ** 2, axis=1))
    return np.asarray(num / np.maximum(den, 1e-6 * den.max()), dtype=np.float64), Rld


C1_FLOOR_BOUND = 2e-12


def test_roundoff_floor_C1():
    """The FP64 oracle on the 4^3, P = 3, Re 30 Taylor-Green state against the
    extended-precision evaluation of the same operator (basis tables and
    constants also formed in extended precision).  Measured per variable:
    5.8e-13, 9.4e-13, 4.5e-13, 3.9e-13, 5.8e-13 -- the fluxes are O(100)
    (energy) while the residual is O(0.1), so FP64 rounding of the flux terms
    leaves about 1e-12 of the residual.  The device residual is held to
    max(1e-12, 4 x this floor) against the extended-precision result."""
    prm = dg.Params(N=4, P=3, Re=30.0)
    q = dg.tgv_initial_condition(prm)
    floor, Rld = roundoff_floor(q, prm)
    print("FP64 round-off floor per variable:", floor)
    assert Rld.dtype == np.longdouble
    assert np.all(floor < C1_FLOOR_BOUND), floor
    # the floor is a real measurement, not an identity: the FP64 result differs
    assert np.max(floor) > 0.0
