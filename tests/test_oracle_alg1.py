"""Pins of the oracle's Algorithm 1 pieces: the discrete-increment forcing
target, the post-step correction, and a network that reads and forces a
subset of the variables (Sec. 2.1, 2.2, Algorithm 1)."""
import numpy as np
import pytest

import synthetic
from oracle import dg, forcing, projection, rk
from oracle.basis import Basis


def _smooth_state(N, P, seed=3):
    """TGV plus a smooth perturbation, so that every variable varies."""
    prm = dg.Params(N=N, P=P, Re=400.0)
    q = dg.tgv_initial_condition(prm)
    x = dg.node_coordinates(prm)
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.02, 0.05, size=5)
    for v in range(5):
        scale = 1.0 if v < 4 else 10.0
        q[v] = q[v] + scale * a[v] * np.sin(x[0] + 2 * x[1] + v) * np.cos(x[2] - v)
    return q


def test_increment_target_vanishes_for_equal_orders():
    """P_HO = P_LO and one high-order step per low-order step: both evolutions
    are the same uncorrected step from the same state, so s = 0."""
    prm = dg.Params(N=2, P=3, Re=400.0)
    q = _smooth_state(2, 3)
    x, y, q1 = forcing.increment_target(q, prm, prm, 1e-3, 1)
    R = dg.residual(q, prm)
    assert np.max(np.abs(y)) < 1e-10 * np.max(np.abs(R))
    assert np.array_equal(forcing.rows_to_field(x, 5, 64), dg.to_flat(projection.project(q, 3, 3)))


def test_increment_target_is_conservative():
    """Both evolutions conserve and G keeps element integrals: every variable's
    integral of s vanishes."""
    prm_hi = dg.Params(N=2, P=5, Re=400.0)
    prm_lo = dg.Params(N=2, P=3, Re=400.0)
    q = _smooth_state(2, 5)
    dt = 1e-3
    x, y, q1 = forcing.increment_target(q, prm_hi, prm_lo, dt, 2)
    yb = dg.to_blocks(forcing.rows_to_field(y, 5, 64), 2, 3)
    Wq = dg.quadrature_weights(Basis(3)) * prm_lo.J
    R = dg.residual(q, prm_hi)
    for v in range(5):
        scale = np.sum(dg.quadrature_weights(Basis(5)) * prm_hi.J * np.abs(R[v]))
        assert abs(np.sum(Wq * yb[v])) < 1e-11 * max(scale, 1.0)


def test_increment_target_tends_to_the_instantaneous_target():
    """As dt -> 0 the discrete increment tends to Eq. (5)'s target
    G p_HO(q) - p_LO(G q), with an error of first order in dt."""
    prm_hi = dg.Params(N=2, P=5, Re=400.0)
    prm_lo = dg.Params(N=2, P=3, Re=400.0)
    q = _smooth_state(2, 5, seed=4)
    _, y5 = forcing.forcing_target(q, prm_hi, prm_lo)
    errs = []
    for dt in (4e-4, 2e-4, 1e-4):
        _, y, _ = forcing.increment_target(q, prm_hi, prm_lo, dt, 1)
        errs.append(np.max(np.abs(y - y5)))
    scale = np.max(np.abs(y5))
    assert errs[-1] < 0.02 * scale
    for a, b in zip(errs[:-1], errs[1:]):
        assert 1.7 < a / b < 2.3


def test_increment_target_advances_the_high_order_state():
    prm_hi = dg.Params(N=2, P=4, Re=400.0)
    prm_lo = dg.Params(N=2, P=2, Re=400.0)
    q = _smooth_state(2, 4)
    _, _, q1 = forcing.increment_target(q, prm_hi, prm_lo, 1e-3, 3)
    ref = q
    for _ in range(3):
        ref = rk.rk3_step(ref, 1e-3 / 3, lambda s, t: dg.residual(s, prm_hi))
    assert np.array_equal(q1, ref)


def _const_net(n_in, n_out, bias):
    """A network whose output is its last bias: W = 0 everywhere."""
    dims = [n_in, 16, 16, n_out]
    params = []
    for l in range(3):
        W = np.zeros((dims[l + 1], dims[l]))
        b = np.zeros(dims[l + 1]) if l < 2 else np.asarray(bias, dtype=np.float64)
        params.append((W, b))
    return params


def test_post_step_correction_closed_form():
    """With a constant forcing s = sigma_out c + mu_out on the momenta, the
    corrected step is the uncorrected one plus dt s."""
    prm = dg.Params(N=2, P=3, Re=400.0)
    q = _smooth_state(2, 3)
    n_p = 64
    rng = np.random.default_rng(11)
    c = rng.standard_normal(3 * n_p)
    norm = forcing.Normalisation(np.zeros(5), np.ones(5), np.full(5, 0.25), np.full(5, 2.0))
    params = _const_net(3 * n_p, 3 * n_p, c)
    dt = 1e-3
    q1 = forcing.post_corrected_step(q, prm, dt, params, norm)
    q_unc = rk.rk3_step(q, dt, lambda s, t: dg.residual(s, prm))
    s = np.zeros((5, 8, n_p))
    for j, v in enumerate(forcing.MOMENTUM):
        s[v] = 2.0 * c[j * n_p:(j + 1) * n_p][None, :] + 0.25
    assert np.max(np.abs(q1 - (q_unc + dt * dg.to_blocks(s, 2, 3)))) < 1e-14 * np.max(np.abs(q))
    # a zero network leaves the uncorrected step
    zero = forcing.Normalisation(np.zeros(5), np.ones(5), np.zeros(5), np.ones(5))
    q0 = forcing.post_corrected_step(q, prm, dt, _const_net(3 * n_p, 3 * n_p, np.zeros(3 * n_p)), zero)
    assert np.array_equal(q0, q_unc)


def test_variable_selection():
    """The forcing ignores unselected inputs, is zero on unselected outputs,
    and with every variable selected is the full network."""
    rng = np.random.default_rng(12)
    E, n_p = 4, 8
    q = rng.standard_normal((5, E, n_p))
    dims = [3 * n_p, 12, 12, 3 * n_p]
    params = [(W.astype(np.float64), b.astype(np.float64) + 0.05) for W, b in synthetic.mlp_init(dims, 5)]
    norm = forcing.Normalisation(rng.standard_normal(5), rng.uniform(0.5, 2, 5), rng.standard_normal(5),
                                 rng.uniform(0.5, 2, 5), mask=(1, 1, 0, 1, 1))
    s = forcing.network_forcing(q, params, norm, "relu", forcing.MOMENTUM, forcing.MOMENTUM)
    q2 = q.copy()
    q2[[0, 4]] = rng.standard_normal((2, E, n_p))
    s2 = forcing.network_forcing(q2, params, norm, "relu", forcing.MOMENTUM, forcing.MOMENTUM)
    assert np.array_equal(s, s2)
    assert np.all(s[[0, 2, 4]] == 0) and np.any(s[1] != 0) and np.any(s[3] != 0)
    # input columns of an unselected variable with zero weights: the full network
    full = [(W.copy(), b.copy()) for W, b in params]
    W0 = np.zeros((12, 5 * n_p))
    for j, v in enumerate(forcing.MOMENTUM):
        W0[:, v * n_p:(v + 1) * n_p] = params[0][0][:, j * n_p:(j + 1) * n_p]
    full[0] = (W0, params[0][1])
    WL = np.zeros((5 * n_p, 12))
    bL = np.zeros(5 * n_p)
    for j, v in enumerate(forcing.MOMENTUM):
        WL[v * n_p:(v + 1) * n_p] = params[-1][0][j * n_p:(j + 1) * n_p]
        bL[v * n_p:(v + 1) * n_p] = params[-1][1][j * n_p:(j + 1) * n_p]
    full[-1] = (WL, bL)
    mask_full = norm.mask * np.array([0, 1, 1, 1, 0])
    norm_full = forcing.Normalisation(norm.mu_in, norm.sigma_in, norm.mu_out, norm.sigma_out, mask=mask_full)
    s_full = forcing.network_forcing(q, full, norm_full, "relu")
    assert np.max(np.abs(s - s_full)) < 1e-13 * np.max(np.abs(s))


def test_column_statistics_on_a_constructed_dataset():
    """Column c of the constructed rows has mean c and standard deviation
    c + 1 exactly (values c +- (c + 1) in alternate rows)."""
    rows, cols = 10, 40
    sign = np.where(np.arange(rows) % 2 == 0, 1.0, -1.0)[:, None]
    c = np.arange(cols, dtype=np.float64)[None, :]
    X = c + (c + 1) * sign
    Y = -2.0 * X
    n = forcing.column_normalisation_from_pairs(X, Y)
    mi, si, mo, so = n.columns
    assert np.allclose(mi, np.arange(cols), atol=1e-13) and np.allclose(si, np.arange(cols) + 1, atol=1e-13)
    assert np.allclose(mo, -2 * np.arange(cols), atol=1e-12) and np.allclose(so, 2 * (np.arange(cols) + 1), atol=1e-12)


def test_column_normalisation_maps_nodes_of_the_selected_variables():
    """With equal input and output maps an identity network returns its
    input, node by node, for the selected variables only; per-variable maps
    are the special case of constant columns."""
    rng = np.random.default_rng(14)
    E, n_p = 3, 8
    q = rng.standard_normal((5, E, n_p))
    mu = rng.standard_normal(5 * n_p)
    sd = rng.uniform(0.5, 2.0, 5 * n_p)
    norm = forcing.Normalisation(np.zeros(5), np.ones(5), np.zeros(5), np.ones(5), columns=(mu, sd, mu, sd))
    ident = [(np.eye(3 * n_p), np.zeros(3 * n_p))]
    s = forcing.network_forcing(q, ident, norm, "tanh", forcing.MOMENTUM, forcing.MOMENTUM)
    assert np.max(np.abs(s[1:4] - q[1:4])) < 1e-14 and np.all(s[[0, 4]] == 0)
    # constant columns per variable = the per-variable normalisation
    pv = rng.uniform(0.5, 2.0, 5)
    pm = rng.standard_normal(5)
    colw = forcing.Normalisation(pm, pv, pm[::-1], pv[::-1],
                                 columns=(np.repeat(pm, n_p), np.repeat(pv, n_p), np.repeat(pm[::-1], n_p),
                                          np.repeat(pv[::-1], n_p)))
    varw = forcing.Normalisation(pm, pv, pm[::-1], pv[::-1])
    params = [(rng.standard_normal((5 * n_p, 5 * n_p)) / 6, rng.standard_normal(5 * n_p))]
    assert np.array_equal(forcing.network_forcing(q, params, colw), forcing.network_forcing(q, params, varw))
