"""Corrective forcing: the network's forcing s(q) added to the low-order
operator (Eq. (4)), and the training target of Eq. (5).

Test infrastructure only (see ``oracle/__init__``).

Network input and output per element e (Sec. 2.2): the element's nodal state
flattened variable-major, x[v * n_p + n] = q[v][e][n], normalised per
variable, xhat_v = (x_v - mu_in[v]) / sigma_in[v]; the network output yhat is
mapped back with s_v = mask[v] (sigma_out[v] yhat_v + mu_out[v]).  The paper
feeds only the momentum and forces only the momentum (mask (0,1,1,1,0)); the
workload measured here feeds and forces all five variables.

The network may also see and force a subset of the variables (in_vars,
out_vars): its input row is then the selected variables' nodal values only,
and the forcing of the other variables is zero.  The paper's network reads
and forces the three momenta (Sec. 2.2).

Training target (Eq. (5), with the low-order state equal to the filtered
high-order one, as Algorithm 1 sets it before each low-order step):
    x = G q_HO,    y = G p_HO(q_HO) - p_LO(G q_HO).

Algorithm 1's own target is the discrete increment over one low-order step
dt_n: with q_NN^n = G q_HO^n advanced one uncorrected low-order step to
q_NN^{n+1}, and q_HO advanced over the same interval in m high-order steps,
    s_n = (G q_HO^{n+1} - q_NN^{n+1}) / dt_n,   paired with x = q_NN^n;
the low-order evolution then corrects after each uncorrected step,
q^{n+1} <- q^{n+1} + dt_n s_n, with s_n evaluated on q^n.
"""
import numpy as np

from . import dg, mlp, projection, rk
from .basis import Basis

ALL_VARS = (0, 1, 2, 3, 4)
MOMENTUM = (1, 2, 3)


class Normalisation:
    """Affine maps of the network input and output: per variable (mu_in[5],
    ...), or per node of the element row (columns: mu_in, sigma_in, mu_out,
    sigma_out each of length 5 n_p, column v n_p + n), the paper's rescaling
    of the values at each node (Sec. 2.2)."""

    def __init__(self, mu_in, sigma_in, mu_out, sigma_out, mask=(1, 1, 1, 1, 1), columns=None):
        self.mu_in = np.asarray(mu_in, dtype=np.float64)
        self.sigma_in = np.asarray(sigma_in, dtype=np.float64)
        self.mu_out = np.asarray(mu_out, dtype=np.float64)
        self.sigma_out = np.asarray(sigma_out, dtype=np.float64)
        self.mask = np.asarray(mask, dtype=np.float64)
        self.columns = None if columns is None else [np.asarray(c, dtype=np.float64) for c in columns]

    def as_array(self):
        return np.concatenate([self.mu_in, self.sigma_in, self.mu_out, self.sigma_out])

    def maps(self, iv, ov, n_p):
        """(shift_in, scale_in, shift_out, scale_out) over the network's
        input columns (variables iv) and output columns (variables ov)."""
        if self.columns is None:
            return (np.repeat(self.mu_in[iv], n_p), np.repeat(self.sigma_in[iv], n_p),
                    np.repeat(self.mu_out[ov], n_p), np.repeat(self.sigma_out[ov], n_p))

        def take(c, vs):
            return np.concatenate([c[v * n_p:(v + 1) * n_p] for v in vs])

        mi, si, mo, so = self.columns
        return take(mi, iv), take(si, iv), take(mo, ov), take(so, ov)


def element_rows(q_flat):
    """q[v][e][n] -> X[e][v * n_p + n]."""
    nv, E, n_p = q_flat.shape
    return np.transpose(q_flat, (1, 0, 2)).reshape(E, nv * n_p)


def rows_to_field(Y, nv, n_p):
    E = Y.shape[0]
    return np.transpose(Y.reshape(E, nv, n_p), (1, 0, 2))


def network_forcing(q_flat, params, norm, act="tanh", in_vars=ALL_VARS, out_vars=ALL_VARS):
    """s(q) for every element; q_flat[5][E][n_p] -> s[5][E][n_p].  The
    network reads the variables in_vars and forces the variables out_vars."""
    nv, E, n_p = q_flat.shape
    iv, ov = list(in_vars), list(out_vars)
    X = element_rows(q_flat[iv])
    shift_in, scale_in, shift_out, scale_out = norm.maps(iv, ov, n_p)
    xhat = (X - shift_in) / scale_in
    yhat = mlp.forward(params, xhat, act)[-1]
    s_sel = yhat * scale_out + shift_out
    s_sel = s_sel * np.repeat(norm.mask[ov], n_p)
    s = np.zeros_like(np.asarray(q_flat, dtype=np.float64))
    s[ov] = rows_to_field(s_sel, len(ov), n_p)
    return s


def corrected_rhs(q_blocks, prm, params=None, norm=None, act="tanh", basis=None, in_vars=ALL_VARS,
                  out_vars=ALL_VARS):
    """Right-hand side of Eq. (4): p_LO(q) + s(q) (s omitted when params is None)."""
    R = dg.residual(q_blocks, prm, basis)
    if params is None:
        return R
    s = network_forcing(dg.to_flat(q_blocks), params, norm, act, in_vars, out_vars)
    return R + dg.to_blocks(s, prm.N, prm.P)


def forcing_target(q_hi, prm_hi, prm_lo):
    """(x, y) of Eq. (5) for one high-order snapshot, as rows [E][5 n_p_lo]."""
    P_hi, P_lo = prm_hi.P, prm_lo.P
    R_hi = dg.residual(q_hi, prm_hi, Basis(P_hi))
    q_lo = projection.project(q_hi, P_hi, P_lo)
    y = projection.project(R_hi, P_hi, P_lo) - dg.residual(q_lo, prm_lo, Basis(P_lo))
    return element_rows(dg.to_flat(q_lo)), element_rows(dg.to_flat(y))


def normalisation_from_pairs(X, Y, nv=5):
    """Per-variable mean and standard deviation of the training pairs, the
    standard deviation floored at 1e-12 max(1, |mean|)."""
    n_p = X.shape[1] // nv

    def stats(A):
        A3 = A.reshape(A.shape[0], nv, n_p)
        mu = A3.mean(axis=(0, 2))
        sd = A3.std(axis=(0, 2))
        sd = np.maximum(sd, 1e-12 * np.maximum(1.0, np.abs(mu)))
        return mu, sd

    mi, si = stats(np.asarray(X, dtype=np.float64))
    mo, so = stats(np.asarray(Y, dtype=np.float64))
    return Normalisation(mi, si, mo, so)


def column_normalisation_from_pairs(X, Y):
    """Mean and standard deviation of every column (node of a variable) of
    the training pairs, the standard deviation floored at 1e-12 max(1, |mean|);
    the per-variable statistics are kept beside them."""
    def stats(A):
        A = np.asarray(A, dtype=np.float64)
        mu = A.mean(axis=0)
        sd = np.maximum(A.std(axis=0), 1e-12 * np.maximum(1.0, np.abs(mu)))
        return mu, sd

    base = normalisation_from_pairs(X, Y)
    mi, si = stats(X)
    mo, so = stats(Y)
    return Normalisation(base.mu_in, base.sigma_in, base.mu_out, base.sigma_out, columns=(mi, si, mo, so))


def increment_target(q_hi, prm_hi, prm_lo, dt_lo, m_sub):
    """One low-order step of Algorithm 1's high-order evolution.

    Sets the low-order state to the filtered high-order one, advances it one
    uncorrected low-order step of dt_lo, advances the high-order state over
    the same interval in m_sub steps of dt_lo / m_sub, filters it, and forms
    the discrete forcing s = (G q_HO^{n+1} - q_NN^{n+1}) / dt_lo.
    Returns (x rows = q_NN^n, y rows = s, q_HO^{n+1}); rows [E][5 n_p_lo]."""
    P_hi, P_lo = prm_hi.P, prm_lo.P
    b_hi, b_lo = Basis(P_hi), Basis(P_lo)
    q_nn = projection.project(q_hi, P_hi, P_lo)
    q_nn1 = rk.rk3_step(q_nn, dt_lo, lambda q, t: dg.residual(q, prm_lo, b_lo))
    q_hi1 = rk.integrate(q_hi, dt_lo / m_sub, m_sub, lambda q, t: dg.residual(q, prm_hi, b_hi))
    s = (projection.project(q_hi1, P_hi, P_lo) - q_nn1) / dt_lo
    return element_rows(dg.to_flat(q_nn)), element_rows(dg.to_flat(s)), q_hi1


def post_corrected_step(q_blocks, prm, dt, params, norm, act="relu", in_vars=MOMENTUM, out_vars=MOMENTUM,
                        basis=None):
    """Algorithm 1's low-order step: the uncorrected step q^n -> q^{n+1}, then
    q^{n+1} + dt s(q^n)."""
    basis = basis or Basis(prm.P)
    s = network_forcing(dg.to_flat(q_blocks), params, norm, act, in_vars, out_vars)
    q1 = rk.rk3_step(q_blocks, dt, lambda q, t: dg.residual(q, prm, basis))
    return q1 + dt * dg.to_blocks(s, prm.N, prm.P)
