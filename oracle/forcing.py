"""Corrective forcing: the network's forcing s(q) added to the low-order
operator (Eq. (4)), and the training target of Eq. (5).

Test infrastructure only (see ``oracle/__init__``).

Network input and output per element e (Sec. 2.2): the element's nodal state
flattened variable-major, x[v * n_p + n] = q[v][e][n], normalised per
variable, xhat_v = (x_v - mu_in[v]) / sigma_in[v]; the network output yhat is
mapped back with s_v = mask[v] (sigma_out[v] yhat_v + mu_out[v]).  The paper
feeds only the momentum and forces only the momentum (mask (0,1,1,1,0)); the
workload measured here feeds and forces all five variables.

Training target (Eq. (5), with the low-order state equal to the filtered
high-order one, as Algorithm 1 sets it before each low-order step):
    x = G q_HO,    y = G p_HO(q_HO) - p_LO(G q_HO).
"""
import numpy as np

from . import dg, mlp, projection
from .basis import Basis


class Normalisation:
    """Per-variable affine maps of the network input and output."""

    def __init__(self, mu_in, sigma_in, mu_out, sigma_out, mask=(1, 1, 1, 1, 1)):
        self.mu_in = np.asarray(mu_in, dtype=np.float64)
        self.sigma_in = np.asarray(sigma_in, dtype=np.float64)
        self.mu_out = np.asarray(mu_out, dtype=np.float64)
        self.sigma_out = np.asarray(sigma_out, dtype=np.float64)
        self.mask = np.asarray(mask, dtype=np.float64)

    def as_array(self):
        return np.concatenate([self.mu_in, self.sigma_in, self.mu_out, self.sigma_out])


def element_rows(q_flat):
    """q[v][e][n] -> X[e][v * n_p + n]."""
    nv, E, n_p = q_flat.shape
    return np.transpose(q_flat, (1, 0, 2)).reshape(E, nv * n_p)


def rows_to_field(Y, nv, n_p):
    E = Y.shape[0]
    return np.transpose(Y.reshape(E, nv, n_p), (1, 0, 2))


def network_forcing(q_flat, params, norm, act="tanh"):
    """s(q) for every element; q_flat[5][E][n_p] -> s[5][E][n_p]."""
    nv, E, n_p = q_flat.shape
    X = element_rows(q_flat)
    scale_in = np.repeat(norm.sigma_in, n_p)
    shift_in = np.repeat(norm.mu_in, n_p)
    yhat = mlp.forward(params, (X - shift_in) / scale_in, act)[-1]
    s = yhat * np.repeat(norm.sigma_out, n_p) + np.repeat(norm.mu_out, n_p)
    s = s * np.repeat(norm.mask, n_p)
    return rows_to_field(s, nv, n_p)


def corrected_rhs(q_blocks, prm, params=None, norm=None, act="tanh", basis=None):
    """Right-hand side of Eq. (4): p_LO(q) + s(q) (s omitted when params is None)."""
    R = dg.residual(q_blocks, prm, basis)
    if params is None:
        return R
    s = network_forcing(dg.to_flat(q_blocks), params, norm, act)
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
