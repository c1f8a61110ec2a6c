"""Method of manufactured solutions for the oracle's DG operator: order of
accuracy of the whole space-time discretisation (Eq. (1) with RK3).

A smooth periodic state q_e(x, t) with every component varying is made an
exact solution by adding S = dq_e/dt + div f^a(q_e) - div f^nu(q_e, grad q_e)
(App. A), derived symbolically.  Over the short horizon T = 0.1 the L2 error
at t = T falls between the consistency rate h^P and the asymptotic h^(P+1)
(measured: 2.44 Euler, 2.53 viscous at P = 2; 2.88 and 2.84 at T = 0.4); a
dropped term, a wrong sign or index anywhere in the operator gives O(1)
errors and a rate near zero.
"""
import numpy as np
import pytest

from oracle import dg, rk
from oracle.basis import Basis


def _manufactured(prm):
    import sympy as sp
    x, y, z, t = sp.symbols("x y z t", real=True)
    X = (x, y, z)
    g = prm.gamma
    rho = 1 + sp.Rational(1, 5) * sp.sin(x) * sp.cos(y) * sp.sin(z + t)
    vel = [sp.Rational(1, 2) * sp.sin(x - t) * sp.cos(z),
           sp.Rational(3, 10) * sp.cos(y + t) * sp.sin(x),
           sp.Rational(1, 5) * sp.sin(z) * sp.cos(y - t)]
    p = 10 + sp.Rational(1, 2) * sp.cos(x + y - t)
    E = p / (g - 1) + rho * sum(v * v for v in vel) / 2
    q = [rho] + [rho * v for v in vel] + [E]
    flux = []
    T = p / rho
    div = sum(sp.diff(vel[a], X[a]) for a in range(3))
    for b in range(3):
        F = [rho * vel[b]] + [rho * vel[a] * vel[b] + (p if a == b else 0) for a in range(3)] + [(E + p) * vel[b]]
        if prm.viscous:
            tau = [prm.mu * (sp.diff(vel[a], X[b]) + sp.diff(vel[b], X[a])) - (sp.Rational(2, 3) * prm.mu * div if a == b else 0)
                   for a in range(3)]
            F[1] -= tau[0]
            F[2] -= tau[1]
            F[3] -= tau[2]
            F[4] -= sum(vel[a] * tau[a] for a in range(3)) + prm.kappa * sp.diff(T, X[b])
        flux.append(F)
    S = [sp.diff(q[v], t) + sum(sp.diff(flux[b][v], X[b]) for b in range(3)) for v in range(5)]
    fq = sp.lambdify((x, y, z, t), q, "numpy")
    fS = sp.lambdify((x, y, z, t), S, "numpy")
    return fq, fS


def _stack(vals, shape):
    return np.stack([np.broadcast_to(np.asarray(v, dtype=np.float64), shape) for v in vals])


def _l2_error(N, P, viscous, T=0.1):
    prm = dg.Params(N=N, P=P, Re=20.0, viscous=viscous)
    b = Basis(P)
    fq, fS = _manufactured(prm)
    X, Y, Z = dg.node_coordinates(prm, b)
    q = _stack(fq(X, Y, Z, 0.0), X.shape)
    dt0 = 0.25 * dg.stable_dt(q, prm)
    n, dt = dg.steps_for(T, dt0)
    q = rk.integrate(q, dt, n, lambda qq, tt: dg.residual(qq, prm, b, source=_stack(fS(X, Y, Z, tt), X.shape)))
    err = q - _stack(fq(X, Y, Z, T), X.shape)
    Wq = dg.quadrature_weights(b) * prm.J
    return np.sqrt(sum(np.sum(Wq * err[v] ** 2) for v in range(5)))


@pytest.mark.slow
@pytest.mark.parametrize("viscous,min_order", [(False, 2.3), (True, 2.2)])
def test_mms_order_of_accuracy_P2(viscous, min_order):
    e4 = _l2_error(4, 2, viscous)
    e8 = _l2_error(8, 2, viscous)
    order = np.log2(e4 / e8)
    assert order >= min_order, (e4, e8, order)
