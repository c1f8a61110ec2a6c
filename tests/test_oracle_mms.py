"""Method of manufactured solutions for the oracle's DG operator: order of
accuracy of the whole space-time discretisation (Eq. (1) with RK3).

A smooth periodic state q_e(x, t) with every component varying is made an
exact solution by adding S = dq_e/dt + div f^a(q_e) - div f^nu(q_e, grad q_e)
(App. A), derived symbolically.  The L2 error at T = 0.4 on 4^3 and 8^3
elements gives the order of accuracy, gated at P + 1/2 for the Euler
equations and at P with viscosity (BR1 can lose up to one order where
diffusion dominates).  Measured: P = 2: 2.88 Euler, 2.84 viscous; P = 3:
3.66 Euler, 3.58 viscous.  The time step is the Eq. (7) one; a quarter of it
changes the errors in the fourth digit, so the temporal error is negligible.
A dropped term, a wrong sign or index anywhere in the operator gives O(1)
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


def _l2_error(N, P, viscous, T=0.4):
    prm = dg.Params(N=N, P=P, Re=20.0, viscous=viscous)
    b = Basis(P)
    fq, fS = _manufactured(prm)
    X, Y, Z = dg.node_coordinates(prm, b)
    q = _stack(fq(X, Y, Z, 0.0), X.shape)
    dt0 = dg.stable_dt(q, prm)
    n, dt = dg.steps_for(T, dt0)
    q = rk.integrate(q, dt, n, lambda qq, tt: dg.residual(qq, prm, b, source=_stack(fS(X, Y, Z, tt), X.shape)))
    err = q - _stack(fq(X, Y, Z, T), X.shape)
    Wq = dg.quadrature_weights(b) * prm.J
    return np.sqrt(sum(np.sum(Wq * err[v] ** 2) for v in range(5)))


@pytest.mark.slow
@pytest.mark.parametrize("P,viscous", [(2, False), (2, True), (3, False), (3, True)])
def test_mms_order_of_accuracy(P, viscous):
    e4 = _l2_error(4, P, viscous)
    e8 = _l2_error(8, P, viscous)
    order = np.log2(e4 / e8)
    min_order = P if viscous else P + 0.5
    print(f"P = {P}, viscous = {viscous}: L2 errors {e4:.4e} {e8:.4e}, order {order:.3f}")
    assert order >= min_order, (e4, e8, order)
