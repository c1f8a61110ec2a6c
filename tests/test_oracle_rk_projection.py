"""Pins of the oracle's time integrator (Sec. 3.1) and filter G (Sec. 2)."""
import numpy as np
import pytest

from oracle import dg, projection, rk
from oracle.basis import Basis, lagrange_eval


def test_rk3_stability_polynomial():
    """On y' = lambda y one step multiplies by 1 + z + z^2/2 + z^3/6, z = lambda dt."""
    for z in (0.3, -1.7, 0.5 + 1.2j, -2.0 + 0.1j):
        out = rk.rk3_step(np.array([1.0 + 0j]), 1.0, lambda y, t: z * y)
        assert abs(out[0] - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-15 * max(1, abs(z) ** 3)


def test_rk3_third_order_on_nonautonomous_ode():
    """y' = cos(t) y, y(0) = 1 has y = exp(sin t); the error falls as dt^3."""
    errs = []
    for n in (20, 40, 80):
        y = rk.integrate(np.array([1.0]), 2.0 / n, n, lambda y, t: np.cos(t) * y)
        errs.append(abs(y[0] - np.exp(np.sin(2.0))))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 2.8), orders


@pytest.mark.parametrize("P_src,P_dst", [(8, 3), (8, 6), (6, 3), (5, 5), (4, 2)])
def test_filter_reproduces_low_degree_polynomials(P_src, P_dst):
    G1 = projection.projection_matrix(P_src, P_dst)
    xs, xd = Basis(P_src).nodes, Basis(P_dst).nodes
    for m in range(P_dst + 1):
        assert np.max(np.abs(G1 @ xs ** m - xd ** m)) < 1e-13


@pytest.mark.parametrize("P_src,P_dst", [(8, 3), (8, 6), (5, 2)])
def test_filter_is_the_l2_projection(P_src, P_dst):
    """Brute force: least-squares fit of degree <= P_dst to the source
    polynomial, on a dense Gauss rule, evaluated at the destination nodes."""
    rng = np.random.default_rng(11)
    src = Basis(P_src)
    xd = Basis(P_dst).nodes
    u = rng.standard_normal(src.n)                       # nodal values of a degree-P_src polynomial
    xq, wq = np.polynomial.legendre.leggauss(40)
    uq = lagrange_eval(src.nodes, xq) @ u
    V = np.vander(xq, P_dst + 1, increasing=True)
    coef = np.linalg.solve(V.T @ (wq[:, None] * V), V.T @ (wq * uq))
    ref = np.vander(xd, P_dst + 1, increasing=True) @ coef
    assert np.max(np.abs(projection.projection_matrix(P_src, P_dst) @ u - ref)) < 1e-12


def test_filter_inverts_interpolation_and_keeps_means():
    for P_src, P_dst in ((8, 3), (6, 3), (8, 6)):
        src, dst = Basis(P_src), Basis(P_dst)
        E1 = lagrange_eval(dst.nodes, src.nodes)            # LO nodal -> HO nodal
        G1 = projection.projection_matrix(P_src, P_dst)
        assert np.max(np.abs(G1 @ E1 - np.eye(dst.n))) < 1e-13
        rng = np.random.default_rng(P_src)
        u = rng.standard_normal(src.n)
        assert abs(dst.weights @ (G1 @ u) - src.weights @ u) < 1e-13


def test_filter_3d_keeps_element_integrals():
    prm = dg.Params(N=2, P=6, Re=100.0)
    rng = np.random.default_rng(12)
    q = rng.standard_normal((5, 2, 2, 2, 7, 7, 7))
    ql = projection.project(q, 6, 3)
    wh = dg.quadrature_weights(Basis(6))
    wl = dg.quadrature_weights(Basis(3))
    assert np.max(np.abs((wh * q).sum(axis=(-3, -2, -1)) - (wl * ql).sum(axis=(-3, -2, -1)))) < 1e-13
