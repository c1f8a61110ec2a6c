"""Nodal Lagrange basis on Gauss-Legendre points (Sec. 2.6: nodal DGSEM).

Test infrastructure only (see ``oracle/__init__``).

The DGSEM of the paper (Sec. 2.6, Kopriva's formulation) collocates the
solution at the P+1 Gauss-Legendre points of [-1, 1] in each direction.  This
module builds, in float64 with plain product formulas:

* ``nodes``, ``weights``  Gauss-Legendre points xi_i and weights w_i,
* ``D``                   derivative matrix D[i, j] = l_j'(xi_i),
* ``bp``, ``bm``          boundary vectors b+_j = l_j(+1), b-_j = l_j(-1),
* ``legendre``            Legendre polynomials L_k (used by the filter G).
"""
import numpy as np


def legendre(n, x, dtype=np.float64):
    """Legendre polynomial L_n(x) and its derivative, by the three-term recurrence
    (k+1) L_{k+1} = (2k+1) x L_k - k L_{k-1}."""
    x = np.asarray(x, dtype=dtype)
    l_prev = np.ones_like(x)
    if n == 0:
        return l_prev, np.zeros_like(x)
    l_cur = x.copy()
    dl_prev = np.zeros_like(x)
    dl_cur = np.ones_like(x)
    for k in range(1, n):
        l_next = ((2 * k + 1) * x * l_cur - k * l_prev) / (k + 1)
        # derivative of the recurrence: (k+1) L'_{k+1} = (2k+1)(L_k + x L'_k) - k L'_{k-1}
        dl_next = ((2 * k + 1) * (l_cur + x * dl_cur) - k * dl_prev) / (k + 1)
        l_prev, l_cur = l_cur, l_next
        dl_prev, dl_cur = dl_cur, dl_next
    return l_cur, dl_cur


def gauss_legendre(P, dtype=np.float64):
    """The P+1 roots of L_{P+1} (ascending) and the Gauss weights
    w_i = 2 / ((1 - x_i^2) L'_{P+1}(x_i)^2), found by Newton's method."""
    n = P + 1
    i = np.arange(n, dtype=np.float64)
    x = (-np.cos(np.pi * (i + 0.75) / (n + 0.5))).astype(dtype)  # ascending initial guesses
    # stop once a step is below the type's rounding at |x| ~ 1
    tol = 1e-17 if np.dtype(dtype) == np.float64 else 1e-21
    for _ in range(100):
        val, der = legendre(n, x, dtype)
        dx = val / der
        x = x - dx
        if np.max(np.abs(dx)) < tol:
            break
    _, der = legendre(n, x, dtype)
    w = 2.0 / ((1.0 - x * x) * der * der)
    return x, w


def lagrange_eval(nodes, t):
    """Matrix L[a, j] = l_j(t_a) of the Lagrange polynomials through ``nodes``,
    by the product formula l_j(t) = prod_{k != j} (t - x_k) / (x_j - x_k)."""
    t = np.atleast_1d(np.asarray(t, dtype=nodes.dtype))
    n = len(nodes)
    L = np.ones((len(t), n), dtype=nodes.dtype)
    for j in range(n):
        for k in range(n):
            if k != j:
                L[:, j] *= (t - nodes[k]) / (nodes[j] - nodes[k])
    return L


def lagrange_deriv(nodes, t):
    """Matrix Ld[a, j] = l_j'(t_a), by differentiating the product formula:
    l_j'(t) = sum_{m != j} 1/(x_j - x_m) prod_{k != j, m} (t - x_k)/(x_j - x_k)."""
    t = np.atleast_1d(np.asarray(t, dtype=nodes.dtype))
    n = len(nodes)
    Ld = np.zeros((len(t), n), dtype=nodes.dtype)
    for j in range(n):
        for m in range(n):
            if m == j:
                continue
            term = np.full(len(t), 1 / (nodes[j] - nodes[m]), dtype=nodes.dtype)
            for k in range(n):
                if k != j and k != m:
                    term *= (t - nodes[k]) / (nodes[j] - nodes[k])
            Ld[:, j] += term
    return Ld


class Basis:
    """Gauss-Legendre nodal basis of order P (P+1 points per direction);
    dtype=np.longdouble builds every table in 80-bit extended precision."""

    def __init__(self, P, dtype=np.float64):
        self.P = P
        self.n = P + 1
        self.nodes, self.weights = gauss_legendre(P, dtype)
        self.D = lagrange_deriv(self.nodes, self.nodes)          # D[i, j] = l_j'(xi_i)
        self.bp = lagrange_eval(self.nodes, 1.0)[0]               # l_j(+1)
        self.bm = lagrange_eval(self.nodes, -1.0)[0]              # l_j(-1)
