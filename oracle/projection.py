"""The filter G of Sec. 2: nodal -> modal (Legendre) -> truncate -> nodal.

Test infrastructure only (see ``oracle/__init__``).

Sec. 2 defines G as a linear map from the high-order to the low-order DOFs and
Sec. 2.6 describes it as the usual DG modal filter: transform the nodal values
to Legendre modes, drop the modes above the low order, and re-evaluate at the
low-order nodes.  Per direction, with Gauss quadrature of the source order
(exact for the products involved), the modal coefficient of L_k is
    c_k = (2k+1)/2 sum_j w_j L_k(xi_j) u_j,
and the low-order nodal value at xi'_a is sum_{k <= P_dst} c_k L_k(xi'_a).
The 3D filter is the tensor product of the 1D one along x, y and z.
"""
import numpy as np

from .basis import Basis, legendre
from .dg import apply_line


def projection_matrix(P_src, P_dst):
    """G1[a, j]: 1D filter from P_src nodal values to P_dst nodal values."""
    if P_dst > P_src:
        raise ValueError("the filter maps to an order not above the source")
    src, dst = Basis(P_src), Basis(P_dst)
    G1 = np.zeros((dst.n, src.n))
    for k in range(P_dst + 1):
        Ld, _ = legendre(k, dst.nodes)
        Ls, _ = legendre(k, src.nodes)
        G1 += (2 * k + 1) / 2.0 * np.outer(Ld, src.weights * Ls)
    return G1


def project(q, P_src, P_dst):
    """Apply G = G1 (x) G1 (x) G1 to a block array [..., k, j, i]."""
    G1 = projection_matrix(P_src, P_dst)
    out = q
    for d in range(3):
        out = apply_line(out, G1, d)
    return out
