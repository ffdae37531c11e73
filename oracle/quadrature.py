"""Gauss-Legendre quadrature on each 1D element.

Paper Sec. 2.1, the table comparing MLP and C-HiDeNN: C-HiDeNN integrates
with Gaussian quadrature.  The
paper gives no point count; this oracle uses the count the workload states
(5 by default), the same on every element.
"""
import numpy as np


def gauss_points(nodes, n_gauss):
    """Gauss points and weights of every element [x_e, x_{e+1}].

    Returns (xg, wg, elem) with xg, wg of shape ((n-1)*n_gauss,), element-major
    (point g of element e at index e*n_gauss+g), and elem[k] = element of point k.
    The weights include the Jacobian (x_{e+1}-x_e)/2.
    """
    xi, w = np.polynomial.legendre.leggauss(n_gauss)
    nodes = np.asarray(nodes, dtype=np.float64)
    xg, wg, el = [], [], []
    for e in range(len(nodes) - 1):
        lo, hi = nodes[e], nodes[e + 1]
        half = 0.5 * (hi - lo)
        for g in range(n_gauss):
            xg.append(lo + half * (1.0 + xi[g]))
            wg.append(half * w[g])
            el.append(e)
    return np.array(xg), np.array(wg), np.array(el, dtype=np.int64)
