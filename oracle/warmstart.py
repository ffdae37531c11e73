"""Data of the learned warm start (oracle; test infrastructure only).

The network learns a slab's factors from its parameters and its carried
initial condition.  Readings (the paper has no learned part; these fix the
interface the device code follows):

  * canonical form of converged factors: modes ordered by
    lambda_m = prod_d ||U_d[:, m]||_2 (largest first, ties by index), columns
    of dims d >= 1 scaled to unit 2-norm with the sign that makes their
    largest-magnitude entry (first on ties) positive; scale and sign go into
    U_0, so the field is unchanged.  Modes with a zero column stay as they are.
  * coarse factors: the fine factor's C-HiDeNN interpolant sampled at the
    coarse nodes (uniform, end points included); prolongation back to the
    fine nodes interpolates the coarse nodal values with the C-HiDeNN basis of
    the coarse grid.  By the Kronecker-delta property sampling after
    prolongation returns the coarse values.
  * input features: (P, r, k, y0) mapped linearly to [-1, 1] over their
    sampling ranges, then the carried field sampled on a 4 x 4 x 4 coarse grid.
  * fallback: a warm start is dropped for the plain initialisation when its
    residual after sweep 1 exceeds the median of the plain initialisation's
    sweep-1 residuals, or when the residual grows from sweep 1 to sweep 2.
"""
import numpy as np

from . import basis, reconstruct

PARAM_RANGES = {"power": (100.0, 300.0), "radius": (0.030, 0.080), "k": (0.010, 0.030), "y0": (0.3, 0.7)}


def canonicalize(U):
    D = len(U)
    M = U[0].shape[1]
    nrm = np.array([[np.linalg.norm(U[d][:, m]) for m in range(M)] for d in range(D)])
    lam = np.prod(nrm, axis=0)
    order = sorted(range(M), key=lambda m: (-lam[m], m))
    out = [np.zeros_like(u) for u in U]
    for r, m in enumerate(order):
        cols = [U[d][:, m].copy() for d in range(D)]
        if np.all(nrm[1:, m] > 0):
            for d in range(1, D):
                i = int(np.argmax(np.abs(cols[d])))
                s = 1.0 if cols[d][i] >= 0 else -1.0
                cols[0] = cols[0] * (s * nrm[d, m])
                cols[d] = cols[d] * (s / nrm[d, m])
        for d in range(D):
            out[d][:, r] = cols[d]
    return out


def coarse_nodes(ax, nc):
    return np.linspace(ax.lo, ax.hi, nc)


def sample(ax, U, nc):
    """Fine factor (n x M) -> values at nc coarse nodes."""
    return reconstruct.factor_at(ax.nodes(), ax.s, ax.a, ax.p, U, coarse_nodes(ax, nc))


def prolong(ax, Uc, s=2, a=20.0, p=2):
    """Coarse nodal values (nc x M) -> fine factor by C-HiDeNN interpolation on the coarse grid."""
    return reconstruct.factor_at(coarse_nodes(ax, Uc.shape[0]), s, a, p, Uc, ax.nodes())


def param_features(case):
    v = []
    for name, (lo, hi) in PARAM_RANGES.items():
        v.append(2.0 * (getattr(case, name) - lo) / (hi - lo) - 1.0)
    return np.array(v)


def ic_features(axes, V, nc=4):
    """Carried field prod_d V_d sampled on nc^3 coarse points (zeros without one)."""
    if V is None or V[0].shape[1] == 0:
        return np.zeros(nc ** 3)
    Phis = [sample(ax, Vd, nc) for ax, Vd in zip(axes[:3], V)]
    return reconstruct.reconstruct_grid(Phis).reshape(-1)


def restart_plain(rho1, rho2, plain_median_rho1):
    """True when the warm start lost: its sweep-1 residual is above the plain
    start's median, it grew from sweep 1 to 2, or either residual is not a
    number (a breakdown counts as a loss)."""
    return not (rho1 <= plain_median_rho1) or not (rho2 <= rho1)
