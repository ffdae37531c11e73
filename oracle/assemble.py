"""1D Gauss-quadrature matrices and load vectors (oracle).

Paper Sec. 2.5: after substituting the 1D C-HiDeNN interpolation into the weak
form, every term factors into 1D integrals over one dimension -- the stiffness
int B_i B_j dx, the mass-type int N_i N_j dt, the coefficient-weighted mass
int N_i k N_j dk, the time-derivative int N_i dN_j/dt dt, and the forcing
int N_i f dx.  Test index first, trial index second.

Each matrix is the quadrature sum written out:  A[i,j] = sum_g w_g a_i(x_g) b_j(x_g),
i.e. A = Phi_a^T diag(w) Phi_b with Phi the (points x nodes) shape matrices.
The boundary point mass e_b e_b^T (a convection face) is included for the
optional Neumann-convection term of Sec. 2.4.
"""
import numpy as np
import scipy.sparse as sp

from . import basis, quadrature

KINDS = ("mass", "stiff", "ddt", "wmass", "bmass", "wstiff", "wddt")


class Dim1D:
    """One dimension: nodes, hyperparameters, Gauss rule and shape matrices."""

    def __init__(self, nodes, s, a, p, n_gauss=5, fixed=()):
        self.nodes = np.asarray(nodes, dtype=np.float64)
        self.n = len(self.nodes)
        self.s, self.a, self.p, self.n_gauss = s, a, p, n_gauss
        self.fixed = tuple(int(f) for f in fixed)
        self.xg, self.wg, self.elem = quadrature.gauss_points(self.nodes, n_gauss)
        self.Ng, self.Bg = basis.shape_matrices(self.nodes, s, a, p, self.xg)

    def matrix(self, kind, coef=None, bnode=None, dcoef=None):
        """Sparse n x n matrix of one kind.

        Kinds 'wmass' (int c N_i N_j), 'wstiff' (int c B_i B_j) and 'wddt'
        (int N_i d/dx (c N_j) = int N_i (c' N_j + c B_j), the time derivative
        of a product with a solution-dependent coefficient, Appendix A) take
        coef = callable c(x) or values at the Gauss points; 'wddt' also takes
        dcoef = c' likewise.  Kind 'bmass' takes bnode = the boundary node."""
        W = sp.diags(self.wg)
        val = lambda f: f(self.xg) if callable(f) else np.asarray(f, dtype=np.float64)
        if kind == "mass":
            A = self.Ng.T @ W @ self.Ng
        elif kind == "stiff":
            A = self.Bg.T @ W @ self.Bg
        elif kind == "ddt":
            A = self.Ng.T @ W @ self.Bg
        elif kind == "wmass":
            A = self.Ng.T @ sp.diags(self.wg * val(coef)) @ self.Ng
        elif kind == "wstiff":
            A = self.Bg.T @ sp.diags(self.wg * val(coef)) @ self.Bg
        elif kind == "wddt":
            A = self.Ng.T @ sp.diags(self.wg * val(dcoef)) @ self.Ng + self.Ng.T @ sp.diags(self.wg * val(coef)) @ self.Bg
        elif kind == "bmass":
            A = sp.csr_matrix(([1.0], ([bnode], [bnode])), shape=(self.n, self.n))
        else:
            raise ValueError(kind)
        return sp.csr_matrix(A)

    def load(self, f):
        """Load vector F[i] = int Ntilde_i f dx for a callable f or Gauss values."""
        fv = f(self.xg) if callable(f) else np.asarray(f, dtype=np.float64)
        return np.asarray(self.Ng.T @ (self.wg * fv)).ravel()

    def loads(self, fs):
        """n x R matrix of load vectors, one column per function."""
        return np.stack([self.load(f) for f in fs], axis=1) if fs else np.zeros((self.n, 0))
