"""1D C-HiDeNN shape functions and derivatives (oracle).

Paper Sec. 2.1, Eq. (1): inside element e the field is
    u(x) = sum_{i in A^e} N_i(x) sum_{j in A_s^i} W^i_j(x) u_j = sum_k Ntilde_k(x) u_k,
with N_i the linear finite-element hats of the element's two nodes and W^i_j the
convolution patch function of node i's patch, controlled by patch size s,
dilation a and reproducing order p.  Sec. 2.5 writes the 1D derivative
Btilde_k = dNtilde_k/dx used by the stiffness and time-derivative integrals.

The paper defers the patch-function definition to its references.  Readings
taken here (all stated in the design notes):
  * patch of node i = nodes max(0,i-s) .. min(n-1,i+s) (truncated at the ends);
  * W^i_j(x) = radial-basis interpolation with polynomial reproduction: the
    cardinal functions of  [R P; P^T 0][c; b] = [u; 0]  on the patch, with
    R_jk = phi(|x_j - x_k| / (a h_i)),  P_jq = xi_j^q  (q = 0..p),
    xi = (x - x_i)/h_i,  h_i = mean node spacing of the patch (for s = 0, of
    the node's two adjacent elements);
  * phi = cubic B-spline kernel (zero beyond z = 1);
  * a point lying on an interior node belongs to the element on its right,
    the last node belongs to the last element.
Requires 0 <= p <= s so that every (truncated) patch has at least p+1 nodes.

parity unpinned: none -- every function here is pinned by tests/test_oracle_basis.py.
"""
import numpy as np
import scipy.sparse as sp


def phi(z):
    """Cubic B-spline kernel: 2/3-4z^2+4z^3 on [0,1/2], 4/3-4z+4z^2-4z^3/3 on (1/2,1], 0 beyond."""
    z = abs(z)
    if z <= 0.5:
        return 2.0 / 3.0 - 4.0 * z * z + 4.0 * z ** 3
    if z <= 1.0:
        return 4.0 / 3.0 - 4.0 * z + 4.0 * z * z - 4.0 / 3.0 * z ** 3
    return 0.0


def dphi(z):
    """d phi / dz for z >= 0."""
    z = abs(z)
    if z <= 0.5:
        return -8.0 * z + 12.0 * z * z
    if z <= 1.0:
        return -4.0 + 8.0 * z - 4.0 * z * z
    return 0.0


def patch(n, i, s):
    """Node indices of node i's patch."""
    return list(range(max(0, i - s), min(n - 1, i + s) + 1))


def patch_function(nodes, i, s, a, p, x):
    """W^i_j(x) and dW^i_j/dx for every j in node i's patch.

    Returns (js, W, dW)."""
    js = patch(len(nodes), i, s)
    xp = np.asarray(nodes, dtype=np.float64)[js]
    npatch = len(js)
    if npatch < p + 1:
        raise ValueError("patch smaller than p+1 nodes (need p <= s)")
    lo, hi = max(0, i - max(s, 1)), min(len(nodes) - 1, i + max(s, 1))
    h = (nodes[hi] - nodes[lo]) / (hi - lo)
    L = a * h
    xi = lambda t: (t - nodes[i]) / h
    size = npatch + p + 1
    G = np.zeros((size, size))
    for j in range(npatch):
        for k in range(npatch):
            G[j, k] = phi(abs(xp[j] - xp[k]) / L)
        for q in range(p + 1):
            G[j, npatch + q] = xi(xp[j]) ** q
            G[npatch + q, j] = xi(xp[j]) ** q
    rhs = np.zeros((size, 2))
    for j in range(npatch):
        d = x - xp[j]
        rhs[j, 0] = phi(abs(d) / L)
        rhs[j, 1] = dphi(abs(d) / L) * np.sign(d) / L
    for q in range(p + 1):
        rhs[npatch + q, 0] = xi(x) ** q
        rhs[npatch + q, 1] = q * xi(x) ** (q - 1) / h if q > 0 else 0.0
    sol = np.linalg.solve(G, rhs)
    return js, sol[:npatch, 0], sol[:npatch, 1]


def element_of(nodes, x):
    """Element e with x in [x_e, x_{e+1}); the last node maps to the last element."""
    n = len(nodes)
    e = int(np.searchsorted(nodes, x, side="right")) - 1
    return min(max(e, 0), n - 2)


def shape_at(nodes, s, a, p, x):
    """C-HiDeNN shape values and derivatives at one point.

    Returns (e, {k: (Ntilde_k(x), Btilde_k(x))}) over the nodes whose functions
    are nonzero on x's element."""
    nodes = np.asarray(nodes, dtype=np.float64)
    e = element_of(nodes, x)
    x0, x1 = nodes[e], nodes[e + 1]
    he = x1 - x0
    hats = ((e, (x1 - x) / he, -1.0 / he), (e + 1, (x - x0) / he, 1.0 / he))
    out = {}
    for i, Ni, dNi in hats:
        js, W, dW = patch_function(nodes, i, s, a, p, x)
        for j, w, dw in zip(js, W, dW):
            N0, B0 = out.get(j, (0.0, 0.0))
            out[j] = (N0 + Ni * w, B0 + dNi * w + Ni * dw)
    return e, out


def shape_matrices(nodes, s, a, p, pts):
    """Sparse (n_pts x n) matrices of Ntilde_k(pts) and Btilde_k(pts)."""
    rows, cols, nv, bv = [], [], [], []
    for r, x in enumerate(pts):
        _, vals = shape_at(nodes, s, a, p, float(x))
        for k, (N, B) in vals.items():
            rows.append(r)
            cols.append(k)
            nv.append(N)
            bv.append(B)
    shape = (len(pts), len(nodes))
    Nm = sp.csr_matrix((nv, (rows, cols)), shape=shape)
    Bm = sp.csr_matrix((bv, (rows, cols)), shape=shape)
    return Nm, Bm
