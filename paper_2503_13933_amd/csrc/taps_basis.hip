// 1D C-HiDeNN basis, separable source factors, Gauss-quadrature assembly and
// TD interpolation kernels (paper Sec. 2.1, 2.3, 2.4, 2.5).
//
// These run once per problem (setup) or once per output grid, so they favour
// simple one-thread-per-output layouts; the per-point patch systems are tiny
// (at most 2s+1+p+1 <= 11 unknowns) and solved in thread-private memory.
#include "taps_internal.hpp"

namespace {

constexpr int kMaxPatch = 2 * TAPS_MAX_S + 1;
constexpr int kMaxSys = kMaxPatch + TAPS_MAX_S + 1;
constexpr int kMaxL = 2 * TAPS_MAX_S + 2;

struct BasisArgs {
  const double* x;
  int n, s, p;
  double a;
};

// Cubic B-spline kernel and its derivative (argument >= 0).
__device__ inline double kernel_phi(double z) {
  z = fabs(z);
  if (z <= 0.5) return 2.0 / 3.0 - 4.0 * z * z + 4.0 * z * z * z;
  if (z <= 1.0) return 4.0 / 3.0 - 4.0 * z + 4.0 * z * z - (4.0 / 3.0) * z * z * z;
  return 0.0;
}
__device__ inline double kernel_dphi(double z) {
  z = fabs(z);
  if (z <= 0.5) return -8.0 * z + 12.0 * z * z;
  if (z <= 1.0) return -4.0 + 8.0 * z - 4.0 * z * z;
  return 0.0;
}

// Patch function W^i_j(xq) and its derivative for j = j0 .. j0+np-1: the
// cardinal functions of radial-basis interpolation with degree-p polynomial
// reproduction on node i's patch (Sec. 2.1, convolution patch function).
__device__ void patch_weights(const BasisArgs& B, int i, double xq, double* W, double* dW,
                              int* j0_out, int* np_out) {
  const int lo = max(0, i - B.s), hi = min(B.n - 1, i + B.s);
  const int np = hi - lo + 1;
  const int sh = max(B.s, 1);
  const int hlo = max(0, i - sh), hhi = min(B.n - 1, i + sh);
  const double h = (B.x[hhi] - B.x[hlo]) / double(hhi - hlo);
  const double L = B.a * h;
  const double xi0 = B.x[i];
  const int sz = np + B.p + 1;
  double G[kMaxSys][kMaxSys];
  double r0[kMaxSys], r1[kMaxSys];
  for (int j = 0; j < np; ++j) {
    const double xj = B.x[lo + j];
    for (int k = 0; k < np; ++k) G[j][k] = kernel_phi(fabs(xj - B.x[lo + k]) / L);
    const double xi = (xj - xi0) / h;
    double pw = 1.0;
    for (int q = 0; q <= B.p; ++q) {
      G[j][np + q] = pw;
      G[np + q][j] = pw;
      pw *= xi;
    }
    const double dd = xq - xj;
    r0[j] = kernel_phi(fabs(dd) / L);
    const double sg = dd > 0.0 ? 1.0 : (dd < 0.0 ? -1.0 : 0.0);
    r1[j] = kernel_dphi(fabs(dd) / L) * sg / L;
  }
  for (int q = 0; q <= B.p; ++q)
    for (int k = 0; k <= B.p; ++k) G[np + q][np + k] = 0.0;
  {
    const double xi = (xq - xi0) / h;
    double pw = 1.0, dpw = 0.0;  // xi^q and q xi^(q-1)
    for (int q = 0; q <= B.p; ++q) {
      r0[np + q] = pw;
      r1[np + q] = dpw / h;
      dpw = (q + 1) * pw;
      pw *= xi;
    }
  }
  // Gaussian elimination with partial pivoting, two right-hand sides.
  for (int c = 0; c < sz; ++c) {
    int piv = c;
    double best = fabs(G[c][c]);
    for (int r = c + 1; r < sz; ++r)
      if (fabs(G[r][c]) > best) {
        best = fabs(G[r][c]);
        piv = r;
      }
    if (piv != c) {
      for (int k = 0; k < sz; ++k) {
        double t = G[c][k];
        G[c][k] = G[piv][k];
        G[piv][k] = t;
      }
      double t0 = r0[c]; r0[c] = r0[piv]; r0[piv] = t0;
      double t1 = r1[c]; r1[c] = r1[piv]; r1[piv] = t1;
    }
    const double inv = 1.0 / G[c][c];
    for (int r = c + 1; r < sz; ++r) {
      const double f = G[r][c] * inv;
      if (f == 0.0) continue;
      for (int k = c; k < sz; ++k) G[r][k] -= f * G[c][k];
      r0[r] -= f * r0[c];
      r1[r] -= f * r1[c];
    }
  }
  for (int c = sz - 1; c >= 0; --c) {
    double a0 = r0[c], a1 = r1[c];
    for (int k = c + 1; k < sz; ++k) {
      a0 -= G[c][k] * r0[k];
      a1 -= G[c][k] * r1[k];
    }
    r0[c] = a0 / G[c][c];
    r1[c] = a1 / G[c][c];
  }
  for (int j = 0; j < np; ++j) {
    W[j] = r0[j];
    dW[j] = r1[j];
  }
  *j0_out = lo;
  *np_out = np;
}

// Element containing xq: largest e with x[e] <= xq, clamped to [0, n-2].
__device__ inline int element_of(const double* x, int n, double xq) {
  int lo = 0, hi = n - 1;  // invariant: answer in [lo, hi)
  if (xq < x[0]) return 0;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (x[mid] <= xq) lo = mid; else hi = mid;
  }
  return min(lo, n - 2);
}

// Ntilde and Btilde of the L = 2s+2 window nodes at xq (Sec. 2.1, Eq. (1):
// hats of the element's two nodes times their patch functions).
__device__ void shape_point(const BasisArgs& B, double xq, int* first, double* N, double* dN) {
  const int Lw = 2 * B.s + 2;
  const int e = element_of(B.x, B.n, xq);
  const int f = min(max(e - B.s, 0), B.n - Lw);
  for (int l = 0; l < Lw; ++l) {
    N[l] = 0.0;
    dN[l] = 0.0;
  }
  const double x0 = B.x[e], x1 = B.x[e + 1], he = x1 - x0;
  for (int t = 0; t < 2; ++t) {
    const int i = e + t;
    const double Ni = t == 0 ? (x1 - xq) / he : (xq - x0) / he;
    const double dNi = t == 0 ? -1.0 / he : 1.0 / he;
    double W[kMaxPatch], dW[kMaxPatch];
    int j0, np;
    patch_weights(B, i, xq, W, dW, &j0, &np);
    for (int jj = 0; jj < np; ++jj) {
      const int l = j0 + jj - f;
      N[l] += Ni * W[jj];
      dN[l] += dNi * W[jj] + Ni * dW[jj];
    }
  }
  *first = f;
}

struct GaussRule {
  double xi[TAPS_MAX_GAUSS];
  double w[TAPS_MAX_GAUSS];
};

__global__ void k_gauss(const double* __restrict__ x, int n, int ng, GaussRule rule,
                        double* __restrict__ xg, double* __restrict__ wg) {
  const long idx = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (idx >= long(n - 1) * ng) return;
  const int e = int(idx / ng), g = int(idx % ng);
  const double lo = x[e], hi = x[e + 1], half = 0.5 * (hi - lo);
  xg[idx] = lo + half * (1.0 + rule.xi[g]);
  wg[idx] = half * rule.w[g];
}

__global__ void k_shape(BasisArgs B, int npts, const double* __restrict__ pts, double* __restrict__ N,
                        double* __restrict__ dN, int* __restrict__ first) {
  const int pidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (pidx >= npts) return;
  const int Lw = 2 * B.s + 2;
  double n_[kMaxL], d_[kMaxL];
  int f;
  shape_point(B, pts[pidx], &f, n_, d_);
  for (int l = 0; l < Lw; ++l) {
    N[long(pidx) * Lw + l] = n_[l];
    if (dN) dN[long(pidx) * Lw + l] = d_[l];
  }
  first[pidx] = f;
}

struct SourceArgs {
  int kind, npts, ncols, nparams;
  double prm[8];
};

__global__ void k_source(SourceArgs S, const double* __restrict__ pts, const double* __restrict__ centers,
                         BasisArgs B, double* __restrict__ out) {
  const long idx = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (idx >= long(S.npts) * S.ncols) return;
  const int c = int(idx / S.npts), p = int(idx % S.npts);
  const double x = pts[p];
  double v = 0.0;
  switch (S.kind) {
    case TAPS_SRC_GAUSS: {
      const double dx = x - centers[c];
      v = S.prm[0] * exp(-2.0 * dx * dx / (S.prm[1] * S.prm[1]));
      break;
    }
    case TAPS_SRC_TOPLAYER:
      v = (S.prm[0] - x <= S.prm[1]) ? 1.0 : 0.0;
      break;
    case TAPS_SRC_POLY: {
      double pw = 1.0;
      for (int q = 0; q < S.nparams; ++q) {
        v += S.prm[q] * pw;
        pw *= x;
      }
      break;
    }
    case TAPS_SRC_SIN:
      v = S.prm[0] * sin(S.prm[1] * x);
      break;
    case TAPS_SRC_NODAL: {
      double n_[kMaxL], d_[kMaxL];
      int f;
      shape_point(B, x, &f, n_, d_);
      const int l = c - f;
      v = (l >= 0 && l < 2 * B.s + 2) ? n_[l] : 0.0;
      break;
    }
    case TAPS_SRC_EXPQUAD: {
      const double* r = centers + 8L * c;   // s, beta, lambda, p0, p1, p2, q0, q1
      const double xi = x - r[0];
      v = ((r[5] * xi + r[4]) * xi + r[3]) * exp(-r[1] * xi * xi + r[2] * x) + (r[6] + r[7] * x);
      break;
    }
  }
  out[idx] = v;
}

constexpr int kMaxAssembleKinds = 8;

// NODAL source columns: one thread per point computes the point's shape
// values once and writes every column (nonzero only in its window), column
// by column so that neighbouring points' stores are adjacent.
__global__ void k_source_nodal(int npts, int ncols, const double* __restrict__ pts, BasisArgs B,
                               double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  double n_[kMaxL], d_[kMaxL];
  int f;
  shape_point(B, pts[p], &f, n_, d_);
  const int L = 2 * B.s + 2;
  for (int c = 0; c < ncols; ++c) {
    const int l = c - f;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxL; ++k) v = (k == l && k < L) ? n_[k] : v;
    out[long(c) * npts + p] = v;
  }
}

struct BandArgs {
  int n, s, ng, K;
  int kinds[kMaxAssembleKinds];
  int bnode[kMaxAssembleKinds];
};

// Band entry (kind kk, row i, offset o): sum over the elements that contain
// both node i and node j = i+o-w of the Gauss sum of the kind's integrand.
__global__ void k_band(BandArgs A, const double* __restrict__ Ng, const double* __restrict__ dNg,
                       const int* __restrict__ firstg, const double* __restrict__ wg,
                       const double* __restrict__ coef, double* __restrict__ band) {
  const int w = 2 * A.s + 1, BW = 2 * w + 1, Lw = 2 * A.s + 2;
  const long ngp = long(A.n - 1) * A.ng;
  const long idx = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (idx >= long(A.K) * A.n * BW) return;
  const int kk = int(idx / (long(A.n) * BW));
  const int rem = int(idx % (long(A.n) * BW));
  const int i = rem / BW, o = rem % BW;
  const int j = i + o - w;
  double val = 0.0;
  if (j >= 0 && j < A.n) {
    const int kind = A.kinds[kk];
    if (kind == TAPS_BMASS) {
      val = (i == A.bnode[kk] && j == i) ? 1.0 : 0.0;
    } else {
      const int elo = max(max(i, j) - A.s - 1, 0), ehi = min(min(i, j) + A.s, A.n - 2);
      for (int e = elo; e <= ehi; ++e) {
        for (int g = 0; g < A.ng; ++g) {
          const long P = long(e) * A.ng + g;
          const int f = firstg[P];
          const bool dtest = kind == TAPS_STIFF || kind == TAPS_WSTIFF;
          const bool dtrial = kind == TAPS_STIFF || kind == TAPS_WSTIFF || kind == TAPS_DDT || kind == TAPS_WDDT;
          const double ai = dtest ? dNg[P * Lw + (i - f)] : Ng[P * Lw + (i - f)];
          const double bj = dtrial ? dNg[P * Lw + (j - f)] : Ng[P * Lw + (j - f)];
          const bool weighted = kind == TAPS_WMASS || kind == TAPS_WSTIFF || kind == TAPS_WDDT;
          const double c = weighted ? wg[P] * coef[P] : wg[P];
          val += c * ai * bj;
          if (kind == TAPS_WDDT)   // + int Ntilde_i c' Ntilde_j
            val += wg[P] * coef[ngp + P] * ai * Ng[P * Lw + (j - f)];
        }
      }
    }
  }
  band[idx] = val;
}

// Load vector entry F[i][r] = sum_{elements around i} sum_g w_g Ntilde_i f_r.
__global__ void k_load(int n, int s, int ng, int R, const double* __restrict__ Ng,
                       const int* __restrict__ firstg, const double* __restrict__ wg,
                       const double* __restrict__ fg, double* __restrict__ F) {
  const long idx = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (idx >= long(n) * R) return;
  const int r = int(idx / n), i = int(idx % n);
  const int Lw = 2 * s + 2;
  const long ngp = long(n - 1) * ng;
  const int elo = max(i - s - 1, 0), ehi = min(i + s, n - 2);
  double val = 0.0;
  for (int e = elo; e <= ehi; ++e)
    for (int g = 0; g < ng; ++g) {
      const long P = long(e) * ng + g;
      val += wg[P] * Ng[P * Lw + (i - firstg[P])] * fg[long(r) * ngp + P];
    }
  F[long(i) * R + r] = val;
}

__global__ void k_interp(int npts, int L, const double* __restrict__ N, const int* __restrict__ first,
                         int n, int M, const double* __restrict__ U, double* __restrict__ Phi) {
  const long idx = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (idx >= long(npts) * M) return;
  const int p = int(idx / M), m = int(idx % M);
  const int f = first[p];
  if (f < 0 || f + L > n) {  // inconsistent window: flag instead of reading out of bounds
    Phi[idx] = __builtin_nan("");
    return;
  }
  double v = 0.0;
  for (int l = 0; l < L; ++l) v += N[long(p) * L + l] * U[long(f + l) * M + m];
  Phi[idx] = v;
}

// Y = alpha diag-scaled (A X): one thread per output entry (i, c); the band
// row i is read once per column, X rows i-w..i+w stay in cache across c.
__global__ void k_band_apply(int n, int w, const double* __restrict__ band, int ncols, const double* __restrict__ X,
                             int ldx, const double* __restrict__ scale, double alpha, double* __restrict__ Y, int ldy) {
  const long idx = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (idx >= long(n) * ncols) return;
  const int i = int(idx / ncols), c = int(idx - long(i) * ncols);
  const int BW = 2 * w + 1;
  const int j0 = max(0, i - w), j1 = min(n - 1, i + w);
  double v = 0.0;
  for (int j = j0; j <= j1; ++j) v += band[long(i) * BW + (j - i + w)] * X[long(j) * ldx + c];
  Y[long(i) * ldy + c] = alpha * (scale ? scale[c] : 1.0) * v;
}

struct TdInnerArgs {
  int D, Ma, Mb;
  int n[TAPS_MAX_DIMS], w[TAPS_MAX_DIMS];
  const double* band[TAPS_MAX_DIMS];
  const double* A[TAPS_MAX_DIMS];
  const double* B[TAPS_MAX_DIMS];
};

// G[m][m'] = prod_d A_d[:, m]^T S_d B_d[:, m'] (S_d banded): block (m, m'),
// rows strided over the threads, one block-wide sum per dim in a fixed order.
__global__ __launch_bounds__(256) void k_td_gram(TdInnerArgs T, double* __restrict__ G) {
  __shared__ double red[256];
  const int m = blockIdx.x, mp = blockIdx.y, tid = threadIdx.x;
  double prod = 1.0;
  for (int d = 0; d < T.D; ++d) {
    const int n = T.n[d], w = T.w[d], BW = 2 * w + 1;
    const double* A = T.A[d];
    const double* B = T.B[d];
    const double* band = T.band[d];
    double acc = 0.0;
    for (int i = tid; i < n; i += 256) {
      double sb = 0.0;
      for (int j = max(0, i - w); j <= min(n - 1, i + w); ++j) sb += band[long(i) * BW + (j - i + w)] * B[long(j) * T.Mb + mp];
      acc += A[long(i) * T.Ma + m] * sb;
    }
    red[tid] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    prod *= red[0];
    __syncthreads();
  }
  if (tid == 0) G[long(m) * T.Mb + mp] = prod;
}

// out[Ma*Mb] = sum of every entry of G, in row order.
__global__ void k_td_total(int len, double* __restrict__ G) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int t = 0; t < len; ++t) s += G[t];
  G[len] = s;
}

BasisArgs basis_args(const taps_basis1d_t* b) {
  BasisArgs B;
  B.x = b->d_x;
  B.n = b->n_nodes;
  B.s = b->s;
  B.p = b->p;
  B.a = b->a;
  return B;
}

inline int grid_for(long work, int block) { return int((work + block - 1) / block); }

}  // namespace

using namespace taps;

extern "C" {

taps_status taps_gauss_points(taps_handle_t h, const taps_basis1d_t* b, double* d_xg, double* d_wg,
                              hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  TAPS_TRY(check_basis(h, b));
  if (!d_xg || !d_wg) return fail(h, TAPS_ERR_INVALID, "null output");
  GaussRule rule;
  gauss_legendre(b->n_gauss, rule.xi, rule.w);
  const long work = long(b->n_nodes - 1) * b->n_gauss;
  k_gauss<<<grid_for(work, 256), 256, 0, stream>>>(b->d_x, b->n_nodes, b->n_gauss, rule, d_xg, d_wg);
  TAPS_LAUNCHED(h, "k_gauss");
  return TAPS_OK;
}

taps_status taps_shape1d(taps_handle_t h, const taps_basis1d_t* b, int32_t n_pts, const double* d_pts,
                         double* d_N, double* d_dN, int32_t* d_first, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  TAPS_TRY(check_basis(h, b));
  if (n_pts < 0) return fail(h, TAPS_ERR_INVALID, "n_pts < 0");
  if (n_pts == 0) return TAPS_OK;
  if (!d_pts || !d_N || !d_first) return fail(h, TAPS_ERR_INVALID, "null pointer");
  k_shape<<<grid_for(n_pts, 128), 128, 0, stream>>>(basis_args(b), n_pts, d_pts, d_N, d_dN, d_first);
  TAPS_LAUNCHED(h, "k_shape");
  return TAPS_OK;
}

taps_status taps_source1d(taps_handle_t h, taps_source_kind kind, int32_t n_pts, const double* d_pts,
                          int32_t n_cols, int32_t n_params, const double* params,
                          const double* d_centers, const taps_basis1d_t* basis, double* d_out,
                          hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (n_pts < 0 || n_cols < 0) return fail(h, TAPS_ERR_INVALID, "negative size");
  if (n_pts == 0 || n_cols == 0) return TAPS_OK;
  if (!d_pts || !d_out) return fail(h, TAPS_ERR_INVALID, "null pointer");
  if (n_params < 0 || n_params > 8 || (n_params > 0 && !params))
    return fail(h, TAPS_ERR_INVALID, "n_params must be 0..8 with params");
  SourceArgs S{};
  S.kind = kind;
  S.npts = n_pts;
  S.ncols = n_cols;
  S.nparams = n_params;
  for (int q = 0; q < n_params; ++q) S.prm[q] = params[q];
  BasisArgs B{};
  switch (kind) {
    case TAPS_SRC_GAUSS:
      if (!d_centers || n_params < 2) return fail(h, TAPS_ERR_INVALID, "GAUSS needs centers, amp, radius");
      break;
    case TAPS_SRC_TOPLAYER:
      if (n_params < 2) return fail(h, TAPS_ERR_INVALID, "TOPLAYER needs surface and depth");
      break;
    case TAPS_SRC_POLY:
    case TAPS_SRC_SIN:
      if (n_cols != 1) return fail(h, TAPS_ERR_INVALID, "POLY/SIN take one column");
      if (kind == TAPS_SRC_SIN && n_params < 2) return fail(h, TAPS_ERR_INVALID, "SIN needs amp, omega");
      break;
    case TAPS_SRC_EXPQUAD:
      if (!d_centers) return fail(h, TAPS_ERR_INVALID, "EXPQUAD needs 8 coefficients per column");
      break;
    case TAPS_SRC_NODAL:
      TAPS_TRY(check_basis(h, basis));
      if (n_cols != basis->n_nodes) return fail(h, TAPS_ERR_INVALID, "NODAL needs n_cols = n_nodes");
      B = basis_args(basis);
      break;
    default:
      return fail(h, TAPS_ERR_INVALID, "unknown source kind %d", int(kind));
  }
  if (kind == TAPS_SRC_NODAL) {
    k_source_nodal<<<grid_for(n_pts, 128), 128, 0, stream>>>(n_pts, n_cols, d_pts, B, d_out);
    TAPS_LAUNCHED(h, "k_source_nodal");
    return TAPS_OK;
  }
  k_source<<<grid_for(long(n_pts) * n_cols, 256), 256, 0, stream>>>(S, d_pts, d_centers, B, d_out);
  TAPS_LAUNCHED(h, "k_source");
  return TAPS_OK;
}

taps_status taps_assemble1d(taps_handle_t h, const taps_basis1d_t* b, int32_t n_kinds,
                            const int32_t* kinds, const double* d_coef_g, const int32_t* bnode,
                            double* d_band, int32_t n_loads, const double* d_f_g, double* d_F,
                            hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  TAPS_TRY(check_basis(h, b));
  if (n_kinds < 0 || n_kinds > kMaxAssembleKinds)
    return fail(h, TAPS_ERR_UNSUPPORTED, "n_kinds=%d outside 0..%d", n_kinds, kMaxAssembleKinds);
  if (n_kinds > 0 && (!kinds || !d_band)) return fail(h, TAPS_ERR_INVALID, "null kinds/band");
  if (n_loads < 0) return fail(h, TAPS_ERR_INVALID, "n_loads < 0");
  if (n_loads > 0 && (!d_f_g || !d_F)) return fail(h, TAPS_ERR_INVALID, "null load pointers");
  BandArgs A{};
  A.n = b->n_nodes;
  A.s = b->s;
  A.ng = b->n_gauss;
  A.K = n_kinds;
  for (int k = 0; k < n_kinds; ++k) {
    if (kinds[k] < TAPS_MASS || kinds[k] > TAPS_WDDT) return fail(h, TAPS_ERR_INVALID, "kind %d", kinds[k]);
    if ((kinds[k] == TAPS_WMASS || kinds[k] == TAPS_WSTIFF || kinds[k] == TAPS_WDDT) && !d_coef_g)
      return fail(h, TAPS_ERR_INVALID, "weighted kind %d needs coefficients", kinds[k]);
    A.kinds[k] = kinds[k];
    A.bnode[k] = -1;
    if (kinds[k] == TAPS_BMASS) {
      if (!bnode || bnode[k] < 0 || bnode[k] >= b->n_nodes)
        return fail(h, TAPS_ERR_INVALID, "BMASS needs a node index");
      A.bnode[k] = bnode[k];
    }
  }
  const long ngp = long(b->n_nodes - 1) * b->n_gauss;
  const int Lw = 2 * b->s + 2;
  Bump bump;
  const size_t o_xg = bump.take(ngp * 8), o_wg = bump.take(ngp * 8);
  const size_t o_N = bump.take(ngp * Lw * 8), o_dN = bump.take(ngp * Lw * 8);
  const size_t o_f = bump.take(ngp * 4);
  TAPS_TRY(need_ws(h, bump.off, stream));
  char* ws = static_cast<char*>(h->ws);
  double* xg = reinterpret_cast<double*>(ws + o_xg);
  double* wg = reinterpret_cast<double*>(ws + o_wg);
  double* Ng = reinterpret_cast<double*>(ws + o_N);
  double* dNg = reinterpret_cast<double*>(ws + o_dN);
  int* firstg = reinterpret_cast<int*>(ws + o_f);
  TAPS_TRY(taps_gauss_points(h, b, xg, wg, stream));
  TAPS_TRY(taps_shape1d(h, b, int32_t(ngp), xg, Ng, dNg, firstg, stream));
  if (n_kinds > 0) {
    const long work = long(n_kinds) * b->n_nodes * band_width(b->s);
    k_band<<<grid_for(work, 256), 256, 0, stream>>>(A, Ng, dNg, firstg, wg, d_coef_g, d_band);
    TAPS_LAUNCHED(h, "k_band");
  }
  if (n_loads > 0) {
    const long work = long(b->n_nodes) * n_loads;
    k_load<<<grid_for(work, 256), 256, 0, stream>>>(b->n_nodes, b->s, b->n_gauss, n_loads, Ng, firstg, wg,
                                                    d_f_g, d_F);
    TAPS_LAUNCHED(h, "k_load");
  }
  return TAPS_OK;
}

taps_status taps_load1d(taps_handle_t h, int32_t n_nodes, int32_t s, int32_t n_gauss, const double* d_N,
                        const int32_t* d_first, const double* d_wg, int32_t n_loads, const double* d_f_g,
                        double* d_F, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (n_nodes < 2 * s + 2 || n_nodes < 2 || s < 0 || s > TAPS_MAX_S || n_gauss < 1 || n_gauss > TAPS_MAX_GAUSS ||
      n_loads < 0)
    return fail(h, TAPS_ERR_INVALID, "n_nodes=%d s=%d n_gauss=%d n_loads=%d", n_nodes, s, n_gauss, n_loads);
  if (n_loads == 0) return TAPS_OK;
  if (!d_N || !d_first || !d_wg || !d_f_g || !d_F) return fail(h, TAPS_ERR_INVALID, "null pointer");
  const long work = long(n_nodes) * n_loads;
  k_load<<<grid_for(work, 256), 256, 0, stream>>>(n_nodes, s, n_gauss, n_loads, d_N, d_first, d_wg, d_f_g, d_F);
  TAPS_LAUNCHED(h, "k_load");
  return TAPS_OK;
}

taps_status taps_band_apply(taps_handle_t h, int32_t n, int32_t s, const double* d_band, int32_t n_cols,
                            const double* d_X, int32_t ldx, const double* d_scale, double alpha, double* d_Y,
                            int32_t ldy, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (n < 1 || n_cols < 0 || s < 0 || s > TAPS_MAX_S) return fail(h, TAPS_ERR_INVALID, "n=%d n_cols=%d s=%d", n, n_cols, s);
  if (ldx < n_cols || ldy < n_cols) return fail(h, TAPS_ERR_INVALID, "leading dimensions %d, %d < %d", ldx, ldy, n_cols);
  if (n_cols == 0) return TAPS_OK;
  if (!d_band || !d_X || !d_Y) return fail(h, TAPS_ERR_INVALID, "null pointer");
  k_band_apply<<<grid_for(long(n) * n_cols, 256), 256, 0, stream>>>(n, 2 * s + 1, d_band, n_cols, d_X, ldx, d_scale,
                                                                     alpha, d_Y, ldy);
  TAPS_LAUNCHED(h, "k_band_apply");
  return TAPS_OK;
}

taps_status taps_td_inner(taps_handle_t h, int32_t D, const int32_t* n, const int32_t* s,
                          const double* const* d_band, int32_t Ma, const double* const* d_A, int32_t Mb,
                          const double* const* d_B, double* d_out, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (D < 1 || D > TAPS_MAX_DIMS || Ma < 1 || Mb < 1 || Ma > 1024 || Mb > 1024)
    return fail(h, TAPS_ERR_INVALID, "D=%d Ma=%d Mb=%d", D, Ma, Mb);
  if (!n || !s || !d_band || !d_A || !d_B || !d_out) return fail(h, TAPS_ERR_INVALID, "null pointer");
  TdInnerArgs T{};
  T.D = D;
  T.Ma = Ma;
  T.Mb = Mb;
  for (int d = 0; d < D; ++d) {
    if (n[d] < 1 || s[d] < 0 || s[d] > TAPS_MAX_S) return fail(h, TAPS_ERR_INVALID, "dim %d: n=%d s=%d", d, n[d], s[d]);
    if (!d_band[d] || !d_A[d] || !d_B[d]) return fail(h, TAPS_ERR_INVALID, "dim %d: null pointer", d);
    T.n[d] = n[d];
    T.w[d] = 2 * s[d] + 1;
    T.band[d] = d_band[d];
    T.A[d] = d_A[d];
    T.B[d] = d_B[d];
  }
  k_td_gram<<<dim3(Ma, Mb), 256, 0, stream>>>(T, d_out);
  TAPS_LAUNCHED(h, "k_td_gram");
  k_td_total<<<1, 64, 0, stream>>>(Ma * Mb, d_out);
  TAPS_LAUNCHED(h, "k_td_total");
  return TAPS_OK;
}

taps_status taps_interp1d(taps_handle_t h, int32_t n_pts, int32_t L, const double* d_N,
                          const int32_t* d_first, int32_t n_nodes, int32_t M, const double* d_U,
                          double* d_Phi, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (n_pts < 0 || L < 1 || M < 1 || n_nodes < L) return fail(h, TAPS_ERR_INVALID, "bad sizes");
  if (n_pts == 0) return TAPS_OK;
  if (!d_N || !d_first || !d_U || !d_Phi) return fail(h, TAPS_ERR_INVALID, "null pointer");
  k_interp<<<grid_for(long(n_pts) * M, 256), 256, 0, stream>>>(n_pts, L, d_N, d_first, n_nodes, M, d_U, d_Phi);
  TAPS_LAUNCHED(h, "k_interp");
  return TAPS_OK;
}

}  // extern "C"
