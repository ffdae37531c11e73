// Block-banded solve of the dim-d system (paper Sec. 2.6: with every factor
// but U^[d] fixed, the Galerkin condition is the linear system
// K^[d] U^[d] = Q^[d]; node-major it is block-banded with M x M blocks
// B_ij = sum_k A^k_d[i][j] C^k and block half-bandwidth w = 2s+1).
//
// One workgroup walks the block chain i = 0..n-1 (block LU without pivoting,
// right-looking, only the (w+1) x (w+1) active window is live):
//   P = B_kk ; P^-1 by Gauss-Jordan in LDS ; y_k = P^-1 b_k
//   Z_kj = P^-1 B_kj (j = k+1..k+w)        -- kept for back substitution
//   B_ij -= B_ik Z_kj, b_i -= B_ik y_k     (i, j = k+1..k+w)
// then x_k = y_k - sum_j Z_kj x_j from the last block row up.
// The window lives in an L2-resident ring buffer indexed by (i mod (w+1),
// j mod (w+1)); the pivot block, the column panel B_{k+1..k+w,k} and the
// row panel Z_{k,k+1..k+w} live in LDS.  Rows of fixed nodes are identity
// rows with zero right-hand side and their columns are zeroed, which keeps
// X = 0 there.
#include "taps_device.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstring>

namespace {

constexpr int kThreads = 256;
constexpr int kTI = 4;  // register tile of the trailing update (rows)
constexpr int kTJ = 4;  // (cols)

struct SolveArgs {
  int n, M, s, K;
  const double* band;   // K x n x (4s+3)
  const double* C;      // K x M x M
  const double* Q;      // n x M
  const uint8_t* fixed; // n or null
  double* X;            // n x M
  double* Zst;          // n x M x (w M)
  double* Yst;          // n x M
  double* win;          // (w+1)^2 x M x M
  double* rhs;          // (w+1) x M
  int* info;
};

__device__ inline bool is_fixed(const SolveArgs& A, int i) { return A.fixed && A.fixed[i]; }

// Write the original block B_ij (|i-j| <= w) into the window ring.
__device__ void build_block(const SolveArgs& A, int i, int j, double* dst) {
  const int M = A.M, MM = M * M, w = 2 * A.s + 1, BW = 2 * w + 1;
  const bool fi = is_fixed(A, i), fj = is_fixed(A, j);
  double coef[TAPS_MAX_KINDS];
  for (int k = 0; k < A.K; ++k) coef[k] = A.band[(long(k) * A.n + i) * BW + (j - i + w)];
  for (int t = threadIdx.x; t < MM; t += blockDim.x) {
    double v;
    if (fi) {
      v = (i == j && (t / M) == (t % M)) ? 1.0 : 0.0;
    } else if (fj) {
      v = 0.0;
    } else {
      v = 0.0;
      for (int k = 0; k < A.K; ++k) v += coef[k] * A.C[long(k) * MM + t];
    }
    dst[t] = v;
  }
}

__device__ void build_rhs(const SolveArgs& A, int i, double* dst) {
  const bool fi = is_fixed(A, i);
  for (int m = threadIdx.x; m < A.M; m += blockDim.x) dst[m] = fi ? 0.0 : A.Q[long(i) * A.M + m];
}

__global__ __launch_bounds__(kThreads) void k_block_lu(SolveArgs A) {
  extern __shared__ double lds[];
  const int M = A.M, MM = M * M, w = 2 * A.s + 1, W1 = w + 1, n = A.n, wM = w * M;
  double* sP = lds;            // M x M   pivot block -> its inverse
  double* Lp = sP + MM;        // (w M) x M column panel  (also row-panel staging M x (w M))
  double* Zp = Lp + w * MM;    // M x (w M)  Z row panel
  double* sb = Zp + w * MM;    // M   b_k
  double* sy = sb + M;         // M   y_k
  __shared__ int s_info;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) s_info = 0;
  auto WIN = [&](int i, int j) { return A.win + (long(i % W1) * W1 + (j % W1)) * MM; };
  auto RHS = [&](int i) { return A.rhs + long(i % W1) * M; };

  // initial window rows/cols 0..min(w, n-1)
  const int init_hi = min(w, n - 1);
  for (int i = 0; i <= init_hi; ++i) {
    for (int j = 0; j <= init_hi; ++j) build_block(A, i, j, WIN(i, j));
    build_rhs(A, i, RHS(i));
  }
  __syncthreads();

  for (int k = 0; k < n; ++k) {
    const int wa = min(w, n - 1 - k);  // active neighbours below / right
    if (k > 0) {
      const int t = k + w;
      if (t < n) {
        for (int j = k; j <= t; ++j) build_block(A, t, j, WIN(t, j));
        for (int i = k; i < t; ++i) build_block(A, i, t, WIN(i, t));
        build_rhs(A, t, RHS(t));
      }
      __syncthreads();
    }
    // ---- pivot block inverse (Gauss-Jordan, in place, no pivoting)
    {
      const double* P = WIN(k, k);
      for (int t = tid; t < MM; t += nt) sP[t] = P[t];
      const double* b = RHS(k);
      for (int m = tid; m < M; m += nt) sb[m] = b[m];
    }
    __syncthreads();
    for (int r = 0; r < M; ++r) {
      const double piv = sP[r * M + r];
      if (tid == 0 && s_info == 0 && (!(fabs(piv) > 0.0) || !isfinite(piv))) s_info = k + 1;
      const double inv = 1.0 / piv;
      for (int j = tid; j < M; j += nt)
        if (j != r) sP[r * M + j] *= inv;
      __syncthreads();
      for (int t = tid; t < MM; t += nt) {
        const int i = t / M, j = t % M;
        if (i != r && j != r) sP[t] -= sP[i * M + r] * sP[r * M + j];
      }
      __syncthreads();
      for (int i = tid; i < M; i += nt) {
        if (i != r) sP[i * M + r] *= -inv;
        else sP[r * M + r] = inv;
      }
      __syncthreads();
    }
    // y_k = P^-1 b_k ; stage the row panel B_{k, k+1..k+wa} (M x wa M) in Lp
    for (int m = tid; m < M; m += nt) {
      double v = 0.0;
      for (int q = 0; q < M; ++q) v += sP[m * M + q] * sb[q];
      sy[m] = v;
      A.Yst[long(k) * M + m] = v;
    }
    const int waM = wa * M;
    for (int t = tid; t < M * waM; t += nt) {
      const int q = t / waM, J = t % waM;
      const int jj = J / M, c = J % M;
      Lp[q * waM + J] = WIN(k, k + 1 + jj)[q * M + c];
    }
    __syncthreads();
    // Z = P^-1 (row panel), kept in LDS and stored for back substitution
    for (int t = tid; t < M * waM; t += nt) {
      const int q = t / waM, J = t % waM;
      double v = 0.0;
      for (int u = 0; u < M; ++u) v += sP[q * M + u] * Lp[u * waM + J];
      Zp[q * waM + J] = v;
      A.Zst[(long(k) * M + q) * wM + J] = v;
    }
    __syncthreads();
    // column panel B_{k+1..k+wa, k} -> Lp ((wa M) x M)
    for (int t = tid; t < waM * M; t += nt) {
      const int I = t / M, q = t % M;
      const int ii = I / M, r = I % M;
      Lp[t] = WIN(k + 1 + ii, k)[r * M + q];
    }
    __syncthreads();
    // trailing update of the window and the right-hand sides
    const int nti = (waM + kTI - 1) / kTI, ntj = (waM + kTJ - 1) / kTJ;
    for (int T = tid; T < nti * ntj; T += nt) {
      const int I0 = (T / ntj) * kTI, J0 = (T % ntj) * kTJ;
      double acc[kTI][kTJ];
      for (int a = 0; a < kTI; ++a)
        for (int b = 0; b < kTJ; ++b) acc[a][b] = 0.0;
      for (int q = 0; q < M; ++q) {
        double av[kTI], bv[kTJ];
        for (int a = 0; a < kTI; ++a) av[a] = (I0 + a < waM) ? Lp[(I0 + a) * M + q] : 0.0;
        for (int b = 0; b < kTJ; ++b) bv[b] = (J0 + b < waM) ? Zp[q * waM + J0 + b] : 0.0;
        for (int a = 0; a < kTI; ++a)
          for (int b = 0; b < kTJ; ++b) acc[a][b] += av[a] * bv[b];
      }
      for (int a = 0; a < kTI; ++a) {
        const int I = I0 + a;
        if (I >= waM) break;
        const int bi = k + 1 + I / M, r = I % M;
        for (int b = 0; b < kTJ; ++b) {
          const int J = J0 + b;
          if (J >= waM) break;
          double* blk = WIN(bi, k + 1 + J / M);
          blk[r * M + (J % M)] -= acc[a][b];
        }
      }
    }
    for (int I = tid; I < waM; I += nt) {
      double v = 0.0;
      for (int q = 0; q < M; ++q) v += Lp[I * M + q] * sy[q];
      RHS(k + 1 + I / M)[I % M] -= v;
    }
    __syncthreads();
  }

  // ---- back substitution: x_k = y_k - sum_j Z_kj x_j
  const int parts = max(1, nt / M);
  double* sx = lds;                 // ring of (w+1) x M solved rows
  double* spart = lds + W1 * M;     // parts x M partial sums
  for (int k = n - 1; k >= 0; --k) {
    const int wa = min(w, n - 1 - k);
    const int waM = wa * M;
    if (tid < parts * M) {
      const int m = tid % M, part = tid / M;
      const int per = (waM + parts - 1) / parts;
      const int jb = part * per, je = min(waM, jb + per);
      double v = 0.0;
      const double* zrow = A.Zst + (long(k) * M + m) * wM;
      for (int J = jb; J < je; ++J) v += zrow[J] * sx[((k + 1 + J / M) % W1) * M + (J % M)];
      spart[part * M + m] = v;
    }
    __syncthreads();
    for (int m = tid; m < M; m += nt) {
      double v = A.Yst[long(k) * M + m];
      for (int part = 0; part < parts; ++part) v -= spart[part * M + m];
      sx[(k % W1) * M + m] = v;
      A.X[long(k) * M + m] = v;
    }
    __syncthreads();
  }
  if (tid == 0) A.info[0] = s_info;
}

size_t lu_lds_allowed = 0;
// ---------------------------------------------------------------------------
// Matrix-core variant of the same block LU (same math, same window ring):
// 512 threads, the pivot inverse by a double-buffered Gauss-Jordan (one
// barrier per pivot), and both block products -- Z = P^-1 (row panel) and
// the trailing update B_ij -= B_ik Z_kj -- on v_mfma_f64_16x16x4f64.
// LDS holds the operands in fragment-friendly layouts (contiguous along the
// 16-wide output index): LpT[q][I] = -B_{k+1+I/M, k}[I%M][q] and
// Zp[q][J] = Z_{k, k+1+J/M}[q][J%M], inner index q padded to a multiple of 4
// with zero rows.  MFMA f64 16x16x4 lane layout: A[l%16][l/16], B[l/16][l%16],
// D[l/16 + 4i][l%16] (i = 0..3).
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kThreadsMfma = 512;

__device__ inline v4d mfma16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ void block_lu_mfma_body(const SolveArgs& A) {
  extern __shared__ double lds[];
  const int M = A.M, MM = M * M, w = 2 * A.s + 1, W1 = w + 1, n = A.n, wM = w * M;
  const int M4 = (M + 3) & ~3;
  const int P16 = ((wM + 15) / 16) * 16;
  double* LpT = lds;              // M4 x P16
  double* Zp = LpT + M4 * P16;    // M4 x P16
  double* sPa = Zp + M4 * P16;    // M x M
  double* sPb = sPa + MM;         // M x M
  double* sb = sPb + MM;          // M
  double* sy = sb + M;            // M
  __shared__ int s_info;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
  if (tid == 0) s_info = 0;
  auto WIN = [&](int i, int j) { return A.win + (long(i % W1) * W1 + (j % W1)) * MM; };
  auto RHS = [&](int i) { return A.rhs + long(i % W1) * M; };
  // zero the K-padding rows once; they are never written afterwards
  for (int t = tid; t < (M4 - M) * P16; t += nt) {
    LpT[M * P16 + t] = 0.0;
    Zp[M * P16 + t] = 0.0;
  }
  const int init_hi = min(w, n - 1);
  for (int i = 0; i <= init_hi; ++i) {
    for (int j = 0; j <= init_hi; ++j) build_block(A, i, j, WIN(i, j));
    build_rhs(A, i, RHS(i));
  }
  __syncthreads();

  for (int k = 0; k < n; ++k) {
    const int wa = min(w, n - 1 - k);
    const int waM = wa * M;
    if (k > 0) {
      const int t = k + w;
      if (t < n) {
        for (int j = k; j <= t; ++j) build_block(A, t, j, WIN(t, j));
        for (int i = k; i < t; ++i) build_block(A, i, t, WIN(i, t));
        build_rhs(A, t, RHS(t));
      }
      __syncthreads();
    }
    // pivot block, right-hand side and the row panel B_{k, k+1..k+wa} (staged in LpT as [t][J])
    {
      const double* P = WIN(k, k);
      for (int t = tid; t < MM; t += nt) sPa[t] = P[t];
      const double* b = RHS(k);
      for (int m = tid; m < M; m += nt) sb[m] = b[m];
      for (int t = tid; t < M * waM; t += nt) {
        const int q = t / waM, J = t % waM;
        LpT[q * P16 + J] = WIN(k, k + 1 + J / M)[q * M + (J % M)];
      }
    }
    __syncthreads();
    // Gauss-Jordan inverse, double buffered: every entry of the next buffer
    // depends on the current one only, so one barrier per pivot
    double* cur = sPa;
    double* nxt = sPb;
    for (int r = 0; r < M; ++r) {
      const double p = cur[r * M + r];
      if (tid == 0 && s_info == 0 && (!(fabs(p) > 0.0) || !isfinite(p))) s_info = k + 1;
      const double ip = 1.0 / p;
      for (int t = tid; t < MM; t += nt) {
        const int i = t / M, j = t % M;
        double v;
        if (i == r) v = (j == r) ? ip : cur[r * M + j] * ip;
        else if (j == r) v = -cur[i * M + r] * ip;
        else v = cur[t] - cur[i * M + r] * (cur[r * M + j] * ip);
        nxt[t] = v;
      }
      __syncthreads();
      double* tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
    // y_k = P^-1 b_k
    for (int m = tid; m < M; m += nt) {
      double v = 0.0;
      for (int q = 0; q < M; ++q) v += cur[m * M + q] * sb[q];
      sy[m] = v;
      A.Yst[long(k) * M + m] = v;
    }
    // Z = P^-1 (row panel) on the matrix cores: tiles of 16 (rows q) x 16 (cols J)
    {
      const int tr = (M + 15) / 16, tc = (waM + 15) / 16;
      for (int T = wave; T < tr * tc; T += nwaves) {
        const int q0 = (T / tc) * 16, J0 = (T % tc) * 16;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        const int ar = q0 + (lane & 15);
        const int bc = J0 + (lane & 15);
        for (int kk = 0; kk < M4; kk += 4) {
          const int kx = kk + (lane >> 4);
          const double a = (ar < M && kx < M) ? cur[ar * M + kx] : 0.0;
          const double b = (kx < M && bc < waM) ? LpT[kx * P16 + bc] : 0.0;
          acc = mfma16x16x4(a, b, acc);
        }
        for (int i = 0; i < 4; ++i) {
          const int q = q0 + (lane >> 4) + 4 * i;
          if (q < M && bc < waM) {
            Zp[q * P16 + bc] = acc[i];
            A.Zst[(long(k) * M + q) * wM + bc] = acc[i];
          }
        }
      }
    }
    __syncthreads();
    // -(column panel)^T -> LpT[q][I]
    for (int t = tid; t < waM * M; t += nt) {
      const int I = t / M, q = t % M;
      LpT[q * P16 + I] = -WIN(k + 1 + I / M, k)[(I % M) * M + q];
    }
    __syncthreads();
    // trailing update B_ij += (-L) Z on the matrix cores, accumulating into the window
    {
      const int tt = (waM + 15) / 16;
      for (int T = wave; T < tt * tt; T += nwaves) {
        const int I0 = (T / tt) * 16, J0 = (T % tt) * 16;
        const int col = J0 + (lane & 15);
        double* cp[4];
        v4d acc;
        for (int i = 0; i < 4; ++i) {
          const int row = I0 + (lane >> 4) + 4 * i;
          cp[i] = (row < waM && col < waM)
                      ? WIN(k + 1 + row / M, k + 1 + col / M) + (row % M) * M + (col % M)
                      : nullptr;
          acc[i] = cp[i] ? *cp[i] : 0.0;
        }
        const int ar = I0 + (lane & 15);
        for (int kk = 0; kk < M4; kk += 4) {
          const int kx = kk + (lane >> 4);
          acc = mfma16x16x4(LpT[kx * P16 + ar], Zp[kx * P16 + col], acc);
        }
        for (int i = 0; i < 4; ++i)
          if (cp[i]) *cp[i] = acc[i];
      }
    }
    for (int I = tid; I < waM; I += nt) {
      double v = 0.0;
      for (int q = 0; q < M; ++q) v += LpT[q * P16 + I] * sy[q];
      RHS(k + 1 + I / M)[I % M] += v;
    }
    __syncthreads();
  }

  // back substitution: x_k = y_k - sum_j Z_kj x_j
  const int parts = max(1, nt / M);
  double* sx = lds;
  double* spart = lds + W1 * M;
  for (int k = n - 1; k >= 0; --k) {
    const int wa = min(w, n - 1 - k);
    const int waM = wa * M;
    if (tid < parts * M) {
      const int m = tid % M, part = tid / M;
      const int per = (waM + parts - 1) / parts;
      const int jb = part * per, je = min(waM, jb + per);
      double v = 0.0;
      const double* zrow = A.Zst + (long(k) * M + m) * wM;
      for (int J = jb; J < je; ++J) v += zrow[J] * sx[((k + 1 + J / M) % W1) * M + (J % M)];
      spart[part * M + m] = v;
    }
    __syncthreads();
    for (int m = tid; m < M; m += nt) {
      double v = A.Yst[long(k) * M + m];
      for (int part = 0; part < parts; ++part) v -= spart[part * M + m];
      sx[(k % W1) * M + m] = v;
      A.X[long(k) * M + m] = v;
    }
    __syncthreads();
  }
  if (tid == 0) A.info[0] = s_info;
}

__global__ __launch_bounds__(kThreadsMfma) void k_block_lu_mfma(SolveArgs A) { block_lu_mfma_body(A); }

// Batched: one workgroup per (active) system; all share M and s, n may differ.
__global__ __launch_bounds__(kThreadsMfma) void k_block_lu_mfma_batched(const SolveArgs* __restrict__ args,
                                                                        const int* __restrict__ active) {
  const SolveArgs A = args[active[blockIdx.x]];
  block_lu_mfma_body(A);
}

size_t lu_mfma_lds_allowed = 0;
size_t lu_mfma_batched_lds_allowed = 0;


constexpr int kResRows = taps::dev::kResRows;


// Per chunk of kResRows rows: R = sum_k A^k U (C^k)^T - Q on the chunk, and the
// chunk's sums of R^2 and Q^2 over free rows -> part[2*block], part[2*block+1].
// V^k = U (C^k)^T is formed on the chunk plus a halo of w rows in LDS.
__global__ void k_residual_part(int n, int M, int s, int K, const double* __restrict__ band,
                                const double* __restrict__ C, const double* __restrict__ U,
                                const double* __restrict__ Q, const uint8_t* __restrict__ fixed,
                                double* __restrict__ part) {
  taps::dev::residual_part(blockIdx.x, n, M, s, K, band, C, U, Q, fixed, part + 2 * blockIdx.x);
}

// Relative backward error of one dim solve from the per-chunk sums:
// sqrt(sum R^2 / sum Q^2) over the free rows.
__global__ void k_berr_final(int nparts, const double* __restrict__ part, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double r = 0.0, q = 0.0;
  for (int b = 0; b < nparts; ++b) {
    r += part[2 * b];
    q += part[2 * b + 1];
  }
  out[0] = q > 0.0 ? sqrt(r / q) : sqrt(r);
}

size_t res_lds_allowed = 0;

}  // namespace

namespace taps {

int dim_residual_nparts(int n) { return cdiv(n, kResRows); }

taps_status dim_residual_parts(taps_handle* h, const taps_problem_t* p, int d, const double* d_C,
                               const double* d_U, const double* d_Q, double* parts, int* nparts,
                               hipStream_t stream) {
  const int nb = cdiv(p->n[d], kResRows);
  const int w = 2 * p->s[d] + 1;
  const int hr = kResRows + 2 * w;
  const size_t lds = size_t(2 * hr * p->M + p->M * p->M + kResRows * p->M) * 8;
  if (lds > 160 * 1024 - 4096) return fail(h, TAPS_ERR_UNSUPPORTED, "residual needs %zu bytes of LDS", lds);
  TAPS_TRY(allow_lds(h, k_residual_part, lds, &res_lds_allowed));
  k_residual_part<<<nb, 256, lds, stream>>>(p->n[d], p->M, p->s[d], p->n_kinds[d], p->d_band[d], d_C, d_U, d_Q,
                                            p->d_fixed[d], parts);
  TAPS_LAUNCHED(h, "k_residual_part");
  *nparts = nb;
  return TAPS_OK;
}

// Algorithmic flops of the block LU solve (what the method needs, not what
// the kernel spends: the pivot is counted as an LU, not an explicit inverse).
double solve_flops(int n, int M, int w) {
  const double m3 = double(M) * M * M, m2 = double(M) * M;
  double f = 0.0;
  for (int k = 0; k < n; ++k) {
    const double wa = double(std::min(w, n - 1 - k));
    f += (2.0 / 3.0) * m3 + 2.0 * wa * m3 + 2.0 * wa * wa * m3 + (2.0 + 4.0 * wa) * m2;
  }
  return f;
}

double solve_bytes(int n, int M, int w, int K) {
  return 8.0 * (double(K) * n * (2 * w + 1) + double(K) * M * M + 2.0 * n * M);
}

size_t solve_mfma_lds_bytes(int M, int s) {
  const int w = 2 * s + 1;
  const size_t M4 = (M + 3) & ~3, P16 = ((w * M + 15) / 16) * 16;
  const size_t fwd = (2 * M4 * P16 + 2 * size_t(M) * M + 2 * size_t(M)) * 8;
  const size_t back = size_t(w + 1 + max(1, kThreadsMfma / M)) * M * 8;
  return fwd > back ? fwd : back;
}

size_t solve_lds_bytes(int M, int s) {
  const int w = 2 * s + 1;
  const size_t fwd = size_t(M) * M * (2 * w + 1) * 8 + 2 * size_t(M) * 8;
  const size_t back = size_t(w + 1 + max(1, kThreads / M)) * M * 8;
  return fwd > back ? fwd : back;
}

taps_status solve_dim_impl(taps_handle* h, const taps_problem_t* p, int d, const double* d_C,
                           const double* d_Q, double* d_X, int* d_info, double* d_berr, hipStream_t stream) {
  const int n = p->n[d], M = p->M, s = p->s[d], w = 2 * s + 1;
  const size_t lds_mfma = solve_mfma_lds_bytes(M, s);
  const bool use_mfma = lds_mfma <= 160 * 1024 - 64 && !getenv("TAPS_SOLVE_VECTOR");
  const size_t lds = use_mfma ? lds_mfma : solve_lds_bytes(M, s);
  if (lds > 160 * 1024 - 64)
    return fail(h, TAPS_ERR_UNSUPPORTED, "M=%d with s=%d needs %zu bytes of LDS (max 163840)", M, s, lds);
  Bump bump;
  const size_t o_Z = bump.take(size_t(n) * M * w * M * 8);
  const size_t o_Y = bump.take(size_t(n) * M * 8);
  const size_t o_W = bump.take(size_t(w + 1) * (w + 1) * M * M * 8);
  const size_t o_R = bump.take(size_t(w + 1) * M * 8);
  const size_t o_P = bump.take(size_t(dim_residual_nparts(n)) * 2 * 8);
  TAPS_TRY(need_ws(h, bump.off, stream));
  char* ws = static_cast<char*>(h->ws);
  SolveArgs A;
  A.n = n;
  A.M = M;
  A.s = s;
  A.K = p->n_kinds[d];
  A.band = p->d_band[d];
  A.C = d_C;
  A.Q = d_Q;
  A.fixed = p->d_fixed[d];
  A.X = d_X;
  A.Zst = reinterpret_cast<double*>(ws + o_Z);
  A.Yst = reinterpret_cast<double*>(ws + o_Y);
  A.win = reinterpret_cast<double*>(ws + o_W);
  A.rhs = reinterpret_cast<double*>(ws + o_R);
  A.info = d_info;
  size_t slot;
  if (use_mfma) {
    TAPS_TRY(allow_lds(h, k_block_lu_mfma, lds, &lu_mfma_lds_allowed));
    TAPS_TRY(prof_begin(h, TAPS_PROF_SOLVE, stream, &slot));
    k_block_lu_mfma<<<1, kThreadsMfma, lds, stream>>>(A);
    TAPS_LAUNCHED(h, "k_block_lu_mfma");
  } else {
    TAPS_TRY(allow_lds(h, k_block_lu, lds, &lu_lds_allowed));
    TAPS_TRY(prof_begin(h, TAPS_PROF_SOLVE, stream, &slot));
    k_block_lu<<<1, kThreads, lds, stream>>>(A);
    TAPS_LAUNCHED(h, "k_block_lu");
  }
  TAPS_TRY(prof_end(h, slot, solve_flops(n, M, w), solve_bytes(n, M, w, A.K), stream));
  if (d_berr) {
    double* parts = reinterpret_cast<double*>(ws + o_P);
    int nb = 0;
    TAPS_TRY(dim_residual_parts(h, p, d, d_C, d_X, d_Q, parts, &nb, stream));
    k_berr_final<<<1, 64, 0, stream>>>(nb, parts, d_berr);
    TAPS_LAUNCHED(h, "k_berr_final");
  }
  return TAPS_OK;
}

// ---- batched solve (used by the batched Algorithm-1 driver)
size_t solve_args_bytes() { return sizeof(SolveArgs); }

size_t solve_ws_bytes(int n, int M, int s) {
  const int w = 2 * s + 1;
  Bump bump;
  bump.take(size_t(n) * M * w * M * 8);
  bump.take(size_t(n) * M * 8);
  bump.take(size_t(w + 1) * (w + 1) * M * M * 8);
  bump.take(size_t(w + 1) * M * 8);
  return bump.off;
}

// Fill the device argument record of one system into host memory `dst`
// (sizeof(SolveArgs) bytes); `ws` is the system's own solve workspace.
void solve_args_fill(void* dst, const taps_problem_t* p, int d, const double* d_C, const double* d_Q,
                     double* d_X, int* d_info, void* ws) {
  const int n = p->n[d], M = p->M, s = p->s[d], w = 2 * s + 1;
  Bump bump;
  const size_t o_Z = bump.take(size_t(n) * M * w * M * 8);
  const size_t o_Y = bump.take(size_t(n) * M * 8);
  const size_t o_W = bump.take(size_t(w + 1) * (w + 1) * M * M * 8);
  const size_t o_R = bump.take(size_t(w + 1) * M * 8);
  char* base = static_cast<char*>(ws);
  SolveArgs A;
  A.n = n;
  A.M = M;
  A.s = s;
  A.K = p->n_kinds[d];
  A.band = p->d_band[d];
  A.C = d_C;
  A.Q = d_Q;
  A.fixed = p->d_fixed[d];
  A.X = d_X;
  A.Zst = reinterpret_cast<double*>(base + o_Z);
  A.Yst = reinterpret_cast<double*>(base + o_Y);
  A.win = reinterpret_cast<double*>(base + o_W);
  A.rhs = reinterpret_cast<double*>(base + o_R);
  A.info = d_info;
  memcpy(dst, &A, sizeof(A));
}

bool solve_batched_supported(int M, int s) { return solve_mfma_lds_bytes(M, s) <= 160 * 1024 - 64; }

taps_status solve_batched_launch(taps_handle* h, int n_active, const void* d_args, const int* d_active,
                                 int M, int s, double flops, double bytes, hipStream_t stream) {
  const size_t lds = solve_mfma_lds_bytes(M, s);
  TAPS_TRY(allow_lds(h, k_block_lu_mfma_batched, lds, &lu_mfma_batched_lds_allowed));
  size_t slot;
  TAPS_TRY(prof_begin(h, TAPS_PROF_SOLVE, stream, &slot));
  k_block_lu_mfma_batched<<<n_active, kThreadsMfma, lds, stream>>>(static_cast<const SolveArgs*>(d_args),
                                                                    d_active);
  TAPS_LAUNCHED(h, "k_block_lu_mfma_batched");
  TAPS_TRY(prof_end(h, slot, flops, bytes, stream));
  return TAPS_OK;
}

taps_status berr_final_launch(taps_handle* h, int nparts, const double* parts, double* out, hipStream_t stream) {
  k_berr_final<<<1, 64, 0, stream>>>(nparts, parts, out);
  TAPS_LAUNCHED(h, "k_berr_final");
  return TAPS_OK;
}

}  // namespace taps

using namespace taps;

extern "C" taps_status taps_solve_dim(taps_handle_t h, const taps_problem_t* prob, int32_t d,
                                      const double* d_C, const double* d_Q, double* d_X,
                                      int32_t* d_info, double* d_berr, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  TAPS_TRY(check_problem(h, prob));
  if (d < 0 || d >= prob->D) return fail(h, TAPS_ERR_INVALID, "dim %d out of range", d);
  if (!d_C || !d_Q || !d_X || !d_info) return fail(h, TAPS_ERR_INVALID, "null pointer");
  return solve_dim_impl(h, prob, d, d_C, d_Q, d_X, d_info, d_berr, stream);
}
