// Device bodies of the contraction, residual and balancing kernels, written
// once and launched both per problem (single-problem calls) and over a batch
// of problems (one block index per problem).  Each body takes its block
// coordinates explicitly.
#pragma once

#include "taps_internal.hpp"

namespace taps {
namespace dev {

constexpr int kGramRows = 64;   // rows of U per Gram partial block
constexpr int kLgCols = 64;     // load columns per load-Gram block
constexpr int kLgRows = 256;    // rows per load-Gram split
constexpr int kLgStage = 32;    // rows staged in LDS at a time
constexpr int kQRows = 64;      // rows of Q per force block
constexpr int kQStage = 32;     // load columns staged in LDS at a time
constexpr int kResRows = 64;    // rows per residual partial block

inline int gram_lds_doubles(int M, int s) { return (2 * kGramRows + 2 * (2 * s + 1)) * M; }
inline int residual_lds_doubles(int M, int s) {
  const int hr = kResRows + 2 * (2 * s + 1);
  return 2 * hr * M + M * M + kResRows * M;
}

// Partial of G^k = U^T A^k U over rows [chunk*kGramRows, +kGramRows): the
// chunk of U plus a halo of w rows goes to LDS, V = A^k U on the chunk rows,
// then U_chunk^T V.  part: K x M x M for this chunk.
__device__ inline void gram_partial(int chunk, int n, int M, int s, int K, const double* __restrict__ band,
                                    const double* __restrict__ U, double* __restrict__ part) {
  extern __shared__ double lds[];
  const int w = 2 * s + 1, BW = 2 * w + 1;
  const int r0 = chunk * kGramRows;
  const int rows = min(kGramRows, n - r0);
  double* sU = lds;                            // (kGramRows + 2w) x M
  double* sV = lds + (kGramRows + 2 * w) * M;  // kGramRows x M
  const int halo_rows = rows + 2 * w;
  for (int t = threadIdx.x; t < halo_rows * M; t += blockDim.x) {
    const int rr = t / M, m = t % M;
    const int g = r0 - w + rr;
    sU[rr * M + m] = (g >= 0 && g < n) ? U[long(g) * M + m] : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    const double* bk = band + long(k) * n * BW;
    for (int t = threadIdx.x; t < rows * M; t += blockDim.x) {
      const int i = t / M, m = t % M;
      const double* brow = bk + long(r0 + i) * BW;
      double v = 0.0;
      for (int o = 0; o < BW; ++o) v += brow[o] * sU[(i + o) * M + m];
      sV[i * M + m] = v;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < M * M; t += blockDim.x) {
      const int m = t / M, nn = t % M;
      double acc = 0.0;
      for (int i = 0; i < rows; ++i) acc += sU[(i + w) * M + m] * sV[i * M + nn];
      part[long(k) * M * M + t] = acc;
    }
    __syncthreads();
  }
}

// out[t] = sum_b part[b][t] in block order, for t in this block's range.
__device__ inline void sum_parts(int tblock, int nparts, long len, const double* __restrict__ part,
                                 double* __restrict__ out) {
  const long t = tblock * long(blockDim.x) + threadIdx.x;
  if (t >= len) return;
  double acc = 0.0;
  for (int b = 0; b < nparts; ++b) acc += part[long(b) * len + t];
  out[t] = acc;
}

// Partial of L = F^T U for load columns [ctile*kLgCols, +kLgCols) over rows of
// split `split`.  part layout: [split][Rc][M].
__device__ inline void lgram_partial(int ctile, int split, int n, int Rc, int M, const double* __restrict__ F,
                                     const double* __restrict__ U, double* __restrict__ part) {
  __shared__ double sF[kLgStage][kLgCols + 1];
  __shared__ double sU[kLgStage * TAPS_MAX_M];
  const int c0 = ctile * kLgCols;
  const int rbeg = split * kLgRows, rend = min(n, rbeg + kLgRows);
  const int nout = kLgCols * M;
  constexpr int kPer = (kLgCols * TAPS_MAX_M + 255) / 256;
  double acc[kPer];
  for (int q = 0; q < kPer; ++q) acc[q] = 0.0;
  for (int i0 = rbeg; i0 < rend; i0 += kLgStage) {
    const int rows = min(kLgStage, rend - i0);
    for (int t = threadIdx.x; t < kLgStage * kLgCols; t += blockDim.x) {
      const int r = t / kLgCols, c = t % kLgCols;
      sF[r][c] = (r < rows && c0 + c < Rc) ? F[long(i0 + r) * Rc + c0 + c] : 0.0;
    }
    for (int t = threadIdx.x; t < kLgStage * M; t += blockDim.x) {
      const int r = t / M;
      sU[t] = (r < rows) ? U[long(i0) * M + t] : 0.0;
    }
    __syncthreads();
    for (int q = 0; q < kPer; ++q) {
      const int o = threadIdx.x + q * blockDim.x;
      if (o < nout) {
        const int c = o / M, m = o % M;
        double a = acc[q];
        for (int r = 0; r < rows; ++r) a += sF[r][c] * sU[r * M + m];
        acc[q] = a;
      }
    }
    __syncthreads();
  }
  for (int q = 0; q < kPer; ++q) {
    const int o = threadIdx.x + q * blockDim.x;
    if (o < nout) {
      const int c = o / M, m = o % M;
      if (c0 + c < Rc) part[(long(split) * Rc + c0 + c) * M + m] = acc[q];
    }
  }
}

struct CoupleArgs {
  int D, M, T, d, Kd;
  int tk[TAPS_MAX_TERMS][TAPS_MAX_DIMS];
  double gamma[TAPS_MAX_TERMS];
  const double* gram[TAPS_MAX_DIMS];  // dim e's Grams (n_kinds[e] x M x M)
};

// C^k_d[m][n] = sum over terms whose dim-d matrix is k of
// gamma * prod_{e != d} G_e^{kind(term, e)}[m][n]  (Hadamard product).
__device__ inline void couple(int tblock, const CoupleArgs& A, double* __restrict__ C) {
  const int t = tblock * blockDim.x + threadIdx.x;
  const int MM = A.M * A.M;
  if (t >= A.Kd * MM) return;
  const int k = t / MM, mn = t % MM;
  double acc = 0.0;
  for (int tau = 0; tau < A.T; ++tau) {
    if (A.tk[tau][A.d] != k) continue;
    double prod = A.gamma[tau];
    for (int e = 0; e < A.D; ++e) {
      if (e == A.d) continue;
      prod *= A.gram[e][long(A.tk[tau][e]) * MM + mn];
    }
    acc += prod;
  }
  C[t] = acc;
}

struct WeightArgs {
  int D, M, R, d, Rc;
  const double* lgram[TAPS_MAX_DIMS];  // Rc_e x M
  const int* col[TAPS_MAX_DIMS];       // R entries or null (identity)
  const int* ptr;                      // dim d grouping (null = identity)
  const int* idx;
};

// Wt[c][m] = sum over load terms r with col_d(r) = c of prod_{e != d} L_e[col_e(r)][m].
__device__ inline void load_weights(int tblock, const WeightArgs& A, double* __restrict__ Wt) {
  const long t = tblock * long(blockDim.x) + threadIdx.x;
  if (t >= long(A.Rc) * A.M) return;
  const int c = int(t / A.M), m = int(t % A.M);
  const int rb = A.ptr ? A.ptr[c] : c;
  const int re = A.ptr ? A.ptr[c + 1] : c + 1;
  double acc = 0.0;
  for (int q = rb; q < re; ++q) {
    const int r = A.ptr ? A.idx[q] : q;
    double prod = 1.0;
    for (int e = 0; e < A.D; ++e) {
      if (e == A.d) continue;
      const int ce = A.col[e] ? A.col[e][r] : r;
      prod *= A.lgram[e][long(ce) * A.M + m];
    }
    acc += prod;
  }
  Wt[t] = acc;
}

// Q = F_d Wt for rows [rblock*kQRows, +kQRows), load columns staged in LDS.
__device__ inline void force(int rblock, int n, int Rc, int M, const double* __restrict__ F,
                             const double* __restrict__ Wt, double* __restrict__ Q) {
  __shared__ double sF[kQRows][kQStage + 1];
  __shared__ double sW[kQStage * TAPS_MAX_M];
  const int r0 = rblock * kQRows;
  const int rows = min(kQRows, n - r0);
  const int nout = kQRows * M;
  constexpr int kPer = (kQRows * TAPS_MAX_M + 255) / 256;
  double acc[kPer];
  for (int q = 0; q < kPer; ++q) acc[q] = 0.0;
  for (int c0 = 0; c0 < Rc; c0 += kQStage) {
    const int cols = min(kQStage, Rc - c0);
    for (int t = threadIdx.x; t < kQRows * kQStage; t += blockDim.x) {
      const int r = t / kQStage, c = t % kQStage;
      sF[r][c] = (r < rows && c < cols) ? F[long(r0 + r) * Rc + c0 + c] : 0.0;
    }
    for (int t = threadIdx.x; t < kQStage * M; t += blockDim.x) {
      const int c = t / M;
      sW[t] = (c < cols) ? Wt[long(c0) * M + t] : 0.0;
    }
    __syncthreads();
    for (int q = 0; q < kPer; ++q) {
      const int o = threadIdx.x + q * blockDim.x;
      if (o < nout) {
        const int r = o / M, m = o % M;
        double a = acc[q];
        for (int c = 0; c < cols; ++c) a += sF[r][c] * sW[c * M + m];
        acc[q] = a;
      }
    }
    __syncthreads();
  }
  for (int q = 0; q < kPer; ++q) {
    const int o = threadIdx.x + q * blockDim.x;
    if (o < nout) {
      const int r = o / M, m = o % M;
      if (r < rows) Q[long(r0 + r) * M + m] = acc[q];
    }
  }
}

// Per chunk of kResRows rows: R = sum_k A^k U (C^k)^T - Q and the chunk's
// sums of R^2 and Q^2 over free rows -> part[0], part[1].  V^k = U (C^k)^T is
// formed on the chunk plus a halo of w rows in LDS.
__device__ inline void residual_part(int chunk, int n, int M, int s, int K, const double* __restrict__ band,
                                     const double* __restrict__ C, const double* __restrict__ U,
                                     const double* __restrict__ Q, const uint8_t* __restrict__ fixed,
                                     double* __restrict__ part) {
  extern __shared__ double lds[];
  const int w = 2 * s + 1, BW = 2 * w + 1, MM = M * M;
  const int r0 = chunk * kResRows;
  const int rows = min(kResRows, n - r0);
  const int hr = rows + 2 * w;
  double* sU = lds;          // hr x M
  double* sV = sU + hr * M;  // hr x M
  double* sC = sV + hr * M;  // M x M
  double* sR = sC + MM;      // rows x M
  __shared__ double red[2][256];
  for (int t = threadIdx.x; t < hr * M; t += blockDim.x) {
    const int rr = t / M, m = t % M;
    const int g = r0 - w + rr;
    sU[t] = (g >= 0 && g < n) ? U[long(g) * M + m] : 0.0;
  }
  for (int t = threadIdx.x; t < rows * M; t += blockDim.x) sR[t] = -Q[long(r0) * M + t];
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    for (int t = threadIdx.x; t < MM; t += blockDim.x) sC[t] = C[long(k) * MM + t];
    __syncthreads();
    for (int t = threadIdx.x; t < hr * M; t += blockDim.x) {
      const int rr = t / M, m = t % M;
      double v = 0.0;
      for (int q = 0; q < M; ++q) v += sU[rr * M + q] * sC[m * M + q];
      sV[t] = v;
    }
    __syncthreads();
    const double* bk = band + long(k) * n * BW;
    for (int t = threadIdx.x; t < rows * M; t += blockDim.x) {
      const int i = t / M, m = t % M;
      const double* brow = bk + long(r0 + i) * BW;
      double v = 0.0;
      for (int o = 0; o < BW; ++o) v += brow[o] * sV[(i + o) * M + m];
      sR[t] += v;
    }
    __syncthreads();
  }
  double rr2 = 0.0, qq2 = 0.0;
  for (int t = threadIdx.x; t < rows * M; t += blockDim.x) {
    const int i = t / M;
    if (fixed && fixed[r0 + i]) continue;
    const double q = Q[long(r0) * M + t];
    rr2 += sR[t] * sR[t];
    qq2 += q * q;
  }
  red[0][threadIdx.x] = rr2;
  red[1][threadIdx.x] = qq2;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      red[0][threadIdx.x] += red[0][threadIdx.x + st];
      red[1][threadIdx.x] += red[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[0] = red[0][0];
    part[1] = red[1][0];
  }
}

struct BalanceArgs {
  int D, M;
  int n[TAPS_MAX_DIMS];
  double* U[TAPS_MAX_DIMS];
};

// Mode m: column norms of every dim, geometric mean, rescale (skipped when a
// norm is below 1e-300).  Block of 256 threads.
__device__ inline void balance(int m, const BalanceArgs& A) {
  __shared__ double red[256];
  __shared__ double nrm[TAPS_MAX_DIMS];
  for (int e = 0; e < A.D; ++e) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < A.n[e]; i += blockDim.x) {
      const double v = A.U[e][long(i) * A.M + m];
      acc += v * v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) nrm[e] = sqrt(red[0]);
    __syncthreads();
  }
  bool tiny = false;
  double lg = 0.0;
  for (int e = 0; e < A.D; ++e) {
    tiny = tiny || !(nrm[e] >= 1e-300);
    lg += log(nrm[e]);
  }
  if (tiny) return;
  const double g = exp(lg / A.D);
  for (int e = 0; e < A.D; ++e) {
    const double f = g / nrm[e];
    for (int i = threadIdx.x; i < A.n[e]; i += blockDim.x) A.U[e][long(i) * A.M + m] *= f;
  }
}

}  // namespace dev
}  // namespace taps
