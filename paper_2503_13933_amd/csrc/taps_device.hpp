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
constexpr int kQRows = 64;      // rows of Q per force block
constexpr int kResRows = 64;    // rows per residual partial block

inline int gram_lds_doubles(int M, int s) {
  return (2 * kGramRows + 2 * (2 * s + 1)) * (M | 1) + kGramRows * (2 * (2 * s + 1) + 1);
}

// v_mfma_f64_16x16x4f64 operands of lane l: A[l%16][l/16], B[l/16][l%16];
// result D[l/16 + 4j][l%16], j = 0..3.
typedef double rv4d __attribute__((ext_vector_type(4)));
// two doubles at an 8-byte-aligned address (one 16-byte load)
typedef double f64x2u __attribute__((ext_vector_type(2), aligned(8)));
__device__ inline rv4d mfma_f64(double a, double b, rv4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Rows g0 .. g0+nrows-1 of a row-major matrix with M columns into LDS rows
// 0 .. nrows-1 (row stride L), zero outside rows [0, n): rows over the 4
// waves of the block, columns over the lanes, eight rows per wave loaded
// before any is stored so their memory latencies overlap.
template <class P>
__device__ inline void stage_rows(double* dst, int L, P src, int M, int g0, int n, int nrows) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c = lane; c < M; c += 64) {
    for (int r = wv; r < nrows; r += 32) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int rr = r + 4 * u, g = g0 + rr;
        v[u] = (rr < nrows && g >= 0 && g < n) ? src[long(g) * M + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (r + 4 * u < nrows) dst[(r + 4 * u) * L + c] = v[u];
    }
  }
}

inline int residual_lds_doubles(int M, int s) { return (kResRows + 2 * (2 * s + 1) + M) * (M | 1); }

// V = A^k U on 16 chunk rows i0.. (i0 wave-uniform), one column per lane:
// the column's 15 + BW halo values sit in registers and each output takes
// BW of them (a sliding window); the band coefficients (sB, the chunk's band
// rows) are the same for every lane.  Rows past the chunk's end give zero.
template <int BW>
__device__ inline void band_rows16(const double* sB, int i0, int rows, const double* sU, double* sV, int L, int M,
                                   int lane) {
  constexpr int R = 16;
  for (int c = lane; c < M; c += 64) {
    double u[R + BW - 1];
#pragma unroll
    for (int t = 0; t < R + BW - 1; ++t) u[t] = sU[(i0 + t) * L + c];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double v = 0.0;
      if (i0 + i < rows) {
#pragma unroll
        for (int o = 0; o < BW; ++o) v = fma(sB[(i0 + i) * BW + o], u[i + o], v);
      }
      sV[(i0 + i) * L + c] = v;
    }
  }
}

// Partial of G^k = U^T A^k U over rows [chunk*kGramRows, +kGramRows): the
// chunk of U plus a halo of w rows goes to LDS (rows over the waves, columns
// over the lanes) and the chunk's band rows of kind k after it, V = A^k U on
// the chunk rows (16 rows per wave, see band_rows16), then U_chunk^T V on the
// matrix cores, the rows of the chunk
// being the contracted index (16 steps of 4, operands of four steps loaded
// together); the 16 x 16 tiles of the M x M result are dealt to the 4 waves.
// Operand rows and columns past M read neighbouring LDS entries and only
// reach result entries past M, which are not stored.
// part: K x M x M for this chunk.
template <int BW>
__device__ inline void gram_partial_bw(int chunk, int n, int M, int K, const double* __restrict__ band_,
                                       const double* __restrict__ U_, double* __restrict__ part_) {
  const auto band = gp(band_);
  const auto U = gp(U_);
  const auto part = gp(part_);
  extern __shared__ double lds[];
  constexpr int w = (BW - 1) / 2;
  const int L = M | 1, MM = M * M;
  const int r0 = chunk * kGramRows;
  const int rows = min(kGramRows, n - r0);
  const int halo_rows = kGramRows + 2 * w;
  double* sU = lds;                  // halo_rows x L
  double* sV = sU + halo_rows * L;   // kGramRows x L
  double* sB = sV + kGramRows * L;   // rows x BW
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  stage_rows(sU, L, U, M, r0 - w, n, halo_rows);
  const int nt = (M + 15) / 16;
  for (int k = 0; k < K; ++k) {
    __syncthreads();   // sB and sV free
    const auto brows = band + (long(k) * n + r0) * BW;
    for (int t = tid; t < rows * BW; t += blockDim.x) sB[t] = brows[t];
    __syncthreads();
    band_rows16<BW>(sB, 16 * wv, rows, sU, sV, L, M, lane);
    __syncthreads();
    for (int tile = wv; tile < nt * nt; tile += 4) {
      const int tr = tile / nt, tc = tile - (tile / nt) * nt;
      const int ma = tr * 16 + (lane & 15), nb = tc * 16 + (lane & 15);
      rv4d acc = {0.0, 0.0, 0.0, 0.0};
      for (int kk0 = 0; kk0 < kGramRows / 4; kk0 += 4) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = 4 * (kk0 + u) + (lane >> 4);
          a[u] = sU[(i + w) * L + ma];
          b[u] = sV[i * L + nb];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = mfma_f64(a[u], b[u], acc);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = tr * 16 + (lane >> 4) + 4 * j;
        if (m < M && nb < M) part[long(k) * MM + m * M + nb] = acc[j];
      }
    }
  }
}

__device__ inline void gram_partial(int chunk, int n, int M, int s, int K, const double* __restrict__ band,
                                    const double* __restrict__ U, double* __restrict__ part) {
  switch (s) {
    case 0: gram_partial_bw<3>(chunk, n, M, K, band, U, part); break;
    case 1: gram_partial_bw<7>(chunk, n, M, K, band, U, part); break;
    case 2: gram_partial_bw<11>(chunk, n, M, K, band, U, part); break;
    default: gram_partial_bw<15>(chunk, n, M, K, band, U, part); break;
  }
}

// out[t] = sum_b part[b][t] in block order, for t in this block's range.
template <int NS>
__device__ inline void sum_parts_n(int s0, int nparts, long len, const double* __restrict__ part_,
                                   double* __restrict__ out_) {
  const auto part = gp(part_);
  const auto out = gp(out_);
  if (s0 * long(blockDim.x) >= len) return;
  long t[NS];
  double acc[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    t[u] = (s0 + u) * long(blockDim.x) + threadIdx.x;
    acc[u] = 0.0;
  }
  for (int b = 0; b < nparts; ++b) {
#pragma unroll
    for (int u = 0; u < NS; ++u) acc[u] += part[long(b) * len + min(t[u], len - 1)];
  }
#pragma unroll
  for (int u = 0; u < NS; ++u)
    if (t[u] < len) out[t[u]] = acc[u];
}
__device__ inline void sum_parts(int tblock, int nparts, long len, const double* __restrict__ part,
                                 double* __restrict__ out) {
  sum_parts_n<1>(tblock, nparts, len, part, out);
}

// Partial of L = F^T U for load columns [ctile*kLgCols, +kLgCols) over rows
// [split*rows, +rows) (rows a multiple of 16), on the matrix cores: wave v owns load columns
// [16v, 16v+16) of the tile, the rows are the contracted index, and the
// M columns of U are covered in passes of up to NCT 16-wide tiles (as in
// the force).  Operands
// are read from global memory (16 consecutive doubles per row and step).
// part layout: [split][Rc][M].
template <int NCT = 4>
__device__ inline void lgram_partial(int ctile, int split, int rows, int n, int Rc, int M,
                                     const double* __restrict__ F_, const double* __restrict__ U_,
                                     double* __restrict__ part_) {
  const auto F = gp(F_);
  const auto U = gp(U_);
  const auto part = gp(part_);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int cw = ctile * kLgCols + wv * 16;
  if (cw >= Rc) return;
  const int rbeg = split * rows, rend = min(n, rbeg + rows);
  const int ca = cw + (lane & 15);
  const int nct = (M + 15) / 16;
  for (int ct0 = 0; ct0 < nct; ct0 += NCT) {
    rv4d acc[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[c] = rv4d{0.0, 0.0, 0.0, 0.0};
    // 16 rows per pass, all operands of a pass loaded together and the next
    // pass's requested before this pass's products
    auto load = [&](int i0, double (&a)[4], double (&b)[4][NCT]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 4 * u + (lane >> 4);
        const bool ok = i < rend;
        a[u] = (ok && ca < Rc) ? F[long(i) * Rc + ca] : 0.0;
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
          const int m = (ct0 + c) * 16 + (lane & 15);
          b[u][c] = (ok && ct0 + c < nct && m < M) ? U[long(i) * M + m] : 0.0;
        }
      }
    };
    double an[4], bn[4][NCT];
    if (rbeg < rend) load(rbeg, an, bn);
    for (int i0 = rbeg; i0 < rend; i0 += 16) {
      double a[4], b[4][NCT];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = an[u];
#pragma unroll
        for (int c = 0; c < NCT; ++c) b[u][c] = bn[u][c];
      }
      if (i0 + 16 < rend) load(i0 + 16, an, bn);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int c = 0; c < NCT; ++c)
          if (ct0 + c < nct) acc[c] = mfma_f64(a[u], b[u][c], acc[c]);   // guard, not exit: stays unrolled
      }
    }
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int m = (ct0 + c) * 16 + (lane & 15);
      if (ct0 + c >= nct || m >= M) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int cc = cw + (lane >> 4) + 4 * j;
        if (cc < Rc) part[(long(split) * Rc + cc) * M + m] = acc[c][j];
      }
    }
  }
}

struct CoupleArgs {
  int D, M, T, d, Kd;   // d and Kd: the dim and its kind count (single-problem launches)
  int tk[TAPS_MAX_TERMS][TAPS_MAX_DIMS];
  double gamma[TAPS_MAX_TERMS];
  const double* gram[TAPS_MAX_DIMS];  // dim e's Grams (n_kinds[e] x M x M)
};

// C^k_d[m][n] = sum over terms whose dim-d matrix is k of
// gamma * prod_{e != d} G_e^{kind(term, e)}[m][n]  (Hadamard product).
// NS consecutive slices of blockDim.x entries from slice s0 on, stored after
// all their loads (one store per slice would otherwise order the next
// slice's loads behind it).
template <int NS>
__device__ inline void couple_n(int s0, const CoupleArgs& A, int d, int Kd, double* __restrict__ C) {
  const int MM = A.M * A.M, len = Kd * MM;
  if (s0 * int(blockDim.x) >= len) return;
  int t[NS], k[NS], mn[NS];
  double acc[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    t[u] = (s0 + u) * blockDim.x + threadIdx.x;
    const int tc = min(t[u], len - 1);
    k[u] = tc / MM;
    mn[u] = tc - k[u] * MM;
    acc[u] = 0.0;
  }
  for (int tau = 0; tau < A.T; ++tau) {
    const int kt = A.tk[tau][d];
    double prod[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) prod[u] = A.gamma[tau];
    for (int e = 0; e < A.D; ++e) {
      if (e == d) continue;
      const auto g = gp(A.gram[e]) + long(A.tk[tau][e]) * MM;
#pragma unroll
      for (int u = 0; u < NS; ++u) prod[u] *= g[mn[u]];
    }
#pragma unroll
    for (int u = 0; u < NS; ++u)
      if (k[u] == kt) acc[u] += prod[u];
  }
#pragma unroll
  for (int u = 0; u < NS; ++u)
    if (t[u] < len) gp(C)[t[u]] = acc[u];
}
__device__ inline void couple(int tblock, const CoupleArgs& A, double* __restrict__ C) {
  couple_n<1>(tblock, A, A.d, A.Kd, C);
}

struct WeightArgs {
  int D, M, R, d, Rc;
  const double* lgram[TAPS_MAX_DIMS];  // Rc_e x M
  const int* col[TAPS_MAX_DIMS];       // R entries or null (identity)
  const int* ptr;                      // dim d grouping (null = identity)
  const int* idx;
  double* P;                           // R x M per-term products (ptr order)
};

// Per-term products, one thread per (term, mode), terms in the grouping order
// of dim d: P[q][m] = prod_{e != d} L_e[col_e(r)][m], r = idx[q].  Every
// thread's loads depend only on its own term, so the whole table fills in a
// few memory latencies.
// NS consecutive slices of blockDim.x items from slice s0 on, every load of
// a kind issued for all slices before any is used (the index, column-map and
// load-Gram reads form a dependent chain per item), the products stored last.
template <int NS>
__device__ inline void load_terms_n(int s0, const WeightArgs& A) {
  const int M = A.M, RM = A.R * M;   // R M < 2^31
  if (RM <= 0 || s0 * int(blockDim.x) >= RM) return;
  int t[NS], m[NS], r[NS];
  double prod[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    t[u] = (s0 + u) * blockDim.x + threadIdx.x;
    const int tc = min(t[u], RM - 1);
    const int q = tc / M;
    m[u] = tc - q * M;
    r[u] = q;
    prod[u] = 1.0;
  }
  if (A.ptr) {
#pragma unroll
    for (int u = 0; u < NS; ++u) r[u] = gp(A.idx)[r[u]];
  }
  for (int e = 0; e < A.D; ++e) {
    if (e == A.d) continue;
    int ce[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) ce[u] = A.col[e] ? gp(A.col[e])[r[u]] : r[u];
    double lv[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) lv[u] = gp(A.lgram[e])[long(ce[u]) * M + m[u]];
#pragma unroll
    for (int u = 0; u < NS; ++u) prod[u] *= lv[u];
  }
#pragma unroll
  for (int u = 0; u < NS; ++u)
    if (t[u] < RM) gp(A.P)[t[u]] = prod[u];
}
__device__ inline void load_terms(int tblock, const WeightArgs& A) { load_terms_n<1>(tblock, A); }

// Wt[c][m] = sum of P[q][m] over the terms q of group c (ptr[c] .. ptr[c+1]),
// in term order; independent contiguous loads.
__device__ inline void load_weights(int tblock, const WeightArgs& A, double* __restrict__ Wt) {
  const int t = tblock * blockDim.x + threadIdx.x;   // Rc M < 2^31
  const int M = A.M;
  if (t >= A.Rc * M) return;
  const int c = t / M, m = t - c * M;
  const int rb = A.ptr ? gp(A.ptr)[c] : c;
  const int re = A.ptr ? gp(A.ptr)[c + 1] : c + 1;
  const auto P = gp(A.P) + m;
  double acc = 0.0;
  int q = rb;
  for (; q + 4 <= re; q += 4) {
    const double p0 = P[long(q) * M], p1 = P[long(q + 1) * M], p2 = P[long(q + 2) * M], p3 = P[long(q + 3) * M];
    acc = (((acc + p0) + p1) + p2) + p3;
  }
  for (; q < re; ++q) acc += P[long(q) * M];
  gp(Wt)[t] = acc;
}

// Long groups with the per-term products formed in place (no product
// table): block (c, s) takes slice s of wsl equal slices of group c's terms
// and sums prod_{e != d} L_e[col_e(r)][m] over them, as 256/L row lanes x L
// mode lanes (L = M rounded up to 32 or 64); the row lanes are summed in a
// fixed order and the slice's sum goes to out[(c wsl + s) M + m] (the load
// weights themselves when wsl = 1).
__device__ inline void load_weights_fused(int c, int s, int wsl, const WeightArgs& A, double* __restrict__ out) {
  __shared__ double red[256];
  const int M = A.M, L = M <= 32 ? 32 : 64, lanes = 256 / L;
  const int m = threadIdx.x % L, lr = threadIdx.x / L, mc = min(m, M - 1);
  const int rb = A.ptr ? gp(A.ptr)[c] : c;
  const int re = A.ptr ? gp(A.ptr)[c + 1] : c + 1;
  const int len = (re - rb + wsl - 1) / wsl;
  const int q0 = rb + s * len, q1 = min(re, q0 + len);
  // four terms per step, every load of a kind issued for all four before
  // any is used (index -> column map -> load Gram is a dependent chain)
  constexpr int NT = 4;
  double acc[NT] = {0.0, 0.0, 0.0, 0.0};
  for (int q = q0 + lr; q < q1; q += NT * lanes) {
    int r[NT];
    double prod[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int qt = min(q + t * lanes, q1 - 1);
      r[t] = A.ptr ? gp(A.idx)[qt] : qt;
      prod[t] = (q + t * lanes < q1) ? 1.0 : 0.0;
    }
    for (int e = 0; e < A.D; ++e) {
      if (e == A.d) continue;
      int ce[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) ce[t] = A.col[e] ? gp(A.col[e])[r[t]] : r[t];
      double lv[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) lv[t] = gp(A.lgram[e])[long(ce[t]) * M + mc];
#pragma unroll
      for (int t = 0; t < NT; ++t) prod[t] *= lv[t];
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] += prod[t];
  }
  red[threadIdx.x] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (lr == 0 && m < M) {
    double t = 0.0;
    for (int k = 0; k < lanes; ++k) t += red[k * L + m];
    gp(out)[(long(c) * wsl + s) * M + m] = t;
  }
  __syncthreads();
}

// Q = F_d Wt for rows [rblock*kQRows, +kQRows) on the matrix cores: wave v
// owns rows [16v, 16v+16) of the block, the load columns are the contracted
// index (passes of 16 columns in four steps, operands loaded together), and
// the M columns are covered in passes of up to NCT 16-wide tiles (NCT = 4
// covers any M; the batched kernels instantiate the smallest that covers
// their M, which holds fewer operand registers).  In a pass
// from column c0, lane group g = l/16 takes columns c0 + 4g .. c0 + 4g + 3, one
// per step (the Wt rows follow the same assignment), so each lane reads its
// four F entries as two 16-byte loads: 64 contiguous bytes of four rows' lines
// per instruction pair instead of four loads of 8 bytes per row.
// (load columns [c_lo, c_hi) only: the batched driver splits long load
// rows over several work items and sums their partial Q afterwards)
template <int NCT = 4>
__device__ inline void force(int rblock, int n, int Rc, int M, const double* __restrict__ F_,
                             const double* __restrict__ Wt_, double* __restrict__ Q_, int c_lo = 0,
                             int c_hi = 0x7fffffff) {
  const auto F = gp(F_);
  const auto Wt = gp(Wt_);
  const auto Q = gp(Q_);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rw = rblock * kQRows + wv * 16;
  if (rw >= n) return;
  const int ia = rw + (lane & 15);
  const int nct = (M + 15) / 16;
  for (int ct0 = 0; ct0 < nct; ct0 += NCT) {
    rv4d acc[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[c] = rv4d{0.0, 0.0, 0.0, 0.0};
    // 16 load columns per pass, all operands of a pass loaded together and
    // the next pass's requested before this pass's products
    const int c_end = min(Rc, c_hi);
    auto load = [&](int c0, double (&a)[4], double (&b)[4][NCT]) {
      const int kb = c0 + 4 * (lane >> 4);
      if (ia < n && kb + 3 < c_end) {
        const gmem<f64x2u>* p = reinterpret_cast<const gmem<f64x2u>*>(F + long(ia) * Rc + kb);
        const f64x2u lo = p[0], hi = p[1];
        a[0] = lo.x;
        a[1] = lo.y;
        a[2] = hi.x;
        a[3] = hi.y;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = (ia < n && kb + u < c_end) ? F[long(ia) * Rc + kb + u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool ok = kb + u < c_end;
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
          const int m = (ct0 + c) * 16 + (lane & 15);
          b[u][c] = (ok && ct0 + c < nct && m < M) ? Wt[long(kb + u) * M + m] : 0.0;
        }
      }
    };
    // the next pass's operands requested before this pass's products
    auto mma = [&](const double (&a)[4], const double (&b)[4][NCT]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int c = 0; c < NCT; ++c)
          if (ct0 + c < nct) acc[c] = mfma_f64(a[u], b[u][c], acc[c]);   // guard, not exit: stays unrolled
      }
    };
    double an[4], bn[4][NCT];
    load(c_lo, an, bn);
    for (int c0 = c_lo; c0 < c_end; c0 += 16) {
      double a[4], b[4][NCT];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = an[u];
#pragma unroll
        for (int c = 0; c < NCT; ++c) b[u][c] = bn[u][c];
      }
      if (c0 + 16 < c_end) load(c0 + 16, an, bn);
      mma(a, b);
    }
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int m = (ct0 + c) * 16 + (lane & 15);
      if (ct0 + c >= nct || m >= M) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = rw + (lane >> 4) + 4 * j;
        if (i < n) Q[long(i) * M + m] = acc[c][j];
      }
    }
  }
}

// Per chunk of kResRows rows: R = sum_k (A^k U) (C^k)^T - Q and the chunk's
// sums of R^2 and Q^2 over free rows -> part[0], part[1].  256 threads: wave
// v owns rows [16v, 16v+16) of the chunk.  The chunk of U with a halo of w
// rows and C^k sit in LDS (odd row stride L); the banded product W^k = A^k U
// is formed directly as the A operands of v_mfma_f64_16x16x4f64 (lane l:
// row l%16, column 4kk + l/16) and multiplied by (C^k)^T on the matrix cores,
// up to four 16-column tiles of R per pass.
// (BW = 2(2s+1)+1 band entries per row, a template argument so that the
// band coefficients and the A-operand sums are exactly BW long)
template <int BW, int NCT = 4>
__device__ inline void residual_part_bw(int chunk, int n, int M, int K, const double* __restrict__ band_,
                                        const double* __restrict__ C_, const double* __restrict__ U_,
                                        const double* __restrict__ Q_, const uint8_t* __restrict__ fixed_,
                                        double* __restrict__ part_) {
  const auto band = gp(band_);
  const auto C = gp(C_);
  const auto U = gp(U_);
  const auto Q = gp(Q_);
  const auto fixed = gp(fixed_);
  const auto part = gp(part_);
  extern __shared__ double lds[];
  constexpr int w = (BW - 1) / 2;
  const int L = M | 1;
  const int r0 = chunk * kResRows;
  const int rows = min(kResRows, n - r0);
  const int hr = kResRows + 2 * w;
  double* sU = lds;            // hr x L (halo rows r0-w ..)
  double* sC = sU + hr * L;    // M x L
  __shared__ double red[4][2];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  stage_rows(sU, L, U, M, r0 - w, n, hr);
  const int i_a = wv * 16 + (lane & 15);    // chunk row of this lane's A operands
  const int ksteps = (M + 3) / 4, nct = (M + 15) / 16;
  double rr2 = 0.0, qq2 = 0.0;
  for (int ct0 = 0; ct0 < nct; ct0 += NCT) {
    rv4d acc[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[c] = rv4d{0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < K; ++k) {
      __syncthreads();   // sU staged / sC free
      for (int c = lane; c < M; c += 64)   // rows wv, wv+4, ..: four loads in flight, then four stores
        for (int rb = wv; rb < M; rb += 16) {
          double cv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) cv[u] = C[(long(k) * M + min(rb + 4 * u, M - 1)) * M + c];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (rb + 4 * u < M) sC[(rb + 4 * u) * L + c] = cv[u];
        }
      double bc[BW];
      const auto brow = band + (long(k) * n + r0 + min(i_a, rows - 1)) * BW;
#pragma unroll
      for (int o = 0; o < BW; ++o) {
        const double bv = brow[o];
        bc[o] = (i_a < rows) ? bv : 0.0;
      }
      __syncthreads();
      for (int kk = 0; kk < ksteps; ++kk) {
        const int q = 4 * kk + (lane >> 4);
        double a = 0.0;
        if (q < M) {
#pragma unroll
          for (int o = 0; o < BW; ++o) a += bc[o] * sU[(i_a + o) * L + q];
        }
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
          if (ct0 + c < nct) {
            const int m = (ct0 + c) * 16 + (lane & 15);
            const double b = (m < M && q < M) ? sC[m * L + q] : 0.0;
            acc[c] = mfma_f64(a, b, acc[c]);
          }
        }
      }
    }
    // R = acc - Q on this pass's tiles; lane holds rows l/16 + 4j, column l%16
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int m = (ct0 + c) * 16 + (lane & 15);
      if (ct0 + c >= nct || m >= M) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = wv * 16 + (lane >> 4) + 4 * j;
        if (i >= rows || (fixed && fixed[r0 + i])) continue;
        const double qv = Q[long(r0 + i) * M + m];
        const double r = acc[c][j] - qv;
        rr2 += r * r;
        qq2 += qv * qv;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    rr2 += __shfl_xor(rr2, o);
    qq2 += __shfl_xor(qq2, o);
  }
  if (lane == 0) {
    red[wv][0] = rr2;
    red[wv][1] = qq2;
  }
  __syncthreads();
  if (tid == 0) {
    part[0] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
    part[1] = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
  }
}

__device__ inline void residual_part(int chunk, int n, int M, int s, int K, const double* __restrict__ band,
                                     const double* __restrict__ C, const double* __restrict__ U,
                                     const double* __restrict__ Q, const uint8_t* __restrict__ fixed,
                                     double* __restrict__ part) {
  switch (s) {
    case 0: residual_part_bw<3>(chunk, n, M, K, band, C, U, Q, fixed, part); break;
    case 1: residual_part_bw<7>(chunk, n, M, K, band, C, U, Q, fixed, part); break;
    case 2: residual_part_bw<11>(chunk, n, M, K, band, C, U, Q, fixed, part); break;
    default: residual_part_bw<15>(chunk, n, M, K, band, C, U, Q, fixed, part); break;
  }
}

struct BalanceArgs {
  int D, M;
  int n[TAPS_MAX_DIMS];
  double* U[TAPS_MAX_DIMS];
  // cached Grams of each dim (K x M x M) and load Grams (Rc x M), rescaled
  // with the factors for the dims of the scale mask (batched driver)
  int K[TAPS_MAX_DIMS], Rc[TAPS_MAX_DIMS];
  double* gram[TAPS_MAX_DIMS];
  double* lgram[TAPS_MAX_DIMS];
  // factors at the start of the sweep (same layout as U; null: no change
  // measured) and where the relative change of the sweep goes (one double)
  const double* snap[TAPS_MAX_DIMS];
  double* change;
  // where the per-dim mode factors go (D x M; null: the Grams of the scale
  // mask are rescaled inside the balancing block itself)
  double* fac;
};

// Copy of every factor of one problem (the start of a sweep), one block of
// 256 threads walking the contiguous n_d x M arrays.
__device__ inline void snapshot(const BalanceArgs& A) {
  if (!A.change) return;
  for (int e = 0; e < A.D; ++e) {
    const auto src = gp(A.U[e]);
    const auto dst = gp(const_cast<double*>(A.snap[e]));
    const long len = long(A.n[e]) * A.M;
    long i = threadIdx.x;
    for (; i + 3 * 256 < len; i += 4 * 256) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = src[i + u * 256];
#pragma unroll
      for (int u = 0; u < 4; ++u) dst[i + u * 256] = v[u];
    }
    for (; i < len; i += 256) dst[i] = src[i];
  }
}

// Every mode m of one problem: column norms of every dim, their geometric
// mean g, U_e[:, m] *= g / ||U_e[:, m]|| (skipped for a mode with a norm below
// 1e-300).  With a snapshot, the relative change of the sweep,
// sqrt(sum_e ||U_e - snap_e||_F^2 / sum_e ||U_e||_F^2) of the balanced
// factors, is written to *change (the paper's stop rule, Sec. 2.6).  Block of 256 threads as 4 row phases x 64 mode lanes, so each row
// of a factor is read and written as one contiguous segment; the row phases
// are summed in a fixed order.  For the dims in scale_mask the cached Grams
// follow the factors without being recomputed: G^k[m][n] *= f_m f_n and
// L[c][m] *= f_m (f = the factor applied to column m).
__device__ inline void balance(const BalanceArgs& A, unsigned scale_mask = 0) {
  __shared__ double part[4][64];
  __shared__ double fac[TAPS_MAX_DIMS][64];
  const int m = threadIdx.x & 63, ph = threadIdx.x >> 6, M = A.M;
  for (int e = 0; e < A.D; ++e) {
    // rows ph, ph+4, ... of column m, eight rows loaded before they are used
    const auto Ue = gp(A.U[e]);
    const int n = A.n[e];
    double acc = 0.0;
    if (m < M) {
      double a4[4] = {0.0, 0.0, 0.0, 0.0};
      int i = ph;
      for (; i + 28 < n; i += 32) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = Ue[long(i + 4 * u) * M + m];
#pragma unroll
        for (int u = 0; u < 8; ++u) a4[u & 3] += v[u] * v[u];
      }
      for (; i < n; i += 4) {
        const double v = Ue[long(i) * M + m];
        a4[0] += v * v;
      }
      acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    }
    part[ph][m] = acc;
    __syncthreads();
    if (ph == 0) fac[e][m] = sqrt(((part[0][m] + part[1][m]) + part[2][m]) + part[3][m]);
    __syncthreads();
  }
  if (ph == 0 && m < M) {
    bool tiny = false;
    double lg = 0.0;
    for (int e = 0; e < A.D; ++e) {
      tiny = tiny || !(fac[e][m] >= 1e-300);
      lg += log(fac[e][m]);
    }
    const double g = exp(lg / A.D);
    for (int e = 0; e < A.D; ++e) fac[e][m] = tiny ? 1.0 : g / fac[e][m];
  }
  __syncthreads();
  double dsum = 0.0, nsum = 0.0;
  if (m < M)
    for (int e = 0; e < A.D; ++e) {
      const double f = fac[e][m];
      const auto Ue = gp(A.U[e]);
      const int n = A.n[e];
      int i = ph;
      if (A.change) {
        const auto Se = gp(A.snap[e]);
        for (; i + 28 < n; i += 32) {
          double v[8], o[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            v[u] = Ue[long(i + 4 * u) * M + m];
            o[u] = Se[long(i + 4 * u) * M + m];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const double x = v[u] * f, dx = x - o[u];
            Ue[long(i + 4 * u) * M + m] = x;
            dsum += dx * dx;
            nsum += x * x;
          }
        }
        for (; i < n; i += 4) {
          const double x = Ue[long(i) * M + m] * f, dx = x - Se[long(i) * M + m];
          Ue[long(i) * M + m] = x;
          dsum += dx * dx;
          nsum += x * x;
        }
        continue;
      }
      for (; i + 28 < n; i += 32) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = Ue[long(i + 4 * u) * M + m];
#pragma unroll
        for (int u = 0; u < 8; ++u) Ue[long(i + 4 * u) * M + m] = v[u] * f;
      }
      for (; i < n; i += 4) Ue[long(i) * M + m] *= f;
    }
  if (A.change) {
    // block sum in a fixed order: lanes of a wave by shuffles, then the waves
    for (int o = 32; o > 0; o >>= 1) {
      dsum += __shfl_xor(dsum, o);
      nsum += __shfl_xor(nsum, o);
    }
    __syncthreads();
    if (m == 0) {
      part[ph][0] = dsum;
      part[ph][1] = nsum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double dd = (part[0][0] + part[1][0]) + (part[2][0] + part[3][0]);
      const double nn = (part[0][1] + part[1][1]) + (part[2][1] + part[3][1]);
      *A.change = nn > 0.0 ? sqrt(dd / nn) : (dd > 0.0 ? INFINITY : 0.0);
    }
  }
  if (A.fac) {
    if (ph == 0 && m < M)
      for (int e = 0; e < A.D; ++e) gp(A.fac)[e * M + m] = fac[e][m];
    return;
  }
  for (int e = 0; e < A.D; ++e) {
    if (!(scale_mask & (1u << e))) continue;
    const int MM = M * M;
    const auto G = gp(A.gram[e]), LG = gp(A.lgram[e]);
    for (int t = threadIdx.x; t < A.K[e] * MM; t += blockDim.x) {
      const int r = t - (t / MM) * MM, mm = r / M, nn = r - (r / M) * M;
      G[t] *= fac[e][mm] * fac[e][nn];
    }
    for (int t = threadIdx.x; t < A.Rc[e] * M; t += blockDim.x) LG[t] *= fac[e][t - (t / M) * M];
  }
}

// The Grams and load Grams of the dims in scale_mask follow the factors
// balance() applied (A.fac): G^k[m][n] *= f_m f_n, L[c][m] *= f_m, for the
// entries [t0, t0 + blockDim.x) of the mask's dims laid end to end.
__device__ inline void rescale_grams(const BalanceArgs& A, unsigned scale_mask, long t0) {
  const int M = A.M, MM = M * M;
  long t = t0 + threadIdx.x;
  for (int e = 0; e < A.D; ++e) {
    if (!(scale_mask & (1u << e))) continue;
    const long g = long(A.K[e]) * MM, l = long(A.Rc[e]) * M;
    const auto f = gp(A.fac) + e * M;
    if (t < g) {
      const int r = int(t % MM), mm = r / M, nn = r - mm * M;
      gp(A.gram[e])[t] *= f[mm] * f[nn];
      return;
    }
    t -= g;
    if (t < l) {
      gp(A.lgram[e])[t] *= f[int(t % M)];
      return;
    }
    t -= l;
  }
}

}  // namespace dev
}  // namespace taps
