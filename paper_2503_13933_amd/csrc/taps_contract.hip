// Grams, load Grams, Hadamard couplings and the force of the dim-d system
// (paper Sec. 2.5: the 1D integrals of the other dimensions collapse into
// M x M coefficient matrices that multiply entrywise; the forcing term gives
// Q^[d]).  All reductions are two-stage with a fixed summation order, so two
// runs give bitwise equal results.
#include "taps_internal.hpp"

namespace {

constexpr int kGramRows = 64;   // rows of U per Gram partial block
constexpr int kLgCols = 64;     // load columns per load-Gram block
constexpr int kLgRows = 256;    // rows per load-Gram split
constexpr int kLgStage = 32;    // rows staged in LDS at a time
constexpr int kQRows = 64;      // rows of Q per force block
constexpr int kQStage = 32;     // load columns staged in LDS at a time

// Stage 1 of G^k = U^T A^k U: one block per chunk of kGramRows rows.  The chunk
// of U plus a halo of w rows each side goes to LDS; V = A^k U is formed on the
// chunk rows, then the chunk's contribution U_chunk^T V is written as a partial.
__global__ void k_gram_partial(int n, int M, int s, int K, const double* __restrict__ band,
                               const double* __restrict__ U, double* __restrict__ part) {
  extern __shared__ double lds[];
  const int w = 2 * s + 1, BW = 2 * w + 1;
  const int r0 = blockIdx.x * kGramRows;
  const int rows = min(kGramRows, n - r0);
  double* sU = lds;                                 // (kGramRows + 2w) x M
  double* sV = lds + (kGramRows + 2 * w) * M;       // kGramRows x M
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
      part[(long(blockIdx.x) * K + k) * M * M + t] = acc;
    }
    __syncthreads();
  }
}

// Stage 2: out[t] = sum_b part[b][t] in block order.
__global__ void k_sum_parts(int nparts, long len, const double* __restrict__ part, double* __restrict__ out) {
  const long t = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (t >= len) return;
  double acc = 0.0;
  for (int b = 0; b < nparts; ++b) acc += part[long(b) * len + t];
  out[t] = acc;
}

// Stage 1 of L = F^T U: block (column tile, row split) accumulates
// sum_{i in split} F[i][c] U[i][m] for its kLgCols columns.
__global__ void k_lgram_partial(int n, int Rc, int M, const double* __restrict__ F,
                                const double* __restrict__ U, double* __restrict__ part) {
  __shared__ double sF[kLgStage][kLgCols + 1];
  __shared__ double sU[kLgStage * TAPS_MAX_M];
  const int c0 = blockIdx.x * kLgCols;
  const int rbeg = blockIdx.y * kLgRows, rend = min(n, rbeg + kLgRows);
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
  // partial layout: [split][Rc][M]
  for (int q = 0; q < kPer; ++q) {
    const int o = threadIdx.x + q * blockDim.x;
    if (o < nout) {
      const int c = o / M, m = o % M;
      if (c0 + c < Rc) part[(long(blockIdx.y) * Rc + c0 + c) * M + m] = acc[q];
    }
  }
}

struct CoupleArgs {
  int D, M, T, d;
  int tk[TAPS_MAX_TERMS][TAPS_MAX_DIMS];
  double gamma[TAPS_MAX_TERMS];
  const double* gram[TAPS_MAX_DIMS];  // cache base of dim e's Grams (n_kinds[e] x M x M)
  int Kd;
};

// C^k_d[m][n] = sum over terms whose dim-d matrix is k of
// gamma * prod_{e != d} G_e^{kind(term, e)}[m][n]  (Hadamard product).
__global__ void k_couple(CoupleArgs A, double* __restrict__ C) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
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
  const double* lgram[TAPS_MAX_DIMS];     // Rc_e x M
  const int* col[TAPS_MAX_DIMS];          // R entries or null (identity)
  const int* ptr;                         // dim d grouping (null = identity)
  const int* idx;
};

// Wt[c][m] = sum over load terms r with col_d(r) = c of prod_{e != d} L_e[col_e(r)][m].
__global__ void k_load_weights(WeightArgs A, double* __restrict__ Wt) {
  const long t = blockIdx.x * long(blockDim.x) + threadIdx.x;
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

// Q = F_d Wt: block per kQRows rows, load columns staged through LDS.
__global__ void k_force(int n, int Rc, int M, const double* __restrict__ F, const double* __restrict__ Wt,
                        double* __restrict__ Q) {
  __shared__ double sF[kQRows][kQStage + 1];
  __shared__ double sW[kQStage * TAPS_MAX_M];
  const int r0 = blockIdx.x * kQRows;
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

size_t gram_lds_allowed = 0;

}  // namespace

namespace taps {

size_t cache_gram_off(const taps_problem_t* p, int e) {
  size_t off = 0;
  for (int f = 0; f < e; ++f)
    off += align256(size_t(p->n_kinds[f]) * p->M * p->M * 8) + align256(size_t(p->R_cols[f]) * p->M * 8);
  return off;
}
size_t cache_lgram_off(const taps_problem_t* p, int e) {
  return cache_gram_off(p, e) + align256(size_t(p->n_kinds[e]) * p->M * p->M * 8);
}
size_t cache_total(const taps_problem_t* p) { return cache_gram_off(p, p->D); }

taps_status prepare_cache(taps_handle* h, const taps_problem_t* p, hipStream_t stream) {
  bool same = h->sig_D == p->D && h->sig_M == p->M;
  for (int d = 0; same && d < p->D; ++d)
    same = h->sig_n[d] == p->n[d] && h->sig_k[d] == p->n_kinds[d] && h->sig_r[d] == p->R_cols[d];
  if (!same) {
    h->gc.valid = 0;
    h->sig_D = p->D;
    h->sig_M = p->M;
    for (int d = 0; d < p->D; ++d) {
      h->sig_n[d] = p->n[d];
      h->sig_k[d] = p->n_kinds[d];
      h->sig_r[d] = p->R_cols[d];
    }
  }
  void* buf = h->cache;
  size_t have = h->cache_bytes;
  const size_t need = cache_total(p);
  if (need > have) {
    TAPS_TRY(grow(h, &buf, &have, need, stream));
    h->cache = static_cast<double*>(buf);
    h->cache_bytes = have;
    h->gc.valid = 0;
  }
  h->gc.base = h->cache;
  return TAPS_OK;
}

taps_status refresh_grams(taps_handle* h, const taps_problem_t* p, taps_gram_cache* gc, uint32_t mask,
                          const double* const* d_U, hipStream_t stream) {
  const int M = p->M;
  for (int e = 0; e < p->D; ++e) {
    if (!(mask & (1u << e))) continue;
    if (!d_U[e]) return fail(h, TAPS_ERR_INVALID, "factor of dim %d is null", e);
    const int n = p->n[e], K = p->n_kinds[e], Rc = p->R_cols[e];
    const int w = 2 * p->s[e] + 1;
    // --- Grams
    const int chunks = cdiv(n, kGramRows);
    const size_t part_g = size_t(chunks) * K * M * M * 8;
    const int ctiles = cdiv(Rc, kLgCols), splits = cdiv(n, kLgRows);
    const size_t part_l = size_t(splits) * Rc * M * 8;
    TAPS_TRY(need_ws(h, align256(part_g) + align256(part_l), stream));
    double* pg = static_cast<double*>(h->ws);
    double* pl = reinterpret_cast<double*>(static_cast<char*>(h->ws) + align256(part_g));
    double* gram = gc->base + cache_gram_off(p, e) / 8;
    double* lgram = gc->base + cache_lgram_off(p, e) / 8;
    const size_t lds = size_t(2 * kGramRows + 2 * w) * M * 8;
    TAPS_TRY(allow_lds(h, k_gram_partial, lds, &gram_lds_allowed));
    size_t slot;
    TAPS_TRY(prof_begin(h, TAPS_PROF_CONTRACT, stream, &slot));
    k_gram_partial<<<chunks, 256, lds, stream>>>(n, M, p->s[e], K, p->d_band[e], d_U[e], pg);
    TAPS_LAUNCHED(h, "k_gram_partial");
    const long glen = long(K) * M * M;
    k_sum_parts<<<cdiv(glen, 256), 256, 0, stream>>>(chunks, glen, pg, gram);
    TAPS_LAUNCHED(h, "k_sum_parts(gram)");
    // --- load Grams
    dim3 grid(ctiles, splits);
    k_lgram_partial<<<grid, 256, 0, stream>>>(n, Rc, M, p->d_F[e], d_U[e], pl);
    TAPS_LAUNCHED(h, "k_lgram_partial");
    const long llen = long(Rc) * M;
    k_sum_parts<<<cdiv(llen, 256), 256, 0, stream>>>(splits, llen, pl, lgram);
    TAPS_LAUNCHED(h, "k_sum_parts(lgram)");
    {
      const double bw = 2 * w + 1;
      const double fl = double(K) * (2.0 * bw * n * M + 2.0 * n * double(M) * M) + 2.0 * n * double(Rc) * M;
      const double by = 8.0 * (double(n) * M + K * n * bw + double(n) * Rc + K * double(M) * M + double(Rc) * M);
      TAPS_TRY(prof_end(h, slot, fl, by, stream));
    }
    gc->valid |= (1u << e);
  }
  return TAPS_OK;
}

taps_status couple_and_force(taps_handle* h, const taps_problem_t* p, const taps_gram_cache* gc, int d,
                             double* d_C, double* d_Q, hipStream_t stream) {
  const int M = p->M;
  CoupleArgs ca{};
  ca.D = p->D;
  ca.M = M;
  ca.T = p->T;
  ca.d = d;
  ca.Kd = p->n_kinds[d];
  for (int t = 0; t < p->T; ++t) {
    ca.gamma[t] = p->gamma[t];
    for (int e = 0; e < p->D; ++e) ca.tk[t][e] = p->term_kind[t][e];
  }
  for (int e = 0; e < p->D; ++e) ca.gram[e] = gc->base + cache_gram_off(p, e) / 8;
  size_t slot;
  TAPS_TRY(prof_begin(h, TAPS_PROF_CONTRACT, stream, &slot));
  k_couple<<<cdiv(long(ca.Kd) * M * M, 256), 256, 0, stream>>>(ca, d_C);
  TAPS_LAUNCHED(h, "k_couple");

  const int Rc = p->R_cols[d];
  TAPS_TRY(need_ws(h, size_t(Rc) * M * 8, stream));
  double* Wt = static_cast<double*>(h->ws);
  WeightArgs wa{};
  wa.D = p->D;
  wa.M = M;
  wa.R = p->R;
  wa.d = d;
  wa.Rc = Rc;
  for (int e = 0; e < p->D; ++e) {
    wa.lgram[e] = gc->base + cache_lgram_off(p, e) / 8;
    wa.col[e] = p->d_load_col[e];
  }
  wa.ptr = p->d_load_ptr[d];
  wa.idx = p->d_load_idx[d];
  k_load_weights<<<cdiv(long(Rc) * M, 256), 256, 0, stream>>>(wa, Wt);
  TAPS_LAUNCHED(h, "k_load_weights");
  k_force<<<cdiv(p->n[d], kQRows), 256, 0, stream>>>(p->n[d], Rc, M, p->d_F[d], Wt, d_Q);
  TAPS_LAUNCHED(h, "k_force");
  const double n = p->n[d];
  const double fl = 2.0 * n * Rc * M + double(p->R) * (p->D - 1) * M + double(ca.Kd) * p->T * (p->D - 1) * M * M;
  const double by = 8.0 * (n * Rc + double(Rc) * M + n * M + double(ca.Kd) * M * M);
  TAPS_TRY(prof_end(h, slot, fl, by, stream));
  return TAPS_OK;
}

}  // namespace taps

using namespace taps;

extern "C" taps_status taps_contract(taps_handle_t h, const taps_problem_t* prob, int32_t d,
                                     uint32_t stale_mask, const double* const* d_U, double* d_C,
                                     double* d_Q, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  TAPS_TRY(check_problem(h, prob));
  if (d < 0 || d >= prob->D) return fail(h, TAPS_ERR_INVALID, "dim %d out of range", d);
  if (!d_U || !d_C || !d_Q) return fail(h, TAPS_ERR_INVALID, "null pointer");
  TAPS_TRY(prepare_cache(h, prob, stream));
  const uint32_t all = (prob->D >= 32) ? 0xffffffffu : ((1u << prob->D) - 1u);
  const uint32_t need = all & ~(1u << d);
  const uint32_t refresh = (stale_mask | ~h->gc.valid) & need;
  TAPS_TRY(refresh_grams(h, prob, &h->gc, refresh, d_U, stream));
  if (stale_mask & (1u << d)) h->gc.valid &= ~(1u << d);
  return couple_and_force(h, prob, &h->gc, d, d_C, d_Q, stream);
}
