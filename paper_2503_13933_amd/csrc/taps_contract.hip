// Grams, load Grams, Hadamard couplings and the force of the dim-d system
// (paper Sec. 2.5: the 1D integrals of the other dimensions collapse into
// M x M coefficient matrices that multiply entrywise; the forcing term gives
// Q^[d]).  All reductions are two-stage with a fixed summation order, so two
// runs give bitwise equal results.
#include "taps_device.hpp"

namespace {

using namespace taps::dev;

__global__ __launch_bounds__(256) void k_gram_partial(int n, int M, int s, int K, const double* __restrict__ band,
                               const double* __restrict__ U, double* __restrict__ part) {
  gram_partial(blockIdx.x, n, M, s, K, band, U, part + long(blockIdx.x) * K * M * M);
}

__global__ void k_sum_parts(int nparts, long len, const double* __restrict__ part, double* __restrict__ out) {
  sum_parts(blockIdx.x, nparts, len, part, out);
}

__global__ __launch_bounds__(256) void k_lgram_partial(int n, int Rc, int M, const double* __restrict__ F, const double* __restrict__ U,
                                double* __restrict__ part) {
  lgram_partial(blockIdx.x, blockIdx.y, kLgRows, n, Rc, M, F, U, part);
}

__global__ void k_couple(CoupleArgs A, double* __restrict__ C) { couple(blockIdx.x, A, C); }

__global__ void k_load_terms(WeightArgs A) { load_terms(blockIdx.x, A); }
__global__ void k_load_weights(WeightArgs A, double* __restrict__ Wt) { load_weights(blockIdx.x, A, Wt); }

__global__ __launch_bounds__(256) void k_force(int n, int Rc, int M, const double* __restrict__ F, const double* __restrict__ Wt,
                        double* __restrict__ Q) {
  force(blockIdx.x, n, Rc, M, F, Wt, Q);
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
    const size_t lds = size_t(gram_lds_doubles(M, p->s[e])) * 8;
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
  TAPS_TRY(need_ws(h, size_t(Rc + p->R) * M * 8, stream));
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
  wa.P = Wt + size_t(Rc) * M;
  k_load_terms<<<cdiv(long(p->R) * M, 256), 256, 0, stream>>>(wa);
  TAPS_LAUNCHED(h, "k_load_terms");
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
