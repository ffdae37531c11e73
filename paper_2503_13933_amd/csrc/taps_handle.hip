// Handle lifetime, workspace, argument validation and the host Gauss rule.
#include "taps_internal.hpp"

#include <new>

namespace taps {

void gauss_legendre(int n, double* xi, double* w) {
  // Roots of the Legendre polynomial P_n by Newton iteration from the
  // Chebyshev-like initial guess cos(pi (k + 3/4) / (n + 1/2)); weights
  // 2 / ((1 - x^2) P_n'(x)^2).  Symmetric pairs are filled from one root.
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < (n + 1) / 2; ++k) {
    double x = std::cos(pi * (k + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? x : p1;
      double pm = (n == 1) ? 1.0 : p0;
      dp = n * (x * pn - pm) / (x * x - 1.0);
      double dx = pn / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) {
        // one more evaluation of the derivative at the converged root
        p0 = 1.0;
        p1 = x;
        for (int j = 2; j <= n; ++j) {
          double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
          p0 = p1;
          p1 = p2;
        }
        pn = (n == 1) ? x : p1;
        pm = (n == 1) ? 1.0 : p0;
        dp = n * (x * pn - pm) / (x * x - 1.0);
        break;
      }
    }
    double wk = 2.0 / ((1.0 - x * x) * dp * dp);
    // ascending order: the negative root first
    xi[k] = -x;
    w[k] = wk;
    xi[n - 1 - k] = x;
    w[n - 1 - k] = wk;
  }
  if (n % 2 == 1) xi[n / 2] = 0.0;
}

taps_status check_basis(taps_handle* h, const taps_basis1d_t* b) {
  if (!b) return fail(h, TAPS_ERR_INVALID, "basis is null");
  if (!b->d_x) return fail(h, TAPS_ERR_INVALID, "basis node pointer is null");
  if (b->s < 0 || b->s > TAPS_MAX_S)
    return fail(h, TAPS_ERR_UNSUPPORTED, "patch size s=%d outside 0..%d", b->s, TAPS_MAX_S);
  if (b->p < 0 || b->p > b->s)
    return fail(h, TAPS_ERR_UNSUPPORTED, "reproducing order p=%d needs 0 <= p <= s=%d", b->p, b->s);
  if (!(b->a > 0.0)) return fail(h, TAPS_ERR_INVALID, "dilation a must be positive");
  if (b->n_nodes < 2 || b->n_nodes < 2 * b->s + 2)
    return fail(h, TAPS_ERR_UNSUPPORTED, "n_nodes=%d below max(2, 2s+2)", b->n_nodes);
  if (b->n_gauss < 1 || b->n_gauss > TAPS_MAX_GAUSS)
    return fail(h, TAPS_ERR_UNSUPPORTED, "n_gauss=%d outside 1..%d", b->n_gauss, TAPS_MAX_GAUSS);
  return TAPS_OK;
}

taps_status check_problem(taps_handle* h, const taps_problem_t* p) {
  if (!p) return fail(h, TAPS_ERR_INVALID, "problem is null");
  if (p->D < 1 || p->D > TAPS_MAX_DIMS) return fail(h, TAPS_ERR_UNSUPPORTED, "D=%d", p->D);
  if (p->M < 1 || p->M > TAPS_MAX_M) return fail(h, TAPS_ERR_UNSUPPORTED, "M=%d", p->M);
  if (p->T < 1 || p->T > TAPS_MAX_TERMS) return fail(h, TAPS_ERR_UNSUPPORTED, "T=%d", p->T);
  if (p->R < 1) return fail(h, TAPS_ERR_INVALID, "R=%d", p->R);
  for (int d = 0; d < p->D; ++d) {
    if (p->s[d] < 0 || p->s[d] > TAPS_MAX_S)
      return fail(h, TAPS_ERR_UNSUPPORTED, "dim %d: s=%d", d, p->s[d]);
    if (p->n[d] < 2 * p->s[d] + 2 || p->n[d] < 2)
      return fail(h, TAPS_ERR_UNSUPPORTED, "dim %d: n=%d below 2s+2", d, p->n[d]);
    if (p->n_kinds[d] < 1 || p->n_kinds[d] > TAPS_MAX_KINDS)
      return fail(h, TAPS_ERR_UNSUPPORTED, "dim %d: n_kinds=%d", d, p->n_kinds[d]);
    if (!p->d_band[d]) return fail(h, TAPS_ERR_INVALID, "dim %d: band pointer is null", d);
    if (p->R_cols[d] < 1 || !p->d_F[d]) return fail(h, TAPS_ERR_INVALID, "dim %d: no load columns", d);
    bool any = p->d_load_col[d] || p->d_load_ptr[d] || p->d_load_idx[d];
    bool all = p->d_load_col[d] && p->d_load_ptr[d] && p->d_load_idx[d];
    if (any && !all) return fail(h, TAPS_ERR_INVALID, "dim %d: load map needs col, ptr and idx", d);
    if (!any && p->R_cols[d] != p->R)
      return fail(h, TAPS_ERR_INVALID, "dim %d: identity load map needs R_cols == R", d);
  }
  for (int t = 0; t < p->T; ++t)
    for (int d = 0; d < p->D; ++d)
      if (p->term_kind[t][d] < 0 || p->term_kind[t][d] >= p->n_kinds[d])
        return fail(h, TAPS_ERR_INVALID, "term %d dim %d: kind %d out of range", t, d, p->term_kind[t][d]);
  return TAPS_OK;
}

taps_status prof_begin(taps_handle* h, int family, hipStream_t stream, size_t* slot) {
  *slot = size_t(-1);
  if (!h->prof.on) return TAPS_OK;
  auto& P = h->prof;
  if (2 * (P.used + 1) > P.ev.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      TAPS_HIP(h, hipEventCreate(&e));
      P.ev.push_back(e);
    }
    P.fam.push_back(family);
  }
  P.fam[P.used] = family;
  TAPS_HIP(h, hipEventRecord(P.ev[2 * P.used], stream));
  *slot = P.used++;
  return TAPS_OK;
}

taps_status prof_end(taps_handle* h, size_t slot, double flops, double bytes, hipStream_t stream) {
  if (slot == size_t(-1)) return TAPS_OK;
  auto& P = h->prof;
  TAPS_HIP(h, hipEventRecord(P.ev[2 * slot + 1], stream));
  P.flops[P.fam[slot]] += flops;
  P.bytes[P.fam[slot]] += bytes;
  return TAPS_OK;
}

}  // namespace taps

namespace {
// does nothing: its dispatches mark where a profiled region starts and ends
// in an external kernel trace or counter run
__global__ void k_prof_mark(int) {}
}  // namespace

extern "C" {

taps_status taps_profile_enable(taps_handle_t h, int32_t enable) {
  if (!h) return TAPS_ERR_INVALID;
  k_prof_mark<<<1, 64, 0, nullptr>>>(enable);
  TAPS_LAUNCHED(h, "k_prof_mark");
  if (enable) {
    h->prof.used = 0;
    for (int f = 0; f < kProfFamilies; ++f) h->prof.flops[f] = h->prof.bytes[f] = 0.0;
  }
  h->prof.on = enable != 0;
  return TAPS_OK;
}

taps_status taps_profile_read(taps_handle_t h, taps_prof_family family, int32_t* launches, double* total_ms,
                              double* flops, double* bytes) {
  if (!h) return TAPS_ERR_INVALID;
  if (family != TAPS_PROF_SOLVE && family != TAPS_PROF_CONTRACT && family != TAPS_PROF_RECON &&
      family != TAPS_PROF_EIG && family != TAPS_PROF_SCHUR)
    return taps::fail(h, TAPS_ERR_INVALID, "unknown family %d", int(family));
  auto& P = h->prof;
  int cnt = 0;
  double ms = 0.0;
  for (size_t i = 0; i < P.used; ++i) {
    if (P.fam[i] != family) continue;
    TAPS_HIP(h, hipEventSynchronize(P.ev[2 * i + 1]));
    float t = 0.0f;
    TAPS_HIP(h, hipEventElapsedTime(&t, P.ev[2 * i], P.ev[2 * i + 1]));
    ms += t;
    ++cnt;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = ms;
  if (flops) *flops = P.flops[family];
  if (bytes) *bytes = P.bytes[family];
  return TAPS_OK;
}

taps_status taps_create(taps_handle_t* out) {
  if (!out) return TAPS_ERR_INVALID;
  *out = nullptr;
  taps_handle* h = new (std::nothrow) taps_handle();
  if (!h) return TAPS_ERR_ALLOC;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return TAPS_ERR_HIP;
  }
  if (hipMalloc(reinterpret_cast<void**>(&h->d_small), 1024) != hipSuccess) {
    delete h;
    return TAPS_ERR_ALLOC;
  }
  const taps_status st = taps::recon_scratch_attach(h);
  if (st != TAPS_OK) {
    (void)hipFree(h->d_small);
    delete h;
    return st;
  }
  *out = h;
  return TAPS_OK;
}

taps_status taps_destroy(taps_handle_t h) {
  if (!h) return TAPS_OK;
  (void)hipDeviceSynchronize();
  if (h->ws) (void)hipFree(h->ws);
  if (h->cache) (void)hipFree(h->cache);
  for (auto e : h->prof.ev) (void)hipEventDestroy(e);
  if (h->side) (void)hipFree(h->side);
  if (h->batch) (void)hipFree(h->batch);
  if (h->stage) (void)hipHostFree(h->stage);
  if (h->stage_ev) (void)hipEventDestroy(h->stage_ev);
  if (h->d_small) (void)hipFree(h->d_small);
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->gstream) (void)hipStreamDestroy(h->gstream);
  delete h;
  return TAPS_OK;
}

taps_status taps_set_tuning(taps_handle_t h, const taps_tuning_t* t) {
  if (!h) return TAPS_ERR_INVALID;
  if (!t || t->graph_sweeps < 0 || t->graph_sweeps > 16)
    return taps::fail(h, TAPS_ERR_INVALID, "graph_sweeps must be 0..16");
  if (t->solver != 0 && t->solver != 1) return taps::fail(h, TAPS_ERR_INVALID, "solver must be 0 or 1");
  if (t->lgram_rows != 0 && (t->lgram_rows < 16 || t->lgram_rows > 4096 || t->lgram_rows % 16))
    return taps::fail(h, TAPS_ERR_INVALID, "lgram_rows must be 0 or a multiple of 16 in 16..4096");
  h->tune = *t;
  return TAPS_OK;
}

taps_status taps_get_tuning(taps_handle_t h, taps_tuning_t* t) {
  if (!h) return TAPS_ERR_INVALID;
  if (!t) return taps::fail(h, TAPS_ERR_INVALID, "null pointer");
  *t = h->tune;
  return TAPS_OK;
}

const char* taps_last_error(taps_handle_t h) { return h ? h->err.c_str() : "null handle"; }

taps_status taps_reserve(taps_handle_t h, size_t bytes) {
  if (!h) return TAPS_ERR_INVALID;
  return taps::need_ws(h, bytes, nullptr);
}

size_t taps_workspace_bytes(taps_handle_t h) { return h ? h->ws_bytes + h->cache_bytes : 0; }

}  // extern "C"
