// Projected residual, mode balancing and the Algorithm 1 driver
// (paper Sec. 2.5, the block-diagonal nonlinear system; Sec. 2.6, subspace
// iteration).
#include "taps_device.hpp"

#include <vector>


namespace {

struct ResFinal {
  int D;
  int nparts[TAPS_MAX_DIMS];
  const double* part[TAPS_MAX_DIMS];
};

__global__ void k_residual_final(ResFinal A, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double rs = 0.0, qs = 0.0;
  for (int d = 0; d < A.D; ++d) {
    double r = 0.0, q = 0.0;
    for (int b = 0; b < A.nparts[d]; ++b) {
      r += A.part[d][2 * b];
      q += A.part[d][2 * b + 1];
    }
    out[d] = r;
    rs += r;
    qs += q;
  }
  out[A.D] = qs;
  out[A.D + 1] = (qs > 0.0) ? sqrt(rs / qs) : sqrt(rs);
}

using taps::dev::BalanceArgs;

__global__ __launch_bounds__(256) void k_balance(BalanceArgs A) { taps::dev::balance(A); }

__global__ __launch_bounds__(256) void k_snapshot(BalanceArgs A) { taps::dev::snapshot(A); }

__global__ void k_first_info(int D, const int* __restrict__ infos, int* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int v = 0;
  for (int d = 0; d < D && v == 0; ++d) v = infos[d];
  out[0] = v;
}


}  // namespace

using namespace taps;

namespace {

// Driver region of the handle: C and Q of the dim being solved, residual
// partials of every dim, one info word per dim.
struct DriverBufs {
  double* C;
  double* Q;
  double* parts;
  double* berr;
  int* infos;
  double* snap;  // factors at the start of a sweep (sum_d n_d M doubles)
};

taps_status driver_bufs(taps_handle* h, const taps_problem_t* p, DriverBufs* out, hipStream_t stream) {
  int Kmax = 1, nmax = 1, parts_total = 0;
  size_t nsum = 0;
  for (int d = 0; d < p->D; ++d) {
    Kmax = std::max(Kmax, p->n_kinds[d]);
    nmax = std::max(nmax, p->n[d]);
    parts_total += dim_residual_nparts(p->n[d]);
    nsum += size_t(p->n[d]);
  }
  Bump b;
  const size_t oC = b.take(size_t(Kmax) * p->M * p->M * 8);
  const size_t oQ = b.take(size_t(nmax) * p->M * 8);
  const size_t oP = b.take(size_t(parts_total) * 2 * 8);
  const size_t oB = b.take(TAPS_MAX_DIMS * 8);
  const size_t oI = b.take(TAPS_MAX_DIMS * 4);
  const size_t oS = b.take(nsum * p->M * 8);
  TAPS_TRY(grow(h, &h->side, &h->side_bytes, b.off, stream));
  char* base = static_cast<char*>(h->side);
  out->C = reinterpret_cast<double*>(base + oC);
  out->Q = reinterpret_cast<double*>(base + oQ);
  out->parts = reinterpret_cast<double*>(base + oP);
  out->berr = reinterpret_cast<double*>(base + oB);
  out->infos = reinterpret_cast<int*>(base + oI);
  out->snap = reinterpret_cast<double*>(base + oS);
  return TAPS_OK;
}

taps_status residual_impl(taps_handle* h, const taps_problem_t* p, const double* const* d_U, double* d_out,
                          hipStream_t stream) {
  TAPS_TRY(prepare_cache(h, p, stream));
  DriverBufs db;
  TAPS_TRY(driver_bufs(h, p, &db, stream));
  const uint32_t all = (1u << p->D) - 1u;
  TAPS_TRY(refresh_grams(h, p, &h->gc, all, d_U, stream));
  ResFinal rf{};
  rf.D = p->D;
  int off = 0;
  for (int d = 0; d < p->D; ++d) {
    TAPS_TRY(couple_and_force(h, p, &h->gc, d, db.C, db.Q, stream));
    int nb = 0;
    TAPS_TRY(dim_residual_parts(h, p, d, db.C, d_U[d], db.Q, db.parts + 2 * off, &nb, stream));
    rf.nparts[d] = nb;
    rf.part[d] = db.parts + 2 * off;
    off += nb;
  }
  k_residual_final<<<1, 64, 0, stream>>>(rf, d_out);
  TAPS_LAUNCHED(h, "k_residual_final");
  return TAPS_OK;
}

// snap: sum_d n_d M doubles holding the factors of the sweep's start (null:
// no change measured); change: where the relative change goes.
BalanceArgs balance_args(const taps_problem_t* p, double* const* d_U, double* snap, double* change) {
  BalanceArgs ba{};
  ba.D = p->D;
  ba.M = p->M;
  size_t off = 0;
  for (int d = 0; d < p->D; ++d) {
    ba.n[d] = p->n[d];
    ba.U[d] = d_U[d];
    ba.snap[d] = snap ? snap + off : nullptr;
    off += size_t(p->n[d]) * p->M;
  }
  ba.change = snap ? change : nullptr;
  return ba;
}

taps_status balance_impl(taps_handle* h, const taps_problem_t* p, double* const* d_U, hipStream_t stream,
                         double* snap = nullptr, double* change = nullptr) {
  const BalanceArgs ba = balance_args(p, d_U, snap, change);
  k_balance<<<1, 256, 0, stream>>>(ba);
  TAPS_LAUNCHED(h, "k_balance");
  h->gc.valid = 0;  // every Gram changes scale
  return TAPS_OK;
}

taps_status sweep_impl(taps_handle* h, const taps_problem_t* p, double* const* d_U, int* d_info,
                       double* d_berr, hipStream_t stream, double* d_change = nullptr) {
  TAPS_TRY(prepare_cache(h, p, stream));
  DriverBufs db;
  TAPS_TRY(driver_bufs(h, p, &db, stream));
  if (d_change) {
    k_snapshot<<<1, 256, 0, stream>>>(balance_args(p, d_U, db.snap, d_change));
    TAPS_LAUNCHED(h, "k_snapshot");
  }
  const uint32_t all = (1u << p->D) - 1u;
  h->gc.valid = 0;  // the factors passed in need not be those the cache was built from
  for (int d = 0; d < p->D; ++d) {
    const uint32_t need = all & ~(1u << d);
    TAPS_TRY(refresh_grams(h, p, &h->gc, need & ~h->gc.valid, d_U, stream));
    TAPS_TRY(couple_and_force(h, p, &h->gc, d, db.C, db.Q, stream));
    TAPS_TRY(solve_dim_impl(h, p, d, db.C, db.Q, d_U[d], db.infos + d, (d_berr ? d_berr : db.berr) + d, stream));
    h->gc.valid &= ~(1u << d);
  }
  TAPS_TRY(balance_impl(h, p, d_U, stream, d_change ? db.snap : nullptr, d_change));
  if (d_info) {
    k_first_info<<<1, 64, 0, stream>>>(p->D, db.infos, d_info);
    TAPS_LAUNCHED(h, "k_first_info");
  }
  return TAPS_OK;
}

}  // namespace

namespace taps {

// Launchers shared with the batched driver.
taps_status balance_launch(taps_handle* h, const taps_problem_t* p, double* const* d_U, hipStream_t stream) {
  BalanceArgs ba{};
  ba.D = p->D;
  ba.M = p->M;
  for (int d = 0; d < p->D; ++d) {
    ba.n[d] = p->n[d];
    ba.U[d] = d_U[d];
  }
  k_balance<<<1, 256, 0, stream>>>(ba);
  TAPS_LAUNCHED(h, "k_balance");
  return TAPS_OK;
}

taps_status residual_final_launch(taps_handle* h, int D, const int* nparts, double* const* parts, double* out,
                                  hipStream_t stream) {
  ResFinal rf{};
  rf.D = D;
  for (int d = 0; d < D; ++d) {
    rf.nparts[d] = nparts[d];
    rf.part[d] = parts[d];
  }
  k_residual_final<<<1, 64, 0, stream>>>(rf, out);
  TAPS_LAUNCHED(h, "k_residual_final");
  return TAPS_OK;
}

}  // namespace taps

namespace {

taps_status check_factors(taps_handle* h, const taps_problem_t* p, const void* const* d_U) {
  if (!d_U) return fail(h, TAPS_ERR_INVALID, "factor array is null");
  for (int d = 0; d < p->D; ++d)
    if (!d_U[d]) return fail(h, TAPS_ERR_INVALID, "factor %d is null", d);
  return TAPS_OK;
}

}  // namespace

extern "C" {

taps_status taps_residual(taps_handle_t h, const taps_problem_t* prob, const double* const* d_U,
                          double* d_out, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  TAPS_TRY(check_problem(h, prob));
  TAPS_TRY(check_factors(h, prob, reinterpret_cast<const void* const*>(d_U)));
  if (!d_out) return fail(h, TAPS_ERR_INVALID, "null output");
  return residual_impl(h, prob, d_U, d_out, stream);
}

taps_status taps_balance(taps_handle_t h, const taps_problem_t* prob, double* const* d_U,
                         hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  TAPS_TRY(check_problem(h, prob));
  TAPS_TRY(check_factors(h, prob, reinterpret_cast<const void* const*>(d_U)));
  return balance_impl(h, prob, d_U, stream);
}

taps_status taps_sweep(taps_handle_t h, const taps_problem_t* prob, double* const* d_U, int32_t* d_info,
                       double* d_berr, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  TAPS_TRY(check_problem(h, prob));
  TAPS_TRY(check_factors(h, prob, reinterpret_cast<const void* const*>(d_U)));
  return sweep_impl(h, prob, d_U, d_info, d_berr, stream);
}

taps_status taps_als(taps_handle_t h, const taps_problem_t* prob, double* const* d_U, double tol,
                     double change_tol, int32_t iter_max, int32_t* sweeps, double* rho, double* change,
                     double* history, double* change_history, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  TAPS_TRY(check_problem(h, prob));
  TAPS_TRY(check_factors(h, prob, reinterpret_cast<const void* const*>(d_U)));
  if (!sweeps || !rho) return fail(h, TAPS_ERR_INVALID, "null output");
  if (iter_max < 1) return fail(h, TAPS_ERR_INVALID, "iter_max < 1");
  const int D = prob->D;
  double* d_res = h->d_small;                               // D+2 doubles
  double* d_be = h->d_small + 32;                           // D doubles
  int* d_inf = reinterpret_cast<int*>(h->d_small + 64);    // one word
  double* d_chg = h->d_small + 80;                          // one double
  double res[TAPS_MAX_DIMS + 2], be[TAPS_MAX_DIMS], chg = NAN;
  int info = 0;
  *sweeps = 0;
  *rho = NAN;
  if (change) *change = NAN;
  // the change needs a copy of the factors per sweep: only when asked for
  const bool want_change = change || change_history || change_tol > 0.0;
  for (int it = 0; it < iter_max; ++it) {
    TAPS_TRY(sweep_impl(h, prob, d_U, d_inf, d_be, stream, want_change ? d_chg : nullptr));
    TAPS_TRY(residual_impl(h, prob, d_U, d_res, stream));
    TAPS_HIP(h, hipMemcpyAsync(res, d_res, size_t(D + 2) * 8, hipMemcpyDeviceToHost, stream));
    TAPS_HIP(h, hipMemcpyAsync(be, d_be, size_t(D) * 8, hipMemcpyDeviceToHost, stream));
    TAPS_HIP(h, hipMemcpyAsync(&info, d_inf, 4, hipMemcpyDeviceToHost, stream));
    if (want_change) TAPS_HIP(h, hipMemcpyAsync(&chg, d_chg, 8, hipMemcpyDeviceToHost, stream));
    TAPS_HIP(h, hipStreamSynchronize(stream));
    *sweeps = it + 1;
    int bad = -1;
    for (int d = 0; d < D && bad < 0; ++d)
      if (!(be[d] <= TAPS_BERR_LIMIT)) bad = d;
    *rho = (info || bad >= 0) ? NAN : res[D + 1];
    if (info || bad >= 0) chg = NAN;
    if (history) history[it] = *rho;
    if (change_history) change_history[it] = chg;
    if (change) *change = chg;
    if (info) {
      if (info < 0)
        fail(h, TAPS_OK, "sweep %d: eigen stage of the fast diagonalisation failed (info %d)", it + 1, info);
      else
        fail(h, TAPS_OK, "sweep %d: zero or non-finite pivot (info %d)", it + 1, info);
      break;
    }
    if (bad >= 0) {
      fail(h, TAPS_OK, "sweep %d: dim %d solve backward error %.3e above %.0e", it + 1, bad, be[bad],
           TAPS_BERR_LIMIT);
      break;
    }
    if (!(*rho > tol)) break;
    if (change_tol > 0.0 && chg <= change_tol) break;
  }
  return TAPS_OK;
}

}  // extern "C"
