// Batched Algorithm 1 (paper Sec. 2.6) over many independent problems --
// slabs, parameter queries -- that share D, M and the patch size of each dim
// (grid sizes may differ).  Every dim step solves all active systems in one
// launch, one workgroup per system; problems that reach the tolerance (or
// break down) are predicated off on the host after each sweep.
#include "taps_internal.hpp"

#include <algorithm>
#include <cstring>
#include <vector>

using namespace taps;

namespace {

struct ProbLayout {
  size_t cache, C, Q, ws, parts, out, info;  // byte offsets in the batch buffer
  int nparts[TAPS_MAX_DIMS];
  int part_off[TAPS_MAX_DIMS];              // in units of 2 doubles
};

}  // namespace

extern "C" taps_status taps_als_batched(taps_handle_t h, int32_t B, const taps_problem_t* probs,
                                        double* const* d_U, double tol, int32_t iter_max, int32_t* sweeps,
                                        double* rho, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (B < 1 || !probs || !d_U || !sweeps || !rho) return fail(h, TAPS_ERR_INVALID, "bad batch arguments");
  if (iter_max < 1) return fail(h, TAPS_ERR_INVALID, "iter_max < 1");
  const taps_problem_t& p0 = probs[0];
  for (int b = 0; b < B; ++b) {
    TAPS_TRY(check_problem(h, &probs[b]));
    const taps_problem_t& p = probs[b];
    if (p.D != p0.D || p.M != p0.M)
      return fail(h, TAPS_ERR_INVALID, "problem %d: D and M must match the batch", b);
    for (int d = 0; d < p.D; ++d) {
      if (p.s[d] != p0.s[d]) return fail(h, TAPS_ERR_INVALID, "problem %d dim %d: patch size differs", b, d);
      if (!d_U[size_t(b) * p.D + d]) return fail(h, TAPS_ERR_INVALID, "problem %d factor %d is null", b, d);
    }
  }
  const int D = p0.D, M = p0.M;
  for (int d = 0; d < D; ++d)
    if (!solve_batched_supported(M, p0.s[d]))
      return fail(h, TAPS_ERR_UNSUPPORTED, "batched solve needs M=%d, s=%d to fit LDS", M, p0.s[d]);

  // ---- layout of the batch buffer
  const size_t args_sz = solve_args_bytes();
  Bump bump;
  const size_t o_args = bump.take(args_sz * size_t(D) * B);
  const size_t o_active = bump.take(size_t(B) * 4);
  const size_t o_outs = bump.take(size_t(B) * (2 * D + 2) * 8);
  const size_t o_infos = bump.take(size_t(B) * D * 4);
  std::vector<ProbLayout> L(B);
  for (int b = 0; b < B; ++b) {
    const taps_problem_t& p = probs[b];
    int Kmax = 1, nmax = 1, tot = 0;
    size_t ws = 0;
    for (int d = 0; d < D; ++d) {
      Kmax = std::max(Kmax, p.n_kinds[d]);
      nmax = std::max(nmax, p.n[d]);
      ws = std::max(ws, solve_ws_bytes(p.n[d], M, p.s[d]));
      L[b].nparts[d] = dim_residual_nparts(p.n[d]);
      L[b].part_off[d] = tot;
      tot += L[b].nparts[d];
    }
    L[b].cache = bump.take(cache_total(&p));
    L[b].C = bump.take(size_t(Kmax) * M * M * 8);
    L[b].Q = bump.take(size_t(nmax) * M * 8);
    L[b].ws = bump.take(ws);
    L[b].parts = bump.take(size_t(tot) * 2 * 8);
  }
  TAPS_TRY(grow(h, &h->batch, &h->batch_bytes, bump.off, stream));
  char* base = static_cast<char*>(h->batch);
  double* outs = reinterpret_cast<double*>(base + o_outs);  // [b]: res (D+2), berr (D)
  int* infos = reinterpret_cast<int*>(base + o_infos);       // [b][d]
  int* d_active = reinterpret_cast<int*>(base + o_active);
  auto C_of = [&](int b) { return reinterpret_cast<double*>(base + L[b].C); };
  auto Q_of = [&](int b) { return reinterpret_cast<double*>(base + L[b].Q); };
  auto parts_of = [&](int b) { return reinterpret_cast<double*>(base + L[b].parts); };
  auto U_of = [&](int b) { return d_U + size_t(b) * D; };

  // solve argument records for every (dim, problem)
  std::vector<char> args(args_sz * size_t(D) * B);
  for (int d = 0; d < D; ++d)
    for (int b = 0; b < B; ++b)
      solve_args_fill(args.data() + (size_t(d) * B + b) * args_sz, &probs[b], d, C_of(b), Q_of(b),
                      U_of(b)[d], infos + size_t(b) * D + d, base + L[b].ws);
  TAPS_HIP(h, hipMemcpyAsync(base + o_args, args.data(), args.size(), hipMemcpyHostToDevice, stream));

  std::vector<taps_gram_cache> gc(B);
  for (int b = 0; b < B; ++b) gc[b].base = reinterpret_cast<double*>(base + L[b].cache);
  std::vector<int> active(B), next;
  for (int b = 0; b < B; ++b) {
    active[b] = b;
    sweeps[b] = 0;
    rho[b] = NAN;
  }
  TAPS_HIP(h, hipMemcpyAsync(d_active, active.data(), size_t(B) * 4, hipMemcpyHostToDevice, stream));
  std::vector<double> h_outs(size_t(B) * (2 * D + 2));
  std::vector<int> h_infos(size_t(B) * D);
  const uint32_t all = (1u << D) - 1u;

  for (int it = 0; it < iter_max && !active.empty(); ++it) {
    for (int b : active) gc[b].valid = 0;
    for (int d = 0; d < D; ++d) {
      const uint32_t need = all & ~(1u << d);
      double fl = 0.0, by = 0.0;
      for (int b : active) {
        const taps_problem_t& p = probs[b];
        TAPS_TRY(refresh_grams(h, &p, &gc[b], need & ~gc[b].valid, U_of(b), stream));
        TAPS_TRY(couple_and_force(h, &p, &gc[b], d, C_of(b), Q_of(b), stream));
        fl += solve_flops(p.n[d], M, 2 * p.s[d] + 1);
        by += solve_bytes(p.n[d], M, 2 * p.s[d] + 1, p.n_kinds[d]);
      }
      TAPS_TRY(solve_batched_launch(h, int(active.size()), base + o_args + size_t(d) * B * args_sz, d_active, M,
                                    p0.s[d], fl, by, stream));
      for (int b : active) {
        gc[b].valid &= ~(1u << d);
        int nb = 0;
        TAPS_TRY(dim_residual_parts(h, &probs[b], d, C_of(b), U_of(b)[d], Q_of(b), parts_of(b), &nb, stream));
        TAPS_TRY(berr_final_launch(h, nb, parts_of(b), outs + size_t(b) * (2 * D + 2) + (D + 2) + d, stream));
      }
    }
    for (int b : active) {
      const taps_problem_t& p = probs[b];
      TAPS_TRY(balance_launch(h, &p, U_of(b), stream));
      gc[b].valid = 0;
      TAPS_TRY(refresh_grams(h, &p, &gc[b], all, U_of(b), stream));
      double* parts[TAPS_MAX_DIMS];
      for (int d = 0; d < D; ++d) {
        TAPS_TRY(couple_and_force(h, &p, &gc[b], d, C_of(b), Q_of(b), stream));
        parts[d] = parts_of(b) + 2 * L[b].part_off[d];
        int nb = 0;
        TAPS_TRY(dim_residual_parts(h, &p, d, C_of(b), U_of(b)[d], Q_of(b), parts[d], &nb, stream));
      }
      TAPS_TRY(residual_final_launch(h, D, L[b].nparts, parts, outs + size_t(b) * (2 * D + 2), stream));
    }
    TAPS_HIP(h, hipMemcpyAsync(h_outs.data(), outs, h_outs.size() * 8, hipMemcpyDeviceToHost, stream));
    TAPS_HIP(h, hipMemcpyAsync(h_infos.data(), infos, h_infos.size() * 4, hipMemcpyDeviceToHost, stream));
    TAPS_HIP(h, hipStreamSynchronize(stream));
    next.clear();
    for (int b : active) {
      const double* o = h_outs.data() + size_t(b) * (2 * D + 2);
      bool broke = false;
      for (int d = 0; d < D; ++d)
        broke = broke || h_infos[size_t(b) * D + d] != 0 || !(o[D + 2 + d] <= TAPS_BERR_LIMIT);
      sweeps[b] = it + 1;
      rho[b] = broke ? NAN : o[D + 1];
      if (!broke && rho[b] > tol) next.push_back(b);
    }
    if (next.size() != active.size() && !next.empty())
      TAPS_HIP(h, hipMemcpyAsync(d_active, next.data(), next.size() * 4, hipMemcpyHostToDevice, stream));
    active.swap(next);
    // keep the staged active list alive until the copy has run
    TAPS_HIP(h, hipStreamSynchronize(stream));
  }
  return TAPS_OK;
}
