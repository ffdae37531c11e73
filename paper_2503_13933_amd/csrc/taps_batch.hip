// Batched Algorithm 1 (paper Sec. 2.6) over many independent problems --
// slabs, parameter queries -- that share D, M and the patch size of each dim
// (grid sizes may differ).  Every step of a sweep is one launch over all
// active problems: Gram refreshes, couplings, forces, the dim solves (one
// workgroup per system), the backward-error check, balancing and the
// residual.  The row-chunked contraction kernels (Gram, load Gram, force,
// residual) are persistent: a fixed grid of workgroups strides over the work
// items -- one per (problem, row chunk), or (problem, column tile, row split)
// for the load Gram -- of exactly the active problems however uneven their
// sizes.  Item w belongs to the active problem a with pref[a] <= w <
// pref[a+1] (a binary search in a per-kind prefix table of the active
// problems' item counts, read from device memory, so a captured graph stays
// valid while the table changes).  Problems that reach the tolerance or break
// down are predicated off on the host after each sweep by shrinking the
// active list and its prefix tables.
#include "taps_device.hpp"

#include <algorithm>
#include <cstring>
#include <unordered_set>
#include <vector>

using namespace taps;
using namespace taps::dev;

namespace {

// Device record of one problem of the batch.
struct BProb {
  int D, M;
  int n[TAPS_MAX_DIMS], s[TAPS_MAX_DIMS], K[TAPS_MAX_DIMS], Rc[TAPS_MAX_DIMS];
  const double* band[TAPS_MAX_DIMS];
  const double* F[TAPS_MAX_DIMS];
  const uint8_t* fixed[TAPS_MAX_DIMS];
  double* U[TAPS_MAX_DIMS];
  double* gram[TAPS_MAX_DIMS];
  double* lgram[TAPS_MAX_DIMS];
  int roff[TAPS_MAX_DIMS];  // residual partial offset of dim d (units of 2 doubles)
  double* C;
  double* Q;
  double* Wt;
  double* gpart;
  double* lpart;
  double* qpart;  // partial forces of split load rows ([split][n M])
  double* wpart;  // partial load weights of sliced long groups ([group][slice][M])
  double* rparts;
  double* outs;  // res (D+2), backward error per dim (D), relative change of the sweep (1)
};

enum { kItGram = 0, kItLgram = 1, kItForce = 2, kItRes = 3, kItKinds = 4 };
// load columns per force work item where a dim's loads are split (long load
// rows: the force of a few problems with tens of thousands of load terms
// would otherwise run on a few waves per SIMD with its loads exposed)
constexpr int kForceCols = 1024;
// terms per slice of a long load group (load weights formed in place)
constexpr int kWSlice = 512;
// persistent grid sizes (a few items per workgroup at full batches)
constexpr int kPersistLds = 4096, kPersistStream = 8192;

// Work item w -> (active problem index in P, item index within the problem).
// pref has nact + 1 entries (pref[nact] the item count); owner[w] is the
// active index a with pref[a] <= w < pref[a + 1], written by kb_owner_fill
// whenever the active set changes, so an item is located by one load.
struct Item {
  int b, c;
};
__device__ inline Item locate(const int* __restrict__ act, const int* __restrict__ pref,
                              const int* __restrict__ owner, int w) {
  const int a = owner[w];
  return Item{act[a], w - pref[a]};
}

// owner tables of every (kind, dim): one thread per active problem fills
// its items' entries (grid.y = kind * D + dim)
struct OwnerOffsets {
  int off[kItKinds * TAPS_MAX_DIMS];
};
__global__ void kb_owner_fill(const int* __restrict__ pref, int* __restrict__ owner, OwnerOffsets oo, int nact,
                              int B) {
  const int kd = blockIdx.y;
  const int* pr = pref + size_t(kd) * (B + 1);
  int* ow = owner + oo.off[kd];
  for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < nact; a += gridDim.x * blockDim.x)
    for (int w = pr[a]; w < pr[a + 1]; ++w) ow[w] = a;
}

// One instantiation per band width BW = 4s + 3 (a launch's problems share
// the patch size of each dim), so a kernel holds the registers of its own
// band width only; at most 168 registers: three workgroups per CU, as many
// as the LDS allows.
template <int BW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void kb_gram_partial(
    const BProb* __restrict__ P, const int* __restrict__ act, const int* __restrict__ pref,
    const int* __restrict__ owner, int nact, int e) {
  const int nit = pref[nact];
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item x = locate(act, pref, owner, w);
    const BProb& q = P[x.b];
    gram_partial_bw<BW>(x.c, q.n[e], q.M, q.K[e], q.band[e], q.U[e], q.gpart + long(x.c) * q.K[e] * q.M * q.M);
    __syncthreads();   // LDS free for the next item
  }
}

// The elementwise kernels (sums of partials, couplings, load terms and
// weights) run kVB slices of 256 items per block: a grid with one slice per
// block has tens of thousands of tiny blocks, and their dispatch, not their
// work, then sets the time.
constexpr int kVB = 8;

__global__ void kb_gram_sum(const BProb* __restrict__ P, const int* __restrict__ act, int e) {
  const BProb& q = P[act[blockIdx.y]];
  const int chunks = (q.n[e] + kGramRows - 1) / kGramRows;
  sum_parts_n<kVB>(blockIdx.x * kVB, chunks, long(q.K[e]) * q.M * q.M, q.gpart, q.gram[e]);
}

// (NCT 16-column tiles per pass, the fewest that cover M: three waves per
// SIMD up to 48 modes)
template <int NCT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void kb_lgram_partial(
    const BProb* __restrict__ P, const int* __restrict__ act, const int* __restrict__ pref,
    const int* __restrict__ owner, int nact, int e, int rows) {
  const int nit = pref[nact];
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item x = locate(act, pref, owner, w);
    const BProb& q = P[x.b];
    const int splits = (q.n[e] + rows - 1) / rows;
    const int ct = x.c / splits;
    lgram_partial<NCT>(ct, x.c - ct * splits, rows, q.n[e], q.Rc[e], q.M, q.F[e], q.U[e], q.lpart);
  }
}

__global__ void kb_lgram_sum(const BProb* __restrict__ P, const int* __restrict__ act, int e, int rows) {
  const BProb& q = P[act[blockIdx.y]];
  const int splits = (q.n[e] + rows - 1) / rows;
  sum_parts_n<kVB>(blockIdx.x * kVB, splits, long(q.Rc[e]) * q.M, q.lpart, q.lgram[e]);
}

// one coupling record per problem (its term table), for every dim
__global__ void kb_couple(const BProb* __restrict__ P, const CoupleArgs* __restrict__ CA,
                          const int* __restrict__ act, int d) {
  const int b = act[blockIdx.y];
  couple_n<kVB>(blockIdx.x * kVB, CA[b], d, P[b].K[d], P[b].C);
}

__global__ void kb_load_terms(const WeightArgs* __restrict__ WA, const int* __restrict__ act, int d, int D) {
  load_terms_n<kVB>(blockIdx.x * kVB, WA[long(act[blockIdx.y]) * D + d]);
}

__global__ void kb_load_weights(const BProb* __restrict__ P, const WeightArgs* __restrict__ WA,
                                const int* __restrict__ act, int d, int D) {
  const int b = act[blockIdx.y];
#pragma unroll
  for (int u = 0; u < kVB; ++u) load_weights(blockIdx.x * kVB + u, WA[long(b) * D + d], P[b].Wt);
}

// Long groups, products formed in place: block x = group * wsl + slice
// (blocks past a problem's group count return); wsl = 1 writes the load
// weights directly, otherwise per-slice partials summed by kb_wsum.
__global__ __launch_bounds__(256) void kb_load_weights_fused(const BProb* __restrict__ P,
                                                             const WeightArgs* __restrict__ WA,
                                                             const int* __restrict__ act, int d, int D, int wsl) {
  const int b = act[blockIdx.y];
  const WeightArgs& A = WA[long(b) * D + d];
  const int c = blockIdx.x / wsl, sl = blockIdx.x - c * wsl;
  if (c >= A.Rc) return;
  load_weights_fused(c, sl, wsl, A, wsl == 1 ? P[b].Wt : P[b].wpart);
}

__global__ void kb_wsum(const BProb* __restrict__ P, const WeightArgs* __restrict__ WA, const int* __restrict__ act,
                        int d, int D, int wsl) {
  const int b = act[blockIdx.y];
  const BProb& q = P[b];
  const int M = q.M, Rc = WA[long(b) * D + d].Rc;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Rc * M) return;
  const int c = t / M, m = t - c * M;
  const auto part = gp(q.wpart) + long(c) * wsl * M + m;
  double acc = 0.0;
  for (int sl = 0; sl < wsl; ++sl) acc += part[long(sl) * M];
  gp(q.Wt)[t] = acc;
}

// split = 0: item = row block, Q written directly; split = 1: item = (row
// block, column range of kForceCols), partial Q per range, summed by
// kb_force_sum.  (NCT as in the load Gram: 152 registers at NCT = 3, three
// waves per SIMD.)
template <int NCT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void kb_force(
    const BProb* __restrict__ P, const int* __restrict__ act, const int* __restrict__ pref,
    const int* __restrict__ owner, int nact, int d, int split) {
  const int nit = pref[nact];
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item x = locate(act, pref, owner, w);
    const BProb& q = P[x.b];
    if (!split) {
      force<NCT>(x.c, q.n[d], q.Rc[d], q.M, q.F[d], q.Wt, q.Q);
    } else {
      const int ns = (q.Rc[d] + kForceCols - 1) / kForceCols, rb = x.c / ns, sp = x.c - rb * ns;
      force<NCT>(rb, q.n[d], q.Rc[d], q.M, q.F[d], q.Wt, q.qpart + long(sp) * q.n[d] * q.M, sp * kForceCols,
                 (sp + 1) * kForceCols);
    }
  }
}

__global__ void kb_force_sum(const BProb* __restrict__ P, const int* __restrict__ act, int d) {
  const BProb& q = P[act[blockIdx.y]];
  const int ns = (q.Rc[d] + kForceCols - 1) / kForceCols;
  sum_parts_n<kVB>(blockIdx.x * kVB, ns, long(q.n[d]) * q.M, q.qpart, q.Q);
}

// (one instantiation per band width, as the Gram partials, and per number
// of 16-column tiles per pass, three up to 48 modes: up to s = 1, 128
// registers, four workgroups per CU, as many as the LDS allows; three for
// the wider bands, whose windows would spill at 128)
template <int BW, int NCT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BW <= 7 ? 4 : 3))) void kb_residual_part(
    const BProb* __restrict__ P, const int* __restrict__ act, const int* __restrict__ pref,
    const int* __restrict__ owner, int nact, int d) {
  const int nit = pref[nact];
  for (int w = blockIdx.x; w < nit; w += gridDim.x) {
    const Item x = locate(act, pref, owner, w);
    const BProb& q = P[x.b];
    residual_part_bw<BW, NCT>(x.c, q.n[d], q.M, q.K[d], q.band[d], q.C, q.U[d], q.Q, q.fixed[d],
                              q.rparts + 2 * (q.roff[d] + x.c));
    __syncthreads();   // LDS free for the next item
  }
}

// the instantiations of both, by patch size s (band width 4s + 3) and, for
// the residual, the number of modes
typedef void (*persist_fn)(const BProb*, const int*, const int*, const int*, int, int);
persist_fn gram_partial_for(int s) {
  switch (s) {
    case 0: return kb_gram_partial<3>;
    case 1: return kb_gram_partial<7>;
    case 2: return kb_gram_partial<11>;
    default: return kb_gram_partial<15>;
  }
}
persist_fn residual_part_for(int s, int M) {
  if (M <= 48) {
    switch (s) {
      case 0: return kb_residual_part<3, 3>;
      case 1: return kb_residual_part<7, 3>;
      case 2: return kb_residual_part<11, 3>;
      default: return kb_residual_part<15, 3>;
    }
  }
  switch (s) {
    case 0: return kb_residual_part<3, 4>;
    case 1: return kb_residual_part<7, 4>;
    case 2: return kb_residual_part<11, 4>;
    default: return kb_residual_part<15, 4>;
  }
}

// One thread per active problem: backward error of dim d from its partials.
__global__ void kb_berr_final(const BProb* __restrict__ P, const int* __restrict__ act, int nact, int d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nact) return;
  const BProb& q = P[act[i]];
  const int nb = (q.n[d] + kResRows - 1) / kResRows;
  const double* part = q.rparts + 2 * q.roff[d];
  double r = 0.0, s = 0.0;
  for (int c = 0; c < nb; ++c) {
    r += part[2 * c];
    s += part[2 * c + 1];
  }
  q.outs[q.D + 2 + d] = s > 0.0 ? sqrt(r / s) : sqrt(r);
}

// One thread per active problem: per-dim ||R_d||^2, sum ||Q_d||^2 and rho.
__global__ void kb_residual_final(const BProb* __restrict__ P, const int* __restrict__ act, int nact) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nact) return;
  const BProb& q = P[act[i]];
  double rs = 0.0, qs = 0.0;
  for (int d = 0; d < q.D; ++d) {
    const int nb = (q.n[d] + kResRows - 1) / kResRows;
    const double* part = q.rparts + 2 * q.roff[d];
    double r = 0.0, s = 0.0;
    for (int c = 0; c < nb; ++c) {
      r += part[2 * c];
      s += part[2 * c + 1];
    }
    q.outs[d] = r;
    rs += r;
    qs += s;
  }
  q.outs[q.D] = qs;
  q.outs[q.D + 1] = qs > 0.0 ? sqrt(rs / qs) : sqrt(rs);
}

__global__ __launch_bounds__(256) void kb_balance(const BalanceArgs* __restrict__ BA, const int* __restrict__ act,
                                                   unsigned scale_mask) {
  balance(BA[act[blockIdx.x]], scale_mask);
}

// the Gram rescaling of the balance over many blocks per problem (a large
// load Gram rescaled by the one balancing block took milliseconds)
__global__ __launch_bounds__(256) void kb_rescale_grams(const BalanceArgs* __restrict__ BA,
                                                        const int* __restrict__ act, unsigned scale_mask) {
  const BalanceArgs& A = BA[act[blockIdx.y]];
#pragma unroll
  for (int u = 0; u < kVB; ++u) rescale_grams(A, scale_mask, (long(blockIdx.x) * kVB + u) * blockDim.x);
}

__global__ __launch_bounds__(256) void kb_snapshot(const BalanceArgs* __restrict__ BA, const int* __restrict__ act) {
  snapshot(BA[act[blockIdx.x]]);
}

size_t gram_lds_allowed[4] = {}, res_lds_allowed[4] = {};   // per patch size 0..3

// grid sizes per dim (maxima over the batch; blocks past a problem's own
// extent return at once)
struct Sizes {
  int chunks[TAPS_MAX_DIMS], ctiles[TAPS_MAX_DIMS], splits[TAPS_MAX_DIMS], gram[TAPS_MAX_DIMS];
  int lgram[TAPS_MAX_DIMS], rblocks[TAPS_MAX_DIMS], cpl[TAPS_MAX_DIMS], wt[TAPS_MAX_DIMS];
  int rchunks[TAPS_MAX_DIMS], rc[TAPS_MAX_DIMS], qlen[TAPS_MAX_DIMS], fsplit[TAPS_MAX_DIMS], wsl[TAPS_MAX_DIMS];
  int max_terms = 1;
  Sizes() {
    for (int d = 0; d < TAPS_MAX_DIMS; ++d) {
      chunks[d] = ctiles[d] = splits[d] = gram[d] = lgram[d] = rblocks[d] = cpl[d] = wt[d] = rchunks[d] = rc[d] = 1;
      qlen[d] = 1;
      fsplit[d] = 0;
      wsl[d] = 1;
    }
  }
};

}  // namespace

extern "C" taps_status taps_als_batched(taps_handle_t h, int32_t B, const taps_problem_t* probs,
                                        double* const* d_U, double tol, double change_tol, int32_t iter_max,
                                        int32_t* sweeps, double* rho, double* change, hipStream_t stream) {
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
  const int D = p0.D, M = p0.M, MM = M * M;
  // the relative change of a sweep needs the factors of its start (one copy
  // per sweep); measured only when asked for or used by the stop rule
  const bool want_change = change != nullptr || change_tol > 0.0;
  // per dim: fast diagonalisation when selected and every system of the
  // batch has two kinds, block LU otherwise
  std::vector<char> use_fd(D, 0);
  for (int d = 0; d < D; ++d) {
    bool fd = h->tune.solver == 1;
    for (int b = 0; b < B && fd; ++b) fd = solve_fd_supported(M, p0.s[d], probs[b].n_kinds[d]);
    use_fd[d] = fd;
    int kmax = 1;
    for (int b = 0; b < B; ++b) kmax = std::max(kmax, probs[b].n_kinds[d]);
    if (!fd && !solve_batched_supported(M, p0.s[d], kmax))
      return fail(h, TAPS_ERR_UNSUPPORTED, "batched block LU needs M=%d, s=%d to fit LDS and at most 4 kinds (%d)", M,
                  p0.s[d], kmax);
  }

  // ---- layout of the batch buffer
  const size_t args_sz = solve_args_bytes();
  const int lg_rows = h->tune.lgram_rows > 0 ? h->tune.lgram_rows : kLgRows;
  Sizes Z;
  for (int d = 0; d < D; ++d)
    for (int b = 0; b < B; ++b)
      if (probs[b].R_cols[d] > kForceCols) Z.fsplit[d] = 1;
  // dims whose load map is the identity in every problem: the per-term
  // products are the load weights themselves, written straight into Wt
  std::vector<char> ident(D, 1);
  for (int d = 0; d < D; ++d)
    for (int b = 0; b < B; ++b)
      if (probs[b].d_load_col[d]) ident[d] = 0;
  // long groups (on average 64 terms or more per load column in every
  // problem): the products formed in place, each group cut into Z.wsl slices
  // of at most about kWSlice terms on average
  std::vector<char> long_groups(D, 1);
  for (int d = 0; d < D; ++d) {
    for (int b = 0; b < B; ++b) {
      const taps_problem_t& p = probs[b];
      if (long(p.R) < 64L * p.R_cols[d]) long_groups[d] = 0;
      Z.wsl[d] = std::max(Z.wsl[d], cdiv(cdiv(p.R, p.R_cols[d]), kWSlice));
    }
    if (!long_groups[d] || ident[d]) Z.wsl[d] = 1;
  }
  Bump bump;
  const size_t o_args = bump.take(args_sz * size_t(D) * B);
  const size_t o_prob = bump.take(sizeof(BProb) * size_t(B));
  const size_t o_cpl = bump.take(sizeof(CoupleArgs) * size_t(B));
  const size_t o_wa = bump.take(sizeof(WeightArgs) * size_t(B) * D);
  const size_t o_bal = bump.take(sizeof(BalanceArgs) * size_t(B));
  const size_t o_active = bump.take(size_t(B) * 4);
  const int NO = 2 * D + 3;  // outputs per problem
  const size_t o_outs = bump.take(size_t(B) * NO * 8);
  const size_t o_infos = bump.take(size_t(B) * D * 4);
  // work items of every (kind, dim) per problem, their totals over the batch,
  // and the prefix tables over the active problems (B + 1 entries each)
  auto items_of = [&](int kind, int b, int d) -> int {
    const taps_problem_t& p = probs[b];
    switch (kind) {
      case kItGram: return cdiv(p.n[d], kGramRows);
      case kItLgram: return cdiv(p.R_cols[d], kLgCols) * cdiv(p.n[d], lg_rows);
      case kItForce: return cdiv(p.n[d], kQRows) * (Z.fsplit[d] ? cdiv(p.R_cols[d], kForceCols) : 1);
      default: return cdiv(p.n[d], kResRows);
    }
  };
  std::vector<long> it_full(kItKinds * D, 0);
  for (int b = 0; b < B; ++b)
    for (int k = 0; k < kItKinds; ++k)
      for (int d = 0; d < D; ++d) it_full[k * D + d] += items_of(k, b, d);
  const size_t o_pref = bump.take(size_t(kItKinds) * D * (B + 1) * 4);
  OwnerOffsets own_off{};
  long own_total = 0;
  for (int kd = 0; kd < kItKinds * D; ++kd) {
    own_off.off[kd] = int(own_total);
    own_total += it_full[kd];
  }
  if (own_total >= (1L << 31)) return fail(h, TAPS_ERR_UNSUPPORTED, "too many work items in one batch");
  const size_t o_owner = bump.take(size_t(std::max(1L, own_total)) * 4);
  std::vector<BProb> bp(B);
  std::vector<size_t> o_cache(B), o_C(B), o_Q(B), o_Wt(B), o_gp(B), o_lp(B), o_rp(B), o_ws(B), wt_doubles(B);
  std::vector<size_t> o_snap(B), o_qp(B), o_fac(B), o_wp(B);
  long rescale_len = 1;   // Gram and load-Gram entries of all dims, largest problem
  for (int b = 0; b < B; ++b) {
    const taps_problem_t& p = probs[b];
    int Kmax = 1, nmax = 1, tot = 0;
    size_t ws = 0, gp = 0, lp = 0, wt = 0, nsum = 0, qp = 0, wp = 0;
    for (int d = 0; d < D; ++d) {
      const int ch = cdiv(p.n[d], kGramRows), ct = cdiv(p.R_cols[d], kLgCols), sp = cdiv(p.n[d], lg_rows);
      Kmax = std::max(Kmax, p.n_kinds[d]);
      nmax = std::max(nmax, p.n[d]);
      ws = std::max(ws, solve_ws_bytes(p.n[d], M, p.s[d], use_fd[d]));
      gp = std::max(gp, size_t(ch) * p.n_kinds[d] * MM * 8);
      lp = std::max(lp, size_t(sp) * p.R_cols[d] * M * 8);
      wt = std::max(wt, size_t(p.R_cols[d]) * M * 8);
      Z.max_terms = std::max(Z.max_terms, cdiv(long(p.R) * M, 256));
      bp[b].roff[d] = tot;
      nsum += size_t(p.n[d]);
      tot += cdiv(p.n[d], kResRows);
      Z.chunks[d] = std::max(Z.chunks[d], ch);
      Z.ctiles[d] = std::max(Z.ctiles[d], ct);
      Z.splits[d] = std::max(Z.splits[d], sp);
      Z.gram[d] = std::max(Z.gram[d], cdiv(long(p.n_kinds[d]) * MM, 256));
      Z.lgram[d] = std::max(Z.lgram[d], cdiv(long(p.R_cols[d]) * M, 256));
      Z.rblocks[d] = std::max(Z.rblocks[d], cdiv(p.n[d], kQRows));
      Z.cpl[d] = std::max(Z.cpl[d], cdiv(long(p.n_kinds[d]) * MM, 256));
      Z.wt[d] = std::max(Z.wt[d], cdiv(long(p.R_cols[d]) * M, 256));
      Z.rchunks[d] = std::max(Z.rchunks[d], cdiv(p.n[d], kResRows));
      Z.rc[d] = std::max(Z.rc[d], p.R_cols[d]);
      Z.qlen[d] = std::max(Z.qlen[d], cdiv(long(p.n[d]) * M, 256));
      if (Z.fsplit[d]) qp = std::max(qp, size_t(cdiv(p.R_cols[d], kForceCols)) * p.n[d] * M * 8);
      if (Z.wsl[d] > 1) wp = std::max(wp, size_t(p.R_cols[d]) * Z.wsl[d] * M * 8);
    }
    o_cache[b] = bump.take(cache_total(&p));
    o_C[b] = bump.take(size_t(Kmax) * MM * 8);
    o_Q[b] = bump.take(size_t(nmax) * M * 8);
    o_Wt[b] = bump.take(wt + size_t(p.R) * M * 8);   // Wt, then the per-term products
    wt_doubles[b] = wt / 8;
    o_gp[b] = bump.take(gp);
    o_lp[b] = bump.take(lp);
    o_rp[b] = bump.take(size_t(tot) * 2 * 8);
    o_ws[b] = bump.take(ws);
    o_snap[b] = bump.take(nsum * M * 8);
    o_fac[b] = bump.take(size_t(D) * M * 8);
    o_wp[b] = bump.take(wp);
    long rl = 0;
    for (int d = 0; d < D; ++d) rl += long(p.n_kinds[d]) * MM + long(p.R_cols[d]) * M;
    rescale_len = std::max(rescale_len, rl);
    o_qp[b] = bump.take(qp);
  }
  TAPS_TRY(grow(h, &h->batch, &h->batch_bytes, bump.off, stream));
  char* base = static_cast<char*>(h->batch);
  double* outs = reinterpret_cast<double*>(base + o_outs);
  int* infos = reinterpret_cast<int*>(base + o_infos);
  int* d_active = reinterpret_cast<int*>(base + o_active);
  const BProb* d_prob = reinterpret_cast<const BProb*>(base + o_prob);
  const CoupleArgs* d_cpl = reinterpret_cast<const CoupleArgs*>(base + o_cpl);
  const WeightArgs* d_wa = reinterpret_cast<const WeightArgs*>(base + o_wa);
  const BalanceArgs* d_bal = reinterpret_cast<const BalanceArgs*>(base + o_bal);
  const int* d_pref = reinterpret_cast<const int*>(base + o_pref);
  auto pref = [&](int kind, int d) { return d_pref + size_t(kind * D + d) * (B + 1); };
  int* d_owner = reinterpret_cast<int*>(base + o_owner);
  auto owner = [&](int kind, int d) { return d_owner + own_off.off[kind * D + d]; };
  // persistent grid of one kernel: its items over the whole batch, capped
  auto pgrid = [&](int kind, int d, int cap) { return unsigned(std::max(1L, std::min(long(cap), it_full[kind * D + d]))); };
  // prefix tables of the active problems' item counts, staged in the
  // handle's pinned staging behind the records (set below)
  const size_t pref_len = size_t(kItKinds) * D * (B + 1);
  int* h_pref = nullptr;
  auto upload_items = [&](const std::vector<int>& act_list, hipStream_t st) -> taps_status {
    for (int k = 0; k < kItKinds; ++k)
      for (int d = 0; d < D; ++d) {
        int* pr = h_pref + size_t(k * D + d) * (B + 1);
        pr[0] = 0;
        for (size_t a = 0; a < act_list.size(); ++a) pr[a + 1] = pr[a] + items_of(k, act_list[a], d);
      }
    TAPS_HIP(h, hipMemcpyAsync(base + o_pref, h_pref, pref_len * 4, hipMemcpyHostToDevice, st));
    TAPS_HIP(h, hipEventRecord(h->stage_ev, st));
    const int na = int(act_list.size());
    kb_owner_fill<<<dim3(cdiv(na, 256), kItKinds * D), 256, 0, st>>>(d_pref, d_owner, own_off, na, B);
    TAPS_LAUNCHED(h, "kb_owner_fill");
    return TAPS_OK;
  };

  // ---- device records, written straight into the handle's pinned staging in
  // the layout of [o_args, o_active + 4B) and sent in one copy; the prefix
  // tables follow them.  Every copy out of the staging is stream-ordered
  // before the launches that read it, and the staging is rewritten only
  // after the stream has drained (the readback of each sweep) or, in the
  // next call, after the event recorded behind the last copy.
  const size_t rec_bytes = o_active + size_t(B) * 4 - o_args;
  TAPS_TRY(stage_reserve(h, align256(rec_bytes) + pref_len * 4));
  char* const stg = static_cast<char*>(h->stage);
  h_pref = reinterpret_cast<int*>(stg + align256(rec_bytes));
  char* const args = stg;
  CoupleArgs* const cpl = reinterpret_cast<CoupleArgs*>(stg + (o_cpl - o_args));
  WeightArgs* const wa = reinterpret_cast<WeightArgs*>(stg + (o_wa - o_args));
  BalanceArgs* const bal = reinterpret_cast<BalanceArgs*>(stg + (o_bal - o_args));
  int* const act_h = reinterpret_cast<int*>(stg + (o_active - o_args));
  for (int b = 0; b < B; ++b) {
    const taps_problem_t& p = probs[b];
    BProb& q = bp[b];
    double* cache = reinterpret_cast<double*>(base + o_cache[b]);
    q.D = D;
    q.M = M;
    for (int d = 0; d < D; ++d) {
      q.n[d] = p.n[d];
      q.s[d] = p.s[d];
      q.K[d] = p.n_kinds[d];
      q.Rc[d] = p.R_cols[d];
      q.band[d] = p.d_band[d];
      q.F[d] = p.d_F[d];
      q.fixed[d] = p.d_fixed[d];
      q.U[d] = d_U[size_t(b) * D + d];
      q.gram[d] = cache + cache_gram_off(&p, d) / 8;
      q.lgram[d] = cache + cache_lgram_off(&p, d) / 8;
    }
    q.C = reinterpret_cast<double*>(base + o_C[b]);
    q.Q = reinterpret_cast<double*>(base + o_Q[b]);
    q.Wt = reinterpret_cast<double*>(base + o_Wt[b]);
    q.gpart = reinterpret_cast<double*>(base + o_gp[b]);
    q.lpart = reinterpret_cast<double*>(base + o_lp[b]);
    q.qpart = reinterpret_cast<double*>(base + o_qp[b]);
    q.wpart = reinterpret_cast<double*>(base + o_wp[b]);
    q.rparts = reinterpret_cast<double*>(base + o_rp[b]);
    q.outs = outs + size_t(b) * NO;
    // only the first T terms and D dims are read: the rest is left as it is
    CoupleArgs& ca = cpl[b];
    ca.D = D;
    ca.M = M;
    ca.T = p.T;
    ca.d = 0;
    ca.Kd = 0;
    for (int t = 0; t < p.T; ++t) {
      ca.gamma[t] = p.gamma[t];
      for (int e = 0; e < D; ++e) ca.tk[t][e] = p.term_kind[t][e];
    }
    for (int e = 0; e < D; ++e) ca.gram[e] = q.gram[e];
    for (int d = 0; d < D; ++d) {
      WeightArgs& w = wa[size_t(b) * D + d];
      w = WeightArgs{};
      w.D = D;
      w.M = M;
      w.R = p.R;
      w.d = d;
      w.Rc = p.R_cols[d];
      for (int e = 0; e < D; ++e) {
        w.lgram[e] = q.lgram[e];
        w.col[e] = p.d_load_col[e];
      }
      w.ptr = p.d_load_ptr[d];
      w.idx = p.d_load_idx[d];
      w.P = ident[d] ? q.Wt : q.Wt + wt_doubles[b];
      solve_args_fill(args + (size_t(d) * B + b) * args_sz, &p, d, q.C, q.Q, q.U[d],
                      infos + size_t(b) * D + d, base + o_ws[b], use_fd[d]);
    }
    bal[b] = BalanceArgs{};
    bal[b].D = D;
    bal[b].M = M;
    double* snap = reinterpret_cast<double*>(base + o_snap[b]);
    for (int d = 0; d < D; ++d) {
      bal[b].n[d] = p.n[d];
      bal[b].U[d] = q.U[d];
      bal[b].K[d] = p.n_kinds[d];
      bal[b].Rc[d] = p.R_cols[d];
      bal[b].gram[d] = q.gram[d];
      bal[b].lgram[d] = q.lgram[d];
      bal[b].snap[d] = snap;
      snap += size_t(p.n[d]) * M;
    }
    bal[b].change = want_change ? q.outs + 2 * D + 2 : nullptr;
    bal[b].fac = reinterpret_cast<double*>(base + o_fac[b]);
  }
  std::vector<int> active(B), next;
  for (int b = 0; b < B; ++b) {
    active[b] = b;
    act_h[b] = b;
    sweeps[b] = 0;
    rho[b] = NAN;
    if (change) change[b] = NAN;
  }
  std::memcpy(stg + (o_prob - o_args), bp.data(), sizeof(BProb) * B);
  TAPS_HIP(h, hipMemcpyAsync(base + o_args, stg, rec_bytes, hipMemcpyHostToDevice, stream));
  TAPS_HIP(h, hipEventRecord(h->stage_ev, stream));
  TAPS_TRY(upload_items(active, stream));
  // captured sweeps run on the handle's own stream: the uploads must have landed
  if (!h->prof.on && h->tune.graph_sweeps > 0) TAPS_HIP(h, hipStreamSynchronize(stream));

  const size_t glds = size_t(gram_lds_doubles(M, *std::max_element(p0.s, p0.s + D))) * 8;
  const size_t rlds = size_t(residual_lds_doubles(M, *std::max_element(p0.s, p0.s + D))) * 8;
  if (rlds > 160 * 1024 - 4096) return fail(h, TAPS_ERR_UNSUPPORTED, "residual needs %zu bytes of LDS", rlds);
  for (int d = 0; d < D; ++d) {
    const int si = std::min(p0.s[d], 3);
    TAPS_TRY(allow_lds(h, gram_partial_for(p0.s[d]), glds, &gram_lds_allowed[si]));
    TAPS_TRY(allow_lds(h, residual_part_for(p0.s[d], M), rlds, &res_lds_allowed[si]));
  }
  for (int d = 0; d < D; ++d)
    TAPS_TRY(use_fd[d] ? fd_prepare(h, M, p0.s[d]) : solve_batched_prepare(h, M, p0.s[d]));

  auto refresh = [&](int e, int nact, hipStream_t st) -> taps_status {
    size_t slot;
    TAPS_TRY(prof_begin(h, TAPS_PROF_CONTRACT, st, &slot));
    gram_partial_for(p0.s[e])<<<pgrid(kItGram, e, kPersistLds), 256, glds, st>>>(d_prob, d_active, pref(kItGram, e),
                                                                       owner(kItGram, e), nact, e);
    TAPS_LAUNCHED(h, "kb_gram_partial");
    kb_gram_sum<<<dim3(cdiv(Z.gram[e], kVB), nact), 256, 0, st>>>(d_prob, d_active, e);
    TAPS_LAUNCHED(h, "kb_gram_sum");
    (M <= 32 ? kb_lgram_partial<2> : M <= 48 ? kb_lgram_partial<3> : kb_lgram_partial<4>)<<<pgrid(kItLgram, e, kPersistStream), 256, 0, st>>>(d_prob, d_active, pref(kItLgram, e),
                                                                        owner(kItLgram, e), nact, e, lg_rows);
    TAPS_LAUNCHED(h, "kb_lgram_partial");
    kb_lgram_sum<<<dim3(cdiv(Z.lgram[e], kVB), nact), 256, 0, st>>>(d_prob, d_active, e, lg_rows);
    TAPS_LAUNCHED(h, "kb_lgram_sum");
    // work of the method: Grams (U read once for all kinds, K M^2 written;
    // flops K (2 bw n M + 2 n M^2)) and load Gram (F and U read, R M written;
    // 2 n R M flops); a load matrix shared by several problems (one grid's
    // time loads) is read once per launch
    // (counted only while profiling: a loop over the problems per launch)
    double fl = 0.0, by = 0.0;
    if (slot != size_t(-1)) {
      std::unordered_set<const double*> seen;
      for (int b : active) {
        const taps_problem_t& p = probs[b];
        const double n = p.n[e], K = p.n_kinds[e], Rc = p.R_cols[e], bw = 4 * p.s[e] + 3;
        const bool first = seen.insert(p.d_F[e]).second;
        fl += K * (2.0 * bw * n * M + 2.0 * n * M * M) + 2.0 * n * Rc * M;
        by += 8.0 * (n * M + K * MM + (first ? n * Rc : 0.0) + Rc * M);
      }
    }
    return prof_end(h, slot, fl, by, st);
  };
  auto system = [&](int d, int nact, hipStream_t st) -> taps_status {
    size_t slot;
    TAPS_TRY(prof_begin(h, TAPS_PROF_CONTRACT, st, &slot));
    kb_couple<<<dim3(cdiv(Z.cpl[d], kVB), nact), 256, 0, st>>>(d_prob, d_cpl, d_active, d);
    TAPS_LAUNCHED(h, "kb_couple");
    if (long_groups[d] && !ident[d]) {
      // products formed in place, group slices summed afterwards
      kb_load_weights_fused<<<dim3(Z.rc[d] * Z.wsl[d], nact), 256, 0, st>>>(d_prob, d_wa, d_active, d, D,
                                                                           Z.wsl[d]);
      TAPS_LAUNCHED(h, "kb_load_weights_fused");
      if (Z.wsl[d] > 1) {
        kb_wsum<<<dim3(cdiv(Z.wt[d], 1), nact), 256, 0, st>>>(d_prob, d_wa, d_active, d, D, Z.wsl[d]);
        TAPS_LAUNCHED(h, "kb_wsum");
      }
    } else {
      kb_load_terms<<<dim3(cdiv(Z.max_terms, kVB), nact), 256, 0, st>>>(d_wa, d_active, d, D);
      TAPS_LAUNCHED(h, "kb_load_terms");
    }
    if (ident[d] || long_groups[d]) {
      // the products are the weights (one term per load column), or the
      // weights were formed in place above
    } else {
      kb_load_weights<<<dim3(cdiv(Z.wt[d], kVB), nact), 256, 0, st>>>(d_prob, d_wa, d_active, d, D);
      TAPS_LAUNCHED(h, "kb_load_weights");
    }
    (M <= 32 ? kb_force<2> : M <= 48 ? kb_force<3> : kb_force<4>)<<<pgrid(kItForce, d, kPersistStream), 256, 0, st>>>(d_prob, d_active, pref(kItForce, d),
                                                                 owner(kItForce, d), nact, d, Z.fsplit[d]);
    TAPS_LAUNCHED(h, "kb_force");
    if (Z.fsplit[d]) {
      kb_force_sum<<<dim3(cdiv(Z.qlen[d], kVB), nact), 256, 0, st>>>(d_prob, d_active, d);
      TAPS_LAUNCHED(h, "kb_force_sum");
    }
    double fl = 0.0, by = 0.0;
    if (slot != size_t(-1)) {
      std::unordered_set<const double*> seen;
      for (int b : active) {
        const taps_problem_t& p = probs[b];
        const double n = p.n[d], Rc = p.R_cols[d];
        const bool first = seen.insert(p.d_F[d]).second;
        fl += 2.0 * n * Rc * M;
        by += 8.0 * ((first ? n * Rc : 0.0) + Rc * M + n * M);
      }
    }
    return prof_end(h, slot, fl, by, st);
  };
  auto residual_parts = [&](int d, int nact, hipStream_t st) -> taps_status {
    residual_part_for(p0.s[d], M)<<<pgrid(kItRes, d, kPersistLds), 256, rlds, st>>>(d_prob, d_active, pref(kItRes, d),
                                                                       owner(kItRes, d), nact, d);
    TAPS_LAUNCHED(h, "kb_residual_part");
    return TAPS_OK;
  };

  // every launch of one sweep over the nact active problems (no host work)
  const uint32_t all = (1u << D) - 1u;
  auto one_sweep = [&](int nact, hipStream_t st) -> taps_status {
    uint32_t valid = 0;
    if (want_change) {
      kb_snapshot<<<nact, 256, 0, st>>>(d_bal, d_active);
      TAPS_LAUNCHED(h, "kb_snapshot");
    }
    for (int d = 0; d < D; ++d) {
      const uint32_t stale = (all & ~(1u << d)) & ~valid;
      for (int e = 0; e < D; ++e)
        if (stale & (1u << e)) TAPS_TRY(refresh(e, nact, st));
      valid |= stale;
      TAPS_TRY(system(d, nact, st));
      double fl = 0.0, by = 0.0;
      if (h->prof.on) {
        for (int b : active) {
          const taps_problem_t& p = probs[b];
          fl += use_fd[d] ? solve_fd_flops(p.n[d], M, p.s[d]) : solve_flops(p.n[d], M, 2 * p.s[d] + 1);
          by += use_fd[d] ? solve_fd_bytes(p.n[d], M, p.s[d]) : solve_bytes(p.n[d], M, 2 * p.s[d] + 1, p.n_kinds[d]);
        }
      }
      const void* d_args = base + o_args + size_t(d) * B * args_sz;
      TAPS_TRY(use_fd[d] ? fd_batched_launch(h, nact, d_args, d_active, M, p0.s[d], fl, by, st)
                         : solve_batched_launch(h, nact, d_args, d_active, M, p0.s[d], fl, by, st));
      valid &= ~(1u << d);
      TAPS_TRY(residual_parts(d, nact, st));
      kb_berr_final<<<cdiv(nact, 64), 64, 0, st>>>(d_prob, d_active, nact, d);
      TAPS_LAUNCHED(h, "kb_berr_final");
    }
    // the Grams still valid (every dim but the last solved) are rescaled with
    // the factors inside the balancing kernel; only the stale ones are recomputed
    kb_balance<<<nact, 256, 0, st>>>(d_bal, d_active, valid);
    TAPS_LAUNCHED(h, "kb_balance");
    kb_rescale_grams<<<dim3(unsigned(cdiv(rescale_len, 256L * kVB)), nact), 256, 0, st>>>(d_bal, d_active, valid);
    TAPS_LAUNCHED(h, "kb_rescale_grams");
    for (int e = 0; e < D; ++e)
      if (!(valid & (1u << e))) TAPS_TRY(refresh(e, nact, st));
    for (int d = 0; d < D; ++d) {
      TAPS_TRY(system(d, nact, st));
      TAPS_TRY(residual_parts(d, nact, st));
    }
    kb_residual_final<<<cdiv(nact, 64), 64, 0, st>>>(d_prob, d_active, nact);
    TAPS_LAUNCHED(h, "kb_residual_final");
    return TAPS_OK;
  };

  // graph mode: K sweeps captured once per launch layout, replayed on the
  // handle's own stream (the caller's stream may be the legacy null stream,
  // which cannot be captured); the uploads above were synchronised already
  const int K = h->prof.on ? 0 : h->tune.graph_sweeps;
  hipStream_t run = stream;
  if (K > 0) {
    if (!h->gstream) TAPS_HIP(h, hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
    run = h->gstream;
  }
  auto graph_for = [&](int nact, int k) -> taps_status {
    std::vector<int64_t> sig = {int64_t(reinterpret_cast<intptr_t>(base)), B, D, M, nact, k, int64_t(glds),
                                int64_t(rlds), Z.max_terms, lg_rows, int64_t(want_change)};
    for (long v : it_full) sig.push_back(v);
    for (int d = 0; d < D; ++d) {
      sig.push_back(p0.s[d] * 2 + use_fd[d]);
      for (int v : {Z.chunks[d], Z.ctiles[d], Z.splits[d], Z.gram[d], Z.lgram[d], Z.rblocks[d], Z.cpl[d], Z.wt[d],
                    Z.rchunks[d], Z.rc[d], int(long_groups[d]), Z.qlen[d], Z.fsplit[d], int(ident[d]), Z.wsl[d]})
        sig.push_back(v);
    }
    if (h->graph_exec && sig == h->graph_sig) return TAPS_OK;
    if (h->graph_exec) {
      TAPS_HIP(h, hipGraphExecDestroy(h->graph_exec));
      h->graph_exec = nullptr;
    }
    TAPS_HIP(h, hipStreamBeginCapture(run, hipStreamCaptureModeThreadLocal));
    taps_status st = TAPS_OK;
    for (int j = 0; j < k && st == TAPS_OK; ++j) st = one_sweep(nact, run);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(run, &graph);
    if (st != TAPS_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (ec != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, TAPS_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ec));
    }
    const hipError_t ei = hipGraphInstantiate(&h->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      (void)hipGetLastError();
      h->graph_exec = nullptr;
      return fail(h, TAPS_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    h->graph_sig = sig;
    return TAPS_OK;
  };

  std::vector<double> h_outs(size_t(B) * NO);
  std::vector<int> h_infos(size_t(B) * D);
  for (int it = 0; it < iter_max && !active.empty();) {
    const int nact = int(active.size());
    int k = 1;
    if (K > 0) {
      k = std::min(K, iter_max - it);
      TAPS_TRY(graph_for(nact, k));
      TAPS_HIP(h, hipGraphLaunch(h->graph_exec, run));
    } else {
      TAPS_TRY(one_sweep(nact, run));
    }
    it += k;
    TAPS_HIP(h, hipMemcpyAsync(h_outs.data(), outs, h_outs.size() * 8, hipMemcpyDeviceToHost, run));
    TAPS_HIP(h, hipMemcpyAsync(h_infos.data(), infos, h_infos.size() * 4, hipMemcpyDeviceToHost, run));
    TAPS_HIP(h, hipStreamSynchronize(run));
    next.clear();
    for (int b : active) {
      const double* o = h_outs.data() + size_t(b) * NO;
      bool broke = false;
      for (int d = 0; d < D; ++d)
        broke = broke || h_infos[size_t(b) * D + d] != 0 || !(o[D + 2 + d] <= TAPS_BERR_LIMIT);
      sweeps[b] = it;
      rho[b] = broke ? NAN : o[D + 1];
      const double chg = broke || !want_change ? NAN : o[2 * D + 2];
      if (change) change[b] = chg;
      if (!broke && rho[b] > tol && !(change_tol > 0.0 && chg <= change_tol)) next.push_back(b);
    }
    if (next.size() != active.size() && !next.empty()) {
      std::memcpy(act_h, next.data(), next.size() * 4);
      TAPS_HIP(h, hipMemcpyAsync(d_active, act_h, next.size() * 4, hipMemcpyHostToDevice, run));
      TAPS_TRY(upload_items(next, run));
    }
    active.swap(next);
  }
  return TAPS_OK;
}
