// Internal plumbing of the TAPS HIP library: handle, workspace, argument
// checks, launch helpers.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/taps.h"

// Grams and load Grams of one problem (per dim e: n_kinds[e] M^2 Grams, then
// R_cols[e] M load Grams) and which dims hold those of the current factors.
struct taps_gram_cache {
  double* base = nullptr;
  uint32_t valid = 0;
};

constexpr int kProfFamilies = 5;   // taps_prof_family values

struct taps_handle {
  // scratch: reused by every call (partial sums, solve factors, C/Q buffers)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // Gram cache of the single-problem calls
  double* cache = nullptr;
  size_t cache_bytes = 0;
  taps_gram_cache gc;
  // shape signature of the problem the cache belongs to
  int32_t sig_D = -1, sig_M = -1;
  int32_t sig_n[TAPS_MAX_DIMS] = {0}, sig_k[TAPS_MAX_DIMS] = {0}, sig_r[TAPS_MAX_DIMS] = {0};
  // driver region: C and Q of the dim being solved, residual partials, info words
  void* side = nullptr;
  size_t side_bytes = 0;
  // small fixed buffer: [0, 64) doubles residual output, then info words
  double* d_small = nullptr;
  // batched driver region (per-problem caches, couplings, solve workspaces)
  void* batch = nullptr;
  size_t batch_bytes = 0;
  // pinned host staging of the batched driver's per-call records, sent in one
  // copy; stage_ev is recorded after that copy and waited on before reuse
  void* stage = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t stage_ev = nullptr;
  std::string err;
  int device = 0;
  // tuning of the batched driver (taps_set_tuning / taps_autotune) and the
  // instantiated graph of its sweeps, reused while the launch layout holds
  taps_tuning_t tune{0};
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t gstream = nullptr;
  std::vector<int64_t> graph_sig;
  // kernel timing (taps_profile_*)
  struct Prof {
    std::vector<hipEvent_t> ev;    // start/stop pairs, reused
    std::vector<int> fam;          // family of each recorded pair
    size_t used = 0;               // pairs recorded since enable
    double flops[kProfFamilies] = {}, bytes[kProfFamilies] = {};
    bool on = false;
  } prof;
};

namespace taps {

inline taps_status fail(taps_handle* h, taps_status st, const char* fmt, ...) {
  if (h) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    h->err = buf;
  }
  return st;
}

#define TAPS_HIP(h, call)                                                               \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      (void)hipGetLastError(); /* clear the sticky error for later launches */         \
      return taps::fail((h), TAPS_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    }                                                                                  \
  } while (0)

#define TAPS_LAUNCHED(h, what)                                                          \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess)                                                              \
      return taps::fail((h), TAPS_ERR_HIP, "launch of %s failed: %s", what, hipGetErrorString(e_)); \
  } while (0)

#define TAPS_TRY(x)                    \
  do {                                 \
    taps_status st_ = (x);             \
    if (st_ != TAPS_OK) return st_;    \
  } while (0)

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Allow `bytes` of dynamic LDS for `kernel` (above 64 KB this must be opted in;
// the limit counts static LDS too, so ask for what the launch needs).
template <typename K>
inline taps_status allow_lds(taps_handle* h, K kernel, size_t bytes, size_t* have) {
  if (bytes <= *have || bytes <= 64 * 1024) return TAPS_OK;
  TAPS_HIP(h, hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  *have = bytes;
  return TAPS_OK;
}

// Pinned host staging of at least `need` bytes, free to overwrite: the last
// copy out of it has ended.
inline taps_status stage_reserve(taps_handle* h, size_t need) {
  if (!h->stage_ev) TAPS_HIP(h, hipEventCreateWithFlags(&h->stage_ev, hipEventDisableTiming));
  else TAPS_HIP(h, hipEventSynchronize(h->stage_ev));
  if (need <= h->stage_bytes) return TAPS_OK;
  if (h->stage) TAPS_HIP(h, hipHostFree(h->stage));
  h->stage = nullptr;
  h->stage_bytes = 0;
  const size_t bytes = align256(need + need / 4);
  if (hipHostMalloc(&h->stage, bytes, hipHostMallocDefault) != hipSuccess) {
    h->stage = nullptr;
    (void)hipGetLastError();
    return fail(h, TAPS_ERR_ALLOC, "hipHostMalloc of %zu bytes failed", bytes);
  }
  h->stage_bytes = bytes;
  return TAPS_OK;
}

// Grow a device buffer (synchronising `stream` first, since old contents may be in use).
inline taps_status grow(taps_handle* h, void** buf, size_t* have, size_t need, hipStream_t stream) {
  if (need <= *have) return TAPS_OK;
  TAPS_HIP(h, hipStreamSynchronize(stream));
  if (*buf) TAPS_HIP(h, hipFree(*buf));
  *buf = nullptr;
  *have = 0;
  size_t bytes = align256(need + need / 4);
  if (hipMalloc(buf, bytes) != hipSuccess) {
    *buf = nullptr;
    (void)hipGetLastError();
    return fail(h, TAPS_ERR_ALLOC, "hipMalloc of %zu bytes failed", bytes);
  }
  *have = bytes;
  return TAPS_OK;
}

inline taps_status need_ws(taps_handle* h, size_t bytes, hipStream_t stream) {
  return grow(h, &h->ws, &h->ws_bytes, bytes, stream);
}

// Bump allocator over the workspace (offsets only; 256-byte aligned).
struct Bump {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  }
};

inline int band_width(int s) { return 4 * s + 3; }
inline int half_band(int s) { return 2 * s + 1; }

inline int cdiv(long a, long b) { return static_cast<int>((a + b - 1) / b); }

// Global-memory view of a pointer.  Pointers read from argument records in
// memory are generic to the compiler, and generic (flat) accesses count
// against the LDS wait counter as well, so a kernel waiting on its LDS reads
// would also wait for every outstanding flat load and store.  Device bodies
// rebind their record pointers through gp() to get global accesses.
template <class T>
using gmem = T __attribute__((address_space(1)));
template <class T>
__device__ inline gmem<T>* gp(T* p) {
  return (gmem<T>*)p;
}

// ---- shared argument checks ------------------------------------------------
taps_status check_basis(taps_handle* h, const taps_basis1d_t* b);
taps_status check_problem(taps_handle* h, const taps_problem_t* p);

// ---- cross-file entry points (implemented in the .hip files) --------------
// Gram cache refresh for the dims in `mask`, given factors d_U.
taps_status refresh_grams(taps_handle* h, const taps_problem_t* p, taps_gram_cache* gc, uint32_t mask,
                          const double* const* d_U, hipStream_t stream);
// Offsets of dim e's Grams / load Grams inside h->cache.
size_t cache_gram_off(const taps_problem_t* p, int e);
size_t cache_lgram_off(const taps_problem_t* p, int e);
size_t cache_total(const taps_problem_t* p);
// Couplings + force of dim d from the cache (cache must be valid for e != d).
taps_status couple_and_force(taps_handle* h, const taps_problem_t* p, const taps_gram_cache* gc, int d,
                             double* d_C, double* d_Q, hipStream_t stream);
// Ensure the cache is sized and signed for problem p.
taps_status prepare_cache(taps_handle* h, const taps_problem_t* p, hipStream_t stream);

// Dim solve (block LU) and the per-chunk sums of R^2 / Q^2 of the dim-d
// system residual sum_k A^k U C^k^T - Q over free rows (2 doubles per chunk).
taps_status solve_dim_impl(taps_handle* h, const taps_problem_t* p, int d, const double* d_C,
                           const double* d_Q, double* d_X, int* d_info, double* d_berr, hipStream_t stream);
int dim_residual_nparts(int n);
taps_status dim_residual_parts(taps_handle* h, const taps_problem_t* p, int d, const double* d_C,
                               const double* d_U, const double* d_Q, double* parts, int* nparts,
                               hipStream_t stream);

// Batched dim solve: one workgroup per system (all systems share M and s).
size_t solve_args_bytes();
// Workspace of one batched dim solve (fd: fast diagonalisation, else block
// LU) and its device argument record.
size_t solve_ws_bytes(int n, int M, int s, bool fd);
void solve_args_fill(void* dst, const taps_problem_t* p, int d, const double* d_C, const double* d_Q,
                     double* d_X, int* d_info, void* ws, bool fd);
bool solve_batched_supported(int M, int s, int K);
// raises the kernel's LDS limit ahead of any launch (not allowed inside a capture)
taps_status solve_batched_prepare(taps_handle* h, int M, int s);
// Fast diagonalisation of two-kind dim systems (solver 1 of the tuning):
// applicability, algorithmic work, LDS set-up and the batched launch (eigen
// stage then banded stage, one workgroup per active system each).
bool solve_fd_supported(int M, int s, int K);
double solve_fd_flops(int n, int M, int s);
double solve_fd_bytes(int n, int M, int s);
taps_status fd_prepare(taps_handle* h, int M, int s);
taps_status fd_batched_launch(taps_handle* h, int n_active, const void* d_args, const int* d_active, int M, int s,
                              double flops, double bytes, hipStream_t stream);
taps_status solve_batched_launch(taps_handle* h, int n_active, const void* d_args, const int* d_active,
                                 int M, int s, double flops, double bytes, hipStream_t stream);
taps_status berr_final_launch(taps_handle* h, int nparts, const double* parts, double* out, hipStream_t stream);
double solve_flops(int n, int M, int w);
double solve_bytes(int n, int M, int w, int K);

// Device address of the allocation-free reconstruction's scratch on the
// handle's GPU (looked up once per GPU by taps_create).
taps_status recon_scratch_attach(taps_handle* h);
taps_status balance_launch(taps_handle* h, const taps_problem_t* p, double* const* d_U, hipStream_t stream);
taps_status residual_final_launch(taps_handle* h, int D, const int* nparts, double* const* parts, double* out,
                                  hipStream_t stream);

// Kernel timing helpers: bracket a launch with events when profiling is on.
taps_status prof_begin(taps_handle* h, int family, hipStream_t stream, size_t* slot);
taps_status prof_end(taps_handle* h, size_t slot, double flops, double bytes, hipStream_t stream);

// Host Gauss-Legendre rule on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, double* xi, double* w);

}  // namespace taps
