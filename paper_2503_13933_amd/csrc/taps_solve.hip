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

using taps::gmem;
using taps::gp;

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

__device__ inline bool is_fixed(const SolveArgs& A, int i) { return A.fixed && gp(A.fixed)[i]; }

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
// Matrix-core variant of the same block LU (same math, same window ring),
// 512 threads = 8 waves, four barriers per block row:
//  (A) build the entering row/column of blocks (couplings held in registers,
//      band coefficients prefetched into LDS during the previous row);
//  (B) stage the pivot block, the row panel [B_{k,k+1..k+wa} | b_k] and the
//      negated column panel in LDS (contiguous copies of the ring), then
//      invert the pivot block by Gauss-Jordan over all 512 threads (two LDS
//      buffers, one barrier per pivot);
//  (C) [Z | y] = P^-1 [row panel | b] in place on v_mfma_f64_16x16x4f64, one
//      16-column strip per wave (its B fragments are read before any write);
//  (D) window and right-hand sides += (-L) [Z | y] on the matrix cores, the
//      window values loaded before the MFMA chain and added after it.
// The row panel is stored K-major (contiguous along the 16-wide output index),
// the column panel row-major with an odd row stride; the inner index is padded
// to a multiple of 4 with zeros.  MFMA f64 16x16x4 lane
// layout: A[l%16][l/16], B[l/16][l%16], D[l/16 + 4i][l%16] (i = 0..3).
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kThreadsMfma = 512;
// kinds the matrix-core block LU holds couplings for in registers; systems
// with more kinds go to the vector kernel
constexpr int kLuKinds = 4;
constexpr int kMaxBlk = 2 * (2 * TAPS_MAX_S + 1) + 1;  // entering blocks per row

__device__ inline v4d mfma16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Quotient by a kernel-constant divisor through its float reciprocal: exact
// for 0 <= a < 2^20 and divisors <= 64 (the error of (a + 1/2)/d stays below
// 1/(2d)).
__device__ inline int fdiv(int a, float inv) { return int((float(a) + 0.5f) * inv); }

// Raw buffer resource over [base, base + bytes).  The address unit returns 0
// for loads and drops stores whose offset lies outside the range, so a lane
// with nothing to do is given kOOB instead of a branch: every wave then issues
// the same memory operations and the compiler waits on exact counts rather
// than draining the queue (vector loads and stores share one counter).
typedef unsigned int u32x2 __attribute__((__vector_size__(8)));
constexpr int kOOB = 0x7ffffff0;
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base, long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), 0x00020000);
}
__device__ inline double bload(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ inline void bstore(__amdgpu_buffer_rsrc_t r, int off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

// Gauss-Jordan inverse of an M x M block P by the whole workgroup.  S0 holds
// P row-major, which read column-major is P^T; the elimination runs on that
// array (every pivot reads one buffer and writes the other, so one barrier per
// pivot) and the last pivot stores its result transposed, which leaves P^-1
// column-major (S[j*M + i] = P^-1[i][j]) in S0 (M even) or S1 (M odd).  Each
// thread owns the entries t = tid + u*nt (i = t % M, j = t / M; indices of
// t >= M*M are clamped by the caller and their results discarded).  A pivot
// step is branch-free: all its reads are issued first, and every thread
// stores every entry (discarded ones to a sink), so no read is deferred into
// a predicated region.
template <int KE>
__device__ bool gj_block(int M, double* S0, double* S1, const int* ei, const int* ej) {
  __shared__ double sink;  // target of the discarded entries t >= M*M
  const int MM = M * M, tid = threadIdx.x, nt = blockDim.x;
  bool bad = false;
  double* cur = S0;
  double* nxt = S1;
  for (int r = 0; r < M; ++r) {
    const double p = cur[r * M + r];
    double aij[KE], air[KE], arj[KE];
#pragma unroll
    for (int u = 0; u < KE; ++u) {
      aij[u] = cur[ej[u] * M + ei[u]];
      air[u] = cur[r * M + ei[u]];
      arj[u] = cur[ej[u] * M + r];
    }
    bad = bad || !(fabs(p) > 0.0) || !isfinite(p);
    const double ip = 1.0 / p;
#pragma unroll
    for (int u = 0; u < KE; ++u) {
      const int i = ei[u], j = ej[u];
      double v = aij[u] - air[u] * (arj[u] * ip);
      v = (j == r) ? -air[u] * ip : v;
      v = (i == r) ? ((j == r) ? ip : aij[u] * ip) : v;
      *((tid + u * nt < MM) ? &nxt[r == M - 1 ? i * M + j : j * M + i] : &sink) = v;
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  return bad;
}

template <int MP>
__device__ void block_lu_mfma_body(const SolveArgs& A) {
  extern __shared__ double lds[];
  constexpr int kEnt = (MP * MP + kThreadsMfma - 1) / kThreadsMfma;
  constexpr int kStage = kEnt <= 2 ? 4 : 2;  // blocks staged per round of loads
  const int M = A.M, MM = M * M, w = 2 * A.s + 1, W1 = w + 1, n = A.n, wM = w * M, K = A.K;
  const int BW = 2 * w + 1;
  const int M4 = (M + 3) & ~3;
  const int P16 = ((wM + 1 + 15) / 16) * 16;
  const int R16 = ((wM + 15) / 16) * 16, LDL = M4 + 1;  // odd row stride: no bank conflicts
  double* Lp = lds;               // R16 x LDL: -(column panel), row-major
  double* Zp = Lp + R16 * LDL;    // M4 x P16: [row panel | b], K-major
  double* sG0 = Zp + M4 * P16;    // M x M  Gauss-Jordan buffers
  double* sG1 = sG0 + MM;         // M x M
  const double* sPinv = (M % 2 == 0) ? sG0 : sG1;  // where M pivots leave the inverse
  __shared__ double sCoef[kMaxBlk * kLuKinds];
  __shared__ double sQ[TAPS_MAX_M];
  __shared__ int sFixRow[2 * TAPS_MAX_S + 2];
  __shared__ int s_info;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
  const float invM = 1.0f / float(M), invW1 = 1.0f / float(W1);
  auto slot = [&](int i) { return i - fdiv(i, invW1) * W1; };
  // the window ring and the right-hand-side ring (which follows it in memory)
  // through one buffer resource, addressed by byte offsets
  const int rhs0 = int(A.rhs - A.win) * 8;
  const __amdgpu_buffer_rsrc_t rw = make_rsrc(A.win, long(rhs0) + long(W1) * M * 8);
  const __amdgpu_buffer_rsrc_t rfix = make_rsrc(A.fixed, A.fixed ? n : 0);
  auto woff = [&](int i, int j) { return (slot(i) * W1 + slot(j)) * MM * 8; };
  auto roff = [&](int i) { return rhs0 + slot(i) * M * 8; };
  auto fixed_at = [&](int i) { return int(__builtin_amdgcn_raw_buffer_load_b8(rfix, i, 0, 0)); };
  if (tid == 0) s_info = 0;
  // this thread's entries t = tid + u*nt of an M x M block: row-major row ej,
  // column ei (clamped for t >= M*M)
  int ei[kEnt], ej[kEnt];
#pragma unroll
  for (int u = 0; u < kEnt; ++u) {
    const int t = min(tid + u * nt, MM - 1);
    ej[u] = fdiv(t, invM);
    ei[u] = t - ej[u] * M;
  }
  // couplings at this thread's entries of an M x M block, zero for kinds
  // k >= K; loaded where blocks are built rather than held for the whole
  // kernel (the registers are needed by the update)
  auto load_couplings = [&](double (&cr)[kLuKinds][kEnt]) {
#pragma unroll
    for (int u = 0; u < kEnt; ++u) {
#pragma unroll
      for (int k = 0; k < kLuKinds; ++k) {
        const double c = A.C[long(min(k, K - 1)) * MM + ej[u] * M + ei[u]];
        cr[k][u] = (k < K) ? c : 0.0;
      }
    }
  };
  // zero the K-padding (columns M..M4-1 of Lp, rows M..M4-1 of Zp) and Lp's
  // tail rows once; they are never written afterwards
  for (int t = tid; t < R16 * LDL; t += nt) Lp[t] = 0.0;
  for (int t = tid; t < (M4 - M) * P16; t += nt) Zp[M * P16 + t] = 0.0;
  // block (i, j) of the original matrix, from coefficients cf[K] and the fixed
  // flags (bit 0: row i fixed -> identity or zero block, bit 1: column j fixed)
  // (cf holds kLuKinds values, zero beyond K, read once per block)
  auto build = [&](const double (&creg)[kLuKinds][kEnt], const double* cf, int fix, bool diag, int off) {
    double c[kLuKinds];
#pragma unroll
    for (int k = 0; k < kLuKinds; ++k) c[k] = cf[k];
#pragma unroll
    for (int u = 0; u < kEnt; ++u) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < kLuKinds; ++k) v += c[k] * creg[k][u];
      v = (fix & 2) ? 0.0 : v;
      v = (fix & 1) ? ((diag && ei[u] == ej[u]) ? 1.0 : 0.0) : v;
      const int t = tid + u * nt;
      bstore(rw, t < MM ? off + t * 8 : kOOB, v);
    }
  };
  // initial window rows/cols 0..min(w, n-1)
  {
    double creg[kLuKinds][kEnt];
    load_couplings(creg);
    const int hi = min(w, n - 1);
    for (int i = 0; i <= hi; ++i) {
      for (int j = 0; j <= hi; ++j) {
        double cf[kLuKinds];
#pragma unroll
        for (int k = 0; k < kLuKinds; ++k)
          cf[k] = (k < K) ? A.band[(long(k) * n + i) * BW + (j - i + w)] : 0.0;
        build(creg, cf, (fixed_at(i) ? 1 : 0) | (fixed_at(j) ? 2 : 0), i == j, woff(i, j));
      }
      const double q = fixed_at(i) ? 0.0 : A.Q[long(i) * M + min(tid, M - 1)];
      bstore(rw, tid < M ? roff(i) + tid * 8 : kOOB, q);
    }
  }
  // band coefficients, fixed flags of rows kn..kn+w and the load row of the
  // blocks entering at block row kn (row t = kn + w, columns kn..t, and column
  // t, rows kn..t-1): loaded early into registers, stored to LDS late
  // (thread tid loads coefficient kk = tid % kLuKinds of block
  // b = tid / kLuKinds, zero for kk >= K)
  struct Pre { double cf, q; int fx; };
  auto pre_issue = [&](int kn) {
    Pre pr{0.0, 0.0, 0};
    const int t = kn + w;
    if (t >= n || kn < 1) return pr;
    const int b = min(tid / kLuKinds, 2 * w), kk = tid % kLuKinds;
    const int i = (b <= w) ? t : kn + (b - w - 1);
    const int j = (b <= w) ? kn + b : t;
    const double cf = A.band[(long(min(kk, K - 1)) * n + i) * BW + (j - i + w)];
    pr.cf = (kk < K) ? cf : 0.0;
    pr.q = A.Q[long(t) * M + min(tid, M - 1)];
    pr.fx = fixed_at(kn + min(tid, w));
    return pr;
  };
  auto pre_commit = [&](int kn, const Pre& pr) {
    if (kn + w >= n || kn < 1) return;
    if (tid < (2 * w + 1) * kLuKinds) sCoef[tid] = pr.cf;
    if (tid < M) sQ[tid] = pr.q;
    if (tid <= w) sFixRow[tid] = pr.fx;
  };
  pre_commit(1, pre_issue(1));
  __syncthreads();

  for (int k = 0; k < n; ++k) {
    const int wa = min(w, n - 1 - k);
    const int waM = wa * M;
    // (A) entering blocks: row t = k + w (cols k..t) and column t (rows k..t-1)
    if (k > 0 && k + w < n) {
      const int t = k + w;
      double creg[kLuKinds][kEnt];
      load_couplings(creg);
      for (int b = 0; b < 2 * w + 1; ++b) {
        const int i = (b <= w) ? t : k + (b - w - 1);
        const int j = (b <= w) ? k + b : t;
        build(creg, sCoef + b * kLuKinds, (sFixRow[i - k] ? 1 : 0) | (sFixRow[j - k] ? 2 : 0), i == j,
              woff(i, j));
      }
      bstore(rw, tid < M ? roff(t) + tid * 8 : kOOB, sFixRow[w] ? 0.0 : sQ[min(tid, M - 1)]);
      __syncthreads();
    }
    // (B) stage the pivot block, the row panel [B_{k,k+1..} | b_k] and the
    // negated column panel (blocks b = 0 | 1..wa | wa+1..2wa), several
    // blocks' loads in flight per thread; then invert the pivot block
    {
      const int nb = 2 * wa + 1;
      for (int b0 = 0; b0 < nb; b0 += kStage) {
        double v[kStage][kEnt];
#pragma unroll
        for (int c = 0; c < kStage; ++c) {
          const int b = min(b0 + c, nb - 1);
          const int i = (b <= wa) ? k : k + b - wa;
          const int j = (b <= wa) ? k + b : k;
          const int off = woff(i, j);
#pragma unroll
          for (int u = 0; u < kEnt; ++u) v[c][u] = bload(rw, off + (ej[u] * M + ei[u]) * 8);
        }
#pragma unroll
        for (int c = 0; c < kStage; ++c) {
          const int b = b0 + c;
          if (b < nb) {
#pragma unroll
            for (int u = 0; u < kEnt; ++u) {
              if (tid + u * nt < MM) {
                const int r = ej[u], q = ei[u];
                if (b == 0) sG0[r * M + q] = v[c][u];
                else if (b <= wa) Zp[r * P16 + (b - 1) * M + q] = v[c][u];
                else Lp[((b - wa - 1) * M + r) * LDL + q] = -v[c][u];
              }
            }
          }
        }
      }
      const double bv = bload(rw, roff(k) + min(tid, M - 1) * 8);
      if (tid < M) Zp[tid * P16 + waM] = bv;
    }
    __syncthreads();
    if (gj_block<kEnt>(M, sG0, sG1, ei, ej) && tid == 0 && s_info == 0) s_info = k + 1;
    // (C) [Z | y] = P^-1 [row panel | b], in place, one 16-column strip per wave
    {
      const int ncol = waM + 1;
      const int strips = (ncol + 15) / 16, rtiles = (M + 15) / 16;
      const int ksteps = M4 / 4;
      const __amdgpu_buffer_rsrc_t rz = make_rsrc(A.Zst + long(k) * M * wM, long(M) * wM * 8);
      const __amdgpu_buffer_rsrc_t ry = make_rsrc(A.Yst + long(k) * M, long(M) * 8);
      for (int st = wave; st < strips; st += nwaves) {
        const int col = st * 16 + (lane & 15);
        double bf[MP / 4];
#pragma unroll
        for (int kk = 0; kk < MP / 4; ++kk)
          bf[kk] = (kk < ksteps) ? Zp[(4 * kk + (lane >> 4)) * P16 + col] : 0.0;
        // B fragments of this strip are in registers: rows of Zp may now be overwritten
#pragma unroll 1
        for (int tr = 0; tr < rtiles; ++tr) {
          const int ar = tr * 16 + (lane & 15);
          v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kk = 0; kk < MP / 4; ++kk) {
            const int kx = 4 * kk + (lane >> 4);
            const double a = (ar < M && kx < M) ? sPinv[kx * M + ar] : 0.0;
            acc = mfma16x16x4(a, bf[kk], acc);
          }
          // (elements copied out by name: indexing the accumulator vector in the
          // store loop is not reliably compiled)
          const double zv[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int q = tr * 16 + (lane >> 4) + 4 * i;
            if (q < M && col < ncol) Zp[q * P16 + col] = zv[i];
            bstore(rz, (q < M && col < waM) ? (q * wM + col) * 8 : kOOB, zv[i]);
            bstore(ry, (q < M && col == waM) ? q * 8 : kOOB, zv[i]);
          }
        }
      }
    }
    __syncthreads();
    // (D) window and right-hand sides += (-L) [Z | y]; the next block row's
    // coefficients and the window values of the wave's next tile are loaded
    // while the current tile's MFMA chain runs
    {
      const Pre pr = pre_issue(k + 1);
      const int trows = (waM + 15) / 16, tcols = (waM + 1 + 15) / 16;
      const int ntiles = trows * tcols;
      const int ksteps = M4 / 4;
      const float invTc = 1.0f / float(tcols);
      auto locate = [&](int T, int* o) {
        const int tr = fdiv(T, invTc);
        const int I0 = tr * 16, J0 = (T - tr * tcols) * 16;
        const int col = J0 + (lane & 15);
        const int jb = fdiv(col, invM), cc = col - jb * M;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = I0 + (lane >> 4) + 4 * i;
          const int bi = fdiv(row, invM), r = row - bi * M;
          const int ow = (col < waM) ? woff(k + 1 + bi, k + 1 + jb) + (r * M + cc) * 8 : roff(k + 1 + bi) + r * 8;
          o[i] = (T < ntiles && row < waM && col <= waM) ? ow : kOOB;
        }
      };
      // one tile: (-L)[Z | y] on the matrix cores, added to the window values
      // loaded one tile earlier
      auto tile = [&](int T, const int* o, const double* old) {
        const int I0 = fdiv(T, invTc) * 16, J0 = (T - fdiv(T, invTc) * tcols) * 16;
        const int col = J0 + (lane & 15);
        const int ar = I0 + (lane & 15);
        double af[MP / 4], bfr[MP / 4];
#pragma unroll
        for (int kk = 0; kk < MP / 4; ++kk) {
          const int kx = 4 * kk + (lane >> 4);
          af[kk] = (kk < ksteps) ? Lp[ar * LDL + kx] : 0.0;
          bfr[kk] = (kk < ksteps) ? Zp[kx * P16 + col] : 0.0;
        }
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < MP / 4; ++kk) acc = mfma16x16x4(af[kk], bfr[kk], acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) bstore(rw, o[i], old[i] + acc[i]);
      };
      // two register sets used alternately, so a prefetched value is never
      // copied (a copy would wait for the load)
      int oA[4], oB[4];
      double vA[4], vB[4];
      locate(wave, oA);
#pragma unroll
      for (int i = 0; i < 4; ++i) vA[i] = bload(rw, oA[i]);
      for (int T = wave; T < ntiles; T += 2 * nwaves) {
        locate(T + nwaves, oB);
#pragma unroll
        for (int i = 0; i < 4; ++i) vB[i] = bload(rw, oB[i]);
        tile(T, oA, vA);
        if (T + nwaves >= ntiles) break;
        locate(T + 2 * nwaves, oA);
#pragma unroll
        for (int i = 0; i < 4; ++i) vA[i] = bload(rw, oA[i]);
        tile(T + nwaves, oB, vB);
      }
      pre_commit(k + 1, pr);
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
      for (int J = jb; J < je; ++J) {
        const int bj = fdiv(J, invM);
        v += zrow[J] * sx[slot(k + 1 + bj) * M + (J - bj * M)];
      }
      spart[part * M + m] = v;
    }
    __syncthreads();
    for (int m = tid; m < M; m += nt) {
      double v = A.Yst[long(k) * M + m];
      for (int part = 0; part < parts; ++part) v -= spart[part * M + m];
      sx[slot(k) * M + m] = v;
      A.X[long(k) * M + m] = v;
    }
    __syncthreads();
  }
  if (tid == 0) A.info[0] = s_info;
}

#define TAPS_FOR_MP(X) X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64)

#define TAPS_LU_KERNELS(MP)                                                                          \
  __global__ __launch_bounds__(kThreadsMfma) void k_block_lu_mfma_##MP(SolveArgs A) {                \
    block_lu_mfma_body<MP>(A);                                                                       \
  }                                                                                                  \
  __global__ __launch_bounds__(kThreadsMfma) void k_block_lu_mfma_batched_##MP(                      \
      const SolveArgs* __restrict__ args, const int* __restrict__ active) {                          \
    const SolveArgs A = args[active[blockIdx.x]];                                                    \
    block_lu_mfma_body<MP>(A);                                                                       \
  }
TAPS_FOR_MP(TAPS_LU_KERNELS)

inline int mp_of(int M) { return ((M + 7) / 8) * 8; }

typedef void (*lu_single_fn)(SolveArgs);
typedef void (*lu_batched_fn)(const SolveArgs*, const int*);

lu_single_fn lu_single_for(int M) {
  switch (mp_of(M)) {
#define TAPS_CASE(MP) case MP: return k_block_lu_mfma_##MP;
    TAPS_FOR_MP(TAPS_CASE)
#undef TAPS_CASE
  }
  return nullptr;
}

lu_batched_fn lu_batched_for(int M) {
  switch (mp_of(M)) {
#define TAPS_CASE(MP) case MP: return k_block_lu_mfma_batched_##MP;
    TAPS_FOR_MP(TAPS_CASE)
#undef TAPS_CASE
  }
  return nullptr;
}

size_t lu_mfma_lds_allowed[9] = {0};
size_t lu_mfma_batched_lds_allowed[9] = {0};


constexpr int kResRows = taps::dev::kResRows;


// Per chunk of kResRows rows: R = sum_k A^k U (C^k)^T - Q on the chunk, and the
// chunk's sums of R^2 and Q^2 over free rows -> part[2*block], part[2*block+1]
// (matrix-core body shared with the batched driver).
__global__ __launch_bounds__(256) void k_residual_part(int n, int M, int s, int K, const double* __restrict__ band,
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

// ---------------------------------------------------------------------------
// Fast diagonalisation of a dim system with two 1D matrix kinds (the paper's
// own solver, Sec. 2.6):  A1 X C1^T + A2 X C2^T = Q.  Right-multiplying by
// C1^{-T} gives A1 X + A2 X E = Q C1^{-T} with E = C2^T C1^{-T}.  With the
// complex Schur form E = Z T Z^H and the eigenvectors of T (T Wv = Wv diag(l),
// Wv unit upper triangular), P = Z Wv diagonalises E, and Y = X P decouples
// into M banded systems (A1 + l_m A2) y_m = (Q C1^{-T} P)_m; X = Re(Y P^{-1})
// with P^{-1} = Wv^{-1} Z^H.
//   k_fd_inverse, k_fd_schur, k_fd_vectors (one wave per system for the
//              Schur kernel, four for the other two):
//              C1^{-1} by Gauss-Jordan with partial pivoting and E; Householder
//              Hessenberg form and Francis double-shift QR to the real Schur
//              form (Z accumulated); complex Schur form, Wv and Wv^{-1} by
//              substitution; writes H2 = C1^{-T} Z Wv, H3 = Wv^{-1} Z^H and l
//              to the workspace.
//   k_fd_solve (one workgroup per system): R = Q H2, the M banded complex
//              systems (one lane each; elimination without pivoting over a
//              (w+1)-row window in LDS, U rows kept for back substitution),
//              X = Re(Y H3).  Fixed rows are identity rows with zero right-hand
//              side and zero columns.
// Workspace (doubles, from A.Zst): H2 2M^2 | H3 2M^2 | l 2M | C1inv M^2 |
// T M^2 | Z M^2 | Y 2nM | U store 2 M n (w+1).
struct cplx {
  double r, i;
};
__device__ inline cplx cmk(double r, double i) { return cplx{r, i}; }
__device__ inline cplx cadd(cplx a, cplx b) { return cplx{a.r + b.r, a.i + b.i}; }
__device__ inline cplx csub(cplx a, cplx b) { return cplx{a.r - b.r, a.i - b.i}; }
__device__ inline cplx cmul(cplx a, cplx b) { return cplx{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ inline cplx cconj(cplx a) { return cplx{a.r, -a.i}; }
__device__ inline cplx cscale(cplx a, double s) { return cplx{a.r * s, a.i * s}; }
__device__ inline double cabs2(cplx a) { return hypot(a.r, a.i); }
// Complex array in global memory (real and imaginary parts adjacent):
// entries read as cplx and assigned from cplx through global accesses.
struct GCplx {
  gmem<double>* p;
  struct Ref {
    gmem<double>* q;
    __device__ operator cplx() const { return cplx{q[0], q[1]}; }
    __device__ const Ref& operator=(cplx v) const {
      q[0] = v.r;
      q[1] = v.i;
      return *this;
    }
  };
  __device__ Ref operator[](long i) const { return Ref{p + 2 * i}; }
  __device__ GCplx operator+(long i) const { return GCplx{p + 2 * i}; }
};

// a - l b in four fused multiply-adds
__device__ inline cplx cfms(cplx a, cplx l, cplx b) {
  return cplx{fma(-l.r, b.r, fma(l.i, b.i, a.r)), fma(-l.r, b.i, fma(-l.i, b.r, a.i))};
}
__device__ inline cplx cdivz(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.r) >= fabs(b.i)) {
    const double t = b.i / b.r, d = b.r + b.i * t;
    return cplx{(a.r + a.i * t) / d, (a.i - a.r * t) / d};
  }
  const double t = b.r / b.i, d = b.i + b.r * t;
  return cplx{(a.r * t + a.i) / d, (a.i * t - a.r) / d};
}
__device__ inline cplx csqrtz(cplx z) {
  const double m = cabs2(z);
  double r = sqrt(0.5 * (m + fabs(z.r)));
  if (r == 0.0) return cplx{0.0, 0.0};
  if (z.r >= 0.0) return cplx{r, z.i / (2.0 * r)};
  return cplx{fabs(z.i) / (2.0 * r), z.i >= 0.0 ? r : -r};
}

// largest M of the fast diagonalisation; kernels are instantiated for
// M <= kFdSmallM (the layouts and register tiles of the common sizes) and
// for M <= kFdMaxM
constexpr int kFdSmallM = 48;
constexpr int kFdMaxM = 64;

// Workspace of one fast-diagonalisation solve (inside the first workspace
// region): H2 = C1^{-T} P and H3 = P^{-1} (M x M complex), the eigenvalues
// (M complex), C1^{-1}, E (then the real Schur form T) and the Schur
// vectors Z (M x M each), the right-hand sides / solutions of the
// banded systems (n x M complex, row-major) and their U rows
// (n x (w+1) x M complex).
struct FdWs {
  gmem<double> *H2, *H3, *lam, *C1inv, *T, *Zq, *Y, *U;
};
__device__ inline FdWs fd_ws(const SolveArgs& A) {
  const int M = A.M, MM = M * M;
  FdWs f;
  f.H2 = gp(A.Zst);
  f.H3 = f.H2 + 2 * MM;
  f.lam = f.H3 + 2 * MM;
  f.C1inv = f.lam + 2 * M;
  f.T = f.C1inv + MM;
  f.Zq = f.T + MM;
  f.Y = f.Zq + MM;
  f.U = f.Y + 2 * long(A.n) * M;
  return f;
}

// |re| + |im|: the cheap modulus of the deflation and shift tests.
__device__ inline double cabs1(cplx a) { return fabs(a.r) + fabs(a.i); }
__device__ inline cplx crecip(cplx a) {
  const double id = 1.0 / (a.r * a.r + a.i * a.i);
  return cplx{a.r * id, -a.i * id};
}

// Complex Givens rotation [c s; -conj(s) c] [f; g] = [r; 0], c real:
// c = |f| / r, s = f conj(g) / (|f| r), r = sqrt(|f|^2 + |g|^2), from one
// reciprocal square root of |f|^2 r^2.  Operands of extreme magnitude are
// rescaled first.
__device__ inline void cgivens(cplx f, cplx g, double& c, cplx& s) {
  double f2 = f.r * f.r + f.i * f.i, g2 = g.r * g.r + g.i * g.i;
  if (g2 == 0.0) {
    c = 1.0;
    s = cmk(0.0, 0.0);
    return;
  }
  if (f2 == 0.0) {
    c = 0.0;
    s = cscale(cconj(g), rsqrt(g2));
    return;
  }
  double p = f2 * (f2 + g2);
  if (!(p > 1e-280 && p < 1e280)) {
    const double is = 1.0 / fmax(cabs1(f), cabs1(g));
    f = cscale(f, is);
    g = cscale(g, is);
    f2 = f.r * f.r + f.i * f.i;
    g2 = g.r * g.r + g.i * g.i;
    p = f2 * (f2 + g2);
  }
  const double t = rsqrt(p);
  c = f2 * t;
  s = cscale(cmul(f, cconj(g)), t);
}

// Walk of the M x M index space by one lane of a 64-wide wave: t = lane,
// lane + 64, ... as (row, column) without integer division in the loop.
struct IjWalk {
  int i, j, q, r;
  __device__ IjWalk(int lane, int M, int stride = 64) : i(lane / M), j(lane % M), q(stride / M), r(stride % M) {}
  __device__ void next(int M) {
    i += q;
    j += r;
    if (j >= M) {
      j -= M;
      ++i;
    }
  }
};
// nthr threads (one wave by default) read the row-major M x M matrices
// srcs[0..N) (element t = i M + j)
// and hands entry (i, j) of each to put(i, j, values); sixteen entries per lane
// are loaded before the first is handed on, so the loads' latencies overlap.
template <int N, class Src, class Put>
__device__ inline void stage_square(int M, int lane, const Src* const (&srcs)[N], Put put, int nthr = 64) {
  constexpr int kU = 16;
  const int MM = M * M;
  IjWalk w(lane, M, nthr);
  for (int t0 = lane; t0 < MM; t0 += nthr * kU) {
    double v[kU][N];
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int a = 0; a < N; ++a) v[u][a] = srcs[a][min(t0 + nthr * u, MM - 1)];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (t0 + nthr * u < MM) put(w.i, w.j, v[u]);
      w.next(M);
    }
  }
}

// Eigen stage of the fast diagonalisation for one dim system with two kinds,
// in three kernels of one 64-lane wave per system (split so that the long
// real phases hold little LDS and four systems share a compute unit; the
// inverse and vectors kernels run four waves per system, which share their
// dense products while one wave takes the column-serial parts):
//   inverse: C1^{-1} by Gauss-Jordan with partial pivoting, E = C2^T C1^{-T}
//     (the system becomes A1 X + A2 X E = Q C1^{-T}) to the workspace;
//   schur: Householder reduction of E to Hessenberg form and Francis
//     double-shift QR in real arithmetic to the real Schur form (at most
//     40 M iterations), T and Z to the workspace;
//   vectors: unitary 2 x 2 rotations of the complex-pair blocks to the
//     complex Schur form E = Z T Z^H, eigenvectors Wv of T (unit upper
//     triangular), so P = Z Wv; H2 = C1^{-T} P and H3 = P^{-1} = Wv^{-1} Z^H
//     to the workspace, with the eigenvalues.
// LDS in M x L real units (L = M rounded up to odd, so that column walks over
// the lanes hit distinct banks): inverse 2 (the Gauss-Jordan iterate, in
// place, and C2), schur 2 (Hr, Zr; at the largest M of the layout), vectors 6
// (complex H, Wv, Z; C1^{-1} at the end).
// info word: 0, -1 (C1 singular) or -2 (no convergence); a later kernel
// skips a system whose info is set.
// Orders the LDS accesses of one wave for the compiler.  A workgroup of one
// wave needs no hardware barrier: its LDS accesses complete in issue order.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// sqrt(q), q > 0 and normal: the hardware reciprocal square root estimate,
// one Goldschmidt step for sqrt(q) and 1/(2 sqrt(q)) together, then two
// Newton corrections of the square root.
__device__ inline double nr_sqrt(double q) {
  const double r = __builtin_amdgcn_rsq(q);
  double g = q * r, hh = 0.5 * r;
  const double e = fma(-hh, g, 0.5);
  g = fma(g, e, g);
  hh = fma(hh, e, hh);
  double d = fma(-g, g, q);
  g = fma(d, hh, g);
  d = fma(-g, g, q);
  return fma(d, hh, g);
}
// 1/d, d normal: the hardware reciprocal estimate and two Newton steps.
__device__ inline double nr_rcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

constexpr int kVecThreads = 256;   // the inverse and eigenvector kernels: four waves per system

__device__ void fd_eig_inverse(const SolveArgs& A) {
  extern __shared__ double lds[];
  // four waves per system: Gauss-Jordan on the first (lane = column), the
  // staging and the product E on all of them
  constexpr int NT = kVecThreads;
  const int M = A.M, MM = M * M, L = M | 1, LL = M * L, lane = threadIdx.x;
  double* S0 = lds;                                   // unit 0
  double* C2s = lds + LL;                             // unit 1
  __shared__ int perm[64];
  __shared__ int s_fail;
  const FdWs f = fd_ws(A);
  if (lane == 0) s_fail = 0;
  {
    const auto Cg = gp(A.C);
    const gmem<double>* const src[2] = {Cg, Cg + MM};
    stage_square(M, lane, src, [&](int i, int j, const double* v) {
      S0[i * L + j] = v[0];
      C2s[i * L + j] = v[1];
    }, NT);
  }
  __syncthreads();
  // ---- C1^{-1}: Gauss-Jordan with partial pivoting (row swaps, undone as
  // column swaps at the end), in place: lane j rewrites its column j from
  // its own entries and column r; every batch of rows is read by all lanes
  // (one instruction for the wave) before any lane stores it, and lane r's
  // stores to column r only reach rows the other lanes have read already
  double* cur = S0;
  for (int r = 0; r < M; ++r) {
    // pivot: largest |cur[i][r]|, i >= r (first on ties), by a wave reduction
    double bv = (lane >= r && lane < M) ? fabs(cur[lane * L + r]) : -1.0;
    int bi = lane;
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o);
      const int oi = __shfl_xor(bi, o);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    const int p = bi;
    if (lane == 0) {
      perm[r] = p;
      if (!(bv > 0.0) || !isfinite(bv)) s_fail = 1;
    }
    if (p != r && lane < M) {
      const double t = cur[r * L + lane];
      cur[r * L + lane] = cur[p * L + lane];
      cur[p * L + lane] = t;
    }
    __syncthreads();
    if (lane < M) {   // column lane of the next iterate, rows in batches of 8
      const int j = lane;
      const double ip = 1.0 / cur[r * L + r];
      const double arj = cur[r * L + j] * ip;
      // new entry = alpha a_ij + beta a_ir off the pivot row, rowv on it
      // (column r: -a_ir / p and 1 / p; other columns: a_ij - a_ir a_rj / p
      // and a_rj / p), with per-lane coefficients so the loop has no branches
      const double alpha = (j == r) ? 0.0 : 1.0;
      const double beta = (j == r) ? -ip : -arj;
      const double rowv = (j == r) ? ip : arj;
      for (int i0 = 0; i0 < M; i0 += 8) {
        double aa[8], ar[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {   // clamped rows: every load in bounds, issued together
          const int i = min(i0 + u, M - 1);
          aa[u] = cur[i * L + j];
          ar[u] = cur[i * L + r];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u;
          const double v = (i == r) ? rowv : fma(beta, ar[u], alpha * aa[u]);
          if (i < M) cur[i * L + j] = v;
        }
      }
    }
    __syncthreads();
  }
  for (int r = M - 1; r >= 0; --r) {   // undo the row swaps as column swaps
    const int p = perm[r];
    if (p != r && lane < M) {
      const double t = cur[lane * L + r];
      cur[lane * L + r] = cur[lane * L + p];
      cur[lane * L + p] = t;
    }
    __syncthreads();
  }
  const double* Ci = cur;   // C1^{-1}, kept for E and saved for H2
  {
    IjWalk w(lane, M, NT);
    for (int t = lane; t < MM; t += NT, w.next(M)) f.C1inv[t] = Ci[w.i * L + w.j];
  }
  // ---- E[i][j] = sum_q C2[q][i] C1inv[j][q] to the workspace
  {
    IjWalk w(lane, M, NT);
    for (int t = lane; t < MM; t += NT, w.next(M)) {
      const int i = w.i, j = w.j;
      double e = 0.0;
#pragma unroll 8
      for (int q = 0; q < M; ++q) e += C2s[q * L + i] * Ci[j * L + q];
      f.T[t] = e;
    }
  }
  if (lane == 0) A.info[0] = s_fail ? -1 : 0;
}

// (the Schur kernel's LDS layout is fixed at the largest M of its
// instantiation, MAXM: row stride MAXM + 1 (odd) and Zr at a fixed offset,
// so that every row and column offset of the bulge chase is an immediate of
// the LDS instructions)
constexpr int schur_l(int maxm) { return maxm | 1; }
// the sink takes the three stores of each lane a pass leaves alone: row pass
// at lane + {0, L, 2L}, column passes at 3 lane + {0, 1, 2}
constexpr int schur_sink(int maxm) { return 2 * schur_l(maxm) + 64 > 3 * 64 ? 2 * schur_l(maxm) + 64 : 3 * 64; }
template <int MAXM>
__device__ void fd_eig_schur(const SolveArgs& A) {
  extern __shared__ double lds[];
  const int M = A.M, MM = M * M, lane = threadIdx.x;
  constexpr int L = schur_l(MAXM);
  double* Hr = lds;                                   // MAXM x L
  double* Zr = lds + MAXM * L;                        // MAXM x L
  double* Dm = lds + 2 * MAXM * L;                    // schur_sink: stores of lanes a chase step leaves alone
  __shared__ int s_fail;
  const FdWs f = fd_ws(A);
  if (A.info[0] != 0) return;
  if (lane == 0) s_fail = 0;
  {
    const gmem<double>* const src[1] = {f.T};
    stage_square(M, lane, src, [&](int i, int j, const double* v) {
      Hr[i * L + j] = v[0];
      Zr[i * L + j] = (i == j) ? 1.0 : 0.0;
    });
  }
  wave_sync();
  // ---- Householder Hessenberg form, Zr accumulated.  The rows (left) and
  // columns (right) past k are read once into registers in batches of 8
  // (static, at most MAXM / 8 batches; clamped entries weigh 0), all
  // loads before the first use, and updated from there.
  constexpr int kHB = MAXM / 8;
  for (int k = 0; k + 2 < M; ++k) {
    // the Householder vector, in registers of every lane: column k below the
    // diagonal read by all lanes (one address per load, a broadcast), rows
    // past M - 1 zero; its norm from four partial sums
    double vv[kHB][8];
    double sq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < kHB; ++b) {
      const int i0 = k + 1 + 8 * b;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double xv = (i0 < M) ? Hr[min(i0 + u, M - 1) * L + k] : 0.0;
        vv[b][u] = (i0 + u < M) ? xv : 0.0;
        sq[u & 3] = fma(vv[b][u], vv[b][u], sq[u & 3]);
      }
    }
    const double ss = (sq[0] + sq[1]) + (sq[2] + sq[3]);
    if (ss == 0.0) continue;
    const double x0 = vv[0][0];
    const double nx = sqrt(ss);
    const double alpha = x0 >= 0.0 ? -nx : nx;
    vv[0][0] = x0 - alpha;
    const double beta = 1.0 / (nx * (nx + fabs(x0)));   // 2 / |v|^2, |v|^2 = 2 nx (nx + |x0|)
    if (lane < M) {   // left: column lane, rows k+1..
      double hv[kHB][8];
#pragma unroll
      for (int b = 0; b < kHB; ++b) {
        const int i0 = k + 1 + 8 * b;
        if (i0 < M) {
#pragma unroll
          for (int u = 0; u < 8; ++u) hv[b][u] = Hr[min(i0 + u, M - 1) * L + lane];
        }
      }
      double ws[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int b = 0; b < kHB; ++b) {
        const int i0 = k + 1 + 8 * b;
        if (i0 < M) {
#pragma unroll
          for (int u = 0; u < 8; ++u) ws[u & 3] = fma(vv[b][u], hv[b][u], ws[u & 3]);
        }
      }
      const double bw = beta * ((ws[0] + ws[1]) + (ws[2] + ws[3]));
#pragma unroll
      for (int b = 0; b < kHB; ++b) {
        const int i0 = k + 1 + 8 * b;
        if (i0 < M) {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (i0 + u < M) Hr[(i0 + u) * L + lane] = hv[b][u] - vv[b][u] * bw;
        }
      }
    }
    wave_sync();
    if (lane < M) {   // right: row lane, columns k+1.. (Hr and Zr)
      double hv[kHB][8], zv[kHB][8];
#pragma unroll
      for (int b = 0; b < kHB; ++b) {
        const int j0 = k + 1 + 8 * b;
        if (j0 < M) {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int j = min(j0 + u, M - 1);
            hv[b][u] = Hr[lane * L + j];
            zv[b][u] = Zr[lane * L + j];
          }
        }
      }
      double us[2] = {0.0, 0.0}, zs[2] = {0.0, 0.0};
#pragma unroll
      for (int b = 0; b < kHB; ++b) {
        const int j0 = k + 1 + 8 * b;
        if (j0 < M) {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            us[u & 1] = fma(hv[b][u], vv[b][u], us[u & 1]);
            zs[u & 1] = fma(zv[b][u], vv[b][u], zs[u & 1]);
          }
        }
      }
      const double bu = beta * (us[0] + us[1]), buz = beta * (zs[0] + zs[1]);
#pragma unroll
      for (int b = 0; b < kHB; ++b) {
        const int j0 = k + 1 + 8 * b;
        if (j0 < M) {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (j0 + u < M) {
              Hr[lane * L + j0 + u] = hv[b][u] - bu * vv[b][u];
              Zr[lane * L + j0 + u] = zv[b][u] - buz * vv[b][u];
            }
          }
        }
      }
    }
    wave_sync();
  }
  // ---- real Schur form by Francis double-shift QR (two shifts per sweep,
  // the eigenvalues of the trailing 2 x 2 block, or an exceptional pair every
  // 10 iterations on one eigenvalue); 3-element Householder reflectors chase
  // the bulge, rows on the column lanes and columns (of Hr and Zr) on the row
  // lanes.  A deflated 2 x 2 block with real eigenvalues is rotated to upper
  // triangular form; one with complex eigenvalues stays.
  // reflector (I - tau u u^T), u = (1, u1, u2), applied to rows k.. of Hr
  // (columns c0..M-1) and to columns k.. of Hr (rows 0..r1) and of Zr;
  // returns this lane's new Hr[lane][k] (rows <= r1)
  auto reflect = [&](int k, int len, double tau, double u1, double u2, int c0, int r1) -> double {
    if (lane >= c0 && lane < M) {
      const double h0 = Hr[k * L + lane], h1 = Hr[(k + 1) * L + lane];
      const double h2 = len == 3 ? Hr[(k + 2) * L + lane] : 0.0;
      const double w = tau * (h0 + u1 * h1 + u2 * h2);
      Hr[k * L + lane] = h0 - w;
      Hr[(k + 1) * L + lane] = h1 - w * u1;
      if (len == 3) Hr[(k + 2) * L + lane] = h2 - w * u2;
    }
    wave_sync();
    double col = 0.0;
    if (lane <= r1) {
      const double h0 = Hr[lane * L + k], h1 = Hr[lane * L + k + 1];
      const double h2 = len == 3 ? Hr[lane * L + k + 2] : 0.0;
      const double w = tau * (h0 + u1 * h1 + u2 * h2);
      col = h0 - w;
      Hr[lane * L + k] = col;
      Hr[lane * L + k + 1] = h1 - w * u1;
      if (len == 3) Hr[lane * L + k + 2] = h2 - w * u2;
    }
    if (lane < M) {
      const double z0 = Zr[lane * L + k], z1 = Zr[lane * L + k + 1];
      const double z2 = len == 3 ? Zr[lane * L + k + 2] : 0.0;
      const double w = tau * (z0 + u1 * z1 + u2 * z2);
      Zr[lane * L + k] = z0 - w;
      Zr[lane * L + k + 1] = z1 - w * u1;
      if (len == 3) Zr[lane * L + k + 2] = z2 - w * u2;
    }
    wave_sync();
    return col;
  };
  // Householder vector of (x, y, z): (I - tau u u^T)(x, y, z)^T = (beta, 0, 0)^T,
  // tau = (beta - x) / beta and u = (1, y, z) / (x - beta) from one reciprocal
  // (norm and reciprocal by Newton iterations from the hardware estimates:
  // no range scaling, the entries are far from under- and overflow).  With
  // y = z = 0 the reflector is the identity (tau = 0); that case is a select
  // on a harmless stand-in norm, not a branch.
  auto house = [](double x, double y, double z, double& tau, double& u1, double& u2) {
    const bool ident = y == 0.0 && z == 0.0;
    const double q = ident ? 1.0 : x * x + y * y + z * z;
    const double nrm = nr_sqrt(q);
    const double beta = x >= 0.0 ? -nrm : nrm;
    const double xb = x - beta;   // |xb| >= nrm > 0
    const double inv = nr_rcp(beta * xb);
    const double sc = beta * inv;
    tau = ident ? 0.0 : -xb * xb * inv;
    u1 = ident ? 0.0 : y * sc;
    u2 = ident ? 0.0 : z * sc;
  };
  // a double held by lane l, to every lane (l wave-uniform)
  auto from_lane = [](double x, int l) -> double {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane(int(b), l), hi = __builtin_amdgcn_readlane(int(b >> 32), l);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
  };
  int hi = M - 1, it = 0, total = 0;
  const int limit = 40 * M;
  while (hi >= 0 && total < limit) {
    // lo: the largest i <= hi whose subdiagonal entry is negligible (0 if none)
    bool neg = false;
    if (lane >= 1 && lane <= hi)
      neg = fabs(Hr[lane * L + lane - 1]) <=
            2.220446049250313e-16 * (fabs(Hr[lane * L + lane]) + fabs(Hr[(lane - 1) * L + lane - 1]));
    const unsigned long long bal = __ballot(neg);
    const int lo = bal ? 63 - __clzll(bal) : 0;
    wave_sync();
    if (lo > 0 && lane == 0) Hr[lo * L + lo - 1] = 0.0;
    if (lo == hi) {
      --hi;
      it = 0;
      wave_sync();
      continue;
    }
    if (lo == hi - 1) {
      // 2 x 2 block: rotate to triangular form when its eigenvalues are real
      const double a = Hr[(hi - 1) * L + hi - 1], b = Hr[(hi - 1) * L + hi], c = Hr[hi * L + hi - 1],
                   d = Hr[hi * L + hi];
      const double p = 0.5 * (a - d), disc = p * p + b * c;
      wave_sync();
      if (disc >= 0.0) {
        const double sq = sqrt(disc);
        const double lam = 0.5 * (a + d) + (p >= 0.0 ? sq : -sq);
        double e0 = b, e1 = lam - a;   // eigenvector of lam, the better conditioned form
        const double f0 = lam - d, f1 = c;
        if (e0 * e0 + e1 * e1 < f0 * f0 + f1 * f1) {
          e0 = f0;
          e1 = f1;
        }
        const double en = sqrt(e0 * e0 + e1 * e1);
        if (en > 0.0) {
          const double cs = e0 / en, sn = e1 / en;   // G = [cs -sn; sn cs]: H <- G^T H G
          const int k = hi - 1;
          if (lane >= k && lane < M) {
            const double h0 = Hr[k * L + lane], h1 = Hr[(k + 1) * L + lane];
            Hr[k * L + lane] = cs * h0 + sn * h1;
            Hr[(k + 1) * L + lane] = cs * h1 - sn * h0;
          }
          wave_sync();
          if (lane <= hi) {
            const double h0 = Hr[lane * L + k], h1 = Hr[lane * L + k + 1];
            Hr[lane * L + k] = cs * h0 + sn * h1;
            Hr[lane * L + k + 1] = cs * h1 - sn * h0;
          }
          if (lane < M) {
            const double z0 = Zr[lane * L + k], z1 = Zr[lane * L + k + 1];
            Zr[lane * L + k] = cs * z0 + sn * z1;
            Zr[lane * L + k + 1] = cs * z1 - sn * z0;
          }
          wave_sync();
          if (lane == 0) Hr[hi * L + hi - 1] = 0.0;
        }
      }
      hi -= 2;
      it = 0;
      wave_sync();
      continue;
    }
    ++it;
    ++total;
    double h11, h12, h21, h22;
    if (it % 10 == 0) {   // exceptional shifts
      const double sx = fabs(Hr[hi * L + hi - 1]) + fabs(Hr[(hi - 1) * L + hi - 2]);
      h11 = 0.75 * sx + Hr[hi * L + hi];
      h12 = -0.4375 * sx;
      h21 = sx;
      h22 = h11;
    } else {
      h11 = Hr[(hi - 1) * L + hi - 1];
      h12 = Hr[(hi - 1) * L + hi];
      h21 = Hr[hi * L + hi - 1];
      h22 = Hr[hi * L + hi];
    }
    const double s = h11 + h22, t = h11 * h22 - h12 * h21;
    const double a00 = Hr[lo * L + lo], a01 = Hr[lo * L + lo + 1], a10 = Hr[(lo + 1) * L + lo],
                 a11 = Hr[(lo + 1) * L + lo + 1], a21 = Hr[(lo + 2) * L + lo + 1];
    double x = a00 * a00 + a01 * a10 - s * a00 + t;
    double y = a10 * (a00 + a11 - s);
    double z = a10 * a21;
    // after the reflector at k, the next bulge column (rows k+1..k+3 of
    // column k) sits in registers of lanes k+1..k+3
    for (int k = lo; k + 1 < hi; ++k) {
      // One step of the chase: the reflector acts on rows k..k+2 (one column
      // per lane) and then on columns k..k+2 (rows 0..r1 of Hr and all rows
      // of Zr, one row per lane).  The row operands and Zr are read before
      // the reflector is known, so those loads overlap its computation; the
      // column operands are read after the row pass has stored (one wave:
      // its LDS accesses complete in issue order), and the Zr pass fills that
      // wait.  Loads run on every lane (lanes past M on row / column M - 1).
      // Every lane stores too: a lane outside a pass (row pass: columns
      // c0..M-1; column pass: rows 0..r1; Zr: rows 0..M-1) stores into the
      // sink, so the step has no branch, and a reflector that is the identity
      // (tau = 0) stores the values it read.
      const int c0 = max(lo, k - 1), r1 = min(k + 3, hi);
      const int lm = min(lane, M - 1);
      const double a0 = Hr[k * L + lm], a1 = Hr[(k + 1) * L + lm], a2 = Hr[(k + 2) * L + lm];
      const double z0 = Zr[lm * L + k], z1 = Zr[lm * L + k + 1], z2 = Zr[lm * L + k + 2];
      double tau, u1, u2;
      house(x, y, z, tau, u1, u2);
      {
        const double w = tau * (a0 + u1 * a1 + u2 * a2);
        double* const p = (lane >= c0 && lane < M) ? Hr + k * L + lane : Dm + lane;
        p[0] = a0 - w;
        p[L] = a1 - w * u1;
        p[2 * L] = a2 - w * u2;
      }
      const double h0 = Hr[lm * L + k], h1 = Hr[lm * L + k + 1], h2 = Hr[lm * L + k + 2];
      {
        const double w = tau * (z0 + u1 * z1 + u2 * z2);
        double* const p = lane < M ? Zr + lane * L + k : Dm + 3 * lane;
        p[0] = z0 - w;
        p[1] = z1 - w * u1;
        p[2] = z2 - w * u2;
      }
      const double w = tau * (h0 + u1 * h1 + u2 * h2);
      const double col = h0 - w;
      {
        double* const p = lane <= r1 ? Hr + lane * L + k : Dm + 3 * lane;
        p[0] = col;
        p[1] = h1 - w * u1;
        p[2] = h2 - w * u2;
      }
      // the next bulge column: rows k+1..k+3 of column k (k + 3 <= hi + 1 <= M)
      x = from_lane(col, k + 1);
      y = from_lane(col, k + 2);
      const double z3 = from_lane(col, k + 3);
      z = (k + 3 <= hi) ? z3 : 0.0;
      wave_sync();
    }
    {
      const int k = hi - 1;
      double tau, u1, u2;
      house(x, y, 0.0, tau, u1, u2);
      wave_sync();
      if (tau != 0.0) reflect(k, 2, tau, u1, 0.0, max(lo, k - 1), hi);
    }
  }
  if (hi >= 0 && lane == 0) s_fail = 2;
  wave_sync();
  {
    IjWalk w(lane, M);
    for (int t = lane; t < MM; t += 64, w.next(M)) {
      f.T[t] = (w.i > w.j + 1) ? 0.0 : Hr[w.i * L + w.j];   // rounding residue below the subdiagonal dropped
      f.Zq[t] = Zr[w.i * L + w.j];
    }
  }
  if (lane == 0 && s_fail) A.info[0] = -2;
}

// ZG: Z lives in the workspace (the right-hand-side region, free until the
// banded stage) instead of LDS, for M whose six LDS units do not fit; the
// lanes of one wave see each other's global stores in issue order.
template <bool ZG>
__device__ void fd_eig_vectors(const SolveArgs& A) {
  extern __shared__ double lds[];
  // four waves per system: the lanes past the first wave take no row or
  // column of their own (they reach the barriers) and share the dense products
  constexpr int NT = kVecThreads;
  const int M = A.M, MM = M * M, L = M | 1, LL = M * L, lane = threadIdx.x;
  cplx* H = reinterpret_cast<cplx*>(lds);            // units 0-1
  cplx* Wv = reinterpret_cast<cplx*>(lds + 2 * LL);   // units 2-3
  const FdWs f = fd_ws(A);
  using ZPtr = typename std::conditional<ZG, GCplx, cplx*>::type;
  ZPtr Z;                                             // units 4-5, or the workspace
  if constexpr (ZG)
    Z = GCplx{f.Y};
  else
    Z = reinterpret_cast<cplx*>(lds + 4 * LL);
  if (A.info[0] != 0) return;
  // ---- complex Schur form: H = Hr, Z = Zr, then each remaining 2 x 2 block
  // (complex eigenvalue pair) is triangularised by a unitary rotation whose
  // first column is the block's eigenvector for mu
  {
    const gmem<double>* const src[2] = {f.T, f.Zq};
    stage_square(M, lane, src, [&](int i, int j, const double* v) {
      H[i * L + j] = cmk(v[0], 0.0);
      Z[i * L + j] = cmk(v[1], 0.0);
    }, NT);
  }
  __syncthreads();
  for (int k = 0; k + 1 < M; ++k) {
    const cplx c = H[(k + 1) * L + k];
    if (c.r == 0.0 && c.i == 0.0) continue;
    const cplx a = H[k * L + k], b = H[k * L + k + 1], d = H[(k + 1) * L + k + 1];
    const cplx tr = cadd(a, d), det = csub(cmul(a, d), cmul(b, c));
    const cplx mu = cadd(cscale(tr, 0.5), csqrtz(csub(cscale(cmul(tr, tr), 0.25), det)));
    cplx e0 = b, e1 = csub(mu, a);
    const cplx f0 = csub(mu, d), f1 = c;
    if (cabs1(e0) + cabs1(e1) < cabs1(f0) + cabs1(f1)) {
      e0 = f0;
      e1 = f1;
    }
    const double en = rsqrt(e0.r * e0.r + e0.i * e0.i + e1.r * e1.r + e1.i * e1.i);
    const cplx g0 = cscale(e0, en), g1 = cscale(e1, en);   // G = [g0 -conj(g1); g1 conj(g0)]
    __syncthreads();
    if (lane >= k && lane < M) {   // rows k, k+1 <- G^H rows
      const cplx h0 = H[k * L + lane], h1 = H[(k + 1) * L + lane];
      H[k * L + lane] = cadd(cmul(cconj(g0), h0), cmul(cconj(g1), h1));
      H[(k + 1) * L + lane] = csub(cmul(g0, h1), cmul(g1, h0));
    }
    __syncthreads();
    if (lane <= k + 1) {           // columns k, k+1 <- columns G
      const cplx h0 = H[lane * L + k], h1 = H[lane * L + k + 1];
      H[lane * L + k] = cadd(cmul(h0, g0), cmul(h1, g1));
      H[lane * L + k + 1] = csub(cmul(h1, cconj(g0)), cmul(h0, cconj(g1)));
    }
    if (lane < M) {
      const cplx z0 = Z[lane * L + k], z1 = Z[lane * L + k + 1];
      Z[lane * L + k] = cadd(cmul(z0, g0), cmul(z1, g1));
      Z[lane * L + k + 1] = csub(cmul(z1, cconj(g0)), cmul(z0, cconj(g1)));
    }
    __syncthreads();
    if (lane == 0) H[(k + 1) * L + k] = cmk(0.0, 0.0);
    __syncthreads();
    ++k;   // the next subdiagonal entry is zero
  }
  // ---- eigenvectors Wv of T (unit upper triangular), one column per lane
  if (lane < M) {
    const int k = lane;
    const cplx tk = H[k * L + k];
    double tn = 0.0;
    for (int i = 0; i <= k; ++i) tn = fmax(tn, cabs1(H[i * L + i]));
    const double small = 2.220446049250313e-16 * fmax(tn, 1e-300);
    for (int i = 0; i < M; ++i) Wv[i * L + k] = cmk(i == k ? 1.0 : 0.0, 0.0);
    for (int i = k - 1; i >= 0; --i) {
      cplx sacc = cmk(0.0, 0.0);
      for (int j = i + 1; j <= k; ++j) sacc = cadd(sacc, cmul(H[i * L + j], Wv[j * L + k]));
      cplx den = csub(H[i * L + i], tk);
      if (cabs1(den) < small) den = cmk(small, 0.0);
      Wv[i * L + k] = cmul(sacc, cscale(crecip(den), -1.0));
    }
    f.lam[2 * k] = tk.r;
    f.lam[2 * k + 1] = tk.i;
  }
  __syncthreads();
  // ---- Winv = Wv^{-1} (unit upper triangular) into H (T no longer needed)
  if (lane < M) {
    const int j = lane;
    for (int i = 0; i < M; ++i) H[i * L + j] = cmk(i == j ? 1.0 : 0.0, 0.0);
    for (int i = j - 1; i >= 0; --i) {
      cplx sacc = cmk(0.0, 0.0);
      for (int k2 = i + 1; k2 <= j; ++k2) sacc = cadd(sacc, cmul(Wv[i * L + k2], H[k2 * L + j]));
      H[i * L + j] = cscale(sacc, -1.0);
    }
  }
  __syncthreads();
  // ---- H3 = Winv Z^H  (H3[m][q] = sum_j Winv[m][j] conj(Z[q][j]))
  {
    IjWalk w(lane, M, NT);
    for (int t = lane; t < MM; t += NT, w.next(M)) {
      const int m = w.i, q = w.j;
      cplx sacc = cmk(0.0, 0.0);
      for (int j = m; j < M; ++j) sacc = cadd(sacc, cmul(H[m * L + j], cconj(Z[q * L + j])));
      f.H3[2 * t] = sacc.r;
      f.H3[2 * t + 1] = sacc.i;
    }
  }
  __syncthreads();
  // ---- ZW = Z Wv into H, then H2 = C1inv^T ZW (H2[q][m] = sum_j C1inv[j][q] ZW[j][m])
  {
    IjWalk w(lane, M, NT);
    for (int t = lane; t < MM; t += NT, w.next(M)) {
      const int i = w.i, m = w.j;
      cplx sacc = cmk(0.0, 0.0);
      for (int j = 0; j <= m; ++j) sacc = cadd(sacc, cmul(Z[i * L + j], Wv[j * L + m]));
      H[i * L + m] = sacc;
    }
  }
  __syncthreads();
  double* Ci2 = lds + 2 * LL;   // C1^{-1} back from the workspace (Wv is dead)
  {
    const gmem<double>* const src[1] = {f.C1inv};
    stage_square(M, lane, src, [&](int i, int j, const double* v) { Ci2[i * L + j] = v[0]; }, NT);
  }
  __syncthreads();
  {
    IjWalk w(lane, M, NT);
    for (int t = lane; t < MM; t += NT, w.next(M)) {
      const int q = w.i, m = w.j;
      cplx sacc = cmk(0.0, 0.0);
      for (int j = 0; j < M; ++j) sacc = cadd(sacc, cscale(H[j * L + m], Ci2[j * L + q]));
      f.H2[2 * t] = sacc.r;
      f.H2[2 * t + 1] = sacc.i;
    }
  }
}

// dst[t] = (src[2t], src[2t+1]) for t < n, by nt threads with sixteen loads in flight each
__device__ inline void stage_cplx(cplx* dst, const gmem<double>* src, int n, int tid, int nt) {
  constexpr int kU = 16;
  for (int t0 = tid; t0 < n; t0 += nt * kU) {
    double re[kU], im[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int t = min(t0 + nt * u, n - 1);
      re[u] = src[2 * t];
      im[u] = src[2 * t + 1];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (t0 + nt * u < n) dst[t0 + nt * u] = cmk(re[u], im[u]);
  }
}
constexpr int kFdThreads = 64;   // one wave: transforms, staging and elimination
// the register-window back substitution forms X itself (its H3 operands held
// in registers) up to the 48-mode layout
template <int MAXM> constexpr bool kFuseOut = MAXM <= 48;

// Banded complex solves (A1 + lambda_m A2) y_m = r_m of the fast
// diagonalisation with the elimination window in registers: lane m owns
// system m and keeps rows k..k+w, columns k..k+w of its partly reduced matrix
// (a (w+1)^2 ring indexed by row and column modulo w+1, so the unrolled steps
// address it statically) plus the right-hand sides of those rows.  Band rows
// (A1, A2 pairs, shared by the M systems) go through a three-chunk LDS ring:
// the wave loads chunk c+2 into registers before eliminating chunk c and
// stores it to LDS after.  The right-hand side entering at step k is loaded
// w+1 steps ahead.  Each step stores row k divided by its pivot: the w upper
// entries (the U row, layout [row][entry][system] so stores and loads are
// coalesced over systems) and the reduced right-hand side; back substitution
// walks the rows upwards with the U rows loaded a few rows ahead and needs no
// division.  Rows beyond n are identity rows, so the last steps need no
// guards.  No pivoting: a zero pivot sets the info word.  One 64-lane wave
// per system set: the elimination is bound by its own instruction stream and
// the U stores, so one wave per SIMD is the useful occupancy.
template <int MAXM, int W>
__device__ void fd_banded_reg(const SolveArgs& A, const FdWs& f, const cplx* sLam, double2* ring, int* s_info) {
  constexpr int W1 = W + 1, BW = 2 * W + 1, CH = W1 * (32 / W1);
  constexpr int SPL = (CH * BW + 63) / 64;   // staged entries per lane and chunk
  const int n = A.n, M = A.M, tid = threadIdx.x, m = tid;
  const auto b1 = gp(A.band);
  const auto b2 = b1 + long(n) * BW;
  const GCplx Yg{f.Y}, Ug{f.U};
  // staged (a1, a2) of band row i, offset o (column i - W + o), with fixed
  // rows (identity), fixed and out-of-range columns (zero) applied
  auto band_pair = [&](int c, int t) -> double2 {
    const int i = c * CH + t / BW, o = t % BW, j = i - W + o;
    double2 v = make_double2(0.0, 0.0);
    if (t >= CH * BW) return v;
    if (i >= n || is_fixed(A, i)) {
      v.x = (o == W) ? 1.0 : 0.0;
    } else if (j >= 0 && j < n && !is_fixed(A, j)) {
      v = make_double2(b1[long(i) * BW + o], b2[long(i) * BW + o]);
    }
    return v;
  };
  auto stage_store = [&](int c, const double2* v) {
    double2* dst = ring + (c % 3) * CH * BW;
#pragma unroll
    for (int u = 0; u < SPL; ++u)
      if (tid + 64 * u < CH * BW) dst[tid + 64 * u] = v[u];
  };
  const int nchunks = (n + W) / CH + 1;   // rows up to n + W are read
  double2 sv[SPL];
#pragma unroll
  for (int u = 0; u < SPL; ++u) sv[u] = band_pair(0, tid + 64 * u);
  stage_store(0, sv);
  if (nchunks > 1) {
#pragma unroll
    for (int u = 0; u < SPL; ++u) sv[u] = band_pair(1, tid + 64 * u);
    stage_store(1, sv);
  }
  __syncthreads();
  const bool act = m < M;
  const cplx lam = act ? sLam[m] : cmk(0.0, 0.0);
  auto E = [&](int i, int o) -> cplx {
    const double2 v = ring[((i / CH) % 3 * CH + i % CH) * BW + o];
    return cmk(v.x + lam.r * v.y, lam.i * v.y);
  };
  auto rhs_at = [&](int i) -> cplx { return i < n ? Yg[long(i) * M + m] : cmk(0.0, 0.0); };
  cplx win[W1][W1], rhs[W1], rnext[W1];
  if (act) {
#pragma unroll
    for (int r = 0; r < W1; ++r) {
#pragma unroll
      for (int c = 0; c < W1; ++c) win[r][c] = E(r, c - r + W);
      rhs[r] = rhs_at(r);
      rnext[r] = rhs_at(r + W1);
    }
  }
  int info = 0;
  // ---- forward elimination, one chunk of CH rows per barrier
  for (int c = 0; c * CH < n; ++c) {
    const bool more = c + 2 < nchunks;
    if (more) {   // loads of chunk c+2, consumed after this chunk's steps
#pragma unroll
      for (int u = 0; u < SPL; ++u) sv[u] = band_pair(c + 2, tid + 64 * u);
    }
    if (act) {
      for (int k0 = c * CH; k0 < (c + 1) * CH && k0 < n; k0 += W1) {
#pragma unroll
        for (int p = 0; p < W1; ++p) {
          const int k = k0 + p;
          if (k < n) {
            const cplx piv = win[p][p];
            const double d = piv.r * piv.r + piv.i * piv.i;
            if (!(d > 0.0) || !(d < INFINITY)) info = info ? info : k + 1;
            const cplx inv = cscale(cconj(piv), nr_rcp(d));
            // row k divided by its pivot (the w upper entries and the reduced
            // right-hand side); the rows below subtract their column-k entry
            // times it, which needs no multiplier per row
            cplx urow[W1];
#pragma unroll
            for (int cc = 1; cc < W1; ++cc) urow[cc] = cmul(inv, win[p][(p + cc) % W1]);
            const cplx yk = cmul(inv, rhs[p]);
#pragma unroll
            for (int r = 1; r < W1; ++r) {
              const int rs = (p + r) % W1;
              const cplx l = win[rs][p];
#pragma unroll
              for (int cc = 1; cc < W1; ++cc) {
                const int cs = (p + cc) % W1;
                win[rs][cs] = cfms(win[rs][cs], l, urow[cc]);
              }
              rhs[rs] = cfms(rhs[rs], l, yk);
            }
            const GCplx u = Ug + (long(k) * W * M + m);
#pragma unroll
            for (int cc = 1; cc < W1; ++cc) u[long(cc - 1) * M] = urow[cc];
            Yg[long(k) * M + m] = yk;
            // slot p now takes row k + W1 (columns k+1 .. k+W1) and column
            // k + W1 (rows k+1 .. k+W)
            const int i = k + W1;
#pragma unroll
            for (int cc = 1; cc <= W1; ++cc) win[p][(p + cc) % W1] = E(i, cc - 1);
#pragma unroll
            for (int r = 1; r < W1; ++r) win[(p + r) % W1][p] = E(k + r, 2 * W + 1 - r);
            rhs[p] = rnext[p];
            rnext[p] = rhs_at(k + 2 * W1);
          }
        }
      }
    }
    if (more) stage_store(c + 2, sv);
    __syncthreads();
  }
  if (act && info) atomicCAS(s_info, 0, info);
  if constexpr (kFuseOut<MAXM>) {
  // ---- back substitution: y_k = yhat_k - sum_c U[k][c] y_{k+c} (row k
  // already divided by its pivot), fused with the transform out: the rows of
  // y go to a ring of two 16-row tiles in LDS (the band ring is dead by now)
  // and each completed tile becomes 16 rows of X = Re(Y H3) on the matrix
  // cores, so y never returns to global memory.  The U rows and reduced
  // right-hand sides are loaded PF rows ahead (a ring of PF row buffers, PF
  // dividing w+1, so slots stay static in the unrolled groups).  Lanes past M
  // follow mode M-1 without storing: the tile products need the whole wave.
  const int MM = M * M;
  cplx* sH = reinterpret_cast<cplx*>(ring);
  stage_cplx(sH, f.H3, MM, tid, 64);
  __syncthreads();
  constexpr int kKS = MAXM / 4, kCT = (MAXM + 15) / 16;
  const int lane = tid, nct = (M + 15) / 16, ksteps = (M + 3) / 4;
  double hr[kCT][kKS], hi[kCT][kKS];
#pragma unroll
  for (int c = 0; c < kCT; ++c) {
    const int mb = c * 16 + (lane & 15);
#pragma unroll
    for (int u = 0; u < kKS; ++u) {
      const int q = 4 * u + (lane >> 4);
      const cplx hb = (u < ksteps && c < nct && q < M && mb < M) ? sH[q * M + mb] : cmk(0.0, 0.0);
      hr[c][u] = hb.r;
      hi[c][u] = hb.i;
    }
  }
  __syncthreads();
  cplx* ytile = sH;   // [2][16][M]
  const auto Xg = gp(A.X);
  auto flush = [&](int t) {   // rows 16t .. 16t+15 of X from tile slot t & 1
    const cplx* yt = ytile + (t & 1) * 16 * M;
    const int ia = t * 16 + (lane & 15);
    const bool row_ok = ia < n && !is_fixed(A, ia);
    double yr[kKS], yi[kKS];
#pragma unroll
    for (int u = 0; u < kKS; ++u) {
      const int mm = 4 * u + (lane >> 4);
      const cplx v = (row_ok && u < ksteps && mm < M) ? yt[(lane & 15) * M + mm] : cmk(0.0, 0.0);
      yr[u] = v.r;
      yi[u] = -v.i;
    }
    v4d ar[kCT], ai[kCT];
#pragma unroll
    for (int c = 0; c < kCT; ++c) ar[c] = ai[c] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < kKS; ++u) {
#pragma unroll
      for (int c = 0; c < kCT; ++c) {
        if (u < ksteps && c < nct) {   // (guards, not loop exits: the loops stay fully unrolled)
          ar[c] = mfma16x16x4(yr[u], hr[c][u], ar[c]);
          ai[c] = mfma16x16x4(yi[u], hi[c][u], ai[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kCT; ++c) {
      const int qb = c * 16 + (lane & 15);
      const v4d x = ar[c] + ai[c];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = t * 16 + (lane >> 4) + 4 * j;
        if (c < nct && i < n && qb < M) Xg[long(i) * M + qb] = x[j];
      }
    }
  };
  {
    const int me = act ? m : M - 1;
    constexpr int PF = W1 / 2 > 0 ? W1 / 2 : 1;
    static_assert(W1 % PF == 0, "prefetch ring must divide the group");
    cplx ub[PF][W], yh[PF], yw[W1];
#pragma unroll
    for (int p = 0; p < W1; ++p) yw[p] = cmk(0.0, 0.0);
#pragma unroll
    for (int j = 1; j <= PF; ++j) {   // rows n-1 .. n-PF into slots k % PF
      const int k = n - j;
      if (k >= 0) {
#pragma unroll
        for (int q = 0; q < PF; ++q)
          if (k % PF == q) {
#pragma unroll
            for (int cc = 0; cc < W; ++cc) ub[q][cc] = Ug[(long(k) * W + cc) * M + me];
            yh[q] = Yg[long(k) * M + me];
          }
      }
    }
    const int gtop = (n - 1) / W1;
    int tp = (n - 1) >> 4;   // the highest tile not yet turned into X
    for (int g = gtop; g >= 0; --g) {
#pragma unroll
      for (int p = W1 - 1; p >= 0; --p) {
        const int k = g * W1 + p;
        if (k < n) {
          const int q = p % PF;
          cplx acc = yh[q];
#pragma unroll
          for (int cc = 1; cc < W1; ++cc) acc = cfms(acc, ub[q][cc - 1], yw[(p + cc) % W1]);
          const cplx y = acc;
          yw[p] = y;
          if (act) ytile[(((k >> 4) & 1) * 16 + (k & 15)) * M + m] = y;
          if (k - PF >= 0) {
#pragma unroll
            for (int cc = 0; cc < W; ++cc) ub[q][cc] = Ug[(long(k - PF) * W + cc) * M + me];
            yh[q] = Yg[long(k - PF) * M + me];
          }
        }
      }
      // every row from g W1 up is done: tiles starting at or above it are complete
      while (tp >= 0 && 16 * tp >= g * W1) {
        wave_sync();
        flush(tp);
        --tp;
      }
    }
  }
  } else {
    // (64-mode layout: y back to global memory, transformed afterwards)
    if (act) {
      constexpr int PF = W1 / 2 > 0 ? W1 / 2 : 1;
      static_assert(W1 % PF == 0, "prefetch ring must divide the group");
      cplx ub[PF][W], yh[PF], yw[W1];
#pragma unroll
      for (int p = 0; p < W1; ++p) yw[p] = cmk(0.0, 0.0);
#pragma unroll
      for (int j = 1; j <= PF; ++j) {
        const int k = n - j;
        if (k >= 0) {
#pragma unroll
          for (int q = 0; q < PF; ++q)
            if (k % PF == q) {
#pragma unroll
              for (int cc = 0; cc < W; ++cc) ub[q][cc] = Ug[(long(k) * W + cc) * M + m];
              yh[q] = Yg[long(k) * M + m];
            }
        }
      }
      const int gtop = (n - 1) / W1;
      for (int g = gtop; g >= 0; --g) {
#pragma unroll
        for (int p = W1 - 1; p >= 0; --p) {
          const int k = g * W1 + p;
          if (k < n) {
            const int q = p % PF;
            cplx acc = yh[q];
#pragma unroll
            for (int cc = 1; cc < W1; ++cc) acc = cfms(acc, ub[q][cc - 1], yw[(p + cc) % W1]);
            const cplx y = acc;
            yw[p] = y;
            Yg[long(k) * M + m] = y;
            if (k - PF >= 0) {
#pragma unroll
              for (int cc = 0; cc < W; ++cc) ub[q][cc] = Ug[(long(k - PF) * W + cc) * M + m];
              yh[q] = Yg[long(k - PF) * M + m];
            }
          }
        }
      }
    }
  }
}

template <int MAXM>
__device__ __attribute__((always_inline)) void fd_solve_body(const SolveArgs& A) {
  extern __shared__ double lds[];
  const int M = A.M, MM = M * M, n = A.n, w = 2 * A.s + 1, BW = 2 * w + 1, W1 = w + 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  // LDS: the eigenvalues, then one region used in turn by H2 (transform
  // in), the staged band chunks (register window) or per-system row rings
  // (other patch sizes), and H3 (transform out)
  cplx* sLam = reinterpret_cast<cplx*>(lds);    // M
  cplx* win = sLam + M;
  cplx* sH = win;                                // M x M, H2 then H3
  const FdWs f = fd_ws(A);
  __shared__ int s_info;
  if (tid == 0) s_info = 0;
  if (A.info[0] != 0) return;   // the eigen stage failed: leave its code
  for (int m = tid; m < M; m += nt) sLam[m] = cmk(f.lam[2 * m], f.lam[2 * m + 1]);
  stage_cplx(sH, f.H2, MM, tid, nt);
  __syncthreads();
  const GCplx Y{f.Y};   // n x M
  const GCplx U{f.U};   // M x n x (w+1)
  const auto Qg = gp(A.Q);
  const auto Xg = gp(A.X);
  // ---- R = Q H2 (fixed rows zero) on the matrix cores: per 16-row tile
  // (tiles dealt to the waves) the Q operands of every step are loaded once
  // for all mode tiles, and the next tile's operands are loaded before this
  // tile's products; real and imaginary parts in two accumulators sharing
  // the Q operand (lane l: row l%16, q = 4kk + l/16).  The H2 operands are
  // the same for every row tile: they sit in registers for the whole
  // transform, and each mode tile has its own accumulators, so the products
  // of one step are independent of each other.
  constexpr int kKS = MAXM / 4, kCT = (MAXM + 15) / 16;
  const int wave = tid >> 6, lane = tid & 63, nwv = nt >> 6;
  const int nrt = (n + 15) / 16, nct = (M + 15) / 16, ksteps = (M + 3) / 4;
  // operand u of mode tile c (lane l: mode 16 c + l%16, q = 4 u + l/16) of an
  // M x M complex matrix in LDS; zero outside
  auto b_operands = [&](double (*br)[kKS], double (*bi)[kKS]) {
#pragma unroll
    for (int c = 0; c < kCT; ++c) {
      const int mb = c * 16 + (lane & 15);
#pragma unroll
      for (int u = 0; u < kKS; ++u) {
        const int q = 4 * u + (lane >> 4);
        const cplx hb = (u < ksteps && c < nct && q < M && mb < M) ? sH[q * M + mb] : cmk(0.0, 0.0);
        br[c][u] = hb.r;
        bi[c][u] = hb.i;
      }
    }
  };
  {
    double an[kKS];
    auto load_q = [&](int tr, double* dst) {
      const int ia = tr * 16 + (lane & 15);
      const int ic = min(ia, n - 1);
#pragma unroll
      for (int u = 0; u < kKS; ++u) {
        const int q = 4 * u + (lane >> 4);
        dst[u] = (u < ksteps && q < M) ? Qg[long(ic) * M + q] : 0.0;
      }
    };
    if (wave < nrt) load_q(wave, an);
    double hr[kCT][kKS], hi[kCT][kKS];
    b_operands(hr, hi);
    for (int tr = wave; tr < nrt; tr += nwv) {
      double av[kKS];
      const int ia = tr * 16 + (lane & 15);
      const bool row_ok = ia < n && !is_fixed(A, ia);
#pragma unroll
      for (int u = 0; u < kKS; ++u) av[u] = row_ok ? an[u] : 0.0;
      if (tr + nwv < nrt) load_q(tr + nwv, an);
      v4d are[kCT], aim[kCT];
#pragma unroll
      for (int c = 0; c < kCT; ++c) are[c] = aim[c] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < kKS; ++u) {
#pragma unroll
        for (int c = 0; c < kCT; ++c) {
          if (u < ksteps && c < nct) {   // (guards, not loop exits: the loops stay fully unrolled)
            are[c] = mfma16x16x4(av[u], hr[c][u], are[c]);
            aim[c] = mfma16x16x4(av[u], hi[c][u], aim[c]);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < kCT; ++c) {
        const int mb = c * 16 + (lane & 15);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int i = tr * 16 + (lane >> 4) + 4 * j;
          if (c < nct && i < n && mb < M) Y[long(i) * M + mb] = cmk(are[c][j], aim[c][j]);
        }
      }
    }
  }
  __syncthreads();
  // ---- banded systems (A1 + l_m A2) y = r
  if (w == 5 || w == 3 || w == 1) {
    double2* ring = reinterpret_cast<double2*>(win);
    if (w == 5) fd_banded_reg<MAXM, 5>(A, f, sLam, ring, &s_info);
    if (w == 3) fd_banded_reg<MAXM, 3>(A, f, sLam, ring, &s_info);
    if (w == 1) fd_banded_reg<MAXM, 1>(A, f, sLam, ring, &s_info);
  } else if (tid < M) {   // any patch size: one lane per system, ring of rows in LDS
    const auto b1 = gp(A.band);
    const auto b2 = b1 + long(n) * BW;
    const int m = tid;
    const cplx lam = sLam[m];
    cplx* wr = win + long(m) * W1 * BW;   // ring of w+1 rows, entry c <-> column (row - w + c)
    auto entry = [&](int i, int j) -> cplx {   // original matrix entry, fixed rows/cols applied
      if (j < 0 || j >= n || j < i - w || j > i + w) return cmk(0.0, 0.0);
      const bool fi = is_fixed(A, i), fj = is_fixed(A, j);
      if (fi) return cmk(i == j ? 1.0 : 0.0, 0.0);
      if (fj) return cmk(0.0, 0.0);
      const double a1 = b1[long(i) * BW + (j - i + w)], a2 = b2[long(i) * BW + (j - i + w)];
      return cmk(a1 + lam.r * a2, lam.i * a2);
    };
    auto load_row = [&](int i) {
      cplx* row = wr + (i % W1) * BW;
      for (int c = 0; c < BW; ++c) row[c] = entry(i, i - w + c);
    };
    for (int i = 0; i < min(W1, n); ++i) load_row(i);
    for (int k = 0; k < n; ++k) {
      cplx* rk = wr + (k % W1) * BW;          // row k: column k at c = w
      const cplx piv = rk[w];
      if (!(cabs2(piv) > 0.0) || !isfinite(piv.r) || !isfinite(piv.i)) {
        atomicCAS(&s_info, 0, k + 1);
      }
      const cplx yk = Y[long(k) * M + m];
      for (int i = k + 1; i <= min(k + w, n - 1); ++i) {
        cplx* ri = wr + (i % W1) * BW;          // row i: column k at c = w - (i - k)
        const int ci = w - (i - k);
        const cplx l = cdivz(ri[ci], piv);
        ri[ci] = cmk(0.0, 0.0);
        for (int c = 1; c <= w; ++c) ri[ci + c] = csub(ri[ci + c], cmul(l, rk[w + c]));
        Y[long(i) * M + m] = csub(Y[long(i) * M + m], cmul(l, yk));
      }
      // keep U row k (diagonal and w upper entries), then bring in row k+w+1
      for (int c = 0; c <= w; ++c) U[(long(m) * n + k) * W1 + c] = rk[w + c];
      if (k + W1 < n) load_row(k + W1);
    }
    for (int k = n - 1; k >= 0; --k) {
      const GCplx uk = U + (long(m) * n + k) * W1;
      cplx sacc = Y[long(k) * M + m];
      for (int c = 1; c <= w && k + c < n; ++c) sacc = csub(sacc, cmul(uk[c], Y[long(k + c) * M + m]));
      Y[long(k) * M + m] = cdivz(sacc, uk[0]);
    }
  }
  __syncthreads();
  // ---- X = Re(Y H3) = Yr H3r - Yi H3i (fixed rows zero) on the matrix
  // cores, row tiles as above (Y operands of every step loaded once per row
  // tile, the next tile's before this tile's products; H3 operands in
  // registers; the two products of a step go to two accumulators per mode
  // tile, summed at the store).  The register-window solves formed X
  // during their back substitution already.
  const bool x_done = kFuseOut<MAXM> && (w == 5 || w == 3 || w == 1);
  if (!x_done) stage_cplx(sH, f.H3, MM, tid, nt);
  __syncthreads();
  if (!x_done) {
    double anr[kKS], ani[kKS];
    auto load_y = [&](int tr, double* dr, double* di) {
      const int ic = min(tr * 16 + (lane & 15), n - 1);
#pragma unroll
      for (int u = 0; u < kKS; ++u) {
        const int m = 4 * u + (lane >> 4);
        const cplx v = (u < ksteps && m < M) ? cplx(Y[long(ic) * M + m]) : cmk(0.0, 0.0);
        dr[u] = v.r;
        di[u] = v.i;
      }
    };
    if (wave < nrt) load_y(wave, anr, ani);
    double hr[kCT][kKS], hi[kCT][kKS];
    b_operands(hr, hi);
    for (int tr = wave; tr < nrt; tr += nwv) {
      double yr[kKS], yi[kKS];
      const int ia = tr * 16 + (lane & 15);
      const bool row_ok = ia < n && !is_fixed(A, ia);
#pragma unroll
      for (int u = 0; u < kKS; ++u) {
        yr[u] = row_ok ? anr[u] : 0.0;
        yi[u] = row_ok ? -ani[u] : 0.0;
      }
      if (tr + nwv < nrt) load_y(tr + nwv, anr, ani);
      v4d ar[kCT], ai[kCT];
#pragma unroll
      for (int c = 0; c < kCT; ++c) ar[c] = ai[c] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < kKS; ++u) {
#pragma unroll
        for (int c = 0; c < kCT; ++c) {
          if (u < ksteps && c < nct) {
            ar[c] = mfma16x16x4(yr[u], hr[c][u], ar[c]);
            ai[c] = mfma16x16x4(yi[u], hi[c][u], ai[c]);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < kCT; ++c) {
        const int qb = c * 16 + (lane & 15);
        const v4d x = ar[c] + ai[c];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int i = tr * 16 + (lane >> 4) + 4 * j;
          if (c < nct && i < n && qb < M) Xg[long(i) * M + qb] = x[j];
        }
      }
    }
  }
  if (tid == 0 && s_info) A.info[0] = s_info;
}

__global__ __launch_bounds__(kVecThreads) void k_fd_inverse(const SolveArgs* __restrict__ args,
                                                   const int* __restrict__ active) {
  const SolveArgs A = args[active[blockIdx.x]];
  fd_eig_inverse(A);
}
template <int MAXM>
__global__ __launch_bounds__(64) void k_fd_schur(const SolveArgs* __restrict__ args, const int* __restrict__ active) {
  const SolveArgs A = args[active[blockIdx.x]];
  fd_eig_schur<MAXM>(A);
}
template <bool ZG>
__global__ __launch_bounds__(kVecThreads) void k_fd_vectors(const SolveArgs* __restrict__ args,
                                                   const int* __restrict__ active) {
  const SolveArgs A = args[active[blockIdx.x]];
  fd_eig_vectors<ZG>(A);
}
template <int MAXM>
__global__ __launch_bounds__(kFdThreads, 1) void k_fd_solve(const SolveArgs* __restrict__ args,
                                                         const int* __restrict__ active) {
  const SolveArgs A = args[active[blockIdx.x]];
  fd_solve_body<MAXM>(A);
}
__global__ __launch_bounds__(kVecThreads) void k_fd_inverse_one(SolveArgs A) { fd_eig_inverse(A); }
template <int MAXM>
__global__ __launch_bounds__(64) void k_fd_schur_one(SolveArgs A) { fd_eig_schur<MAXM>(A); }
template <bool ZG>
__global__ __launch_bounds__(kVecThreads) void k_fd_vectors_one(SolveArgs A) { fd_eig_vectors<ZG>(A); }
template <int MAXM>
__global__ __launch_bounds__(kFdThreads, 1) void k_fd_solve_one(SolveArgs A) { fd_solve_body<MAXM>(A); }

// dynamic LDS of the three eigen-stage kernels, in M x L real units
constexpr size_t kFdLdsCap = 160 * 1024 - 2048;
size_t fd_inverse_lds(int M) { return size_t(2) * M * (M | 1) * 8; }
int fd_maxm(int M) { return M <= kFdSmallM ? kFdSmallM : kFdMaxM; }
size_t fd_schur_lds(int M) {
  const int mx = fd_maxm(M);
  return (size_t(2) * mx * schur_l(mx) + schur_sink(mx)) * 8;
}
// Z goes to the workspace when the six units do not fit
bool fd_vectors_zg(int M) { return size_t(6) * M * (M | 1) * 8 > kFdLdsCap; }
size_t fd_vectors_lds(int M) { return size_t(fd_vectors_zg(M) ? 4 : 6) * M * (M | 1) * 8; }
size_t fd_solve_lds(int M, int s) {
  const int w = 2 * s + 1;
  const bool reg = (w == 1 || w == 3 || w == 5);
  const size_t rows = size_t(M) * (w + 1) * (2 * w + 1);                      // per-system row rings
  const size_t ring = size_t(3) * ((w + 1) * (32 / (w + 1))) * (2 * w + 1);   // staged band chunks
  // (register-window solves: also two 16-row tiles of y for the fused transform out)
  return (size_t(M) + std::max(std::max(size_t(M) * M, reg ? ring : rows), reg ? size_t(32) * M : size_t(0))) * 16;
}
size_t fd_inverse_allowed = 0, fd_inverse1_allowed = 0;

bool fd_supported(int M, int s, int K) {
  return K == 2 && M <= kFdMaxM && fd_vectors_lds(M) <= kFdLdsCap && fd_inverse_lds(M) <= kFdLdsCap &&
         fd_solve_lds(M, s) <= kFdLdsCap;
}

// Launches of one instantiation: MAXM the layout and register-tile size
// (kFdSmallM or kFdMaxM), ZG whether the vectors kernel keeps Z in the
// workspace.  Flops and bytes as the library counts them (fd_eig_*, fd_*).
template <int MAXM> size_t fd_schur_lds_ok = 0;
template <int MAXM> size_t fd_schur1_lds_ok = 0;
template <bool ZG> size_t fd_vectors_lds_ok = 0;
template <bool ZG> size_t fd_vectors1_lds_ok = 0;
template <int MAXM> size_t fd_solve_lds_ok = 0;
template <int MAXM> size_t fd_solve1_lds_ok = 0;
double fd_schur_flops(int M);
double fd_schur_bytes(int M);
double fd_eig_flops(int M);
double fd_eig_bytes(int M);
double fd_flops(int n, int M, int w);
double fd_bytes(int n, int M, int w);

template <int MAXM, bool ZG>
taps_status fd_single_t(taps_handle* h, const SolveArgs& A, int n, int M, int s, hipStream_t stream) {
  const int w = 2 * s + 1;
  TAPS_TRY(taps::allow_lds(h, k_fd_inverse_one, fd_inverse_lds(M), &fd_inverse1_allowed));
  TAPS_TRY(taps::allow_lds(h, k_fd_schur_one<MAXM>, fd_schur_lds(M), &fd_schur1_lds_ok<MAXM>));
  TAPS_TRY(taps::allow_lds(h, k_fd_vectors_one<ZG>, fd_vectors_lds(M), &fd_vectors1_lds_ok<ZG>));
  TAPS_TRY(taps::allow_lds(h, k_fd_solve_one<MAXM>, fd_solve_lds(M, s), &fd_solve1_lds_ok<MAXM>));
  size_t slot, sslot;
  TAPS_TRY(taps::prof_begin(h, TAPS_PROF_EIG, stream, &slot));
  k_fd_inverse_one<<<1, kVecThreads, fd_inverse_lds(M), stream>>>(A);
  TAPS_LAUNCHED(h, "k_fd_inverse");
  TAPS_TRY(taps::prof_begin(h, TAPS_PROF_SCHUR, stream, &sslot));
  k_fd_schur_one<MAXM><<<1, 64, fd_schur_lds(M), stream>>>(A);
  TAPS_LAUNCHED(h, "k_fd_schur");
  TAPS_TRY(taps::prof_end(h, sslot, fd_schur_flops(M), fd_schur_bytes(M), stream));
  k_fd_vectors_one<ZG><<<1, kVecThreads, fd_vectors_lds(M), stream>>>(A);
  TAPS_LAUNCHED(h, "k_fd_vectors");
  TAPS_TRY(taps::prof_end(h, slot, fd_eig_flops(M), fd_eig_bytes(M), stream));
  TAPS_TRY(taps::prof_begin(h, TAPS_PROF_SOLVE, stream, &slot));
  k_fd_solve_one<MAXM><<<1, kFdThreads, fd_solve_lds(M, s), stream>>>(A);
  TAPS_LAUNCHED(h, "k_fd_solve");
  return taps::prof_end(h, slot, fd_flops(n, M, w), fd_bytes(n, M, w), stream);
}

template <int MAXM, bool ZG>
taps_status fd_prepare_t(taps_handle* h, int M, int s) {
  TAPS_TRY(taps::allow_lds(h, k_fd_inverse, fd_inverse_lds(M), &fd_inverse_allowed));
  TAPS_TRY(taps::allow_lds(h, k_fd_schur<MAXM>, fd_schur_lds(M), &fd_schur_lds_ok<MAXM>));
  TAPS_TRY(taps::allow_lds(h, k_fd_vectors<ZG>, fd_vectors_lds(M), &fd_vectors_lds_ok<ZG>));
  return taps::allow_lds(h, k_fd_solve<MAXM>, fd_solve_lds(M, s), &fd_solve_lds_ok<MAXM>);
}

template <int MAXM, bool ZG>
taps_status fd_batched_t(taps_handle* h, int n_active, const SolveArgs* args, const int* d_active, int M, int s,
                         double flops, double bytes, hipStream_t stream) {
  size_t slot, sslot;
  TAPS_TRY(taps::prof_begin(h, TAPS_PROF_EIG, stream, &slot));
  k_fd_inverse<<<n_active, kVecThreads, fd_inverse_lds(M), stream>>>(args, d_active);
  TAPS_LAUNCHED(h, "k_fd_inverse");
  TAPS_TRY(taps::prof_begin(h, TAPS_PROF_SCHUR, stream, &sslot));
  k_fd_schur<MAXM><<<n_active, 64, fd_schur_lds(M), stream>>>(args, d_active);
  TAPS_LAUNCHED(h, "k_fd_schur");
  TAPS_TRY(taps::prof_end(h, sslot, n_active * fd_schur_flops(M), n_active * fd_schur_bytes(M), stream));
  k_fd_vectors<ZG><<<n_active, kVecThreads, fd_vectors_lds(M), stream>>>(args, d_active);
  TAPS_LAUNCHED(h, "k_fd_vectors");
  TAPS_TRY(taps::prof_end(h, slot, n_active * fd_eig_flops(M), n_active * fd_eig_bytes(M), stream));
  TAPS_TRY(taps::prof_begin(h, TAPS_PROF_SOLVE, stream, &slot));
  k_fd_solve<MAXM><<<n_active, kFdThreads, fd_solve_lds(M, s), stream>>>(args, d_active);
  TAPS_LAUNCHED(h, "k_fd_solve");
  return taps::prof_end(h, slot, flops, bytes, stream);
}

// Algorithmic work of the fast diagonalisation's two stages.  Eigen stage
// per system, in units of M^3 real flops: C1^{-1} 2, E 2, Schur form with
// Schur vectors 25 (the usual Hessenberg + QR count), triangular eigenvectors
// and their inverse 4/3 each, H3 4, Z Wv 4, H2 4.  Banded stage: the two
// complex transforms (4 n M^2 each) and M banded complex eliminations with
// back substitution, 8 n (w+1)(w+2) each.
double fd_eig_flops(int M) { return 44.0 * M * double(M) * M; }
// the real Schur kernel alone: Hessenberg reduction and Francis QR with the
// Schur vectors accumulated; E read, T and Z written
double fd_schur_flops(int M) { return 25.0 * M * double(M) * M; }
double fd_schur_bytes(int M) { return 24.0 * M * double(M); }
double fd_eig_bytes(int M) { return 8.0 * (2.0 * M * M) + 16.0 * (2.0 * M * M + M) + 8.0 * M * M; }
double fd_flops(int n, int M, int w) {
  return 8.0 * n * double(M) * M + 8.0 * M * double(n) * (w + 1) * (w + 2);
}

// Algorithmic bytes of the banded stage: what the method itself must move --
// the two bands, Q read and X written once each, and the two complex M x M
// transforms.  The kernel's own scratch (complex right-hand sides and the
// pivot-scaled U rows it writes and reads back) is not counted: it shows in
// the memory counters, not here.
double fd_bytes(int n, int M, int w) {
  return 8.0 * (2.0 * n * (2 * w + 1) + 2.0 * n * M) + 16.0 * (2.0 * M * M);
}

}  // namespace

namespace taps {

int dim_residual_nparts(int n) { return cdiv(n, kResRows); }

taps_status dim_residual_parts(taps_handle* h, const taps_problem_t* p, int d, const double* d_C,
                               const double* d_U, const double* d_Q, double* parts, int* nparts,
                               hipStream_t stream) {
  const int nb = cdiv(p->n[d], kResRows);
  const size_t lds = size_t(taps::dev::residual_lds_doubles(p->M, p->s[d])) * 8;
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
  const size_t M4 = (M + 3) & ~3, P16 = ((w * M + 1 + 15) / 16) * 16;
  const size_t R16 = ((w * M + 15) / 16) * 16;
  const size_t fwd = (R16 * (M4 + 1) + M4 * P16 + 2 * size_t(M) * M) * 8;
  const size_t back = size_t(w + 1 + max(1, kThreadsMfma / M)) * M * 8;
  return fwd > back ? fwd : back;
}

size_t solve_lds_bytes(int M, int s) {
  const int w = 2 * s + 1;
  const size_t fwd = size_t(M) * M * (2 * w + 1) * 8 + 2 * size_t(M) * 8;
  const size_t back = size_t(w + 1 + max(1, kThreads / M)) * M * 8;
  return fwd > back ? fwd : back;
}

// Doubles of the first workspace region: the block LU's stored factors, or
// the fast diagonalisation's transforms, eigenvalues, C1^{-1}, complex
// right-hand sides and banded U rows, whichever is larger.
size_t fd_doubles(int n, int M, int s) {
  // the right-hand-side region also holds the vectors kernel's complex Z
  // (M x (M | 1)) when that does not fit LDS
  return size_t(7) * M * M + 2 * size_t(M) + std::max(2 * size_t(n) * M * (2 * s + 3), 2 * size_t(M) * (M | 1));
}

size_t zst_doubles(int n, int M, int s) {
  const size_t w = 2 * s + 1, lu = size_t(n) * M * w * M;
  return std::max(lu, fd_doubles(n, M, s));
}

taps_status solve_dim_impl(taps_handle* h, const taps_problem_t* p, int d, const double* d_C,
                           const double* d_Q, double* d_X, int* d_info, double* d_berr, hipStream_t stream) {
  const int n = p->n[d], M = p->M, s = p->s[d], w = 2 * s + 1;
  const size_t lds_mfma = solve_mfma_lds_bytes(M, s);
  const bool use_mfma = lds_mfma <= 160 * 1024 - 64 && p->n_kinds[d] <= kLuKinds && !getenv("TAPS_SOLVE_VECTOR");
  const size_t lds = use_mfma ? lds_mfma : solve_lds_bytes(M, s);
  const bool use_fd = h->tune.solver == 1 && fd_supported(M, s, p->n_kinds[d]);
  if (!use_fd && lds > 160 * 1024 - 64)
    return fail(h, TAPS_ERR_UNSUPPORTED, "M=%d with s=%d needs %zu bytes of LDS (max 163840)", M, s, lds);
  Bump bump;
  const size_t o_Z = bump.take(zst_doubles(n, M, s) * 8);
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
  if (use_fd) {
    if (M <= kFdSmallM)
      TAPS_TRY((fd_single_t<kFdSmallM, false>(h, A, n, M, s, stream)));
    else if (fd_vectors_zg(M))
      TAPS_TRY((fd_single_t<kFdMaxM, true>(h, A, n, M, s, stream)));
    else
      TAPS_TRY((fd_single_t<kFdMaxM, false>(h, A, n, M, s, stream)));
  } else if (use_mfma) {
    lu_single_fn fn = lu_single_for(M);
    TAPS_TRY(allow_lds(h, fn, lds, &lu_mfma_lds_allowed[mp_of(M) / 8]));
    TAPS_TRY(prof_begin(h, TAPS_PROF_SOLVE, stream, &slot));
    fn<<<1, kThreadsMfma, lds, stream>>>(A);
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

size_t solve_ws_bytes(int n, int M, int s, bool fd) {
  if (fd) return fd_doubles(n, M, s) * 8;
  const int w = 2 * s + 1;
  Bump bump;
  bump.take(zst_doubles(n, M, s) * 8);
  bump.take(size_t(n) * M * 8);
  bump.take(size_t(w + 1) * (w + 1) * M * M * 8);
  bump.take(size_t(w + 1) * M * 8);
  return bump.off;
}

// Fill the device argument record of one system into host memory `dst`
// (sizeof(SolveArgs) bytes); `ws` is the system's own solve workspace.
void solve_args_fill(void* dst, const taps_problem_t* p, int d, const double* d_C, const double* d_Q,
                     double* d_X, int* d_info, void* ws, bool fd) {
  const int n = p->n[d], M = p->M, s = p->s[d], w = 2 * s + 1;
  Bump bump;
  const size_t o_Z = bump.take(zst_doubles(n, M, s) * 8);
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
  A.Yst = fd ? nullptr : reinterpret_cast<double*>(base + o_Y);   // the fast diagonalisation
  A.win = fd ? nullptr : reinterpret_cast<double*>(base + o_W);   // uses the first region only
  A.rhs = fd ? nullptr : reinterpret_cast<double*>(base + o_R);
  A.info = d_info;
  memcpy(dst, &A, sizeof(A));
}

bool solve_batched_supported(int M, int s, int K) {
  return solve_mfma_lds_bytes(M, s) <= 160 * 1024 - 64 && K <= kLuKinds;
}

bool solve_fd_supported(int M, int s, int K) { return fd_supported(M, s, K); }
double solve_fd_flops(int n, int M, int s) { return fd_flops(n, M, 2 * s + 1); }
double solve_fd_bytes(int n, int M, int s) { return fd_bytes(n, M, 2 * s + 1); }

taps_status fd_prepare(taps_handle* h, int M, int s) {
  if (M <= kFdSmallM) return fd_prepare_t<kFdSmallM, false>(h, M, s);
  return fd_vectors_zg(M) ? fd_prepare_t<kFdMaxM, true>(h, M, s) : fd_prepare_t<kFdMaxM, false>(h, M, s);
}

taps_status fd_batched_launch(taps_handle* h, int n_active, const void* d_args, const int* d_active, int M, int s,
                              double flops, double bytes, hipStream_t stream) {
  const SolveArgs* args = static_cast<const SolveArgs*>(d_args);
  if (M <= kFdSmallM)
    return fd_batched_t<kFdSmallM, false>(h, n_active, args, d_active, M, s, flops, bytes, stream);
  if (fd_vectors_zg(M)) return fd_batched_t<kFdMaxM, true>(h, n_active, args, d_active, M, s, flops, bytes, stream);
  return fd_batched_t<kFdMaxM, false>(h, n_active, args, d_active, M, s, flops, bytes, stream);
}

taps_status solve_batched_prepare(taps_handle* h, int M, int s) {
  return allow_lds(h, lu_batched_for(M), solve_mfma_lds_bytes(M, s), &lu_mfma_batched_lds_allowed[mp_of(M) / 8]);
}

taps_status solve_batched_launch(taps_handle* h, int n_active, const void* d_args, const int* d_active,
                                 int M, int s, double flops, double bytes, hipStream_t stream) {
  const size_t lds = solve_mfma_lds_bytes(M, s);
  lu_batched_fn fn = lu_batched_for(M);
  TAPS_TRY(allow_lds(h, fn, lds, &lu_mfma_batched_lds_allowed[mp_of(M) / 8]));
  size_t slot;
  TAPS_TRY(prof_begin(h, TAPS_PROF_SOLVE, stream, &slot));
  fn<<<n_active, kThreadsMfma, lds, stream>>>(static_cast<const SolveArgs*>(d_args), d_active);
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
