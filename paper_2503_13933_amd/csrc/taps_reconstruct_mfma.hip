// Reduced-precision reconstruction of the rank-M field on the matrix cores
// (paper Sec. 2.3, TD interpolation):
//   u[i][j][k] = sum_m Phi_0[i][m] s_k[m] Phi_1[j][m],   s_k[m] = w_m Phi_2[k][m].
// Per plane k this is an (n0 x M) x (M x n1) product whose inner index carries
// the diagonal s_k.  The scaling is folded into the left operand once per
// (workgroup, plane), A'_k = Phi_0 diag(s_k), and the right operand Phi_1 is
// streamed through every j tile, so the per-plane cost outside the MFMA chain
// is 64 x M multiplies per wave.
//
// Rounding points (the error statement follows from them):
//   BF16: Phi_0, Phi_1, w, Phi_2 rounded to FP32; s = fl32(w * Phi_2);
//         a' = bf16(fl32(Phi_0 * s)); b = bf16(Phi_1); products exact in FP32,
//         accumulated in FP32 by v_mfma_f32_16x16x32_bf16.
//   FP32: the same in FP32 throughout (v_mfma_f32_16x16x4_f32).
//
// Workgroup = 4 waves for one plane.  BF16: 512 rows of i, each wave owning
// 128 rows (eight 16-row tiles, scaled Phi_0 operands in registers); FP32: 256
// rows, four tiles per wave.  Each wave walks the j tiles of 16 columns, Phi_1
// operands loaded three tiles ahead.  The BF16 Phi_1 is staged tile-ordered:
// for each 16-column tile and 32-mode step, the 64 lanes' 16-byte operands lie
// contiguously, so one load instruction reads 1 KB in 8 whole cache lines (the
// row-major layout touches 16 lines, half of each, and its loads bounded the
// kernel well below the matrix cores' rate); eight row tiles per wave halve
// the operand bytes per product against four.  Lanes with no row or
// column load and store through buffer resources with out-of-range offsets,
// which the address unit turns into zeros and dropped stores.
//
// MFMA lane layouts (checked on the device): A[l%16][kgroup l/16],
// B[kgroup l/16][l%16], D[4*(l/16) + r][l%16] for r = 0..3.  Accumulator
// elements are copied to a plain array before the buffer stores: storing
// acc[q] straight from the accumulator registers made this compiler emit the
// first element for every q, and indexing the 128-bit load result of a
// generic vector type element by element made it load one word for all four;
// whole-vector bit casts and named components avoid both.
#include <type_traits>
#include "taps_internal.hpp"

#include <cmath>
#include <mutex>
#include <vector>

// Scratch of taps_reconstruct_noalloc (staged factors and per-block partial
// records of one call), for callers that cannot allocate.  One copy per GPU,
// held until the process ends; host code reaches it only through the device
// address recon_scratch_attach() looked up for that GPU.
static __device__ __align__(256) char scratch[TAPS_NOALLOC_SCRATCH_BYTES];

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((__vector_size__(16)));

constexpr int kWaves = 4;
constexpr int kTilesF32 = 4;   // 16-row tiles per wave, FP32 kernel
constexpr int kTilesBF16 = 8;  // 16-row tiles per wave, BF16 kernel
constexpr int kOOB = 0x7ffffff0;

// rows of i per workgroup
constexpr int rows_wg(bool bf) { return kWaves * 16 * (bf ? kTilesBF16 : kTilesF32); }

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base, long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), 0x00020000);
}

// Per-field operands of a batched call (row blockIdx.y of a device table);
// a single call passes its pointers directly and a null table.
struct ConvJob {
  const double* P;
  void* out;
};
struct ReconJob {
  const float* P0f;
  const void* P1;
  const double* P2;
  const double* mw;
  float* out;
  double* rec;
};
struct PlaneJob {
  const double* rec;
  double* out;
};

// FP64 factor (n x M) -> T (n x Mp), zero-padded columns (conversion through FP32).
template <typename T>
__global__ void k_recon_convert(int n, int M, int Mp, const double* __restrict__ P, T* __restrict__ out,
                                const ConvJob* __restrict__ tab) {
  if (tab) {
    P = tab[blockIdx.y].P;
    out = static_cast<T*>(tab[blockIdx.y].out);
  }
  const long idx = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= long(n) * Mp) return;
  const int i = int(idx / Mp), m = int(idx - long(i) * Mp);
  const float v = (m < M) ? float(P[long(i) * M + m]) : 0.0f;
  out[idx] = T(v);
}

// FP64 factor (n x M) -> BF16 in the tile order of k_recon_bf16's streamed
// operand: element e of lane l of (tile jt, step ks) at ((jt KS + ks) 64 + l) 8 + e
// holds row 16 jt + l%16, mode 32 ks + 8 (l/16) + e; rows past n and modes
// past M are zero.  ntj = ceil(n / 16) tiles, KS = Mp / 32 steps.
__global__ void k_recon_convert_tiled(int n, int M, int KS, const double* __restrict__ P, __bf16* __restrict__ out,
                                      const ConvJob* __restrict__ tab) {
  if (tab) {
    P = tab[blockIdx.y].P;
    out = static_cast<__bf16*>(tab[blockIdx.y].out);
  }
  const long idx = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const long ntj = (n + 15) / 16;
  if (idx >= ntj * KS * 512) return;
  const int e = int(idx & 7), l = int((idx >> 3) & 63);
  const long t = idx >> 9;  // jt KS + ks
  const int ks = int(t % KS), jt = int(t / KS);
  const int j = 16 * jt + (l & 15), m = 32 * ks + 8 * (l >> 4) + e;
  const float v = (j < n && m < M) ? float(P[long(j) * M + m]) : 0.0f;
  out[idx] = __bf16(v);
}

struct Reduce {
  float mx;
  double ss;
  unsigned int cnt;  // the wave's count (the same in every lane: ballots counted on the scalar unit)
};

// Epilogue of one 16 x 16 tile of the products.  They are formed transposed
// (streamed Phi_1 rows as the MFMA's first operand), so lane l holds, for row
// i = (tile's first row) + l%16, the four consecutive columns j0 .. j0+3 with
// j0 = 16 jt + 4 (l/16): one 16-byte store per lane.  Store the values, or
// fold them into {max, sum of squares, count(u > thr)}: the maximum and the
// squares per lane (ss: the squares of a j tile's values summed in FP32,
// added to r.ss in FP64 by the caller), the count per wave from ballots of
// the compares, popcounted on the scalar unit; thrf is thr rounded down to
// FP32, so v > thrf exactly when v > thr.  FULL (wave-uniform: a tile wholly
// inside the plane) takes the unpredicated path.
template <int MODE, bool FULL>
__device__ inline void epilogue(const f32x4& acc, int i, int j0, int n0, int n1, bool jfull, float thrf, Reduce& r,
                                float& ss, __amdgpu_buffer_rsrc_t ro) {
  const float v[4] = {acc.x, acc.y, acc.z, acc.w};
  if (MODE == TAPS_STORE) {
    if (jfull) {
      const int off = (i < n0) ? (i * n1 + j0) * 4 : kOOB;
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, acc), ro, off, 0, 0);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int off = (i < n0 && j0 + q < n1) ? (i * n1 + j0 + q) * 4 : kOOB;
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[q]), ro, off, 0, 0);
      }
    }
  } else {
    // the same compare (and ballot) on both paths, so it is formed once
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const unsigned long long gt = __ballot(v[q] > thrf);
      if (FULL) {
        r.mx = fmaxf(r.mx, v[q]);
        ss = fmaf(v[q], v[q], ss);
        r.cnt += __builtin_popcountll(gt);
      } else {
        const bool ok = i < n0 && j0 + q < n1;
        r.mx = ok ? fmaxf(r.mx, v[q]) : r.mx;
        ss = ok ? fmaf(v[q], v[q], ss) : ss;
        r.cnt += __builtin_popcountll(gt & __ballot(ok));
      }
    }
  }
}

// Workgroup reduction of {max, sum of squares, count} into one record.
__device__ void reduce_store(Reduce r, double* rec) {
  __shared__ double sred[kWaves][3];
  for (int off = 32; off > 0; off >>= 1) {
    r.mx = fmaxf(r.mx, __shfl_xor(r.mx, off));
    r.ss += __shfl_xor(r.ss, off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sred[wave][0] = r.mx;
    sred[wave][1] = r.ss;
    sred[wave][2] = double(r.cnt);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = -INFINITY, ss = 0.0, cnt = 0.0;
    for (int w = 0; w < kWaves; ++w) {
      mx = fmax(mx, sred[w][0]);
      ss += sred[w][1];
      cnt += sred[w][2];
    }
    rec[0] = mx;
    rec[1] = ss;
    rec[2] = cnt;
    rec[3] = 0.0;
  }
}

// Scale factors of plane k in LDS: s[m] = fl32(fl32(w_m) * fl32(Phi_2[k][m])).
__device__ void plane_scale(float* s, int k, int M, int Mp, const double* P2, const double* mw) {
  for (int m = threadIdx.x; m < Mp; m += blockDim.x)
    s[m] = (m < M) ? float(mw ? mw[m] : 1.0) * float(P2[long(k) * M + m]) : 0.0f;
  __syncthreads();
}

// BF16 x BF16 -> FP32.  KS = Mp / 32 inner steps of 32 modes; lane group
// g = l/16 of step ks covers modes 32 ks + 8 g + (0..7).  P1t is Phi_1 in
// the tile order of k_recon_convert_tiled.
template <int KS, int MODE>
__global__ __launch_bounds__(kWaves * 64) void k_recon_bf16(int n0, int n1, int nrb, int M, const float* __restrict__ P0f,
                                                            const __bf16* __restrict__ P1t, const double* __restrict__ P2,
                                                            const double* __restrict__ mw, float thrf, float* __restrict__ out,
                                                            double* __restrict__ rec, const ReconJob* __restrict__ tab) {
  if (tab) {
    const ReconJob& J = tab[blockIdx.y];
    P0f = J.P0f;
    P1t = static_cast<const __bf16*>(J.P1);
    P2 = J.P2;
    mw = J.mw;
    out = J.out;
    rec = J.rec;
  }
  constexpr int Mp = 32 * KS, RT = kTilesBF16;
  __shared__ __align__(16) float s[Mp];
  const int k = blockIdx.x / nrb, rb = blockIdx.x - k * nrb;
  const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: tile tests branch on the scalar unit
  plane_scale(s, k, M, Mp, P2, mw);
  const int ibase = rb * rows_wg(true) + wave * 16 * RT;
  // scaled operands a'[i][m] = bf16(P0f[i][m] * s[m]), kept as packed words
  // (held as eight separate halves they were re-packed at every use)
  // (rows past n0 read row n0-1 and are zeroed: no load is predicated)
  u32x4 a[RT][KS];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int i = ibase + 16 * rt + c16;
    const f32x4* row = reinterpret_cast<const f32x4*>(P0f + long(min(i, n0 - 1)) * Mp);
    const float keep = (i < n0) ? 1.0f : 0.0f;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int q4 = (32 * ks + 8 * g) / 4;
      const f32x4 x0 = row[q4], x1 = row[q4 + 1];
      const f32x4 s0 = reinterpret_cast<const f32x4*>(s)[q4], s1 = reinterpret_cast<const f32x4*>(s)[q4 + 1];
      bf16x8 v;
      v[0] = __bf16(x0.x * s0.x * keep);
      v[1] = __bf16(x0.y * s0.y * keep);
      v[2] = __bf16(x0.z * s0.z * keep);
      v[3] = __bf16(x0.w * s0.w * keep);
      v[4] = __bf16(x1.x * s1.x * keep);
      v[5] = __bf16(x1.y * s1.y * keep);
      v[6] = __bf16(x1.z * s1.z * keep);
      v[7] = __bf16(x1.w * s1.w * keep);
      a[rt][ks] = __builtin_bit_cast(u32x4, v);
    }
  }
  const int ntj = (n1 + 15) / 16;
  const __amdgpu_buffer_rsrc_t rb1 = make_rsrc(P1t, long(ntj) * 16 * Mp * 2);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(out + (MODE == TAPS_STORE ? long(k) * n0 * n1 : 0),
                                              MODE == TAPS_STORE ? long(n0) * n1 * 4 : 0);
  auto bload = [&](int jt, bf16x8* b) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int off = (jt < ntj) ? ((jt * KS + ks) * 64 + lane) * 16 : kOOB;
      b[ks] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rb1, off, 0, 0));
    }
  };
  Reduce red{-INFINITY, 0.0, 0u};
  const bool rows_full = ibase + 16 * RT <= n0;
  // ALL: every tile of this wave lies inside the plane (its rows, and a
  // multiple of 16 columns), so no tile needs the per-tile test
  bool hot = false;   // wave-uniform: the wave's previous tile held a value above thr
  auto tile = [&](int jt, const bf16x8* b, auto all) {
    const bool jfull = 16 * jt + 16 <= n1;
    const bool full = decltype(all)::value || (rows_full && jfull);
    float ss = 0.0f;
    if (MODE == TAPS_REDUCE && full && !hot) {
      // after a cold tile: the whole tile's products first, then the fold:
      // the squares in the same order as the per-row-tile epilogue, the
      // maximum, and the count only when some value of the tile exceeds thr
      // (most of a field lies below it; otherwise every compare would be
      // false), so a cold tile needs no compares and no ballots (a
      // wave-uniform branch).  After a hot tile the per-row-tile epilogue,
      // which overlaps the compares with the next row tile's products, folds
      // the next one (the same values either way)
      f32x4 acc[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        acc[rt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
          acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[ks], __builtin_bit_cast(bf16x8, a[rt][ks]), acc[rt],
                                                            0, 0, 0);
      }
      float t = -INFINITY;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        ss = fmaf(acc[rt].x, acc[rt].x, ss);
        ss = fmaf(acc[rt].y, acc[rt].y, ss);
        ss = fmaf(acc[rt].z, acc[rt].z, ss);
        ss = fmaf(acc[rt].w, acc[rt].w, ss);
        t = fmaxf(fmaxf(fmaxf(fmaxf(t, acc[rt].x), acc[rt].y), acc[rt].z), acc[rt].w);
      }
      red.mx = fmaxf(red.mx, t);
      hot = __ballot(t > thrf) != 0;
      if (hot) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          red.cnt += __builtin_popcountll(__ballot(acc[rt].x > thrf)) + __builtin_popcountll(__ballot(acc[rt].y > thrf)) +
                     __builtin_popcountll(__ballot(acc[rt].z > thrf)) + __builtin_popcountll(__ballot(acc[rt].w > thrf));
      }
    } else {
      const unsigned int cnt0 = red.cnt;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[ks], __builtin_bit_cast(bf16x8, a[rt][ks]), acc, 0, 0, 0);
        const int i = ibase + 16 * rt + c16;
        if (full)
          epilogue<MODE, true>(acc, i, 16 * jt + 4 * g, n0, n1, jfull, thrf, red, ss, ro);
        else
          epilogue<MODE, false>(acc, i, 16 * jt + 4 * g, n0, n1, jfull, thrf, red, ss, ro);
      }
      hot = red.cnt != cnt0;
    }
    if (MODE == TAPS_REDUCE) red.ss += double(ss);
  };
  // four register sets in rotation: tile jt's operands were requested three
  // tiles earlier (an L2 round trip outlasts one tile's MFMA chain)
  auto run = [&](auto all) {
    bf16x8 b0[KS], b1[KS], b2[KS], b3[KS];
    bload(0, b0);
    bload(1, b1);
    bload(2, b2);
    for (int jt = 0; jt < ntj; jt += 4) {
      bload(jt + 3, b3);
      tile(jt, b0, all);
      if (jt + 1 >= ntj) break;
      bload(jt + 4, b0);
      tile(jt + 1, b1, all);
      if (jt + 2 >= ntj) break;
      bload(jt + 5, b1);
      tile(jt + 2, b2, all);
      if (jt + 3 >= ntj) break;
      bload(jt + 6, b2);
      tile(jt + 3, b3, all);
    }
  };
  if (rows_full && n1 % 16 == 0)
    run(std::true_type{});
  else
    run(std::false_type{});
  if (MODE == TAPS_REDUCE) reduce_store(red, rec + (long(k) * nrb + rb) * 4);
}

// FP32 x FP32 -> FP32.  S = Mp / 4 instructions of K = 4; in instruction q
// lane group g takes mode g*S + q, so each lane's modes are contiguous.
template <int S, int MODE>
__global__ __launch_bounds__(kWaves * 64) void k_recon_fp32(int n0, int n1, int nrb, int M, const float* __restrict__ P0f,
                                                            const float* __restrict__ P1f, const double* __restrict__ P2,
                                                            const double* __restrict__ mw, float thrf, float* __restrict__ out,
                                                            double* __restrict__ rec, const ReconJob* __restrict__ tab) {
  if (tab) {
    const ReconJob& J = tab[blockIdx.y];
    P0f = J.P0f;
    P1f = static_cast<const float*>(J.P1);
    P2 = J.P2;
    mw = J.mw;
    out = J.out;
    rec = J.rec;
  }
  constexpr int Mp = 4 * S;
  __shared__ __align__(16) float s[Mp];
  const int k = blockIdx.x / nrb, rb = blockIdx.x - k * nrb;
  const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: tile tests branch on the scalar unit
  plane_scale(s, k, M, Mp, P2, mw);
  const int ibase = rb * rows_wg(false) + wave * 16 * kTilesF32;
  // (rows past n0 read row n0-1 and are zeroed: no load is predicated)
  float a[4][S];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
    const int i = ibase + 16 * rt + c16;
    const f32x4* row = reinterpret_cast<const f32x4*>(P0f + long(min(i, n0 - 1)) * Mp + g * S);
    const f32x4* sv = reinterpret_cast<const f32x4*>(s + g * S);
    const float keep = (i < n0) ? 1.0f : 0.0f;
#pragma unroll
    for (int q4 = 0; q4 < S / 4; ++q4) {
      const f32x4 x = row[q4], sc = sv[q4];
      a[rt][4 * q4 + 0] = x.x * sc.x * keep;
      a[rt][4 * q4 + 1] = x.y * sc.y * keep;
      a[rt][4 * q4 + 2] = x.z * sc.z * keep;
      a[rt][4 * q4 + 3] = x.w * sc.w * keep;
    }
  }
  const __amdgpu_buffer_rsrc_t rb1 = make_rsrc(P1f, long(n1) * Mp * 4);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(out + (MODE == TAPS_STORE ? long(k) * n0 * n1 : 0),
                                              MODE == TAPS_STORE ? long(n0) * n1 * 4 : 0);
  auto bload = [&](int jt, float* b) {
    const int j = 16 * jt + c16;
#pragma unroll
    for (int q4 = 0; q4 < S / 4; ++q4) {
      const int off = (j < n1) ? (j * Mp + g * S + 4 * q4) * 4 : kOOB;
      const f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rb1, off, 0, 0));
      b[4 * q4 + 0] = v.x;
      b[4 * q4 + 1] = v.y;
      b[4 * q4 + 2] = v.z;
      b[4 * q4 + 3] = v.w;
    }
  };
  Reduce red{-INFINITY, 0.0, 0u};
  const bool rows_full = ibase + 16 * kTilesF32 <= n0;
  // ALL: every tile of this wave inside the plane (as in the BF16 kernel)
  auto tile = [&](int jt, const float* b, auto all) {
    f32x4 acc[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      acc[rt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q = 0; q < S; ++q) acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(b[q], a[rt][q], acc[rt], 0, 0, 0);
    }
    const bool jfull = 16 * jt + 16 <= n1;
    const bool full = decltype(all)::value || (rows_full && jfull);
    float ss = 0.0f;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int i = ibase + 16 * rt + c16;
      if (full)
        epilogue<MODE, true>(acc[rt], i, 16 * jt + 4 * g, n0, n1, jfull, thrf, red, ss, ro);
      else
        epilogue<MODE, false>(acc[rt], i, 16 * jt + 4 * g, n0, n1, jfull, thrf, red, ss, ro);
    }
    if (MODE == TAPS_REDUCE) red.ss += double(ss);
  };
  const int ntj = (n1 + 15) / 16;
  auto run = [&](auto all) {
    float bA[S], bB[S];
    bload(0, bA);
    for (int jt = 0; jt < ntj; jt += 2) {
      bload(jt + 1, bB);
      tile(jt, bA, all);
      if (jt + 1 >= ntj) break;
      bload(jt + 2, bA);
      tile(jt + 1, bB, all);
    }
  };
  if (rows_full && n1 % 16 == 0)
    run(std::true_type{});
  else
    run(std::false_type{});
  if (MODE == TAPS_REDUCE) reduce_store(red, rec + (long(k) * nrb + rb) * 4);
}

// Per-plane combination of the workgroup records (fixed order).
__global__ void k_recon_plane_mfma(int nrb, int n2, const double* __restrict__ rec, double* __restrict__ out,
                                   const PlaneJob* __restrict__ tab) {
  if (tab) {
    rec = tab[blockIdx.y].rec;
    out = tab[blockIdx.y].out;
  }
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n2) return;
  double mx = -INFINITY, ss = 0.0, cnt = 0.0;
  for (int t = 0; t < nrb; ++t) {
    const double* r = rec + (long(k) * nrb + t) * 4;
    mx = fmax(mx, r[0]);
    ss += r[1];
    cnt += r[2];
  }
  out[long(k) * 4 + 0] = mx;
  out[long(k) * 4 + 1] = ss;
  out[long(k) * 4 + 2] = cnt;
  out[long(k) * 4 + 3] = 0.0;
}

typedef void (*recon_fn)(dim3, hipStream_t, int, int, int, int, const float*, const void*, const double*,
                         const double*, float, float*, double*, const ReconJob*);

template <int KS, int MODE>
void launch_bf16(dim3 grid, hipStream_t st, int n0, int n1, int nrb, int M, const float* P0f, const void* P1,
                 const double* P2, const double* mw, float thr, float* out, double* rec, const ReconJob* tab) {
  k_recon_bf16<KS, MODE><<<grid, kWaves * 64, 0, st>>>(n0, n1, nrb, M, P0f, static_cast<const __bf16*>(P1), P2, mw,
                                                      thr, out, rec, tab);
}
template <int S, int MODE>
void launch_fp32(dim3 grid, hipStream_t st, int n0, int n1, int nrb, int M, const float* P0f, const void* P1,
                 const double* P2, const double* mw, float thr, float* out, double* rec, const ReconJob* tab) {
  k_recon_fp32<S, MODE><<<grid, kWaves * 64, 0, st>>>(n0, n1, nrb, M, P0f, static_cast<const float*>(P1), P2, mw,
                                                     thr, out, rec, tab);
}

}  // namespace

namespace taps {

// Accounting of one reconstruction call for the profiler family RECON:
// flops = 2 n0 n1 n2 M (the method's modes, not the padded ones the
// matrix cores execute); bytes = stored field
// (STORE) + factors read once.
double recon_flops(int n0, int n1, int n2, int M) { return 2.0 * n0 * double(n1) * n2 * M; }

// B fields of one shape: d_Phi holds 3 factor pointers per field, d_mode_w
// one pointer per field (or is null), d_out one output per field.  B = 1
// passes the pointers to the kernels directly; B > 1 uploads per-field tables
// (grid.y = field) into the workspace behind the staged factors.
// ext (with ext_cap bytes) replaces the handle workspace when given: then
// nothing is allocated and no kernel is timed.
taps_status reconstruct_mfma_fields(taps_handle* h, int B, const int32_t* n_pts, const double* const* d_Phi,
                                    int32_t M, const double* const* d_mode_w, taps_prec prec, taps_recon_mode mode,
                                    void* const* d_out, double thr, hipStream_t stream, char* ext = nullptr,
                                    size_t ext_cap = 0) {
  const int n0 = n_pts[0], n1 = n_pts[1], n2 = n_pts[2];
  const bool bf = (prec == TAPS_BF16);
  const int Mp = bf ? 32 * cdiv(M, 32) : 16 * cdiv(M, 16);
  if (long(n0) * n1 * 4 >= (1L << 31) || long(n1) * Mp * 4 >= (1L << 31))
    return fail(h, TAPS_ERR_UNSUPPORTED, "plane %d x %d too large for 32-bit offsets", n0, n1);
  const int nrb = cdiv(n0, rows_wg(bf));
  if (long(nrb) * n2 >= (1L << 31)) return fail(h, TAPS_ERR_UNSUPPORTED, "grid too large");
  if (B > 65535) return fail(h, TAPS_ERR_UNSUPPORTED, "%d fields in one call (max 65535)", B);
  const bool st = (mode == TAPS_STORE);
  Bump bump;
  const size_t s_P0 = size_t(n0) * Mp * 4, s_P1 = bf ? size_t(cdiv(n1, 16)) * 16 * Mp * 2 : size_t(n1) * Mp * 4;
  const size_t s_R = st ? 0 : size_t(n2) * nrb * 4 * 8;
  std::vector<size_t> o_P0(B), o_P1(B), o_R(B);
  for (int b = 0; b < B; ++b) {
    o_P0[b] = bump.take(s_P0);
    o_P1[b] = bump.take(s_P1);
    o_R[b] = bump.take(s_R);
  }
  const size_t o_tab = bump.take(B > 1 ? size_t(B) * (2 * sizeof(ConvJob) + sizeof(ReconJob) + sizeof(PlaneJob)) : 0);
  if (ext && bump.off > ext_cap)
    return fail(h, TAPS_ERR_UNSUPPORTED, "this reconstruction needs %zu bytes of scratch; the allocation-free entry "
                "point has %zu", bump.off, ext_cap);
  if (ext && B > 1) return fail(h, TAPS_ERR_INVALID, "allocation-free reconstruction takes one field");
  if (!ext) TAPS_TRY(need_ws(h, bump.off, stream));
  char* ws = ext ? ext : static_cast<char*>(h->ws);
  auto P0f = [&](int b) { return reinterpret_cast<float*>(ws + o_P0[b]); };
  auto P1 = [&](int b) { return static_cast<void*>(ws + o_P1[b]); };
  auto rec = [&](int b) { return reinterpret_cast<double*>(ws + o_R[b]); };
  const ConvJob* t_c0 = nullptr;
  const ConvJob* t_c1 = nullptr;
  const ReconJob* t_r = nullptr;
  const PlaneJob* t_p = nullptr;
  if (B > 1) {
    std::vector<char> tab(size_t(B) * (2 * sizeof(ConvJob) + sizeof(ReconJob) + sizeof(PlaneJob)));
    ConvJob* c0 = reinterpret_cast<ConvJob*>(tab.data());
    ConvJob* c1 = c0 + B;
    ReconJob* rj = reinterpret_cast<ReconJob*>(c1 + B);
    PlaneJob* pj = reinterpret_cast<PlaneJob*>(rj + B);
    for (int b = 0; b < B; ++b) {
      c0[b] = ConvJob{d_Phi[3 * b], P0f(b)};
      c1[b] = ConvJob{d_Phi[3 * b + 1], P1(b)};
      rj[b] = ReconJob{P0f(b), P1(b), d_Phi[3 * b + 2], d_mode_w ? d_mode_w[b] : nullptr,
                       st ? static_cast<float*>(d_out[b]) : nullptr, rec(b)};
      pj[b] = PlaneJob{rec(b), static_cast<double*>(d_out[b])};
    }
    // pageable source: the runtime stages it before returning
    TAPS_HIP(h, hipMemcpyAsync(ws + o_tab, tab.data(), tab.size(), hipMemcpyHostToDevice, stream));
    t_c0 = reinterpret_cast<const ConvJob*>(ws + o_tab);
    t_c1 = t_c0 + B;
    t_r = reinterpret_cast<const ReconJob*>(t_c1 + B);
    t_p = reinterpret_cast<const PlaneJob*>(t_r + B);
  }
  const dim3 g0(cdiv(long(n0) * Mp, 256), B), g1(cdiv(long(n1) * Mp, 256), B);
  k_recon_convert<float><<<g0, 256, 0, stream>>>(n0, M, Mp, d_Phi[0], P0f(0), t_c0);
  TAPS_LAUNCHED(h, "k_recon_convert");
  if (bf)
    k_recon_convert_tiled<<<dim3(cdiv(long(cdiv(n1, 16)) * 16 * Mp, 256), B), 256, 0, stream>>>(
        n1, M, Mp / 32, d_Phi[1], static_cast<__bf16*>(P1(0)), t_c1);
  else
    k_recon_convert<float><<<g1, 256, 0, stream>>>(n1, M, Mp, d_Phi[1], static_cast<float*>(P1(0)), t_c1);
  TAPS_LAUNCHED(h, "k_recon_convert");
  const dim3 grid(unsigned(long(nrb) * n2), B);
  float* out0 = st ? static_cast<float*>(d_out[0]) : nullptr;
  recon_fn fn = nullptr;
  if (bf) {
    if (Mp == 32) fn = st ? launch_bf16<1, TAPS_STORE> : launch_bf16<1, TAPS_REDUCE>;
    else fn = st ? launch_bf16<2, TAPS_STORE> : launch_bf16<2, TAPS_REDUCE>;
  } else {
    switch (Mp / 4) {
      case 4: fn = st ? launch_fp32<4, TAPS_STORE> : launch_fp32<4, TAPS_REDUCE>; break;
      case 8: fn = st ? launch_fp32<8, TAPS_STORE> : launch_fp32<8, TAPS_REDUCE>; break;
      case 12: fn = st ? launch_fp32<12, TAPS_STORE> : launch_fp32<12, TAPS_REDUCE>; break;
      default: fn = st ? launch_fp32<16, TAPS_STORE> : launch_fp32<16, TAPS_REDUCE>; break;
    }
  }
  size_t slot = 0;
  if (!ext) TAPS_TRY(prof_begin(h, TAPS_PROF_RECON, stream, &slot));
  // largest float <= thr (for u > thr decided in FP32 exactly as in FP64)
  float thrf = float(thr);
  if (double(thrf) > thr) thrf = std::nextafter(thrf, -INFINITY);
  fn(grid, stream, n0, n1, nrb, M, P0f(0), P1(0), d_Phi[2], d_mode_w ? d_mode_w[0] : nullptr, thrf, out0, rec(0),
     t_r);
  TAPS_LAUNCHED(h, bf ? "k_recon_bf16" : "k_recon_fp32");
  if (!ext)
    TAPS_TRY(prof_end(h, slot, B * recon_flops(n0, n1, n2, M),
                      B * ((st ? 4.0 * n0 * double(n1) * n2 : 0.0) + 4.0 * (double(n0) + n1) * Mp), stream));
  if (!st) {
    k_recon_plane_mfma<<<dim3(cdiv(n2, 64), B), 64, 0, stream>>>(nrb, n2, rec(0), static_cast<double*>(d_out[0]),
                                                               t_p);
    TAPS_LAUNCHED(h, "k_recon_plane_mfma");
  }
  return TAPS_OK;
}

taps_status reconstruct_mfma(taps_handle* h, const int32_t* n_pts, const double* const* d_Phi, int32_t M,
                             const double* d_mode_w, taps_prec prec, taps_recon_mode mode, void* d_out, double thr,
                             hipStream_t stream) {
  const double* const mw[1] = {d_mode_w};
  void* const out[1] = {d_out};
  return reconstruct_mfma_fields(h, 1, n_pts, d_Phi, M, d_mode_w ? mw : nullptr, prec, mode, out, thr, stream,
                                 nullptr, 0);
}

namespace {
constexpr int kScratchDevices = 64;
std::mutex scratch_mu;
char* scratch_ptr[kScratchDevices] = {};  // device address of `scratch` on each GPU
}  // namespace

// Looks up the device address of the no-alloc scratch on the handle's GPU
// (which must be current), once per GPU; taps_create calls it.
taps_status recon_scratch_attach(taps_handle* h) {
  if (h->device < 0 || h->device >= kScratchDevices)
    return fail(h, TAPS_ERR_UNSUPPORTED, "device %d beyond the %d the library tracks", h->device, kScratchDevices);
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_ptr[h->device]) return TAPS_OK;
  void* ptr = nullptr;
  TAPS_HIP(h, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return fail(h, TAPS_ERR_HIP, "no device address for the reconstruction scratch");
  scratch_ptr[h->device] = static_cast<char*>(ptr);
  return TAPS_OK;
}

char* recon_scratch(taps_handle* h) {
  std::lock_guard<std::mutex> lock(scratch_mu);
  return (h->device >= 0 && h->device < kScratchDevices) ? scratch_ptr[h->device] : nullptr;
}

}  // namespace taps
