// Learned warm start: canonical form of CP factors, the warm-start network's
// forward and backward passes on the matrix cores, squared-error loss, Adam.
//
// Network layers x_{l+1} = GELU(W_l x_l + b_l) (last layer linear).  Forward:
// the layer input is rounded to BF16 once (stored in the activation cache,
// row stride ldw = width rounded up to 32, zero padded) and multiplied with
// the BF16 weights by v_mfma_f32_16x16x32_bf16, FP32 accumulation; one wave
// per 16 x 16 output tile.  Backward: dz = dy * GELU'(z), then dW = dz^T x^
// and dx = dz W^ on v_mfma_f32_16x16x4_f32 (BF16 values are exact in FP32),
// db by column sums.  MFMA lane layouts: A[l%16][k group l/16],
// B[k group l/16][l%16], D[4*(l/16) + r][l%16].
#include "taps_internal.hpp"

#include <cmath>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((__vector_size__(16)));

inline int ldw(int w) { return (w + 31) / 32 * 32; }

__device__ inline float bf16_bits_to_f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// FP32 -> BF16 bits, round to nearest, ties to even (NaN kept quiet).
__device__ inline uint16_t f_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// GELU(z) = z Phi(z), Phi(z) = erfc(-z/sqrt 2)/2: the complementary form keeps
// full relative accuracy in the negative tail, where 1 + erf cancels.
__device__ inline float phi_cdf(float z) { return 0.5f * erfcf(-z * 0.70710678118654752f); }
__device__ inline float gelu(float z) { return z * phi_cdf(z); }
__device__ inline float gelu_grad(float z) { return phi_cdf(z) + z * expf(-0.5f * z * z) * 0.39894228040143268f; }

struct CacheLayout {
  size_t x[TAPS_MLP_MAX_LAYERS], z[TAPS_MLP_MAX_LAYERS], bytes;
};

CacheLayout cache_layout(const taps_mlp_t* net, int B) {
  CacheLayout c{};
  size_t off = 0;
  for (int l = 0; l < net->n_layers; ++l) {
    c.x[l] = off;
    off += taps::align256(size_t(B) * ldw(net->width[l]) * 2);
    c.z[l] = off;
    off += taps::align256(size_t(B) * net->width[l + 1] * 4);
  }
  c.bytes = off;
  return c;
}

// First layer input: FP32 (B x w) -> BF16 bits (B x ld), zero padding.
__global__ void k_mlp_input(int B, int w, int ld, const float* __restrict__ X, uint16_t* __restrict__ xh) {
  const long idx = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (idx >= long(B) * ld) return;
  const int b = int(idx / ld), i = int(idx - long(b) * ld);
  xh[idx] = (i < w) ? f_to_bf16_bits(X[long(b) * w + i]) : uint16_t(0);
}

// One 16 x 16 tile of z = x^ W^T + b per wave; grid (B tiles, out tiles
// covering the next layer's padded width).
__global__ __launch_bounds__(64) void k_mlp_fwd(int B, int ld, int out, int ld_next, const uint16_t* __restrict__ xh,
                                                const uint16_t* __restrict__ W, const float* __restrict__ bias,
                                                float* __restrict__ z, int act, uint16_t* __restrict__ xh_next,
                                                float* __restrict__ Y) {
  const int lane = threadIdx.x, g = lane >> 4, c16 = lane & 15;
  const int b0 = blockIdx.x * 16, o0 = blockIdx.y * 16;
  const int br = min(b0 + c16, B - 1), orow = min(o0 + c16, out - 1);
  const bool bok = b0 + c16 < B, ook = o0 + c16 < out;
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < ld; k0 += 32) {
    u32x4 xa = *reinterpret_cast<const u32x4*>(xh + long(br) * ld + k0 + 8 * g);
    u32x4 wb = *reinterpret_cast<const u32x4*>(W + long(orow) * ld + k0 + 8 * g);
    const u32x4 zero = {0u, 0u, 0u, 0u};
    xa = bok ? xa : zero;
    wb = ook ? wb : zero;
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, xa), __builtin_bit_cast(bf16x8, wb), acc,
                                                  0, 0, 0);
  }
  const float v[4] = {acc.x, acc.y, acc.z, acc.w};
  const int o = o0 + c16;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = b0 + 4 * g + q;
    if (b >= B) continue;
    if (o < out) {
      const float zz = v[q] + bias[o];
      z[long(b) * out + o] = zz;
      if (act) xh_next[long(b) * ld_next + o] = f_to_bf16_bits(gelu(zz));
      else Y[long(b) * out + o] = zz;
    } else if (act && o < ld_next) {
      xh_next[long(b) * ld_next + o] = 0;
    }
  }
}

// dz = dy * GELU'(z) (act) or dy.
__global__ void k_mlp_dz(long n, const float* __restrict__ z, const float* __restrict__ dy, int act,
                         float* __restrict__ dz) {
  const long idx = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (idx >= n) return;
  dz[idx] = act ? dy[idx] * gelu_grad(z[idx]) : dy[idx];
}

// gW (out x ld) = dz^T x^ : tile (o, i), inner index the batch.
__global__ __launch_bounds__(64) void k_mlp_dw(int B, int out, int ld, const float* __restrict__ dz,
                                               const uint16_t* __restrict__ xh, float* __restrict__ gW) {
  const int lane = threadIdx.x, g = lane >> 4, c16 = lane & 15;
  const int o0 = blockIdx.x * 16, i0 = blockIdx.y * 16;
  const int oc = min(o0 + c16, out - 1);
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < B; k0 += 4) {
    const int b = min(k0 + g, B - 1);
    const bool ok = k0 + g < B;
    const float a = (ok && o0 + c16 < out) ? dz[long(b) * out + oc] : 0.0f;
    const float x = ok ? bf16_bits_to_f(xh[long(b) * ld + i0 + c16]) : 0.0f;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, x, acc, 0, 0, 0);
  }
  const float v[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int o = o0 + 4 * g + q;
    if (o < out) gW[long(o) * ld + i0 + c16] = v[q];
  }
}

// gb[o] = sum_b dz[b][o] (fixed order).
__global__ void k_mlp_db(int B, int out, const float* __restrict__ dz, float* __restrict__ gb) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= out) return;
  float s = 0.0f;
  for (int b = 0; b < B; ++b) s += dz[long(b) * out + o];
  gb[o] = s;
}

// dx (B x in) = dz W^ : tile (b, i), inner index the layer output.
__global__ __launch_bounds__(64) void k_mlp_dx(int B, int out, int in, int ld, const float* __restrict__ dz,
                                               const uint16_t* __restrict__ W, float* __restrict__ dx) {
  const int lane = threadIdx.x, g = lane >> 4, c16 = lane & 15;
  const int b0 = blockIdx.x * 16, i0 = blockIdx.y * 16;
  const int bc = min(b0 + c16, B - 1);
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < out; k0 += 4) {
    const int o = min(k0 + g, out - 1);
    const bool ok = k0 + g < out;
    const float a = (ok && b0 + c16 < B) ? dz[long(bc) * out + o] : 0.0f;
    const float w = ok ? bf16_bits_to_f(W[long(o) * ld + i0 + c16]) : 0.0f;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, w, acc, 0, 0, 0);
  }
  const float v[4] = {acc.x, acc.y, acc.z, acc.w};
  const int i = i0 + c16;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = b0 + 4 * g + q;
    if (b < B && i < in) dx[long(b) * in + i] = v[q];
  }
}

// Mean squared error, one workgroup (deterministic order).
__global__ __launch_bounds__(1024) void k_mse(long n, const float* __restrict__ Y, const float* __restrict__ T,
                                              float* __restrict__ dY, double* __restrict__ loss) {
  __shared__ double part[1024];
  double s = 0.0;
  const double inv = 1.0 / double(n);
  for (long i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = double(Y[i]) - double(T[i]);  // exact for FP32 operands
    s += d * d;
    dY[i] = float(2.0 * d * inv);
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) part[threadIdx.x] += part[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = part[0] * inv;
}

__global__ void k_adam(long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2,
                       uint16_t* __restrict__ p16) {
  const long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (p16) p16[i] = f_to_bf16_bits(pi);
}

struct CanonArgs {
  int n[TAPS_MAX_DIMS];
  const double* U[TAPS_MAX_DIMS];
  double* out[TAPS_MAX_DIMS];
};

// Canonical form of D factors (one workgroup; sizes and pointers by value).
__global__ __launch_bounds__(256) void k_canonicalize(int D, int M, CanonArgs A) {
  const int* n_arr = A.n;
  const double* const* U = A.U;
  double* const* out = A.out;
  __shared__ double nrm[TAPS_MAX_DIMS][TAPS_MAX_M];
  __shared__ double sgn[TAPS_MAX_DIMS][TAPS_MAX_M];
  __shared__ double fac[TAPS_MAX_DIMS][TAPS_MAX_M];
  __shared__ int rank[TAPS_MAX_M];
  const int tid = threadIdx.x;
  for (int t = tid; t < D * M; t += blockDim.x) {
    const int d = t / M, m = t - d * M;
    const int n = n_arr[d];
    double s = 0.0, best = -1.0, sign = 1.0;
    for (int i = 0; i < n; ++i) {
      const double x = U[d][long(i) * M + m];
      s += x * x;
      if (fabs(x) > best) {
        best = fabs(x);
        sign = x < 0.0 ? -1.0 : 1.0;
      }
    }
    nrm[d][m] = sqrt(s);
    sgn[d][m] = sign;
  }
  __syncthreads();
  for (int m = tid; m < M; m += blockDim.x) {
    double lam = 1.0;
    bool zero = false;
    for (int d = 0; d < D; ++d) {
      lam *= nrm[d][m];
      zero = zero || (d > 0 && !(nrm[d][m] > 0.0));
    }
    double f0 = 1.0;
    for (int d = 1; d < D; ++d) {
      fac[d][m] = zero ? 1.0 : sgn[d][m] / nrm[d][m];
      f0 *= zero ? 1.0 : sgn[d][m] * nrm[d][m];
    }
    fac[0][m] = f0;
    int r = 0;
    for (int q = 0; q < M; ++q) {
      double lq = 1.0;
      for (int d = 0; d < D; ++d) lq *= nrm[d][q];
      r += (lq > lam || (lq == lam && q < m)) ? 1 : 0;
    }
    rank[m] = r;
  }
  __syncthreads();
  for (int d = 0; d < D; ++d) {
    const int n = n_arr[d];
    for (long t = tid; t < long(n) * M; t += blockDim.x) {
      const int i = int(t / M), m = int(t - long(i) * M);
      out[d][long(i) * M + rank[m]] = U[d][t] * fac[d][m];
    }
  }
}

taps_status check_net(taps_handle* h, const taps_mlp_t* net, int B) {
  if (!net || net->n_layers < 1 || net->n_layers > TAPS_MLP_MAX_LAYERS)
    return taps::fail(h, TAPS_ERR_INVALID, "network: bad layer count");
  if (B < 1) return taps::fail(h, TAPS_ERR_INVALID, "batch %d", B);
  for (int l = 0; l <= net->n_layers; ++l)
    if (net->width[l] < 1 || net->width[l] > 4096) return taps::fail(h, TAPS_ERR_INVALID, "width[%d]=%d", l, net->width[l]);
  for (int l = 0; l < net->n_layers; ++l)
    if (!net->d_W[l] || !net->d_b[l]) return taps::fail(h, TAPS_ERR_INVALID, "layer %d: null weights", l);
  return TAPS_OK;
}

}  // namespace

using namespace taps;

extern "C" {

size_t taps_mlp_cache_bytes(const taps_mlp_t* net, int32_t B) {
  if (!net || net->n_layers < 1 || net->n_layers > TAPS_MLP_MAX_LAYERS || B < 1) return 0;
  return cache_layout(net, B).bytes;
}

taps_status taps_mlp_forward(taps_handle_t h, const taps_mlp_t* net, int32_t B, const float* d_X, void* d_cache,
                             float* d_Y, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  TAPS_TRY(check_net(h, net, B));
  if (!d_X || !d_cache || !d_Y) return fail(h, TAPS_ERR_INVALID, "null pointer");
  const CacheLayout c = cache_layout(net, B);
  char* cache = static_cast<char*>(d_cache);
  const int L = net->n_layers;
  const int ld0 = ldw(net->width[0]);
  k_mlp_input<<<cdiv(long(B) * ld0, 256), 256, 0, stream>>>(B, net->width[0], ld0, d_X,
                                                            reinterpret_cast<uint16_t*>(cache + c.x[0]));
  TAPS_LAUNCHED(h, "k_mlp_input");
  for (int l = 0; l < L; ++l) {
    const int out = net->width[l + 1], ld = ldw(net->width[l]);
    const bool act = l < L - 1;
    const int ld_next = act ? ldw(out) : out;
    dim3 grid(cdiv(B, 16), cdiv(act ? ld_next : out, 16));
    k_mlp_fwd<<<grid, 64, 0, stream>>>(B, ld, out, ld_next, reinterpret_cast<const uint16_t*>(cache + c.x[l]),
                                       net->d_W[l], net->d_b[l], reinterpret_cast<float*>(cache + c.z[l]), act ? 1 : 0,
                                       act ? reinterpret_cast<uint16_t*>(cache + c.x[l + 1]) : nullptr,
                                       act ? nullptr : d_Y);
    TAPS_LAUNCHED(h, "k_mlp_fwd");
  }
  return TAPS_OK;
}

taps_status taps_mlp_backward(taps_handle_t h, const taps_mlp_t* net, int32_t B, const void* d_cache,
                              const float* d_dY, float* const* d_gW, float* const* d_gb, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  TAPS_TRY(check_net(h, net, B));
  if (!d_cache || !d_dY || !d_gW || !d_gb) return fail(h, TAPS_ERR_INVALID, "null pointer");
  const int L = net->n_layers;
  for (int l = 0; l < L; ++l)
    if (!d_gW[l] || !d_gb[l]) return fail(h, TAPS_ERR_INVALID, "layer %d: null gradient", l);
  int wmax = 0;
  for (int l = 0; l <= L; ++l) wmax = std::max(wmax, net->width[l]);
  Bump bump;
  const size_t o_dz = bump.take(size_t(B) * wmax * 4);
  const size_t o_g0 = bump.take(size_t(B) * wmax * 4);
  const size_t o_g1 = bump.take(size_t(B) * wmax * 4);
  TAPS_TRY(need_ws(h, bump.off, stream));
  char* ws = static_cast<char*>(h->ws);
  float* dz = reinterpret_cast<float*>(ws + o_dz);
  float* gbuf[2] = {reinterpret_cast<float*>(ws + o_g0), reinterpret_cast<float*>(ws + o_g1)};
  const CacheLayout c = cache_layout(net, B);
  const char* cache = static_cast<const char*>(d_cache);
  const float* dy = d_dY;
  for (int l = L - 1; l >= 0; --l) {
    const int out = net->width[l + 1], in = net->width[l], ld = ldw(in);
    const long nz = long(B) * out;
    k_mlp_dz<<<cdiv(nz, 256), 256, 0, stream>>>(nz, reinterpret_cast<const float*>(cache + c.z[l]), dy,
                                                l < L - 1 ? 1 : 0, dz);
    TAPS_LAUNCHED(h, "k_mlp_dz");
    const uint16_t* xh = reinterpret_cast<const uint16_t*>(cache + c.x[l]);
    k_mlp_dw<<<dim3(cdiv(out, 16), ld / 16), 64, 0, stream>>>(B, out, ld, dz, xh, d_gW[l]);
    TAPS_LAUNCHED(h, "k_mlp_dw");
    k_mlp_db<<<cdiv(out, 128), 128, 0, stream>>>(B, out, dz, d_gb[l]);
    TAPS_LAUNCHED(h, "k_mlp_db");
    if (l > 0) {
      float* dx = gbuf[l & 1];
      k_mlp_dx<<<dim3(cdiv(B, 16), cdiv(in, 16)), 64, 0, stream>>>(B, out, in, ld, dz, net->d_W[l], dx);
      TAPS_LAUNCHED(h, "k_mlp_dx");
      dy = dx;
    }
  }
  return TAPS_OK;
}

taps_status taps_mlp_mse(taps_handle_t h, int64_t n, const float* d_Y, const float* d_T, float* d_dY, double* d_loss,
                         hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (n < 1 || !d_Y || !d_T || !d_dY || !d_loss) return fail(h, TAPS_ERR_INVALID, "bad arguments");
  k_mse<<<1, 1024, 0, stream>>>(n, d_Y, d_T, d_dY, d_loss);
  TAPS_LAUNCHED(h, "k_mse");
  return TAPS_OK;
}

taps_status taps_adam_step(taps_handle_t h, int64_t n, float* d_p, const float* d_g, float* d_m, float* d_v, double lr,
                           double b1, double b2, double eps, int32_t t, uint16_t* d_p16, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (n < 0 || t < 1 || !(b1 >= 0.0 && b1 < 1.0) || !(b2 >= 0.0 && b2 < 1.0))
    return fail(h, TAPS_ERR_INVALID, "bad Adam arguments");
  if (n == 0) return TAPS_OK;
  if (!d_p || !d_g || !d_m || !d_v) return fail(h, TAPS_ERR_INVALID, "null pointer");
  const double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
  k_adam<<<cdiv(n, 256), 256, 0, stream>>>(n, d_p, d_g, d_m, d_v, float(lr), float(b1), float(b2), float(eps),
                                           float(c1), float(c2), d_p16);
  TAPS_LAUNCHED(h, "k_adam");
  return TAPS_OK;
}

taps_status taps_canonicalize(taps_handle_t h, int32_t D, const int32_t* n, int32_t M, const double* const* d_U,
                              double* const* d_out, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (D < 1 || D > TAPS_MAX_DIMS || M < 1 || M > TAPS_MAX_M || !n || !d_U || !d_out)
    return fail(h, TAPS_ERR_INVALID, "bad arguments");
  for (int d = 0; d < D; ++d)
    if (n[d] < 1 || !d_U[d] || !d_out[d] || d_U[d] == d_out[d]) return fail(h, TAPS_ERR_INVALID, "dim %d", d);
  CanonArgs a{};
  for (int d = 0; d < D; ++d) {
    a.n[d] = n[d];
    a.U[d] = d_U[d];
    a.out[d] = d_out[d];
  }
  k_canonicalize<<<1, 256, 0, stream>>>(D, M, a);
  TAPS_LAUNCHED(h, "k_canonicalize");
  return TAPS_OK;
}

}  // extern "C"
