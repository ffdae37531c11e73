// Reconstruction of the rank-M field on a 3D grid (paper Sec. 2.3, TD
// interpolation: u = sum_m prod_d Phi_d[i_d, m] with Phi_d = Ntilde_d U_d).
//
// Per z-plane k the field is a rank-M product  Phi_0 diag(w o Phi_2[k,:]) Phi_1^T,
// i.e. an (n0 x M) x (M x n1) GEMM with a per-plane diagonal scaling.  The FP64
// path is plain FMA; the reduced-precision paths live in the MFMA kernels of
// taps_reconstruct_mfma.hip.
#include "taps_internal.hpp"

namespace taps {
taps_status reconstruct_mfma(taps_handle* h, const int32_t* n_pts, const double* const* d_Phi, int32_t M,
                             const double* d_mode_w, taps_prec prec, taps_recon_mode mode, void* d_out,
                             double thr, hipStream_t stream);
taps_status reconstruct_mfma_fields(taps_handle* h, int B, const int32_t* n_pts, const double* const* d_Phi,
                                    int32_t M, const double* const* d_mode_w, taps_prec prec, taps_recon_mode mode,
                                    void* const* d_out, double thr, hipStream_t stream, char* ext = nullptr,
                                    size_t ext_cap = 0);
char* recon_scratch(taps_handle* h);
}

namespace {
taps_status fp64_reduce(taps_handle* h, const int32_t* n_pts, const double* const* d_Phi, int32_t M,
                        const double* d_mode_w, double* out, double thr, double* t, hipStream_t stream);
}

namespace {

constexpr int kTile = 16;  // 16 x 16 (i, j) outputs per block, one plane

// FP64: block = (i-tile, j-tile, plane k).  The plane's scaled mode weights and
// the two factor tiles are staged in LDS.
__global__ void k_recon_fp64(int n0, int n1, int n2, int M, const double* __restrict__ P0,
                             const double* __restrict__ P1, const double* __restrict__ P2,
                             const double* __restrict__ mw, int mode, double thr, double* __restrict__ out) {
  __shared__ double s0[kTile][TAPS_MAX_M + 1];
  __shared__ double s1[kTile][TAPS_MAX_M + 1];
  __shared__ double sw[TAPS_MAX_M];
  __shared__ double red[3][256];
  const int i0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile, k = blockIdx.z;
  const int tid = threadIdx.x;
  for (int m = tid; m < M; m += blockDim.x) sw[m] = P2[long(k) * M + m] * (mw ? mw[m] : 1.0);
  for (int t = tid; t < kTile * M; t += blockDim.x) {
    const int r = t / M, m = t % M;
    s0[r][m] = (i0 + r < n0) ? P0[long(i0 + r) * M + m] : 0.0;
    s1[r][m] = (j0 + r < n1) ? P1[long(j0 + r) * M + m] : 0.0;
  }
  __syncthreads();
  const int ti = tid / kTile, tj = tid % kTile;
  const int i = i0 + ti, j = j0 + tj;
  double u = 0.0;
  for (int m = 0; m < M; ++m) u += s0[ti][m] * sw[m] * s1[tj][m];
  const bool in = (i < n0 && j < n1);
  if (mode == TAPS_STORE) {
    if (in) out[(long(k) * n0 + i) * n1 + j] = u;
    return;
  }
  red[0][tid] = in ? u : -INFINITY;
  red[1][tid] = in ? u * u : 0.0;
  red[2][tid] = (in && u > thr) ? 1.0 : 0.0;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (tid < st) {
      red[0][tid] = fmax(red[0][tid], red[0][tid + st]);
      red[1][tid] += red[1][tid + st];
      red[2][tid] += red[2][tid + st];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const long tile = (long(k) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    out[tile * 4 + 0] = red[0][0];
    out[tile * 4 + 1] = red[1][0];
    out[tile * 4 + 2] = red[2][0];
    out[tile * 4 + 3] = 0.0;
  }
}

// Per-plane reduction of the per-tile records (fixed order).
__global__ void k_recon_plane(int tiles_per_plane, int n2, const double* __restrict__ tiles,
                              double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n2) return;
  double mx = -INFINITY, ss = 0.0, cnt = 0.0;
  for (int t = 0; t < tiles_per_plane; ++t) {
    const double* r = tiles + (long(k) * tiles_per_plane + t) * 4;
    mx = fmax(mx, r[0]);
    ss += r[1];
    cnt += r[2];
  }
  out[long(k) * 4 + 0] = mx;
  out[long(k) * 4 + 1] = ss;
  out[long(k) * 4 + 2] = cnt;
  out[long(k) * 4 + 3] = 0.0;
}

}  // namespace

using namespace taps;

extern "C" taps_status taps_reconstruct(taps_handle_t h, const int32_t* n_pts, const double* const* d_Phi,
                                        int32_t M, const double* d_mode_w, taps_prec prec,
                                        taps_recon_mode mode, void* d_out, double thr, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (!n_pts || !d_Phi || !d_out) return fail(h, TAPS_ERR_INVALID, "null pointer");
  if (M < 1 || M > TAPS_MAX_M) return fail(h, TAPS_ERR_UNSUPPORTED, "M=%d", M);
  for (int d = 0; d < 3; ++d) {
    if (n_pts[d] < 1) return fail(h, TAPS_ERR_INVALID, "n_pts[%d]=%d", d, n_pts[d]);
    if (!d_Phi[d]) return fail(h, TAPS_ERR_INVALID, "Phi[%d] is null", d);
  }
  if (mode != TAPS_STORE && mode != TAPS_REDUCE) return fail(h, TAPS_ERR_INVALID, "mode %d", int(mode));
  if (prec == TAPS_FP32 || prec == TAPS_BF16)
    return reconstruct_mfma(h, n_pts, d_Phi, M, d_mode_w, prec, mode, d_out, thr, stream);
  if (prec != TAPS_FP64) return fail(h, TAPS_ERR_INVALID, "precision %d", int(prec));
  const int n0 = n_pts[0], n1 = n_pts[1], n2 = n_pts[2];
  dim3 grid(cdiv(n0, kTile), cdiv(n1, kTile), n2);
  if (mode == TAPS_STORE) {
    k_recon_fp64<<<grid, kTile * kTile, 0, stream>>>(n0, n1, n2, M, d_Phi[0], d_Phi[1], d_Phi[2], d_mode_w,
                                                     mode, thr, static_cast<double*>(d_out));
    TAPS_LAUNCHED(h, "k_recon_fp64");
    return TAPS_OK;
  }
  const long tiles = long(grid.x) * grid.y * n2;
  TAPS_TRY(need_ws(h, size_t(tiles) * 4 * 8, stream));
  return fp64_reduce(h, n_pts, d_Phi, M, d_mode_w, static_cast<double*>(d_out), thr, static_cast<double*>(h->ws),
                     stream);
}

extern "C" taps_status taps_reconstruct_noalloc(taps_handle_t h, const int32_t* n_pts, const double* const* d_Phi,
                                                int32_t M, const double* d_mode_w, taps_prec prec,
                                                taps_recon_mode mode, void* d_out, double thr, hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (!n_pts || !d_Phi || !d_out) return fail(h, TAPS_ERR_INVALID, "null pointer");
  if (M < 1 || M > TAPS_MAX_M) return fail(h, TAPS_ERR_UNSUPPORTED, "M=%d", M);
  for (int d = 0; d < 3; ++d) {
    if (n_pts[d] < 1) return fail(h, TAPS_ERR_INVALID, "n_pts[%d]=%d", d, n_pts[d]);
    if (!d_Phi[d]) return fail(h, TAPS_ERR_INVALID, "Phi[%d] is null", d);
  }
  if (mode != TAPS_STORE && mode != TAPS_REDUCE) return fail(h, TAPS_ERR_INVALID, "mode %d", int(mode));
  if (prec != TAPS_FP64 && prec != TAPS_FP32 && prec != TAPS_BF16)
    return fail(h, TAPS_ERR_INVALID, "precision %d", int(prec));
  int dev = -1;
  TAPS_HIP(h, hipGetDevice(&dev));
  if (dev != h->device)
    return fail(h, TAPS_ERR_INVALID, "handle belongs to device %d, device %d is current", h->device, dev);
  char* ext = recon_scratch(h);
  if (!ext) return fail(h, TAPS_ERR_HIP, "reconstruction scratch not attached on device %d", dev);
  if (prec == TAPS_FP32 || prec == TAPS_BF16) {
    const double* const mw[1] = {d_mode_w};
    void* const out[1] = {d_out};
    return reconstruct_mfma_fields(h, 1, n_pts, d_Phi, M, d_mode_w ? mw : nullptr, prec, mode, out, thr, stream, ext,
                                   TAPS_NOALLOC_SCRATCH_BYTES);
  }
  const int n0 = n_pts[0], n1 = n_pts[1], n2 = n_pts[2];
  if (mode == TAPS_STORE) {
    dim3 grid(cdiv(n0, kTile), cdiv(n1, kTile), n2);
    k_recon_fp64<<<grid, kTile * kTile, 0, stream>>>(n0, n1, n2, M, d_Phi[0], d_Phi[1], d_Phi[2], d_mode_w,
                                                     mode, thr, static_cast<double*>(d_out));
    TAPS_LAUNCHED(h, "k_recon_fp64");
    return TAPS_OK;
  }
  const size_t need = size_t(cdiv(n0, kTile)) * cdiv(n1, kTile) * n2 * 4 * 8;
  if (need > TAPS_NOALLOC_SCRATCH_BYTES)
    return fail(h, TAPS_ERR_UNSUPPORTED, "this reconstruction needs %zu bytes of scratch; the allocation-free entry "
                "point has %zu", need, size_t(TAPS_NOALLOC_SCRATCH_BYTES));
  return fp64_reduce(h, n_pts, d_Phi, M, d_mode_w, static_cast<double*>(d_out), thr, reinterpret_cast<double*>(ext),
                     stream);
}

namespace {

// FP64 REDUCE: per-tile records into t (one record of 4 doubles per 2D tile
// and plane), then one record per plane into out.
taps_status fp64_reduce(taps_handle* h, const int32_t* n_pts, const double* const* d_Phi, int32_t M,
                        const double* d_mode_w, double* out, double thr, double* t, hipStream_t stream) {
  const int n0 = n_pts[0], n1 = n_pts[1], n2 = n_pts[2];
  dim3 grid(cdiv(n0, kTile), cdiv(n1, kTile), n2);
  const taps_recon_mode mode = TAPS_REDUCE;
  k_recon_fp64<<<grid, kTile * kTile, 0, stream>>>(n0, n1, n2, M, d_Phi[0], d_Phi[1], d_Phi[2], d_mode_w, mode,
                                                   thr, t);
  TAPS_LAUNCHED(h, "k_recon_fp64");
  k_recon_plane<<<cdiv(n2, 64), 64, 0, stream>>>(int(grid.x * grid.y), n2, t, out);
  TAPS_LAUNCHED(h, "k_recon_plane");
  return TAPS_OK;
}

}  // namespace

extern "C" taps_status taps_reconstruct_batched(taps_handle_t h, int32_t B, const int32_t* n_pts,
                                                const double* const* d_Phi, int32_t M,
                                                const double* const* d_mode_w, taps_prec prec,
                                                taps_recon_mode mode, void* const* d_out, double thr,
                                                hipStream_t stream) {
  if (!h) return TAPS_ERR_INVALID;
  if (B < 1 || !n_pts || !d_Phi || !d_out) return fail(h, TAPS_ERR_INVALID, "bad batched reconstruction arguments");
  if (M < 1 || M > TAPS_MAX_M) return fail(h, TAPS_ERR_UNSUPPORTED, "M=%d", M);
  for (int d = 0; d < 3; ++d)
    if (n_pts[d] < 1) return fail(h, TAPS_ERR_INVALID, "n_pts[%d]=%d", d, n_pts[d]);
  for (int b = 0; b < B; ++b) {
    if (!d_out[b]) return fail(h, TAPS_ERR_INVALID, "output %d is null", b);
    for (int d = 0; d < 3; ++d)
      if (!d_Phi[3 * b + d]) return fail(h, TAPS_ERR_INVALID, "field %d: Phi[%d] is null", b, d);
  }
  if (mode != TAPS_STORE && mode != TAPS_REDUCE) return fail(h, TAPS_ERR_INVALID, "mode %d", int(mode));
  if (prec == TAPS_FP32 || prec == TAPS_BF16)
    return reconstruct_mfma_fields(h, B, n_pts, d_Phi, M, d_mode_w, prec, mode, d_out, thr, stream);
  if (prec != TAPS_FP64) return fail(h, TAPS_ERR_INVALID, "precision %d", int(prec));
  for (int b = 0; b < B; ++b)   // FP64: one field after the other
    TAPS_TRY(taps_reconstruct(h, n_pts, d_Phi + 3 * b, M, d_mode_w ? d_mode_w[b] : nullptr, prec, mode, d_out[b],
                              thr, stream));
  return TAPS_OK;
}
