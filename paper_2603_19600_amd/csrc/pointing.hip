// Pointing operator kernels: ang2pix, P (gather), P^T (scatter-add), the fused
// diagonal-noise normal operator and the block-Jacobi accumulation.
//
// Every kernel expands the pointing on the fly (PointingOperator, section
// "Software Design", "Map-making classes"): theta/phi/psi are streamed once,
// coalesced along time, and the pixel and the polariser weights are rebuilt in
// registers; nothing per-sample is stored.
#include "common.h"

namespace fx {

// ---------------------------------------------------------------------------
// ang2pix over a flat array.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ang2pix(int32_t nside, const T *__restrict__ theta,
                                                    const T *__restrict__ phi, int64_t n,
                                                    int64_t *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
    out[i] = ang2pix_ring(nside, (double)theta[i], (double)phi[i]);
}

template <typename T>
furax_status launch_ang2pix(int32_t nside, const T *theta, const T *phi, int64_t n, int64_t *out,
                            hipStream_t s) {
  if (n == 0) return FURAX_OK;
  const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 65536);
  hipLaunchKernelGGL(k_ang2pix<T>, dim3((unsigned)blocks), dim3(kBlock), 0, s, nside, theta, phi,
                     n, out);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status launch_ang2pix<float>(int32_t, const float *, const float *, int64_t,
                                            int64_t *, hipStream_t);
template furax_status launch_ang2pix<double>(int32_t, const double *, const double *, int64_t,
                                             int64_t *, hipStream_t);

// ---------------------------------------------------------------------------
// Fill kernel (used instead of a memset so that captured graphs stay safe).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_zero(uint4 *__restrict__ p, int64_t n16,
                                                 uint8_t *__restrict__ tail, int64_t ntail) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  for (int64_t i = t; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (t < ntail) tail[t] = 0;
}

furax_status zero_async(void *ptr, size_t bytes, hipStream_t s) {
  if (bytes == 0) return FURAX_OK;
  // Every buffer the library clears is at least 16-byte aligned (allocator
  // or map planes of 8-byte elements starting at an aligned base).
  const int64_t n16 = (int64_t)(bytes / 16);
  const int64_t ntail = (int64_t)(bytes % 16);
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n16 + kBlock - 1) / kBlock, 8192));
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                     static_cast<uint4 *>(ptr), n16,
                     static_cast<uint8_t *>(ptr) + n16 * 16, ntail);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}

// ---------------------------------------------------------------------------
// P: tod[k,i] = g_k (I[p] + c Q[p] + s U[p]).
// ---------------------------------------------------------------------------
template <typename T, typename MT>
__global__ void __launch_bounds__(kBlock) k_apply(PtArgs<T> a, const MT *__restrict__ map,
                                                  int64_t npix, T *__restrict__ tod) {
  const int64_t nch = chunks_per_det(a.n_samp);
  const int64_t k = blockIdx.x / nch;
  const int64_t base = (blockIdx.x % nch) * kChunk + threadIdx.x;
  const T g = gain_of(a, k);
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t i = base + (int64_t)it * kBlock;
    if (i >= a.n_samp) break;
    const Geom<T> gm = sample_geom(a, k, i);
    T y = 0;
    if (gm.pix >= 0) {
      y = (T)map[gm.pix] + gm.c * (T)map[npix + gm.pix] + gm.s * (T)map[2 * npix + gm.pix];
      y = g * y;
    }
    tod[k * a.n_samp + i] = y;
  }
}

template <typename T>
furax_status launch_pointing_apply(const PtArgs<T> &a, const void *map, bool map_f64, T *tod,
                                   hipStream_t s) {
  if (a.n_samp == 0) return FURAX_OK;
  const int64_t npix = 12ll * a.nside * a.nside;
  const int64_t blocks = a.n_det * chunks_per_det(a.n_samp);
  if (map_f64)
    hipLaunchKernelGGL((k_apply<T, double>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a,
                       static_cast<const double *>(map), npix, tod);
  else
    hipLaunchKernelGGL((k_apply<T, float>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a,
                       static_cast<const float *>(map), npix, tod);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status launch_pointing_apply<float>(const PtArgs<float> &, const void *, bool,
                                                   float *, hipStream_t);
template furax_status launch_pointing_apply<double>(const PtArgs<double> &, const void *, bool,
                                                    double *, hipStream_t);

// ---------------------------------------------------------------------------
// P^T: map[:, p] += g_k w_k d[k,i] (1, c, s), products in T, sums in FP64.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_transpose_atomic(PtArgs<T> a, const T *__restrict__ tod,
                                                             int64_t npix, const double *w_det,
                                                             double *__restrict__ map) {
  const int64_t nch = chunks_per_det(a.n_samp);
  const int64_t k = blockIdx.x / nch;
  const int64_t base = (blockIdx.x % nch) * kChunk + threadIdx.x;
  T g = gain_of(a, k);
  if (w_det) g = g * (T)w_det[k];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t i = base + (int64_t)it * kBlock;
    if (i >= a.n_samp) break;
    const Geom<T> gm = sample_geom(a, k, i);
    if (gm.pix < 0) continue;
    const T v = g * tod[k * a.n_samp + i];
    atomicAdd(&map[gm.pix], (double)v);
    atomicAdd(&map[npix + gm.pix], (double)(v * gm.c));
    atomicAdd(&map[2 * npix + gm.pix], (double)(v * gm.s));
  }
}

template <typename T>
furax_status launch_pointing_transpose(const PtArgs<T> &a, const T *tod, double *map,
                                       bool /*tod_scaled_by_w*/, const double *w_det,
                                       hipStream_t s) {
  if (a.n_samp == 0) return FURAX_OK;
  const int64_t npix = 12ll * a.nside * a.nside;
  const int64_t blocks = a.n_det * chunks_per_det(a.n_samp);
  hipLaunchKernelGGL(k_transpose_atomic<T>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a, tod,
                     npix, w_det, map);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status launch_pointing_transpose<float>(const PtArgs<float> &, const float *,
                                                       double *, bool, const double *,
                                                       hipStream_t);
template furax_status launch_pointing_transpose<double>(const PtArgs<double> &, const double *,
                                                        double *, bool, const double *,
                                                        hipStream_t);

// ---------------------------------------------------------------------------
// Fused q = P^T diag(w) P p for diagonal noise: one pass over the pointing.
// map_lo is an FP32 copy of p for the FP32 path (null: read p in FP64).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fused_diag(PtArgs<T> a, const T *__restrict__ map_lo,
                                                       const double *__restrict__ p, int64_t npix,
                                                       const double *__restrict__ w_det,
                                                       double *__restrict__ q) {
  const int64_t nch = chunks_per_det(a.n_samp);
  const int64_t k = blockIdx.x / nch;
  const int64_t base = (blockIdx.x % nch) * kChunk + threadIdx.x;
  const T g = gain_of(a, k);
  const T w = (T)w_det[k];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t i = base + (int64_t)it * kBlock;
    if (i >= a.n_samp) break;
    const Geom<T> gm = sample_geom(a, k, i);
    if (gm.pix < 0) continue;
    T y;
    if (map_lo)
      y = map_lo[gm.pix] + gm.c * map_lo[npix + gm.pix] + gm.s * map_lo[2 * npix + gm.pix];
    else
      y = (T)p[gm.pix] + gm.c * (T)p[npix + gm.pix] + gm.s * (T)p[2 * npix + gm.pix];
    y = g * y;
    const T v = g * (w * y);
    atomicAdd(&q[gm.pix], (double)v);
    atomicAdd(&q[npix + gm.pix], (double)(v * gm.c));
    atomicAdd(&q[2 * npix + gm.pix], (double)(v * gm.s));
  }
}

template <typename T>
furax_status launch_fused_diag(const PtArgs<T> &a, const T *map_lo, const double *p,
                               const double *w_det, double *q, hipStream_t s) {
  if (a.n_samp == 0) return FURAX_OK;
  const int64_t npix = 12ll * a.nside * a.nside;
  const int64_t blocks = a.n_det * chunks_per_det(a.n_samp);
  hipLaunchKernelGGL(k_fused_diag<T>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a, map_lo, p,
                     npix, w_det, q);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status launch_fused_diag<float>(const PtArgs<float> &, const float *,
                                               const double *, const double *, double *,
                                               hipStream_t);
template furax_status launch_fused_diag<double>(const PtArgs<double> &, const double *,
                                                const double *, const double *, double *,
                                                hipStream_t);

// ---------------------------------------------------------------------------
// Block-Jacobi accumulation: M_p += g^2 w_k (1,c,s)^T (1,c,s), hits_p += 1.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bj_build(PtArgs<T> a, int64_t npix,
                                                     const double *__restrict__ w_det,
                                                     double *__restrict__ M6,
                                                     int32_t *__restrict__ hits) {
  const int64_t nch = chunks_per_det(a.n_samp);
  const int64_t k = blockIdx.x / nch;
  const int64_t base = (blockIdx.x % nch) * kChunk + threadIdx.x;
  const double g = a.gain ? a.gain[k] : 1.0;
  const double w = g * g * w_det[k];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t i = base + (int64_t)it * kBlock;
    if (i >= a.n_samp) break;
    const Geom<T> gm = sample_geom(a, k, i);
    if (gm.pix < 0) continue;
    const double c = (double)gm.c, s = (double)gm.s;
    const double wc = w * c, ws = w * s;
    atomicAdd(&M6[gm.pix], w);
    atomicAdd(&M6[npix + gm.pix], wc);
    atomicAdd(&M6[2 * npix + gm.pix], ws);
    atomicAdd(&M6[3 * npix + gm.pix], wc * c);
    atomicAdd(&M6[4 * npix + gm.pix], wc * s);
    atomicAdd(&M6[5 * npix + gm.pix], ws * s);
    atomicAdd(&hits[gm.pix], 1);
  }
}

template <typename T>
furax_status launch_bj_build(const PtArgs<T> &a, const double *w_det, double *M6, int32_t *hits,
                             hipStream_t s) {
  if (a.n_samp == 0) return FURAX_OK;
  const int64_t npix = 12ll * a.nside * a.nside;
  const int64_t blocks = a.n_det * chunks_per_det(a.n_samp);
  hipLaunchKernelGGL(k_bj_build<T>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a, npix, w_det,
                     M6, hits);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status launch_bj_build<float>(const PtArgs<float> &, const double *, double *,
                                             int32_t *, hipStream_t);
template furax_status launch_bj_build<double>(const PtArgs<double> &, const double *, double *,
                                              int32_t *, hipStream_t);

// ---------------------------------------------------------------------------
// Closed-form inverse of each pixel's symmetric 3x3 block, 1-norm rcond.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_bj_invert(int64_t npix, const double *__restrict__ M6,
                                                      const int32_t *__restrict__ hits,
                                                      double rcond_min, int32_t min_hits,
                                                      const uint8_t *__restrict__ force_valid,
                                                      double *__restrict__ Minv6,
                                                      uint8_t *__restrict__ valid,
                                                      double *__restrict__ rcond_out) {
#pragma clang fp contract(off)
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < npix; p += stride) {
    const double a = M6[p], b = M6[npix + p], c = M6[2 * npix + p];
    const double d = M6[3 * npix + p], e = M6[4 * npix + p], f = M6[5 * npix + p];
    const double A = d * f - e * e, B = c * e - b * f, C = b * e - c * d;
    const double D = a * f - c * c, E = b * c - a * e, F = a * d - b * b;
    const double det = a * A + b * B + c * C;
    const double ia = A / det, ib = B / det, ic = C / det;
    const double id = D / det, ie = E / det, iff = F / det;
    const double n1 = fmax(fmax(fabs(a) + fabs(b) + fabs(c), fabs(b) + fabs(d) + fabs(e)),
                           fabs(c) + fabs(e) + fabs(f));
    const double n1i = fmax(fmax(fabs(ia) + fabs(ib) + fabs(ic), fabs(ib) + fabs(id) + fabs(ie)),
                            fabs(ic) + fabs(ie) + fabs(iff));
    double rc = 1.0 / (n1 * n1i);
    if (!(rc - rc == 0.0) || det == 0.0) rc = 0.0;
    bool ok;
    if (force_valid) ok = force_valid[p] != 0;
    else ok = (hits[p] >= min_hits) && (rc >= rcond_min);
    Minv6[p] = ok ? ia : 0.0;
    Minv6[npix + p] = ok ? ib : 0.0;
    Minv6[2 * npix + p] = ok ? ic : 0.0;
    Minv6[3 * npix + p] = ok ? id : 0.0;
    Minv6[4 * npix + p] = ok ? ie : 0.0;
    Minv6[5 * npix + p] = ok ? iff : 0.0;
    if (valid) valid[p] = ok ? 1 : 0;
    if (rcond_out) rcond_out[p] = rc;
  }
}

furax_status launch_bj_invert(int64_t npix, const double *M6, const int32_t *hits,
                              double rcond_min, int32_t min_hits, const uint8_t *force_valid,
                              double *Minv6, uint8_t *valid, double *rcond, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((npix + kBlock - 1) / kBlock, 16384);
  hipLaunchKernelGGL(k_bj_invert, dim3((unsigned)blocks), dim3(kBlock), 0, s, npix, M6, hits,
                     rcond_min, min_hits, force_valid, Minv6, valid, rcond);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}

}  // namespace fx
