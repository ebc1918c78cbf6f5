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
// Sample tiles.
// ---------------------------------------------------------------------------
Tiling make_tiling(int64_t n_det, int64_t n_samp, int32_t nside, int64_t target_samples,
                   int32_t min_log2ts) {
  Tiling t;
  // At most 256 detectors per tile: with a +-1 deg focal plane they cover a
  // patch a few tens of pixels wide, so a 64-sample stretch of all of them
  // revisits each pixel ~10 times at nside 512.
  t.dets = (int32_t)std::min<int64_t>(n_det, 256);
  int32_t l2 = nside >= 1024 ? 5 : 6;
  while (((int64_t)t.dets << l2) < target_samples && l2 < 10) ++l2;
  l2 = std::max(l2, min_log2ts);
  // never longer than the stream rounded up to a power of two
  int32_t cap = 0;
  while (((int64_t)1 << cap) < n_samp) ++cap;
  t.log2ts = std::min(l2, cap);
  t.n_tb = (n_samp + ((int64_t)1 << t.log2ts) - 1) >> t.log2ts;
  t.n_dg = (n_det + t.dets - 1) / t.dets;
  return t;
}

// Block index -> logical tile, keeping consecutive time blocks of one detector
// group on the same XCD (workgroups are dealt round-robin over the 8 XCDs), so
// the map lines a tile touches are likely already in that XCD's L2.
__device__ __forceinline__ int64_t tile_of_block(int64_t bid, int64_t nblocks) {
  const int64_t per = nblocks / 8;
  if (per == 0 || bid >= per * 8) return bid;
  return (bid % 8) * per + bid / 8;
}

// 2 alpha_i for the tile's samples t0 .. t0 + 2^log2ts - 1, into LDS.
template <typename T>
__device__ __forceinline__ void fill_two_alpha(const PtArgs<T> &a, int64_t t0, int32_t log2ts,
                                               double *ta, int nthreads) {
  if (!a.hwp) return;
  for (int t = threadIdx.x; t < (1 << log2ts); t += nthreads)
    ta[t] = 2.0 * hwp_alpha(t0 + t, a.hwp_num_mod, a.hwp_den, a.hwp_phase0);
}

template <typename MT>
__device__ __forceinline__ void load_iqu(const MT *__restrict__ m, MapLayout l, int32_t pix,
                                         MT &I, MT &Q, MT &U) {
  const int64_t o = (int64_t)pix * l.ps;
  I = m[o];
  Q = m[o + l.cs];
  U = m[o + 2 * l.cs];
}

// ---------------------------------------------------------------------------
// P: tod[k,i] = g_k (I[p] + c Q[p] + s U[p]).
// ---------------------------------------------------------------------------
constexpr int kApplyThreads = 256;
constexpr int kMaxTileSamples = 1024;   // longest tile (2^10 samples per detector)

template <typename T, typename MT>
__global__ void __launch_bounds__(kApplyThreads) k_apply(PtArgs<T> a, const MT *__restrict__ map,
                                                         MapLayout ml, Tiling tl,
                                                         T *__restrict__ tod, GeomCache<T> gc) {
  __shared__ double ta[kMaxTileSamples];
  const int64_t tile = tile_of_block(blockIdx.x, tl.blocks());
  const int64_t d0 = (tile / tl.n_tb) * tl.dets;
  const int64_t t0 = (tile % tl.n_tb) << tl.log2ts;
  const int32_t tsm = (1 << tl.log2ts) - 1;
  const int32_t nsamp = tl.dets << tl.log2ts;
  fill_two_alpha(a, t0, tl.log2ts, ta, kApplyThreads);
  __syncthreads();
  for (int32_t s = threadIdx.x; s < nsamp; s += kApplyThreads) {
    const int64_t k = d0 + (s >> tl.log2ts);
    const int64_t i = t0 + (s & tsm);
    if (k >= a.n_det || i >= a.n_samp) continue;
    const int64_t off = k * a.n_samp + i;
    const Geom<T> gm = sample_geom_ta(a, k, off, ta[s & tsm]);
    T y = 0;
    if (gm.pix >= 0) {
      MT I, Q, U;
      load_iqu(map, ml, gm.pix, I, Q, U);
      y = (T)I + gm.c * (T)Q + gm.s * (T)U;
      y = gain_of(a, k) * y;
    }
    tod[off] = y;
    if (gc.pix) {
      gc.pix[off] = gm.pix;
      gc.c[off] = gm.c;
      gc.s[off] = gm.s;
    }
  }
}

template <typename T>
furax_status launch_pointing_apply(const PtArgs<T> &a, const void *map, bool map_f64,
                                   MapLayout ml, T *tod, hipStream_t s, GeomCache<T> gc) {
  if (a.n_samp == 0) return FURAX_OK;
  const Tiling tl = make_tiling(a.n_det, a.n_samp, a.nside, 4096, 6);
  if (map_f64)
    hipLaunchKernelGGL((k_apply<T, double>), dim3((unsigned)tl.blocks()), dim3(kApplyThreads), 0,
                       s, a, static_cast<const double *>(map), ml, tl, tod, gc);
  else
    hipLaunchKernelGGL((k_apply<T, float>), dim3((unsigned)tl.blocks()), dim3(kApplyThreads), 0,
                       s, a, static_cast<const float *>(map), ml, tl, tod, gc);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status launch_pointing_apply<float>(const PtArgs<float> &, const void *, bool,
                                                   MapLayout, float *, hipStream_t,
                                                   GeomCache<float>);
template furax_status launch_pointing_apply<double>(const PtArgs<double> &, const void *, bool,
                                                    MapLayout, double *, hipStream_t,
                                                    GeomCache<double>);

// ---------------------------------------------------------------------------
// P^T scatter-add with LDS privatisation.
//
// Each workgroup owns one tile of samples and an open-addressing hash table
// in LDS (kHashSlots pixel keys and three FP64 sums per slot).  A sample
// claims its pixel's slot with a compare-and-swap on the key (linear
// probing), then adds its three contributions with LDS FP64 atomics.  After
// the tile, every occupied slot is flushed to the global map with FP64
// atomics, so global atomic traffic falls from 3 per sample to 3 per distinct
// pixel per tile.  A sample that finds no slot within kMaxProbe probes goes
// straight to global memory, so the result never depends on the table size.
// ---------------------------------------------------------------------------
constexpr int kHashSlots = 4096;        // 4096 x (4 + 24) B = 112 KB of LDS
constexpr int kScatterThreads = 1024;
constexpr int kMaxProbe = 64;
constexpr int32_t kEmpty = -1;

// MODE 0: v from tod, geometry recomputed; 1: fused diagonal normal operator;
// 2: v from tod, geometry read from the cache written by the gather.
template <typename T, typename MT, int MODE>
__global__ void __launch_bounds__(kScatterThreads)
k_scatter(PtArgs<T> a, const T *__restrict__ tod, const double *__restrict__ w_det,
          const MT *__restrict__ pmap, MapLayout pl, Tiling tl, double *__restrict__ q,
          MapLayout ql, GeomCache<T> gc) {
  __shared__ int32_t keys[kHashSlots];
  __shared__ double acc[3][kHashSlots];
  __shared__ double ta[kMaxTileSamples];
  for (int h = threadIdx.x; h < kHashSlots; h += kScatterThreads) {
    keys[h] = kEmpty;
    acc[0][h] = 0.0;
    acc[1][h] = 0.0;
    acc[2][h] = 0.0;
  }
  __syncthreads();

  const int64_t tile = tile_of_block(blockIdx.x, tl.blocks());
  const int64_t d0 = (tile / tl.n_tb) * tl.dets;
  const int64_t t0 = (tile % tl.n_tb) << tl.log2ts;
  const int32_t tsm = (1 << tl.log2ts) - 1;
  const int32_t nsamp = tl.dets << tl.log2ts;
  if constexpr (MODE != 2) fill_two_alpha(a, t0, tl.log2ts, ta, kScatterThreads);
  __syncthreads();
  volatile int32_t *vkeys = keys;
  for (int32_t s = threadIdx.x; s < nsamp; s += kScatterThreads) {
    const int64_t k = d0 + (s >> tl.log2ts);
    const int64_t i = t0 + (s & tsm);
    if (k >= a.n_det || i >= a.n_samp) continue;
    const int64_t off = k * a.n_samp + i;
    Geom<T> gm;
    if constexpr (MODE == 2) {
      gm.pix = gc.pix[off];
      if (gm.pix < 0) continue;
      gm.c = gc.c[off];
      gm.s = gc.s[off];
    } else {
      gm = sample_geom_ta(a, k, off, ta[s & tsm]);
      if (gm.pix < 0) continue;
    }
    const T g = gain_of(a, k);
    T v;
    if constexpr (MODE == 1) {
      MT I, Q, U;
      load_iqu(pmap, pl, gm.pix, I, Q, U);
      const T y = g * ((T)I + gm.c * (T)Q + gm.s * (T)U);
      v = g * ((T)w_det[k] * y);
    } else {
      v = g * tod[off];
      if (w_det) v = v * (T)w_det[k];
    }
    const double v0 = (double)v, v1 = (double)(v * gm.c), v2 = (double)(v * gm.s);
    uint32_t h = ((uint32_t)gm.pix * 2654435761u) >> (32 - 12);   // 12 = log2(kHashSlots)
    bool placed = false;
    for (int probe = 0; probe < kMaxProbe; ++probe) {
      int32_t cur = vkeys[h];
      if (cur == kEmpty) cur = atomicCAS(&keys[h], kEmpty, gm.pix);
      if (cur == kEmpty || cur == gm.pix) {
        placed = true;
        break;
      }
      h = (h + 1) & (kHashSlots - 1);
    }
    if (placed) {
      atomicAdd(&acc[0][h], v0);
      atomicAdd(&acc[1][h], v1);
      atomicAdd(&acc[2][h], v2);
    } else {
      const int64_t o = (int64_t)gm.pix * ql.ps;
      atomicAdd(&q[o], v0);
      atomicAdd(&q[o + ql.cs], v1);
      atomicAdd(&q[o + 2 * ql.cs], v2);
    }
  }
  __syncthreads();
  for (int h = threadIdx.x; h < kHashSlots; h += kScatterThreads) {
    const int32_t key = keys[h];
    if (key == kEmpty) continue;
    const int64_t o = (int64_t)key * ql.ps;
    atomicAdd(&q[o], acc[0][h]);
    atomicAdd(&q[o + ql.cs], acc[1][h]);
    atomicAdd(&q[o + 2 * ql.cs], acc[2][h]);
  }
}

template <typename T>
furax_status launch_scatter(const PtArgs<T> &a, const T *tod, const double *w_det,
                            const void *pmap, bool pmap_f64, MapLayout pl, double *q,
                            MapLayout ql, hipStream_t s, GeomCache<T> gc) {
  if (a.n_samp == 0) return FURAX_OK;
  const Tiling tl = make_tiling(a.n_det, a.n_samp, a.nside, 8192, 6);
  const dim3 grid((unsigned)tl.blocks()), blk(kScatterThreads);
  if (tod && gc.pix) {
    hipLaunchKernelGGL((k_scatter<T, double, 2>), grid, blk, 0, s, a, tod, w_det,
                       (const double *)nullptr, pl, tl, q, ql, gc);
  } else if (tod) {
    hipLaunchKernelGGL((k_scatter<T, double, 0>), grid, blk, 0, s, a, tod, w_det,
                       (const double *)nullptr, pl, tl, q, ql, gc);
  } else if (pmap_f64) {
    hipLaunchKernelGGL((k_scatter<T, double, 1>), grid, blk, 0, s, a, tod, w_det,
                       static_cast<const double *>(pmap), pl, tl, q, ql, gc);
  } else {
    hipLaunchKernelGGL((k_scatter<T, float, 1>), grid, blk, 0, s, a, tod, w_det,
                       static_cast<const float *>(pmap), pl, tl, q, ql, gc);
  }
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status launch_scatter<float>(const PtArgs<float> &, const float *, const double *,
                                            const void *, bool, MapLayout, double *, MapLayout,
                                            hipStream_t, GeomCache<float>);
template furax_status launch_scatter<double>(const PtArgs<double> &, const double *,
                                             const double *, const void *, bool, MapLayout,
                                             double *, MapLayout, hipStream_t,
                                             GeomCache<double>);

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
