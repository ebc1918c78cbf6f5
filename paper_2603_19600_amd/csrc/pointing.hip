// Pointing operator kernels: ang2pix, P (gather), P^T (scatter-add), the fused
// diagonal-noise normal operator and the block-Jacobi accumulation.
//
// Every kernel expands the pointing on the fly (PointingOperator, section
// "Software Design", "Map-making classes"): theta/phi/psi are streamed once,
// coalesced along time -- or, with quaternion pointing, each sample's attitude
// is composed from the boresight's and its detector's -- and the pixel and the
// polariser weights are rebuilt in registers; nothing per-sample is stored.
#include "common.h"
#include "tiles.h"

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
  t.dets = (int32_t)std::min<int64_t>(n_det, kMaxTileDets);
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


// ---------------------------------------------------------------------------
// P: tod[k,i] = g_k (I[p] + c Q[p] + s U[p]).  With pix_out, the pixel of
// every sample (-1 when flagged) is also written, for the P^T that follows in
// the same normal-operator application.
// ---------------------------------------------------------------------------
constexpr int kApplyThreads = 256;

template <typename T, typename MT, bool IL, bool QUAT>
__global__ void __launch_bounds__(kApplyThreads) k_apply(PtArgs<T> a, const MT *__restrict__ map,
                                                         int64_t map_cs, Tiling tl,
                                                         T *__restrict__ tod,
                                                         int32_t *__restrict__ pix_out,
                                                         uint16_t *__restrict__ local_out,
                                                         int32_t local_mask) {
  __shared__ TileConsts tc;
  __shared__ Quat tq[QUAT ? kMaxTileDets : 1];
  __shared__ double2 turn4a[QUAT ? kMaxTileSamples : 1];
  int64_t dg, tb;
  tile_coords(tl, tile_of_block(blockIdx.x, tl.blocks()), dg, tb);
  const int64_t d0 = dg * tl.dets;
  const int64_t t0 = tb << tl.log2ts;
  const int32_t nsamp = tl.dets << tl.log2ts;
  load_tile_consts(a, nullptr, tl, d0, t0, tc);
  if constexpr (QUAT) load_tile_quats(a, tl, d0, tq);
  __syncthreads();
  if constexpr (QUAT) {
    if (a.hwp && !a.dpsi) {
      load_tile_turns(tc, tl, turn4a);
      __syncthreads();
    }
  }
  // quaternion attitudes take more registers per sample in flight: two
  // samples per thread there (four waves per SIMD instead of three) measured
  // faster; the FP64 angle planes keep four (three waves)
  constexpr int KB = QUAT ? 2 : kBatch;
  for (int32_t s0 = threadIdx.x; s0 < nsamp; s0 += KB * kApplyThreads) {
    Slot sl[KB];
    int32_t px[KB], tag[KB];
    T c[KB], s[KB];
    if constexpr (QUAT) {
      Quat qb[KB];
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        sl[b] = slot_of(tl, d0, t0, s0 + b * kApplyThreads, a.n_det, a.n_samp, tc.det);
        qb[b] = load_quat(a.qb, t0 + sl[b].il < a.n_samp ? t0 + sl[b].il : 0);
      }
#pragma unroll
      for (int b = 0; b < KB; ++b)
        quat_slot(a, tc, turn4a, sl[b], quat_dir(qmul(qb[b], tq[sl[b].kl])), px[b], c[b], s[b]);
    } else {
      T th[KB], ph[KB], ps[KB];
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        sl[b] = slot_of(tl, d0, t0, s0 + b * kApplyThreads, a.n_det, a.n_samp, tc.det);
        th[b] = ld_stream(a.theta + sl[b].off);
        ph[b] = ld_stream(a.phi + sl[b].off);
        ps[b] = ld_stream(a.psi + sl[b].off);
      }
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        px[b] = pixel_of(a, th[b], ph[b]);
        pol_weights(a, tc, sl[b], ps[b], c[b], s[b]);
      }
    }
    MT I[KB], Q[KB], U[KB];
#pragma unroll
    for (int b = 0; b < KB; ++b)
      load_iqu<IL>(map, map_cs, px[b] >= 0 ? px[b] : 0, I[b], Q[b], U[b], tag[b]);
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      if (!sl[b].in) continue;
      const T y = (T)I[b] + c[b] * (T)Q[b] + s[b] * (T)U[b];
      st_stream(tod + sl[b].off, px[b] >= 0 ? (T)tc.gain[sl[b].kl] * y : (T)0);
      if (pix_out) st_stream(pix_out + sl[b].off, px[b]);
      if (local_out)
        st_stream(local_out + sl[b].off,
                  (uint16_t)(px[b] >= 0 ? (uint16_t)(tag[b] & local_mask) : 0xffff));
    }
  }
}


template <typename T, typename MT, bool QUAT>
static void launch_apply(const PtArgs<T> &a, const MT *m, MapLayout ml, bool il, const Tiling &tl,
                         T *tod, hipStream_t s, int32_t *pix_out, uint16_t *local_out,
                         int32_t local_mask) {
  const dim3 grid((unsigned)tl.blocks()), blk(kApplyThreads);
  if (il)
    hipLaunchKernelGGL((k_apply<T, MT, true, QUAT>), grid, blk, 0, s, a, m, ml.cs, tl, tod,
                       pix_out, local_out, local_mask);
  else
    hipLaunchKernelGGL((k_apply<T, MT, false, QUAT>), grid, blk, 0, s, a, m, ml.cs, tl, tod,
                       pix_out, local_out, local_mask);
}

template <typename T>
furax_status launch_pointing_apply(const PtArgs<T> &a, const void *map, bool map_f64,
                                   MapLayout ml, T *tod, hipStream_t s, int32_t *pix_out,
                                   uint16_t *local_out, int32_t local_mask) {
  if (a.n_samp == 0) return FURAX_OK;
  const Tiling tl = tiling_for(a, 4096);
  const bool il = ml.ps == 4;
  if (a.qb) {
    if (map_f64)
      launch_apply<T, double, true>(a, static_cast<const double *>(map), ml, il, tl, tod, s,
                                    pix_out, local_out, local_mask);
    else
      launch_apply<T, float, true>(a, static_cast<const float *>(map), ml, il, tl, tod, s,
                                   pix_out, local_out, local_mask);
  } else {
    if (map_f64)
      launch_apply<T, double, false>(a, static_cast<const double *>(map), ml, il, tl, tod, s,
                                     pix_out, local_out, local_mask);
    else
      launch_apply<T, float, false>(a, static_cast<const float *>(map), ml, il, tl, tod, s,
                                    pix_out, local_out, local_mask);
  }
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status launch_pointing_apply<float>(const PtArgs<float> &, const void *, bool,
                                                   MapLayout, float *, hipStream_t, int32_t *,
                                                   uint16_t *, int32_t);
template furax_status launch_pointing_apply<double>(const PtArgs<double> &, const void *, bool,
                                                    MapLayout, double *, hipStream_t, int32_t *,
                                                    uint16_t *, int32_t);

// q(c, pix) += v (1, cos, sin) over the tile's samples, where
//   MODE 0: v = g_k w_k tod[k,i], geometry recomputed from the pointing;
//   MODE 1: v = g_k w_k g_k (P p)[k,i], the fused diagonal-noise normal
//           operator (p read from pmap, interleaved when IL);
//   MODE 2: v = g_k w_k tod[k,i], pixel read from pix_in (written by the P of
//           the same application), weights recomputed from psi.
// w_k = w_det[k], or 1 when w_det is null.
template <typename T, typename MT, int MODE, bool IL, bool QUAT>
__global__ void __launch_bounds__(kScatterThreads)
k_scatter(PtArgs<T> a, const T *__restrict__ tod, const double *__restrict__ w_det,
          const MT *__restrict__ pmap, int64_t p_cs, Tiling tl, double *__restrict__ q,
          MapLayout ql, const int32_t *__restrict__ pix_in) {
  // quaternion samples carry a boresight attitude each: fewer in flight per
  // thread keeps the 1024-thread workgroup within its register budget
  constexpr int KB = QUAT ? 2 : kBatch;
  __shared__ int32_t keys[kHashSlots];
  __shared__ double acc[3][kHashSlots];
  __shared__ TileConsts tc;
  __shared__ Quat tq[QUAT ? kMaxTileDets : 1];
  __shared__ double2 turn4a[QUAT ? kMaxTileSamples : 1];
  for (int h = threadIdx.x; h < kHashSlots; h += kScatterThreads) {
    keys[h] = kEmpty;
    acc[0][h] = 0.0;
    acc[1][h] = 0.0;
    acc[2][h] = 0.0;
  }
  int64_t dg, tb;
  tile_coords(tl, tile_of_block(blockIdx.x, tl.blocks()), dg, tb);
  const int64_t d0 = dg * tl.dets;
  const int64_t t0 = tb << tl.log2ts;
  const int32_t nsamp = tl.dets << tl.log2ts;
  load_tile_consts(a, w_det, tl, d0, t0, tc);
  if constexpr (QUAT) load_tile_quats(a, tl, d0, tq);
  __syncthreads();
  if constexpr (QUAT) {
    if (a.hwp && !a.dpsi) {
      load_tile_turns(tc, tl, turn4a);
      __syncthreads();
    }
  }

  for (int32_t s0 = threadIdx.x; s0 < nsamp; s0 += KB * kScatterThreads) {
    Slot sl[KB];
    int32_t px[KB];
    T v[KB], c[KB], s[KB];
    if constexpr (QUAT) {
      Quat qb[KB];
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        sl[b] = slot_of(tl, d0, t0, s0 + b * kScatterThreads, a.n_det, a.n_samp, tc.det);
        qb[b] = load_quat(a.qb, t0 + sl[b].il < a.n_samp ? t0 + sl[b].il : 0);
        if constexpr (MODE == 2) px[b] = pix_in[sl[b].off];
        if constexpr (MODE != 1) v[b] = ld_stream(tod + sl[b].off);
      }
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        int32_t pq;
        quat_slot(a, tc, turn4a, sl[b], quat_dir(qmul(qb[b], tq[sl[b].kl])), pq, c[b], s[b]);
        if constexpr (MODE != 2) px[b] = pq;
        if (!sl[b].in) px[b] = -1;
      }
    } else {
      T th[KB], ph[KB], ps[KB];
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        sl[b] = slot_of(tl, d0, t0, s0 + b * kScatterThreads, a.n_det, a.n_samp, tc.det);
        ps[b] = ld_stream(a.psi + sl[b].off);
        if constexpr (MODE == 2) {
          px[b] = pix_in[sl[b].off];
        } else {
          th[b] = ld_stream(a.theta + sl[b].off);
          ph[b] = ld_stream(a.phi + sl[b].off);
        }
        if constexpr (MODE != 1) v[b] = ld_stream(tod + sl[b].off);
      }
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        if constexpr (MODE != 2) px[b] = pixel_of(a, th[b], ph[b]);
        if (!sl[b].in) px[b] = -1;
        pol_weights(a, tc, sl[b], ps[b], c[b], s[b]);
      }
    }
    if constexpr (MODE == 1) {
      MT I[KB], Q[KB], U[KB];
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        int32_t tag;
        load_iqu<IL>(pmap, p_cs, px[b] >= 0 ? px[b] : 0, I[b], Q[b], U[b], tag);
      }
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        const T g = (T)tc.gain[sl[b].kl];
        const T y = g * ((T)I[b] + c[b] * (T)Q[b] + s[b] * (T)U[b]);
        v[b] = g * ((T)tc.w[sl[b].kl] * y);
      }
    } else {
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        v[b] = (T)tc.gain[sl[b].kl] * v[b];
        if (w_det) v[b] = v[b] * (T)tc.w[sl[b].kl];
      }
    }
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      if (px[b] < 0) continue;
      hash_add(keys, acc, px[b], (double)v[b], (double)(v[b] * c[b]), (double)(v[b] * s[b]), q,
               ql);
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

template <typename T, bool QUAT>
static void launch_scatter_k(const PtArgs<T> &a, const T *tod, const double *w_det,
                             const void *pmap, bool pmap_f64, MapLayout pl, double *q,
                             MapLayout ql, hipStream_t s, const int32_t *pix_in) {
  const Tiling tl = tiling_for(a, 8192);
  const dim3 grid((unsigned)tl.blocks()), blk(kScatterThreads);
  const double *nul = nullptr;
  if (tod && pix_in) {
    hipLaunchKernelGGL((k_scatter<T, double, 2, false, QUAT>), grid, blk, 0, s, a, tod, w_det,
                       nul, int64_t(0), tl, q, ql, pix_in);
  } else if (tod) {
    hipLaunchKernelGGL((k_scatter<T, double, 0, false, QUAT>), grid, blk, 0, s, a, tod, w_det,
                       nul, int64_t(0), tl, q, ql, pix_in);
  } else {
    const bool il = pl.ps == 4;
    if (pmap_f64) {
      const double *m = static_cast<const double *>(pmap);
      if (il)
        hipLaunchKernelGGL((k_scatter<T, double, 1, true, QUAT>), grid, blk, 0, s, a, tod,
                           w_det, m, pl.cs, tl, q, ql, pix_in);
      else
        hipLaunchKernelGGL((k_scatter<T, double, 1, false, QUAT>), grid, blk, 0, s, a, tod,
                           w_det, m, pl.cs, tl, q, ql, pix_in);
    } else {
      const float *m = static_cast<const float *>(pmap);
      if (il)
        hipLaunchKernelGGL((k_scatter<T, float, 1, true, QUAT>), grid, blk, 0, s, a, tod,
                           w_det, m, pl.cs, tl, q, ql, pix_in);
      else
        hipLaunchKernelGGL((k_scatter<T, float, 1, false, QUAT>), grid, blk, 0, s, a, tod,
                           w_det, m, pl.cs, tl, q, ql, pix_in);
    }
  }
}

template <typename T>
furax_status launch_scatter(const PtArgs<T> &a, const T *tod, const double *w_det,
                            const void *pmap, bool pmap_f64, MapLayout pl, double *q,
                            MapLayout ql, hipStream_t s, const int32_t *pix_in) {
  if (a.n_samp == 0) return FURAX_OK;
  if (a.qb)
    launch_scatter_k<T, true>(a, tod, w_det, pmap, pmap_f64, pl, q, ql, s, pix_in);
  else
    launch_scatter_k<T, false>(a, tod, w_det, pmap, pmap_f64, pl, q, ql, s, pix_in);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status launch_scatter<float>(const PtArgs<float> &, const float *, const double *,
                                            const void *, bool, MapLayout, double *, MapLayout,
                                            hipStream_t, const int32_t *);
template furax_status launch_scatter<double>(const PtArgs<double> &, const double *,
                                             const double *, const void *, bool, MapLayout,
                                             double *, MapLayout, hipStream_t, const int32_t *);

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
// Inverse of each pixel's symmetric 3x3 block from its Cholesky factorisation
// M = L L^T (the blocks are sums of w (1,c,s)^T (1,c,s), w > 0, so positive
// semi-definite), and its 1-norm reciprocal condition number.  The Cholesky
// route is backward stable: a block that is singular in exact arithmetic (all
// of the pixel's samples at one polariser angle, or at two angles pi/2 apart)
// meets a pivot that is not positive or of rounding size, so its inverse is
// huge and its rcond tiny, where the adjugate formula's cofactors would all be
// rounding noise with a ratio of order one.  A non-positive pivot gives
// inverse 0 and rcond 0.  M^-1 = L^-T L^-1, L^-1 by forward substitution.
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
    const double l11 = sqrt(a);
    const double l21 = b / l11;
    const double l31 = c / l11;
    const double t22 = d - l21 * l21;
    const double l22 = sqrt(t22);
    const double l32 = (e - l31 * l21) / l22;
    const double t33 = f - l31 * l31 - l32 * l32;
    const double l33 = sqrt(t33);
    const double i11 = 1.0 / l11, i22 = 1.0 / l22, i33 = 1.0 / l33;
    const double i21 = -(l21 * i11) * i22;
    const double i32 = -(l32 * i22) * i33;
    const double i31 = -(l31 * i11 + l32 * i21) * i33;
    double ia = i11 * i11 + i21 * i21 + i31 * i31;
    double ib = i21 * i22 + i31 * i32;
    double ic = i31 * i33;
    double id = i22 * i22 + i32 * i32;
    double ie = i32 * i33;
    double iff = i33 * i33;
    const bool fin = ia - ia == 0.0 && ib - ib == 0.0 && ic - ic == 0.0 && id - id == 0.0 &&
                     ie - ie == 0.0 && iff - iff == 0.0;
    const bool chol = a > 0.0 && t22 > 0.0 && t33 > 0.0 && fin;
    if (!chol) ia = ib = ic = id = ie = iff = 0.0;
    const double n1 = fmax(fmax(fabs(a) + fabs(b) + fabs(c), fabs(b) + fabs(d) + fabs(e)),
                           fabs(c) + fabs(e) + fabs(f));
    const double n1i = fmax(fmax(fabs(ia) + fabs(ib) + fabs(ic), fabs(ib) + fabs(id) + fabs(ie)),
                            fabs(ic) + fabs(ie) + fabs(iff));
    double rc = 1.0 / (n1 * n1i);
    if (!chol || !(rc - rc == 0.0)) rc = 0.0;
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
