// Sample tiles shared by the kernels that expand the pointing per sample
// (P, the LDS-privatised P^T, the chi-square gradient): a workgroup owns a
// tile of detectors x consecutive samples, stages per-tile constants in LDS
// and keeps several samples' memory chains in flight per thread.
#pragma once

#include "common.h"

namespace fx {

// Block index -> logical tile, keeping consecutive logical tiles on the same
// XCD (workgroups are dealt round-robin over the 8 XCDs), so the map lines a
// tile touches are likely already in that XCD's L2.
__device__ __forceinline__ int64_t tile_of_block(int64_t bid, int64_t nblocks) {
  const int64_t per = nblocks / 8;
  if (per == 0 || bid >= per * 8) return bid;
  return (bid % 8) * per + bid / 8;
}

// Logical tile -> (detector group, time block).  Time blocks are the outer
// index and detector groups the inner one: the groups of one time block look
// at the same patch of sky (every group spans the whole focal plane), so they
// run next to each other on one XCD and share its L2 copy of the map lines,
// instead of each XCD walking one group along the scan and fetching the same
// lines again.
__device__ __forceinline__ void tile_coords(const Tiling &tl, int64_t tile, int64_t &dg,
                                            int64_t &tb) {
  tb = tile / tl.n_dg;
  dg = tile - tb * tl.n_dg;
}


// Samples per thread whose memory traffic is issued together.  A sample's
// work is a chain of dependent accesses (pointing -> pixel -> map value, or
// pixel -> hash slot); issuing the loads of kBatch samples before using any
// of them keeps kBatch chains in flight per thread instead of one.
constexpr int kBatch = 4;

// Where slot s of a tile lives: detector k, sample offset within the tile's
// time block, flat TOD offset.  Slots past the stream (ragged last time block
// or detector group) get offset 0, so their loads stay in bounds; their
// results are discarded.
struct Slot {
  int64_t k, off;
  int32_t kl, il;   // detector and sample index within the tile
  bool in;
};

__device__ __forceinline__ Slot slot_of(const Tiling &tl, int64_t d0, int64_t t0, int32_t s,
                                        int64_t n_det, int64_t n_samp,
                                        const int32_t *tile_det) {
  Slot r;
  r.kl = s >> tl.log2ts;
  r.il = s & ((1 << tl.log2ts) - 1);
  const int64_t i = t0 + r.il;
  r.in = s < (tl.dets << tl.log2ts) && d0 + r.kl < n_det && i < n_samp;
  r.k = r.in ? (int64_t)tile_det[r.kl] : 0;
  r.off = r.in ? r.k * n_samp + i : 0;
  return r;
}

// The detector taking tile position d0 + j (within n_det).
template <typename T>
__device__ __forceinline__ int64_t tile_detector(const PtArgs<T> &a, int64_t idx) {
  return a.det_perm ? (int64_t)a.det_perm[idx] : idx;
}

// Per-tile constants staged in LDS once per workgroup: the HWP term
// 2 alpha_i of each of the tile's samples and each detector's gain, angle
// offset and noise weight, so the per-sample work reads them from LDS.
constexpr int kMaxTileSamples = 1024;   // longest tile (2^10 samples per detector)

struct TileConsts {
  double two_alpha[kMaxTileSamples];
  double gain[kMaxTileDets], dpsi[kMaxTileDets], w[kMaxTileDets];
  int32_t det[kMaxTileDets];   // the detector at each tile position
};

template <typename T>
__device__ __forceinline__ void load_tile_consts(const PtArgs<T> &a, const double *w_det,
                                                 const Tiling &tl, int64_t d0, int64_t t0,
                                                 TileConsts &tc) {
  if (a.hwp) {
    for (int t = threadIdx.x; t < (1 << tl.log2ts); t += blockDim.x)
      tc.two_alpha[t] = 2.0 * hwp_alpha(t0 + t, a.hwp_num_mod, a.hwp_den, a.hwp_phase0);
  }
  for (int j = threadIdx.x; j < tl.dets; j += blockDim.x) {
    const int64_t k = d0 + j < a.n_det ? tile_detector(a, d0 + j) : 0;
    tc.det[j] = (int32_t)k;
    tc.gain[j] = a.gain ? a.gain[k] : 1.0;
    tc.dpsi[j] = a.dpsi ? a.dpsi[k] : 0.0;
    tc.w[j] = w_det ? w_det[k] : 1.0;
  }
}

// Polariser weights of a sample from its angle psi, its detector's angle
// offset and the HWP term: cos / sin of 2 (psi + dpsi_k + 2 alpha_i).
template <typename T>
__device__ __forceinline__ void pol_weights(const PtArgs<T> &a, const TileConsts &tc,
                                            const Slot &sl, T psi, T &c, T &s) {
#pragma clang fp contract(off)
  double pe = (double)psi;
  if (a.dpsi) pe = pe + tc.dpsi[sl.kl];
  if (a.hwp) pe = pe + tc.two_alpha[sl.il];
  weights(2.0 * pe, c, s);
}

template <typename T>
__device__ __forceinline__ int32_t pixel_of(const PtArgs<T> &a, T theta, T phi) {
  int32_t p = ang2pix_ring(a.nside, (double)theta, (double)phi);
  if (p >= 0 && a.valid && !a.valid[p]) p = -1;
  return p;
}

// Quaternion pointing: the tile's detector attitudes are staged in LDS next to
// the other per-detector constants; a slot's geometry then needs its boresight
// attitude (shared by all detectors of the time block, so cache-resident) and
// one Hamilton product.
template <typename T>
__device__ __forceinline__ void load_tile_quats(const PtArgs<T> &a, const Tiling &tl, int64_t d0,
                                                Quat *tq) {
  for (int j = threadIdx.x; j < tl.dets; j += blockDim.x)
    tq[j] = load_quat(a.qd, d0 + j < a.n_det ? tile_detector(a, d0 + j) : 0);
}

// With a HWP and no angle offsets the turn of the polariser weights is by
// 4 alpha_i alone: its cosine and sine are tabulated per tile sample in LDS
// (turn4a), so no sample evaluates a sine or cosine.
__device__ __forceinline__ void load_tile_turns(const TileConsts &tc, const Tiling &tl,
                                                double2 *turn4a) {
  for (int t = threadIdx.x; t < (1 << tl.log2ts); t += blockDim.x) {
    double sn, cs;
    sincos(2.0 * tc.two_alpha[t], &sn, &cs);
    turn4a[t] = make_double2(cs, sn);
  }
}

template <typename T>
__device__ __forceinline__ void quat_slot(const PtArgs<T> &a, const TileConsts &tc,
                                          const double2 *turn4a, const Slot &sl,
                                          const QuatDir &d, int32_t &pix, T &c, T &s) {
#pragma clang fp contract(off)
  pix = zphi2pix_ring(a.nside, d.z, d.phi);
  if (pix >= 0 && a.valid && !a.valid[pix]) pix = -1;
  if (a.hwp && !a.dpsi) {
    double c2, s2;
    quat_c2s2(d, c2, s2);
    const double2 tn = turn4a[sl.il];
    turn_weights(c2, s2, (T)tn.x, (T)tn.y, c, s);
    return;
  }
  double beta = a.dpsi ? tc.dpsi[sl.kl] : 0.0;
  if (a.hwp) beta = beta + tc.two_alpha[sl.il];
  quat_weights(d, a.dpsi || a.hwp, beta, c, s);
}

// Stokes values of pixel pix of a map: planar [3][npix] (IL = false, cs =
// npix) or interleaved [npix][4] (IL = true; one 16- or 32-byte load, whose
// 4th lane -- a tag, the pixel's nested index as integer bits in the solver's
// maps -- comes with it).
template <bool IL, typename MT>
__device__ __forceinline__ void load_iqu(const MT *__restrict__ m, int64_t cs, int32_t pix,
                                         MT &I, MT &Q, MT &U, int32_t &tag) {
  tag = 0;
  if constexpr (IL) {
    if constexpr (sizeof(MT) == 4) {
      const float4 v = reinterpret_cast<const float4 *>(m)[pix];
      I = v.x;
      Q = v.y;
      U = v.z;
      tag = __float_as_int(v.w);
    } else {
      const double2 *q = reinterpret_cast<const double2 *>(m) + 2 * (int64_t)pix;
      const double2 v0 = q[0], v1 = q[1];
      I = v0.x;
      Q = v0.y;
      U = v1.x;
      tag = (int32_t)__double_as_longlong(v1.y);
    }
  } else {
    I = m[pix];
    Q = m[cs + pix];
    U = m[2 * cs + pix];
  }
}

// Tile shape of the pointing kernels.  A tile's time runs are at least 128
// bytes of each pointing plane, so a wave's loads cover whole cache lines.
inline Tiling tiling_for(const PtArgs<float> &a, int64_t target) {
  return make_tiling(a.n_det, a.n_samp, a.nside, target, 5);
}
inline Tiling tiling_for(const PtArgs<double> &a, int64_t target) {
  return make_tiling(a.n_det, a.n_samp, a.nside, target, 4);
}

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

__device__ __forceinline__ void hash_add(int32_t *keys, double (*acc)[kHashSlots], int32_t pix,
                                         double v0, double v1, double v2, double *__restrict__ q,
                                         const MapLayout &ql) {
  volatile int32_t *vkeys = keys;
  uint32_t h = ((uint32_t)pix * 2654435761u) >> (32 - 12);   // 12 = log2(kHashSlots)
  bool placed = false;
  for (int probe = 0; probe < kMaxProbe; ++probe) {
    int32_t cur = vkeys[h];
    if (cur == kEmpty) cur = atomicCAS(&keys[h], kEmpty, pix);
    if (cur == kEmpty || cur == pix) {
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
    const int64_t o = (int64_t)pix * ql.ps;
    atomicAdd(&q[o], v0);
    atomicAdd(&q[o + ql.cs], v1);
    atomicAdd(&q[o + 2 * ql.cs], v2);
  }
}

}  // namespace fx
