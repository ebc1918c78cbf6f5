// Chi-square of the data model (Eq. (1) with T = 0), its gradient, and the
// vector-Jacobian product of the signal s = P(m; g, dpsi) used by the
// differentiable path (sections "Summary" and "Research Impact Statement":
// JAX autodiff, here a hand-written adjoint).
//
//   s[k,i]     = g_k s1[k,i],  s1 = I[p] + Q[p] cos 2 psi_eff + U[p] sin 2 psi_eff
//   ds/dm      : P (adjoint: P^T, a scatter-add)
//   ds/dg_k    : s1[k,i], the unit-gain signal
//   ds/ddpsi_k : g_k (-2 Q[p] sin 2 psi_eff + 2 U[p] cos 2 psi_eff)
//
// and, with r = d - s and u = N^-1 r (diagonal N), chi2 = r^T N^-1 r has
//   d chi2 / dm = -2 P^T (g u),  d chi2 / dg_k = -2 sum_i u s1,
//   d chi2 / ddpsi_k = -2 sum_i u g_k (-2 Q sin + 2 U cos).
//
// One kernel serves the three uses.  It walks the same detector x time tiles
// as P, expands the pointing once per sample (never stored), gathers the map,
// and in the same pass
//   * sums r u per tile (chi-square),
//   * adds the map contributions into an LDS hash of the tile's pixels,
//     flushed with one FP64 global atomic per touched pixel and Stokes value,
//   * reduces the per-detector gain and angle terms over each 64-sample group
//     of a detector with a wave shuffle tree, written once per group.
// Per-detector and chi-square partials are then summed in a fixed order, so
// those results are reproducible bit for bit; the map gradient's atomics make
// its last bits depend on scheduling.
#include <mutex>
#include <string>

#include "common.h"
#include "reduce.h"
#include "tiles.h"

namespace fx {

constexpr int kGradThreads = 1024;
constexpr int kGradGroupsMax = 256;     // 64-sample (or whole-row) groups per tile
constexpr int64_t kGradTileSamples = 16384;

enum GradMode { kModeChi2 = 0, kModeGrad = 1, kModeVjp = 2 };

// Tile of the gradient kernels: at most kGradTileSamples slots, so that a
// tile holds at most kGradGroupsMax groups of min(64, tile length) slots.
template <typename T>
static Tiling grad_tiling(const PtArgs<T> &a) {
  return tiling_for(a, kGradTileSamples);
}

// MODE kModeChi2: chi_part[tile] = sum r u, u_out = u (if given).
// MODE kModeGrad: the same, and the gradient of chi2 (scale -2 applied here
//                 for the map, in k_det_final for the detector terms).
// MODE kModeVjp:  u = tod (a cotangent), gradient terms with scale 1.
// grad_map: planar [3][npix] FP64, accumulated (or null); det_part:
// [2][n_det][n_tb] FP64 (or null): per time block, the unscaled per-detector
// sums of u s1 and u g ds/ddpsi.
template <typename T, typename MT, bool QUAT, int MODE>
__global__ void __launch_bounds__(kGradThreads)
k_grad_tile(PtArgs<T> a, const MT *__restrict__ m, int64_t npix, Tiling tl,
            const T *__restrict__ tod, const double *__restrict__ w_det, double map_scale,
            double *__restrict__ grad_map, double *__restrict__ det_part,
            double *__restrict__ chi_part, T *__restrict__ u_out) {
  constexpr int KB = QUAT ? 2 : kBatch;
  __shared__ int32_t keys[kHashSlots];
  __shared__ double acc[3][kHashSlots];
  __shared__ TileConsts tc;
  __shared__ Quat tq[QUAT ? kMaxTileDets : 1];
  __shared__ double2 turn4a[QUAT ? kMaxTileSamples : 1];
  __shared__ double grp[2][kGradGroupsMax];
  __shared__ double red[kGradThreads / 64];
  const bool want_map = grad_map != nullptr && MODE != kModeChi2;
  const bool want_det = det_part != nullptr && MODE != kModeChi2;
  if (want_map) {
    for (int h = threadIdx.x; h < kHashSlots; h += kGradThreads) {
      keys[h] = kEmpty;
      acc[0][h] = 0.0;
      acc[1][h] = 0.0;
      acc[2][h] = 0.0;
    }
  }
  int64_t dg, tb;
  tile_coords(tl, tile_of_block(blockIdx.x, tl.blocks()), dg, tb);
  const int64_t d0 = dg * tl.dets;
  const int64_t t0 = tb << tl.log2ts;
  const int32_t nsamp = tl.dets << tl.log2ts;
  const int32_t log2G = tl.log2ts < 6 ? tl.log2ts : 6;   // group: min(64, tile length) slots
  const int32_t G = 1 << log2G;
  load_tile_consts(a, w_det, tl, d0, t0, tc);
  if constexpr (QUAT) load_tile_quats(a, tl, d0, tq);
  __syncthreads();
  if constexpr (QUAT) {
    if (a.hwp && !a.dpsi) {
      load_tile_turns(tc, tl, turn4a);
      __syncthreads();
    }
  }
  const int lane = threadIdx.x & 63;
  double chi = 0.0;
  for (int32_t s0 = threadIdx.x; s0 < nsamp; s0 += KB * kGradThreads) {
    Slot sl[KB];
    int32_t px[KB];
    T c[KB], s[KB], dv[KB];
    if constexpr (QUAT) {
      Quat qb[KB];
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        sl[b] = slot_of(tl, d0, t0, s0 + b * kGradThreads, a.n_det, a.n_samp, tc.det);
        qb[b] = load_quat(a.qb, t0 + sl[b].il < a.n_samp ? t0 + sl[b].il : 0);
        dv[b] = ld_stream(tod + sl[b].off);
      }
#pragma unroll
      for (int b = 0; b < KB; ++b)
        quat_slot(a, tc, turn4a, sl[b], quat_dir(qmul(qb[b], tq[sl[b].kl])), px[b], c[b], s[b]);
    } else {
      T th[KB], ph[KB], ps[KB];
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        sl[b] = slot_of(tl, d0, t0, s0 + b * kGradThreads, a.n_det, a.n_samp, tc.det);
        th[b] = ld_stream(a.theta + sl[b].off);
        ph[b] = ld_stream(a.phi + sl[b].off);
        ps[b] = ld_stream(a.psi + sl[b].off);
        dv[b] = ld_stream(tod + sl[b].off);
      }
#pragma unroll
      for (int b = 0; b < KB; ++b) {
        px[b] = pixel_of(a, th[b], ph[b]);
        pol_weights(a, tc, sl[b], ps[b], c[b], s[b]);
      }
    }
    MT I[KB], Q[KB], U[KB];
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      int32_t tag;
      load_iqu<false>(m, npix, px[b] >= 0 ? px[b] : 0, I[b], Q[b], U[b], tag);
    }
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      const bool live = sl[b].in && px[b] >= 0;
      const T g = (T)tc.gain[sl[b].kl];
      const T s1 = live ? (T)I[b] + c[b] * (T)Q[b] + s[b] * (T)U[b] : (T)0;
      T u;
      if constexpr (MODE == kModeVjp) {
        u = sl[b].in ? dv[b] : (T)0;
      } else {
        const T r = sl[b].in ? dv[b] - g * s1 : (T)0;
        u = (T)tc.w[sl[b].kl] * r;
        chi += (double)r * (double)u;
        if (u_out && sl[b].in) st_stream(u_out + sl[b].off, u);
      }
      if constexpr (MODE != kModeChi2) {
        if (want_det) {
          // per-group sums of u s1 and u g (-2 Q sin + 2 U cos), fixed tree
          const T ds = live ? (T)(-2) * (T)Q[b] * s[b] + (T)2 * (T)U[b] * c[b] : (T)0;
          double e0 = live ? (double)(u * s1) : 0.0;
          double e1 = live ? (double)(u * (g * ds)) : 0.0;
          for (int off = G >> 1; off >= 1; off >>= 1) {
            e0 += __shfl_down(e0, off, G);
            e1 += __shfl_down(e1, off, G);
          }
          if ((lane & (G - 1)) == 0) {
            const int32_t gi = (s0 + b * kGradThreads) >> log2G;
            if (gi < kGradGroupsMax) {
              grp[0][gi] = e0;
              grp[1][gi] = e1;
            }
          }
        }
        if (want_map && live) {
          const T v = (T)map_scale * (g * u);
          hash_add(keys, acc, px[b], (double)v, (double)(v * c[b]), (double)(v * s[b]),
                   grad_map, MapLayout{npix, 1});
        }
      }
    }
  }
  // chi-square partial of the tile: wave sums, then the waves in order
  if (MODE != kModeVjp && chi_part) {
    double w = chi;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) w += __shfl_down(w, off, 64);
    if (lane == 0) red[threadIdx.x >> 6] = w;
  }
  __syncthreads();
  if (MODE != kModeVjp && chi_part && threadIdx.x == 0) {
    double t = 0.0;
    for (int j = 0; j < kGradThreads / 64; ++j) t += red[j];
    chi_part[blockIdx.x] = t;
  }
  if (MODE != kModeChi2 && want_det) {
    // detector kl's groups kl * gpd .. (kl + 1) * gpd - 1, summed in order
    const int32_t gpd = 1 << (tl.log2ts - log2G);
    for (int kl = threadIdx.x; kl < tl.dets; kl += kGradThreads) {
      if (d0 + kl >= a.n_det) continue;
      const int64_t k = tc.det[kl];
      double t0s = 0.0, t1s = 0.0;
      for (int j = 0; j < gpd; ++j) {
        t0s += grp[0][kl * gpd + j];
        t1s += grp[1][kl * gpd + j];
      }
      det_part[k * tl.n_tb + tb] = t0s;
      det_part[(a.n_det + k) * tl.n_tb + tb] = t1s;
    }
  }
  if (MODE != kModeChi2 && want_map) {
    for (int h = threadIdx.x; h < kHashSlots; h += kGradThreads) {
      const int32_t key = keys[h];
      if (key == kEmpty) continue;
      atomicAdd(&grad_map[key], acc[0][h]);
      atomicAdd(&grad_map[npix + key], acc[1][h]);
      atomicAdd(&grad_map[2 * npix + key], acc[2][h]);
    }
  }
}

// One workgroup per detector: gg[k] = scale sum_tb det_part[0][k][tb],
// gd[k] = scale sum_tb det_part[1][k][tb], each thread summing a strided
// share in order and the workgroup's shares combined by a fixed tree.
__global__ void __launch_bounds__(kBlock) k_det_final(int64_t n_det, int64_t n_tb, double scale,
                                                      const double *__restrict__ det_part,
                                                      double *__restrict__ gg,
                                                      double *__restrict__ gd) {
  __shared__ double red[2][kBlock];
  const int64_t k = blockIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t j = threadIdx.x; j < n_tb; j += kBlock) {
    s0 += det_part[k * n_tb + j];
    s1 += det_part[(n_det + k) * n_tb + j];
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  __syncthreads();
  for (int w = kBlock / 2; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (gg) gg[k] = scale * red[0][0];
    if (gd) gd[k] = scale * red[1][0];
  }
}

// One workgroup: out = sum of partial[0 .. count), in a fixed order.
__global__ void __launch_bounds__(kBlock) k_sum_to(const double *__restrict__ partial,
                                                   int64_t count, double *__restrict__ out) {
  __shared__ double red[kBlock];
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += kBlock) t += partial[i];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int w = kBlock / 2; w >= 1; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

template <typename T, typename MT, int MODE>
static void launch_grad(const PtArgs<T> &a, const MT *m, int64_t npix, const Tiling &tl,
                        const T *tod, const double *w_det, double map_scale, double *grad_map,
                        double *det_part, double *chi_part, T *u_out, hipStream_t s) {
  const dim3 grid((unsigned)tl.blocks()), blk(kGradThreads);
  if (a.qb)
    hipLaunchKernelGGL((k_grad_tile<T, MT, true, MODE>), grid, blk, 0, s, a, m, npix, tl, tod,
                       w_det, map_scale, grad_map, det_part, chi_part, u_out);
  else
    hipLaunchKernelGGL((k_grad_tile<T, MT, false, MODE>), grid, blk, 0, s, a, m, npix, tl, tod,
                       w_det, map_scale, grad_map, det_part, chi_part, u_out);
}

template <typename T, int MODE>
static void launch_grad_any(int32_t map_dt, const PtArgs<T> &a, const void *m, int64_t npix,
                            const Tiling &tl, const T *tod, const double *w_det, double map_scale,
                            double *grad_map, double *det_part, double *chi_part, T *u_out,
                            hipStream_t s) {
  if (map_dt == FURAX_F64)
    launch_grad<T, double, MODE>(a, static_cast<const double *>(m), npix, tl, tod, w_det,
                                 map_scale, grad_map, det_part, chi_part, u_out, s);
  else
    launch_grad<T, float, MODE>(a, static_cast<const float *>(m), npix, tl, tod, w_det, map_scale,
                                grad_map, det_part, chi_part, u_out, s);
}

// Scratch of the gradient passes: chi-square partials [tiles] and the
// per-detector partials [2][n_det][n_tb].
template <typename T>
static size_t grad_scratch_doubles(const PtArgs<T> &a, bool det) {
  const Tiling tl = grad_tiling(a);
  return (size_t)tl.blocks() + (det ? (size_t)2 * a.n_det * tl.n_tb : 0);
}

template <typename T>
furax_status chi2_impl(const furax_pointing *P, const furax_noise *N, int32_t map_dt,
                       const void *map, const T *tod, double *chi2_out, T *resid_w,
                       hipStream_t s) {
  if (P->n_samp == 0) return zero_async(chi2_out, sizeof(double), s);
  const int64_t npix = npix_of(P->nside);
  const PtArgs<T> a = pt_args<T>(P, nullptr);
  const Tiling tl = grad_tiling(a);
  DevBuf part;
  FX_TRY(part.alloc(sizeof(double) * grad_scratch_doubles(a, false), s));
  double *chi_part = static_cast<double *>(part.ptr);
  launch_grad_any<T, kModeChi2>(map_dt, a, map, npix, tl, tod, N->inv_var, 1.0, nullptr, nullptr,
                                chi_part, resid_w, s);
  FX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(kBlock), 0, s, chi_part, tl.blocks(), chi2_out);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status chi2_impl<float>(const furax_pointing *, const furax_noise *, int32_t,
                                       const void *, const float *, double *, float *,
                                       hipStream_t);
template furax_status chi2_impl<double>(const furax_pointing *, const furax_noise *, int32_t,
                                        const void *, const double *, double *, double *,
                                        hipStream_t);

// The gradient pass proper, shared by the chi-square gradient (MODE
// kModeGrad: u = N^-1 (d - P m), scale -2, chi2 written when chi2_out is
// given) and the VJP of a cotangent (kModeVjp, scale 1).
template <typename T, int MODE>
static furax_status grad_pass(const furax_pointing *P, const furax_noise *N, int32_t map_dt,
                              const void *map, const T *tod, double *chi2_out, double *grad_map,
                              double *grad_gain, double *grad_dpsi, hipStream_t s,
                              double *ext_scratch = nullptr, size_t ext_doubles = 0) {
  const double scale = MODE == kModeGrad ? -2.0 : 1.0;
  const bool det = grad_gain || grad_dpsi;
  if (P->n_samp == 0) {
    if (grad_gain) FX_TRY(zero_async(grad_gain, sizeof(double) * P->n_det, s));
    if (grad_dpsi) FX_TRY(zero_async(grad_dpsi, sizeof(double) * P->n_det, s));
    if (chi2_out) FX_TRY(zero_async(chi2_out, sizeof(double), s));
    return FURAX_OK;
  }
  const int64_t npix = npix_of(P->nside);
  const PtArgs<T> a = pt_args<T>(P, nullptr);
  const Tiling tl = grad_tiling(a);
  const size_t need = grad_scratch_doubles(a, det);
  DevBuf part;
  double *chi_part = ext_scratch;
  if (ext_scratch) {
    if (need > ext_doubles)
      return set_error(FURAX_EUNSUPPORTED,
                       "this problem needs " + std::to_string(need) +
                           " FP64 partial sums, more than the " + std::to_string(ext_doubles) +
                           " of the library's static scratch; use furax_chi2_grad");
  } else {
    FX_TRY(part.alloc(sizeof(double) * need, s));
    chi_part = static_cast<double *>(part.ptr);
  }
  double *det_part = det ? chi_part + tl.blocks() : nullptr;
  launch_grad_any<T, MODE>(map_dt, a, map, npix, tl, tod,
                           MODE == kModeGrad ? N->inv_var : nullptr, scale, grad_map, det_part,
                           MODE == kModeGrad ? chi_part : nullptr, nullptr, s);
  FX_HIP(hipGetLastError());
  if (det) {
    hipLaunchKernelGGL(k_det_final, dim3((unsigned)P->n_det), dim3(kBlock), 0, s, P->n_det,
                       tl.n_tb, scale, det_part, grad_gain, grad_dpsi);
    FX_HIP(hipGetLastError());
  }
  if (MODE == kModeGrad && chi2_out) {
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(kBlock), 0, s, chi_part, tl.blocks(), chi2_out);
    FX_HIP(hipGetLastError());
  }
  return FURAX_OK;
}

template <typename T>
furax_status vjp_impl(const furax_pointing *P, int32_t map_dt, const void *map, const T *cot,
                      double *grad_map, double *grad_gain, double *grad_dpsi, hipStream_t s) {
  return grad_pass<T, kModeVjp>(P, nullptr, map_dt, map, cot, nullptr, grad_map, grad_gain,
                                grad_dpsi, s);
}
template furax_status vjp_impl<float>(const furax_pointing *, int32_t, const void *,
                                      const float *, double *, double *, double *, hipStream_t);
template furax_status vjp_impl<double>(const furax_pointing *, int32_t, const void *,
                                       const double *, double *, double *, double *, hipStream_t);

template <typename T>
furax_status chi2_grad_impl(const furax_pointing *P, const furax_noise *N, int32_t map_dt,
                            const void *map, const T *tod, double *chi2_out, double *grad_map,
                            double *grad_gain, double *grad_dpsi, hipStream_t s) {
  return grad_pass<T, kModeGrad>(P, N, map_dt, map, tod, chi2_out, grad_map, grad_gain,
                                 grad_dpsi, s);
}
template furax_status chi2_grad_impl<float>(const furax_pointing *, const furax_noise *, int32_t,
                                            const void *, const float *, double *, double *,
                                            double *, double *, hipStream_t);
template furax_status chi2_grad_impl<double>(const furax_pointing *, const furax_noise *, int32_t,
                                             const void *, const double *, double *, double *,
                                             double *, double *, hipStream_t);

// ---------------------------------------------------------------------------
// The chi-square gradient without any allocation, for callers that cannot
// allocate (HIP graph capture, serving loops).  Its partial sums live in a
// file-scope device array: every GPU the library runs on holds its own copy
// (kNoAllocScratchDoubles FP64 values, 16 MiB) until the process ends.  Host
// code never passes the array's name to a kernel: its device address is looked
// up once per device with hipGetSymbolAddress, with that device current, and
// that address is what the kernels receive.  Every partial sum is written
// before it is read, so nothing needs clearing between calls; calls that
// overlap on one GPU share the array and race.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchDoubles = (size_t)1 << 21;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

static furax_status scratch_of_current_device(double **out) {
  int dev = 0;
  FX_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(FURAX_EUNSUPPORTED, "device ordinal beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    FX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return FURAX_OK;
}

template <typename T>
furax_status chi2_grad_noalloc_impl(const furax_pointing *P, const furax_noise *N,
                                    int32_t map_dt, const void *map, const T *tod,
                                    double *chi2_out, double *grad_map, double *grad_gain,
                                    double *grad_dpsi, hipStream_t s) {
  double *ws = nullptr;
  FX_TRY(scratch_of_current_device(&ws));
  return grad_pass<T, kModeGrad>(P, N, map_dt, map, tod, chi2_out, grad_map, grad_gain,
                                 grad_dpsi, s, ws, kNoAllocScratchDoubles);
}
template furax_status chi2_grad_noalloc_impl<float>(const furax_pointing *, const furax_noise *,
                                                    int32_t, const void *, const float *, double *,
                                                    double *, double *, double *, hipStream_t);
template furax_status chi2_grad_noalloc_impl<double>(const furax_pointing *, const furax_noise *,
                                                     int32_t, const void *, const double *,
                                                     double *, double *, double *, double *,
                                                     hipStream_t);

}  // namespace fx
