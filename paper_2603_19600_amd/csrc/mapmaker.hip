// Normal operator A = P^T N^-1 P and the block-Jacobi PCG map-maker.
//
// The solver is the iterative inverse of Table 1 (A.I(solver, preconditioner))
// applied to the estimator of Eq. (2) with T = 0, preconditioned by the
// block-Jacobi preconditioner of "Map-making classes".  All scalars of the
// recurrence (<p,q>, alpha, <r,z>, beta, |r|) live in device memory and are
// produced by deterministic two-pass FP64 reductions, so an iteration never
// waits on the host; a device-side stop flag freezes the iterate on
// convergence or breakdown.
#include <cmath>
#include <cstring>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "common.h"
#include "reduce.h"

namespace fx {

template <typename T>
furax_status launch_bj_build(const PtArgs<T> &a, const double *w_det, double *M6, int32_t *hits,
                             hipStream_t s);
furax_status launch_bj_invert(int64_t npix, const double *M6, const int32_t *hits,
                              double rcond_min, int32_t min_hits, const uint8_t *force_valid,
                              double *Minv6, uint8_t *valid, double *rcond, hipStream_t s);


struct PcgScalars {
  double rz, pq, alpha, beta, rr, bnorm, rel, rtol;
  int32_t stop;      // 0 running, 1 rtol reached, 2 breakdown
  int32_t iters;
};

__device__ __forceinline__ bool finite_pos(double v) { return v > 0.0 && v - v == 0.0; }

// partial[block] = this block's share of <p, q>, p planar [3][npix], q interleaved [npix][4].
//
// The vector passes touch valid pixels only.  On the others x, r, z and p are
// 0 from the initialisation on and stay 0 (p = 0 there gives <p, q> nothing),
// and in ring order the unobserved pixels come in long stretches, so whole
// waves skip their loads and stores: the passes move the observed part of the
// sky instead of all of it.
__global__ void __launch_bounds__(kBlock) k_dot_pq(int64_t npix, const double *__restrict__ p,
                                                   const double *__restrict__ q,
                                                   const uint8_t *__restrict__ valid,
                                                   double *__restrict__ partial) {
  double v[1] = {0.0};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npix; i += stride) {
    if (!valid[i]) continue;
    v[0] += p[i] * q[4 * i] + p[npix + i] * q[4 * i + 1] + p[2 * npix + i] * q[4 * i + 2];
  }
  block_sum<1>(v, partial + blockIdx.x, kRedBlocks);
}

// After the initial residual: partial[0] = <r,z>, partial[1] = <b,b>.
__global__ void __launch_bounds__(kBlock) k_init_final(const double *__restrict__ partial,
                                                       double rtol, PcgScalars *sc, double *hist) {
  double v[2];
  final_sum<2>(partial, v);
  if (threadIdx.x != 0) return;
  sc->rz = v[0];
  sc->rtol = rtol;
  sc->bnorm = sqrt(v[1]);
  sc->iters = 0;
  sc->stop = 0;
  // b = 0 is solved by x = 0; a non-finite or non-positive <r,z> is a breakdown
  sc->rel = v[1] == 0.0 ? 0.0 : 1.0;
  if (hist) hist[0] = sc->rel;
  if (v[1] == 0.0) sc->stop = 1;
  else if (!finite_pos(v[0]) || !finite_pos(v[1])) sc->stop = 2;
}

__global__ void __launch_bounds__(kBlock) k_pq_final(const double *__restrict__ partial,
                                                     PcgScalars *sc) {
  double v[1];
  final_sum<1>(partial, v);
  if (threadIdx.x != 0 || sc->stop) return;
  sc->pq = v[0];
  if (!finite_pos(v[0])) sc->stop = 2;
  else sc->alpha = sc->rz / v[0];
}

// x += alpha p; r -= alpha q (q interleaved); z = Minv r; partials of <r,z> and <r,r>.
// The operator kernels do not flag samples of invalid pixels; q there holds
// contributions that flagging would have dropped, so r is kept at 0 on invalid
// pixels -- they are skipped, and x, r, z keep the 0 of the initialisation
// (p, z and Minv are 0 there, so the valid pixels see exactly the flagged
// operator).
__global__ void __launch_bounds__(kBlock) k_update1(int64_t npix, double *__restrict__ x,
                                                    double *__restrict__ r,
                                                    const double *__restrict__ p,
                                                    const double *__restrict__ q,
                                                    const double *__restrict__ Mi,
                                                    const uint8_t *__restrict__ valid,
                                                    double *__restrict__ z,
                                                    const PcgScalars *__restrict__ sc,
                                                    double *__restrict__ partial) {
  if (sc->stop) return;
  const double alpha = sc->alpha;
  double v[2] = {0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npix; i += stride) {
    if (!valid[i]) continue;
    double rr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t j = c * npix + i;
      x[j] = x[j] + alpha * p[j];
      rr[c] = r[j] - alpha * q[4 * i + c];
      r[j] = rr[c];
    }
    const double a = Mi[i], b = Mi[npix + i], cc = Mi[2 * npix + i];
    const double d = Mi[3 * npix + i], e = Mi[4 * npix + i], f = Mi[5 * npix + i];
    const double z0 = a * rr[0] + b * rr[1] + cc * rr[2];
    const double z1 = b * rr[0] + d * rr[1] + e * rr[2];
    const double z2 = cc * rr[0] + e * rr[1] + f * rr[2];
    z[i] = z0;
    z[npix + i] = z1;
    z[2 * npix + i] = z2;
    v[0] += rr[0] * z0 + rr[1] * z1 + rr[2] * z2;
    v[1] += rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2];
  }
  block_sum<2>(v, partial + blockIdx.x, kRedBlocks);
}

__global__ void __launch_bounds__(kBlock) k_rz_final(const double *__restrict__ partial,
                                                     PcgScalars *sc, double *hist, int32_t nhist) {
  double v[2];
  final_sum<2>(partial, v);
  if (threadIdx.x != 0 || sc->stop) return;
  const int32_t it = sc->iters + 1;
  sc->iters = it;
  sc->rr = v[1];
  const double rel = sqrt(v[1]) / sc->bnorm;
  sc->rel = rel;
  if (hist && it < nhist) hist[it] = rel;
  if (rel <= sc->rtol) {
    sc->stop = 1;
  } else if (!finite_pos(v[0])) {
    sc->stop = 2;
  } else {
    sc->beta = v[0] / sc->rz;
    sc->rz = v[0];
  }
}

// p = z + beta p, and its interleaved gather copy pg in the path's precision
// (valid pixels; p and pg stay 0 on the others).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_update2(int64_t npix, double *__restrict__ p,
                                                    const double *__restrict__ z,
                                                    T *__restrict__ pg,
                                                    const uint8_t *__restrict__ valid,
                                                    const PcgScalars *__restrict__ sc) {
  if (sc->stop) return;
  const double beta = sc->beta;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npix; i += stride) {
    if (!valid[i]) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = z[c * npix + i] + beta * p[c * npix + i];
      p[c * npix + i] = v;
      pg[4 * i + c] = (T)v;
    }
  }
}

// The 4th lane of pixel i of an interleaved gather map carries a tag as
// integer bits: the pixel's nested index when tag is given (read back by P to
// label each sample with its superpixel offset), else 0.
template <typename T>
__device__ __forceinline__ void set_tag(T *g, int64_t i, const int32_t *tag) {
  const int32_t v = tag ? tag[i] : 0;
  if constexpr (sizeof(T) == 8) reinterpret_cast<int64_t *>(g)[4 * i + 3] = v;
  else reinterpret_cast<int32_t *>(g)[4 * i + 3] = v;
}

// z = Minv r (initial), r = b on valid pixels (0 elsewhere), p = z, x = 0;
// partials of <r,z>, <b,b>.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_init_vectors(int64_t npix, const double *__restrict__ b,
                                                         const uint8_t *__restrict__ valid,
                                                         double *__restrict__ x,
                                                         double *__restrict__ r,
                                                         double *__restrict__ z,
                                                         double *__restrict__ p,
                                                         T *__restrict__ pg,
                                                         const int32_t *__restrict__ tag,
                                                         const double *__restrict__ Mi,
                                                         double *__restrict__ partial) {
  double v[2] = {0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npix; i += stride) {
    double rr[3];
    const bool ok = valid[i] != 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rr[c] = ok ? b[c * npix + i] : 0.0;
      r[c * npix + i] = rr[c];
      x[c * npix + i] = 0.0;
    }
    const double a = Mi[i], bb = Mi[npix + i], cc = Mi[2 * npix + i];
    const double d = Mi[3 * npix + i], e = Mi[4 * npix + i], f = Mi[5 * npix + i];
    const double zz[3] = {a * rr[0] + bb * rr[1] + cc * rr[2], bb * rr[0] + d * rr[1] + e * rr[2],
                          cc * rr[0] + e * rr[1] + f * rr[2]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      z[c * npix + i] = zz[c];
      p[c * npix + i] = zz[c];
      pg[4 * i + c] = (T)zz[c];
      v[0] += rr[c] * zz[c];
      v[1] += rr[c] * rr[c];
    }
    set_tag(pg, i, tag);
  }
  block_sum<2>(v, partial + blockIdx.x, kRedBlocks);
}

__global__ void k_diag_weights(int64_t n_det, const double *__restrict__ inv_var,
                               const double *__restrict__ lags, int64_t lag_stride,
                               double *__restrict__ w) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_det) return;
  w[k] = inv_var ? inv_var[k] : lags[k * lag_stride];
}

static int64_t map_blocks(int64_t n) {
  return std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, kRedBlocks));
}

// ---------------------------------------------------------------------------
// Normal operator.
// ---------------------------------------------------------------------------
static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct NormalLayout {
  size_t spec = 0, y = 0, z = 0, pg = 0, qi = 0, wdet = 0, gpix = 0, total = 0;
  bool sp = false;   // band noise with the superpixel-major P^T
};

// Workspace of the normal operator: per-detector diagonal weights, the band
// kernel's spectrum and two TOD buffers (band noise), and the interleaved
// gather copy of p and the interleaved FP64 accumulator of q.  With band
// noise and no superpixel plan (nside not a power of two) also the ring pixel
// of every sample (int32), which P writes and the tiled P^T reads back; with
// the plan, P^T reads each sample's pixel offset from the plan.
template <typename T>
static NormalLayout normal_layout(const furax_pointing *P, const furax_noise *N) {
  NormalLayout L;
  size_t off = 0;
  const size_t tod = (size_t)P->n_det * P->n_samp * sizeof(T);
  const int64_t npix = npix_of(P->nside);
  L.wdet = off; off += align256(sizeof(double) * P->n_det);
  if (N->kind != 0) {   // band N^-1 or F_T: P, the weight and P^T as separate kernels
    L.spec = off; off += align256(noise_workspace_bytes<T>(N));
    L.y = off; off += align256(tod);
    L.z = off; off += align256(tod);
    const size_t S = (size_t)P->n_det * P->n_samp;
    if (sp_supported(P->nside, (int64_t)S)) {
      L.sp = true;
    } else {
      L.gpix = off; off += align256(sizeof(int32_t) * S);
    }
  }
  L.pg = off; off += align256(sizeof(T) * 4 * npix);
  L.qi = off; off += align256(sizeof(double) * 4 * npix);
  L.total = off;
  return L;
}

// Everything the normal operator needs besides p and q, prepared once.
template <typename T>
struct NormalPlan {
  const furax_pointing *P;
  const furax_noise *N;
  PtArgs<T> a;
  char *work;
  NormalLayout L;
  int64_t npix;
  bool use_sp = false;   // superpixel-major P^T (power-of-two nside)
  SpPlan sp;
};

template <typename T>
static furax_status normal_prepare(NormalPlan<T> &pl, hipStream_t s) {
  const furax_noise *N = pl.N;
  double *w = reinterpret_cast<double *>(pl.work + pl.L.wdet);
  hipLaunchKernelGGL(k_diag_weights, dim3((unsigned)((pl.P->n_det + 255) / 256)), dim3(256), 0, s,
                     pl.P->n_det, N->kind != 1 ? N->inv_var : nullptr,
                     N->kind == 1 ? N->toeplitz : nullptr, N->toeplitz_stride, w);
  FX_HIP(hipGetLastError());
  if (N->kind != 0) FX_TRY(noise_prepare<T>(N, pl.work + pl.L.spec, s));
  return FURAX_OK;
}

// Superpixel tables, runs, run-sorted sample copies and chunk partials of the
// plan's pointing (power-of-two nside).  With M6/hits, the block-Jacobi
// blocks are accumulated on the way.
template <typename T>
static furax_status sp_prepare(NormalPlan<T> &pl, const double *w, double *M6, int32_t *hits,
                               hipStream_t s) {
  const int64_t S = pl.P->n_det * pl.P->n_samp;
  FX_TRY(sp_nest_tables(pl.sp, pl.P->nside, s));
  DevBuf plane;
  FX_TRY(plane.alloc(sizeof(int32_t) * S, s));
  int32_t *np = static_cast<int32_t *>(plane.ptr);
  FX_TRY(sp_nest_plane<T>(pl.sp, pl.a, np, s));
  FX_TRY(sp_build_runs<T>(pl.sp, pl.a, np, M6 ? 7 : 3, s));
  if (M6) FX_TRY(sp_bj_build<T>(pl.sp, pl.a, w, M6, hits, s));
  pl.a.det_perm = pl.sp.det_perm;   // P's tiles take the detectors in sky order
  return FURAX_OK;
}

// Events recorded on the stream between the phases of one PCG iteration:
// e[0] before P, e[1] after P, e[2] after N^-1, e[3] after P^T, e[4] after the
// map-domain updates (the diagonal-noise path fuses the three operator phases
// into the P^T one).
struct PhaseEvents {
  hipEvent_t e[5];
};

// A named range for the profiler's marker trace (rocprofv3 --marker-trace)
// around the host code that enqueues one PCG iteration or one phase of the
// operator; the calls do nothing unless a tool listens.
struct Range {
  explicit Range(const char *name) { roctxRangePush(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range &) = delete;
  Range &operator=(const Range &) = delete;
};

static furax_status mark(const PhaseEvents *ev, int i, hipStream_t s) {
  if (ev) FX_HIP(hipEventRecord(ev->e[i], s));
  return FURAX_OK;
}

// q = P^T N^-1 P p with p given as its interleaved gather copy pg (precision T;
// on the superpixel path its 4th lane holds the nested index) and q an
// interleaved [npix][4] FP64 accumulator (overwritten).
template <typename T>
static furax_status normal_run(const NormalPlan<T> &pl, const T *pg, double *q, hipStream_t s,
                               const PhaseEvents *ev = nullptr) {
  const double *w = reinterpret_cast<const double *>(pl.work + pl.L.wdet);
  constexpr bool f64 = sizeof(T) == 8;
  FX_TRY(mark(ev, 0, s));
  if (pl.N->kind == 0) {
    FX_TRY(mark(ev, 1, s));
    FX_TRY(mark(ev, 2, s));
    FX_TRY(zero_async(q, sizeof(double) * 4 * pl.npix, s));
    FX_TRY(launch_scatter<T>(pl.a, nullptr, w, pg, f64, kInterleaved, q, kInterleaved, s));
    return mark(ev, 3, s);
  }
  T *y = reinterpret_cast<T *>(pl.work + pl.L.y);
  T *z = reinterpret_cast<T *>(pl.work + pl.L.z);
  if (pl.use_sp) {
    {
      Range r("P");
      FX_TRY(launch_pointing_apply<T>(pl.a, pg, f64, kInterleaved, y, s));
    }
    FX_TRY(mark(ev, 1, s));
    {
      Range r("N^-1");
      FX_TRY(noise_run<T>(pl.N, y, z, pl.work + pl.L.spec, s));
    }
    FX_TRY(mark(ev, 2, s));
    {
      Range r("P^T");
      FX_TRY(sp_transpose<T>(pl.sp, pl.a, z, nullptr, q, kInterleaved, s));
    }
    return mark(ev, 3, s);
  }
  int32_t *pix = reinterpret_cast<int32_t *>(pl.work + pl.L.gpix);
  FX_TRY(launch_pointing_apply<T>(pl.a, pg, f64, kInterleaved, y, s, pix));
  FX_TRY(mark(ev, 1, s));
  FX_TRY(noise_run<T>(pl.N, y, z, pl.work + pl.L.spec, s));
  FX_TRY(mark(ev, 2, s));
  FX_TRY(zero_async(q, sizeof(double) * 4 * pl.npix, s));
  FX_TRY(launch_scatter<T>(pl.a, z, nullptr, nullptr, f64, kInterleaved, q, kInterleaved, s, pix));
  return mark(ev, 3, s);
}

// planar FP64 [3][npix] -> interleaved [npix][4] of T (4th lane 0), zero on
// pixels with valid = 0 (when valid is given).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_to_interleaved(int64_t npix, const double *__restrict__ p,
                                                           const uint8_t *__restrict__ valid,
                                                           const int32_t *__restrict__ tag,
                                                           T *__restrict__ g) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npix; i += stride) {
    const bool ok = !valid || valid[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) g[4 * i + c] = ok ? (T)p[c * npix + i] : (T)0;
    set_tag(g, i, tag);
  }
}

__global__ void __launch_bounds__(kBlock) k_from_interleaved(int64_t npix, const double *__restrict__ qi,
                                                             const uint8_t *__restrict__ valid,
                                                             double *__restrict__ q) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npix; i += stride) {
    const bool ok = !valid || valid[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) q[c * npix + i] = ok ? qi[4 * i + c] : 0.0;
  }
}

int64_t normal_workspace_bytes(const furax_pointing *P, const furax_noise *N, int32_t prec) {
  return prec == FURAX_F32 ? (int64_t)normal_layout<float>(P, N).total
                           : (int64_t)normal_layout<double>(P, N).total;
}

template <typename T>
furax_status normal_apply_impl(const furax_pointing *P, const furax_noise *N, const double *p,
                               double *q, const uint8_t *valid, void *work, hipStream_t s) {
  NormalPlan<T> pl;
  pl.P = P;
  pl.N = N;
  // Flagging the samples of invalid pixels is done in the map domain: p is
  // zeroed there on input (so those samples read 0) and q on output (so what
  // they scatter is dropped), which is the flagged operator exactly.
  pl.a = pt_args<T>(P, nullptr);
  pl.L = normal_layout<T>(P, N);
  pl.npix = npix_of(P->nside);
  pl.use_sp = N->kind != 0 && pl.L.sp;
  DevBuf own;
  if (!work) {
    FX_TRY(own.alloc(pl.L.total, s));
    work = own.ptr;
  }
  pl.work = static_cast<char *>(work);
  FX_TRY(normal_prepare<T>(pl, s));
  furax_status st = FURAX_OK;
  if (pl.use_sp) st = sp_prepare<T>(pl, nullptr, nullptr, nullptr, s);
  if (st == FURAX_OK) {
    T *pg = reinterpret_cast<T *>(pl.work + pl.L.pg);
    double *qi = reinterpret_cast<double *>(pl.work + pl.L.qi);
    const unsigned nb = (unsigned)map_blocks(pl.npix);
    hipLaunchKernelGGL(k_to_interleaved<T>, dim3(nb), dim3(kBlock), 0, s, pl.npix, p, valid,
                       pl.use_sp ? pl.sp.r2n : nullptr, pg);
    st = hipGetLastError() == hipSuccess ? FURAX_OK : set_error(FURAX_EHIP, "launch failed");
    if (st == FURAX_OK) st = normal_run<T>(pl, pg, qi, s);
    if (st == FURAX_OK) {
      hipLaunchKernelGGL(k_from_interleaved, dim3(nb), dim3(kBlock), 0, s, pl.npix, qi, valid, q);
      st = hipGetLastError() == hipSuccess ? FURAX_OK : set_error(FURAX_EHIP, "launch failed");
    }
  }
  pl.sp.release(s);
  return st;
}
template furax_status normal_apply_impl<float>(const furax_pointing *, const furax_noise *,
                                               const double *, double *, const uint8_t *, void *,
                                               hipStream_t);
template furax_status normal_apply_impl<double>(const furax_pointing *, const furax_noise *,
                                                const double *, double *, const uint8_t *, void *,
                                                hipStream_t);

template <typename T>
furax_status bj_build_impl(const furax_pointing *P, const furax_noise *N, double *M6,
                           int32_t *hits, hipStream_t s) {
  const int64_t npix = npix_of(P->nside);
  DevBuf wbuf;
  FX_TRY(wbuf.alloc(sizeof(double) * P->n_det, s));
  double *w = static_cast<double *>(wbuf.ptr);
  hipLaunchKernelGGL(k_diag_weights, dim3((unsigned)((P->n_det + 255) / 256)), dim3(256), 0, s,
                     P->n_det, N->kind != 1 ? N->inv_var : nullptr,
                     N->kind == 1 ? N->toeplitz : nullptr, N->toeplitz_stride, w);
  FX_HIP(hipGetLastError());
  FX_TRY(zero_async(M6, sizeof(double) * 6 * npix, s));
  FX_TRY(zero_async(hits, sizeof(int32_t) * npix, s));
  return launch_bj_build<T>(pt_args<T>(P, nullptr), w, M6, hits, s);
}
template furax_status bj_build_impl<float>(const furax_pointing *, const furax_noise *, double *,
                                           int32_t *, hipStream_t);
template furax_status bj_build_impl<double>(const furax_pointing *, const furax_noise *, double *,
                                            int32_t *, hipStream_t);

// ---------------------------------------------------------------------------
// PCG session.
// ---------------------------------------------------------------------------
}  // namespace fx

struct furax_pcg_state {
  furax_pointing P;
  furax_noise N;
  furax_pcg_opts opt;
  hipStream_t s = nullptr;
  int64_t npix = 0;
  int32_t precision = FURAX_F64;
  char *mem = nullptr;       // one stream-ordered allocation for everything
  size_t mem_bytes = 0;
  double *x, *r, *z, *p, *q, *Minv, *partial, *hist;   // q: interleaved [npix][4]
  void *pg;                                               // interleaved gather copy of p
  uint8_t *valid;
  fx::PcgScalars *sc;
  fx::NormalPlan<float> pl32;
  fx::NormalPlan<double> pl64;
  int32_t nhist = 0;
  int32_t iters_launched = 0;
  bool timing = false;
  std::vector<fx::PhaseEvents> events;   // pool, reused after each read
  int32_t n_timed = 0;
};

namespace fx {

template <typename T>
static furax_status pcg_setup(furax_pcg_state *h, const void *tod) {
  hipStream_t s = h->s;
  const int64_t npix = h->npix;
  NormalPlan<T> &pl = [&]() -> NormalPlan<T> & {
    if constexpr (sizeof(T) == 4) return h->pl32;
    else return h->pl64;
  }();
  pl.P = &h->P;
  pl.N = &h->N;
  pl.npix = npix;
  pl.L = normal_layout<T>(&h->P, &h->N);

  // Memory map of the session.
  const size_t vec = align256(sizeof(double) * 3 * npix);
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off += align256(b); return o; };
  const size_t o_x = take(vec), o_r = take(vec), o_z = take(vec), o_p = take(vec);
  const size_t o_q = take(sizeof(double) * 4 * npix);
  const size_t o_minv = take(sizeof(double) * 6 * npix);
  const size_t o_valid = take(npix);
  const size_t o_pg = take(sizeof(T) * 4 * npix);
  const size_t o_part = take(sizeof(double) * 2 * kRedBlocks);
  const size_t o_sc = take(sizeof(PcgScalars));
  h->nhist = h->opt.max_iter + 1;
  const size_t o_hist = take(sizeof(double) * h->nhist);
  const size_t o_work = take(pl.L.total);
  h->mem_bytes = off;
  if (hipMallocAsync((void **)&h->mem, off, s) != hipSuccess)
    return set_error(FURAX_ENOMEM, "PCG workspace allocation failed");
  char *m = h->mem;
  h->x = (double *)(m + o_x);
  h->r = (double *)(m + o_r);
  h->z = (double *)(m + o_z);
  h->p = (double *)(m + o_p);
  h->q = (double *)(m + o_q);
  h->Minv = (double *)(m + o_minv);
  h->valid = (uint8_t *)(m + o_valid);
  h->pg = m + o_pg;
  h->partial = (double *)(m + o_part);
  h->sc = (PcgScalars *)(m + o_sc);
  h->hist = (double *)(m + o_hist);
  pl.work = m + o_work;
  // Before the first iteration the unaccumulated blocks M6 (6 planes) live in
  // the adjacent p and q vectors (3 + 4 npix doubles >= 6 npix) and the hit
  // counts in x; both are consumed by the inversion before those vectors are
  // initialised.
  double *M6 = h->p;
  int32_t *hits = reinterpret_cast<int32_t *>(h->x);

  // Preconditioner: M6 (in p,q), hits (in x), then Minv and valid.
  pl.a = pt_args<T>(&h->P, nullptr);
  FX_TRY(normal_prepare<T>(pl, s));
  const double *w = reinterpret_cast<const double *>(pl.work + pl.L.wdet);
  const int64_t S = h->P.n_det * h->P.n_samp;
  pl.use_sp = sp_supported(h->P.nside, S);
  if (pl.use_sp) {
    // superpixel plan (kept for the iterations) and the blocks on the way
    FX_TRY(sp_prepare<T>(pl, w, M6, hits, s));
    pl.use_sp = h->N.kind != 0 && pl.L.sp;
  } else {
    FX_TRY(zero_async(M6, sizeof(double) * 6 * npix, s));
    FX_TRY(zero_async(hits, sizeof(int32_t) * npix, s));
    FX_TRY(launch_bj_build<T>(pl.a, w, M6, hits, s));
  }
  FX_TRY(launch_bj_invert(npix, M6, hits, h->opt.rcond_min, h->opt.min_hits, h->opt.valid_in,
                          h->Minv, h->valid, nullptr, s));

  // Right-hand side b = P^T N^-1 d into the z buffer.  Samples in invalid
  // pixels only add to b on those pixels, which k_init_vectors drops: that is
  // b with those samples flagged.  The iterations flag the same way (p is 0 on
  // invalid pixels and r is kept at 0 there), so pl.a carries no mask.
  double *b = h->z;
  const T *d = static_cast<const T *>(tod);
  const T *zt = d;
  const double *wd = w;
  if (h->N.kind != 0) {
    T *zbuf = reinterpret_cast<T *>(pl.work + pl.L.z);
    FX_TRY(noise_run<T>(&h->N, d, zbuf, pl.work + pl.L.spec, s));
    zt = zbuf;
    wd = nullptr;
  }
  if (pl.sp.lab) {
    FX_TRY(sp_transpose<T>(pl.sp, pl.a, zt, wd, b, planar_layout(npix), s));
  } else {
    FX_TRY(zero_async(b, sizeof(double) * 3 * npix, s));
    FX_TRY(launch_scatter<T>(pl.a, zt, wd, nullptr, false, planar_layout(npix), b,
                              planar_layout(npix), s));
  }
  if (!pl.use_sp && pl.sp.n2r) {   // diagonal noise: tables no longer needed
    pl.sp.release(s);
    pl.a.det_perm = nullptr;
  }
  // r = b (copied into r), x = 0, z = Minv r, p = z.  b lives in z; k_init_vectors
  // reads b[i] before writing z[i] for the same i, element by element.
  hipLaunchKernelGGL(k_init_vectors<T>, dim3((unsigned)kRedBlocks), dim3(kBlock), 0, s, npix, b,
                     h->valid, h->x, h->r, h->z, h->p, static_cast<T *>(h->pg),
                     pl.use_sp ? pl.sp.r2n : nullptr, h->Minv, h->partial);
  FX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_init_final, dim3(1), dim3(kBlock), 0, s, h->partial, h->opt.rtol, h->sc,
                     h->hist);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}

template <typename T>
static furax_status pcg_step(furax_pcg_state *h) {
  hipStream_t s = h->s;
  NormalPlan<T> &pl = [&]() -> NormalPlan<T> & {
    if constexpr (sizeof(T) == 4) return h->pl32;
    else return h->pl64;
  }();
  const PhaseEvents *ev = nullptr;
  if (h->timing) {
    if ((size_t)h->n_timed == h->events.size()) {
      PhaseEvents pe;
      for (hipEvent_t &e : pe.e) FX_HIP(hipEventCreate(&e));
      h->events.push_back(pe);
    }
    ev = &h->events[h->n_timed++];
  }
  Range it("pcg_iteration");
  FX_TRY(normal_run<T>(pl, static_cast<const T *>(h->pg), h->q, s, ev));
  Range up("pcg_update");
  hipLaunchKernelGGL(k_dot_pq, dim3((unsigned)kRedBlocks), dim3(kBlock), 0, s, h->npix, h->p, h->q,
                     h->valid, h->partial);
  hipLaunchKernelGGL(k_pq_final, dim3(1), dim3(kBlock), 0, s, h->partial, h->sc);
  hipLaunchKernelGGL(k_update1, dim3((unsigned)kRedBlocks), dim3(kBlock), 0, s, h->npix, h->x,
                     h->r, h->p, h->q, h->Minv, h->valid, h->z, h->sc, h->partial);
  hipLaunchKernelGGL(k_rz_final, dim3(1), dim3(kBlock), 0, s, h->partial, h->sc, h->hist,
                     h->nhist);
  hipLaunchKernelGGL(k_update2<T>, dim3((unsigned)map_blocks(h->npix)), dim3(kBlock), 0, s,
                     h->npix, h->p, h->z, static_cast<T *>(h->pg), h->valid, h->sc);
  FX_HIP(hipGetLastError());
  return mark(ev, 4, s);
}

furax_status pcg_set_timing(furax_pcg h, int32_t enable) {
  h->timing = enable != 0;
  return FURAX_OK;
}

furax_status pcg_read_timing(furax_pcg h, furax_pcg_timing *out) {
  FX_HIP(hipStreamSynchronize(h->s));
  furax_pcg_timing t = {0, 0.0, 0.0, 0.0, 0.0};
  for (int32_t i = 0; i < h->n_timed; ++i) {
    float ms[4];
    for (int j = 0; j < 4; ++j)
      FX_HIP(hipEventElapsedTime(&ms[j], h->events[i].e[j], h->events[i].e[j + 1]));
    t.ms_apply += ms[0];
    t.ms_noise += ms[1];
    t.ms_transpose += ms[2];
    t.ms_update += ms[3];
  }
  t.iters = h->n_timed;
  h->n_timed = 0;
  *out = t;
  return FURAX_OK;
}

furax_status pcg_create(const furax_pointing *P, const furax_noise *N, int32_t tod_dt,
                        const void *tod, const furax_pcg_opts *opt, hipStream_t s,
                        furax_pcg *out) {
  furax_pcg_state *h = new (std::nothrow) furax_pcg_state();
  if (!h) return set_error(FURAX_ENOMEM, "host allocation failed");
  h->P = *P;
  h->N = *N;
  h->opt = *opt;
  h->s = s;
  h->npix = npix_of(P->nside);
  h->precision = opt->precision;
  furax_status st = opt->precision == FURAX_F32 ? pcg_setup<float>(h, tod) : pcg_setup<double>(h, tod);
  if (st != FURAX_OK) {
    h->pl32.sp.release(s);
    h->pl64.sp.release(s);
    if (h->mem) (void)hipFreeAsync(h->mem, s);
    (void)hipStreamSynchronize(s);
    delete h;
    return st;
  }
  *out = h;
  return FURAX_OK;
}

furax_status pcg_iterate(furax_pcg h, int32_t n_iter) {
  for (int32_t i = 0; i < n_iter; ++i) {
    if (h->iters_launched >= h->opt.max_iter) break;
    if (!h->opt.no_early_exit) {
      int32_t stop = 0;
      FX_HIP(hipMemcpyAsync(&stop, &h->sc->stop, sizeof(int32_t), hipMemcpyDeviceToHost, h->s));
      FX_HIP(hipStreamSynchronize(h->s));
      if (stop) break;
    }
    FX_TRY(h->precision == FURAX_F32 ? pcg_step<float>(h) : pcg_step<double>(h));
    ++h->iters_launched;
  }
  return FURAX_OK;
}

__global__ void k_copy_out(int64_t npix, const double *__restrict__ x,
                           const uint8_t *__restrict__ valid, double *__restrict__ out,
                           uint8_t *__restrict__ vout) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npix; i += stride) {
    const bool ok = valid[i] != 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * npix + i] = ok ? x[c * npix + i] : 0.0;
    if (vout) vout[i] = valid[i];
  }
}

__global__ void k_count_valid(int64_t npix, const uint8_t *__restrict__ valid, double *partial) {
  double v[1] = {0.0};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < npix; i += stride)
    v[0] += valid[i] ? 1.0 : 0.0;
  block_sum<1>(v, partial + blockIdx.x, kRedBlocks);
}

__global__ void k_count_final(const double *partial, PcgScalars *sc, double *out) {
  double v[1];
  final_sum<1>(partial, v);
  if (threadIdx.x == 0) out[0] = v[0];
}

furax_status pcg_finish(furax_pcg h, double *map_out, uint8_t *valid_out, furax_pcg_info *info) {
  hipStream_t s = h->s;
  if (map_out) {
    hipLaunchKernelGGL(k_copy_out, dim3((unsigned)map_blocks(h->npix)), dim3(kBlock), 0, s,
                       h->npix, h->x, h->valid, map_out, valid_out);
    FX_HIP(hipGetLastError());
  }
  // n_valid via a deterministic count into the q buffer's first element
  hipLaunchKernelGGL(k_count_valid, dim3((unsigned)kRedBlocks), dim3(kBlock), 0, s, h->npix,
                     h->valid, h->partial);
  hipLaunchKernelGGL(k_count_final, dim3(1), dim3(kBlock), 0, s, h->partial, h->sc, h->q);
  FX_HIP(hipGetLastError());
  PcgScalars sc;
  double nvalid = 0.0;
  FX_HIP(hipMemcpyAsync(&sc, h->sc, sizeof(sc), hipMemcpyDeviceToHost, s));
  FX_HIP(hipMemcpyAsync(&nvalid, h->q, sizeof(double), hipMemcpyDeviceToHost, s));
  std::vector<double> hist;
  if (info && info->resid_history && !h->opt.no_early_exit) {
    hist.resize(h->nhist);
    FX_HIP(hipMemcpyAsync(hist.data(), h->hist, sizeof(double) * h->nhist, hipMemcpyDeviceToHost, s));
  }
  FX_HIP(hipStreamSynchronize(s));
  if (info) {
    info->iters = sc.iters;
    info->stop_reason = sc.stop;
    info->rel_resid = sc.rel;
    info->n_valid = (int64_t)nvalid;
    if (info->resid_history && !hist.empty())
      std::memcpy(info->resid_history, hist.data(), sizeof(double) * (sc.iters + 1));
  }
  if (sc.stop == 2) return set_error(FURAX_EBREAKDOWN, "PCG breakdown (<p,Ap> or <r,z> not positive and finite)");
  if (sc.stop == 0 && h->opt.rtol > 0.0) return set_error(FURAX_ENOTCONV, "PCG reached max_iter before rtol");
  return FURAX_OK;
}

furax_status pcg_destroy(furax_pcg h) {
  if (!h) return FURAX_OK;
  for (fx::PhaseEvents &pe : h->events)
    for (hipEvent_t e : pe.e) (void)hipEventDestroy(e);
  h->pl32.sp.release(h->s);
  h->pl64.sp.release(h->s);
  if (h->mem) FX_HIP(hipFreeAsync(h->mem, h->s));
  FX_HIP(hipStreamSynchronize(h->s));
  delete h;
  return FURAX_OK;
}

}  // namespace fx
