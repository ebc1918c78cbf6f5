// Gap filling by constrained Gaussian realisations (the symmetric band-Toeplitz
// operator's second use named after Table 2): for each detector with missing
// samples G and valid samples V, noise covariance N (band-Toeplitz lags c) and
// an unconstrained realisation n supplied by the caller,
//     d_G = n_G + N_GV N_VV^-1 (d_V - n_V),   d_V unchanged.
//
// N_VV^-1 is applied by conjugate gradients on every detector at once: the
// operator is v -> mask_V(N mask_V(v)) with N applied by the same overlap-save
// kernels as the weights, the preconditioner is 1 / c_k[0], and every
// detector has its own scalars (alpha_k, beta_k), so the detectors' solves are
// independent.  The iterate x itself is never formed: the fill needs only
// N_GV x = sum_i alpha_i (N p_i)_G, and N p_i is the product each iteration
// computes anyway, so y_G accumulates alpha_i q_i on the missing samples and
// no final product is needed.  Vectors are FP64 in both TOD precisions.
// Per-detector sums are taken in two fixed-order stages (chunk partials, then
// one pass over them), so results do not depend on scheduling.
//
// Where N is applied by the 32768-sample FP64 overlap-save kernel (bands
// above 2560 lags), that kernel also forms the new direction as it loads its
// input and adds each block's share of p . (mask q) after its output
// (noise_run_gap): an iteration is then the transform and one vector pass
// (the step) instead of the transform and three.
#include <algorithm>
#include <cstddef>
#include <utility>

#include "common.h"
#include "reduce.h"

namespace fx {

constexpr int kGapChunks = 64;   // workgroups per detector in the vector passes

struct GapDet {
  double rz, pq, rr, bb, alpha, beta, inv_c0;
};

__device__ __forceinline__ void chunk_range(int64_t n, int64_t c, int64_t &i0, int64_t &i1) {
  i0 = n * c / kGapChunks;
  i1 = n * (c + 1) / kGapChunks;
}

// r = b = valid (d - n), y = 0, p = z = r / c0; partials of r z, b b and of
// the number of missing samples.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gap_init(const T *__restrict__ d,
                                                     const T *__restrict__ nr,
                                                     const uint8_t *__restrict__ gaps, int64_t n,
                                                     const GapDet *__restrict__ det,
                                                     double *__restrict__ y, double *__restrict__ r,
                                                     double *__restrict__ p,
                                                     double *__restrict__ part) {
  const int64_t k = blockIdx.y;
  int64_t i0, i1;
  chunk_range(n, blockIdx.x, i0, i1);
  const double ic = det[k].inv_c0;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
    const int64_t o = k * n + i;
    const bool g = gaps[o] != 0;
    const double v = g ? 0.0 : (double)d[o] - (double)nr[o];
    const double z = v * ic;
    y[o] = 0.0;
    r[o] = v;
    p[o] = z;
    acc[0] += v * z;
    acc[1] += v * v;
    acc[2] += g ? 1.0 : 0.0;
  }
  block_sum<3>(acc, part + (k * kGapChunks + blockIdx.x) * 3, 1);
}

// Partials of p (mask_V q) (q = N p is left unmasked: its missing samples
// feed the fill).
__global__ void __launch_bounds__(kBlock) k_gap_pq(const double *__restrict__ p,
                                                   const double *__restrict__ q,
                                                   const uint8_t *__restrict__ gaps, int64_t n,
                                                   double *__restrict__ part) {
  const int64_t k = blockIdx.y;
  int64_t i0, i1;
  chunk_range(n, blockIdx.x, i0, i1);
  double acc[1] = {0.0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
    const int64_t o = k * n + i;
    acc[0] += p[o] * (gaps[o] ? 0.0 : q[o]);
  }
  block_sum<1>(acc, part + (k * kGapChunks + blockIdx.x), 1);
}

// Per-detector scalars from the chunk partials (one thread per detector, the
// chunks summed in order).  stage 0: after init (rz, bb); 1: alpha = rz / pq
// (0 when pq or rz is not positive and finite: that detector is done);
// 2: beta = rz_new / rz, rr.  With rel_out, the largest |r_k| / |b_k| goes there
// (0 for a detector with b_k = 0, which then takes alpha = 0 throughout).
__global__ void __launch_bounds__(kBlock) k_gap_scalars(int64_t n_det, int32_t stage,
                                                        int64_t n_part,
                                                        const double *__restrict__ part,
                                                        GapDet *__restrict__ det,
                                                        double *__restrict__ rel_out) {
  __shared__ double red[kBlock];
  double worst = 0.0;
  for (int64_t k = threadIdx.x; k < n_det; k += kBlock) {
    GapDet g = det[k];
    if (stage == 0) {
      double a = 0.0, b = 0.0, m = 0.0;
      for (int c = 0; c < kGapChunks; ++c) {
        a += part[(k * kGapChunks + c) * 3];
        b += part[(k * kGapChunks + c) * 3 + 1];
        m += part[(k * kGapChunks + c) * 3 + 2];
      }
      // a detector with no missing sample needs no solve: mark it converged
      g.rz = m > 0.0 ? a : 0.0;
      g.bb = m > 0.0 ? b : 0.0;
      g.rr = g.bb;
    } else if (stage == 1) {
      // n_part partials per detector: the vector pass's chunks, or the fused
      // transform's blocks
      double a = 0.0;
      for (int64_t c = 0; c < n_part; ++c) a += part[k * n_part + c];
      g.pq = a;
      const bool ok = a > 0.0 && g.rz > 0.0 && (g.rz / a) - (g.rz / a) == 0.0;
      g.alpha = ok ? g.rz / a : 0.0;
    } else {
      double a = 0.0, b = 0.0;
      for (int c = 0; c < kGapChunks; ++c) {
        a += part[(k * kGapChunks + c) * 2];
        b += part[(k * kGapChunks + c) * 2 + 1];
      }
      g.beta = (g.alpha != 0.0 && g.rz > 0.0) ? a / g.rz : 0.0;
      g.rz = g.bb > 0.0 ? a : 0.0;   // a detector with nothing to solve stays done
      g.rr = b;
    }
    det[k] = g;
    const double rel = g.bb > 0.0 ? sqrt(g.rr / g.bb) : 0.0;
    worst = fmax(worst, rel);
  }
  red[threadIdx.x] = worst;
  __syncthreads();
  for (int w = kBlock / 2; w >= 1; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && rel_out) *rel_out = red[0];
}

// On valid samples r -= alpha q, on missing ones y += alpha q (the fill's
// N_GV x, accumulated); partials of r z (z = r / c0) and r r.
__global__ void __launch_bounds__(kBlock) k_gap_step(double *__restrict__ y,
                                                     double *__restrict__ r,
                                                     const double *__restrict__ q,
                                                     const uint8_t *__restrict__ gaps, int64_t n,
                                                     const GapDet *__restrict__ det,
                                                     double *__restrict__ part) {
  const int64_t k = blockIdx.y;
  int64_t i0, i1;
  chunk_range(n, blockIdx.x, i0, i1);
  const double a = det[k].alpha, ic = det[k].inv_c0;
  double acc[2] = {0.0, 0.0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
    const int64_t o = k * n + i;
    const double qv = q[o];
    if (gaps[o]) {
      y[o] += a * qv;
    } else {
      const double rv = r[o] - a * qv;
      r[o] = rv;
      acc[0] += rv * (rv * ic);
      acc[1] += rv * rv;
    }
  }
  block_sum<2>(acc, part + (k * kGapChunks + blockIdx.x) * 2, 1);
}

// p = z + beta p.
__global__ void __launch_bounds__(kBlock) k_gap_dir(double *__restrict__ p,
                                                    const double *__restrict__ r, int64_t n,
                                                    const GapDet *__restrict__ det) {
  const int64_t k = blockIdx.y;
  int64_t i0, i1;
  chunk_range(n, blockIdx.x, i0, i1);
  const double b = det[k].beta, ic = det[k].inv_c0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
    const int64_t o = k * n + i;
    p[o] = r[o] * ic + b * p[o];
  }
}

__global__ void __launch_bounds__(kBlock) k_gap_inv_c0(int64_t n_det, const double *__restrict__ c,
                                                       int64_t stride, GapDet *__restrict__ det) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n_det) return;
  GapDet g{};
  g.inv_c0 = 1.0 / c[k * stride];
  det[k] = g;
}

// out = d on valid samples, n + y on missing ones (y = N_GV x, or 0 for white
// noise).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gap_out(const T *__restrict__ d,
                                                    const T *__restrict__ nr,
                                                    const uint8_t *__restrict__ gaps,
                                                    const double *__restrict__ y, int64_t S,
                                                    T *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t o = (int64_t)blockIdx.x * kBlock + threadIdx.x; o < S; o += stride)
    out[o] = gaps[o] ? (T)((double)nr[o] + (y ? y[o] : 0.0)) : d[o];
}

template <typename T>
furax_status gap_fill_impl(const furax_noise *C, const uint8_t *gaps, const T *d, const T *nr,
                           T *out, const furax_gapfill_opts *opt, furax_gapfill_info *info,
                           hipStream_t s) {
  const int64_t n = C->n_samp, nd = C->n_det, S = nd * n;
  if (info) {
    info->iters = 0;
    info->rel_resid = 0.0;
  }
  if (S == 0) return FURAX_OK;
  const unsigned ob = (unsigned)std::min<int64_t>((S + kBlock - 1) / kBlock, 65536);
  if (C->kind == 0) {   // white covariance: nothing to constrain
    hipLaunchKernelGGL(k_gap_out<T>, dim3(ob), dim3(kBlock), 0, s, d, nr, gaps,
                       (const double *)nullptr, S, out);
    FX_HIP(hipGetLastError());
    return FURAX_OK;
  }
  // y, r, p, q [S] FP64 (and with the fused transform a second direction
  // buffer); spectrum; per-detector scalars and chunk / block partials
  const int64_t nblk = noise_gap_blocks(C);
  const int nvec = nblk > 0 ? 5 : 4;
  const size_t vb = sizeof(double) * (size_t)S;
  const size_t spec_b = noise_workspace_bytes<double>(C);
  const size_t part_b = sizeof(double) * std::max<int64_t>(3 * kGapChunks, nblk) * nd;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  DevBuf mem;
  FX_TRY(mem.alloc(nvec * al(vb) + al(spec_b) + al(part_b) + al(sizeof(GapDet) * nd) + 256, s));
  char *base = static_cast<char *>(mem.ptr);
  double *y = reinterpret_cast<double *>(base);
  double *r = reinterpret_cast<double *>(base + al(vb));
  double *p = reinterpret_cast<double *>(base + 2 * al(vb));
  double *q = reinterpret_cast<double *>(base + 3 * al(vb));
  double *p_alt = nblk > 0 ? reinterpret_cast<double *>(base + 4 * al(vb)) : nullptr;
  char *spec = base + nvec * al(vb);
  double *part = reinterpret_cast<double *>(spec + al(spec_b));
  GapDet *det = reinterpret_cast<GapDet *>(reinterpret_cast<char *>(part) + al(part_b));
  double *rel = reinterpret_cast<double *>(reinterpret_cast<char *>(det) + al(sizeof(GapDet) * nd));
  FX_TRY(noise_prepare<double>(C, spec, s));
  hipLaunchKernelGGL(k_gap_inv_c0, dim3((unsigned)((nd + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, nd, C->toeplitz, C->toeplitz_stride, det);
  const dim3 grid(kGapChunks, (unsigned)nd);
  hipLaunchKernelGGL(k_gap_init<T>, grid, dim3(kBlock), 0, s, d, nr, gaps, n, det, y, r, p, part);
  hipLaunchKernelGGL(k_gap_scalars, dim3(1), dim3(kBlock), 0, s, nd, 0, (int64_t)kGapChunks, part,
                     det, rel);
  FX_HIP(hipGetLastError());
  double worst = 0.0;
  FX_HIP(hipMemcpyAsync(&worst, rel, sizeof(double), hipMemcpyDeviceToHost, s));
  FX_HIP(hipStreamSynchronize(s));
  int32_t it = 0;
  // per-detector beta and 1 / c0 inside the GapDet records, read with a stride
  const double *det_words = reinterpret_cast<const double *>(det);
  constexpr int64_t kDetStride = sizeof(GapDet) / sizeof(double);
  static_assert(sizeof(GapDet) % sizeof(double) == 0, "GapDet holds doubles only");
  double *p_cur = p;
  while (it < opt->max_iter && worst > opt->rtol) {
    if (nblk > 0) {
      // p_alt = z + beta p_cur (beta = 0 at the first iteration: p_alt = z),
      // q = N p_alt and the blocks' partials of p_alt . (mask q), in one kernel
      const GapFuse g{r, p_alt, gaps, det_words + offsetof(GapDet, inv_c0) / sizeof(double),
                      det_words + offsetof(GapDet, beta) / sizeof(double), kDetStride, part};
      FX_TRY(noise_run_gap(C, p_cur, q, spec, g, s));
      std::swap(p_cur, p_alt);
      hipLaunchKernelGGL(k_gap_scalars, dim3(1), dim3(kBlock), 0, s, nd, 1, nblk, part, det, rel);
      hipLaunchKernelGGL(k_gap_step, grid, dim3(kBlock), 0, s, y, r, q, gaps, n, det, part);
      hipLaunchKernelGGL(k_gap_scalars, dim3(1), dim3(kBlock), 0, s, nd, 2, (int64_t)kGapChunks,
                         part, det, rel);
    } else {
      FX_TRY(noise_run<double>(C, p, q, spec, s));
      hipLaunchKernelGGL(k_gap_pq, grid, dim3(kBlock), 0, s, p, q, gaps, n, part);
      hipLaunchKernelGGL(k_gap_scalars, dim3(1), dim3(kBlock), 0, s, nd, 1, (int64_t)kGapChunks,
                         part, det, rel);
      hipLaunchKernelGGL(k_gap_step, grid, dim3(kBlock), 0, s, y, r, q, gaps, n, det, part);
      hipLaunchKernelGGL(k_gap_scalars, dim3(1), dim3(kBlock), 0, s, nd, 2, (int64_t)kGapChunks,
                         part, det, rel);
      hipLaunchKernelGGL(k_gap_dir, grid, dim3(kBlock), 0, s, p, r, n, det);
    }
    FX_HIP(hipGetLastError());
    ++it;
    FX_HIP(hipMemcpyAsync(&worst, rel, sizeof(double), hipMemcpyDeviceToHost, s));
    FX_HIP(hipStreamSynchronize(s));
    if (!(worst - worst == 0.0)) break;   // non-finite: stop, report it
  }
  // the constrained realisation from the accumulated y_G = N_GV x
  hipLaunchKernelGGL(k_gap_out<T>, dim3(ob), dim3(kBlock), 0, s, d, nr, gaps, y, S, out);
  FX_HIP(hipGetLastError());
  FX_HIP(hipStreamSynchronize(s));
  if (info) {
    info->iters = it;
    info->rel_resid = worst;
  }
  if (!(worst - worst == 0.0)) return set_error(FURAX_EBREAKDOWN, "gap-fill CG breakdown");
  if (opt->rtol > 0.0 && worst > opt->rtol)
    return set_error(FURAX_ENOTCONV, "gap-fill CG reached max_iter before rtol");
  return FURAX_OK;
}
template furax_status gap_fill_impl<float>(const furax_noise *, const uint8_t *, const float *,
                                           const float *, float *, const furax_gapfill_opts *,
                                           furax_gapfill_info *, hipStream_t);
template furax_status gap_fill_impl<double>(const furax_noise *, const uint8_t *, const double *,
                                            const double *, double *, const furax_gapfill_opts *,
                                            furax_gapfill_info *, hipStream_t);

}  // namespace fx
