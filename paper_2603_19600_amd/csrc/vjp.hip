// Chi-square of the data model (Eq. (1) with T = 0) and the vector-Jacobian
// product of the signal s = P(m; g, dpsi) used by the differentiable path
// (sections "Summary" and "Research Impact Statement": JAX autodiff, here a
// hand-written adjoint).
//
//   s[k,i]     = g_k (I[p] + Q[p] cos 2 psi_eff + U[p] sin 2 psi_eff)
//   ds/dm      : P (adjoint: P^T, a scatter-add)
//   ds/dg_k    : (P_1 m)[k,i], the unit-gain signal
//   ds/ddpsi_k : g_k (-2 Q[p] sin 2 psi_eff + 2 U[p] cos 2 psi_eff)
//
// Pointing is recomputed from theta/phi/psi in every pass, never stored.
// Products are formed in the pointing precision; every sum is FP64 and the
// per-detector sums are deterministic (fixed partial layout, fixed order).
#include "common.h"
#include "reduce.h"

namespace fx {

constexpr int kDetParts = 64;   // partial sums per detector

template <typename T, typename MT>
__device__ __forceinline__ void read_map(const MT *__restrict__ m, int64_t npix, int32_t p,
                                         T &I, T &Q, T &U) {
  I = (T)m[p];
  Q = (T)m[npix + p];
  U = (T)m[2 * npix + p];
}

// chi2 = sum_k w_k sum_i (d - s)^2 for diagonal N; optionally u = w_k (d - s).
template <typename T, typename MT>
__global__ void __launch_bounds__(kBlock) k_chi2(PtArgs<T> a, const MT *__restrict__ m,
                                                 int64_t npix, const T *__restrict__ d,
                                                 const double *__restrict__ w_det,
                                                 T *__restrict__ u_out,
                                                 double *__restrict__ partial) {
  double acc[1] = {0.0};
  const int64_t total = a.n_det * a.n_samp;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total; idx += stride) {
    const int64_t k = idx / a.n_samp, i = idx - k * a.n_samp;
    const Geom<T> gm = sample_geom(a, k, i);
    T s = 0;
    if (gm.pix >= 0) {
      T I, Q, U;
      read_map<T, MT>(m, npix, gm.pix, I, Q, U);
      s = gain_of(a, k) * (I + gm.c * Q + gm.s * U);
    }
    const T r = d[idx] - s;
    const T u = (T)w_det[k] * r;
    if (u_out) u_out[idx] = u;
    acc[0] += (double)r * (double)u;
  }
  block_sum<1>(acc, partial + blockIdx.x, kRedBlocks);
}

__global__ void __launch_bounds__(kBlock) k_sum_to(const double *__restrict__ partial,
                                                   double *__restrict__ out) {
  double v[1];
  final_sum<1>(partial, v);
  if (threadIdx.x == 0) out[0] = v[0];
}

// grad_map += P^T u (gains included); per-detector partials of
//   gg = sum u (P_1 m),   gd = sum u g (-2 Q sin + 2 U cos).
template <typename T, typename MT>
__global__ void __launch_bounds__(kBlock) k_vjp(PtArgs<T> a, const MT *__restrict__ m,
                                                int64_t npix, const T *__restrict__ u,
                                                double *__restrict__ grad_map,
                                                double *__restrict__ partial /* [2][n_det][kDetParts] */) {
  const int64_t k = blockIdx.x / kDetParts;
  const int part = blockIdx.x % kDetParts;
  const T g = gain_of(a, k);
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)part * kBlock + threadIdx.x; i < a.n_samp;
       i += (int64_t)kDetParts * kBlock) {
    const Geom<T> gm = sample_geom(a, k, i);
    if (gm.pix < 0) continue;
    const T uu = u[k * a.n_samp + i];
    if (grad_map) {
      const T v = g * uu;
      atomicAdd(&grad_map[gm.pix], (double)v);
      atomicAdd(&grad_map[npix + gm.pix], (double)(v * gm.c));
      atomicAdd(&grad_map[2 * npix + gm.pix], (double)(v * gm.s));
    }
    if (m) {
      T I, Q, U;
      read_map<T, MT>(m, npix, gm.pix, I, Q, U);
      const T s1 = I + gm.c * Q + gm.s * U;
      const T ds = (T)(-2) * Q * gm.s + (T)2 * U * gm.c;
      acc[0] += (double)(uu * s1);
      acc[1] += (double)(uu * (g * ds));
    }
  }
  block_sum<2>(acc, partial + k * kDetParts + part, a.n_det * kDetParts);
}

__global__ void k_det_final(int64_t n_det, const double *__restrict__ partial,
                            double *__restrict__ gg, double *__restrict__ gd) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_det) return;
  double s0 = 0.0, s1 = 0.0;
  for (int j = 0; j < kDetParts; ++j) {
    s0 += partial[k * kDetParts + j];
    s1 += partial[n_det * kDetParts + k * kDetParts + j];
  }
  if (gg) gg[k] = s0;
  if (gd) gd[k] = s1;
}

template <typename T>
furax_status chi2_impl(const furax_pointing *P, const furax_noise *N, int32_t map_dt,
                       const void *map, const T *tod, double *chi2_out, T *resid_w,
                       hipStream_t s) {
  const int64_t npix = npix_of(P->nside);
  DevBuf part;
  FX_TRY(part.alloc(sizeof(double) * kRedBlocks, s));
  double *partial = static_cast<double *>(part.ptr);
  const PtArgs<T> a = pt_args<T>(P, nullptr);
  if (map_dt == FURAX_F64)
    hipLaunchKernelGGL((k_chi2<T, double>), dim3(kRedBlocks), dim3(kBlock), 0, s, a,
                       static_cast<const double *>(map), npix, tod, N->inv_var, resid_w, partial);
  else
    hipLaunchKernelGGL((k_chi2<T, float>), dim3(kRedBlocks), dim3(kBlock), 0, s, a,
                       static_cast<const float *>(map), npix, tod, N->inv_var, resid_w, partial);
  hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(kBlock), 0, s, partial, chi2_out);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status chi2_impl<float>(const furax_pointing *, const furax_noise *, int32_t,
                                       const void *, const float *, double *, float *,
                                       hipStream_t);
template furax_status chi2_impl<double>(const furax_pointing *, const furax_noise *, int32_t,
                                        const void *, const double *, double *, double *,
                                        hipStream_t);

template <typename T>
furax_status vjp_impl(const furax_pointing *P, int32_t map_dt, const void *map, const T *cot,
                      double *grad_map, double *grad_gain, double *grad_dpsi, hipStream_t s) {
  if (P->n_samp == 0) {
    if (grad_gain) FX_TRY(zero_async(grad_gain, sizeof(double) * P->n_det, s));
    if (grad_dpsi) FX_TRY(zero_async(grad_dpsi, sizeof(double) * P->n_det, s));
    return FURAX_OK;
  }
  const int64_t npix = npix_of(P->nside);
  const bool need_det = grad_gain || grad_dpsi;
  DevBuf part;
  FX_TRY(part.alloc(sizeof(double) * 2 * P->n_det * kDetParts, s));
  double *partial = static_cast<double *>(part.ptr);
  const PtArgs<T> a = pt_args<T>(P, nullptr);
  const int64_t blocks = P->n_det * kDetParts;
  if (map_dt == FURAX_F64)
    hipLaunchKernelGGL((k_vjp<T, double>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a,
                       need_det ? static_cast<const double *>(map) : nullptr, npix, cot, grad_map,
                       partial);
  else
    hipLaunchKernelGGL((k_vjp<T, float>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a,
                       need_det ? static_cast<const float *>(map) : nullptr, npix, cot, grad_map,
                       partial);
  FX_HIP(hipGetLastError());
  if (need_det) {
    hipLaunchKernelGGL(k_det_final, dim3((unsigned)((P->n_det + 255) / 256)), dim3(256), 0, s,
                       P->n_det, partial, grad_gain, grad_dpsi);
    FX_HIP(hipGetLastError());
  }
  return FURAX_OK;
}
template furax_status vjp_impl<float>(const furax_pointing *, int32_t, const void *,
                                      const float *, double *, double *, double *, hipStream_t);
template furax_status vjp_impl<double>(const furax_pointing *, int32_t, const void *,
                                       const double *, double *, double *, double *, hipStream_t);

}  // namespace fx
