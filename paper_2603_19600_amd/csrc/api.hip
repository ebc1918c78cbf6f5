// C-ABI entry points: argument validation (before any launch), dtype
// dispatch and status/error plumbing.  No C++ exception crosses the boundary.
#include <cstdio>
#include <cstring>
#include <string>

#include "common.h"

namespace fx {

static thread_local std::string g_last_error = "no error";

furax_status set_error(furax_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

furax_status hip_error(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return FURAX_EHIP;
}

furax_status DevBuf::alloc(size_t bytes, hipStream_t s) {
  stream = s;
  if (bytes == 0) return FURAX_OK;
  if (hipMallocAsync(&ptr, bytes, s) != hipSuccess) {
    ptr = nullptr;
    return set_error(FURAX_ENOMEM, "stream-ordered device allocation failed");
  }
  return FURAX_OK;
}

int64_t npix_of(int64_t nside) { return 12 * nside * nside; }

static bool dtype_ok(int32_t dt) { return dt == FURAX_F32 || dt == FURAX_F64; }

furax_status check_pointing(const furax_pointing *P) {
  if (!P) return set_error(FURAX_EINVAL, "pointing descriptor is NULL");
  if (P->nside < 1 || P->nside > kMaxNside)
    return set_error(FURAX_EINVAL, "nside must be in [1, 8192]");
  if (P->n_det < 1) return set_error(FURAX_EINVAL, "n_det must be >= 1");
  if (P->n_samp < 0) return set_error(FURAX_EINVAL, "n_samp must be >= 0");
  if (P->n_det > ((int64_t)1 << 31) || P->n_samp > ((int64_t)1 << 40))
    return set_error(FURAX_EINVAL, "pointing too large");
  if (!dtype_ok(P->dtype)) return set_error(FURAX_EINVAL, "pointing dtype must be F32 or F64");
  if (P->bore_quat || P->det_quat) {
    if (P->theta || P->phi || P->psi)
      return set_error(FURAX_EINVAL, "give either theta/phi/psi or quaternions, not both");
    if (!P->det_quat || (P->n_samp > 0 && !P->bore_quat))
      return set_error(FURAX_EINVAL, "quaternion pointing needs bore_quat and det_quat");
    if ((reinterpret_cast<uintptr_t>(P->bore_quat) | reinterpret_cast<uintptr_t>(P->det_quat)) & 15)
      return set_error(FURAX_EINVAL, "quaternion arrays must be 16-byte aligned");
  } else if (P->n_samp > 0 && (!P->theta || !P->phi || !P->psi)) {
    return set_error(FURAX_EINVAL, "theta, phi and psi must be non-NULL");
  }
  if (P->hwp != 0 && P->hwp != 1) return set_error(FURAX_EINVAL, "hwp must be 0 or 1");
  if (P->hwp && (P->hwp_den <= 0 || P->hwp_num < 0))
    return set_error(FURAX_EINVAL, "hwp requires hwp_den > 0 and hwp_num >= 0");
  if (P->hwp && !(P->hwp_phase0 - P->hwp_phase0 == 0.0))
    return set_error(FURAX_EINVAL, "hwp_phase0 must be finite");
  // per-detector chunks must fit a 1-D grid
  const int64_t blocks = P->n_det * chunks_per_det(P->n_samp);
  if (blocks > 0x7fffffffLL) return set_error(FURAX_EINVAL, "too many samples for one launch");
  return FURAX_OK;
}

template <typename T>
int64_t os_max_band();

furax_status check_noise(const furax_noise *N, int64_t n_det, int64_t n_samp, int32_t dt) {
  if (!N) return set_error(FURAX_EINVAL, "noise descriptor is NULL");
  if (N->n_det != n_det || N->n_samp != n_samp)
    return set_error(FURAX_EINVAL, "noise n_det/n_samp do not match the data");
  if (N->n_det < 1 || N->n_samp < 0) return set_error(FURAX_EINVAL, "bad noise shape");
  if (N->kind == 0) {
    if (!N->inv_var) return set_error(FURAX_EINVAL, "diagonal noise needs inv_var");
    return FURAX_OK;
  }
  if (N->kind == 2) {
    if (!N->inv_var) return set_error(FURAX_EINVAL, "template deprojection needs inv_var");
    if (N->tmpl_order < 0 || N->tmpl_order > kMaxTmplOrder)
      return set_error(FURAX_EINVAL, "tmpl_order must be in [0, 7]");
    if (N->tmpl_seg_len <= N->tmpl_order)
      return set_error(FURAX_EINVAL, "tmpl_seg_len must exceed tmpl_order");
    if (N->n_samp > 0 && N->n_samp <= N->tmpl_order)
      return set_error(FURAX_EINVAL, "a stream needs more samples than tmpl_order");
    if (N->n_det * std::max<int64_t>(1, N->n_samp / N->tmpl_seg_len) > 0x7fffffffLL)
      return set_error(FURAX_EINVAL, "too many template segments for one launch");
    return FURAX_OK;
  }
  if (N->kind != 1) return set_error(FURAX_EINVAL, "noise kind must be 0, 1 or 2");
  if (!N->toeplitz) return set_error(FURAX_EINVAL, "band noise needs toeplitz lags");
  if (N->bandwidth < 1) return set_error(FURAX_EINVAL, "bandwidth must be >= 1");
  if (N->bandwidth > n_samp && n_samp > 0)
    return set_error(FURAX_EINVAL, "bandwidth must not exceed n_samp");
  if (N->toeplitz_stride != 0 && N->toeplitz_stride != N->bandwidth)
    return set_error(FURAX_EINVAL, "toeplitz_stride must be 0 or bandwidth");
  const int64_t bmax = dt == FURAX_F32 ? os_max_band<float>() : os_max_band<double>();
  if (N->bandwidth > bmax)
    return set_error(FURAX_EUNSUPPORTED, "band-Toeplitz supports b <= 8192");
  return FURAX_OK;
}

furax_status launch_ang2pix_any(int32_t nside, int32_t dt, const void *th, const void *ph,
                                int64_t n, int64_t *out, hipStream_t s);

template <typename T>
furax_status launch_ang2pix(int32_t nside, const T *theta, const T *phi, int64_t n, int64_t *out,
                            hipStream_t s);
template <typename T>
furax_status normal_apply_impl(const furax_pointing *P, const furax_noise *N, const double *p,
                               double *q, const uint8_t *valid, void *work, hipStream_t s);
template <typename T>
furax_status bj_build_impl(const furax_pointing *P, const furax_noise *N, double *M6,
                           int32_t *hits, hipStream_t s);
furax_status launch_bj_invert(int64_t npix, const double *M6, const int32_t *hits,
                              double rcond_min, int32_t min_hits, const uint8_t *force_valid,
                              double *Minv6, uint8_t *valid, double *rcond, hipStream_t s);
int64_t normal_workspace_bytes(const furax_pointing *P, const furax_noise *N, int32_t prec);
furax_status pcg_create(const furax_pointing *P, const furax_noise *N, int32_t tod_dt,
                        const void *tod, const furax_pcg_opts *opt, hipStream_t s,
                        furax_pcg *out);
furax_status pcg_iterate(furax_pcg h, int32_t n_iter);
furax_status pcg_finish(furax_pcg h, double *map_out, uint8_t *valid_out, furax_pcg_info *info);
furax_status pcg_destroy(furax_pcg h);
furax_status pcg_set_timing(furax_pcg h, int32_t enable);
furax_status pcg_read_timing(furax_pcg h, furax_pcg_timing *out);
template <typename T>
furax_status chi2_impl(const furax_pointing *P, const furax_noise *N, int32_t map_dt,
                       const void *map, const T *tod, double *chi2_out, T *resid_w,
                       hipStream_t s);
template <typename T>
furax_status chi2_grad_impl(const furax_pointing *P, const furax_noise *N, int32_t map_dt,
                            const void *map, const T *tod, double *chi2_out, double *grad_map,
                            double *grad_gain, double *grad_dpsi, hipStream_t s);
template <typename T>
furax_status chi2_grad_noalloc_impl(const furax_pointing *P, const furax_noise *N,
                                    int32_t map_dt, const void *map, const T *tod,
                                    double *chi2_out, double *grad_map, double *grad_gain,
                                    double *grad_dpsi, hipStream_t s);
template <typename T>
furax_status vjp_impl(const furax_pointing *P, int32_t map_dt, const void *map, const T *cot,
                      double *grad_map, double *grad_gain, double *grad_dpsi, hipStream_t s);
void release_twiddles();

static furax_status check_pcg_opts(const furax_pcg_opts *o, const furax_pointing *P) {
  if (!o) return set_error(FURAX_EINVAL, "options are NULL");
  if (o->max_iter < 0) return set_error(FURAX_EINVAL, "max_iter must be >= 0");
  if (!(o->rtol >= 0.0)) return set_error(FURAX_EINVAL, "rtol must be >= 0");
  if (o->precision != P->dtype)
    return set_error(FURAX_EINVAL, "precision must equal the pointing dtype");
  if (!(o->rcond_min >= 0.0) && !o->valid_in) return set_error(FURAX_EINVAL, "rcond_min must be >= 0");
  return FURAX_OK;
}

// Device copy used as the bandwidth ceiling beside the kernels and as the
// reference of known size for the traffic counters (not a step of the method).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ void __launch_bounds__(kBlock) k_stream_copy(const u32x4 *__restrict__ src,
                                                        u32x4 *__restrict__ dst, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += stride) {
    if constexpr (NT) {
      __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
    } else {
      dst[i] = src[i];
    }
  }
}

}  // namespace fx

using namespace fx;

extern "C" {

const char *furax_last_error(void) { return g_last_error.c_str(); }

int32_t furax_version(void) { return 200; }

void furax_release_caches(void) { release_twiddles(); }

furax_status furax_ang2pix(int64_t nside, int32_t dt, const void *theta, const void *phi,
                           int64_t n, int64_t *pix_out, hipStream_t stream) {
  if (nside < 1 || nside > kMaxNside) return set_error(FURAX_EINVAL, "nside must be in [1, 8192]");
  if (!dtype_ok(dt)) return set_error(FURAX_EINVAL, "dtype must be F32 or F64");
  if (n < 0) return set_error(FURAX_EINVAL, "n must be >= 0");
  if (n > 0 && (!theta || !phi || !pix_out)) return set_error(FURAX_EINVAL, "NULL array");
  if (dt == FURAX_F32)
    return launch_ang2pix<float>((int32_t)nside, (const float *)theta, (const float *)phi, n,
                                 pix_out, stream);
  return launch_ang2pix<double>((int32_t)nside, (const double *)theta, (const double *)phi, n,
                                pix_out, stream);
}

furax_status furax_pointing_apply(const furax_pointing *P, int32_t map_dt, const void *map,
                                  int32_t tod_dt, void *tod, hipStream_t stream) {
  FX_TRY(check_pointing(P));
  if (!dtype_ok(map_dt) || !dtype_ok(tod_dt)) return set_error(FURAX_EINVAL, "bad dtype");
  if (tod_dt != P->dtype) return set_error(FURAX_EINVAL, "tod dtype must equal the pointing dtype");
  if (P->dtype == FURAX_F64 && map_dt != FURAX_F64)
    return set_error(FURAX_EINVAL, "FP64 pointing needs an FP64 map");
  if (P->n_samp > 0 && (!map || !tod)) return set_error(FURAX_EINVAL, "NULL map or tod");
  if (P->dtype == FURAX_F32)
    return launch_pointing_apply<float>(pt_args<float>(P, nullptr), map, map_dt == FURAX_F64,
                                        planar_layout(npix_of(P->nside)), (float *)tod, stream);
  return launch_pointing_apply<double>(pt_args<double>(P, nullptr), map, true,
                                       planar_layout(npix_of(P->nside)), (double *)tod, stream);
}

furax_status furax_pointing_transpose(const furax_pointing *P, int32_t tod_dt, const void *tod,
                                      double *map, int32_t accumulate, hipStream_t stream) {
  FX_TRY(check_pointing(P));
  if (tod_dt != P->dtype) return set_error(FURAX_EINVAL, "tod dtype must equal the pointing dtype");
  if (!map || (P->n_samp > 0 && !tod)) return set_error(FURAX_EINVAL, "NULL map or tod");
  if (!accumulate) FX_TRY(zero_async(map, sizeof(double) * 3 * npix_of(P->nside), stream));
  if (P->dtype == FURAX_F32)
    return launch_scatter<float>(pt_args<float>(P, nullptr), (const float *)tod, nullptr, nullptr,
                                 false, planar_layout(npix_of(P->nside)), map,
                                 planar_layout(npix_of(P->nside)), stream);
  return launch_scatter<double>(pt_args<double>(P, nullptr), (const double *)tod, nullptr, nullptr,
                                false, planar_layout(npix_of(P->nside)), map,
                                planar_layout(npix_of(P->nside)), stream);
}

furax_status furax_gap_fill(const furax_noise *C, int32_t dt, const uint8_t *gaps,
                            const void *tod, const void *noise_real, void *out,
                            const furax_gapfill_opts *opt, furax_gapfill_info *info,
                            hipStream_t stream) {
  if (!C) return set_error(FURAX_EINVAL, "covariance descriptor is NULL");
  if (!dtype_ok(dt)) return set_error(FURAX_EINVAL, "bad dtype");
  if (C->kind != 0 && C->kind != 1)
    return set_error(FURAX_EINVAL, "gap filling needs a white (0) or band (1) covariance");
  FX_TRY(check_noise(C, C->n_det, C->n_samp, FURAX_F64));   // the solve runs in FP64
  if (C->kind == 0 && !C->inv_var) return set_error(FURAX_EINVAL, "white covariance needs inv_var");
  if (!opt) return set_error(FURAX_EINVAL, "NULL options");
  if (opt->max_iter < 0 || !(opt->rtol >= 0.0) || !(opt->rtol - opt->rtol == 0.0))
    return set_error(FURAX_EINVAL, "max_iter must be >= 0 and rtol finite and >= 0");
  if (C->n_samp > 0 && (!gaps || !tod || !noise_real || !out))
    return set_error(FURAX_EINVAL, "NULL gaps, tod, noise_real or out");
  if (dt == FURAX_F32)
    return gap_fill_impl<float>(C, gaps, static_cast<const float *>(tod),
                                static_cast<const float *>(noise_real), static_cast<float *>(out),
                                opt, info, stream);
  return gap_fill_impl<double>(C, gaps, static_cast<const double *>(tod),
                               static_cast<const double *>(noise_real), static_cast<double *>(out),
                               opt, info, stream);
}

furax_status furax_template_fit(const furax_noise *N, int32_t dt, const void *tod, double *amp,
                                hipStream_t stream) {
  if (!N) return set_error(FURAX_EINVAL, "noise descriptor is NULL");
  if (!dtype_ok(dt)) return set_error(FURAX_EINVAL, "bad dtype");
  FX_TRY(check_noise(N, N->n_det, N->n_samp, dt));
  if (N->kind != 2) return set_error(FURAX_EINVAL, "template fit needs a noise model of kind 2");
  if (N->n_samp > 0 && (!tod || !amp)) return set_error(FURAX_EINVAL, "NULL tod or amp");
  if (dt == FURAX_F32)
    return launch_deproject<float>(N, static_cast<const float *>(tod), nullptr, amp, stream);
  return launch_deproject<double>(N, static_cast<const double *>(tod), nullptr, amp, stream);
}

furax_status furax_noise_apply(const furax_noise *N, int32_t dt, const void *tod_in,
                               void *tod_out, hipStream_t stream) {
  if (!N) return set_error(FURAX_EINVAL, "noise descriptor is NULL");
  if (!dtype_ok(dt)) return set_error(FURAX_EINVAL, "bad dtype");
  FX_TRY(check_noise(N, N->n_det, N->n_samp, dt));
  if (N->n_samp > 0 && (!tod_in || !tod_out)) return set_error(FURAX_EINVAL, "NULL tod");
  const size_t es = dt == FURAX_F32 ? 4 : 8;
  if (N->kind == 1 && N->n_samp > 0) {
    const char *a = (const char *)tod_in, *b = (const char *)tod_out;
    const size_t bytes = es * N->n_det * N->n_samp;
    if (a < b + bytes && b < a + bytes)
      return set_error(FURAX_EINVAL, "band noise needs non-overlapping input and output");
  }
  DevBuf work;
  const size_t wb = dt == FURAX_F32 ? noise_workspace_bytes<float>(N) : noise_workspace_bytes<double>(N);
  FX_TRY(work.alloc(wb, stream));
  if (dt == FURAX_F32)
    return launch_noise<float>(N, (const float *)tod_in, (float *)tod_out, work.ptr, wb, stream);
  return launch_noise<double>(N, (const double *)tod_in, (double *)tod_out, work.ptr, wb, stream);
}

furax_status furax_bj_build(const furax_pointing *P, const furax_noise *N, double *M6,
                            int32_t *hits, hipStream_t stream) {
  FX_TRY(check_pointing(P));
  FX_TRY(check_noise(N, P->n_det, P->n_samp, P->dtype));
  if (!M6 || !hits) return set_error(FURAX_EINVAL, "NULL output");
  if (P->dtype == FURAX_F32) return bj_build_impl<float>(P, N, M6, hits, stream);
  return bj_build_impl<double>(P, N, M6, hits, stream);
}

furax_status furax_bj_invert(int64_t npix, const double *M6, const int32_t *hits,
                             double rcond_min, int32_t min_hits, double *Minv6, uint8_t *valid,
                             double *rcond, hipStream_t stream) {
  if (npix < 1) return set_error(FURAX_EINVAL, "npix must be >= 1");
  if (!M6 || !hits || !Minv6) return set_error(FURAX_EINVAL, "NULL array");
  if (!(rcond_min >= 0.0)) return set_error(FURAX_EINVAL, "rcond_min must be >= 0");
  return launch_bj_invert(npix, M6, hits, rcond_min, min_hits, nullptr, Minv6, valid, rcond,
                          stream);
}

int64_t furax_normal_workspace_bytes(const furax_pointing *P, const furax_noise *N,
                                     int32_t precision) {
  if (check_pointing(P) != FURAX_OK || !dtype_ok(precision)) return -1;
  if (check_noise(N, P->n_det, P->n_samp, precision) != FURAX_OK) return -1;
  return normal_workspace_bytes(P, N, precision);
}

furax_status furax_normal_apply(const furax_pointing *P, const furax_noise *N, int32_t precision,
                                const double *p, double *q, const uint8_t *valid, void *work,
                                hipStream_t stream) {
  FX_TRY(check_pointing(P));
  if (precision != P->dtype) return set_error(FURAX_EINVAL, "precision must equal the pointing dtype");
  FX_TRY(check_noise(N, P->n_det, P->n_samp, precision));
  if (!p || !q) return set_error(FURAX_EINVAL, "NULL p or q");
  if (precision == FURAX_F32) return normal_apply_impl<float>(P, N, p, q, valid, work, stream);
  return normal_apply_impl<double>(P, N, p, q, valid, work, stream);
}

furax_status furax_pcg_create(const furax_pointing *P, const furax_noise *N, int32_t tod_dt,
                              const void *tod, const furax_pcg_opts *opt, hipStream_t stream,
                              furax_pcg *out) {
  if (!out) return set_error(FURAX_EINVAL, "NULL handle output");
  *out = nullptr;
  FX_TRY(check_pointing(P));
  FX_TRY(check_pcg_opts(opt, P));
  FX_TRY(check_noise(N, P->n_det, P->n_samp, P->dtype));
  if (tod_dt != P->dtype) return set_error(FURAX_EINVAL, "tod dtype must equal the pointing dtype");
  if (P->n_samp > 0 && !tod) return set_error(FURAX_EINVAL, "NULL tod");
  return pcg_create(P, N, tod_dt, tod, opt, stream, out);
}

furax_status furax_pcg_iterate(furax_pcg h, int32_t n_iter) {
  if (!h) return set_error(FURAX_EINVAL, "NULL handle");
  if (n_iter < 0) return set_error(FURAX_EINVAL, "n_iter must be >= 0");
  return pcg_iterate(h, n_iter);
}

furax_status furax_pcg_finish(furax_pcg h, double *map_out, uint8_t *valid_out,
                              furax_pcg_info *info) {
  if (!h) return set_error(FURAX_EINVAL, "NULL handle");
  return pcg_finish(h, map_out, valid_out, info);
}

furax_status furax_pcg_destroy(furax_pcg h) { return pcg_destroy(h); }

furax_status furax_pcg_set_timing(furax_pcg h, int32_t enable) {
  if (!h) return set_error(FURAX_EINVAL, "NULL handle");
  return pcg_set_timing(h, enable);
}

furax_status furax_pcg_read_timing(furax_pcg h, furax_pcg_timing *out) {
  if (!h || !out) return set_error(FURAX_EINVAL, "NULL handle or output");
  return pcg_read_timing(h, out);
}

furax_status furax_pcg_mapmake(const furax_pointing *P, const furax_noise *N, int32_t tod_dt,
                               const void *tod, double *map_out, uint8_t *valid_out,
                               const furax_pcg_opts *opt, furax_pcg_info *info,
                               hipStream_t stream) {
  if (!map_out) return set_error(FURAX_EINVAL, "NULL map_out");
  furax_pcg h = nullptr;
  FX_TRY(furax_pcg_create(P, N, tod_dt, tod, opt, stream, &h));
  furax_status st = pcg_iterate(h, opt->max_iter);
  if (st == FURAX_OK) st = pcg_finish(h, map_out, valid_out, info);
  const std::string keep = g_last_error;
  const furax_status st2 = pcg_destroy(h);
  g_last_error = keep;
  return st != FURAX_OK ? st : st2;
}

furax_status furax_chi2(const furax_pointing *P, const furax_noise *N, int32_t map_dt,
                        const void *map, const void *tod, double *chi2_out, void *resid_w,
                        hipStream_t stream) {
  FX_TRY(check_pointing(P));
  FX_TRY(check_noise(N, P->n_det, P->n_samp, P->dtype));
  if (N->kind != 0) return set_error(FURAX_EUNSUPPORTED, "chi2 supports diagonal noise only");
  if (!dtype_ok(map_dt)) return set_error(FURAX_EINVAL, "bad map dtype");
  if (P->dtype == FURAX_F64 && map_dt != FURAX_F64)
    return set_error(FURAX_EINVAL, "FP64 pointing needs an FP64 map");
  if (!map || !chi2_out || (P->n_samp > 0 && !tod)) return set_error(FURAX_EINVAL, "NULL array");
  if (P->dtype == FURAX_F32)
    return chi2_impl<float>(P, N, map_dt, map, (const float *)tod, chi2_out, (float *)resid_w,
                            stream);
  return chi2_impl<double>(P, N, map_dt, map, (const double *)tod, chi2_out, (double *)resid_w,
                           stream);
}

furax_status furax_chi2_grad(const furax_pointing *P, const furax_noise *N, int32_t map_dt,
                             const void *map, const void *tod, double *chi2_out, double *grad_map,
                             double *grad_gain, double *grad_dpsi, hipStream_t stream) {
  FX_TRY(check_pointing(P));
  FX_TRY(check_noise(N, P->n_det, P->n_samp, P->dtype));
  if (N->kind != 0) return set_error(FURAX_EUNSUPPORTED, "chi2 supports diagonal noise only");
  if (!dtype_ok(map_dt)) return set_error(FURAX_EINVAL, "bad map dtype");
  if (P->dtype == FURAX_F64 && map_dt != FURAX_F64)
    return set_error(FURAX_EINVAL, "FP64 pointing needs an FP64 map");
  if (!map || (P->n_samp > 0 && !tod)) return set_error(FURAX_EINVAL, "NULL array");
  if (P->dtype == FURAX_F32)
    return chi2_grad_impl<float>(P, N, map_dt, map, (const float *)tod, chi2_out, grad_map,
                                 grad_gain, grad_dpsi, stream);
  return chi2_grad_impl<double>(P, N, map_dt, map, (const double *)tod, chi2_out, grad_map,
                                grad_gain, grad_dpsi, stream);
}

furax_status furax_chi2_grad_noalloc(const furax_pointing *P, const furax_noise *N,
                                     int32_t map_dt, const void *map, const void *tod,
                                     double *chi2_out, double *grad_map, double *grad_gain,
                                     double *grad_dpsi, hipStream_t stream) {
  FX_TRY(check_pointing(P));
  FX_TRY(check_noise(N, P->n_det, P->n_samp, P->dtype));
  if (N->kind != 0) return set_error(FURAX_EUNSUPPORTED, "chi2 supports diagonal noise only");
  if (!dtype_ok(map_dt)) return set_error(FURAX_EINVAL, "bad map dtype");
  if (P->dtype == FURAX_F64 && map_dt != FURAX_F64)
    return set_error(FURAX_EINVAL, "FP64 pointing needs an FP64 map");
  if (!map || (P->n_samp > 0 && !tod)) return set_error(FURAX_EINVAL, "NULL array");
  if (P->dtype == FURAX_F32)
    return chi2_grad_noalloc_impl<float>(P, N, map_dt, map, (const float *)tod, chi2_out,
                                         grad_map, grad_gain, grad_dpsi, stream);
  return chi2_grad_noalloc_impl<double>(P, N, map_dt, map, (const double *)tod, chi2_out,
                                        grad_map, grad_gain, grad_dpsi, stream);
}

furax_status furax_pointing_vjp(const furax_pointing *P, int32_t map_dt, const void *map,
                                const void *tod_cot, double *grad_map, double *grad_gain,
                                double *grad_dpsi, hipStream_t stream) {
  FX_TRY(check_pointing(P));
  if (!dtype_ok(map_dt)) return set_error(FURAX_EINVAL, "bad map dtype");
  if (P->dtype == FURAX_F64 && map_dt != FURAX_F64)
    return set_error(FURAX_EINVAL, "FP64 pointing needs an FP64 map");
  if (P->n_samp > 0 && !tod_cot) return set_error(FURAX_EINVAL, "NULL cotangent");
  if ((grad_gain || grad_dpsi) && !map) return set_error(FURAX_EINVAL, "NULL map");
  if (P->dtype == FURAX_F32)
    return vjp_impl<float>(P, map_dt, map, (const float *)tod_cot, grad_map, grad_gain, grad_dpsi,
                           stream);
  return vjp_impl<double>(P, map_dt, map, (const double *)tod_cot, grad_map, grad_gain, grad_dpsi,
                          stream);
}

furax_status furax_stream_copy(const void *src, void *dst, int64_t bytes, int32_t nontemporal,
                               hipStream_t stream) {
  if (bytes < 0 || (bytes & 15)) return set_error(FURAX_EINVAL, "bytes must be a multiple of 16");
  if (bytes > 0 && (!src || !dst)) return set_error(FURAX_EINVAL, "NULL buffer");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
    return set_error(FURAX_EINVAL, "buffers must be 16-byte aligned");
  if (bytes == 0) return FURAX_OK;
  const int64_t n16 = bytes / 16;
  // a few waves of workgroups per CU, each thread streaming many 16-byte words
  const unsigned grid = (unsigned)std::min<int64_t>((n16 + kBlock - 1) / kBlock, 256 * 32);
  if (nontemporal)
    hipLaunchKernelGGL(fx::k_stream_copy<true>, dim3(grid), dim3(kBlock), 0, stream,
                       static_cast<const fx::u32x4 *>(src), static_cast<fx::u32x4 *>(dst), n16);
  else
    hipLaunchKernelGGL(fx::k_stream_copy<false>, dim3(grid), dim3(kBlock), 0, stream,
                       static_cast<const fx::u32x4 *>(src), static_cast<fx::u32x4 *>(dst), n16);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}

}  // extern "C"
