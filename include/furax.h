/*
 * furax.h -- C ABI of the MI355X (gfx950) map-making hot path.
 *
 * The library applies the operators of the generalised-least-squares
 * map-making problem of the paper's Eq. (1)-(2) with no templates:
 *
 *     d = P m + n,      m_hat = (P^T N^-1 P)^-1 P^T N^-1 d,
 *
 * where P is the pointing operator (section "Software Design": the
 * PointingOperator / IndexOperator / QURotationOperator / HWPOperator /
 * LinearPolarizerOperator of Tables 2-3, collapsed by the rotation-merging and
 * HWP-commutation rules of "Algebraic reductions"), N^-1 is block-diagonal over
 * detectors (HomothetyOperator or SymmetricBandToeplitzOperator, Table 2), and
 * the inverse is taken by block-Jacobi preconditioned conjugate gradients
 * ("Map-making classes": BJPreconditioner; Table 1: A.I(solver, preconditioner)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array pointer is a DEVICE pointer (HBM of the current HIP device)
 *    unless marked HOST.  The caller owns every buffer; the library never
 *    frees caller memory and never keeps a pointer after a call returns
 *    (except inside a furax_pcg handle, see below).
 *  - Maps are planar Stokes IQU, [3][npix] row-major (I plane, then Q, then U),
 *    npix = 12 nside^2, HEALPix RING ordering.
 *  - Time-ordered data (TOD) and pointing planes are [n_det][n_samp] row-major.
 *  - Angles are radians.  theta is colatitude in [0, pi], phi longitude.
 *  - A sample whose theta/phi is non-finite or whose theta is outside [0, pi]
 *    has pixel -1: it reads 0 in P and contributes nothing to P^T.
 *  - Pixel indices are computed in FP64 without fused multiply-add, so they
 *    are bit-identical to a plain IEEE FP64 evaluation of the ring-scheme
 *    formulas (up to a 1-ulp difference of the cosine, see ang2pix).
 *  - Every call validates all arguments BEFORE any launch and returns
 *    FURAX_EINVAL with no side effect on a bad argument.  HIP failures return
 *    FURAX_EHIP.  furax_last_error() gives a thread-local message for the last
 *    non-OK status.  No C++ exception crosses this boundary.
 *  - Calls taking a hipStream_t enqueue their work on that stream and return
 *    without synchronising (except where stated), so buffers must stay valid
 *    until the stream reaches that point.  Stream 0 is the legacy default stream.
 */
#ifndef FURAX_H
#define FURAX_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FURAX_OK = 0,
  FURAX_EINVAL = 1,        /* invalid argument; nothing was launched            */
  FURAX_ENOMEM = 2,        /* device allocation failed                          */
  FURAX_EHIP = 3,          /* a HIP runtime call failed                         */
  FURAX_EBREAKDOWN = 4,    /* PCG breakdown: <p,Ap> <= 0, <r,z> <= 0 or non-finite */
  FURAX_ENOTCONV = 5,      /* PCG reached max_iter without meeting rtol         */
  FURAX_EUNSUPPORTED = 6   /* valid but unsupported combination (e.g. band too wide) */
} furax_status;

typedef enum { FURAX_F32 = 0, FURAX_F64 = 1 } furax_dtype;

/* The pointing operator P: StokesIQU map (HEALPix ring, nside) -> TOD.
 *
 *   tod[k,i] = g_k * ( I[p] + Q[p] cos(2 psi_eff) + U[p] sin(2 psi_eff) ),
 *   p        = ang2pix_ring(nside, theta[k,i], phi[k,i]),
 *   psi_eff  = psi[k,i] + dpsi_k + 2 alpha_i                     (hwp = 1)
 *            = psi[k,i] + dpsi_k                                  (hwp = 0),
 *   alpha_i  = 2 pi ((hwp_num * i) mod hwp_den) / hwp_den + hwp_phase0.
 *
 * The merged angle follows from adding consecutive QU rotations and from the
 * ideal-HWP identity R(t) o HWP = HWP o R(-t) ("Algebraic reductions"); the
 * HWP angle is formed from integers so that long scans keep full precision.
 * Pointing is expanded on the fly at every application, never stored
 * (PointingOperator, "Map-making classes").
 *
 * Two representations of the pointing are accepted:
 *  - angle planes: theta, phi, psi given per sample (bore_quat = det_quat =
 *    NULL), in the dtype of the struct;
 *  - boresight quaternions (theta = phi = psi = NULL): the time-dependent
 *    telescope attitude q_b[i] ([n_samp][4] FP64, (w, x, y, z), unit norm)
 *    and each detector's fixed attitude relative to it q_k ([n_det][4] FP64).
 *    Every application expands, per sample, q = q_b[i] (x) q_k (Hamilton
 *    product), the line of sight d = R(q) z_hat and the polarisation
 *    direction e = R(q) x_hat; then
 *        p   = ring pixel of (z = d_z clipped to [-1, 1], phi = atan2(d_y, d_x)),
 *        psi = atan2(-e . e_phi, -e . e_theta)   (from local north towards
 *              west, the HEALPix convention; 0 where both vanish),
 *    and the formulas above apply with that psi.  The rotation is evaluated
 *    in FP64 without fused multiply-add in both precisions, so pixels are
 *    those of a plain IEEE evaluation (up to a 1-ulp difference of atan2).
 *    dtype then selects the TOD precision and the precision of the
 *    polariser products.  Both arrays must be 16-byte aligned.  The per-sample
 *    pointing stream disappears: 32 bytes per time sample serve every
 *    detector. */
typedef struct {
  int64_t nside;           /* 1 <= nside <= 8192                                     */
  int64_t n_det, n_samp;   /* n_det >= 1, n_samp >= 0                                */
  int32_t dtype;           /* furax_dtype of theta/phi/psi                           */
  const void *theta;       /* [n_det][n_samp], or NULL with bore_quat                */
  const void *phi;         /* [n_det][n_samp], or NULL with bore_quat                */
  const void *psi;         /* [n_det][n_samp], or NULL with bore_quat                */
  const double *gain;      /* [n_det] or NULL (all 1)                                */
  const double *dpsi;      /* [n_det] or NULL (all 0): polarisation-angle offsets    */
  int32_t hwp;             /* 0: no half-wave plate, 1: ideal HWP                    */
  int64_t hwp_num;         /* HWP turns per hwp_den samples (f_hwp / f_samp = num/den) */
  int64_t hwp_den;         /* > 0 when hwp = 1                                       */
  double hwp_phase0;       /* HWP angle at sample 0                                  */
  const double *bore_quat; /* [n_samp][4] or NULL: boresight attitude per sample     */
  const double *det_quat;  /* [n_det][4] (with bore_quat): detector attitudes        */
} furax_pointing;

/* The weight of the estimator, block-diagonal over detectors
 * (BlockDiagonalOperator of Table 2): N^-1, or with templates the weighting
 * and deprojection operator F_T of Eq. (3).
 *  kind 0 (HomothetyOperator / DiagonalOperator): z[k,i] = inv_var[k] y[k,i].
 *  kind 1 (SymmetricBandToeplitzOperator): truncated linear convolution of each
 *     detector's stream with its symmetric band of lags t[0..b-1],
 *         z[k,i] = sum_{|tau| <= b-1, 0 <= i+tau < n_samp} t_k[|tau|] y[k,i+tau],
 *     applied by overlap-save blocks with a real FFT (the paper's overlap-save
 *     method).  Both precisions support b <= 8192 (FP64 with b > 4096 also needs
 *     n_samp < 2^28, else FURAX_EUNSUPPORTED).
 *  kind 2 (template deprojection, Eq. (3) with TemplateOperator templates):
 *         z = F_T y,  F_T = W - W T (T^T W T)^-1 T^T W,  W = diag(inv_var[k]),
 *     where T holds, per detector and per segment of tmpl_seg_len samples
 *     (the last segment running to the end of the stream, so segments have
 *     tmpl_seg_len to 2 tmpl_seg_len - 1 samples, or the whole stream when it
 *     is shorter), the Legendre polynomials P_0 .. P_tmpl_order of
 *     x = (2 (i - i0) + 1) / len - 1.  F_T removes every baseline of that form
 *     from each segment: z = w_k (y - T_s (T_s^T T_s)^-1 T_s^T y).  Needs
 *     0 <= tmpl_order <= 7, tmpl_seg_len > tmpl_order and n_samp > tmpl_order.
 *     The projections are accumulated in FP64 in both precisions. */
typedef struct {
  int32_t kind;            /* 0 diagonal, 1 symmetric band-Toeplitz, 2 template deprojection */
  int64_t n_det, n_samp;   /* must equal the pointing's when used together           */
  const double *inv_var;   /* kinds 0 and 2: [n_det]                                 */
  int64_t bandwidth;       /* kind 1: b >= 1 lags                                    */
  const double *toeplitz;  /* kind 1: [1][b] (stride 0) or [n_det][b] (stride b)     */
  int64_t toeplitz_stride; /* 0: one kernel shared by all detectors; b: per detector */
  int64_t tmpl_seg_len;    /* kind 2: samples per template segment                   */
  int32_t tmpl_order;      /* kind 2: highest Legendre degree of the baselines       */
} furax_noise;

/* HEALPix ring-scheme pixel of each direction (Landscape types, section
 * "Software Design"; the ring-scheme formulas of Gorski et al. 2005).
 * theta, phi: [n] of dtype dt.  pix_out: [n] int64, -1 for invalid input.
 * FP64 arithmetic without contraction; FP32 input is promoted exactly.  The
 * device cosine may differ from another libm's by 1 ulp, which can move a
 * direction lying within ~1 ulp of a pixel boundary. */
furax_status furax_ang2pix(int64_t nside, int32_t dt, const void *theta, const void *phi,
                           int64_t n, int64_t *pix_out, hipStream_t stream);

/* tod = P map.  map: [3][npix] of dtype map_dt; tod: [n_det][n_samp] of dtype
 * tod_dt (overwritten).  Supported: all-F64; F32 pointing with F32 tod and an
 * F32 or F64 map. */
furax_status furax_pointing_apply(const furax_pointing *P, int32_t map_dt, const void *map,
                                  int32_t tod_dt, void *tod, hipStream_t stream);

/* map (+)= P^T tod (the transpose of IndexOperator: a scatter-add binning).
 * tod: [n_det][n_samp] of dtype tod_dt (same dtype as the pointing, or F64
 * tod with F32 pointing); map: [3][npix] FP64, overwritten (accumulate = 0)
 * or added to (accumulate = 1).  Products are formed in the pointing dtype and
 * accumulated in FP64 (LDS-privatised per tile, then FP64 atomics), so the
 * summation order, hence the last bits, may vary from run to run. */
furax_status furax_pointing_transpose(const furax_pointing *P, int32_t tod_dt, const void *tod,
                                      double *map, int32_t accumulate, hipStream_t stream);

/* tod_out = N^-1 tod_in for TOD [n_det][n_samp] of dtype dt.  For kind 0
 * tod_in may equal tod_out; for kind 1 the buffers must not overlap. */
furax_status furax_noise_apply(const furax_noise *N, int32_t dt, const void *tod_in,
                               void *tod_out, hipStream_t stream);

/* Block-Jacobi preconditioner ("BJPreconditioner", "Map-making classes"):
 * per-pixel 3x3 blocks of P^T diag(N^-1) P, where diag(N^-1) is inv_var[k]
 * (kinds 0 and 2: the weight without its template projection) or t_k[0]
 * (kind 1).
 *   M6:   [6][npix] FP64 out: entries II, IQ, IU, QQ, QU, UU.
 *   hits: [npix] int32 out: unflagged samples per pixel (exact).
 * furax_bj_invert then writes Minv6 [6][npix] and valid [npix] (1 iff
 * hits >= min_hits and the 1-norm reciprocal condition number
 * 1/(|M|_1 |M^-1|_1) >= rcond_min; Minv is 0 elsewhere) and, if rcond is not
 * NULL, rcond [npix] FP64.  M^-1 comes from the Cholesky factorisation of the
 * (positive semi-definite) block, so a block that is singular in exact
 * arithmetic gets a tiny rcond; a non-positive pivot gives rcond 0 and
 * Minv 0. */
furax_status furax_bj_build(const furax_pointing *P, const furax_noise *N, double *M6,
                            int32_t *hits, hipStream_t stream);
furax_status furax_bj_invert(int64_t npix, const double *M6, const int32_t *hits,
                             double rcond_min, int32_t min_hits, double *Minv6,
                             uint8_t *valid, double *rcond, hipStream_t stream);

/* q = P^T N^-1 P p, the normal operator of Eq. (2), applied as the
 * block decomposition sum_k P_k^T N_k^-1 P_k ("Algebraic reductions").
 *   precision: F64 (plain FP64 throughout) or F32 (FP32 pointing, TOD and
 *              FFT arithmetic; FP64 accumulation of q); must equal P->dtype.
 *   p: [3][npix] FP64 in.  q: [3][npix] FP64 out (overwritten).
 *   valid: [npix] uint8 or NULL.  When given, samples in pixels with
 *          valid = 0 are flagged (read 0, contribute nothing).
 *   work: device scratch of furax_normal_workspace_bytes() bytes, or NULL to
 *         let the library allocate it stream-ordered for this call.
 * With band N and a power-of-two nside the call also builds, stream-ordered,
 * the per-sample schedule of its P^T (samples sorted by nested superpixel of
 * 1024 pixels) and frees it before returning; a PCG session builds that
 * schedule once and reuses it for every iteration.  Its P^T adds each
 * superpixel's samples into FP64 sums with several waves at once, so the
 * summation order, hence the last bits of q, may vary from run to run. */
int64_t furax_normal_workspace_bytes(const furax_pointing *P, const furax_noise *N,
                                     int32_t precision);
furax_status furax_normal_apply(const furax_pointing *P, const furax_noise *N, int32_t precision,
                                const double *p, double *q, const uint8_t *valid, void *work,
                                hipStream_t stream);

/* Block-Jacobi PCG map-maker: solves (P^T N^-1 P) m = P^T N^-1 d for the
 * valid pixels (Eq. (2) with T = 0, as the estimator (H.T @ N.I @ H).I @
 * H.T @ N.I of the section's listing).  Samples falling in invalid pixels are
 * flagged in both P and P^T.  x0 = 0; stop when |r|_2/|b|_2 <= rtol or after
 * max_iter iterations.  Dot products and scalars are FP64 on the device
 * (deterministic two-pass reductions); x and r are FP64 in both precisions. */
typedef struct {
  int32_t max_iter;        /* >= 0                                                   */
  double rtol;             /* >= 0; 0 runs exactly max_iter iterations              */
  int32_t precision;       /* furax_dtype: F64 plain, or F32 (FP32 TOD/pointing math) */
  double rcond_min;        /* validity threshold on the 3x3 blocks (e.g. 1e-3)      */
  int32_t min_hits;        /* validity threshold on hits (e.g. 3)                   */
  const uint8_t *valid_in; /* [npix] or NULL: use this mask instead of the thresholds */
  int32_t no_early_exit;   /* 1: never read the residual back; run max_iter iterations */
} furax_pcg_opts;

typedef struct {
  int32_t iters;           /* iterations performed                                  */
  int32_t stop_reason;     /* 0 max_iter, 1 rtol reached, 2 breakdown               */
  double rel_resid;        /* |r|_2 / |b|_2 at exit                                 */
  double *resid_history;   /* HOST [max_iter + 1] or NULL: |r_k|/|b| for k = 0..iters */
  int64_t n_valid;         /* number of valid pixels                                */
} furax_pcg_info;

/* One call: build the preconditioner and the right-hand side, iterate, write
 * map_out [3][npix] FP64 (0 on invalid pixels) and valid_out [npix] (or NULL).
 * Allocates its workspace stream-ordered on `stream` and is synchronous on
 * return.  Returns FURAX_OK, FURAX_ENOTCONV (max_iter reached with rtol > 0;
 * the map is still written) or FURAX_EBREAKDOWN (the last good iterate is
 * written). */
furax_status furax_pcg_mapmake(const furax_pointing *P, const furax_noise *N, int32_t tod_dt,
                               const void *tod, double *map_out, uint8_t *valid_out,
                               const furax_pcg_opts *opt, furax_pcg_info *info,
                               hipStream_t stream);

/* The same solver as a resumable session, so that a caller can time or
 * checkpoint individual iterations.  furax_pcg_create copies *P, *N and *opt
 * (not the arrays they point to, which must stay valid until
 * furax_pcg_destroy), builds the preconditioner and b = P^T N^-1 d, and sets
 * x0 = 0, r0 = b, z0 = M^-1 r0, p0 = z0.  furax_pcg_iterate runs up to
 * n_iter further iterations without any host synchronisation when
 * opt->no_early_exit = 1 (it then never detects convergence or breakdown;
 * furax_pcg_finish checks them).  furax_pcg_finish synchronises, writes the
 * current iterate and fills info (resid_history is filled only for sessions
 * created with no_early_exit = 0). */
typedef struct furax_pcg_state *furax_pcg;
furax_status furax_pcg_create(const furax_pointing *P, const furax_noise *N, int32_t tod_dt,
                              const void *tod, const furax_pcg_opts *opt, hipStream_t stream,
                              furax_pcg *out);
furax_status furax_pcg_iterate(furax_pcg h, int32_t n_iter);
furax_status furax_pcg_finish(furax_pcg h, double *map_out, uint8_t *valid_out,
                              furax_pcg_info *info);
furax_status furax_pcg_destroy(furax_pcg h);

/* Device time of each phase of the iterations, for profiling a session.
 * After furax_pcg_set_timing(h, 1), every furax_pcg_iterate iteration records
 * HIP events on the session's stream between its phases (a few microseconds
 * per iteration).  furax_pcg_read_timing synchronises the stream, returns the
 * sums over the iterations timed since the previous read and resets them.
 * With diagonal noise, P, N^-1 and P^T are one fused kernel, reported as
 * ms_transpose (ms_apply = ms_noise = 0). */
typedef struct {
  int32_t iters;           /* timed iterations                                      */
  double ms_apply;         /* P: pointing expanded, map gathered into the TOD      */
  double ms_noise;         /* N^-1                                                  */
  double ms_transpose;     /* P^T: binning into the map                            */
  double ms_update;        /* dot products, preconditioner, vector updates         */
} furax_pcg_timing;
furax_status furax_pcg_set_timing(furax_pcg h, int32_t enable);
furax_status furax_pcg_read_timing(furax_pcg h, furax_pcg_timing *out);

/* Chi-square of the data model Eq. (1) and its vector-Jacobian product
 * (the differentiable path of "Summary" / "Research Impact Statement").
 * With s = P m (gains and angle offsets of P included) and r = d - s:
 *   furax_chi2:         chi2 = r^T N^-1 r (diagonal N only), written to
 *                       *chi2_out (device FP64 scalar); u = N^-1 r is written
 *                       to resid_w [n_det][n_samp] (dtype of P) if not NULL.
 *   furax_pointing_vjp: for a TOD cotangent u (dtype of P),
 *     grad_map  [3][npix] FP64  (+)= P^T u               (accumulated),
 *     grad_gain [n_det] FP64     = sum_i u[k,i] (P_1 m)[k,i]   (P_1: unit gain),
 *     grad_dpsi [n_det] FP64     = sum_i u[k,i] g_k (-2 Q sin 2psi_eff + 2 U cos 2psi_eff),
 *   i.e. the transpose of the Jacobian of s with respect to (m, g, dpsi).
 *   Any of grad_map / grad_gain / grad_dpsi may be NULL to skip it. Pointing
 *   is recomputed, not stored. */
furax_status furax_chi2(const furax_pointing *P, const furax_noise *N, int32_t map_dt,
                        const void *map, const void *tod, double *chi2_out, void *resid_w,
                        hipStream_t stream);
furax_status furax_pointing_vjp(const furax_pointing *P, int32_t map_dt, const void *map,
                                const void *tod_cot, double *grad_map, double *grad_gain,
                                double *grad_dpsi, hipStream_t stream);

/* The gradient of chi2 = r^T N^-1 r, r = d - P m (diagonal N), with respect
 * to the map, the detector gains and the polarisation-angle offsets, in one
 * pass over the pointing (recomputed, not stored):
 *   grad_map  [3][npix] FP64 (+)= -2 P^T (N^-1 r)                (accumulated),
 *   grad_gain [n_det] FP64     =  -2 sum_i u[k,i] (P_1 m)[k,i],    u = N^-1 r,
 *   grad_dpsi [n_det] FP64     =  -2 sum_i u[k,i] g_k (-2 Q sin 2psi_eff + 2 U cos 2psi_eff),
 *   chi2_out  (device FP64 scalar, or NULL) = chi2 at the same point.
 * Any output may be NULL to skip it.  tod: [n_det][n_samp] of the pointing's
 * dtype; the map as for furax_chi2.  The per-detector sums and chi2 are
 * deterministic (fixed-order FP64 reductions); the map gradient is binned in
 * LDS per sample tile and flushed with FP64 atomics, so its last bits may
 * vary from run to run.  Allocates its partial sums stream-ordered. */
furax_status furax_chi2_grad(const furax_pointing *P, const furax_noise *N, int32_t map_dt,
                             const void *map, const void *tod, double *chi2_out, double *grad_map,
                             double *grad_gain, double *grad_dpsi, hipStream_t stream);

/* Template fit of a noise model of kind 2 (TemplateOperator, Eq. (1)/(3)):
 * the amplitudes t = (T^T W T)^-1 T^T W y of every detector's and segment's
 * Legendre baselines, e.g. of the residual d - P m after a solve.
 *   tod: [n_det][n_samp] of dtype dt.  amp: [n_det][n_seg][tmpl_order + 1]
 *   FP64 out, n_seg = max(1, n_samp / tmpl_seg_len) (segments as for F_T). */
furax_status furax_template_fit(const furax_noise *N, int32_t dt, const void *tod, double *amp,
                                hipStream_t stream);

/* Gap filling by constrained Gaussian realisations (the band-Toeplitz
 * operator's use named after Table 2).  For every detector with missing
 * samples G and valid samples V:
 *     out_G = n_G + N_GV N_VV^-1 (d_V - n_V),    out_V = d_V,
 * where N is the noise COVARIANCE described by C (kind 1: band-Toeplitz
 * autocorrelation lags c[0..b-1], b <= 8192, truncated at the stream's ends;
 * kind 0: white, then out_G = n_G) and n is an unconstrained realisation of
 * it drawn by the caller.  N_VV^-1 is applied by conjugate gradients on all
 * detectors at once (each with its own scalars), preconditioned by 1/c_k[0],
 * in FP64 whatever dt is, until every detector's |r|/|b| <= rtol or max_iter.
 *   gaps: [n_det][n_samp] uint8, nonzero = missing.  tod, noise_real, out:
 *   [n_det][n_samp] of dtype dt (out may alias tod or noise_real).
 * Allocates 4 FP64 TOD-sized vectors stream-ordered; synchronous on return.
 * Returns FURAX_ENOTCONV when max_iter is reached with rtol > 0 (out is
 * still written) and FURAX_EBREAKDOWN on a non-finite residual. */
typedef struct {
  int32_t max_iter;        /* >= 0                                                   */
  double rtol;             /* >= 0                                                   */
} furax_gapfill_opts;
typedef struct {
  int32_t iters;           /* CG iterations performed                                */
  double rel_resid;        /* largest |r_k| / |b_k| over the detectors at exit       */
} furax_gapfill_info;
furax_status furax_gap_fill(const furax_noise *C, int32_t dt, const uint8_t *gaps,
                            const void *tod, const void *noise_real, void *out,
                            const furax_gapfill_opts *opt, furax_gapfill_info *info,
                            hipStream_t stream);

/* furax_chi2_grad for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments and results as furax_chi2_grad; it calls no hipMalloc,
 * hipFree or allocating library routine.  Its FP64 partial sums live in a
 * static device array of 2^21 values (16 MiB) that every GPU the library runs
 * on holds until the process ends (its address is looked up on the first call
 * on each device).  A problem needing more partial sums than that -- one per
 * sample tile plus two per detector and time block, e.g. 64 detectors x 2^20
 * samples needs 5.3e5 -- returns FURAX_EUNSUPPORTED with nothing launched.
 * Calls that overlap on one GPU (concurrent streams or threads) share the
 * array and race; serialise them.  Every partial sum is written before it is
 * read, so consecutive calls need no clearing. */
furax_status furax_chi2_grad_noalloc(const furax_pointing *P, const furax_noise *N,
                                     int32_t map_dt, const void *map, const void *tod,
                                     double *chi2_out, double *grad_map, double *grad_gain,
                                     double *grad_dpsi, hipStream_t stream);

/* Measurement utility, not a step of the method: dst[0 .. bytes) =
 * src[0 .. bytes) on the device (bytes a multiple of 16, both buffers 16-byte
 * aligned and not overlapping).  nontemporal = 1 moves the data with
 * non-temporal loads and stores, the cache policy of the kernels' pointing and
 * TOD streams; 0 with plain ones.  It gives the achievable read + write HBM
 * bandwidth beside the kernels, and a kernel of known traffic that calibrates
 * the profiler's memory counters. */
furax_status furax_stream_copy(const void *src, void *dst, int64_t bytes, int32_t nontemporal,
                               hipStream_t stream);

/* Thread-local description of the last non-OK status (never NULL). */
const char *furax_last_error(void);
/* Frees the library's per-device FFT twiddle tables (rebuilt on demand). */
void furax_release_caches(void);
/* ABI version: major * 10000 + minor * 100 + patch. */
int32_t furax_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FURAX_H */
