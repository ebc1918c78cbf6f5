// Internal declarations shared by the library's translation units: device-side
// pointing math, kernel argument bundles and host-side error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

#include "furax.h"

namespace fx {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxNside = 8192;
constexpr int kMaxTmplOrder = 7;   // highest Legendre degree of the deprojected baselines

// ---------------------------------------------------------------------------
// Host-side status plumbing.
// ---------------------------------------------------------------------------
furax_status set_error(furax_status st, const std::string &msg);
furax_status hip_error(hipError_t e, const char *what);

#define FX_HIP(call)                                                   \
  do {                                                                 \
    hipError_t fx_e_ = (call);                                         \
    if (fx_e_ != hipSuccess) return ::fx::hip_error(fx_e_, #call);     \
  } while (0)

#define FX_TRY(call)                                                   \
  do {                                                                 \
    furax_status fx_s_ = (call);                                       \
    if (fx_s_ != FURAX_OK) return fx_s_;                               \
  } while (0)

// ---------------------------------------------------------------------------
// Pointing operator arguments as passed to kernels (by value).
// ---------------------------------------------------------------------------
template <typename T>
struct PtArgs {
  const T *theta, *phi, *psi;
  const double *gain;   // may be null
  const double *dpsi;   // may be null
  int64_t n_det, n_samp;
  int32_t nside;
  int32_t hwp;
  int64_t hwp_num_mod, hwp_den;   // hwp_num reduced mod hwp_den
  double hwp_phase0;
  const uint8_t *valid; // [npix] or null: samples in pixels with valid == 0 are flagged
  const double *qb;     // [n_samp][4] boresight attitudes, or null (angle planes)
  const double *qd;     // [n_det][4] detector attitudes (with qb)
  // [n_det] or null: the order in which sample tiles take the detectors (a
  // permutation that puts detectors seeing the same sky next to each other)
  const int32_t *det_perm;
};

// HEALPix ring-scheme pixel in FP64 (ring-scheme formulas of Gorski et al.
// 2005) of the direction with z = cos(theta) and longitude phi, both already
// validated.  Every operation is rounded on its own (no contraction) so that
// the result equals a plain IEEE evaluation of the same expression sequence.
__device__ __forceinline__ int32_t pix_of_z(int32_t n, double z, double phi) {
#pragma clang fp contract(off)
  const double N = (double)n;
  const double two_pi = 2.0 * kPi;
  constexpr double half_pi_c = 0.5 * kPi;
  const double half_pi = half_pi_c;
  const double za = fabs(z);
  // fmod(phi, 2 pi) is phi itself on [0, 2 pi): skip the library call there
  double phr = (phi >= 0.0 && phi < two_pi) ? phi : fmod(phi, two_pi);
  if (phr < 0.0) phr = phr + two_pi;
  // tt = phr / (pi/2) rounded as IEEE division does, from phr * RN(2/pi) and
  // one residual correction (Markstein): equal to the quotient for phr >
  // 2^-900; below that tt only meets 0.5 + tt and floors, which round alike.
  constexpr double inv_half_pi = 1.0 / half_pi_c;
  const double q0 = phr * inv_half_pi;
  const double tt = fma(fma(-q0, half_pi, phr), inv_half_pi, q0);   // in [0, 4]
  int32_t pix;
  if (za <= 2.0 / 3.0) {
    const double t1 = N * (0.5 + tt);
    const double t2 = (0.75 * N) * z;
    const int32_t jp = (int32_t)floor(t1 - t2);
    const int32_t jm = (int32_t)floor(t1 + t2);
    const int32_t ir = n + 1 + jp - jm;                 // 1 .. 2n+1
    const int32_t kshift = 1 - (ir & 1);
    int32_t ip = (jp + jm - n + kshift + 1) / 2;        // in [0, 4n + 1]
    if (ip >= 4 * n) ip -= 4 * n;                       // ip mod 4n
    pix = 2 * n * (n - 1) + (ir - 1) * (4 * n) + ip;
  } else {
    const double tp = tt - floor(tt);
    const double w = N * sqrt(3.0 * (1.0 - za));
    const int32_t jp = (int32_t)floor(tp * w);
    const int32_t jm = (int32_t)floor((1.0 - tp) * w);
    const int32_t ir = jp + jm + 1;                     // 1 .. n
    int32_t ip = (int32_t)floor(tt * (double)ir);       // in [0, 4 ir]
    if (ip >= 4 * ir) ip -= 4 * ir;                     // ip mod 4 ir
    pix = (z > 0.0) ? 2 * ir * (ir - 1) + ip : 12 * n * n - 2 * ir * (ir + 1) + ip;
  }
  return ((uint32_t)pix < (uint32_t)(12 * n * n)) ? pix : -1;
}

// ---------------------------------------------------------------------------
// cos t for t in [0, pi] in FP64, within one ulp: a colatitude needs neither
// the general range reduction nor both of the sine and cosine series that a
// library cos evaluates for every argument.
//
// Reduction: t <= pi/4 is kept (x = t); above, x = c - t with c = pi/2 (up to
// 3 pi/4) or c = pi, c held as hi + lo.  hi - t is exact (Sterbenz: t lies in
// [hi/2, 2 hi] on each sub-range) and lo joins it by Fast2Sum, so x + xl
// equals c - t to ~2^-106 relative with |x| <= pi/4.  Then
//   cos t = cos x (t <= pi/4),  sin x (middle),  -cos x (t >= 3 pi/4).
// The series are Taylor's, truncated where the next term is below 2^-60 of
// the value on |x| <= pi/4 (sin to x^17, cos to x^18), with the coefficients
// RN(1/n!).  Both kernels evaluate the small terms first and add the leading
// one last, with the tail xl entering to first order, after the kernels of
// Sun's fdlibm (k_sin, k_cos): for cos, 1 - x^2/2 is rounded to w and its
// rounding error (1 - w) - x^2/2, exact by Sterbenz, is added back.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sin_kernel(double x, double xl) {
#pragma clang fp contract(off)
  constexpr double S1 = -1.0 / 6.0, S2 = 1.0 / 120.0, S3 = -1.0 / 5040.0,
                   S4 = 1.0 / 362880.0, S5 = -1.0 / 39916800.0, S6 = 1.0 / 6227020800.0,
                   S7 = -1.0 / 1307674368000.0, S8 = 1.0 / 355687428096000.0;
  const double z = x * x, v = z * x;
  double r = fma(z, S8, S7);
  r = fma(z, r, S6);
  r = fma(z, r, S5);
  r = fma(z, r, S4);
  r = fma(z, r, S3);
  r = fma(z, r, S2);
  r = fma(z, r, S1);                      // sin x = x + v r
  const double tail = fma(-0.5 * z, xl, xl);   // xl cos x to first order
  return x + fma(v, r, tail);
}

__device__ __forceinline__ double cos_kernel(double x, double xl) {
#pragma clang fp contract(off)
  constexpr double C2 = 1.0 / 24.0, C3 = -1.0 / 720.0, C4 = 1.0 / 40320.0,
                   C5 = -1.0 / 3628800.0, C6 = 1.0 / 479001600.0, C7 = -1.0 / 87178291200.0,
                   C8 = 1.0 / 20922789888000.0, C9 = -1.0 / 6402373705728000.0;
  const double z = x * x;
  double r = fma(z, C9, C8);
  r = fma(z, r, C7);
  r = fma(z, r, C6);
  r = fma(z, r, C5);
  r = fma(z, r, C4);
  r = fma(z, r, C3);
  r = fma(z, r, C2);                      // cos x = 1 - z/2 + z^2 r
  const double hz = 0.5 * z, w = 1.0 - hz;
  const double small = fma(z * z, r, -(x * xl));   // - x xl: the tail, to first order
  return w + (((1.0 - w) - hz) + small);
}

__device__ __forceinline__ double cos_0pi(double t) {
#pragma clang fp contract(off)
  constexpr double kPio2Hi = 1.5707963267948966;     // RN(pi/2)
  constexpr double kPio2Lo = 6.123233995736766e-17;  // RN(pi/2 - kPio2Hi)
  constexpr double kPiHi = 3.141592653589793;        // RN(pi)
  constexpr double kPiLo = 1.2246467991473532e-16;   // RN(pi - kPiHi)
  constexpr double kQuarter = 0.7853981633974483;    // ~pi/4
  constexpr double kThreeQuarter = 2.356194490192345;  // ~3 pi/4
  const bool far = t >= kThreeQuarter;
  const double hi = far ? kPiHi : kPio2Hi, lo = far ? kPiLo : kPio2Lo;
  const double xh = hi - t;               // exact
  double x = xh + lo;
  double xl = (xh - x) + lo;              // Fast2Sum: |xh| >= |lo| or xh = 0
  const bool near = t <= kQuarter;
  x = near ? t : x;
  xl = near ? 0.0 : xl;
  if (!near && !far) return sin_kernel(x, xl);
  const double c = cos_kernel(x, xl);
  return far ? -c : c;
}

// Ring pixel of (theta, phi) with z = cos_0pi(theta).  Returns -1 for
// non-finite input or theta outside [0, pi].  FP32 angles are promoted
// exactly.
__device__ __forceinline__ int32_t ang2pix_ring(int32_t n, double theta, double phi) {
  if (!(theta >= 0.0 && theta <= kPi)) return -1;      // also rejects NaN
  if (!(phi - phi == 0.0)) return -1;                   // rejects NaN and +-inf
  return pix_of_z(n, cos_0pi(theta), phi);
}

// Ring pixel of (z, phi); -1 for non-finite input or z outside [-1, 1].
__device__ __forceinline__ int32_t zphi2pix_ring(int32_t n, double z, double phi) {
  if (!(z >= -1.0 && z <= 1.0)) return -1;
  if (!(phi - phi == 0.0)) return -1;
  return pix_of_z(n, z, phi);
}

// ---------------------------------------------------------------------------
// Boresight-quaternion pointing: a sample's attitude is q_b[i] (x) q_k
// (Hamilton product of (w, x, y, z) quaternions), its line of sight
// d = R(q) z_hat and its polarisation direction e = R(q) x_hat.
// ---------------------------------------------------------------------------
struct Quat {
  double w, x, y, z;
};

__device__ __forceinline__ Quat load_quat(const double *q, int64_t idx) {
  const double2 *p = reinterpret_cast<const double2 *>(q + 4 * idx);   // 16-byte aligned
  const double2 a = p[0], b = p[1];
  return {a.x, a.y, b.x, b.y};
}

__device__ __forceinline__ Quat qmul(const Quat &a, const Quat &b) {
#pragma clang fp contract(off)
  return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
          a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
          a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}

// What the pointing needs of an attitude: z = d_z clipped to [-1, 1] (NaN
// kept), phi = atan2(d_y, d_x), and the polarisation direction's components
// towards local west and local north scaled by sin(theta):
//   west  = -e . e_phi   * sin(theta) = d_y e_x - d_x e_y,
//   north = -e . e_theta * sin(theta) = e_z        (e is orthogonal to d),
// so that psi = atan2(west, north).
struct QuatDir {
  double z, phi, west, north;
};

__device__ __forceinline__ QuatDir quat_dir(const Quat &q) {
#pragma clang fp contract(off)
  const double dx = 2.0 * (q.x * q.z + q.w * q.y);
  const double dy = 2.0 * (q.y * q.z - q.w * q.x);
  const double dz = 1.0 - 2.0 * (q.x * q.x + q.y * q.y);
  const double ex = 1.0 - 2.0 * (q.y * q.y + q.z * q.z);
  const double ey = 2.0 * (q.x * q.y + q.w * q.z);
  const double ez = 2.0 * (q.x * q.z - q.w * q.y);
  QuatDir g;
  g.z = dz < -1.0 ? -1.0 : (dz > 1.0 ? 1.0 : dz);
  g.phi = atan2(dy, dx);
  g.west = dy * ex - dx * ey;
  g.north = ez;
  return g;
}

// HWP angle alpha_i = 2 pi ((num * i) mod den) / den + phase0, from integers.
__device__ __forceinline__ double hwp_alpha(int64_t i, int64_t num_mod, int64_t den,
                                            double phase0) {
#pragma clang fp contract(off)
  const int64_t m = (num_mod * (i % den)) % den;
  const double frac = (double)m / (double)den;
  return (2.0 * kPi) * frac + phase0;
}

// Merged polarisation angle times two: 2 (psi + dpsi_k + 2 alpha_i), FP64.
template <typename T>
__device__ __forceinline__ double two_psi_eff(const PtArgs<T> &a, int64_t k, int64_t i,
                                              double psi) {
#pragma clang fp contract(off)
  double pe = psi;
  if (a.dpsi) pe = pe + a.dpsi[k];
  if (a.hwp) pe = pe + 2.0 * hwp_alpha(i, a.hwp_num_mod, a.hwp_den, a.hwp_phase0);
  return 2.0 * pe;
}

// Polariser weights cos / sin of an angle given in FP64.  The FP64 variant
// evaluates them in FP64 (the library's sincos).  The FP32 variant reduces
// the angle in FP64 to r = ang - k pi/2 with k = rint(ang 2/pi), |r| <= pi/4
// (the FP64 error of k pi/2 is ~k 1e-16, far below an FP32 ulp for the
// angles of the method: |ang| < ~100), rounds r to FP32 and evaluates the
// Taylor series of sin r to r^9 / 9! and of cos r to r^10 / 10! by Horner's
// rule (truncation below 3e-9 on |r| <= pi/4), then places the quadrant:
//   k mod 4 = 0: ( cos r,  sin r)    1: (-sin r,  cos r)
//             2: (-cos r, -sin r)    3: ( sin r, -cos r).
__device__ __forceinline__ void weights(double ang, double &c, double &s) {
  sincos(ang, &s, &c);
}
__device__ __forceinline__ void weights(double ang, float &c, float &s) {
  constexpr double kHalfPi = 0.5 * kPi;
  constexpr double kTwoOverPi = 2.0 / kPi;
  const double k = rint(ang * kTwoOverPi);
  const float r = (float)fma(-k, kHalfPi, ang);
  const float r2 = r * r;
  float ps = fmaf(r2, 1.0f / 362880.0f, -1.0f / 5040.0f);
  ps = fmaf(r2, ps, 1.0f / 120.0f);
  ps = fmaf(r2, ps, -1.0f / 6.0f);
  const float sr = fmaf(r * r2, ps, r);
  float pc = fmaf(r2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
  pc = fmaf(r2, pc, -1.0f / 720.0f);
  pc = fmaf(r2, pc, 1.0f / 24.0f);
  pc = fmaf(r2, pc, -0.5f);
  const float cr = fmaf(r2, pc, 1.0f);
  const int q = (int)k;
  const bool swap = (q & 1) != 0;
  const float c0 = swap ? sr : cr, s0 = swap ? cr : sr;
  c = ((q + 1) & 2) ? -c0 : c0;
  s = (q & 2) ? -s0 : s0;
}

// cos / sin of 2 (psi + beta) where psi = atan2(west, north): cos 2 psi and
// sin 2 psi follow from (west, north) algebraically in FP64, and the turn by
// 2 beta (detector angle offset plus twice the HWP angle) is applied with the
// precision's weights() of that angle.  psi = 0 where west = north = 0.
__device__ __forceinline__ void quat_c2s2(const QuatDir &g, double &c2, double &s2) {
#pragma clang fp contract(off)
  const double ww = g.west * g.west, nn = g.north * g.north, r2 = ww + nn;
  c2 = 1.0;
  s2 = 0.0;
  if (r2 > 0.0) {
    // 1 / r2 from the hardware reciprocal and two Newton steps (within an
    // ulp or two; the correctly rounded quotient is not needed here)
    double inv = __builtin_amdgcn_rcp(r2);
    inv = fma(inv, fma(-r2, inv, 1.0), inv);
    inv = fma(inv, fma(-r2, inv, 1.0), inv);
    c2 = (nn - ww) * inv;
    s2 = (2.0 * (g.west * g.north)) * inv;
  }
}

// (c, s) = (c2, s2) turned by the angle whose cosine / sine are (cb, sb).
template <typename T>
__device__ __forceinline__ void turn_weights(double c2, double s2, T cb, T sb, T &c, T &s) {
#pragma clang fp contract(off)
  const T ct = (T)c2, st = (T)s2;
  c = ct * cb - st * sb;
  s = st * cb + ct * sb;
}

template <typename T>
__device__ __forceinline__ void quat_weights(const QuatDir &g, bool has_beta, double beta, T &c,
                                             T &s) {
  double c2, s2;
  quat_c2s2(g, c2, s2);
  if (!has_beta) {
    c = (T)c2;
    s = (T)s2;
    return;
  }
  T cb, sb;
  weights(2.0 * beta, cb, sb);
  turn_weights(c2, s2, cb, sb, c, s);
}

// Geometry of one sample: pixel (or -1) and polariser weights.
template <typename T>
struct Geom {
  int32_t pix;
  T c, s;
};

template <typename T>
__device__ __forceinline__ Geom<T> sample_geom(const PtArgs<T> &a, int64_t k, int64_t i) {
  Geom<T> g;
  if (a.qb) {
#pragma clang fp contract(off)
    const QuatDir d = quat_dir(qmul(load_quat(a.qb, i), load_quat(a.qd, k)));
    g.pix = zphi2pix_ring(a.nside, d.z, d.phi);
    double beta = a.dpsi ? a.dpsi[k] : 0.0;
    if (a.hwp) beta = beta + 2.0 * hwp_alpha(i, a.hwp_num_mod, a.hwp_den, a.hwp_phase0);
    quat_weights(d, a.dpsi || a.hwp, beta, g.c, g.s);
  } else {
    const int64_t off = k * a.n_samp + i;
    g.pix = ang2pix_ring(a.nside, (double)a.theta[off], (double)a.phi[off]);
    weights(two_psi_eff(a, k, i, (double)a.psi[off]), g.c, g.s);
  }
  if (g.pix >= 0 && a.valid && !a.valid[g.pix]) g.pix = -1;
  return g;
}

template <typename T>
__device__ __forceinline__ T gain_of(const PtArgs<T> &a, int64_t k) {
  return a.gain ? (T)a.gain[k] : (T)1;
}

// Streams read or written once per sample (pointing planes, TOD, label
// planes) go through the non-temporal path, so they do not evict the map
// lines that the gathers of neighbouring samples reuse from L1 and L2.
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_stream(T *p, T v) { __builtin_nontemporal_store(v, p); }

// ---------------------------------------------------------------------------
// Launch helpers.
// ---------------------------------------------------------------------------
// Per-sample kernels: one workgroup covers kChunk consecutive samples of one
// detector (kBlock threads x kItems samples, strided so loads coalesce).
constexpr int kBlock = 256;
constexpr int kItems = 4;
constexpr int64_t kChunk = (int64_t)kBlock * kItems;

__host__ __device__ inline int64_t chunks_per_det(int64_t n_samp) { return (n_samp + kChunk - 1) / kChunk; }

// ---------------------------------------------------------------------------
// Host-side validation and conversion of the public structs.
// ---------------------------------------------------------------------------
furax_status check_pointing(const furax_pointing *P);
furax_status check_noise(const furax_noise *N, int64_t n_det, int64_t n_samp, int32_t dt);
int64_t npix_of(int64_t nside);

template <typename T>
PtArgs<T> pt_args(const furax_pointing *P, const uint8_t *valid) {
  PtArgs<T> a;
  a.theta = static_cast<const T *>(P->theta);
  a.phi = static_cast<const T *>(P->phi);
  a.psi = static_cast<const T *>(P->psi);
  a.gain = P->gain;
  a.dpsi = P->dpsi;
  a.n_det = P->n_det;
  a.n_samp = P->n_samp;
  a.nside = (int32_t)P->nside;
  a.hwp = P->hwp;
  a.hwp_den = P->hwp ? P->hwp_den : 1;
  a.hwp_num_mod = P->hwp ? (P->hwp_num % a.hwp_den) : 0;
  a.hwp_phase0 = P->hwp ? P->hwp_phase0 : 0.0;
  a.valid = valid;
  a.qb = P->bore_quat;
  a.qd = P->det_quat;
  a.det_perm = nullptr;
  return a;
}

// Device scratch that a call allocates stream-ordered and frees on exit.
struct DevBuf {
  void *ptr = nullptr;
  hipStream_t stream = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() {
    if (ptr) (void)hipFreeAsync(ptr, stream);
  }
  furax_status alloc(size_t bytes, hipStream_t s);
};

// Addressing of a Stokes map: element (c, pix) lives at base[c * cs + pix * ps].
// Planar [3][npix] maps (the public layout) have cs = npix, ps = 1; the
// solver's internal vectors are interleaved [npix][4] (cs = 1, ps = 4) so that
// the three Stokes values of a pixel share one cache line.
struct MapLayout {
  int64_t cs;
  int32_t ps;
};
inline MapLayout planar_layout(int64_t npix) { return {npix, 1}; }
constexpr MapLayout kInterleaved = {1, 4};

// Sample tiles: a workgroup owns `dets` detectors x `ts` consecutive samples
// (ts a power of two), so that the waves of one CU sweep the same patch of
// sky at the same time and share its map cache lines.
constexpr int kMaxTileDets = 256;   // detectors per tile (LDS tables are sized by it)
struct Tiling {
  int32_t dets, log2ts;
  int64_t n_tb, n_dg;    // time blocks per detector, detector groups
  __host__ __device__ int64_t blocks() const { return n_tb * n_dg; }
};
Tiling make_tiling(int64_t n_det, int64_t n_samp, int32_t nside, int64_t target_samples,
                   int32_t min_log2ts);

// Kernel-launch wrappers implemented in the individual translation units.
//
// tod = P map.  With pix_out (a [n_det][n_samp] int32 plane) the ring pixel
// of every sample, -1 when flagged, is written as well.  With local_out (an
// interleaved map whose 4th lane holds each pixel's nested index as integer
// bits) the sample's offset inside its superpixel, nested & (P - 1), is
// written instead (0xffff when flagged).
template <typename T>
furax_status launch_pointing_apply(const PtArgs<T> &a, const void *map, bool map_f64,
                                   MapLayout ml, T *tod, hipStream_t s,
                                   int32_t *pix_out = nullptr, uint16_t *local_out = nullptr,
                                   int32_t local_mask = 0);
// q(c, pix) += sum over samples of v (1, cos, sin) with
//   v = g_k w_k tod[k,i]               when tod != null (w_det may be null: w = 1), or
//   v = g_k w_k g_k (P p)[k,i]          when tod == null (fused diagonal normal operator;
//                                        p read from pmap with layout pl).
// With pix_in (tod != null), the pixels are read from that plane (written by
// launch_pointing_apply over the same pointing) instead of being recomputed.
// Accumulation is privatised per tile in an LDS hash table of FP64 sums and
// flushed with one FP64 global atomic per touched pixel and Stokes component.
template <typename T>
furax_status launch_scatter(const PtArgs<T> &a, const T *tod, const double *w_det,
                            const void *pmap, bool pmap_f64, MapLayout pl, double *q,
                            MapLayout ql, hipStream_t s, const int32_t *pix_in = nullptr);
// ---------------------------------------------------------------------------
// Superpixel-major accumulation (superpix.hip).
// ---------------------------------------------------------------------------
constexpr int kSpPix = 1024;        // pixels per superpixel (32 x 32 nested block)
// Runs per accumulation workgroup (SpPlan::chunk_runs): 512 with angle
// pointing up to nside 512, where the smaller LDS run table lets three
// workgroups share a CU; 1024 otherwise -- with quaternion pointing the kernel
// is register-bound, and at finer nside runs are shorter, so that smaller
// chunks would hold too few samples to repay their set-up.
constexpr int kChunkRunsSmall = 512;
constexpr int kChunkRunsMax = 1024;
constexpr int64_t kMaxRun = 1024;   // longest run of consecutive samples
constexpr int kChunksPerGroup = 4;  // chunks one P^T workgroup takes in turn

struct SpChunk {
  int64_t r0;   // first run (index into the sorted run list)
  int32_t nr;   // number of runs
  int32_t sp;   // superpixel
  int32_t w;    // samples in the chunk (sum of its run lengths)
  int32_t s0;   // the chunk's first sample in the run-sorted sample order
};

// Everything the superpixel accumulation needs, built once per pointing.
struct SpPlan {
  int32_t nside = 0, log2P = 0, n_values = 0;
  int32_t chunk_runs = kChunkRunsMax;   // runs per chunk: kChunkRunsSmall or kChunkRunsMax
  int64_t npix = 0, n_sp = 0, n_runs = 0, n_chunks = 0, n_groups = 0;
  int32_t *n2r = nullptr, *r2n = nullptr;   // nested -> ring, ring -> nested [npix]
  uint64_t *runs = nullptr;                 // offset << 24 | chunk-local prefix of lengths
  SpChunk *chunks = nullptr;                // [n_chunks], ordered by superpixel
  // a group is up to kChunksPerGroup consecutive chunks of one superpixel,
  // accumulated by one workgroup into one partial: [n_groups + 1] first chunks
  int32_t *groups = nullptr;
  int32_t *sp_group = nullptr;              // [n_sp + 1]: first group of each superpixel
  double *partial = nullptr;                // [n_groups][n_values][P]
  // every scheduled sample in run-sorted order (chunk by chunk, run by run):
  // its pixel's offset inside the superpixel and, with angle pointing, its
  // angle psi (a reordered copy of the input plane), so that P^T reads both
  // contiguously instead of in run-sized pieces of the time-ordered planes
  int64_t n_sorted = 0;
  uint16_t *lab = nullptr;                  // [n_sorted]
  void *psi = nullptr;                      // [n_sorted] of the pointing dtype, or null
  // detectors ordered by the nested index of their first sample's pixel (a
  // Z-order walk over the sky), for the sample tiles of P
  int32_t *det_perm = nullptr;              // [n_det]
  void release(hipStream_t s);
};

// The superpixel path needs a power-of-two nside (the nested scheme) and
// fewer than 2^31 samples (one 32-bit selection / sort).
bool sp_supported(int64_t nside, int64_t S);
furax_status sp_nest_tables(SpPlan &sp, int64_t nside, hipStream_t s);
template <typename T>
furax_status sp_nest_plane(const SpPlan &sp, const PtArgs<T> &a, int32_t *plane, hipStream_t s);
template <typename T>
furax_status sp_build_runs(SpPlan &sp, const PtArgs<T> &a, const int32_t *nest_plane,
                           int32_t n_values, hipStream_t s);
// q = P^T (w tod) in ring order (every pixel written); the per-sample pixel
// offsets (and psi) come from the plan's run-sorted copies.
template <typename T>
furax_status sp_transpose(const SpPlan &sp, const PtArgs<T> &a, const T *tod,
                          const double *w_det, double *q, MapLayout ql, hipStream_t s);
template <typename T>
furax_status sp_bj_build(const SpPlan &sp, const PtArgs<T> &a, const double *w_det, double *M6,
                         int32_t *hits, hipStream_t s);

template <typename T>
furax_status launch_noise(const furax_noise *N, const T *in, T *out, void *work,
                          size_t work_bytes, hipStream_t s);
template <typename T>
size_t noise_workspace_bytes(const furax_noise *N);
// out = F_T in and / or the segments' template amplitudes; Lg: the Cholesky
// factor of full-length segments' Gram matrix (noise_prepare's workspace for a
// "deproj" model), or null to accumulate every segment's own.
template <typename T>
furax_status launch_deproject(const furax_noise *N, const T *in, T *out, double *amp,
                              hipStream_t s, const double *Lg = nullptr);
// Kernel spectrum of a band model (noise_workspace_bytes<T> bytes at spec),
// then the weight (or, for a covariance, N itself) applied to [n_det][n_samp].
template <typename T>
furax_status noise_prepare(const furax_noise *N, void *spec, hipStream_t s);
template <typename T>
furax_status noise_run(const furax_noise *N, const T *in, T *out, const void *spec,
                       hipStream_t s);
// Gap-fill CG work carried by the overlap-save kernel for 32768-sample FP64
// blocks (noise_run_gap): the new direction p = r / c0_k + beta_k p_prev is
// formed as each block loads its input -- the transform's input -- and
// written to p_next on the block's valid outputs, and each block adds its
// share of p . (mask N p) after its output.  Per-detector scalars are read
// with a stride (in doubles) from the solver's per-detector records.
struct GapFuse {
  const double *r;        // [n_det][n]: residual, 0 on missing samples
  double *p_next;         // [n_det][n]
  const uint8_t *gaps;    // [n_det][n]: 1 on missing samples
  const double *inv_c0;   // inv_c0[k * stride]
  const double *beta;     // beta[k * stride]
  int64_t stride;
  double *partial;        // [n_det][blocks]: p . (mask N p) per block
};
// Blocks per detector of the fused path for covariance C, or 0 when C takes
// another overlap-save kernel (then the solver runs its separate passes).
int64_t noise_gap_blocks(const furax_noise *C);
// q = N p_next with p_next formed from p_prev (see GapFuse).
furax_status noise_run_gap(const furax_noise *C, const double *p_prev, double *q,
                           const void *spec, const GapFuse &g, hipStream_t s);

template <typename T>
furax_status gap_fill_impl(const furax_noise *C, const uint8_t *gaps, const T *d, const T *nr,
                           T *out, const furax_gapfill_opts *opt, furax_gapfill_info *info,
                           hipStream_t s);

furax_status zero_async(void *ptr, size_t bytes, hipStream_t s);

}  // namespace fx
