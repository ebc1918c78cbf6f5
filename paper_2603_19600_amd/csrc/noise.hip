// Inverse-noise weighting N^-1, block-diagonal over detectors.
//
//  * diagonal (HomothetyOperator / DiagonalOperator of Table 2): z = w_k y;
//  * symmetric band-Toeplitz (SymmetricBandToeplitzOperator, Table 2, applied
//    by the overlap-save method named in the paragraph after the table):
//        z[i] = sum_{|tau| <= b-1, 0 <= i+tau < n} t[|tau|] y[i+tau].
//
// Overlap-save on gfx950: one workgroup owns one block of L = 2M consecutive
// input samples of one detector (zero outside the detector's stream) and
// produces the V = L - 2(b-1) outputs whose stencil lies inside the block.
// The real block is packed as M complex values (even samples -> real part,
// odd -> imaginary), transformed by a Stockham radix-4 FFT of length M held in
// LDS (128 KB for M = 16384 FP32 or M = 8192 FP64), split into the length-L
// real spectrum, multiplied by the kernel's spectrum -- which is real because
// the kernel is symmetric -- re-packed and transformed back.  The split,
// multiply and re-pack are one pass over (k, M-k) pairs.
#include <map>
#include <mutex>
#include <utility>

#include "common.h"

namespace fx {

template <typename T>
struct C2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ C2<T> cmulc(C2<T> a, C2<T> b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return {a.x * s, a.y * s}; }

// ---------------------------------------------------------------------------
// Stockham autosort FFT of length M = 2^m in LDS, radix 16 in registers.
//
// Each pass loads every butterfly's R inputs (stride M/R) into registers,
// synchronises, multiplies by the twiddles W_M^(r k M/(R Ns)), performs the
// R-point DFT in registers and writes the R outputs at stride Ns, so one LDS
// buffer suffices.  M = 16^a * f with f in {1, 2, 4, 8}: a radix-16 passes
// then one or two radix-4 / radix-2 passes (16384 = 16^3 * 4 takes 4 passes
// instead of 7 radix-4 ones).  The LDS index is padded by one element every
// 16 (pad16) so that the stride-16 accesses of the first pass do not pile onto
// a few banks.  tw[j] = exp(-2 pi i j / L), L = 2M, so W_M^x = tw[2x].  INV
// selects the (unnormalised) inverse transform.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int pad16(int e) { return e + (e >> 4); }

template <typename T, bool INV>
__device__ __forceinline__ void dft4(C2<T> &a0, C2<T> &a1, C2<T> &a2, C2<T> &a3) {
  const C2<T> t0 = cadd(a0, a2), t1 = csub(a0, a2);
  const C2<T> t2 = cadd(a1, a3), t3 = csub(a1, a3);
  const C2<T> it3 = {-t3.y, t3.x};   // i t3
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = INV ? cadd(t1, it3) : csub(t1, it3);
  a3 = INV ? csub(t1, it3) : cadd(t1, it3);
}

template <typename T, bool INV>
__device__ __forceinline__ C2<T> rot16(C2<T> a, int j) {
  // a * W16^j (conjugated for the inverse), j in {1, 2, 3, 4, 6, 9}
  constexpr T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
  constexpr T h = (T)0.70710678118654752440;
  const T sg = INV ? (T)1 : (T)-1;   // sign of the imaginary part of W16
  C2<T> w;
  switch (j) {
    case 1: w = {c1, sg * s1}; break;
    case 2: w = {h, sg * h}; break;
    case 3: w = {s1, sg * c1}; break;
    case 4: return INV ? C2<T>{-a.y, a.x} : C2<T>{a.y, -a.x};
    case 6: w = {-h, sg * h}; break;
    default: w = {-c1, -sg * s1}; break;   // j = 9
  }
  return cmul(a, w);
}

// In-place 16-point DFT: on return v[4 k1 + k2] holds X[k1 + 4 k2].
template <typename T, bool INV>
__device__ __forceinline__ void dft16(C2<T> (&v)[16]) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<T, INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  v[4 + 1] = rot16<T, INV>(v[4 + 1], 1);
  v[4 + 2] = rot16<T, INV>(v[4 + 2], 2);
  v[4 + 3] = rot16<T, INV>(v[4 + 3], 3);
  v[8 + 1] = rot16<T, INV>(v[8 + 1], 2);
  v[8 + 2] = rot16<T, INV>(v[8 + 2], 4);
  v[8 + 3] = rot16<T, INV>(v[8 + 3], 6);
  v[12 + 1] = rot16<T, INV>(v[12 + 1], 3);
  v[12 + 2] = rot16<T, INV>(v[12 + 2], 6);
  v[12 + 3] = rot16<T, INV>(v[12 + 3], 9);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<T, INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
}

template <typename T, bool INV>
__device__ __forceinline__ C2<T> twiddle(C2<T> a, C2<T> w) {
  return INV ? cmulc(a, w) : cmul(a, w);
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations,
// not for its global loads, so loads issued before it (the next block's input)
// stay in flight across the FFT passes.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Passes of the length-M FFT: radix 16 while it divides, then 4 and/or 2.
// Pass p has radix R(p) and span Ns(p) = product of the earlier radices.
template <int M>
struct FftPlan {
  static constexpr int n16 = __builtin_ctz(M) / 4;
  static constexpr int rem = M >> (4 * n16);
  static constexpr int npass = n16 + (rem == 8 ? 2 : (rem > 1 ? 1 : 0));
  static constexpr int R(int p) { return p < n16 ? 16 : (rem == 8 ? (p == n16 ? 4 : 2) : rem); }
  static constexpr int Ns(int p) {
    int n = 1;
    for (int i = 0; i < p; ++i) n *= R(i);
    return n;
  }
  // Twiddle stage t < npass - 1 serves pass t + 1 (pass 0 needs none): its
  // butterfly k (k < Ns) multiplies by powers of w1(k) = exp(-2 pi i k step / L),
  // step = L / (R Ns).  The last stage serves the real-spectrum split, where
  // w1(k) = exp(-2 pi i k / L) for k <= M.
  static constexpr int nstage = npass;
  static constexpr int K(int t) { return t < npass - 1 ? Ns(t + 1) : M + 1; }
  static constexpr int step(int t) { return t < npass - 1 ? 2 * M / (R(t + 1) * Ns(t + 1)) : 1; }
  static constexpr int nlo(int t) { return K(t) < 128 ? K(t) : 128; }
  static constexpr int nhi(int t) { return (K(t) + 127) / 128; }
  static constexpr int off(int t) {
    int o = 0;
    for (int i = 0; i < t; ++i) o += nlo(i) + nhi(i);
    return o;
  }
  static constexpr int total = off(nstage);
};

// w1(k) of one twiddle stage from two small FP64 LDS tables, lo[k mod 128]
// (step k) and hi[k / 128] (step 128 k): consecutive lanes read consecutive
// lo entries, so the lookups do not pile onto a few LDS banks.
struct TwStage {
  const C2<double> *lo, *hi;
  __device__ __forceinline__ C2<double> operator()(int k) const {
    return cmul(hi[k >> 7], lo[k & 127]);
  }
};

template <typename T>
__device__ __forceinline__ C2<T> narrow(C2<double> a) { return {(T)a.x, (T)a.y}; }

template <typename T, int M, int NT, int R, bool INV>
__device__ __forceinline__ void stockham_pass(C2<T> *s, const TwStage &tw, int Ns) {
  constexpr int NB = M / R;
  constexpr int PER = (NB + NT - 1) / NT;
  const int tid = threadIdx.x;
  C2<T> v[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = tid + q * NT;
    if (j < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = s[pad16(j + r * NB)];
    }
  }
  lds_barrier();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = tid + q * NT;
    if (j >= NB) continue;
    const int k = j & (Ns - 1);
    if (Ns > 1) {
      // powers of w1 = exp(-2 pi i k / (R Ns)), squared in FP64
      const C2<double> W1 = tw(k);
      if constexpr (R == 16) {
        const C2<double> W2 = cmul(W1, W1), W4 = cmul(W2, W2), W8 = cmul(W4, W4);
        const C2<T> w1 = narrow<T>(W1), w2 = narrow<T>(W2), w4 = narrow<T>(W4),
                    w8 = narrow<T>(W8);
        const C2<T> w3 = cmul(w1, w2), w5 = cmul(w1, w4), w6 = cmul(w2, w4), w7 = cmul(w3, w4);
        const C2<T> w[16] = {w1, w1, w2, w3, w4, w5, w6, w7, w8, cmul(w1, w8), cmul(w2, w8),
                             cmul(w3, w8), cmul(w4, w8), cmul(w5, w8), cmul(w6, w8), cmul(w7, w8)};
#pragma unroll
        for (int r = 1; r < 16; ++r) v[q][r] = twiddle<T, INV>(v[q][r], w[r]);
      } else if constexpr (R == 4) {
        const C2<double> W2 = cmul(W1, W1), W3 = cmul(W1, W2);
        v[q][1] = twiddle<T, INV>(v[q][1], narrow<T>(W1));
        v[q][2] = twiddle<T, INV>(v[q][2], narrow<T>(W2));
        v[q][3] = twiddle<T, INV>(v[q][3], narrow<T>(W3));
      } else {
        v[q][1] = twiddle<T, INV>(v[q][1], narrow<T>(W1));
      }
    }
    const int d = (j - k) * R + k;
    if constexpr (R == 16) {
      dft16<T, INV>(v[q]);
#pragma unroll
      for (int r = 0; r < 16; ++r) s[pad16(d + r * Ns)] = v[q][4 * (r & 3) + (r >> 2)];
    } else if constexpr (R == 4) {
      dft4<T, INV>(v[q][0], v[q][1], v[q][2], v[q][3]);
#pragma unroll
      for (int r = 0; r < 4; ++r) s[pad16(d + r * Ns)] = v[q][r];
    } else {
      s[pad16(d)] = cadd(v[q][0], v[q][1]);
      s[pad16(d + Ns)] = csub(v[q][0], v[q][1]);
    }
  }
  lds_barrier();
}

template <int M>
__device__ __forceinline__ TwStage stage_of(const C2<double> *tab, int t) {
  using Pl = FftPlan<M>;
  const int o = Pl::off(t);
  return {tab + o, tab + o + Pl::nlo(t)};
}

template <typename T, int M, int NT, bool INV>
__device__ __forceinline__ void fft_lds(C2<T> *s, const C2<double> *tab) {
  using Pl = FftPlan<M>;
  int Ns = 1;
#pragma unroll
  for (int p = 0; p < Pl::n16; ++p) {
    stockham_pass<T, M, NT, 16, INV>(s, stage_of<M>(tab, p > 0 ? p - 1 : 0), Ns);
    Ns *= 16;
  }
  constexpr int q = Pl::n16;   // index of the first non-radix-16 pass
  if constexpr (Pl::rem == 8) {
    stockham_pass<T, M, NT, 4, INV>(s, stage_of<M>(tab, q - 1), Ns);
    stockham_pass<T, M, NT, 2, INV>(s, stage_of<M>(tab, q), Ns * 4);
  } else if constexpr (Pl::rem == 4) {
    stockham_pass<T, M, NT, 4, INV>(s, stage_of<M>(tab, q - 1), Ns);
  } else if constexpr (Pl::rem == 2) {
    stockham_pass<T, M, NT, 2, INV>(s, stage_of<M>(tab, q - 1), Ns);
  }
}


// Block index -> task (detector-major, block-minor) with consecutive blocks
// of one detector kept on the same XCD (workgroups are dealt round-robin over
// the 8 XCDs), so the halo a block shares with its neighbours is read through
// the same L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  const int64_t per = nblocks / 8;
  if (per == 0 || bid >= per * 8) return bid;
  return (bid % 8) * per + bid / 8;
}

// A workgroup transforms a contiguous range of (detector, block) tasks, one
// per workgroup unless PREFETCH: then a persistent workgroup walks a range of
// consecutive blocks and loads the next task's input into registers while the
// current one is transformed (it costs VGPRs the transform also needs, so it
// is kept as an option).
template <typename T, int M, int NT, bool PREFETCH>
__global__ void __launch_bounds__(NT) k_overlap_save(const T *__restrict__ in, T *__restrict__ out,
                                                     int64_t n, int32_t b, int64_t nblk,
                                                     int64_t ntask, const T *__restrict__ spec,
                                                     int64_t spec_stride,
                                                     const C2<double> *__restrict__ tw) {
  __shared__ C2<T> s[M + M / 16];
  constexpr int L = 2 * M;
  using Pl = FftPlan<M>;
  __shared__ C2<double> tab[Pl::total];
  const int V = L - 2 * (b - 1);
  const int tid = threadIdx.x;
  // twiddle stage tables from the FP64 table tw[j] = exp(-2 pi i j / L)
#pragma unroll
  for (int t = 0; t < Pl::nstage; ++t) {
    const int o = Pl::off(t), nl = Pl::nlo(t), st = Pl::step(t);
    for (int i = tid; i < nl; i += NT) tab[o + i] = tw[st * i];
    for (int i = tid; i < Pl::nhi(t); i += NT) tab[o + nl + i] = tw[st * 128 * i];
  }
  const TwStage W = stage_of<M>(tab, Pl::nstage - 1);   // the split's twiddles

  const int64_t t_beg = PREFETCH ? ntask * blockIdx.x / gridDim.x
                                 : xcd_remap(blockIdx.x, (int64_t)gridDim.x);
  const int64_t t_end = PREFETCH ? ntask * (blockIdx.x + 1) / gridDim.x : t_beg + 1;
  constexpr int PER = M / NT;
  static_assert(M % NT == 0, "whole complex values per thread");
  C2<T> buf[PER];
  // input of task t: L real samples from s0 = blk V - (b - 1), zero outside
  // the detector's stream, packed as M complex values (even -> re, odd -> im)
  auto fetch = [&](int64_t t) {
    const int64_t det = t / nblk, blk = t - det * nblk;
    const int64_t s0 = blk * V - (b - 1);
    const T *x = in + det * n;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int64_t g = s0 + 2 * (tid + q * NT);
      buf[q].x = (g >= 0 && g < n) ? x[g] : (T)0;
      buf[q].y = (g + 1 >= 0 && g + 1 < n) ? x[g + 1] : (T)0;
    }
  };
  if (t_beg < t_end) fetch(t_beg);
  for (int64_t t = t_beg; t < t_end; ++t) {
    lds_barrier();   // the previous task's outputs have been read out of LDS
#pragma unroll
    for (int q = 0; q < PER; ++q) s[pad16(tid + q * NT)] = buf[q];
    if (PREFETCH && t + 1 < t_end) fetch(t + 1);   // in flight during this task's transforms
    lds_barrier();
    fft_lds<T, M, NT, false>(s, tab);

    const int64_t det = t / nblk, blk = t - det * nblk;
    const T *H = spec + det * spec_stride;   // H[0..M], already divided by M
    for (int k = tid; k <= M / 2; k += NT) {
      const int k2 = (M - k) & (M - 1);
      const C2<T> z1 = s[pad16(k)], z2 = s[pad16(k2)];
      C2<T> r1, r2;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int kk = h ? k2 : k;
        const C2<T> za = h ? z2 : z1;
        const C2<T> zb = h ? z1 : z2;               // Z[M - kk]
        const C2<T> zc = {zb.x, -zb.y};             // conj(Z[M - kk])
        const C2<T> E = cscale(cadd(za, zc), (T)0.5);
        const C2<T> Dh = cscale(csub(za, zc), (T)0.5);
        const C2<T> O = {Dh.y, -Dh.x};              // (Z[k] - conj Z[M-k]) / (2i)
        const T Hk = H[kk], Hm = H[M - kk];
        const T hp = (Hk + Hm) * (T)0.5, hm = (Hk - Hm) * (T)0.5;
        const C2<T> Wk = narrow<T>(W(kk));          // exp(-2 pi i kk / L)
        const C2<T> A = cadd(cscale(E, hp), cscale(cmul(Wk, O), hm));
        const C2<T> B = cadd(cscale(cmulc(E, Wk), hm), cscale(O, hp));
        const C2<T> r = {A.x - B.y, A.y + B.x};     // A + i B
        if (h) r2 = r; else r1 = r;
      }
      s[pad16(k)] = r1;
      if (k2 != k) s[pad16(k2)] = r2;
    }
    lds_barrier();
    fft_lds<T, M, NT, true>(s, tab);

    const int64_t s0 = blk * V - (b - 1);
    T *z = out + det * n;
    const int lo = b - 1, hi = b - 1 + V;
    for (int m = tid; m < M; m += NT) {
      const int e = 2 * m;
      const C2<T> v = s[pad16(m)];
      if (e >= lo && e < hi && s0 + e < n) z[s0 + e] = v.x;
      if (e + 1 >= lo && e + 1 < hi && s0 + e + 1 < n) z[s0 + e + 1] = v.y;
    }
  }
}

// Spectrum of the symmetric circular kernel of length L = 2M, divided by M:
// H[k] = (t0 + 2 sum_{tau=1}^{b-1} t[tau] cos(2 pi k tau / L)) / M, k = 0..M.
// One wave per frequency k: the lanes split the lags, cos(2 pi k tau / L) is
// read from the FP64 table at the exact integer phase (k tau) mod L, and the
// lanes' partial sums are combined in a fixed order.
__global__ void __launch_bounds__(kBlock) k_spectrum(const double *__restrict__ lags, int32_t b,
                                                     int64_t lag_stride, int32_t M,
                                                     const C2<double> *__restrict__ tw64,
                                                     double *__restrict__ spec64,
                                                     float *__restrict__ spec32) {
  const int64_t kern = blockIdx.y;
  const int k = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k > M) return;
  const double *t = lags + kern * lag_stride;
  const int64_t Lmask = 2 * M - 1;
  double acc = 0.0;
  for (int tau = 1 + lane; tau < b; tau += 64) acc += t[tau] * tw64[((int64_t)k * tau) & Lmask].x;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) {
    const double h = (t[0] + 2.0 * acc) / (double)M;
    if (spec64) spec64[kern * (int64_t)(M + 1) + k] = h;
    if (spec32) spec32[kern * (int64_t)(M + 1) + k] = (float)h;
  }
}

// tw64[j] = exp(-2 pi i j / L) in FP64 (both precisions' FFTs read it).
__global__ void __launch_bounds__(kBlock) k_twiddles(int32_t L, C2<double> *tw64) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= L) return;
  double s, c;
  sincospi(2.0 * (double)j / (double)L, &s, &c);
  tw64[j] = {c, -s};
}

template <typename T, int M, int NT>
__global__ void __launch_bounds__(kBlock) k_diag(const T *__restrict__ in, T *__restrict__ out,
                                                 int64_t n_det, int64_t n,
                                                 const double *__restrict__ w) {
  const int64_t total = n_det * n;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += stride)
    out[i] = (T)w[i / n] * in[i];
}

// ---------------------------------------------------------------------------
// Per-device twiddle tables (content-independent; kept until
// furax_release_caches()).
// ---------------------------------------------------------------------------
struct TwTables {
  C2<double> *tw64 = nullptr;
};
static std::mutex g_tw_mu;
static std::map<std::pair<int, int>, TwTables> g_tw;   // (device, L) -> tables

static furax_status get_twiddles(int L, hipStream_t s, TwTables &out) {
  int dev = 0;
  FX_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_tw_mu);
  auto it = g_tw.find({dev, L});
  if (it != g_tw.end()) {
    out = it->second;
    return FURAX_OK;
  }
  TwTables t;
  if (hipMalloc(&t.tw64, sizeof(C2<double>) * L) != hipSuccess)
    return set_error(FURAX_ENOMEM, "twiddle table allocation failed");
  hipLaunchKernelGGL(k_twiddles, dim3((L + kBlock - 1) / kBlock), dim3(kBlock), 0, s, L, t.tw64);
  FX_HIP(hipGetLastError());
  g_tw[{dev, L}] = t;
  out = t;
  return FURAX_OK;
}

void release_twiddles() {
  std::lock_guard<std::mutex> lk(g_tw_mu);
  for (auto &kv : g_tw) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(kv.first.first);
    (void)hipDeviceSynchronize();
    (void)hipFree(kv.second.tw64);
    (void)hipSetDevice(cur);
  }
  g_tw.clear();
}

// FFT half-length M used for a band of b lags in precision T.
template <typename T>
int os_half_length(int64_t b) {
  const int64_t mmax = sizeof(T) == 4 ? 16384 : 8192;
  int64_t m = 512;
  while (m < 4 * (b - 1) && m < mmax) m *= 2;
  return (int)m;
}

template <typename T>
int64_t os_max_band() { return sizeof(T) == 4 ? 8192 : 4096; }
template int64_t os_max_band<float>();
template int64_t os_max_band<double>();

// Spectrum buffer size for a noise model in precision T.
template <typename T>
size_t noise_workspace_bytes(const furax_noise *N) {
  if (N->kind != 1) return 0;
  const int M = os_half_length<T>(N->bandwidth);
  const int64_t nk = N->toeplitz_stride ? N->n_det : 1;
  return (size_t)nk * (M + 1) * sizeof(T);
}
template size_t noise_workspace_bytes<float>(const furax_noise *);
template size_t noise_workspace_bytes<double>(const furax_noise *);

// Compute the kernel spectrum into `spec` (noise_workspace_bytes<T> bytes).
template <typename T>
furax_status noise_prepare(const furax_noise *N, void *spec, hipStream_t s) {
  if (N->kind != 1) return FURAX_OK;
  const int M = os_half_length<T>(N->bandwidth);
  TwTables tw;
  FX_TRY(get_twiddles(2 * M, s, tw));
  const int64_t nk = N->toeplitz_stride ? N->n_det : 1;
  constexpr int per_block = kBlock / 64;
  dim3 grid((M + 1 + per_block - 1) / per_block, (unsigned)nk);
  hipLaunchKernelGGL(k_spectrum, grid, dim3(kBlock), 0, s, N->toeplitz, (int32_t)N->bandwidth,
                     N->toeplitz_stride, M, tw.tw64,
                     sizeof(T) == 8 ? static_cast<double *>(spec) : nullptr,
                     sizeof(T) == 4 ? static_cast<float *>(spec) : nullptr);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status noise_prepare<float>(const furax_noise *, void *, hipStream_t);
template furax_status noise_prepare<double>(const furax_noise *, void *, hipStream_t);

template <typename T, int M, int NT>
static furax_status launch_os(const furax_noise *N, const T *in, T *out, const T *spec,
                              const C2<double> *tw, hipStream_t s) {
  const int b = (int)N->bandwidth;
  const int64_t V = 2 * M - 2 * (int64_t)(b - 1);
  const int64_t nblk = (N->n_samp + V - 1) / V;
  const int64_t ntask = N->n_det * nblk;
  const int64_t spec_stride = N->toeplitz_stride ? (M + 1) : 0;
  hipLaunchKernelGGL((k_overlap_save<T, M, NT, false>), dim3((unsigned)ntask), dim3(NT), 0, s, in,
                     out, N->n_samp, b, nblk, ntask, spec, spec_stride, tw);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}

// Apply N^-1 given a prepared spectrum (kind 1) or the diagonal weights (kind 0).
template <typename T>
furax_status noise_run(const furax_noise *N, const T *in, T *out, const void *spec,
                       hipStream_t s) {
  if (N->n_samp == 0) return FURAX_OK;
  if (N->kind == 0) {
    const int64_t total = N->n_det * N->n_samp;
    const int64_t blocks = std::min<int64_t>((total + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL((k_diag<T, 0, 0>), dim3((unsigned)blocks), dim3(kBlock), 0, s, in, out,
                       N->n_det, N->n_samp, N->inv_var);
    FX_HIP(hipGetLastError());
    return FURAX_OK;
  }
  const int M = os_half_length<T>(N->bandwidth);
  TwTables tw;
  FX_TRY(get_twiddles(2 * M, s, tw));
  const T *sp = static_cast<const T *>(spec);
  const C2<double> *t = tw.tw64;   // FP64 twiddles for both precisions
  switch (M) {
    case 512: return launch_os<T, 512, 64>(N, in, out, sp, t, s);
    case 1024: return launch_os<T, 1024, 64>(N, in, out, sp, t, s);
    case 2048: return launch_os<T, 2048, 128>(N, in, out, sp, t, s);
    case 4096: return launch_os<T, 4096, 256>(N, in, out, sp, t, s);
    case 8192: return launch_os<T, 8192, 512>(N, in, out, sp, t, s);
    case 16384:
      if constexpr (sizeof(T) == 4) return launch_os<T, 16384, 1024>(N, in, out, sp, t, s);
      break;
  }
  return set_error(FURAX_EUNSUPPORTED, "no overlap-save instance for this band");
}
template furax_status noise_run<float>(const furax_noise *, const float *, float *, const void *,
                                       hipStream_t);
template furax_status noise_run<double>(const furax_noise *, const double *, double *,
                                        const void *, hipStream_t);

template <typename T>
furax_status launch_noise(const furax_noise *N, const T *in, T *out, void *work,
                          size_t work_bytes, hipStream_t s) {
  if (N->kind == 1 && work_bytes < noise_workspace_bytes<T>(N))
    return set_error(FURAX_EINVAL, "noise workspace too small");
  FX_TRY(noise_prepare<T>(N, work, s));
  return noise_run<T>(N, in, out, work, s);
}
template furax_status launch_noise<float>(const furax_noise *, const float *, float *, void *,
                                          size_t, hipStream_t);
template furax_status launch_noise<double>(const furax_noise *, const double *, double *, void *,
                                           size_t, hipStream_t);

}  // namespace fx
