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
// odd -> imaginary), transformed by a Stockham FFT of length M, split into the
// length-L real spectrum, multiplied by the kernel's spectrum -- which is real
// because the kernel is symmetric -- re-packed and transformed back.  The
// split, multiply and re-pack are one 2x2 real mixing of each (k, M-k) pair.
// Three kernels: k_os_r32 (M = 8192, the block in registers, radices 32, 16,
// 16), k_os_r32x (M = 16384, the block in registers, radices 32, 32, 16) and
// k_overlap_save (M <= 4096, and streams too long for 32-bit offsets: the
// block in LDS).
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

// Output k of the real-spectrum split, kernel multiply and re-pack, from the
// packed forward transform Z (za = Z[k], zb = Z[M - k]).  With E and O the
// spectra of the even and odd samples, E = (Z[k] + conj Z[M-k]) / 2,
// O = (Z[k] - conj Z[M-k]) / 2i, the full spectrum is X[k] = E + W^k O and
// X[k + M] = E - W^k O (W = exp(-2 pi i / L)).  Multiplying by the real,
// symmetric kernel spectrum H and re-packing gives E' + i O' with
//   E' = hp E + hm W^k O,  O' = hm conj(W^k) E + hp O,
// hp = (H[k] + H[M-k]) / 2, hm = (H[k] - H[M-k]) / 2 (H already divided by
// M).  Substituting E and O, every term but two cancels:
//   Re out = alpha_k Re Z[k] + beta_k Im Z[M-k],
//   Im out = alpha_k Im Z[k] + beta_k Re Z[M-k],
// alpha_k = hp + Im(W^k) hm, beta_k = Re(W^k) hm, tabulated per k by
// k_spectrum (ab = (alpha_k, beta_k)).
template <typename T>
__device__ __forceinline__ C2<T> split_mul(C2<T> za, C2<T> zb, C2<T> ab) {
  return {ab.x * za.x + ab.y * zb.y, ab.x * za.y + ab.y * zb.x};
}

// Per-kernel layout of the spectrum workspace: H[0..M] (padded to M + 2
// entries) then the split coefficients (alpha_k, beta_k), k = 0..M-1.
__host__ __device__ constexpr int64_t spec_block(int M) { return 3 * (int64_t)M + 2; }
__host__ __device__ constexpr int64_t spec_coef_off(int M) { return (int64_t)M + 2; }

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

// Raw buffer over a row of n values (n sizeof(T) < 2^31 bytes, checked by the
// launcher): a load whose byte offset is at or past the end returns zero and
// a store there is dropped.  Offsets are unsigned and must not wrap: an access
// that belongs before the row's start takes kDropOffset instead.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_buffer(T *p, int64_t n) {
  // dword 3: 32-bit data format, no swizzle, untyped access
  return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)(n * (int64_t)sizeof(T)), 0x00020000);
}
constexpr uint32_t kDropOffset = 0x80000000u;   // past every row the launcher admits

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
}
// Two consecutive values of a row as one access (off: byte offset of the first).
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ C2<double> buf_load2(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
  return __builtin_bit_cast(C2<double>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ C2<float> buf_load2(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return __builtin_bit_cast(C2<float>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void buf_store2(__amdgpu_buffer_rsrc_t r, uint32_t off, C2<double> v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), r, off, 0, 0);
}
// FP32 pairs are stored non-temporally (cache policy nt): measured faster for
// the FP32 transforms, slower for FP64, whose pairs keep the default policy.
__device__ __forceinline__ void buf_store2(__amdgpu_buffer_rsrc_t r, uint32_t off, C2<float> v) {
  constexpr int kNonTemporal = 2;   // the nt bit of the cache-policy operand
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, off, 0, kNonTemporal);
}

// The thread index as a value the compiler cannot move across this point:
// LDS and store addresses derived from it are then computed where they are
// used instead of being hoisted to the kernel's start and held in registers
// for its whole length.
__device__ __forceinline__ int fresh_tid(int tid) {
  int t;
  asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"(tid));
  return t;
}
// Used by the FP32 register FFT, where the registers it frees raise the
// occupancy (four waves per SIMD); the FP64 kernel is held to two by its data
// and runs faster with the hoisted addresses.
template <typename T>
__device__ __forceinline__ int pinned_tid(int tid) {
  if constexpr (sizeof(T) == 4) return fresh_tid(tid);
  else return tid;
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
    const C2<T> *AB = reinterpret_cast<const C2<T> *>(spec + det * spec_stride + spec_coef_off(M));
    for (int k = tid; k <= M / 2; k += NT) {
      const int k2 = (M - k) & (M - 1);
      const C2<T> z1 = s[pad16(k)], z2 = s[pad16(k2)];
      const C2<T> r1 = split_mul<T>(z1, z2, AB[k]);
      const C2<T> r2 = split_mul<T>(z2, z1, AB[k2]);
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

// v[r] *= w1^r for r = 1..15, w1 = narrow(W1).  w2, w4, w8 are squared in
// FP64; the other powers are products in T (w3 = w1 w2, w5 = w1 w4, w6 = w2 w4,
// w7 = w3 w4, w(r+8) = w(r) w8), each applied as soon as it is formed so that
// only w1, w2, w4, w8 stay live.
template <typename T, bool INV>
__device__ __forceinline__ void twiddle16(C2<T> (&v)[16], C2<double> W1) {
  const C2<double> W2 = cmul(W1, W1), W4 = cmul(W2, W2), W8 = cmul(W4, W4);
  const C2<T> w1 = narrow<T>(W1), w2 = narrow<T>(W2), w4 = narrow<T>(W4), w8 = narrow<T>(W8);
  v[8] = twiddle<T, INV>(v[8], w8);
  C2<T> w3 = cmul(w1, w2);
#pragma unroll
  for (int r = 1; r < 8; ++r) {
    C2<T> w;
    switch (r) {
      case 1: w = w1; break;
      case 2: w = w2; break;
      case 3: w = w3; break;
      case 4: w = w4; break;
      case 5: w = cmul(w1, w4); break;
      case 6: w = cmul(w2, w4); break;
      default: w = cmul(w3, w4); break;
    }
    v[r] = twiddle<T, INV>(v[r], w);
    v[r + 8] = twiddle<T, INV>(v[r + 8], cmul(w, w8));
  }
}

// ---------------------------------------------------------------------------
// Register-resident overlap-save for the long blocks (M = 8192 and 16384).
//
// NT threads (256 for M = 8192, 512 for M = 16384) hold the whole packed
// block in registers (32 complex values each) and use LDS only to exchange
// data between passes, through a buffer of HALF the block (64 KB in FP64, 32
// or 64 KB in FP32), in two rounds: so two or more workgroups fit one CU and
// one's HBM traffic overlaps another's FFT.  The first forward pass reads its
// inputs from HBM and the last inverse pass writes its outputs there.  Every
// exchange is static in which half a value travels.  Twiddles come from the
// FP64 table tw[j] = exp(-2 pi i j / L) (L2-resident), one lookup per
// butterfly and pass.
// ---------------------------------------------------------------------------

// Radix-16 butterfly q (j = tid + q NT) of a pass of span Ns, on v[16 q ..]:
// twiddles for k = j mod Ns, then the 16-point DFT (result in dft16 order).
template <typename T, int M, bool INV>
__device__ __forceinline__ void reg_r16(C2<T> *v, int j, int Ns, const C2<double> *tw) {
  constexpr int L = 2 * M;
  const int k = j & (Ns - 1);
  if (Ns > 1) twiddle16<T, INV>(*reinterpret_cast<C2<T>(*)[16]>(v), tw[k * (L / (16 * Ns))]);
  dft16<T, INV>(*reinterpret_cast<C2<T>(*)[16]>(v));
}

// First valid output of a block for a band of b lags, rounded up to even.
__host__ __device__ __forceinline__ int os_pair_lo(int b) { return (b - 1) + ((b - 1) & 1); }

// ---------------------------------------------------------------------------
// Register-resident overlap-save with four exchanges, M = 8192.
//
// 256 threads; the transform takes radices 32, 16, 16 (spans 1, 32, 512)
// forward and 16, 16, 32 (spans 1, 16, 256) inverse: each thread's 32 values are one radix-32
// butterfly in the first forward and last inverse pass.  The last forward
// pass gives thread t the butterflies j and 512 - j (0 and 256 for t = 0),
// whose outputs Z[j + 512 r] and Z[512 - j + 512 (15 - r)] are the pairs
// (k, M - k) of the split, and the split's outputs are the inputs of those
// two butterflies in the first inverse pass: four exchanges per block
// instead of six.  Output r of a 32-point DFT sits at p32(r) (dft32), of a
// 16-point one at p16(r).
// ---------------------------------------------------------------------------
__device__ __forceinline__ constexpr int p16(int r) { return 4 * (r & 3) + (r >> 2); }
__device__ __forceinline__ constexpr int p32(int r) { return (r & 16) + p16(r & 15); }

// a * W32^k (conjugated for the inverse), k in [0, 16)
template <typename T, bool INV>
__device__ __forceinline__ C2<T> rot32(C2<T> a, int k) {
  // cos and sin of pi k / 16
  constexpr double c[16] = {1.0,
                            0.98078528040323044913, 0.92387953251128675613,
                            0.83146961230254523708, 0.70710678118654752440,
                            0.55557023301960222474, 0.38268343236508977173,
                            0.19509032201612826785, 0.0,
                            -0.19509032201612826785, -0.38268343236508977173,
                            -0.55557023301960222474, -0.70710678118654752440,
                            -0.83146961230254523708, -0.92387953251128675613,
                            -0.98078528040323044913};
  constexpr double sn[16] = {0.0,
                             0.19509032201612826785, 0.38268343236508977173,
                             0.55557023301960222474, 0.70710678118654752440,
                             0.83146961230254523708, 0.92387953251128675613,
                             0.98078528040323044913, 1.0,
                             0.98078528040323044913, 0.92387953251128675613,
                             0.83146961230254523708, 0.70710678118654752440,
                             0.55557023301960222474, 0.38268343236508977173,
                             0.19509032201612826785};
  if (k == 0) return a;
  if (k == 8) return INV ? C2<T>{-a.y, a.x} : C2<T>{a.y, -a.x};
  const T sg = INV ? (T)1 : (T)-1;
  return cmul(a, C2<T>{(T)c[k], sg * (T)sn[k]});
}

// In-place 32-point DFT of v[r] = input r: output r ends in v[p32(r)].
template <typename T, bool INV>
__device__ __forceinline__ void dft32(C2<T> (&v)[32]) {
  C2<T> e[16], o[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    e[m] = v[2 * m];
    o[m] = v[2 * m + 1];
  }
  dft16<T, INV>(e);
  dft16<T, INV>(o);
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int k = (p >> 2) + 4 * (p & 3);   // e[p], o[p] hold output k of the halves
    const C2<T> t = rot32<T, INV>(o[p], k);
    v[p] = cadd(e[p], t);
    v[16 + p] = csub(e[p], t);
  }
}

// v[r] *= w^r, r = 0..31 (w = W1, conjugated for the inverse).
template <typename T, bool INV>
__device__ __forceinline__ void twiddle32(C2<T> (&v)[32], C2<double> W1) {
  twiddle16<T, INV>(*reinterpret_cast<C2<T>(*)[16]>(v), W1);
  twiddle16<T, INV>(*reinterpret_cast<C2<T>(*)[16]>(v + 16), W1);
  const C2<double> W2 = cmul(W1, W1), W4 = cmul(W2, W2), W8 = cmul(W4, W4);
  const C2<T> w16 = narrow<T>(cmul(W8, W8));
#pragma unroll
  for (int r = 16; r < 32; ++r) v[r] = twiddle<T, INV>(v[r], w16);
}

// (FP32: registers for four waves per SIMD, LDS for four workgroups per CU;
// FP64: two of each)
template <typename T, bool PAIR>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 4 : 2)
k_os_r32(const T *__restrict__ in, T *__restrict__ out, int64_t n, int32_t b, int64_t nblk,
         const T *__restrict__ spec, int64_t spec_stride, const C2<double> *__restrict__ tw) {
  constexpr int M = 8192, L = 2 * M, HALF = M / 2, NT = 256;
  constexpr int HP = HALF + HALF / 16;   // padded half: pad16(e - HALF) = pad16(e) - HP
  // FP32 (VALU-bound) takes each exchange's LDS slots as one per-thread base
  // plus compile-time offsets; FP64 keeps the slots computed per element.
  constexpr bool kFold = sizeof(T) == 4;
  __shared__ C2<T> s[HP];
  const int tid0 = threadIdx.x;
  const int64_t det = (int64_t)blockIdx.x / nblk, blk = (int64_t)blockIdx.x - det * nblk;
  // valid outputs [lo, lo + V) of the block, lo even (os_pair_lo)
  const int lo = os_pair_lo(b), V = L - 2 * lo;
  const int32_t s0 = (int32_t)(blk * V) - lo;
  C2<T> v[32];

  // ---- forward pass 0 (radix 32, span 1): inputs z[t + 256 r] from HBM
  {
    const int tid = pinned_tid<T>(tid0);
    const __amdgpu_buffer_rsrc_t xr = row_buffer(const_cast<T *>(in) + det * n, n);
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      const int32_t g = s0 + 2 * (tid + NT * r);
      if constexpr (PAIR) {   // n even: a pair is wholly inside or outside the row
        v[r] = buf_load2(xr, g >= 0 ? (uint32_t)g * (uint32_t)sizeof(T) : kDropOffset, T());
      } else {
        v[r].x = buf_load<T>(xr, g >= 0 ? (uint32_t)g * (uint32_t)sizeof(T) : kDropOffset);
        v[r].y = buf_load<T>(xr, g + 1 >= 0 ? (uint32_t)(g + 1) * (uint32_t)sizeof(T) : kDropOffset);
      }
    }
    dft32<T, false>(v);
  }
  // ---- exchange: element 32 t + r (half t / 128, chosen per wave) -> v[16 q + r]
  // = element t + 256 q + 512 r (half r / 8)
  {
    const int tid = pinned_tid<T>(tid0);
    const int hw = __builtin_amdgcn_readfirstlane(tid >> 7);
    C2<T> nv[32];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (hw == h) {
#pragma unroll
        for (int r = 0; r < 32; ++r)
          s[kFold ? 34 * tid - h * HP + r + (r >> 4) : pad16(32 * tid + r - h * HALF)] = v[p32(r)];
      }
      lds_barrier();
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 8 * h; r < 8 * h + 8; ++r)
          nv[16 * q + r] = s[kFold ? pad16(tid) + 272 * q + 544 * (r - 8 * h)
                                   : pad16(tid + NT * q + 512 * r - h * HALF)];
      lds_barrier();
    }
#pragma unroll
    for (int e = 0; e < 32; ++e) v[e] = nv[e];
  }
  // ---- forward pass 1 (radix 16, span 32)
#pragma unroll
  for (int q = 0; q < 2; ++q) reg_r16<T, M, false>(v + 16 * q, pinned_tid<T>(tid0) + NT * q, 32, tw);
  // ---- exchange: butterfly j = t + 256 q writes (j - k) 16 + k + 32 r (k = j mod 32,
  // half q) -> paired layout v[16 e + r] = element j_e + 512 r (half r / 8)
  {
    const int tid = pinned_tid<T>(tid0);
    const int j1 = tid == 0 ? 256 : 512 - tid;
    C2<T> nv[32];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      {
        const int j = tid + NT * h, k = j & 31;
#pragma unroll
        for (int r = 0; r < 16; ++r)
          s[kFold ? 17 * (tid - (tid & 31)) + pad16(tid & 31) + 34 * r
                  : pad16((j - k) * 16 + k + 32 * r - h * HALF)] = v[16 * h + p16(r)];
      }
      lds_barrier();
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int r = 8 * h; r < 8 * h + 8; ++r)
          nv[16 * e + r] = s[kFold ? pad16(e ? j1 : tid) + 544 * (r - 8 * h)
                                   : pad16((e ? j1 : tid) + 512 * r - h * HALF)];
      lds_barrier();
    }
#pragma unroll
    for (int e = 0; e < 32; ++e) v[e] = nv[e];
  }
  // ---- forward pass 2 (radix 16, span 512) on butterflies j0 = t, j1; split and
  // kernel multiply; inverse pass 0 (radix 16, span 1) on the same butterflies
  const int tidp = pinned_tid<T>(tid0);
  const int jp[2] = {tidp, tidp == 0 ? 256 : 512 - tidp};
#pragma unroll
  for (int e = 0; e < 2; ++e) reg_r16<T, M, false>(v + 16 * e, jp[e], 512, tw);
  {
    const C2<T> *AB = reinterpret_cast<const C2<T> *>(spec + det * spec_stride + spec_coef_off(M));
    const bool z0 = tidp == 0;
    C2<T> Z[2][16];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int r = 0; r < 16; ++r) Z[e][r] = v[16 * e + p16(r)];
    C2<T> X[2][16];
    // partner of element j_e + 512 r: butterfly j_(1-e), output 15 - r; for
    // t = 0 (j0 = 0, j1 = 256) each butterfly pairs with itself: output
    // (16 - r) mod 16 of butterfly 0, output 15 - r of butterfly 256.  Outputs
    // (0, r) and (1, 15 - r) use the same two values and are formed together.
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const C2<T> a = Z[0][r], c = Z[1][15 - r];
      const C2<T> pa = z0 ? Z[0][(16 - r) & 15] : c;
      const C2<T> pc = z0 ? Z[1][r] : a;
      X[0][r] = split_mul<T>(a, pa, AB[jp[0] + 512 * r]);
      X[1][15 - r] = split_mul<T>(c, pc, AB[jp[1] + 512 * (15 - r)]);
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      dft16<T, true>(X[e]);
#pragma unroll
      for (int m = 0; m < 16; ++m) v[16 * e + m] = X[e][m];   // output r of butterfly j_e at p16(r)
    }
  }
  // ---- exchange: element 16 j_e + r (half e) -> v[16 q + r] = element t + 256 q + 512 r
  {
    const int tid = pinned_tid<T>(tid0);
    const int j1 = tid == 0 ? 256 : 512 - tid;
    C2<T> nv[32];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int r = 0; r < 16; ++r)
        s[kFold ? 17 * (h ? j1 : tid) - h * HP + r : pad16(16 * (h ? j1 : tid) + r - h * HALF)] =
            v[16 * h + p16(r)];
      lds_barrier();
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 8 * h; r < 8 * h + 8; ++r)
          nv[16 * q + r] = s[kFold ? pad16(tid) + 272 * q + 544 * (r - 8 * h)
                                   : pad16(tid + NT * q + 512 * r - h * HALF)];
      lds_barrier();
    }
#pragma unroll
    for (int e = 0; e < 32; ++e) v[e] = nv[e];
  }
  // ---- inverse pass 1 (radix 16, span 16)
#pragma unroll
  for (int q = 0; q < 2; ++q) reg_r16<T, M, true>(v + 16 * q, pinned_tid<T>(tid0) + NT * q, 16, tw);
  // ---- exchange: butterfly j = t + 256 q writes (j - k) 16 + k + 16 r (k = j mod 16,
  // half q) -> v[r] = element t + 256 r, r < 32 (half r / 16)
  {
    const int tid = pinned_tid<T>(tid0);
    C2<T> nv[32];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      {
        const int j = tid + NT * h, k = j & 15;
#pragma unroll
        for (int r = 0; r < 16; ++r)
          s[kFold ? 17 * (tid - (tid & 15)) + (tid & 15) + 17 * r
                  : pad16((j - k) * 16 + k + 16 * r - h * HALF)] = v[16 * h + p16(r)];
      }
      lds_barrier();
#pragma unroll
      for (int r = 16 * h; r < 16 * h + 16; ++r)
        nv[r] = s[kFold ? pad16(tid) + 272 * (r - 16 * h) : pad16(tid + NT * r - h * HALF)];
      lds_barrier();
    }
#pragma unroll
    for (int e = 0; e < 32; ++e) v[e] = nv[e];
  }
  // ---- inverse pass 2 (radix 32, span 256): outputs element t + 256 r, to HBM
  {
    const int tid = pinned_tid<T>(tid0);
    twiddle32<T, true>(v, tw[2 * tid]);
    dft32<T, true>(v);
    const __amdgpu_buffer_rsrc_t zr = row_buffer(out + det * n, n);
    const int hi = lo + V;
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      const C2<T> w = v[p32(r)];
      const int e = 2 * (tid + NT * r);
      if constexpr (PAIR) {
        buf_store2(zr, e >= lo && e < hi ? (uint32_t)(s0 + e) * (uint32_t)sizeof(T) : kDropOffset, w);
      } else {
        buf_store(zr, e >= lo && e < hi ? (uint32_t)(s0 + e) * (uint32_t)sizeof(T) : kDropOffset, w.x);
        buf_store(zr, e + 1 >= lo && e + 1 < hi ? (uint32_t)(s0 + e + 1) * (uint32_t)sizeof(T)
                                                : kDropOffset, w.y);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The same four-exchange scheme for M = 16384 (32768-sample blocks): 512
// threads of 32 values, radices 32, 32, 16 forward (spans 1, 32, 1024) and
// 16, 32, 32 inverse (spans 1, 16, 512).  The last forward pass pairs
// butterflies j and 1024 - j (0 and 512 for thread 0).  Three of the four
// exchanges move a whole radix-32 butterfly per thread in one round (its 32
// outputs fall in one half, chosen per wave).
// ---------------------------------------------------------------------------
// With GAP (FP64 only) the kernel also carries the gap-fill CG's direction
// update and its p . (mask N p) partial (GapFuse); in is then p_prev.
template <typename T, bool PAIR, bool GAP = false>
__global__ void __launch_bounds__(512, sizeof(T) == 4 ? 4 : 2)
k_os_r32x(const T *__restrict__ in, T *__restrict__ out, int64_t n, int32_t b, int64_t nblk,
          const T *__restrict__ spec, int64_t spec_stride, const C2<double> *__restrict__ tw,
          GapFuse gf = GapFuse{}) {
  static_assert(!GAP || sizeof(T) == 8, "the gap-fill fusion is FP64");
  constexpr int M = 16384, L = 2 * M, HALF = M / 2, NT = 512;
  constexpr int HP = HALF + HALF / 16;   // padded half: pad16(e - HALF) = pad16(e) - HP
  // FP32 (VALU-bound) takes each exchange's LDS slots as one per-thread base
  // plus compile-time offsets; FP64 (bound by its LDS exchanges and memory)
  // measured faster with the slots computed per element.
  constexpr bool kFold = sizeof(T) == 4;
  __shared__ C2<T> s[HP];
  const int tid0 = threadIdx.x;
  const int64_t det = (int64_t)blockIdx.x / nblk, blk = (int64_t)blockIdx.x - det * nblk;
  // valid outputs [lo, lo + V) of the block, lo = b - 1 rounded up to even so
  // that the (even, odd) sample pairs a thread moves are all valid or all not
  const int lo = os_pair_lo(b), V = L - 2 * lo;
  const int32_t s0 = (int32_t)(blk * V) - lo;
  C2<T> v[32];

  // ---- forward pass 0 (radix 32, span 1): inputs z[t + 512 r] from HBM
  {
    const int tid = GAP ? fresh_tid(tid0) : pinned_tid<T>(tid0);
    const __amdgpu_buffer_rsrc_t xr = row_buffer(const_cast<T *>(in) + det * n, n);
#pragma unroll
    for (int r = 0; r < (GAP ? 0 : 32); ++r) {
      const int32_t g = s0 + 2 * (tid + NT * r);   // even
      if constexpr (PAIR) {
        // n even: a pair is wholly before the row, inside it or past its end
        v[r] = buf_load2(xr, g >= 0 ? (uint32_t)g * (uint32_t)sizeof(T) : kDropOffset, T());
      } else {
        v[r].x = buf_load<T>(xr, g >= 0 ? (uint32_t)g * (uint32_t)sizeof(T) : kDropOffset);
        v[r].y = buf_load<T>(xr, g + 1 >= 0 ? (uint32_t)(g + 1) * (uint32_t)sizeof(T) : kDropOffset);
      }
    }
    if constexpr (GAP) {
      // p = r / c0 + beta p_prev, element by element (p_prev and the residual
      // loaded together, four elements at a time: the block's 32 values
      // already take half the registers); the block's valid outputs keep p
      // in p_next for the solver's next step
      const __amdgpu_buffer_rsrc_t rr = row_buffer(const_cast<double *>(gf.r) + det * n, n);
      const __amdgpu_buffer_rsrc_t pn = row_buffer(gf.p_next + det * n, n);
      const double ic = gf.inv_c0[det * gf.stride], be = gf.beta[det * gf.stride];
      const int hi = lo + V;
#pragma unroll
      for (int r = 0; r < 32; ++r) {
        const int32_t g = s0 + 2 * (tid + NT * r);
        const int e = 2 * (tid + NT * r);
        C2<T> rv, pv;
        if constexpr (PAIR) {
          rv = buf_load2(rr, g >= 0 ? (uint32_t)g * (uint32_t)sizeof(T) : kDropOffset, T());
          pv = buf_load2(xr, g >= 0 ? (uint32_t)g * (uint32_t)sizeof(T) : kDropOffset, T());
        } else {
          rv.x = buf_load<T>(rr, g >= 0 ? (uint32_t)g * (uint32_t)sizeof(T) : kDropOffset);
          rv.y = buf_load<T>(rr, g + 1 >= 0 ? (uint32_t)(g + 1) * (uint32_t)sizeof(T) : kDropOffset);
          pv.x = buf_load<T>(xr, g >= 0 ? (uint32_t)g * (uint32_t)sizeof(T) : kDropOffset);
          pv.y = buf_load<T>(xr, g + 1 >= 0 ? (uint32_t)(g + 1) * (uint32_t)sizeof(T) : kDropOffset);
        }
        v[r] = C2<T>{rv.x * ic + be * pv.x, rv.y * ic + be * pv.y};
        if constexpr (PAIR) {
          buf_store2(pn, e >= lo && e < hi ? (uint32_t)(s0 + e) * (uint32_t)sizeof(T) : kDropOffset,
                     v[r]);
        } else {
          buf_store(pn, e >= lo && e < hi ? (uint32_t)(s0 + e) * (uint32_t)sizeof(T) : kDropOffset,
                    v[r].x);
          buf_store(pn, e + 1 >= lo && e + 1 < hi ? (uint32_t)(s0 + e + 1) * (uint32_t)sizeof(T)
                                                  : kDropOffset, v[r].y);
        }
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
    dft32<T, false>(v);
  }
  // ---- exchange: element 32 t + r (half t / 256) -> v[r] = element t + 512 r (half r / 16)
  {
    const int tid = pinned_tid<T>(tid0);
    const int hw = __builtin_amdgcn_readfirstlane(tid >> 8);
    C2<T> nv[32];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (hw == h) {
        const int wb = 34 * tid - h * HP;   // pad16(32 t + r - h HALF) = wb + pad16(r)
#pragma unroll
        for (int r = 0; r < 32; ++r)
          s[kFold ? wb + r + (r >> 4) : pad16(32 * tid + r - h * HALF)] = v[p32(r)];
      }
      lds_barrier();
      const int rb = pad16(tid);           // pad16(t + 512 (r + 16 h) - h HALF) = rb + 544 r
#pragma unroll
      for (int r = 0; r < 16; ++r)
        nv[16 * h + r] = s[kFold ? rb + 544 * r : pad16(tid + NT * (r + 16 * h) - h * HALF)];
      lds_barrier();
    }
#pragma unroll
    for (int e = 0; e < 32; ++e) v[e] = nv[e];
  }
  // ---- forward pass 1 (radix 32, span 32): twiddles w^r, w = tw[32 k], k = t mod 32
  {
    const int tid = pinned_tid<T>(tid0);
    twiddle32<T, false>(v, tw[32 * (tid & 31)]);
    dft32<T, false>(v);
  }
  // ---- exchange: butterfly t writes (t - k) 32 + k + 32 r (k = t mod 32; half
  // t / 256) -> paired layout v[16 e + r] = element j_e + 1024 r (half r / 8)
  {
    const int tid = pinned_tid<T>(tid0);
    const int hw = __builtin_amdgcn_readfirstlane(tid >> 8);
    const int j1 = tid == 0 ? 512 : 1024 - tid;
    const int k = tid & 31;
    C2<T> nv[32];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (hw == h) {
        const int wb = 34 * (tid - k) + k + (k >> 4) - h * HP;
#pragma unroll
        for (int r = 0; r < 32; ++r)
          s[kFold ? wb + 34 * r : pad16((tid - k) * 32 + k + 32 * r - h * HALF)] = v[p32(r)];
      }
      lds_barrier();
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int rb = pad16(e ? j1 : tid);  // pad16(j + 1024 (r + 8 h) - h HALF) = rb + 1088 r
#pragma unroll
        for (int r = 0; r < 8; ++r)
          nv[16 * e + 8 * h + r] =
              s[kFold ? rb + 1088 * r : pad16((e ? j1 : tid) + 1024 * (r + 8 * h) - h * HALF)];
      }
      lds_barrier();
    }
#pragma unroll
    for (int e = 0; e < 32; ++e) v[e] = nv[e];
  }
  // ---- forward pass 2 (radix 16, span 1024) on j0 = t, j1; split and kernel
  // multiply; inverse pass 0 (radix 16, span 1) on the same butterflies
  const int tidp = pinned_tid<T>(tid0);
  const int jp[2] = {tidp, tidp == 0 ? 512 : 1024 - tidp};
#pragma unroll
  for (int e = 0; e < 2; ++e) reg_r16<T, M, false>(v + 16 * e, jp[e], 1024, tw);
  {
    const C2<T> *AB = reinterpret_cast<const C2<T> *>(spec + det * spec_stride + spec_coef_off(M));
    const bool z0 = tidp == 0;
    C2<T> Z[2][16];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int r = 0; r < 16; ++r) Z[e][r] = v[16 * e + p16(r)];
    C2<T> X[2][16];
    // partner of element j_e + 1024 r: butterfly j_(1-e), output 15 - r; for
    // t = 0 (j0 = 0, j1 = 512) each butterfly pairs with itself
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const C2<T> a = Z[0][r], c = Z[1][15 - r];
      const C2<T> pa = z0 ? Z[0][(16 - r) & 15] : c;
      const C2<T> pc = z0 ? Z[1][r] : a;
      X[0][r] = split_mul<T>(a, pa, AB[jp[0] + 1024 * r]);
      X[1][15 - r] = split_mul<T>(c, pc, AB[jp[1] + 1024 * (15 - r)]);
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      dft16<T, true>(X[e]);
#pragma unroll
      for (int m = 0; m < 16; ++m) v[16 * e + m] = X[e][m];
    }
  }
  // ---- exchange: element 16 j_e + r (half e) -> v[r] = element t + 512 r (half r / 16)
  {
    const int tid = pinned_tid<T>(tid0);
    const int j1 = tid == 0 ? 512 : 1024 - tid;
    C2<T> nv[32];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int wb = 17 * (h ? j1 : tid) - h * HP;   // pad16(16 j + r - h HALF), r < 16
#pragma unroll
      for (int r = 0; r < 16; ++r)
        s[kFold ? wb + r : pad16(16 * (h ? j1 : tid) + r - h * HALF)] = v[16 * h + p16(r)];
      lds_barrier();
      const int rb = pad16(tid);
#pragma unroll
      for (int r = 0; r < 16; ++r)
        nv[16 * h + r] = s[kFold ? rb + 544 * r : pad16(tid + NT * (r + 16 * h) - h * HALF)];
      lds_barrier();
    }
#pragma unroll
    for (int e = 0; e < 32; ++e) v[e] = nv[e];
  }
  // ---- inverse pass 1 (radix 32, span 16): w = tw[64 k], k = t mod 16
  {
    const int tid = pinned_tid<T>(tid0);
    twiddle32<T, true>(v, tw[64 * (tid & 15)]);
    dft32<T, true>(v);
  }
  // ---- exchange: butterfly t writes (t - k) 32 + k + 16 r (k = t mod 16; half
  // t / 256) -> v[r] = element t + 512 r (half r / 16)
  {
    const int tid = pinned_tid<T>(tid0);
    const int hw = __builtin_amdgcn_readfirstlane(tid >> 8);
    const int k = tid & 15;
    C2<T> nv[32];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (hw == h) {
        const int wb = 34 * (tid - k) + k - h * HP;   // pad16((t - k) 32 + k + 16 r - h HALF)
#pragma unroll
        for (int r = 0; r < 32; ++r)
          s[kFold ? wb + 17 * r : pad16((tid - k) * 32 + k + 16 * r - h * HALF)] = v[p32(r)];
      }
      lds_barrier();
      const int rb = pad16(tid);
#pragma unroll
      for (int r = 0; r < 16; ++r)
        nv[16 * h + r] = s[kFold ? rb + 544 * r : pad16(tid + NT * (r + 16 * h) - h * HALF)];
      lds_barrier();
    }
#pragma unroll
    for (int e = 0; e < 32; ++e) v[e] = nv[e];
  }
  // ---- inverse pass 2 (radix 32, span 512): outputs element t + 512 r, to HBM
  {
    const int tid = pinned_tid<T>(tid0);
    twiddle32<T, true>(v, tw[2 * tid]);
    dft32<T, true>(v);
    const __amdgpu_buffer_rsrc_t zr = row_buffer(out + det * n, n);
    const int hi = lo + V;
    double acc = 0.0;   // GAP: this thread's share of p . (mask N p)
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      const C2<T> w = v[p32(r)];
      const int e = 2 * (tid + NT * r);   // even, as lo and hi are
      if constexpr (PAIR) {
        buf_store2(zr, e >= lo && e < hi ? (uint32_t)(s0 + e) * (uint32_t)sizeof(T) : kDropOffset, w);
      } else {
        buf_store(zr, e >= lo && e < hi ? (uint32_t)(s0 + e) * (uint32_t)sizeof(T) : kDropOffset, w.x);
        buf_store(zr, e + 1 >= lo && e + 1 < hi ? (uint32_t)(s0 + e + 1) * (uint32_t)sizeof(T)
                                                : kDropOffset, w.y);
      }
      if constexpr (GAP) {
        // the pair (s0 + e, s0 + e + 1) is this block's output: p there is
        // what this thread wrote in the first pass
        const int64_t i0 = (int64_t)s0 + e;
        if (e >= lo && e < hi && i0 < n) {
          const int64_t o = det * n + i0;
          const bool two = i0 + 1 < n;
          const double p0 = gf.p_next[o], p1 = two ? gf.p_next[o + 1] : 0.0;
          const bool v0 = gf.gaps[o] == 0, v1 = two && gf.gaps[o + 1] == 0;
          acc += (v0 ? p0 * w.x : 0.0) + (v1 ? p1 * w.y : 0.0);
        }
        if ((r & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
    if constexpr (GAP) {
      __shared__ double wsum[NT / 64];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) acc += __shfl_down(acc, off, 64);
      if ((tid0 & 63) == 0) wsum[tid0 >> 6] = acc;
      __syncthreads();
      if (tid0 == 0) {
        double t = 0.0;
        for (int w = 0; w < NT / 64; ++w) t += wsum[w];   // fixed order
        gf.partial[det * nblk + blk] = t;
      }
    }
  }
}

// Spectrum of the symmetric circular kernel of length L = 2M, divided by M,
// and the split coefficients of split_mul.  One wave per pair (k, M - k),
// k = 0..M/2: since cos(2 pi (M - k) tau / L) = (-1)^tau cos(2 pi k tau / L),
//   H[k]     = (t0 + 2 (S_even + S_odd)) / M,
//   H[M - k] = (t0 + 2 (S_even - S_odd)) / M,
// with S_even / S_odd the sums of t[tau] cos(2 pi k tau / L) over even / odd
// tau >= 1; then alpha and beta of k and M - k, all in FP64, stored as T.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_spectrum(const double *__restrict__ lags, int32_t b,
                                                     int64_t lag_stride, int32_t M,
                                                     const C2<double> *__restrict__ tw64,
                                                     T *__restrict__ spec) {
  const int64_t kern = blockIdx.y;
  const int k = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k > M / 2) return;
  const double *t = lags + kern * lag_stride;
  const int64_t Lmask = 2 * M - 1;
  double se = 0.0, so = 0.0;
  for (int tau = 1 + lane; tau < b; tau += 64) {
    const double v = t[tau] * tw64[((int64_t)k * tau) & Lmask].x;
    if (tau & 1) so += v;
    else se += v;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    se += __shfl_down(se, off, 64);
    so += __shfl_down(so, off, 64);
  }
  if (lane != 0) return;
  T *H = spec + kern * spec_block(M);
  C2<T> *AB = reinterpret_cast<C2<T> *>(H + spec_coef_off(M));
  const int k2 = M - k;
  const double hk = (t[0] + 2.0 * (se + so)) / (double)M;
  const double hk2 = (t[0] + 2.0 * (se - so)) / (double)M;
  H[k] = (T)hk;
  if (k2 != k) H[k2] = (T)hk2;
  const double hp = 0.5 * (hk + hk2), hm = 0.5 * (hk - hk2);
  const C2<double> w = tw64[k];
  AB[k] = {(T)(hp + w.y * hm), (T)(w.x * hm)};
  if (k2 < M && k2 != k) {
    const C2<double> w2 = tw64[k2];
    AB[k2] = {(T)(hp - w2.y * hm), (T)(-w2.x * hm)};
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

// The register-resident kernels take 32-bit sample offsets (n + 4M < 2^31)
// and address each row as a buffer of fewer than 2^31 bytes.
template <typename T>
static bool os_reg_fits(int64_t n_samp, int64_t M) {
  return n_samp + 4 * M < ((int64_t)1 << 31) && n_samp * (int64_t)sizeof(T) < ((int64_t)1 << 31);
}

// FFT half-length M used for noise model N in precision T: the smallest power
// of two with M >= 4 (b - 1) (at most a quarter of each block is halo),
// capped at 8192; 16384 above 2560 lags in FP64 and 3072 in FP32, where the
// longer block's smaller halo outweighs its slower transform (measured
// crossovers).  A stream too long for the register kernels' 32-bit offsets
// keeps M = 8192 up to 4096 lags, where the LDS kernel can take an FP64 block.
template <typename T>
int os_half_length(const furax_noise *N) {
  const int64_t b = N->bandwidth;
  constexpr int64_t kLong = sizeof(T) == 8 ? 2560 : 3072;
  int64_t m = 512;
  while (m < 4 * (b - 1) && m < 8192) m *= 2;
  if (b > 4096 || (b > kLong && os_reg_fits<T>(N->n_samp, 16384))) m = 16384;
  return (int)m;
}

template <typename T>
int64_t os_max_band() { return 8192; }
template int64_t os_max_band<float>();
template int64_t os_max_band<double>();

constexpr int kMaxDeprojNP = 8;   // template deprojection: Legendre degrees 0..7
static furax_status launch_deproj_gram(const furax_noise *N, double *Lg, hipStream_t s);

// Workspace of a noise model in precision T: the band kernel's spectrum, or
// the template deprojection's Gram factor.
template <typename T>
size_t noise_workspace_bytes(const furax_noise *N) {
  if (N->kind == 2) return sizeof(double) * kMaxDeprojNP * kMaxDeprojNP;   // Gram factor
  if (N->kind != 1) return 0;
  const int M = os_half_length<T>(N);
  const int64_t nk = N->toeplitz_stride ? N->n_det : 1;
  return (size_t)nk * spec_block(M) * sizeof(T);
}
template size_t noise_workspace_bytes<float>(const furax_noise *);
template size_t noise_workspace_bytes<double>(const furax_noise *);

// Compute the kernel spectrum into `spec` (noise_workspace_bytes<T> bytes).
template <typename T>
furax_status noise_prepare(const furax_noise *N, void *spec, hipStream_t s) {
  if (N->kind == 2) return launch_deproj_gram(N, static_cast<double *>(spec), s);
  if (N->kind != 1) return FURAX_OK;
  const int M = os_half_length<T>(N);
  TwTables tw;
  FX_TRY(get_twiddles(2 * M, s, tw));
  const int64_t nk = N->toeplitz_stride ? N->n_det : 1;
  constexpr int per_block = kBlock / 64;
  dim3 grid((M / 2 + 1 + per_block - 1) / per_block, (unsigned)nk);
  hipLaunchKernelGGL(k_spectrum<T>, grid, dim3(kBlock), 0, s, N->toeplitz, (int32_t)N->bandwidth,
                     N->toeplitz_stride, M, tw.tw64, static_cast<T *>(spec));
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
  const int64_t spec_stride = N->toeplitz_stride ? spec_block(M) : 0;
  hipLaunchKernelGGL((k_overlap_save<T, M, NT, false>), dim3((unsigned)ntask), dim3(NT), 0, s, in,
                     out, N->n_samp, b, nblk, ntask, spec, spec_stride, tw);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}

template <typename T>
static furax_status launch_os_r32(const furax_noise *N, const T *in, T *out, const T *spec,
                                  const C2<double> *tw, hipStream_t s) {
  constexpr int M = 8192;
  const int b = (int)N->bandwidth;
  if (!os_reg_fits<T>(N->n_samp, M)) return launch_os<T, M, M / 16>(N, in, out, spec, tw, s);
  const int64_t V = 2 * M - 2 * (int64_t)os_pair_lo(b);
  const int64_t nblk = (N->n_samp + V - 1) / V;
  const int64_t ntask = N->n_det * nblk;
  const int64_t spec_stride = N->toeplitz_stride ? spec_block(M) : 0;
  if (N->n_samp % 2 == 0)
    hipLaunchKernelGGL((k_os_r32<T, true>), dim3((unsigned)ntask), dim3(256), 0, s, in, out,
                       N->n_samp, b, nblk, spec, spec_stride, tw);
  else
    hipLaunchKernelGGL((k_os_r32<T, false>), dim3((unsigned)ntask), dim3(256), 0, s, in, out,
                       N->n_samp, b, nblk, spec, spec_stride, tw);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}

template <typename T>
static furax_status launch_os_r32x(const furax_noise *N, const T *in, T *out, const T *spec,
                                   const C2<double> *tw, hipStream_t s) {
  constexpr int M = 16384;
  const int b = (int)N->bandwidth;
  const int64_t V = 2 * M - 2 * (int64_t)os_pair_lo(b);
  const int64_t nblk = (N->n_samp + V - 1) / V;
  const int64_t ntask = N->n_det * nblk;
  const int64_t spec_stride = N->toeplitz_stride ? spec_block(M) : 0;
  if (!os_reg_fits<T>(N->n_samp, M)) {
    // the LDS kernel holds a whole block: an FP64 32768-sample block does not fit
    if constexpr (sizeof(T) == 8)
      return set_error(FURAX_EUNSUPPORTED, "FP64 band above 4096 lags on streams of 2^28 samples or more");
    else
      return launch_os<T, M, M / 16>(N, in, out, spec, tw, s);
  }
  if (N->n_samp % 2 == 0)
    hipLaunchKernelGGL((k_os_r32x<T, true>), dim3((unsigned)ntask), dim3(512), 0, s, in, out,
                       N->n_samp, b, nblk, spec, spec_stride, tw);
  else
    hipLaunchKernelGGL((k_os_r32x<T, false>), dim3((unsigned)ntask), dim3(512), 0, s, in, out,
                       N->n_samp, b, nblk, spec, spec_stride, tw);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}

// ---------------------------------------------------------------------------
// Template deprojection F_T = W - W T (T^T W T)^-1 T^T W (Eq. (3)) with
// W = w_k I and T the Legendre baselines P_0 .. P_{NP-1} of each segment:
//   z = w_k (y - T_s G^-1 T_s^T y),  G = T_s^T T_s.
// One workgroup per (detector, segment).  Pass 1 accumulates, in FP64, the
// projections T_s^T y over the segment's samples; the partial sums are
// combined in a fixed order (wave shuffles, then the waves in order), and one
// thread solves G c = T_s^T y by Cholesky.  Pass 2 re-reads the segment
// (L2-resident) and writes w_k (y - sum_j c_j P_j).  G depends only on the
// segment's length: every full-length segment takes the Cholesky factor that
// k_deproj_gram computes once per application (the same sums in the same
// order), and only a stream's longer last segment accumulates its own Gram
// sums in pass 1.
// ---------------------------------------------------------------------------
constexpr int kDeprojThreads = 256;

// P_0 .. P_{NP-1} at x in [-1, 1] by the three-term recurrence, each step
// multiplied by the constant 1 / (j + 1) rather than divided (within an ulp of
// the quotient; sample i of a segment of length len sits at
// x = (2 i + 1) / len - 1, taken as (2 i + 1) * (1 / len) - 1 for the same
// reason): the basis is evaluated the same way in every pass and in the Gram
// factor, so the projection stays exact for the basis used.
template <int NP>
__device__ __forceinline__ void legendre_at(double x, double (&P)[NP]) {
#pragma clang fp contract(off)
  P[0] = 1.0;
  if constexpr (NP > 1) P[1] = x;
#pragma unroll
  for (int j = 1; j + 1 < NP; ++j)
    P[j + 1] = ((double)(2 * j + 1) * x * P[j] - (double)j * P[j - 1]) * (1.0 / (double)(j + 1));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Workgroup sums of acc[0..NV) in a fixed order: each wave's shuffle tree,
// then the waves in order; the result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void deproj_reduce(double (&acc)[NV], double (&part)[kDeprojThreads / 64][NV],
                                              double (&r)[NV]) {
  constexpr int NW = kDeprojThreads / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double t = wave_sum(acc[v]);
    if (lane == 0) part[wave][v] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      r[v] = part[0][v];
#pragma unroll
      for (int q = 1; q < NW; ++q) r[v] += part[q][v];
    }
  }
}

// Lower Cholesky factor Lm of G, given as its upper triangle by rows in g.
template <int NP>
__device__ __forceinline__ void gram_cholesky(const double *g, double (&Lm)[NP][NP]) {
#pragma clang fp contract(off)
  int k = 0;
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int l = j; l < NP; ++l) Lm[l][j] = g[k++];   // lower triangle holds G
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    double d = Lm[j][j];
#pragma unroll
    for (int m = 0; m < j; ++m) d -= Lm[j][m] * Lm[j][m];
    d = sqrt(d);
    Lm[j][j] = d;
#pragma unroll
    for (int l = j + 1; l < NP; ++l) {
      double v = Lm[l][j];
#pragma unroll
      for (int m = 0; m < j; ++m) v -= Lm[l][m] * Lm[j][m];
      Lm[l][j] = v / d;
    }
  }
}

// c = G^-1 rhs by forward and back substitution with G = Lm Lm^T.
template <int NP>
__device__ __forceinline__ void chol_solve(const double (&Lm)[NP][NP], const double *rhs,
                                           double (&c)[NP]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    double v = rhs[j];
#pragma unroll
    for (int m = 0; m < j; ++m) v -= Lm[j][m] * c[m];
    c[j] = v / Lm[j][j];
  }
#pragma unroll
  for (int j = NP - 1; j >= 0; --j) {
    double v = c[j];
#pragma unroll
    for (int m = j + 1; m < NP; ++m) v -= Lm[m][j] * c[m];
    c[j] = v / Lm[j][j];
  }
}

// Gram sums of one sample's basis values P, added to g[0..NG).
template <int NP>
__device__ __forceinline__ void gram_add(const double (&P)[NP], double *g) {
#pragma clang fp contract(off)
  int k = 0;
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int l = j; l < NP; ++l) g[k++] += P[j] * P[l];
}

// The Cholesky factor of G for a segment of seg_len samples, into Lg[NP][NP].
template <int NP>
__global__ void __launch_bounds__(kDeprojThreads) k_deproj_gram(int64_t seg_len,
                                                                double *__restrict__ Lg) {
#pragma clang fp contract(off)
  constexpr int NG = NP * (NP + 1) / 2;
  __shared__ double part[kDeprojThreads / 64][NG];
  const double inv_len = 1.0 / (double)seg_len;
  double acc[NG];
#pragma unroll
  for (int v = 0; v < NG; ++v) acc[v] = 0.0;
  for (int64_t i = threadIdx.x; i < seg_len; i += kDeprojThreads) {
    double P[NP];
    legendre_at<NP>((2.0 * (double)i + 1.0) * inv_len - 1.0, P);
    gram_add<NP>(P, acc);
  }
  double r[NG];
  deproj_reduce<NG>(acc, part, r);
  if (threadIdx.x == 0) {
    double Lm[NP][NP];
    gram_cholesky<NP>(r, Lm);
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int l = 0; l < NP; ++l) Lg[j * NP + l] = l <= j ? Lm[j][l] : 0.0;
  }
}

// Lg: the factor of full-length segments from k_deproj_gram, or null (every
// segment accumulates its own Gram sums).
template <typename T, int NP>
__global__ void __launch_bounds__(kDeprojThreads) k_deproject(const T *__restrict__ in,
                                                              T *__restrict__ out, int64_t n,
                                                              int64_t seg_len, int64_t nseg,
                                                              const double *__restrict__ w,
                                                              double *__restrict__ amp,
                                                              const double *__restrict__ Lg) {
#pragma clang fp contract(off)
  constexpr int NG = NP * (NP + 1) / 2;
  constexpr int NV = NP + NG;
  __shared__ double part[kDeprojThreads / 64][NV];
  __shared__ double part_y[kDeprojThreads / 64][NP];
  __shared__ double coef[NP];
  const int64_t det = (int64_t)blockIdx.x / nseg, seg = (int64_t)blockIdx.x - det * nseg;
  const int64_t i0 = seg * seg_len;
  const int64_t len = seg + 1 < nseg ? seg_len : n - i0;
  const T *y = in + det * n + i0;
  T *z = out + det * n + i0;
  const double inv_len = 1.0 / (double)len;
  // workgroup-uniform: a full-length segment with a precomputed factor
  const bool known = Lg != nullptr && len == seg_len;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  if (known) {
    for (int64_t i = threadIdx.x; i < len; i += kDeprojThreads) {
      double P[NP];
      legendre_at<NP>((2.0 * (double)i + 1.0) * inv_len - 1.0, P);
      const double yi = (double)y[i];
#pragma unroll
      for (int j = 0; j < NP; ++j) acc[j] += P[j] * yi;
    }
  } else {
    for (int64_t i = threadIdx.x; i < len; i += kDeprojThreads) {
      double P[NP];
      legendre_at<NP>((2.0 * (double)i + 1.0) * inv_len - 1.0, P);
      const double yi = (double)y[i];
#pragma unroll
      for (int j = 0; j < NP; ++j) acc[j] += P[j] * yi;
      gram_add<NP>(P, acc + NP);
    }
  }
  double r[NV];
  if (known) {
    double a[NP], rp[NP];
#pragma unroll
    for (int v = 0; v < NP; ++v) a[v] = acc[v];
    deproj_reduce<NP>(a, part_y, rp);
#pragma unroll
    for (int v = 0; v < NP; ++v) r[v] = rp[v];
  } else {
    deproj_reduce<NV>(acc, part, r);
  }
  if (threadIdx.x == 0) {
    double Lm[NP][NP];
    if (known) {
#pragma unroll
      for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int l = 0; l < NP; ++l) Lm[j][l] = Lg[j * NP + l];
    } else {
      gram_cholesky<NP>(r + NP, Lm);
    }
    double c[NP];
    chol_solve<NP>(Lm, r, c);
#pragma unroll
    for (int j = 0; j < NP; ++j) coef[j] = c[j];
    if (amp) {   // the template fit (T^T W T)^-1 T^T W y of this segment (w cancels)
#pragma unroll
      for (int j = 0; j < NP; ++j) amp[(int64_t)blockIdx.x * NP + j] = c[j];
    }
  }
  if (!out) return;   // amplitudes only (uniform over the workgroup)
  __syncthreads();
  double c[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) c[j] = coef[j];
  const double wk = w[det];
  for (int64_t i = threadIdx.x; i < len; i += kDeprojThreads) {
    double P[NP];
    legendre_at<NP>((2.0 * (double)i + 1.0) * inv_len - 1.0, P);
    double fit = 0.0;
#pragma unroll
    for (int j = 0; j < NP; ++j) fit += c[j] * P[j];
    // the output is not read again by this kernel: stored non-temporally
    __builtin_nontemporal_store((T)(wk * ((double)y[i] - fit)), z + i);
  }
}

template <typename T, int NP>
static furax_status launch_deproject_np(const furax_noise *N, const T *in, T *out, double *amp,
                                        const double *Lg, hipStream_t s) {
  const int64_t nseg = std::max<int64_t>(1, N->n_samp / N->tmpl_seg_len);
  hipLaunchKernelGGL((k_deproject<T, NP>), dim3((unsigned)(N->n_det * nseg)),
                     dim3(kDeprojThreads), 0, s, in, out, N->n_samp, N->tmpl_seg_len, nseg,
                     N->inv_var, amp, Lg);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}

template <int NP>
static furax_status launch_deproj_gram_np(const furax_noise *N, double *Lg, hipStream_t s) {
  hipLaunchKernelGGL((k_deproj_gram<NP>), dim3(1), dim3(kDeprojThreads), 0, s,
                     (int64_t)N->tmpl_seg_len, Lg);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}

// The full-length segments' Cholesky factor into Lg (kMaxDeprojNP^2 doubles).
static furax_status launch_deproj_gram(const furax_noise *N, double *Lg, hipStream_t s) {
  switch (N->tmpl_order) {
    case 0: return launch_deproj_gram_np<1>(N, Lg, s);
    case 1: return launch_deproj_gram_np<2>(N, Lg, s);
    case 2: return launch_deproj_gram_np<3>(N, Lg, s);
    case 3: return launch_deproj_gram_np<4>(N, Lg, s);
    case 4: return launch_deproj_gram_np<5>(N, Lg, s);
    case 5: return launch_deproj_gram_np<6>(N, Lg, s);
    case 6: return launch_deproj_gram_np<7>(N, Lg, s);
    case 7: return launch_deproj_gram_np<8>(N, Lg, s);
  }
  return set_error(FURAX_EINVAL, "tmpl_order must be in [0, 7]");
}

// out = F_T in (out may be null: amplitudes only); amp [n_det][n_seg][order + 1]
// receives the template fit of each segment when not null.
template <typename T>
furax_status launch_deproject(const furax_noise *N, const T *in, T *out, double *amp,
                              hipStream_t s, const double *Lg) {
  if (N->n_samp == 0) return FURAX_OK;
  switch (N->tmpl_order) {
    case 0: return launch_deproject_np<T, 1>(N, in, out, amp, Lg, s);
    case 1: return launch_deproject_np<T, 2>(N, in, out, amp, Lg, s);
    case 2: return launch_deproject_np<T, 3>(N, in, out, amp, Lg, s);
    case 3: return launch_deproject_np<T, 4>(N, in, out, amp, Lg, s);
    case 4: return launch_deproject_np<T, 5>(N, in, out, amp, Lg, s);
    case 5: return launch_deproject_np<T, 6>(N, in, out, amp, Lg, s);
    case 6: return launch_deproject_np<T, 7>(N, in, out, amp, Lg, s);
    case 7: return launch_deproject_np<T, 8>(N, in, out, amp, Lg, s);
  }
  return set_error(FURAX_EINVAL, "tmpl_order must be in [0, 7]");
}
template furax_status launch_deproject<float>(const furax_noise *, const float *, float *, double *,
                                              hipStream_t, const double *);
template furax_status launch_deproject<double>(const furax_noise *, const double *, double *,
                                               double *, hipStream_t, const double *);

// Apply the weight: N^-1 given a prepared spectrum (kind 1) or the diagonal
// weights (kind 0), or the template deprojection F_T (kind 2).
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
  if (N->kind == 2)
    return launch_deproject<T>(N, in, out, nullptr, s, static_cast<const double *>(spec));
  const int M = os_half_length<T>(N);
  TwTables tw;
  FX_TRY(get_twiddles(2 * M, s, tw));
  const T *sp = static_cast<const T *>(spec);
  const C2<double> *t = tw.tw64;   // FP64 twiddles for both precisions
  switch (M) {
    case 512: return launch_os<T, 512, 64>(N, in, out, sp, t, s);
    case 1024: return launch_os<T, 1024, 64>(N, in, out, sp, t, s);
    case 2048: return launch_os<T, 2048, 128>(N, in, out, sp, t, s);
    case 4096: return launch_os<T, 4096, 256>(N, in, out, sp, t, s);
    case 8192:
      return launch_os_r32<T>(N, in, out, sp, t, s);
    case 16384:
      return launch_os_r32x<T>(N, in, out, sp, t, s);
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

int64_t noise_gap_blocks(const furax_noise *C) {
  constexpr int M = 16384;
  if (C->kind != 1 || C->n_samp == 0) return 0;
  if (os_half_length<double>(C) != M || !os_reg_fits<double>(C->n_samp, M)) return 0;
  const int64_t V = 2 * M - 2 * (int64_t)os_pair_lo((int)C->bandwidth);
  return (C->n_samp + V - 1) / V;
}

furax_status noise_run_gap(const furax_noise *C, const double *p_prev, double *q,
                           const void *spec, const GapFuse &g, hipStream_t s) {
  constexpr int M = 16384;
  const int64_t nblk = noise_gap_blocks(C);
  if (nblk == 0) return set_error(FURAX_EUNSUPPORTED, "no fused gap-fill kernel for this band");
  TwTables tw;
  FX_TRY(get_twiddles(2 * M, s, tw));
  const int b = (int)C->bandwidth;
  const int64_t ntask = C->n_det * nblk;
  const int64_t spec_stride = C->toeplitz_stride ? spec_block(M) : 0;
  const double *sp = static_cast<const double *>(spec);
  if (C->n_samp % 2 == 0)
    hipLaunchKernelGGL((k_os_r32x<double, true, true>), dim3((unsigned)ntask), dim3(512), 0, s,
                       p_prev, q, C->n_samp, b, nblk, sp, spec_stride, tw.tw64, g);
  else
    hipLaunchKernelGGL((k_os_r32x<double, false, true>), dim3((unsigned)ntask), dim3(512), 0, s,
                       p_prev, q, C->n_samp, b, nblk, sp, spec_stride, tw.tw64, g);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}

}  // namespace fx
