// Superpixel-major accumulation for P^T and for the block-Jacobi blocks.
//
// P^T is a per-pixel reduction over every sample that falls in the pixel.
// Sample-ordered tiles can only privatise the hits a pixel gets while the
// focal plane sweeps it once (~13 at nside 512 with 256 detectors); every
// tile then adds its partial sums to the global map with FP64 atomics, which
// this GPU performs past the L2, one memory transaction each.  Here the
// reduction is organised by sky region instead:
//
//  * once per plan, each sample's ring pixel is relabelled by its HEALPix
//    NESTED index, whose high bits name a compact superpixel of kSpPix = 1024
//    pixels (a 32 x 32 block of one base face).  Each detector's stream is cut
//    into runs of consecutive samples that stay in one superpixel, the runs
//    are sorted by superpixel (stably, so the order is deterministic) and
//    grouped into chunks of at most SpPlan::chunk_runs runs;
//  * at every application one workgroup per group of up to kChunksPerGroup
//    chunks of one superpixel streams their runs -- tens of consecutive
//    samples each, so the loads stay coalesced -- and adds into LDS sums
//    indexed directly by the pixel's offset inside the superpixel: no
//    hashing, and nothing atomic outside LDS.  The group writes one partial
//    (24 KB), so the partials' HBM traffic is a quarter of one per chunk;
//  * a second kernel sums each superpixel's group partials in group order
//    and writes every pixel of the output exactly once, in ring order.  The
//    LDS sums of a group are added by several waves at once, so their order,
//    hence the last bits of the result, may differ from run to run.
//
// The plan also keeps, in the run-sorted order, each scheduled sample's pixel
// offset inside its superpixel and (angle pointing) its angle psi, so that
// the accumulation reads them contiguously rather than in run-sized pieces
// of the time-ordered planes, whose partly used cache lines would triple its
// traffic.  P still expands the pointing at every application for its own
// gathers; P^T recomputes the polariser weights from psi (or the
// quaternions) at every application.
#include <algorithm>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace fx {

// ---------------------------------------------------------------------------
// Nested <-> ring relabelling (HEALPix, Gorski et al. 2005).
//
// Nested index n = f nside^2 + interleave(x, y): base face f (0-3 north row,
// 4-7 equatorial row, 8-11 south row), x on the even bits and y on the odd
// bits.  Pixel (x, y) of face f lies on ring (2 + f/4) nside - x - y - 1
// counted from the north pole (1 .. 4 nside - 1).  Along its ring it sits
// (x - y) half-pixels east of the face's own longitude, which is 1, 3, 5, 7
// (north and south rows) or 0, 2, 4, 6 (equatorial row) in units of pi/4; in
// the equatorial belt every other ring is shifted by half a pixel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t even_bits(uint32_t w) {
  w &= 0x55555555u;
  w = (w | (w >> 1)) & 0x33333333u;
  w = (w | (w >> 2)) & 0x0f0f0f0fu;
  w = (w | (w >> 4)) & 0x00ff00ffu;
  w = (w | (w >> 8)) & 0x0000ffffu;
  return w;
}

__device__ __forceinline__ int64_t nest_to_ring(int32_t nside, int64_t n) {
  const int64_t N = nside;
  const int64_t face_pix = N * N;
  const int64_t f = n / face_pix;
  const uint32_t w = (uint32_t)(n - f * face_pix);
  const int64_t x = even_bits(w), y = even_bits(w >> 1);
  const int64_t row = f >> 2;
  const int64_t ring = (2 + row) * N - x - y - 1;
  int64_t nr, before, shift;
  if (ring < N) {                 // north cap: 4 ring pixels per ring step
    nr = ring;
    before = 2 * nr * (nr - 1);
    shift = 0;
  } else if (ring > 3 * N) {      // south cap
    nr = 4 * N - ring;
    before = 12 * N * N - 2 * nr * (nr + 1);
    shift = 0;
  } else {                        // equatorial belt: 4 nside pixels per ring
    nr = N;
    before = 2 * N * (N - 1) + (ring - N) * 4 * N;
    shift = (ring - N) & 1;
  }
  const int64_t face_lon = row == 1 ? 2 * (f & 3) : 2 * (f & 3) + 1;
  int64_t j = (face_lon * nr + x - y + 1 + shift) / 2;   // 1-based position in the ring
  if (j > 4 * nr) j -= 4 * nr;
  else if (j < 1) j += 4 * nr;
  return before + j - 1;
}

__global__ void __launch_bounds__(kBlock) k_nest_tables(int32_t nside, int64_t npix,
                                                        int32_t *__restrict__ n2r,
                                                        int32_t *__restrict__ r2n) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x; n < npix; n += stride) {
    const int64_t r = nest_to_ring(nside, n);   // a bijection onto [0, npix)
    n2r[n] = (int32_t)r;
    if ((uint64_t)r < (uint64_t)npix) r2n[r] = (int32_t)n;
  }
}

// ---------------------------------------------------------------------------
// Plan construction.
// ---------------------------------------------------------------------------
// Nested index of every sample (-1 when the pointing is invalid).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_nest_plane(PtArgs<T> a, const int32_t *__restrict__ r2n,
                                                       int32_t *__restrict__ plane) {
  const int64_t S = a.n_det * a.n_samp;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < S; s += stride) {
    int32_t p;
    if (a.qb) {
      const int64_t k = s / a.n_samp, i = s - k * a.n_samp;
      const QuatDir d = quat_dir(qmul(load_quat(a.qb, i), load_quat(a.qd, k)));
      p = zphi2pix_ring(a.nside, d.z, d.phi);
    } else {
      p = ang2pix_ring(a.nside, (double)a.theta[s], (double)a.phi[s]);
    }
    plane[s] = p >= 0 ? r2n[p] : -1;
  }
}

// A run starts where the superpixel changes, at the start of every detector
// stream and every kMaxRun samples (runs stay short enough to balance).
__global__ void __launch_bounds__(kBlock) k_run_heads(int64_t S, int64_t n_samp, int32_t log2P,
                                                      const int32_t *__restrict__ plane,
                                                      uint8_t *__restrict__ head) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < S; s += stride) {
    const int64_t i = s % n_samp;
    bool h = i == 0 || (i % kMaxRun) == 0;
    if (!h) {
      const int32_t a = plane[s], b = plane[s - 1];
      h = (a < 0 ? -1 : a >> log2P) != (b < 0 ? -1 : b >> log2P);
    }
    head[s] = h ? 1 : 0;
  }
}

// Run r = [heads[r], heads[r+1]): key = its superpixel (n_sp for flagged
// samples, sorted last and dropped), value = offset << 16 | length.
__global__ void __launch_bounds__(kBlock) k_run_make(int64_t n_heads, int64_t S, int32_t log2P,
                                                     int64_t n_sp,
                                                     const int64_t *__restrict__ heads,
                                                     const int32_t *__restrict__ plane,
                                                     uint32_t *__restrict__ key,
                                                     uint64_t *__restrict__ val) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n_heads; r += stride) {
    const int64_t off = heads[r];
    const int64_t end = r + 1 < n_heads ? heads[r + 1] : S;
    const int32_t p = plane[off];
    key[r] = p < 0 ? (uint32_t)n_sp : (uint32_t)(p >> log2P);
    val[r] = ((uint64_t)off << 16) | (uint64_t)(end - off);
  }
}

// Sorted keys -> [first, end) of each superpixel's runs (no atomics).
__global__ void __launch_bounds__(kBlock) k_run_bounds(int64_t n, const uint32_t *__restrict__ key,
                                                       int64_t n_sp, int64_t *__restrict__ first,
                                                       int64_t *__restrict__ last) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n; r += stride) {
    const uint32_t k = key[r];
    if (k >= (uint32_t)n_sp) continue;
    if (r == 0 || key[r - 1] != k) first[k] = r;
    if (r == n - 1 || key[r + 1] != k) last[k] = r + 1;
  }
}

// One workgroup per chunk: replace each run's (offset << 16 | length) by
// (offset << 24 | exclusive prefix of the lengths within the chunk) and record
// the chunk's total sample count.
constexpr int kFinalizeThreads = 1024;
static_assert(kChunkRunsMax <= kFinalizeThreads, "one thread per run");
__global__ void __launch_bounds__(kFinalizeThreads) k_run_finalize(uint64_t *__restrict__ runs,
                                                                   SpChunk *__restrict__ chunks) {
  __shared__ int32_t buf[2][kFinalizeThreads];
  SpChunk &ch = chunks[blockIdx.x];
  const int r = threadIdx.x;
  const uint64_t w = r < ch.nr ? runs[ch.r0 + r] : 0;
  const int32_t len = (int32_t)(w & 0xffff);
  buf[0][r] = len;
  __syncthreads();
  int cur = 0;
  for (int d = 1; d < kFinalizeThreads; d <<= 1) {   // inclusive scan
    const int32_t v = buf[cur][r] + (r >= d ? buf[cur][r - d] : 0);
    buf[cur ^ 1][r] = v;
    cur ^= 1;
    __syncthreads();
  }
  const int32_t incl = buf[cur][r];
  if (r < ch.nr) runs[ch.r0 + r] = ((w >> 16) << 24) | (uint64_t)(incl - len);
  if (r == ch.nr - 1) ch.w = incl;
}

// One workgroup per chunk: the chunk's run table in LDS, then threads over
// consecutive sorted slots (coalesced writes), each finding its run by a
// binary search, copy the sample's pixel offset (nested index minus the
// superpixel's first) and, with angle pointing, its angle psi into the
// run-sorted order.
template <typename T>
__global__ void __launch_bounds__(kFinalizeThreads) k_sp_sort(const uint64_t *__restrict__ runs,
                                                              const SpChunk *__restrict__ chunks,
                                                              const int32_t *__restrict__ nest_plane,
                                                              const T *__restrict__ psi,
                                                              int32_t log2P,
                                                              uint16_t *__restrict__ lab,
                                                              T *__restrict__ psi_out) {
  __shared__ int32_t pre[kChunkRunsMax + 1];
  __shared__ int64_t off[kChunkRunsMax];
  const SpChunk ch = chunks[blockIdx.x];
  const int32_t base = ch.sp << log2P;
  for (int r = threadIdx.x; r < ch.nr; r += kFinalizeThreads) {
    const uint64_t w = runs[ch.r0 + r];
    off[r] = (int64_t)(w >> 24);
    pre[r] = (int32_t)(w & 0xffffff);
  }
  if (threadIdx.x == 0) pre[ch.nr] = ch.w;
  __syncthreads();
  for (int32_t j = threadIdx.x; j < ch.w; j += kFinalizeThreads) {
    int32_t lo = 0, hi = ch.nr;                   // last run with pre <= j
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (pre[mid] <= j) lo = mid;
      else hi = mid;
    }
    const int64_t src = off[lo] + (j - pre[lo]);
    const int64_t dst = (int64_t)ch.s0 + j;
    lab[dst] = (uint16_t)(nest_plane[src] - base);
    if (psi_out) psi_out[dst] = psi[src];
  }
}

// The nested index of each detector's first sample (the largest int32 when
// that sample's pointing is invalid): the key that orders the detectors.
__global__ void __launch_bounds__(kBlock) k_det_keys(int64_t n_det, int64_t n_samp,
                                                     const int32_t *__restrict__ plane,
                                                     int32_t *__restrict__ key) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n_det) return;
  const int32_t v = plane[k * n_samp];
  key[k] = v >= 0 ? v : 0x7fffffff;
}

static unsigned grid_for(int64_t n, int64_t cap = 65536) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, cap));
}

void SpPlan::release(hipStream_t s) {
  for (void *p : {(void *)n2r, (void *)r2n, (void *)runs, (void *)chunks, (void *)groups,
                  (void *)sp_group, (void *)partial, (void *)lab, psi, (void *)det_perm}) {
    if (p) (void)hipFreeAsync(p, s);
  }
  *this = SpPlan();
}

bool sp_supported(int64_t nside, int64_t S) {
  return nside >= 1 && (nside & (nside - 1)) == 0 && S > 0 && S < ((int64_t)1 << 31);
}

furax_status sp_nest_tables(SpPlan &sp, int64_t nside, hipStream_t s) {
  sp.nside = (int32_t)nside;
  sp.npix = 12 * nside * nside;
  int32_t l2 = 0;
  while ((int64_t)1 << (l2 + 1) <= nside && l2 < 5) ++l2;   // superpixel side min(nside, 32)
  sp.log2P = 2 * l2;
  sp.n_sp = sp.npix >> sp.log2P;
  if (hipMallocAsync((void **)&sp.n2r, sizeof(int32_t) * sp.npix, s) != hipSuccess ||
      hipMallocAsync((void **)&sp.r2n, sizeof(int32_t) * sp.npix, s) != hipSuccess)
    return set_error(FURAX_ENOMEM, "superpixel tables: allocation failed");
  hipLaunchKernelGGL(k_nest_tables, dim3(grid_for(sp.npix)), dim3(kBlock), 0, s, sp.nside,
                     sp.npix, sp.n2r, sp.r2n);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}

template <typename T>
furax_status sp_build_runs(SpPlan &sp, const PtArgs<T> &a, const int32_t *plane,
                           int32_t n_values, hipStream_t s) {
  const int64_t S = a.n_det * a.n_samp;
  DevBuf b_head, b_heads, b_nsel, b_key, b_val, b_key2, b_cnt, b_tmp;
  FX_TRY(b_head.alloc(S, s));
  FX_TRY(b_heads.alloc(sizeof(int64_t) * S, s));
  FX_TRY(b_nsel.alloc(sizeof(int64_t), s));
  uint8_t *head = static_cast<uint8_t *>(b_head.ptr);
  int64_t *heads = static_cast<int64_t *>(b_heads.ptr);
  int64_t *nsel = static_cast<int64_t *>(b_nsel.ptr);

  hipLaunchKernelGGL(k_run_heads, dim3(grid_for(S)), dim3(kBlock), 0, s, S, a.n_samp, sp.log2P,
                     plane, head);
  FX_HIP(hipGetLastError());

  // heads = positions of the head flags, in order
  hipcub::CountingInputIterator<int64_t> counting(0);
  size_t tmp_bytes = 0;
  FX_HIP(hipcub::DeviceSelect::Flagged(nullptr, tmp_bytes, counting, head, heads, nsel, (int)S, s));
  FX_TRY(b_tmp.alloc(tmp_bytes, s));
  FX_HIP(hipcub::DeviceSelect::Flagged(b_tmp.ptr, tmp_bytes, counting, head, heads, nsel, (int)S,
                                       s));
  int64_t n_heads = 0;
  FX_HIP(hipMemcpyAsync(&n_heads, nsel, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  FX_HIP(hipStreamSynchronize(s));

  FX_TRY(b_key.alloc(sizeof(uint32_t) * n_heads, s));
  FX_TRY(b_key2.alloc(sizeof(uint32_t) * n_heads, s));
  FX_TRY(b_val.alloc(sizeof(uint64_t) * n_heads, s));
  uint32_t *key = static_cast<uint32_t *>(b_key.ptr), *key2 = static_cast<uint32_t *>(b_key2.ptr);
  uint64_t *val = static_cast<uint64_t *>(b_val.ptr);
  if (hipMallocAsync((void **)&sp.runs, sizeof(uint64_t) * std::max<int64_t>(n_heads, 1), s) !=
      hipSuccess)
    return set_error(FURAX_ENOMEM, "superpixel runs: allocation failed");
  hipLaunchKernelGGL(k_run_make, dim3(grid_for(n_heads)), dim3(kBlock), 0, s, n_heads, S,
                     sp.log2P, sp.n_sp, heads, plane, key, val);
  FX_HIP(hipGetLastError());

  // stable sort of the runs by superpixel
  int end_bit = 1;
  while (((int64_t)1 << end_bit) <= sp.n_sp) ++end_bit;
  size_t sort_bytes = 0;
  FX_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, key, key2, val, sp.runs,
                                            (int)n_heads, 0, end_bit, s));
  DevBuf b_sort;
  FX_TRY(b_sort.alloc(sort_bytes, s));
  FX_HIP(hipcub::DeviceRadixSort::SortPairs(b_sort.ptr, sort_bytes, key, key2, val, sp.runs,
                                            (int)n_heads, 0, end_bit, s));

  // runs per superpixel -> chunk table (host)
  FX_TRY(b_cnt.alloc(sizeof(int64_t) * 2 * sp.n_sp, s));
  int64_t *first_d = static_cast<int64_t *>(b_cnt.ptr), *last_d = first_d + sp.n_sp;
  FX_TRY(zero_async(first_d, sizeof(int64_t) * 2 * sp.n_sp, s));
  hipLaunchKernelGGL(k_run_bounds, dim3(grid_for(n_heads)), dim3(kBlock), 0, s, n_heads, key2,
                     sp.n_sp, first_d, last_d);
  FX_HIP(hipGetLastError());
  std::vector<int64_t> fl(2 * sp.n_sp);
  FX_HIP(hipMemcpyAsync(fl.data(), first_d, sizeof(int64_t) * 2 * sp.n_sp, hipMemcpyDeviceToHost,
                        s));
  FX_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> hc(sp.n_sp);
  for (int64_t p = 0; p < sp.n_sp; ++p) hc[p] = fl[sp.n_sp + p] - fl[p];

  std::vector<SpChunk> ch;
  std::vector<int32_t> first(sp.n_sp + 1);
  sp.chunk_runs = !a.qb && sp.nside <= 512 ? kChunkRunsSmall : kChunkRunsMax;
  const int64_t cr = sp.chunk_runs;
  int64_t r = 0;
  for (int64_t p = 0; p < sp.n_sp; ++p) {
    first[p] = (int32_t)ch.size();
    for (int64_t c = 0; c < hc[p]; c += cr) {
      SpChunk k;
      k.r0 = fl[p] + c;
      k.nr = (int32_t)std::min<int64_t>(cr, hc[p] - c);
      k.sp = (int32_t)p;
      k.w = 0;
      k.s0 = 0;
      ch.push_back(k);
    }
    r += hc[p];
  }
  first[sp.n_sp] = (int32_t)ch.size();
  sp.n_runs = r;
  sp.n_chunks = (int64_t)ch.size();
  sp.n_values = n_values;
  // groups: each superpixel's chunks dealt into ceil(n / kChunksPerGroup)
  // groups of near-equal size, so one workgroup sums several chunks in LDS
  // and writes one partial for them
  const int64_t per_group = kChunksPerGroup;
  std::vector<int32_t> grp, first_grp(sp.n_sp + 1);
  for (int64_t p = 0; p < sp.n_sp; ++p) {
    first_grp[p] = (int32_t)grp.size();
    const int64_t nc = first[p + 1] - first[p];
    const int64_t ng = (nc + per_group - 1) / per_group;
    for (int64_t g = 0; g < ng; ++g) grp.push_back(first[p] + (int32_t)(nc * g / ng));
  }
  first_grp[sp.n_sp] = (int32_t)grp.size();
  sp.n_groups = (int64_t)grp.size();
  grp.push_back((int32_t)sp.n_chunks);
  if (hipMallocAsync((void **)&sp.chunks, sizeof(SpChunk) * std::max<int64_t>(sp.n_chunks, 1), s) !=
          hipSuccess ||
      hipMallocAsync((void **)&sp.groups, sizeof(int32_t) * (sp.n_groups + 1), s) !=
          hipSuccess ||
      hipMallocAsync((void **)&sp.sp_group, sizeof(int32_t) * (sp.n_sp + 1), s) != hipSuccess ||
      hipMallocAsync((void **)&sp.partial,
                     sizeof(double) * std::max<int64_t>(sp.n_groups, 1) * n_values *
                         ((int64_t)1 << sp.log2P),
                     s) != hipSuccess)
    return set_error(FURAX_ENOMEM, "superpixel chunk tables: allocation failed");
  if (sp.n_chunks)
    FX_HIP(hipMemcpyAsync(sp.chunks, ch.data(), sizeof(SpChunk) * sp.n_chunks,
                          hipMemcpyHostToDevice, s));
  FX_HIP(hipMemcpyAsync(sp.groups, grp.data(), sizeof(int32_t) * (sp.n_groups + 1),
                        hipMemcpyHostToDevice, s));
  FX_HIP(hipMemcpyAsync(sp.sp_group, first_grp.data(), sizeof(int32_t) * (sp.n_sp + 1),
                        hipMemcpyHostToDevice, s));
  if (sp.n_chunks) {
    hipLaunchKernelGGL(k_run_finalize, dim3((unsigned)sp.n_chunks), dim3(kFinalizeThreads), 0, s,
                       sp.runs, sp.chunks);
    FX_HIP(hipGetLastError());
    // each chunk's first position in the run-sorted sample order
    FX_HIP(hipMemcpyAsync(ch.data(), sp.chunks, sizeof(SpChunk) * sp.n_chunks,
                          hipMemcpyDeviceToHost, s));
    FX_HIP(hipStreamSynchronize(s));
    int64_t pos = 0;
    for (auto &c : ch) {
      c.s0 = (int32_t)pos;
      pos += c.w;
    }
    sp.n_sorted = pos;
    FX_HIP(hipMemcpyAsync(sp.chunks, ch.data(), sizeof(SpChunk) * sp.n_chunks,
                          hipMemcpyHostToDevice, s));
  }
  if (hipMallocAsync((void **)&sp.lab, sizeof(uint16_t) * std::max<int64_t>(sp.n_sorted, 1), s) !=
          hipSuccess ||
      (!a.qb && hipMallocAsync(&sp.psi, sizeof(T) * std::max<int64_t>(sp.n_sorted, 1), s) !=
                    hipSuccess))
    return set_error(FURAX_ENOMEM, "superpixel sample order: allocation failed");
  // detector order for the sample tiles of P: by the nested index of the
  // first sample, a walk along a space-filling curve, so that detectors a
  // tile takes together look at neighbouring pixels
  {
    DevBuf b_dkey;
    FX_TRY(b_dkey.alloc(sizeof(int32_t) * a.n_det, s));
    hipLaunchKernelGGL(k_det_keys, dim3((unsigned)((a.n_det + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, a.n_det, a.n_samp, plane, static_cast<int32_t *>(b_dkey.ptr));
    FX_HIP(hipGetLastError());
    std::vector<int32_t> dkey(a.n_det), perm(a.n_det);
    FX_HIP(hipMemcpyAsync(dkey.data(), b_dkey.ptr, sizeof(int32_t) * a.n_det,
                          hipMemcpyDeviceToHost, s));
    FX_HIP(hipStreamSynchronize(s));
    for (int64_t k = 0; k < a.n_det; ++k) perm[k] = (int32_t)k;
    std::stable_sort(perm.begin(), perm.end(),
                     [&dkey](int32_t x, int32_t y) { return dkey[x] < dkey[y]; });
    if (hipMallocAsync((void **)&sp.det_perm, sizeof(int32_t) * a.n_det, s) != hipSuccess)
      return set_error(FURAX_ENOMEM, "detector order: allocation failed");
    FX_HIP(hipMemcpyAsync(sp.det_perm, perm.data(), sizeof(int32_t) * a.n_det,
                          hipMemcpyHostToDevice, s));
    FX_HIP(hipStreamSynchronize(s));   // perm dies here
  }
  if (sp.n_chunks) {
    hipLaunchKernelGGL(k_sp_sort<T>, dim3((unsigned)sp.n_chunks), dim3(kFinalizeThreads), 0, s,
                       sp.runs,
                       sp.chunks, plane, a.psi, sp.log2P, sp.lab, static_cast<T *>(sp.psi));
    FX_HIP(hipGetLastError());
  }
  FX_HIP(hipStreamSynchronize(s));   // the host vectors die here
  return FURAX_OK;
}
template furax_status sp_build_runs<float>(SpPlan &, const PtArgs<float> &, const int32_t *,
                                           int32_t, hipStream_t);
template furax_status sp_build_runs<double>(SpPlan &, const PtArgs<double> &, const int32_t *,
                                            int32_t, hipStream_t);

// ---------------------------------------------------------------------------
// Per-chunk accumulation.
//
//   KIND 0 (P^T):  sums[0..2][l] += v (1, c, s),  v = g_k w_k tod[k,i];
//   KIND 1 (BJ):   sums[0..5][l] += w (1, c, s)^T (1, c, s) (upper triangle),
//                  w = g_k^2 w_k, and hits[l] += 1.
//
// The chunk's runs are concatenated into W sample slots; slot j belongs to
// the run r with pre[r] <= j < pre[r+1] (pre: the chunk-local exclusive prefix
// of run lengths, stored with each run by the plan builder).  Lanes take
// consecutive slots, so every lane is busy whatever the run lengths, and the
// loads stay coalesced along each run.  Each run's offset, detector constants
// and HWP phase are staged in LDS once per chunk.  The pixel offset inside the
// superpixel and the angle psi of each slot come from the plan's run-sorted
// copies (lab, psi_s), read contiguously; the TOD is read in place, along
// each run.
// ---------------------------------------------------------------------------
constexpr int kSpThreads = 512;
// Occupancy of the accumulation: with 512 runs per chunk the LDS below (the
// superpixel's sums, a HWP table for periods up to 256 samples, the run table)
// comes to ~50 KB, room for three workgroups per CU, and FP64 then takes two
// slot blocks per wave instead of four, whose wider values would otherwise
// take more registers than three workgroups leave (80 VGPRs with two).  FP64
// quaternion pointing takes two as well (108 VGPRs instead of 156: a second
// workgroup per CU).
template <typename T, bool QUAT, int NR>
constexpr int slot_batch() {
  return sizeof(T) == 8 && (QUAT || NR == kChunkRunsSmall) ? 2 : 4;
}
constexpr int kHwpPeriodMax = 256;            // tabulated HWP periods
constexpr int kHwpTable = kHwpPeriodMax + (int)kMaxRun;

template <int NR>
struct SpRunLds {
  int32_t det[NR], i0[NR];    // detector, first sample index
  int32_t pre[NR + 1];
  int32_t hwp0[NR];           // (first sample index) mod hwp_den
  double gw[NR], dpsi[NR];
};
template <int KIND, int NR>
struct SpLds;
template <int NR>
struct SpLds<0, NR> {
  uint8_t run_start[kSpThreads / 64][64];   // per wave: a run starts at this slot of the block
  double acc[3][kSpPix];
  union {
    double two_alpha[kHwpTable];
    double2 turn4a[kHwpPeriodMax];   // quaternion pointing: (cos, sin) 4 alpha for u < den
  };
  SpRunLds<NR> run;
};
template <int NR>
struct SpLds<1, NR> {
  uint8_t run_start[kSpThreads / 64][64];
  double acc[6][kSpPix];
  int32_t hits[kSpPix];
  union {
    double two_alpha[kHwpTable];
    double2 turn4a[kHwpPeriodMax];   // quaternion pointing: (cos, sin) 4 alpha for u < den
  };
  SpRunLds<NR> run;
};

// Last run r in [lo, hi) with pre[r] <= j (pre ascending, pre[lo] <= j).
__device__ __forceinline__ int32_t run_of(const int32_t *pre, int32_t lo, int32_t hi, int32_t j) {
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= j) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename T, int KIND, bool QUAT, int NR>
__global__ void __launch_bounds__(kSpThreads)
k_sp_accum(PtArgs<T> a, const T *__restrict__ tod, const double *__restrict__ w_det,
           const uint16_t *__restrict__ lab, const T *__restrict__ psi_s,
           const uint64_t *__restrict__ runs, const SpChunk *__restrict__ chunks,
           const int32_t *__restrict__ groups, int32_t log2P, double *__restrict__ partial) {
  __shared__ SpLds<KIND, NR> L;
  constexpr int NV = KIND == 0 ? 3 : 6;
  const int P = 1 << log2P;
  for (int l = threadIdx.x; l < P; l += kSpThreads) {
#pragma unroll
    for (int v = 0; v < NV; ++v) L.acc[v][l] = 0.0;
    if constexpr (KIND == 1) L.hits[l] = 0;
  }
  const bool table = a.hwp && a.hwp_den <= kHwpPeriodMax;
  // quaternion pointing with a HWP and no angle offsets: the weights' turn is
  // by 4 alpha alone, tabulated as its cosine and sine over one HWP period
  const bool qturn = QUAT && table && !a.dpsi;
  if (qturn) {
    for (int u = threadIdx.x; u < (int)a.hwp_den; u += kSpThreads) {
#pragma clang fp contract(off)
      const int64_t m = (a.hwp_num_mod * u) % a.hwp_den;
      const double frac = (double)m / (double)a.hwp_den;
      double sn, cs;
      sincos(2.0 * (2.0 * ((2.0 * kPi) * frac + a.hwp_phase0)), &sn, &cs);
      L.turn4a[u] = make_double2(cs, sn);
    }
  } else if (table) {
    // two_alpha[u] = 2 alpha for a sample index congruent to u mod den, for
    // u < den + kMaxRun, so that (phase of the run's first sample) + offset
    // inside the run indexes it without a modulo
    for (int u = threadIdx.x; u < (int)a.hwp_den + (int)kMaxRun; u += kSpThreads) {
#pragma clang fp contract(off)
      const int64_t m = (a.hwp_num_mod * (u % a.hwp_den)) % a.hwp_den;
      const double frac = (double)m / (double)a.hwp_den;
      L.two_alpha[u] = 2.0 * ((2.0 * kPi) * frac + a.hwp_phase0);
    }
  }
  // the group's chunks in turn, summed into the same LDS accumulators
  const int32_t c_lo = groups[blockIdx.x], c_hi = groups[blockIdx.x + 1];
  for (int32_t ci = c_lo; ci < c_hi; ++ci) {
    const SpChunk ch = chunks[ci];
    if (ci > c_lo) __syncthreads();   // every wave is done with the previous run table
    for (int r = threadIdx.x; r < ch.nr; r += kSpThreads) {
      const uint64_t w = runs[ch.r0 + r];
      const int64_t off = (int64_t)(w >> 24);
      const int64_t k = off / a.n_samp;
      const int64_t i0 = off - k * a.n_samp;
      L.run.pre[r] = (int32_t)(w & 0xffffff);
      L.run.hwp0[r] = table ? (int32_t)(i0 % a.hwp_den) : 0;
      L.run.det[r] = (int32_t)k;
      L.run.i0[r] = (int32_t)i0;
      const double g = a.gain ? a.gain[k] : 1.0;
      const double wk = w_det ? w_det[k] : 1.0;
      L.run.gw[r] = KIND == 0 ? g * wk : g * g * wk;
      L.run.dpsi[r] = a.dpsi ? a.dpsi[k] : 0.0;
    }
    if (threadIdx.x == 0) L.run.pre[ch.nr] = ch.w;
    __syncthreads();

    constexpr int kSlotBatch = slot_batch<T, QUAT, NR>();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int kWaves = kSpThreads / 64;
    // Each wave owns a contiguous range of 64-slot blocks and walks it with a
    // run cursor rb (the run holding the block's first slot); lane l looks at
    // the start of run rb + 1 + l, so a block's lanes see every run that can
    // start inside it.
    const int32_t nblk = (ch.w + 63) >> 6;
    const int32_t b0 = (int32_t)((int64_t)nblk * wave / kWaves);
    const int32_t b1 = (int32_t)((int64_t)nblk * (wave + 1) / kWaves);
    int32_t rb = b0 < b1 ? run_of(L.run.pre, 0, ch.nr, b0 * 64) : 0;
    for (int32_t blk = b0; blk < b1; blk += kSlotBatch) {
      int32_t run[kSlotBatch], lo[kSlotBatch], tt[kSlotBatch];
      int64_t sidx[kSlotBatch];
      bool in[kSlotBatch];
      T z[kSlotBatch], ps[kSlotBatch];
      Quat qb[QUAT ? kSlotBatch : 1], qd[QUAT ? kSlotBatch : 1];
#pragma unroll
      for (int b = 0; b < kSlotBatch; ++b) {
        const int32_t jb = (blk + b) * 64;
        const int32_t j = jb + lane;
        in[b] = blk + b < b1 && j < ch.w;
        // starts of runs rb+1 .. rb+64 relative to the block (>= 1: rb holds jb)
        const int32_t m = rb + 1 + lane;
        const int32_t st = m < ch.nr ? L.run.pre[m] - jb : 65;
        // this lane's run: rb + (number of those starts <= lane).  The lanes
        // mark the block slots where a run starts in the wave's row of LDS
        // flags, and one ballot of the flags gives every lane its count.  A
        // wave's LDS accesses complete in issue order; the wave-scope fences
        // keep the compiler from reordering or merging them.
        uint8_t *fl = L.run_start[wave];
        fl[lane] = 0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (st < 64) fl[st] = 1;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const uint64_t starts = __ballot(fl[lane] != 0);
        run[b] = rb + __popcll(starts & ((2ull << lane) - 1ull));
        rb += __popcll(__ballot(st <= 64));
        const int32_t jj = min(j, ch.w - 1);
        const int32_t r = min(run[b], ch.nr - 1);
        run[b] = r;
        tt[b] = jj - L.run.pre[r];                        // offset inside the run
        sidx[b] = (int64_t)L.run.det[r] * a.n_samp + (L.run.i0[r] + tt[b]);
        const int64_t sj = (int64_t)ch.s0 + jj;           // run-sorted position
        lo[b] = (int32_t)lab[sj];
        if constexpr (KIND == 0) z[b] = tod[sidx[b]];
        if constexpr (QUAT) {
          qb[b] = load_quat(a.qb, L.run.i0[r] + tt[b]);
          qd[b] = load_quat(a.qd, L.run.det[r]);
        } else {
          ps[b] = psi_s[sj];
        }
      }
#pragma unroll
      for (int b = 0; b < kSlotBatch; ++b) {
        if (!in[b] || (uint32_t)lo[b] >= (uint32_t)P) continue;
        const int32_t r = run[b];
        const int32_t t = tt[b];
        // psi_eff = psi + dpsi_k + 2 alpha_i, in the oracle's order (beta: the
        // part that does not come from the pointing)
        double two_a = 0.0;
        if (a.hwp && !qturn) {
          if (table) {
            two_a = L.two_alpha[L.run.hwp0[r] + t];
          } else {
            const int64_t i = (int64_t)L.run.i0[r] + t;
            two_a = 2.0 * hwp_alpha(i, a.hwp_num_mod, a.hwp_den, a.hwp_phase0);
          }
        }
        T c, sn;
        if constexpr (QUAT) {
          const QuatDir qdir = quat_dir(qmul(qb[b], qd[b]));
          if (qturn) {
            double c2, s2;
            quat_c2s2(qdir, c2, s2);
            const double2 tn = L.turn4a[(uint32_t)(L.run.hwp0[r] + t) % (uint32_t)a.hwp_den];
            turn_weights(c2, s2, (T)tn.x, (T)tn.y, c, sn);
          } else {
            double beta = a.dpsi ? L.run.dpsi[r] : 0.0;
            if (a.hwp) beta = beta + two_a;
            quat_weights(qdir, a.dpsi || a.hwp, beta, c, sn);
          }
        } else {
          double pe = (double)ps[b];
          if (a.dpsi) pe = pe + L.run.dpsi[r];
          if (a.hwp) pe = pe + two_a;
          weights(2.0 * pe, c, sn);
        }
        if constexpr (KIND == 0) {
          const T v = (T)L.run.gw[r] * z[b];
          atomicAdd(&L.acc[0][lo[b]], (double)v);
          atomicAdd(&L.acc[1][lo[b]], (double)(v * c));
          atomicAdd(&L.acc[2][lo[b]], (double)(v * sn));
        } else {
          const double w = L.run.gw[r];
          const double cd = (double)c, sd = (double)sn;
          const double wc = w * cd, ws = w * sd;
          atomicAdd(&L.acc[0][lo[b]], w);
          atomicAdd(&L.acc[1][lo[b]], wc);
          atomicAdd(&L.acc[2][lo[b]], ws);
          atomicAdd(&L.acc[3][lo[b]], wc * cd);
          atomicAdd(&L.acc[4][lo[b]], wc * sd);
          atomicAdd(&L.acc[5][lo[b]], ws * sd);
          atomicAdd(&L.hits[lo[b]], 1);
        }
      }
    }
  }
  __syncthreads();
  // partial[group][v][l]
  constexpr int NOUT = KIND == 0 ? 3 : 7;
  double *out = partial + (int64_t)blockIdx.x * NOUT * P;
  for (int l = threadIdx.x; l < P; l += kSpThreads) {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[(int64_t)v * P + l] = L.acc[v][l];
    if constexpr (KIND == 1) out[(int64_t)6 * P + l] = (double)L.hits[l];
  }
}

// Sum each superpixel's group partials (in group order) into the ring-ordered
// output: dst[c * cs + ring * ps] for c < nv, every pixel written once (0 on
// pixels no sample reaches).  With hits, the 7th partial goes to hits[ring].
__global__ void __launch_bounds__(kBlock) k_sp_reduce(int64_t npix, int32_t log2P, int32_t nv,
                                                      const double *__restrict__ partial,
                                                      const int32_t *__restrict__ sp_group,
                                                      const int32_t *__restrict__ n2r,
                                                      double *__restrict__ dst, int64_t cs,
                                                      int32_t ps, int32_t *__restrict__ hits) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int P = 1 << log2P;
  const int nout = hits ? nv + 1 : nv;
  for (int64_t n = (int64_t)blockIdx.x * kBlock + threadIdx.x; n < npix; n += stride) {
    const int64_t sp = n >> log2P;
    const int l = (int)(n & (P - 1));
    const int32_t c0 = sp_group[sp], c1 = sp_group[sp + 1];
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double h = 0.0;
    for (int32_t c = c0; c < c1; ++c) {
      const double *src = partial + (int64_t)c * nout * P + l;
      for (int v = 0; v < nv; ++v) acc[v] += src[(int64_t)v * P];
      if (hits) h += src[(int64_t)nv * P];
    }
    const int64_t r = n2r[n];
    for (int v = 0; v < nv; ++v) dst[v * cs + r * ps] = acc[v];
    if (hits) hits[r] = (int32_t)h;
  }
}

template <typename T, int KIND>
static void launch_sp_accum(const SpPlan &sp, const PtArgs<T> &a, const T *tod,
                            const double *w_det, hipStream_t s) {
  const dim3 grid((unsigned)sp.n_groups), blk(kSpThreads);
  const T *psi = static_cast<const T *>(sp.psi);
  if (a.qb)
    hipLaunchKernelGGL((k_sp_accum<T, KIND, true, kChunkRunsMax>), grid, blk, 0, s, a, tod, w_det,
                       sp.lab, psi, sp.runs, sp.chunks, sp.groups, sp.log2P, sp.partial);
  else if (sp.chunk_runs == kChunkRunsSmall)
    hipLaunchKernelGGL((k_sp_accum<T, KIND, false, kChunkRunsSmall>), grid, blk, 0, s, a, tod,
                       w_det, sp.lab, psi, sp.runs, sp.chunks, sp.groups, sp.log2P, sp.partial);
  else
    hipLaunchKernelGGL((k_sp_accum<T, KIND, false, kChunkRunsMax>), grid, blk, 0, s, a, tod,
                       w_det, sp.lab, psi, sp.runs, sp.chunks, sp.groups, sp.log2P, sp.partial);
}

template <typename T>
furax_status sp_transpose(const SpPlan &sp, const PtArgs<T> &a, const T *tod,
                          const double *w_det, double *q, MapLayout ql, hipStream_t s) {
  if (sp.n_chunks > 0) {
    launch_sp_accum<T, 0>(sp, a, tod, w_det, s);
    FX_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_sp_reduce, dim3(grid_for(sp.npix, 16384)), dim3(kBlock), 0, s, sp.npix,
                     sp.log2P, 3, sp.partial, sp.sp_group, sp.n2r, q, ql.cs, ql.ps,
                     (int32_t *)nullptr);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status sp_transpose<float>(const SpPlan &, const PtArgs<float> &, const float *,
                                          const double *, double *, MapLayout, hipStream_t);
template furax_status sp_transpose<double>(const SpPlan &, const PtArgs<double> &,
                                           const double *, const double *, double *, MapLayout,
                                           hipStream_t);

// Block-Jacobi blocks M6 [6][npix] and hits [npix]; needs a plan built with
// n_values = 7.
template <typename T>
furax_status sp_bj_build(const SpPlan &sp, const PtArgs<T> &a, const double *w_det, double *M6,
                         int32_t *hits, hipStream_t s) {
  if (sp.n_chunks > 0) {
    launch_sp_accum<T, 1>(sp, a, (const T *)nullptr, w_det, s);
    FX_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_sp_reduce, dim3(grid_for(sp.npix, 16384)), dim3(kBlock), 0, s, sp.npix,
                     sp.log2P, 6, sp.partial, sp.sp_group, sp.n2r, M6, sp.npix, 1, hits);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status sp_bj_build<float>(const SpPlan &, const PtArgs<float> &, const double *,
                                         double *, int32_t *, hipStream_t);
template furax_status sp_bj_build<double>(const SpPlan &, const PtArgs<double> &, const double *,
                                          double *, int32_t *, hipStream_t);

template <typename T>
furax_status sp_nest_plane(const SpPlan &sp, const PtArgs<T> &a, int32_t *plane, hipStream_t s) {
  const int64_t S = a.n_det * a.n_samp;
  hipLaunchKernelGGL(k_nest_plane<T>, dim3(grid_for(S)), dim3(kBlock), 0, s, a, sp.r2n, plane);
  FX_HIP(hipGetLastError());
  return FURAX_OK;
}
template furax_status sp_nest_plane<float>(const SpPlan &, const PtArgs<float> &, int32_t *,
                                           hipStream_t);
template furax_status sp_nest_plane<double>(const SpPlan &, const PtArgs<double> &, int32_t *,
                                            hipStream_t);

}  // namespace fx
