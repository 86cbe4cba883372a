// compress.hip -- HIP kernels of the ROIBIN-SZ compression path for gfx950.
//
// Launch sequence over a batch of frames (one launch per step for the whole
// batch; every kernel maps its flat work index to a frame with the prefix
// sums of the batch plan):
//   k_prep      one workgroup per frame: clear the histogram, check the peaks,
//               bucket them by band of segment rows.
//   k_bin       fused ROI mask + b x b background binning + prequantisation +
//               2D Lorenzo + code/outlier + histogram; one wave per tile
//               (segment of bin rows x column group of 64-column strips of a
//               panel), walking it row by row; the codes leave in a sparse
//               form (a zero-map and the bytes of nonzero residuals).
//   k_lorenzo_dims  Lorenzo dimensions 1 and 3: the residuals k_bin's 2D
//               predictor leaves to finish (row ends; the panel axis).
//   k_codebook  one workgroup per frame: Huffman lengths and canonical codes.
//   k_count     one wave per 4096-symbol chunk: its codes gathered into a
//               mask and compacted bytes, its bits and outliers; then one
//               wave per peak: ROI window payload, bit copies.
//   k_scan      one workgroup per frame: chunk bit and outlier offsets.
//   k_encode    one workgroup per run of chunks: bit-packing and outlier
//               indices at the offsets k_scan computed.
//   k_roi_classes, k_roi_book, k_roi_count, k_roi_scan  coded ROI: class
//               histogram, class code, window bits and offsets.
//   k_run_count, k_run_scan  run stage: each chunk's Rice parameter and run
//               bits, then their offsets.
//   k_tail      one workgroup per frame: sizes, capacity, header, chunk
//               boundary words, outlier sections, coded ROI and run section
//               tables.
//   k_roi_pack, k_run_pack  the coded ROI bits and the run codes.
#include <algorithm>

#include <type_traits>

#include "rsz_internal.h"

namespace rsz {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The n lowest bits (n <= 64).
__device__ __forceinline__ uint64_t low_bits(uint32_t n) {
  return n >= 64 ? ~0ull : (1ull << n) - 1ull;
}

// Frame owning flat work item `item`: the largest f with prefix[f] <= item.
__device__ __forceinline__ uint32_t find_frame(const uint32_t *prefix, uint32_t nframes,
                                               uint32_t item) {
  uint32_t lo = 0, hi = nframes;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (prefix[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int32_t load_status(const FrameState *st) {
  return __hip_atomic_load(&st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_status(FrameState *st, int32_t code) {
  atomicCAS(&st->status, (int32_t)RSZ_OK, code);
}

// Exclusive scan over the 256 threads of a workgroup; `total` gets the sum.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *s_tmp, T &total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) s_tmp[wave] = x;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const T t = s_tmp[i];
    if (i < wave) off += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return off + x - v;
}

// ----------------------------------------------------------------- k_prep

// Keys of the band counting sort held in LDS per pass over the peaks.
constexpr uint32_t kPrepKeys = 4096;

__global__ __launch_bounds__(256) void k_prep(BatchPlan bp) {
  const uint32_t f = blockIdx.x;
  const FramePlan &fp = bp.frames[f];
  FrameState *st = fp.st;
  __shared__ int s_bad;
  __shared__ uint32_t s_tmp[4];
  __shared__ uint32_t s_cnt[kPrepKeys];
  // this frame's entries of the frame tables (a later kernel finds a
  // workgroup's or peak's frame with one load instead of a search); written
  // for every frame, failed or not
  for (uint32_t i = bp.tile_prefix[f] + threadIdx.x; i < bp.tile_prefix[f + 1]; i += 256)
    bp.tile_frame[i] = f;
  for (uint32_t i = bp.unit_prefix[f] + threadIdx.x; i < bp.unit_prefix[f + 1]; i += 256)
    bp.unit_frame[i] = f;
  for (uint32_t i = bp.peak_prefix[f] + threadIdx.x; i < bp.peak_prefix[f + 1]; i += 256)
    bp.peak_frame[i] = f;
  {
    // k_count workgroup w takes chunks [4 w, 4 w + 4) of the batch: its
    // entry belongs to the frame holding chunk 4 w
    const uint32_t c0 = bp.chunk_prefix[f], c1 = bp.chunk_prefix[f + 1];
    for (uint32_t w = (c0 + kWaves - 1) / kWaves + threadIdx.x; w < (c1 + kWaves - 1) / kWaves;
         w += 256)
      bp.count_frame[w] = make_uint2(f, w * kWaves - c0);
  }
  for (int i = threadIdx.x; i < kNumSym; i += 256) st->hist[i] = 0;
  if (fp.roi_coding)
    for (int i = threadIdx.x; i < kNumSym; i += 256) fp.roi_hist[i] = 0;
  if (threadIdx.x == 0) {
    s_bad = 0;
    st->status = fp.init_status;
    st->n_out = 0;
    st->T = 0;
    st->total = 0;
    st->Troi = 0;
  }
  if (fp.init_status != RSZ_OK) return;
  // the quantiser's reciprocals, computed here rather than carried in the
  // plan (the device divide and multiply are the IEEE operations, so the
  // bits equal the host's): inv[n] = 1 / (n * 2eb), inv[0] = 0
  if (threadIdx.x <= 64)
    st->inv[threadIdx.x] = threadIdx.x ? 1.0 / ((double)threadIdx.x * fp.step) : 0.0;
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < fp.npeaks; k += 256) {
    const int32_t pa = fp.peaks[3 * k], r = fp.peaks[3 * k + 1], c = fp.peaks[3 * k + 2];
    if (pa < 0 || (uint32_t)pa >= fp.P || r < 0 || (uint32_t)r >= fp.H || c < 0 ||
        (uint32_t)c >= fp.W)
      s_bad = 1;
  }
  __syncthreads();
  if (s_bad) {
    if (threadIdx.x == 0) st->status = RSZ_ERR_PEAK;
    return;
  }
  // Counting sort of the peaks by band (panel, segment of raw rows), so that
  // a k_bin wave scans only the bands its rows can touch.  Keys are taken in
  // passes of kPrepKeys; the order inside a band is irrelevant (the mask is
  // a union).
  const uint32_t nkeys = fp.P * fp.segs;
  const uint32_t band = fp.TH * fp.b;
  uint32_t carry = 0;
  for (uint32_t k0 = 0; k0 < nkeys; k0 += kPrepKeys) {
    const uint32_t kn = min(kPrepKeys, nkeys - k0);
    for (uint32_t i = threadIdx.x; i < kPrepKeys; i += 256) s_cnt[i] = 0;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < fp.npeaks; k += 256) {
      const uint32_t key = (uint32_t)fp.peaks[3 * k] * fp.segs + (uint32_t)fp.peaks[3 * k + 1] / band;
      if (key - k0 < kn) atomicAdd(&s_cnt[key - k0], 1u);
    }
    __syncthreads();
    // exclusive scan, 16 consecutive keys per thread
    constexpr int E = kPrepKeys / 256;
    uint32_t v[E], sum = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      v[e] = s_cnt[threadIdx.x * E + e];
      sum += v[e];
    }
    uint32_t tot;
    uint32_t run = carry + block_exclusive_scan<uint32_t>(sum, s_tmp, tot);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t i = threadIdx.x * E + e;
      s_cnt[i] = run;
      if (i < kn) fp.bstart[k0 + i] = run;
      run += v[e];
    }
    carry += tot;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < fp.npeaks; k += 256) {
      const uint32_t r = (uint32_t)fp.peaks[3 * k + 1], c = (uint32_t)fp.peaks[3 * k + 2];
      const uint32_t key = (uint32_t)fp.peaks[3 * k] * fp.segs + r / band;
      if (key - k0 < kn) fp.bucket[atomicAdd(&s_cnt[key - k0], 1u)] = r << 16 | c;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) fp.bstart[nkeys] = fp.npeaks;
}

// Peaks whose window can touch raw rows [R0, R0 + mrows) of panel p: the
// bucket range of the bands holding rows R0 + h - w + 1 .. R0 + mrows - 1 + h
// (h = w/2), clipped to the panel.
__device__ __forceinline__ void peak_range(const FramePlan &fp, uint32_t p, int64_t R0, int mrows,
                                           uint32_t &k0, uint32_t &k1) {
  const int64_t hw = fp.w / 2;
  const int64_t lo = max(R0 + hw - (int64_t)fp.w + 1, (int64_t)0);
  const int64_t hi = min(R0 + mrows - 1 + hw, (int64_t)fp.H - 1);
  k0 = k1 = 0;
  if (lo > hi) return;
  const int64_t band = (int64_t)fp.TH * fp.b;
  k0 = fp.bstart[(size_t)p * fp.segs + (uint32_t)(lo / band)];
  k1 = fp.bstart[(size_t)p * fp.segs + (uint32_t)(hi / band) + 1];
}

// ------------------------------------------------------------------ k_roi

// ROI payload (Sec. IV-A: each peak's w x w window as a buffer, a constant
// fill outside the panel), the work items of k_count past its chunks: one
// wave per peak, flat over the window's w*w
// pixels, kRoiSlots pixels per lane loaded before any is stored (so a
// window's loads are in flight together: the stores could alias the frame as
// far as the compiler knows).  Window row u = e / w from a multiply-high by
// floor((2^32 - 1) / w) + 1, exact for e < w^2 since w^3 < 2^32.
constexpr uint32_t kRoiSlots = 8;
__device__ __forceinline__ void roi_copy(const BatchPlan &bp, uint32_t kg) {
  const int lane = threadIdx.x & 63;
  if (kg >= bp.total_peaks) return;
  const uint32_t f = bp.peak_frame[kg];
  const FramePlan &fp = bp.frames[f];
  if (fp.roi_coding || load_status(fp.st) != RSZ_OK) return;
  // the section lies inside the output buffer (a stream that does not fit
  // it altogether gets RSZ_ERR_CAPACITY from k_tail, and its bytes are
  // unspecified)
  if (fp.off_roi + 4ull * fp.npeaks * fp.w * fp.w > fp.out_cap) return;
  const uint32_t k = kg - bp.peak_prefix[f];
  const int64_t pa = fp.peaks[3 * k], r = fp.peaks[3 * k + 1], c = fp.peaks[3 * k + 2];
  if (pa < 0 || pa >= fp.P) return;
  const uint32_t w = fp.w, ww = w * w, M = 0xFFFFFFFFu / w + 1u;
  const int64_t h = w / 2, H = fp.H, W = fp.W;
  uint32_t *dst = (uint32_t *)(fp.out + fp.off_roi) + (size_t)k * ww;
  const float *src = fp.frame + (size_t)pa * H * W;
  for (uint32_t e0 = 0; e0 < ww; e0 += 64 * kRoiSlots) {
    uint32_t val[kRoiSlots];
#pragma unroll
    for (uint32_t t = 0; t < kRoiSlots; ++t) {
      const uint32_t e = e0 + 64 * t + lane;
      const uint32_t u = __umulhi(e, M), v = e - u * w;
      const int64_t i = r - h + u, j = c - h + v;
      val[t] = 0u;
      if (e < ww && i >= 0 && i < H && j >= 0 && j < W) val[t] = __float_as_uint(*gm(src + i * W + j));
    }
#pragma unroll
    for (uint32_t t = 0; t < kRoiSlots; ++t) {
      const uint32_t e = e0 + 64 * t + lane;
      if (e < ww) *gm(dst + e) = val[t];
    }
  }
}

// ------------------------------------------------------------------ k_bin

// Histogram update: the zero-residual code 512 is counted from a lane mask
// into a wave-uniform total that is added once at the end; every other code
// is one LDS atomic of its lane (cheaper, measured, than one add per
// distinct code of the wave, which takes up to 64 rounds on a wide residual
// distribution).  vmask: the lanes holding a bin.
__device__ __forceinline__ void wave_histogram(uint32_t code, uint64_t vmask, uint32_t *hist,
                                               uint32_t &c512) {
  const int lane = threadIdx.x & 63;
  c512 += (uint32_t)__builtin_popcountll(
      __builtin_amdgcn_uicmp(code, (uint32_t)kRadius, 32 /* eq */) & vmask);
  uint64_t pending = __builtin_amdgcn_uicmp(code, (uint32_t)kRadius, 33 /* ne */) & vmask;
  if ((pending >> lane) & 1u) atomicAdd(&hist[code], 1u);
}

// The same from the wave's ballot m of the lanes whose residual is not 0
// (code other than 512): the others are counted from the mask alone.
__device__ __forceinline__ void wave_histogram_nz(uint32_t code, uint64_t m, uint64_t vmask,
                                                  uint32_t *hist, uint32_t &c512) {
  const int lane = threadIdx.x & 63;
  c512 += (uint32_t)__builtin_popcountll(vmask & ~m);
  if ((m >> lane) & 1u) atomicAdd(&hist[code], 1u);
}

// Value of lane-1 (lane 0 gets `first`): the left neighbour along a row.
__device__ __forceinline__ int32_t from_left(int32_t v, int32_t first) {
  return __builtin_amdgcn_update_dpp(first, v, 0x138 /* wave_shr:1 */, 0xF, 0xF, false);
}

// Codes travel from the binning kernel to the encoder as one byte per bin:
// r + 128 for |r| <= 127, else 0 with the bin's residual in rbuf (codes
// 1..384 and 640..1023, and the outliers).
__device__ __forceinline__ uint32_t code_byte(int32_t r) {
  return (uint32_t)(r + 127) < 255u ? (uint32_t)(r + 128) : 0u;
}
__device__ __forceinline__ uint32_t code_from_residual(int32_t r) {
  return (r > -kRadius && r < kRadius) ? (uint32_t)(r + kRadius) : 0u;
}

// q = rint(S / den) with den = n*2eb and S/den correctly rounded.  Fast path:
// t1 = S * inv with inv = 1/den correctly rounded differs from the exact
// quotient x by at most (2u + u^2)|x| and from the rounded quotient by at
// most 3.01u|x| (u = 2^-53).  When |t1 - rint(t1)| < 0.5 - 2^-20, t1 lies
// more than 2^-20 from the half-integers around rint(t1); for |x| < 2^31 the
// rounded quotient is then within 2^-22 of t1, on the same side, and rounds
// to the same integer.  Larger |x| make both results exceed 2^28 - 1 (a range
// error either way), and NaN/Inf fail the test.  Otherwise: the divide.
__device__ __forceinline__ int32_t quantize(double S, uint32_t n, double step, double inv,
                                            bool &range_err) {
  if (n == 0) return 0;
  const double t1 = S * inv;
  double t = rint(t1);
  if (!(fabs(t1 - t) < 0.5 - 0x1p-20)) t = rint(S / ((double)n * step));
  if (!(fabs(t) <= kQMax)) {
    range_err = true;
    return 0;
  }
  return (int32_t)t;
}

// Raw pixels of one bin, loaded with clamped (always valid) addresses; the
// inclusion of each pixel is decided after the load.
template <int BB>
struct BinPix {
  float v[BB ? BB : 8][BB ? BB : 8];
  uint32_t m[BB ? BB : 8];   // mask word(s) of each raw row (shifted in reduce)
};

template <int BB, bool VEC, bool BG>
__device__ __forceinline__ void load_bin(BinPix<BB> &px, const float *__restrict__ fr, uint32_t H,
                                         uint32_t W, int b, uint32_t I, uint32_t Jc,
                                         const uint32_t *mask, int64_t R0, int wpr, int mword) {
  constexpr int NB = BB ? BB : 8;
#pragma unroll
  for (int di = 0; di < NB; ++di) {
    if (!BB && di >= b) break;
    const uint32_t i = min(I * b + di, H - 1);
    const float *row = fr + (size_t)i * W;
    const uint32_t j0 = Jc * b;
    if constexpr (VEC && BB == 2) {
      const f32x2 x = *gm((const f32x2 *)(row + j0));
      px.v[di][0] = x.x;
      px.v[di][1] = x.y;
    } else if constexpr (VEC && BB == 4) {
      const f32x4 x = *gm((const f32x4 *)(row + j0));
      px.v[di][0] = x.x;
      px.v[di][1] = x.y;
      px.v[di][2] = x.z;
      px.v[di][3] = x.w;
    } else {
#pragma unroll
      for (int dj = 0; dj < NB; ++dj) {
        if (!BB && dj >= b) break;
        px.v[di][dj] = *gm(row + min(j0 + dj, W - 1));
      }
    }
    if constexpr (BG) {
      // the word holding this lane's first bit; for b not dividing 32 the
      // row's bits may continue in the next word (read in row_bits)
      px.m[di] = mask[(int64_t)(i - R0) * wpr + mword];
    } else {
      px.m[di] = 0u;
    }
  }
}

// Mask bits of bin row di: bit dj = pixel J*b+dj is inside a window.
template <int BB, bool BG>
__device__ __forceinline__ uint32_t row_bits(const BinPix<BB> &px, int di, int b, int mshift,
                                             const uint32_t *mask, int64_t rowoff, int mword) {
  if constexpr (!BG) {
    return 0u;
  } else if constexpr (BB == 1 || BB == 2 || BB == 4 || BB == 8) {
    return px.m[di] >> mshift;
  } else {
    // straddling case: combine with the next word when the bits cross it
    const uint32_t lo = px.m[di] >> mshift;
    const uint32_t hi = (mshift + b > 32) ? (mask[rowoff + mword + 1] << (32 - mshift)) : 0u;
    return lo | hi;
  }
}

// Sum in raster order over the included pixels (fp64, from +0.0), count, and
// quantise.
template <int BB, bool BG>
__device__ __forceinline__ int32_t reduce_bin(const BinPix<BB> &px, uint32_t H, uint32_t W, int b,
                                              uint32_t I, uint32_t J, double step,
                                              const double *inv, bool &range_err, double &S_out,
                                              uint32_t &n_out, int mshift, const uint32_t *mask,
                                              int64_t R0, int wpr, int mword) {
  constexpr int NB = BB ? BB : 8;
  double S = 0.0;
  uint32_t n = 0;
#pragma unroll
  for (int di = 0; di < NB; ++di) {
    if (!BB && di >= b) break;
    const bool rowv = I * b + di < H;
    const int64_t rowoff = (int64_t)(min(I * b + di, H - 1) - R0) * wpr;
    const uint32_t mb = row_bits<BB, BG>(px, di, b, mshift, mask, rowoff, mword);
#pragma unroll
    for (int dj = 0; dj < NB; ++dj) {
      if (!BB && dj >= b) break;
      const bool inc = rowv && (J * b + dj < W) && !((mb >> dj) & 1u);
      const double y = S + (double)px.v[di][dj];
      S = inc ? y : S;
      n += inc ? 1u : 0u;
    }
  }
  S_out = S;
  n_out = n;
  return quantize(S, n, step, inv[n], range_err);
}

// Vector path (b = 2 or 4 with W % b == 0, rows 8- or 16-byte aligned): a
// lane's bin row is one float2/float4 load at a 32-bit byte offset from a
// wave-uniform row pointer, and the b x b pixels reduce branch-free.
template <int BB, bool BG>
__device__ __forceinline__ void load_vec(BinPix<BB> &px, const float *__restrict__ fr, uint32_t H,
                                         uint32_t W, uint32_t I, uint32_t lofs,
                                         const uint32_t *mlane, int64_t R0, int wpr) {
#pragma unroll
  for (int di = 0; di < BB; ++di) {
    const uint32_t i = min(I * BB + di, H - 1);
    const char *row = (const char *)(fr + (size_t)i * W);
    if constexpr (BB == 2) {
      const f32x2 x = *gm((const f32x2 *)(row + lofs));
      px.v[di][0] = x.x;
      px.v[di][1] = x.y;
    } else {
      const f32x4 x = *gm((const f32x4 *)(row + lofs));
      px.v[di][0] = x.x;
      px.v[di][1] = x.y;
      px.v[di][2] = x.z;
      px.v[di][3] = x.w;
    }
    px.m[di] = BG ? mlane[(int)(i - R0) * wpr] : 0u;
  }
}

// The fp64 raster-order sum of the included pixels, their count and q.  An
// excluded pixel enters as -0.0, which leaves any sum unchanged (x + -0 = x
// for every x, zeros included), and the sum starts from the first pixel
// rather than from +0.0.  Both can change only the sign of a zero sum, never
// q; with `exact_S` a final +0.0 restores the sum from +0.0 bit for bit (a
// sum from +0.0 is never -0.0).  rowbits: the in-panel pixels of the bin,
// raster bit order (wave-uniform).
template <int BB, bool BG>
__device__ __forceinline__ int32_t reduce_vec(const BinPix<BB> &px, uint32_t rowbits, int mshift,
                                              const double *inv, double step, bool &range_err,
                                              bool exact_S, double &S_out, uint32_t &n_out) {
  uint32_t inc = rowbits;
  if constexpr (BG) {
    uint32_t mb = 0;
#pragma unroll
    for (int di = 0; di < BB; ++di) mb |= __builtin_amdgcn_ubfe(px.m[di], mshift, BB) << (di * BB);
    inc &= ~mb;
  }
  double S = 0.0;
#pragma unroll
  for (int k = 0; k < BB * BB; ++k) {
    // all ones for an included pixel, else zero: keep its bits or take -0.0
    const uint32_t keep = (uint32_t)__builtin_amdgcn_sbfe((int)inc, k, 1);
    const uint32_t xb = (__float_as_uint(px.v[k / BB][k % BB]) & keep) | (0x80000000u & ~keep);
    const double x = (double)__uint_as_float(xb);
    S = k == 0 ? x : S + x;
  }
  const uint32_t n = __builtin_popcount(inc);
  if (exact_S) {
    S_out = S + 0.0;
    n_out = n;
  }
  // n == 0: inv[0] = 0 and S = -0.0, so t1 = 0 and q = 0 without a branch
  const double t1 = S * inv[n];
  double t = rint(t1);
  if (!(fabs(t1 - t) < 0.5 - 0x1p-20)) t = rint(S / ((double)n * step));
  if (!(fabs(t) <= kQMax)) {
    range_err = true;
    return 0;
  }
  return (int32_t)t;
}

// Wave mask of one segment: raw rows [R0, R0 + mrows) x columns [C0, C0 +
// 32*wpr) of panel p, bit set where a pixel lies in some peak's window.
__device__ __forceinline__ void build_mask(const FramePlan &fp, uint32_t p, uint32_t *mask,
                                           int64_t R0, int mrows, int64_t C0, int wpr) {
  const int lane = threadIdx.x & 63;
  uint32_t pk0, pk1;
  peak_range(fp, p, R0, mrows, pk0, pk1);
  const int64_t hw = fp.w / 2, wwin = fp.w;
  for (int i = lane; i < mrows * wpr; i += 64) mask[i] = 0u;
  wave_sync();
  for (uint32_t k = pk0 + lane; k < pk1; k += 64) {
    const uint32_t rc = fp.bucket[k];
    const int64_t r = rc >> 16, c = rc & 0xFFFFu;
    const int64_t rlo = max(r - hw, max(R0, (int64_t)0));
    const int64_t rhi = min(r - hw + wwin, min(R0 + mrows, (int64_t)fp.H));
    const int64_t clo = max(c - hw, max(C0, (int64_t)0));
    const int64_t chi = min(c - hw + wwin, min(C0 + 32 * (int64_t)wpr, (int64_t)fp.W));
    if (rlo >= rhi || clo >= chi) continue;
    const int b0 = (int)(clo - C0), b1 = (int)(chi - 1 - C0);
    for (int64_t i = rlo; i < rhi; ++i) {
      uint32_t *mr = mask + (i - R0) * wpr;
      for (int wd = b0 >> 5; wd <= (b1 >> 5); ++wd) {
        const int lo = max(b0 - wd * 32, 0), hi = min(b1 - wd * 32, 31);
        const uint32_t m = (hi == 31 ? 0xFFFFFFFFu : ((1u << (hi + 1)) - 1u)) & ~((1u << lo) - 1u);
        atomicOr(&mr[wd], m);
      }
    }
  }
  wave_sync();
}

// Sparse codes of one binning tile, staged so that they reach HBM as whole
// cache lines: the tile's zero-map words and byte counts (one per tile row
// and strip) collect in lanes of a few registers and are stored when the
// tile ends; its code bytes other than 128 go through an LDS ring, written
// 256 at a time.  Partial lines written a few bytes at a time, as a row's
// scattered stores would be, cost far more than the bytes they carry.
constexpr uint32_t kZbRing = 512;
constexpr uint32_t kZbFlush = 256;   // <= kZbRing - 4 * 64: a row adds at most 256
struct SparseStage {
  uint8_t zb[kZbRing];
};

// Writes the ring's bytes [from, to) of the tile (from a multiple of 8, both
// within kZbRing of each other) to zb, 8 bytes a lane; the last 8-byte group
// may carry bytes past `to` (the tile's region holds whole groups).
__device__ __forceinline__ void flush_zb(const SparseStage &stg, uint8_t *zb, uint32_t from,
                                         uint32_t to) {
  const int lane = threadIdx.x & 63;
  for (uint32_t o = from + 8u * lane; o < to; o += 512u)
    *gm((u32x2 *)(zb + o)) = *(const u32x2 *)(stg.zb + (o & (kZbRing - 1)));
}

// Strips of a row whose loads are issued together.
template <int BB>
constexpr int strips_in_flight() {
  return BB == 1 || BB == 2 ? 4 : (BB == 4 ? 2 : 1);
}

// One wave's tile: bin rows [I0, I1) of segment `seg` x the strips of 64 bin
// columns [S0, S0 + ns) of column group `cg` of panel p, walked row by row.
// The Lorenzo predictor of the tile's first row and first column reads the q
// of bin row I0 - 1 and bin column J0 - 1, owned by neighbouring tiles: both
// are recomputed here from the frame (same loads, same sums).
// Dimension 2 finishes every residual here.  Dimension 1 takes r = q - q_left
// along the row; the first bin of a row follows the last bin of the row
// before, which a tile spanning the whole row holds (the halo row for its
// first row).  Where the predecessor lies elsewhere -- the first row of a
// panel, every row of a panel split into column groups -- the first bin gets
// r = q here and k_lorenzo_dims corrects it with the q of the row before's
// last bin, kept in qedge.  Dimension 3 leaves the panel's 2D residual for
// k_lorenzo_dims to difference across panels, and counts no histogram here.
template <int BB, bool VEC, bool BG, bool DEBUG, int DIM>
__device__ __forceinline__ void bin_tile(const FramePlan &fp, uint32_t p, uint32_t seg,
                                         uint32_t cg, uint32_t *hist, uint32_t *mask,
                                         const double *inv, SparseStage *stg) {
  constexpr int G = strips_in_flight<BB>();
  constexpr int NS = group_strips(BB);
  const int lane = threadIdx.x & 63;
  const int b = BB ? BB : (int)fp.b;
  const uint32_t H = fp.H, W = fp.W, Hb = fp.Hb, Wb = fp.Wb;
  const uint32_t S0 = cg * fp.gstrips;
  const int ns = (int)min(fp.gstrips, fp.nstrips - S0);
  const uint32_t J0 = S0 * 64;
  // the mask starts one word left of the group when there is a halo column
  const int lw = cg > 0 ? 1 : 0;
  const int64_t Cm = (int64_t)J0 * b - 32 * lw;
  const int wpr = 2 * b * ns + lw;
  const uint32_t I0 = seg * fp.TH, I1 = min(I0 + fp.TH, Hb);
  const int64_t R0 = (int64_t)I0 * b - b;
  const int mrows = (int)(I1 - I0 + 1) * b;
  const float *fr = fp.frame + (size_t)p * H * W;
  const double step = fp.step;
  const size_t gbase = (size_t)p * Hb * Wb;
  uint8_t *codes = fp.codes2 + gbase;
  int32_t *rbuf = fp.rbuf2 + gbase;
  bool range_err = false;
  uint32_t c512 = 0;
  double Sd;
  uint32_t nd;
  const uint32_t dim = DIM ? (uint32_t)DIM : fp.dim;
  // sparse codes (dimensions 1 and 2): the tile's entries and byte region
  const bool sparse = DIM ? DIM != 3 : fp.sparse != 0;
  const uint32_t tix = (p * fp.cgs + cg) * fp.segs + seg;
  const uint32_t gsl = fp.gstrips;   // strips of a column group
  uint32_t zcount = 0, zflushed = 0;
  // entry (strip s, tile row i) sits in lane (s & 1) * 32 + i of pair s >> 1
  uint32_t zmlo[2] = {0u, 0u}, zmhi[2] = {0u, 0u}, zpv[2] = {0u, 0u};
  if (BG || (DEBUG && fp.dbg_mask)) {
    build_mask(fp, p, mask, R0, mrows, Cm, wpr);
    if (DEBUG && fp.dbg_mask) {
      // this group's words of the full-width mask rows (J0*b is a multiple of 32)
      const uint32_t wprg = (W + 31) / 32;
      const uint32_t wd0 = J0 * b / 32;
      const int64_t nwd = min(2 * b * ns, (int)(wprg - wd0));
      const int64_t rs = (int64_t)I0 * b, re = min((int64_t)I1 * b, (int64_t)H);
      for (int64_t e = lane; e < (re - rs) * nwd; e += 64) {
        const int64_t i = rs + e / nwd, wd = e % nwd;
        fp.dbg_mask[((size_t)p * H + i) * wprg + wd0 + wd] = mask[(i - R0) * wpr + lw + wd];
      }
    }
  }
  // halo column: lane i holds q of bin (I0 - 1 + i, J0 - 1), 0 outside the
  // panel; its pixels sit in the last b bits of mask word 0
  int32_t q_left = 0;
  if (cg > 0) {
    const int64_t Ih = (int64_t)I0 - 1 + lane;
    const bool hv = Ih >= 0 && Ih < (int64_t)I1;
    const uint32_t Ic = (uint32_t)min(max(Ih, (int64_t)0), (int64_t)I1 - 1);
    BinPix<BB> px;
    load_bin<BB, VEC, BG>(px, fr, H, W, b, Ic, J0 - 1, mask, R0, wpr, 0);
    bool herr = false;
    const int32_t qh = reduce_bin<BB, BG>(px, H, W, b, Ic, J0 - 1, step, inv, herr, Sd, nd,
                                          32 - b, mask, R0, wpr, 0);
    q_left = hv ? qh : 0;
    range_err |= hv && herr;
  }
  // column of strip s for this lane and its mask word; idle lanes (past the
  // panel) load the last column, which stays inside the frame
#define RSZ_JC(s) ((J0 + (s) * 64 + lane) < Wb ? (J0 + (s) * 64 + lane) : Wb - 1)
#define RSZ_MW(jc) ((int)((((jc) - J0) * b + 32 * lw) >> 5))
  int32_t q_up[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    q_up[s] = 0;
    if (I0 > 0 && s < ns) {
      const uint32_t jc = RSZ_JC(s);
      BinPix<BB> px;
      load_bin<BB, VEC, BG>(px, fr, H, W, b, I0 - 1, jc, mask, R0, wpr, RSZ_MW(jc));
      const int32_t qh = reduce_bin<BB, BG>(px, H, W, b, I0 - 1, J0 + s * 64 + lane, step, inv,
                                            range_err, Sd, nd, (int)((jc * b) & 31), mask, R0,
                                            wpr, RSZ_MW(jc));
      q_up[s] = J0 + s * 64 + lane < Wb ? qh : 0;
    }
  }
  uint64_t vmask[NS];   // lanes of strip s inside the panel
#pragma unroll
  for (int s = 0; s < NS; ++s) vmask[s] = __builtin_amdgcn_uicmp(J0 + s * 64 + lane, Wb, 36 /* ult */);
  // ql_up[s]: left neighbours of the row above (row I0 - 1 to start)
  int32_t ql_up[NS];
  {
    int32_t lft = __builtin_amdgcn_readlane(q_left, 0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      ql_up[s] = 0;
      if (s < ns) {
        ql_up[s] = from_left(q_up[s], lft);
        lft = __builtin_amdgcn_readlane(q_up[s], 63);
      }
    }
  }
  // dim 1: the tile holds the last bin of each row (last column group); if it
  // spans whole rows, that bin is the raster predecessor of the next row's
  // first bin.  lastq: q of the last bin of the row above (the halo row to
  // start).
  const bool last_group = J0 + (uint32_t)ns * 64 >= Wb;
  const bool whole_rows = J0 == 0 && last_group;
  const int lastlane = (int)((Wb - 1) & 63);
  int32_t lastq = 0;
  if (dim == 1 && whole_rows) {
    int32_t v = q_up[0];
#pragma unroll
    for (int s = 1; s < NS; ++s)
      if (s == ns - 1) v = q_up[s];
    lastq = __builtin_amdgcn_readlane(v, lastlane);
  }
  // A panel row whose last strip holds only a few bins (CSPAD at b = 2: 194
  // = 3 * 64 + 2) would spend a whole strip's work per row on them.  When
  // the group's last strip has rem bins and rem * TH <= 64, its bins of all
  // the tile's rows are done after the row loop in one packed vector (lane =
  // tile row * rem + column), their left neighbours kept per row in qlast.
  // Dimension 1 needs each row's last q before the next row, so it keeps
  // the unpacked strip.
  const uint32_t rem = Wb - (J0 + 64 * (uint32_t)(ns - 1));
  const bool packed = VEC && dim != 1 && last_group && ns >= 2 && rem * fp.TH <= 64;
  const int nsr = packed ? ns - 1 : ns;   // strips done row by row
  int32_t qlast = 0;                      // lane i: q of the row loop's last bin of tile row i
  int32_t qhl = 0;                        // q of bin (I0 - 1, last column of the row loop)
  if (packed) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (s == nsr - 1) qhl = __builtin_amdgcn_readlane(q_up[s], 63);
  }
  // The strips of a row are loaded together; each strip's registers take the
  // next row's loads as soon as the strip is reduced, so that they are in
  // flight while the rest of the row is computed.
  static_assert(G == NS, "one group of strips per row");
  BinPix<BB> px[NS];
#define RSZ_LOAD(s, Irow)                                                                   \
  do {                                                                                      \
    if constexpr (VEC) {                                                                    \
      const uint32_t jv_ = RSZ_JC(s);                                                       \
      load_vec<BB, BG>(px[s], fr, H, W, (Irow), jv_ * (uint32_t)b * 4u, mask + RSZ_MW(jv_), \
                       R0, wpr);                                                            \
    } else {                                                                                \
      const uint32_t jc_ = RSZ_JC(s);                                                       \
      load_bin<BB, VEC, BG>(px[s], fr, H, W, b, (Irow), jc_, mask, R0, wpr, RSZ_MW(jc_));  \
    }                                                                                       \
  } while (0)
  // The row loop is compiled for each count of strips it takes (NSR), so
  // that every strip's loads are unconditional code: with the count a
  // run-time bound the compiler cannot count the loads in flight and waits
  // for all of them at the top of each row.
  auto row_loop = [&](auto nsr_c) __attribute__((always_inline)) {
    constexpr int NSR = decltype(nsr_c)::value;
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (s < NSR) {
        RSZ_LOAD(s, I0);
        // issued in strip order, as the loop issues them (the loop's waits
        // count on strip 0's loads being the oldest on entry too)
        __builtin_amdgcn_sched_barrier(0);
      }
    for (uint32_t I = I0; I < I1; ++I) {
      // q left of the group on this row
      int32_t left = __builtin_amdgcn_readlane(q_left, I - I0 + 1);
      if (dim == 1 && whole_rows && I > 0) left = lastq;
      // in-panel pixels of this bin row (vector path: every column is)
      uint32_t rowbits = 0;
      if constexpr (VEC) rowbits = (1u << (min((uint32_t)BB, H - I * BB) * BB)) - 1u;
      {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if (s >= NSR) break;
          const uint32_t J = J0 + s * 64 + lane;
          const bool colv = J < Wb;
          const uint32_t jc = RSZ_JC(s);
          int32_t qv;
          if constexpr (VEC) {
            qv = reduce_vec<BB, BG>(px[s], rowbits, (int)((jc * b) & 31), inv, step, range_err,
                                    DEBUG, Sd, nd);
          } else {
            qv = reduce_bin<BB, BG>(px[s], H, W, b, I, J, step, inv, range_err, Sd, nd,
                                    (int)((jc * b) & 31), mask, R0, wpr, RSZ_MW(jc));
          }
          // the next row's loads are issued on every row (the last row loads
          // itself again, from cache): a load under a condition leaves the
          // compiler unable to count what is in flight, and it then waits
          // for every load at the top of each row
          RSZ_LOAD(s, min(I + 1, I1 - 1));
          const int32_t q = colv ? qv : 0;
          const int32_t ql = from_left(q, left);
          left = __builtin_amdgcn_readlane(q, 63);
          // residual; codes 1..1023 carry r + 512, 0 marks an outlier
          const int32_t r = dim == 1 ? q - ql : q + ql_up[s] - q_up[s] - ql;
          const uint32_t code = code_from_residual(r);
          if (sparse) {
            // the first bin of a row whose dimension-1 predecessor lies in
            // another tile (k_lorenzo_dims corrects it) always goes to rbuf
            const bool forced = dim == 1 && s == 0 && J == 0 && (!whole_rows || I == 0) &&
                                (p | I) != 0;
            const uint32_t cb = forced ? 0u : code_byte(r);
            const bool nz = colv && cb != 128u;
            const uint64_t m = __ballot(nz);
            if (nz) {
              const uint32_t rank =
                  __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
              stg->zb[(zcount + rank) & (kZbRing - 1)] = (uint8_t)cb;
              if (cb == 0) *gm((int32_t *)((char *)(rbuf + (size_t)I * Wb) + J * 4u)) = r;
            }
            // every lane writes the same wave-uniform entry (no branch)
            const bool here = (uint32_t)lane == (uint32_t)(s & 1) * 32u + (I - I0);
            zmlo[s >> 1] = here ? (uint32_t)m : zmlo[s >> 1];
            zmhi[s >> 1] = here ? (uint32_t)(m >> 32) : zmhi[s >> 1];
            zpv[s >> 1] = here ? zcount : zpv[s >> 1];
            zcount += (uint32_t)__builtin_popcountll(m);
            // m holds exactly the lanes whose code is not 512 (a forced bin
            // with r = 0 is counted through the loop, to the same total)
            if (dim != 3) wave_histogram_nz(code, m, vmask[s], hist, c512);
            if (DEBUG && colv) {
              const size_t g = (size_t)I * Wb + J;
              if (fp.dbg_S) fp.dbg_S[gbase + g] = Sd;
              if (fp.dbg_n) fp.dbg_n[gbase + g] = nd;
              if (fp.dbg_q) fp.dbg_q[gbase + g] = q;
            }
          } else if (colv) {
            const size_t g = (size_t)I * Wb + J;
            const uint32_t cb = code_byte(r);
            // row pointer (wave-uniform) + 32-bit lane offset
            *gm(codes + (size_t)I * Wb + J) = (uint8_t)cb;
            if (cb == 0) *gm((int32_t *)((char *)(rbuf + (size_t)I * Wb) + J * 4u)) = r;
            if (DEBUG) {
              if (fp.dbg_S) fp.dbg_S[gbase + g] = Sd;
              if (fp.dbg_n) fp.dbg_n[gbase + g] = nd;
              if (fp.dbg_q) fp.dbg_q[gbase + g] = q;
            }
          }
          if (!sparse && dim != 3) wave_histogram(code, vmask[s], hist, c512);
          if (dim == 1 && s == ns - 1) lastq = __builtin_amdgcn_readlane(q, lastlane);
          q_up[s] = q;
          ql_up[s] = ql;
        }
      }
      if (packed) qlast = (uint32_t)lane == I - I0 ? left : qlast;
      // the row's last q, for k_lorenzo_dims where it cannot be used here
      if (dim == 1 && last_group && (!whole_rows || I == Hb - 1) && lane == 0)
        fp.qedge[(size_t)p * Hb + I] = lastq;
      if (sparse && zcount - zflushed >= kZbFlush) {
        wave_sync();
        flush_zb(*stg, fp.zb + (size_t)tix * fp.tile_cap, zflushed, zflushed + kZbFlush);
        zflushed += kZbFlush;
        wave_sync();
      }
    }
  };
  switch (nsr) {
    case 1: row_loop(std::integral_constant<int, 1>{}); break;
    case 2: if constexpr (NS >= 2) row_loop(std::integral_constant<int, 2>{}); break;
    case 3: if constexpr (NS >= 3) row_loop(std::integral_constant<int, 3>{}); break;
    default: if constexpr (NS >= 4) row_loop(std::integral_constant<int, 4>{}); break;
  }
  if constexpr (VEC) {
    if (packed) {
      const uint32_t nr = I1 - I0;
      const uint32_t r = (uint32_t)lane / rem, c = (uint32_t)lane - r * rem;
      const bool valid = r < nr;
      const uint32_t I = I0 + min(r, nr - 1), Jb = J0 + 64 * (uint32_t)nsr, J = Jb + c;
      // q of the halo row over the packed columns
      int32_t qh = 0;
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s == nsr) qh = q_up[s];
      BinPix<BB> pxp;
      load_vec<BB, BG>(pxp, fr, H, W, I, J * (uint32_t)b * 4u, mask + RSZ_MW(J), R0, wpr);
      const uint32_t rowbits = (1u << (min((uint32_t)BB, H - I * BB) * BB)) - 1u;
      const int32_t qv = reduce_vec<BB, BG>(pxp, rowbits, (int)((J * b) & 31), inv, step,
                                            range_err, DEBUG, Sd, nd);
      const int32_t q = valid ? qv : 0;
      // neighbours: within the vector, or the row loop's last column (qlast)
      // and the halo row
      const int32_t sl = __shfl(q, max(lane - 1, 0)), su = __shfl(q, max(lane - (int)rem, 0));
      const int32_t sul = __shfl(q, max(lane - (int)rem - 1, 0));
      const int32_t ql0 = __shfl(qlast, (int)r), qlu = __shfl(qlast, (int)r - 1 < 0 ? 0 : (int)r - 1);
      const int32_t qhc = __shfl(qh, (int)c), qhcl = __shfl(qh, c > 0 ? (int)c - 1 : 0);
      const int32_t ql = c > 0 ? sl : ql0;
      const int32_t qu = r > 0 ? su : qhc;
      const int32_t qul = r > 0 ? (c > 0 ? sul : qlu) : (c > 0 ? qhcl : qhl);
      const int32_t res = q + qul - qu - ql;
      const uint32_t code = code_from_residual(res);
      const uint32_t cb = code_byte(res);
      const size_t g = (size_t)I * Wb + J;
      if (sparse) {
        const bool nz = valid && cb != 128u;
        const uint64_t m = __ballot(nz);
        if (nz) {
          const uint32_t rank =
              __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          stg->zb[(zcount + rank) & (kZbRing - 1)] = (uint8_t)cb;
          if (cb == 0) *gm(rbuf + g) = res;
        }
        // entry (strip nsr, tile row i): lane i takes its rem bits, and the
        // count of the set bits before them
        const uint64_t ev = (uint32_t)lane < nr ? (m >> ((uint32_t)lane * rem)) & low_bits(rem) : 0ull;
        const uint32_t ez = zcount + (uint32_t)__builtin_popcountll(m & low_bits((uint32_t)lane * rem));
        const int src = lane - 32 * (nsr & 1);
        const bool here = src >= 0 && (uint32_t)src < nr;
        const uint32_t elo = __shfl((uint32_t)ev, max(src, 0)), ehi = __shfl((uint32_t)(ev >> 32), max(src, 0));
        const uint32_t ezs = __shfl(ez, max(src, 0));
#pragma unroll
        for (int pr = 0; pr < 2; ++pr)
          if (pr == (nsr >> 1) && here) {
            zmlo[pr] = elo;
            zmhi[pr] = ehi;
            zpv[pr] = ezs;
          }
        zcount += (uint32_t)__builtin_popcountll(m);
      } else if (valid) {
        *gm(codes + g) = (uint8_t)cb;
        if (cb == 0) *gm(rbuf + g) = res;
      }
      if (DEBUG && valid) {
        if (fp.dbg_S) fp.dbg_S[gbase + g] = Sd;
        if (fp.dbg_n) fp.dbg_n[gbase + g] = nd;
        if (fp.dbg_q) fp.dbg_q[gbase + g] = q;
      }
      if (dim != 3) wave_histogram(code, __ballot(valid), hist, c512);
    }
  }
  if (sparse) {
    wave_sync();
    flush_zb(*stg, fp.zb + (size_t)tix * fp.tile_cap, zflushed, zcount);
    uint64_t *zm = fp.zm + (size_t)tix * kTileEntries;
    uint16_t *zp = fp.zp + (size_t)tix * kTileEntries;
    *gm(zm + lane) = (uint64_t)zmhi[0] << 32 | zmlo[0];
    *gm(zp + lane) = (uint16_t)zpv[0];
    if (NS > 2 && gsl > 2) {
      *gm(zm + 64 + lane) = (uint64_t)zmhi[1] << 32 | zmlo[1];
      *gm(zp + 64 + lane) = (uint16_t)zpv[1];
    }
    wave_sync();
  }
#undef RSZ_LOAD
#undef RSZ_MW
#undef RSZ_JC
  if (lane == 0 && c512) atomicAdd(&hist[kRadius], c512);   // c512 is a wave total
  if (range_err) set_status(fp.st, RSZ_ERR_RANGE);
}

// BB: the bin factor (1, 2, 4) compiled in, or 0 for any b (one strip per
// column group).  DIM: the Lorenzo dimension compiled in, or 0 for a batch
// mixing dimensions (read per frame).  Workgroup t of a frame: panel, column
// group, then a group of kWaves consecutive segments, one per wave.
template <int BB, bool DEBUG, int DIM, bool VONLY>
__device__ __forceinline__ void k_bin_body(BatchPlan bp) {
  __shared__ uint32_t s_hist[kNumSym];
  __shared__ uint32_t s_mask[kWaves][kMaskWords];
  __shared__ double s_inv[65];
  __shared__ SparseStage s_stage[DIM == 3 ? 1 : kWaves];
  const uint32_t f = bp.tile_frame[blockIdx.x];
  const FramePlan &fp = bp.frames[f];
  for (int i = threadIdx.x; i < kNumSym; i += blockDim.x) s_hist[i] = 0u;
  for (int i = threadIdx.x; i < 65; i += blockDim.x) s_inv[i] = fp.st->inv[i];
  __syncthreads();
  // wave index as a wave-uniform (scalar) value: everything per tile and
  // per row below stays in scalar registers
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t t = blockIdx.x - bp.tile_prefix[f];
  const uint32_t per_panel = fp.groups * fp.cgs;
  const uint32_t panel = t / per_panel, rem = t % per_panel;
  const uint32_t cg = rem / fp.groups, seg = (rem % fp.groups) * bp.bin_waves + wv;
  const bool ok = load_status(fp.st) == RSZ_OK;
  if (ok && seg < fp.segs) {
    const bool bg = fp.mode == RSZ_BIN_BACKGROUND;
    uint32_t *mask = s_mask[wv];
    SparseStage *stg = &s_stage[DIM == 3 ? 0 : wv];
    bool vec = false;
    if constexpr (BB == 2 || BB == 4) {
      vec = fp.vec != 0;
      if (vec) {
        if (bg) bin_tile<BB, true, true, DEBUG, DIM>(fp, panel, seg, cg, s_hist, mask, s_inv, stg);
        else bin_tile<BB, true, false, DEBUG, DIM>(fp, panel, seg, cg, s_hist, mask, s_inv, stg);
      }
    }
    // VONLY: every frame of the batch takes the vector path, and the kernel
    // holds only its registers (the scalar path needs more)
    if (!VONLY && !vec) {
      if (bg) bin_tile<BB, false, true, DEBUG, DIM>(fp, panel, seg, cg, s_hist, mask, s_inv, stg);
      else bin_tile<BB, false, false, DEBUG, DIM>(fp, panel, seg, cg, s_hist, mask, s_inv, stg);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kNumSym; i += blockDim.x)
    if (s_hist[i]) atomicAdd(&fp.st->hist[i], s_hist[i]);
}

template <int BB, bool DEBUG, int DIM>
__global__ __launch_bounds__(256) void k_bin(BatchPlan bp) {
  k_bin_body<BB, DEBUG, DIM, false>(bp);
}

// Batches whose frames all take the vector path, without the scalar path's
// registers.  Four waves per SIMD: with the row loop's loads in strip order
// the kernel holds its strips' loads and its sums in 128 registers without
// spilling (five waves spill 23 registers, and measured 0.17 ms slower on
// the 1000-frame CSPAD batch; six spill more).
template <int BB, int DIM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_bin_vec(
    BatchPlan bp) {
  k_bin_body<BB, false, DIM, true>(bp);
}

// ------------------------------------------------------- k_lorenzo_dims

// Finishes the residuals of frames whose Lorenzo predictor is not 2D (the
// "dimension" of Sec. VI), after k_bin.
//  dim 1: one lane per bin row R = p*Hb + I whose first bin k_bin coded as
//    r = q (the first row of each panel; every row of a panel split into
//    column groups).  That bin follows the last bin of row R - 1 in raster
//    order, so r = q_first(R) - q_last(R - 1) replaces it (q_first is the r
//    k_bin coded, q_last comes from qedge); the histogram moves the bin from
//    the old code to the new one.
//  dim 3: the 3D residual is the difference along the panel axis of the
//    panels' 2D residuals (the operators commute): r3[g] = r2[g] - r2[g -
//    Hb*Wb], or r2[g] on panel 0.  k_bin left r2 in codes2/rbuf2.  A
//    workgroup takes kFixBins3 bins, a lane 16 consecutive code bytes per
//    step: one aligned 16-byte load, and its predecessors' bytes shifted out
//    of two aligned loads (the shift, (-Hb*Wb) mod 16, is the same for every
//    lane).  Equal nonzero bytes on both sides mean r3 = 0: output byte 128,
//    code 512, counted by a popcount.  The few other bytes (residuals that
//    differ, escapes, panel 0) are taken one by one.  It writes the code
//    bytes of r3 to codes (r3 to rbuf where the byte is 0) and counts the
//    histogram.

// 0x80 in each byte of x that is zero, 0 elsewhere.
__device__ __forceinline__ uint32_t zero_bytes(uint32_t x) {
  const uint32_t y = (x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
  return ~(y | x | 0x7F7F7F7Fu);
}
// Bit i (i < 4) set where byte i of m has its top bit set.
__device__ __forceinline__ uint32_t byte_bits(uint32_t m) {
  return ((m >> 7) & 1u) | ((m >> 14) & 2u) | ((m >> 21) & 4u) | ((m >> 28) & 8u);
}

__device__ __forceinline__ int32_t r_of(uint32_t byte, const int32_t *rbuf, uint32_t g) {
  return byte ? (int32_t)byte - 128 : rbuf[g];
}

// The 16 code bytes of bins [g0, g0 + 16) (g0 a multiple of 16) of a frame
// with sparse codes, as the dense form would hold them: 128 where the
// zero-map bit is clear, the stored byte where it is set; bytes past the
// frame read 128.  The bins are taken in pieces that lie within one strip of
// one bin row; a piece's stored bytes start at the entry's count plus the
// set bits before the piece.
__device__ uint4 sparse_group(const FramePlan &fp, uint32_t g0) {
  uint32_t w[4] = {0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u};
  const uint32_t end = min(g0 + 16u, fp.nbins);
  for (uint32_t g = g0; g < end;) {
    const uint32_t R = fdiv(fp.fd_Wb, g), J = g - R * fp.Wb;
    const uint32_t pn = fdiv(fp.fd_Hb, R), I = R - pn * fp.Hb;
    const uint32_t seg = fdiv(fp.fd_TH, I), li = I - seg * fp.TH;
    const uint32_t st = J >> 6, a = J & 63u;
    const uint32_t cg = fdiv(fp.fd_gs, st), ls = st - cg * fp.gstrips;
    const uint32_t tix = (pn * fp.cgs + cg) * fp.segs + seg;
    const size_t e = (size_t)tix * kTileEntries + ls * 32u + li;
    const uint32_t n = min(min(64u - a, fp.Wb - J), end - g);
    const uint64_t word = fp.zm[e];
    uint64_t m = (word >> a) & (n == 64 ? ~0ull : (1ull << n) - 1ull);
    if (m) {
      const uint8_t *zb = fp.zb + (size_t)tix * fp.tile_cap + fp.zp[e] +
                          __builtin_popcountll(word & ((1ull << a) - 1ull));
      for (uint32_t k = 0; m; m &= m - 1, ++k) {
        const uint32_t pos = g - g0 + (uint32_t)__builtin_ctzll(m);
        const uint32_t sh = 8 * (pos & 3);
        w[pos >> 2] = (w[pos >> 2] & ~(0xFFu << sh)) | ((uint32_t)zb[k] << sh);
      }
    }
    g += n;
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// 16 code bytes of bins [g0, g0 + 16): the dense bytes, or the sparse form
// expanded (the dense region is padded to whole chunks, so its 16-byte loads
// stay inside it).
__device__ __forceinline__ uint4 code_group(const FramePlan &fp, uint32_t g0) {
  return fp.sparse ? sparse_group(fp, g0) : *(const uint4 *)(fp.codes + g0);
}

__global__ __launch_bounds__(256) void k_lorenzo_dims(BatchPlan bp) {
  __shared__ uint32_t s_hist[kNumSym];
  const uint32_t f = find_frame(bp.fix_prefix, bp.nframes, blockIdx.x);
  const FramePlan &fp = bp.frames[f];
  if (load_status(fp.st) != RSZ_OK) return;   // the same frame for the whole workgroup
  const uint32_t blk = blockIdx.x - bp.fix_prefix[f];
  if (fp.dim == 1) {
    const uint32_t t = blk * 256 + threadIdx.x;
    const uint32_t R = fp.cgs == 1 ? t * fp.Hb : t;
    if (t >= (fp.cgs == 1 ? fp.P : fp.P * fp.Hb) || R == 0) return;
    const size_t g = (size_t)R * fp.Wb;
    // k_bin stored this bin's r = q as an escape (sparse codes: its byte is 0)
    const int32_t qf = fp.rbuf[g];
    const int32_t prev = fp.qedge[R - 1];
    if (prev == 0) return;
    const int32_t r = qf - prev;   // |q| <= 2^28 - 1
    fp.rbuf[g] = r;
    const uint32_t c0 = code_from_residual(qf), c1 = code_from_residual(r);
    if (c0 != c1) {
      atomicSub(&fp.st->hist[c0], 1u);
      atomicAdd(&fp.st->hist[c1], 1u);
    }
    return;
  }
  for (int i = threadIdx.x; i < kNumSym; i += 256) s_hist[i] = 0u;
  __syncthreads();
  const uint32_t plane = fp.Hb * fp.Wb, nbins = fp.nbins;
  const uint4 *__restrict__ c2v = (const uint4 *)fp.codes2;
  const uint8_t *__restrict__ c2b = fp.codes2;
  const int32_t *__restrict__ rb2 = fp.rbuf2;
  uint4 *__restrict__ cout = (uint4 *)fp.codes;
  int32_t *__restrict__ rout = fp.rbuf;
  // the predecessors of 16 aligned bytes start (-plane) mod 16 bytes into an
  // aligned 16-byte group: words q.. of two consecutive groups, shifted by r bytes
  const uint32_t off = (0u - plane) & 15u, qw = off >> 2, rb = off & 3u;
  constexpr int K = (int)(kFixBins3 / 4096);
  uint32_t ow[K][4], pw[K][4];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t g0 = blk * kFixBins3 + k * 4096 + threadIdx.x * 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) ow[k][i] = pw[k][i] = 0u;
    if (g0 < nbins) {
      const uint4 o = c2v[g0 >> 4];
      ow[k][0] = o.x; ow[k][1] = o.y; ow[k][2] = o.z; ow[k][3] = o.w;
      if (g0 >= plane) {
        const uint32_t a = (g0 - plane) & ~15u;   // group holding byte g0 - plane
        const uint4 lo = c2v[a >> 4];
        const uint4 hi = off ? c2v[(a >> 4) + 1] : make_uint4(0u, 0u, 0u, 0u);
        const uint32_t w8[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          uint32_t a0 = w8[i], a1 = w8[i + 1];
#pragma unroll
          for (int t = 1; t < 4; ++t)
            if (qw == (uint32_t)t) { a0 = w8[(i + t) & 7]; a1 = w8[(i + t + 1) & 7]; }
          pw[k][i] = (uint32_t)((((uint64_t)a1 << 32) | a0) >> (8 * rb));
        }
      } else if (g0 + 16 > plane) {
        for (uint32_t e = plane - g0; e < 16 && g0 + e < nbins; ++e)
          pw[k][e >> 2] |= (uint32_t)c2b[g0 + e - plane] << (8 * (e & 3));
      }
    }
  }
  uint32_t c512 = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t g0 = blk * kFixBins3 + k * 4096 + threadIdx.x * 16;
    if (g0 >= nbins) continue;
    // bytes to take one by one: escapes (code byte 0) on either side, bytes
    // whose 2D residuals differ, bytes of panel 0 and bytes past the frame;
    // every other byte has r3 = 0 (output byte 128, code 512)
    uint32_t slow = 0, outw[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t x = ow[k][i] ^ pw[k][i];
      const uint32_t eq = zero_bytes(x), ze = zero_bytes(ow[k][i]) | zero_bytes(pw[k][i]);
      slow |= byte_bits(~eq | ze) << (4 * i);
      outw[i] = 0x80808080u;
    }
    if (g0 < plane) slow |= plane - g0 >= 16 ? 0xFFFFu : (1u << (plane - g0)) - 1u;
    if (g0 + 16 > nbins) slow |= 0xFFFFu & ~((1u << (nbins - g0)) - 1u);
    c512 += 16 - __builtin_popcount(slow);
    while (slow) {
      const int e = __builtin_ctz(slow);
      slow &= slow - 1;
      const uint32_t g = g0 + e;
      if (g >= nbins) continue;
      const uint32_t b2 = (ow[k][e >> 2] >> (8 * (e & 3))) & 0xFFu;
      const uint32_t bq = (pw[k][e >> 2] >> (8 * (e & 3))) & 0xFFu;
      const uint32_t r2 = b2 ? b2 - 128u : (uint32_t)rb2[g];
      const uint32_t rp = g >= plane ? (bq ? bq - 128u : (uint32_t)rb2[g - plane]) : 0u;
      const uint32_t r = r2 - rp;   // |r3| <= 8 (2^28 - 1) < 2^31
      const uint32_t nb = code_byte((int32_t)r);
      outw[e >> 2] = (outw[e >> 2] & ~(0xFFu << (8 * (e & 3)))) | (nb << (8 * (e & 3)));
      if (nb == 0) rout[g] = (int32_t)r;
      // residual 0 (most of panel 0's bytes) joins the wave's count: one
      // LDS atomic per lane on the same word would serialise the wave
      const uint32_t code = code_from_residual((int32_t)r);
      if (code == (uint32_t)kRadius) ++c512;
      else atomicAdd(&s_hist[code], 1u);
    }
    cout[g0 >> 4] = make_uint4(outw[0], outw[1], outw[2], outw[3]);
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) c512 += __shfl_xor(c512, d);
  if ((threadIdx.x & 63) == 0 && c512) atomicAdd(&s_hist[kRadius], c512);
  __syncthreads();
  uint32_t *ghist = fp.st->hist;
  for (int i = threadIdx.x; i < kNumSym; i += 256)
    if (s_hist[i]) atomicAdd(&ghist[i], s_hist[i]);
}

// ------------------------------------------------------------- k_codebook

// Ascending bitonic sort of key[0, n), n a power of two <= 1024, by the
// workgroup (unique keys).
__device__ void bitonic_sort(uint64_t *key, uint32_t n) {
  for (uint32_t k = 2; k <= n; k <<= 1)
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t t = threadIdx.x; t < n / 2; t += 256) {
        const uint32_t i = 2 * t - (t & (j - 1));
        const uint32_t l = i + j;
        const bool asc = (i & k) == 0;
        const uint64_t a = key[i], c = key[l];
        if ((a > c) == asc) {
          key[i] = c;
          key[l] = a;
        }
      }
      __syncthreads();
    }
}

// Gathers key(s) of the symbols with keep(s) into key[0, n) in symbol order,
// pads with ~0 up to the next power of two and sorts; returns n.
template <class KeyOf>
__device__ uint32_t gather_and_sort(uint64_t *key, uint32_t *s_tmp32, KeyOf key_of) {
  uint64_t kv[4];
  uint32_t cnt = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    kv[e] = key_of(threadIdx.x * 4 + e);
    cnt += kv[e] != ~0ull;
  }
  uint32_t n;
  uint32_t pos = block_exclusive_scan<uint32_t>(cnt, s_tmp32, n);
  uint32_t p2 = 1;
  while (p2 < n) p2 <<= 1;
  for (uint32_t i = n + threadIdx.x; i < p2; i += 256) key[i] = ~0ull;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (kv[e] != ~0ull) key[pos++] = kv[e];
  __syncthreads();
  if (p2 > 1) bitonic_sort(key, p2);
  return n;
}

// Huffman code lengths by the two-queue method over leaves sorted by
// (count, symbol), internal nodes in creation order, a leaf taken first on
// equal weights; lengths above 32 make the counts halve (kept >= 1) and the
// build repeat.  Then canonical codewords in (length, symbol) order.
// Huffman lengths (two-queue rule, halving rebuild above kMaxLen) and
// canonical codewords of the histogram `hist` (kNumSym entries) into
// lens / cw, by one workgroup.
__device__ void build_code(FrameState *st, const uint32_t *hist, uint8_t *lens_out,
                           uint32_t *cw_out) {
  __shared__ uint64_t s_key[kNumSym];
  __shared__ uint32_t s_w[2 * kNumSym];      // node weights: leaves, then internal nodes
  __shared__ uint16_t s_anc[2][2 * kNumSym]; // parents, then ancestors (pointer jumping)
  __shared__ uint16_t s_dep[2][2 * kNumSym];
  __shared__ uint32_t s_weight[kNumSym];
  __shared__ uint8_t s_len[kNumSym];
  __shared__ uint32_t s_blc[kMaxLen + 1];
  __shared__ uint32_t s_first[kMaxLen + 1];
  __shared__ uint32_t s_start[kMaxLen + 1];
  __shared__ uint32_t s_tmp32[4];
  __shared__ int s_maxlen, s_ok;
  if (threadIdx.x == 0) s_ok = load_status(st) == RSZ_OK;
  __syncthreads();
  if (!s_ok) return;
  for (int s = threadIdx.x; s < kNumSym; s += 256) {
    s_weight[s] = hist[s];   // the counts sum to < 2^27
    s_len[s] = 0;
  }
  __syncthreads();
  uint32_t nl;
  int cur = 0;   // pointer-jumping buffer holding the final depths
  for (;;) {
    nl = gather_and_sort(s_key, s_tmp32, [&](uint32_t sym) {
      const uint32_t w = s_weight[sym];
      return w ? (((uint64_t)w << 10) | sym) : ~0ull;
    });
    const uint32_t nn = nl ? 2 * nl - 1 : 0;   // nodes; the root is nn - 1
    for (uint32_t i = threadIdx.x; i < nl; i += 256) s_w[i] = (uint32_t)(s_key[i] >> 10);
    __syncthreads();
    if (threadIdx.x == 0 && nl > 1) {
      // the merge is sequential; the next leaf weight is read ahead
      uint32_t lf = 0, nf = nl, ne = nl;
      uint32_t wl = s_w[0];
      for (uint32_t m = 0; m + 1 < nl; ++m) {
        uint32_t pick[2], wsum = 0;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const bool leaf = nf == ne || (lf < nl && wl <= s_w[nf]);
          if (leaf) {
            pick[t] = lf++;
            wsum += wl;
            wl = lf < nl ? s_w[lf] : 0u;
          } else {
            pick[t] = nf;
            wsum += s_w[nf++];
          }
        }
        s_w[ne] = wsum;
        s_anc[0][pick[0]] = (uint16_t)ne;
        s_anc[0][pick[1]] = (uint16_t)ne;
        ne++;
      }
    }
    __syncthreads();
    // depth of every node by pointer jumping: dep = distance to anc
    const uint32_t root = nn ? nn - 1 : 0;
    for (uint32_t v = threadIdx.x; v < nn; v += 256) {
      s_dep[0][v] = v == root ? 0 : 1;
      if (v == root) s_anc[0][v] = (uint16_t)root;
    }
    __syncthreads();
    cur = 0;
    for (uint32_t span = 1; span < nn; span <<= 1) {
      for (uint32_t v = threadIdx.x; v < nn; v += 256) {
        const uint32_t a = s_anc[cur][v];
        s_dep[cur ^ 1][v] = s_dep[cur][v] + s_dep[cur][a];
        s_anc[cur ^ 1][v] = s_anc[cur][a];
      }
      __syncthreads();
      cur ^= 1;
    }
    if (threadIdx.x == 0) s_maxlen = nl == 1 ? 1 : 0;
    __syncthreads();
    if (nl > 1) {
      uint32_t mx = 0;
      for (uint32_t i = threadIdx.x; i < nl; i += 256) mx = max(mx, (uint32_t)s_dep[cur][i]);
      atomicMax(&s_maxlen, (int)mx);
    }
    __syncthreads();
    if (s_maxlen <= kMaxLen) break;
    for (int s = threadIdx.x; s < kNumSym; s += 256)
      if (s_weight[s]) s_weight[s] = (s_weight[s] >> 1) ? (s_weight[s] >> 1) : 1u;
    __syncthreads();
  }
  // lengths by symbol; a single used symbol gets length 1
  for (uint32_t i = threadIdx.x; i < nl; i += 256)
    s_len[s_key[i] & 1023] = nl == 1 ? 1 : (uint8_t)s_dep[cur][i];
  if (threadIdx.x <= kMaxLen) s_blc[threadIdx.x] = 0;
  __syncthreads();
  // canonical order: the used symbols sorted by (length, symbol)
  const uint32_t nu = gather_and_sort(s_key, s_tmp32, [&](uint32_t sym) {
    const uint32_t L = s_len[sym];
    return L ? (((uint64_t)L << 10) | sym) : ~0ull;
  });
  for (uint32_t i = threadIdx.x; i < nu; i += 256) atomicAdd(&s_blc[s_key[i] >> 10], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t code = 0, start = 0;
    s_blc[0] = 0;
    for (int L = 1; L <= kMaxLen; ++L) {
      code = (code + s_blc[L - 1]) << 1;
      s_first[L] = code;
      s_start[L] = start;
      start += s_blc[L];
    }
  }
  __syncthreads();
  for (int s = threadIdx.x; s < kNumSym; s += 256) {
    lens_out[s] = s_len[s];
    cw_out[s] = 0;
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nu; i += 256) {
    const uint64_t k = s_key[i];
    const uint32_t L = (uint32_t)(k >> 10), sym = (uint32_t)(k & 1023);
    cw_out[sym] = s_first[L] + (i - s_start[L]);
  }
}

__global__ __launch_bounds__(256) void k_codebook(BatchPlan bp) {
  FrameState *st = bp.frames[blockIdx.x].st;
  build_code(st, st->hist, st->lens, st->cw);
}

// Bit k of the result (k = 0..15) is set where byte k of the 16 bytes w
// differs from 0x80, the code byte of residual 0.  Per 32-bit word, x = w ^
// 0x80808080 has a zero byte exactly where w has 0x80, and ((x & 0x7F7F7F7F)
// + 0x7F7F7F7F) | x sets each byte's top bit exactly where that byte of x is
// not zero (no carry crosses a byte).
__device__ __forceinline__ uint32_t non_zero_residuals(const uint32_t (&w)[4]) {
  uint32_t m = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t x = w[e] ^ 0x80808080u;
    const uint32_t hi = (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
    m |= ((hi >> 7) & 1u) << (4 * e) | ((hi >> 15) & 1u) << (4 * e + 1) |
         ((hi >> 23) & 1u) << (4 * e + 2) | (hi >> 31) << (4 * e + 3);
  }
  return m;
}

// Byte k (0..15, any lane value) of the 16 bytes w.
__device__ __forceinline__ uint32_t byte_at(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                            uint32_t k) {
  const uint32_t x = k < 8 ? (k < 4 ? w0 : w1) : (k < 12 ? w2 : w3);
  return (x >> (8 * (k & 3))) & 0xFFu;
}

// Sparse rounds: at most this many bytes per lane differ from residual 0's.
constexpr uint32_t kSparseBytes = 4;

// ---------------------------------------------------------------- k_count

// Exclusive prefix sums over the lanes of a wave, and the wave total.
__device__ __forceinline__ uint64_t wave_exclusive_scan(uint64_t v, uint64_t &total) {
  const int lane = threadIdx.x & 63;
  uint64_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  total = __shfl(x, 63);
  return x - v;
}

__device__ __forceinline__ uint32_t wave_exclusive_scan32(uint32_t v, uint32_t &total) {
  const int lane = threadIdx.x & 63;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  total = __shfl(x, 63);
  return x - v;
}


// Position of a bin of a frame with sparse codes, for walking its bins in
// raster order piece by piece: a piece lies in one strip (64 bin columns) of
// one bin row.  J, I, pn: column, row and panel; seg, li: segment and row
// within it; st, cg, ls: strip, column group and strip within the group.
struct BinCursor {
  uint32_t g, J, I, pn, seg, li, st, cg, ls;
};

__device__ __forceinline__ BinCursor bin_cursor(const FramePlan &fp, uint32_t g) {
  BinCursor c;
  c.g = g;
  const uint32_t R = fdiv(fp.fd_Wb, g);
  c.J = g - R * fp.Wb;
  c.pn = fdiv(fp.fd_Hb, R);
  c.I = R - c.pn * fp.Hb;
  c.seg = fdiv(fp.fd_TH, c.I);
  c.li = c.I - c.seg * fp.TH;
  c.st = c.J >> 6;
  c.cg = fdiv(fp.fd_gs, c.st);
  c.ls = c.st - c.cg * fp.gstrips;
  return c;
}

// The cursor's piece: its binning tile, entry, first column within the
// strip, and length (at most `left` bins).
__device__ __forceinline__ uint32_t cursor_tile(const FramePlan &fp, const BinCursor &c) {
  return (c.pn * fp.cgs + c.cg) * fp.segs + c.seg;
}
__device__ __forceinline__ size_t cursor_entry(const FramePlan &fp, const BinCursor &c) {
  return (size_t)cursor_tile(fp, c) * kTileEntries + c.ls * 32u + c.li;
}
__device__ __forceinline__ uint32_t cursor_len(const FramePlan &fp, const BinCursor &c,
                                               uint32_t left) {
  return min(min(64u - (c.J & 63u), fp.Wb - c.J), left);
}

// Moves the cursor past its piece of n bins (n = cursor_len).
__device__ __forceinline__ void cursor_advance(const FramePlan &fp, BinCursor &c, uint32_t n) {
  c.g += n;
  c.J += n;
  if (c.J < fp.Wb) {   // the next strip of the row
    c.st++;
    if (++c.ls == fp.gstrips) {
      c.ls = 0;
      c.cg++;
    }
    return;
  }
  c.J = c.st = c.cg = c.ls = 0;   // the next row
  if (++c.I == fp.Hb) {
    c.I = c.seg = c.li = 0;
    c.pn++;
  } else if (++c.li == fp.TH) {
    c.li = 0;
    c.seg++;
  }
}

// Calls f(g, n, a, tix, e) for the pieces of bins [g, end) of a frame with
// sparse codes: a is the piece's first column within its strip, tix its
// binning tile, e its entry.
template <class F>
__device__ __forceinline__ void for_pieces(const FramePlan &fp, uint32_t g, uint32_t end, F f) {
  if (g >= end) return;
  BinCursor c = bin_cursor(fp, g);
  while (c.g < end) {
    const uint32_t n = cursor_len(fp, c, end - c.g);
    f(c.g, n, c.J & 63u, cursor_tile(fp, c), cursor_entry(fp, c));
    cursor_advance(fp, c, n);
  }
}

// The chunk form of the codes, which k_count leaves for k_encode: for chunk
// c, cmask[c * 64 + j] has bit k set where bin c * 4096 + 64 j + k carries a
// code byte other than 128 (residual 0), and those bytes follow in bin order
// from codes + c * 4096.
//
// One wave per 4096-symbol chunk, four per workgroup (a workgroup's first
// chunk from count_frame): the chunk form from the sparse codes of k_bin (or
// from the dense bytes of dimension 3, compacted in place), and the chunk's
// bits and outliers.  Lane l takes bins [64 l, 64 l + 64) of the chunk: the
// pieces of its window are located first and their zero-map words loaded
// together, which gives the lane's count of bytes and so (by a wave scan) its
// place in the chunk before any byte is read.  Each piece's bytes are then
// read 16 at a time with aligned word loads and put straight into their
// compacted place in the wave's LDS buffer, which is copied out in whole
// 16-byte stores.  SPARSE: every frame of the batch has sparse codes (the
// kernel holds no dense path).

// Reads the n (<= 64) bytes at zb + o of a tile's byte region (cap bytes, a
// multiple of 16) 16 at a time with aligned word loads; for each, in order,
// calls f(byte).  Words past the region are never read (the index is
// clamped; their bytes are not used).
template <typename F>
__device__ __forceinline__ void for_bytes(const uint8_t *zb, uint32_t cap, uint32_t o, uint32_t n,
                                          F f) {
  const uint32_t *w = (const uint32_t *)zb;
  const uint32_t last = cap / 4u - 1u, sh = o & 3u;
  uint32_t wi = o >> 2;
  for (uint32_t k = 0; k < n; k += 16, wi += 4) {
    const uint32_t cnt = min(n - k, 16u);
    uint32_t d[5];
#pragma unroll
    for (int t = 0; t < 5; ++t)
      d[t] = 4u * t < sh + cnt ? *gm(w + min(wi + (uint32_t)t, last)) : 0u;
    // bytes o + k + 4t .. + 3 (alignbyte takes the byte offset mod 4), as
    // four named words (an indexed array would live in scratch memory)
    const uint32_t e0 = __builtin_amdgcn_alignbyte(d[1], d[0], sh);
    const uint32_t e1 = __builtin_amdgcn_alignbyte(d[2], d[1], sh);
    const uint32_t e2 = __builtin_amdgcn_alignbyte(d[3], d[2], sh);
    const uint32_t e3 = __builtin_amdgcn_alignbyte(d[4], d[3], sh);
    for (uint32_t j = 0; j < cnt; ++j) {
      const uint32_t v = j < 8 ? (j < 4 ? e0 : e1) : (j < 12 ? e2 : e3);
      f((v >> (8 * (j & 3))) & 0xFFu);
    }
  }
}

// The counting of chunk c of a frame by one wave: the lanes' masks (bit k
// of lane l: bin 64 l + k carries a byte other than 128), bits and
// outliers, and the chunk's bytes compacted into comp in bin order (lane l's
// from comp + rank).  lv: the frame's code lengths (16 per lane), which go to
// len4 (the wave's LDS copy).  Every read stays inside the frame's buffers
// whatever they hold.
struct ChunkCount {
  uint64_t mask;
  uint32_t bits, nout, rank, nz_total, nvalid;
};

template <bool SPARSE>
__device__ __forceinline__ ChunkCount count_chunk(const FramePlan &fp, uint32_t c, uint4 lv,
                                                  uint4 *len4, uint8_t *comp) {
  const int lane = threadIdx.x & 63;
  const uint32_t g0 = c * kChunk + lane * 64u;
  const uint32_t end = min(g0 + 64u, fp.nbins);
  const uint32_t nvalid = end > g0 ? end - g0 : 0u;
  const uint8_t *lens = (const uint8_t *)len4;
  uint64_t mask = 0;
  uint32_t bits = 0, nout = 0, at = 0;
  // one code byte of bin g: to its compacted place, its bits and outliers
  auto take = [&](uint32_t b, uint32_t g) {
    comp[at++] = (uint8_t)b;
    const uint32_t code = b ? b + (kRadius - 128) : code_from_residual(*gm(fp.rbuf + g));
    bits += lens[code];
    nout += code == 0;
  };
  // the bytes of one piece: m its bins (from bin g), o the tile offset of
  // its first byte
  auto piece_bytes = [&](uint32_t g, uint32_t tix, uint64_t m, uint32_t o) {
    for_bytes(fp.zb + (size_t)tix * fp.tile_cap, fp.tile_cap, o, (uint32_t)__builtin_popcountll(m),
              [&](uint32_t b) {
                take(b, g + (uint32_t)__builtin_ctzll(m));
                m &= m - 1;
              });
  };
  // the tile offset of a piece's first byte: the entry's count plus the
  // bytes of the strip's columns before column a
  auto piece_start = [](uint64_t word, uint32_t a, uint32_t zp) {
    return zp + (uint32_t)__builtin_popcountll(word & low_bits(a));
  };
  uint32_t nz_total, rank;
  if (SPARSE || fp.sparse) {
    // a window of 64 bins in a row of at least 64 bins meets at most three
    // strip pieces (the end of one strip, a row's last strip, the next row's
    // first); their words are loaded together
    constexpr int kP = 3;
    uint32_t pg[kP], pa[kP], pt[kP], pnn[kP];
    size_t pe[kP];
    bool short_rows = false;
    {
      // lanes past the frame's last bin walk nothing (pnn = 0)
      BinCursor cu = bin_cursor(fp, min(g0, fp.nbins - 1));
      uint32_t left = nvalid;
#pragma unroll
      for (int i = 0; i < kP; ++i) {
        pg[i] = cu.g;
        pa[i] = cu.J & 63u;
        pt[i] = cursor_tile(fp, cu);
        pe[i] = cursor_entry(fp, cu);
        pnn[i] = left ? cursor_len(fp, cu, left) : 0u;
        if (pnn[i]) cursor_advance(fp, cu, pnn[i]);
        left -= pnn[i];
      }
      // wave-uniform: both ways scan the lanes' counts
      short_rows = __ballot(left != 0) != 0;
    }
    if (short_rows) {
      // rows of fewer than 64 bins: piece by piece, the mask first
      for_pieces(fp, g0, end, [&](uint32_t gg, uint32_t n, uint32_t a, uint32_t, size_t e) {
        mask |= ((*gm(fp.zm + e) >> a) & low_bits(n)) << (gg - g0);
      });
      rank = at = wave_exclusive_scan32((uint32_t)__builtin_popcountll(mask), nz_total);
      len4[lane] = lv;
      wave_sync();   // lengths in LDS
      for_pieces(fp, g0, end, [&](uint32_t gg, uint32_t n, uint32_t a, uint32_t tix, size_t e) {
        const uint64_t word = *gm(fp.zm + e);
        const uint64_t m = (word >> a) & low_bits(n);
        if (m) piece_bytes(gg, tix, m, piece_start(word, a, *gm(fp.zp + e)));
      });
    } else {
      uint64_t w[kP], m[kP];
      uint32_t z[kP], po[kP];
#pragma unroll
      for (int i = 0; i < kP; ++i) {
        w[i] = pnn[i] ? *gm(fp.zm + pe[i]) : 0ull;
        z[i] = pnn[i] ? *gm(fp.zp + pe[i]) : 0u;
      }
#pragma unroll
      for (int i = 0; i < kP; ++i) {
        m[i] = (w[i] >> pa[i]) & low_bits(pnn[i]);
        po[i] = piece_start(w[i], pa[i], z[i]);
        mask |= m[i] << (pg[i] - g0);
      }
      rank = at = wave_exclusive_scan32((uint32_t)__builtin_popcountll(mask), nz_total);
      len4[lane] = lv;
      wave_sync();   // lengths in LDS
#pragma unroll
      for (int i = 0; i < kP; ++i)
        if (m[i]) piece_bytes(pg[i], pt[i], m[i], po[i]);
    }
  } else {
    uint32_t dw[16];   // the lane's 64 bytes (the region holds whole chunks)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint4 q = ld16(fp.codes + g0 + 16 * k);
      dw[4 * k] = q.x;
      dw[4 * k + 1] = q.y;
      dw[4 * k + 2] = q.z;
      dw[4 * k + 3] = q.w;
      const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
      mask |= (uint64_t)non_zero_residuals(w4) << (16 * k);
    }
    mask &= low_bits(nvalid);
    rank = at = wave_exclusive_scan32((uint32_t)__builtin_popcountll(mask), nz_total);
    len4[lane] = lv;
    wave_sync();   // lengths in LDS
#pragma unroll
    for (int q = 0; q < 4; ++q)
      for (uint32_t m = (uint32_t)(mask >> (16 * q)) & 0xFFFFu; m; m &= m - 1) {
        const uint32_t k = (uint32_t)__builtin_ctz(m);
        take(byte_at(dw[4 * q], dw[4 * q + 1], dw[4 * q + 2], dw[4 * q + 3], k), g0 + 16 * q + k);
      }
  }
  bits += (nvalid - (uint32_t)__builtin_popcountll(mask)) * lens[kRadius];
  wave_sync();   // the compacted bytes in LDS (dense bytes: every load of the wave is done)
  ChunkCount cc;
  cc.mask = mask;
  cc.bits = bits;
  cc.nout = nout;
  cc.rank = rank;
  cc.nz_total = nz_total;
  cc.nvalid = nvalid;
  return cc;
}

// The frame and chunk of wave wv of k_count's workgroup slot t: the table
// holds the slot's first chunk; the four chunks of a slot may span frames.
__device__ __forceinline__ void slot_chunk(const BatchPlan &bp, uint32_t t, uint32_t wv,
                                           uint32_t &fw, uint32_t &c) {
  const uint2 fc = bp.count_frame[t];
  fw = fc.x;
  c = fc.y + wv;
  while (c >= bp.frames[fw].nchunks) c -= bp.frames[fw].nchunks, ++fw;
}

template <bool SPARSE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_count(BatchPlan bp) {
  __shared__ uint4 s_len4[kWaves][kNumSym / 16];   // each wave's frame code lengths
  __shared__ __align__(16) uint8_t s_comp[kWaves][kChunk];   // each wave's compacted bytes
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t item = blockIdx.x * kWaves + wv;
  if (item >= bp.total_chunks) {
    // the ROI windows' payload, in the same launch (it needs only k_prep's
    // peak check, and this kernel leaves HBM bandwidth to spare)
    roi_copy(bp, item - bp.total_chunks);
    return;
  }
  uint32_t fw, c;
  slot_chunk(bp, blockIdx.x, (uint32_t)wv, fw, c);
  const FramePlan &fp = bp.frames[fw];
  // the status, the code lengths and (inside) the zero-map words are loaded
  // together; the status gates only what the wave writes
  const bool ok = load_status(fp.st) == RSZ_OK;
  const uint4 lv = ((const uint4 *)fp.st->lens)[lane];
  uint8_t *comp = s_comp[wv];
  const ChunkCount cc = count_chunk<SPARSE>(fp, c, lv, s_len4[wv], comp);
  if (!ok) return;   // a frame that failed earlier (k_tail reports it)
  *gm(fp.cmask + (size_t)c * 64 + lane) = cc.mask;
  *gm(fp.lanecnt + (size_t)c * 64 + lane) = cc.bits | cc.nout << 16;
  // whole 16-byte groups (the chunk's region holds 4096 bytes; bytes past
  // nz_total are not read)
  uint8_t *dst = fp.codes + (size_t)c * kChunk;
  for (uint32_t k = 16u * lane; k < cc.nz_total; k += 1024u)
    *gm((u32x4 *)(dst + k)) = *(const u32x4 *)(comp + k);
  uint32_t bits = cc.bits, nout = cc.nout;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    bits += __shfl_xor(bits, d);
    nout += __shfl_xor(nout, d);
  }
  if (lane == 0) {
    fp.chunk_off[c] = bits;
    fp.chunk_oo[c] = nout;
  }
}

// ----------------------------------------------------------------- k_scan

// Exclusive scans of the chunk counts of a frame: chunk bit offsets, chunk
// outlier offsets, and the frame totals.
__global__ __launch_bounds__(256) void k_scan(BatchPlan bp) {
  const FramePlan &fp = bp.frames[blockIdx.x];
  FrameState *st = fp.st;
  __shared__ uint64_t s_tmp[4];
  __shared__ int s_ok;
  if (threadIdx.x == 0) s_ok = load_status(st) == RSZ_OK;
  __syncthreads();
  if (!s_ok) return;
  uint64_t carry = 0;
  for (uint32_t base = 0; base < fp.nchunks; base += 256) {
    const uint32_t c = base + threadIdx.x;
    const uint64_t v = c < fp.nchunks ? (((uint64_t)fp.chunk_oo[c] << 32) | fp.chunk_off[c]) : 0;
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<uint64_t>(v, s_tmp, tot) + carry;
    if (c < fp.nchunks) {
      fp.chunk_off[c] = (uint32_t)ex;
      fp.chunk_oo[c] = (uint32_t)(ex >> 32);
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    st->T = (uint32_t)carry;
    st->n_out = (uint32_t)(carry >> 32);
  }
}

// --------------------------------------------------------------- k_encode

// One workgroup per run of bp.cpw consecutive chunks of a frame; its four
// waves take every fourth chunk, each chunk's bit and outlier offsets come
// from k_scan, so nothing waits across waves.  The chunk's codes come in the
// chunk form of k_count.  When residual 0's codeword is all zeros (the
// canonical code gives it the first codeword whenever it is the only
// shortest symbol) and the chunk's bits fit the wave's LDS words, only the
// bins with other codes are placed: lane i takes the chunk's i-th such bin,
// its position is the bins before it times residual 0's length plus the
// extra length of the other codes before it (a wave scan), and its codeword
// is ORed into the zeroed LDS words, which are stored whole.  Otherwise the
// wave packs the chunk in four rounds of 1024 symbols (16 per lane): a wave
// scan places each lane's bits, the codewords are ORed into the wave's LDS
// words, and the complete words are stored whole; the round's last partial
// word carries into the next.  A chunk's first word, when it starts
// mid-word, is shared with the previous chunk and goes to head[] for k_tail
// to merge.  The words go to fp.bw: the stream's bitstream section, or a
// workspace buffer when the run stage codes them (whose kernels take a
// chunk's first word from head[] themselves).
// Bytes [off, off + 16) of p (p 16-byte aligned, with 32 readable bytes
// from off rounded down to 16): two aligned loads and a byte alignment.
__device__ __forceinline__ void load16_at(const uint8_t *p, uint32_t off, uint32_t (&y)[4]) {
  const uint4 lo = ld16(p + (off & ~15u));
  const uint4 hi = ld16(p + (off & ~15u) + 16);
  const uint32_t x[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
  const uint32_t q = (off >> 2) & 3u, r = off & 3u;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint32_t u = x[i], w = x[i + 1];
#pragma unroll
    for (int t = 1; t < 4; ++t)
      if (q == (uint32_t)t) {
        u = x[i + t];
        w = x[i + t + 1];
      }
    y[i] = __builtin_amdgcn_alignbyte(w, u, r);
  }
}

// The 16 code bytes of bins [16 i, 16 i + 16) of a chunk from its chunk form:
// m (16 bits), the bins whose byte is not 128; their bytes in bin order from
// cb + rank (the region holds 32 bytes past every chunk).
__device__ __forceinline__ uint4 expand16(const uint8_t *cb, uint32_t m, uint32_t rank) {
  uint32_t w[4] = {0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u};
  if (m) {
    uint32_t y[4];
    load16_at(cb, rank, y);
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if ((m >> k) & 1u) {
        w[k >> 2] = (w[k >> 2] & ~(0xFFu << (8 * (k & 3)))) | ((y[0] & 0xFFu) << (8 * (k & 3)));
        y[0] = __builtin_amdgcn_alignbyte(y[1], y[0], 1);
        y[1] = __builtin_amdgcn_alignbyte(y[2], y[1], 1);
        y[2] = __builtin_amdgcn_alignbyte(y[3], y[2], 1);
        y[3] >>= 8;
      }
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Position of the set bit of x with j set bits below it (x has more than j).
__device__ __forceinline__ uint32_t select_bit(uint64_t x, uint32_t j) {
  uint32_t w = (uint32_t)x, pos = 0;
  const uint32_t c = __builtin_popcount(w);
  if (j >= c) {
    j -= c;
    w = (uint32_t)(x >> 32);
    pos = 32;
  }
#pragma unroll
  for (uint32_t half = 16; half; half >>= 1) {
    const uint32_t cl = __builtin_popcount(w & ((1u << half) - 1u));
    if (j >= cl) {
      j -= cl;
      w >>= half;
      pos += half;
    }
  }
  return pos;
}

// ORs the L-bit codeword cw (L >= 1) into the staged words at bit p.
__device__ __forceinline__ void or_codeword(uint32_t *stg, uint32_t p, uint32_t cw, uint32_t L) {
  const uint64_t v = ((uint64_t)cw << (64 - L)) >> (p & 31);
  if (v >> 32) atomicOr(&stg[p >> 5], (uint32_t)(v >> 32));
  if ((uint32_t)v) atomicOr(&stg[(p >> 5) + 1], (uint32_t)v);
}

constexpr int kRoundSyms = 1024;
__global__ __launch_bounds__(256) void k_encode(BatchPlan bp) {
  __shared__ uint8_t s_len[kNumSym];
  __shared__ uint32_t s_cw[kNumSym];
  __shared__ uint32_t s_words[kWaves][kRoundSyms + 1];   // 32 bits per symbol at most
  __shared__ int s_ok;
  const uint32_t f = bp.unit_frame[blockIdx.x];
  const FramePlan &fp = bp.frames[f];
  const FrameState *st = fp.st;
  if (threadIdx.x == 0) s_ok = load_status(st) == RSZ_OK;
  __syncthreads();
  if (!s_ok) return;
  for (int s = threadIdx.x; s < kNumSym; s += 256) {
    s_len[s] = st->lens[s];
    s_cw[s] = st->cw[s];
  }
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t *stg = s_words[wv];
  for (int k = lane; k <= kRoundSyms; k += 64) stg[k] = 0u;
  __syncthreads();   // tables loaded
  const uint32_t c0 = (blockIdx.x - bp.unit_prefix[f]) * bp.cpw;
  const uint32_t c1 = min(c0 + bp.cpw, fp.nchunks);
  uint8_t *o = fp.out;
  const uint64_t cap = fp.out_cap;
  uint32_t *bw = fp.bw;
  const uint64_t bcap = fp.bw_cap;
  for (uint32_t lc = c0 + wv; lc < c1; lc += kWaves) {
    const uint32_t S0 = fp.chunk_off[lc];
    uint32_t oi = fp.chunk_oo[lc];
    if (lane == 0 && fp.off_chunks + 4ull * lc + 4 <= cap)
      *(uint32_t *)(o + fp.off_chunks + 4ull * lc) = S0;
    uint32_t pos = S0 & 31;     // bit position in stg[0]
    uint64_t widx = S0 >> 5;    // stream word of stg[0]
    bool first = (S0 & 31) != 0;
    // the chunk form: lane j holds mask word j and the bytes before it
    const uint8_t *cbytes = fp.codes + (size_t)lc * kChunk;
    const uint64_t mword = *gm(fp.cmask + (size_t)lc * 64 + lane);
    const uint32_t lc_lane = *gm(fp.lanecnt + (size_t)lc * 64 + lane);
    uint32_t nz_total;
    const uint32_t wr = wave_exclusive_scan32((uint32_t)__builtin_popcountll(mword), nz_total);
    const uint32_t nbits = (lc + 1 < fp.nchunks ? fp.chunk_off[lc + 1] : (uint32_t)st->T) - S0;
    const uint32_t L0 = s_len[kRadius];
    if (s_cw[kRadius] == 0 && L0 && pos + nbits <= 32u * kRoundSyms) {
      // residual 0's codeword is all zeros, so its bins only advance the
      // position: lane j places the codewords of its own bins [64 j, 64 j +
      // 64) from its first bit, pb (the bits of the lanes before it, which
      // k_count counted), and its outliers from its first outlier slot
      const uint32_t nw = (pos + nbits + 31) >> 5;
      uint32_t tb, to;
      const uint32_t pb = pos + wave_exclusive_scan32(lc_lane & 0xFFFFu, tb);
      uint32_t oq = oi + wave_exclusive_scan32(lc_lane >> 16, to);
      const uint32_t gl = lc * kChunk + (uint32_t)lane * 64u;
      uint64_t m = mword;
      uint32_t extra = 0;
      for_bytes(cbytes, kChunk, wr, (uint32_t)__builtin_popcountll(m), [&](uint32_t b) {
        const uint32_t k = (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        const uint32_t g = gl + k;
        const uint32_t code = b ? b + (kRadius - 128) : code_from_residual(*gm(fp.rbuf + g));
        const uint32_t L = s_len[code];
        or_codeword(stg, pb + k * L0 + extra, s_cw[code], L);
        extra += L - L0;
        if (code == 0) {
          if (oq < fp.nbins) *gm(fp.obuf + oq) = g;
          ++oq;
        }
      });
      wave_sync();
      for (uint32_t k = lane; k < nw; k += 64) {
        const uint32_t v = stg[k];
        stg[k] = 0u;
        if (k == 0 && first) fp.head[lc] = v;
        else if (widx + k < bcap) *gm(bw + widx + k) = v;
      }
      wave_sync();
      continue;
    }
#pragma unroll 1
    for (int r = 0; r < kChunk / kRoundSyms; ++r) {
      const uint32_t g0 = lc * kChunk + r * kRoundSyms + lane * 16;
      const uint32_t wi = (uint32_t)r * 16 + (lane >> 2), sh = (lane & 3) * 16;
      const uint64_t wm = __shfl(mword, (int)wi);
      const uint4 nx = expand16(cbytes, (uint32_t)(wm >> sh) & 0xFFFFu,
                                (uint32_t)__shfl((int)wr, (int)wi) +
                                    (uint32_t)__builtin_popcountll(wm & low_bits(sh)));
      const uint32_t w4[4] = {nx.x, nx.y, nx.z, nx.w};
      // fast path, the common case: a whole round with no escape byte in the
      // wave, so every code is its byte + 384 and there is no outlier
      uint32_t zero = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) zero |= (w4[e] - 0x01010101u) & ~w4[e] & 0x80808080u;
      if ((lc * kChunk + (r + 1) * kRoundSyms) <= fp.nbins && __ballot(zero != 0) == 0) {
        const uint8_t *lb = s_len + (kRadius - 128);
        const uint32_t *cb = s_cw + (kRadius - 128);
        const uint32_t nz = non_zero_residuals(w4);
        uint32_t tot;
        if (cb[128] == 0 && __ballot(__builtin_popcount(nz) > kSparseBytes) == 0) {
          // residual 0's codeword is all zeros: its bins only advance the
          // position; the few other bytes are placed from their index
          const uint32_t L0 = lb[128];
          uint32_t bits = 16 * L0;
          for (uint32_t m = nz; m; m &= m - 1) bits += lb[byte_at(w4[0], w4[1], w4[2], w4[3], __builtin_ctz(m))] - L0;
          const uint32_t p0 = pos + wave_exclusive_scan32(bits, tot);
          uint32_t extra = 0;
          for (uint32_t m = nz; m; m &= m - 1) {
            const uint32_t k = __builtin_ctz(m), b = byte_at(w4[0], w4[1], w4[2], w4[3], k), L = lb[b];
            const uint32_t p = p0 + k * L0 + extra;
            const uint64_t v = ((uint64_t)cb[b] << (64 - L)) >> (p & 31);
            if (v >> 32) atomicOr(&stg[p >> 5], (uint32_t)(v >> 32));
            if ((uint32_t)v) atomicOr(&stg[(p >> 5) + 1], (uint32_t)v);
            extra += L - L0;
          }
        } else {
          uint32_t bits = 0;
#pragma unroll
          for (int k = 0; k < 16; ++k) bits += lb[(w4[k >> 2] >> (8 * (k & 3))) & 0xFFu];
          uint32_t p = pos + wave_exclusive_scan32(bits, tot);
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const uint32_t b = (w4[k >> 2] >> (8 * (k & 3))) & 0xFFu;
            const uint32_t L = lb[b];
            const uint64_t v = ((uint64_t)cb[b] << (64 - L)) >> (p & 31);
            if (v >> 32) atomicOr(&stg[p >> 5], (uint32_t)(v >> 32));
            if ((uint32_t)v) atomicOr(&stg[(p >> 5) + 1], (uint32_t)v);
            p += L;
          }
        }
        wave_sync();
        const uint32_t end = pos + tot;   // bits in stg
        const uint32_t nw = end >> 5;     // complete words
        for (uint32_t k = lane; k < nw; k += 64) {
          const uint32_t v = stg[k];
          if (k == 0 && first) {
            fp.head[lc] = v;
            continue;
          }
          if (widx + k < bcap) *gm(bw + widx + k) = v;
        }
        if (nw) first = false;
        const uint32_t carry = stg[nw];
        wave_sync();
        for (uint32_t k = lane; k <= nw; k += 64) stg[k] = k == 0 ? carry : 0u;
        wave_sync();
        pos = end & 31;
        widx += nw;
        continue;
      }
      uint32_t code[16];
      uint32_t bits = 0, nout = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const uint32_t g = g0 + k;
        const uint32_t b = (w4[k >> 2] >> (8 * (k & 3))) & 0xFFu;
        code[k] = g < fp.nbins ? b + (kRadius - 128) : 0xFFFFu;
        if (g < fp.nbins && b == 0) code[k] = code_from_residual(*gm(fp.rbuf + g));
        if (g < fp.nbins) {
          bits += s_len[code[k]];
          nout += code[k] == 0;
        }
      }
      uint64_t tot;
      const uint64_t ex = wave_exclusive_scan(((uint64_t)nout << 32) | bits, tot);
      uint32_t p = pos + (uint32_t)ex;
      uint32_t q = oi + (uint32_t)(ex >> 32);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (code[k] == 0xFFFFu) continue;
        const uint32_t L = s_len[code[k]];
        const uint64_t v = ((uint64_t)s_cw[code[k]] << (64 - L)) >> (p & 31);
        atomicOr(&stg[p >> 5], (uint32_t)(v >> 32));
        if ((p & 31) + L > 32) atomicOr(&stg[(p >> 5) + 1], (uint32_t)v);
        p += L;
        if (code[k] == 0) {
          if (q < fp.nbins) *gm(fp.obuf + q) = g0 + k;
          q++;
        }
      }
      wave_sync();
      const uint32_t end = pos + (uint32_t)tot;   // bits in stg
      const uint32_t nw = end >> 5;               // complete words
      for (uint32_t k = lane; k < nw; k += 64) {
        const uint32_t v = stg[k];
        if (k == 0 && first) {
          fp.head[lc] = v;
          continue;
        }
        if (widx + k < bcap) *gm(bw + widx + k) = v;
      }
      if (nw) first = false;
      const uint32_t carry = stg[nw];
      wave_sync();
      for (uint32_t k = lane; k <= nw; k += 64) stg[k] = k == 0 ? carry : 0u;
      wave_sync();
      pos = end & 31;
      widx += nw;
      oi += (uint32_t)(tot >> 32);
    }
    // the chunk's last, partial word: this chunk owns it (the next chunk's
    // bits in it arrive through head[])
    if (pos) {
      const uint32_t v = stg[0];
      if (lane == 0) {
        if (first) fp.head[lc] = v;
        else if (widx < bcap) *gm(bw + widx) = v;
      }
    }
    wave_sync();
    if (lane == 0) stg[0] = 0u;
    wave_sync();
  }
}

// ----------------------------------------------------------------- k_tail

__device__ __forceinline__ void put_u32(uint8_t *o, uint64_t off, uint32_t v) {
  *(uint32_t *)(o + off) = v;
}

__global__ __launch_bounds__(256) void k_tail(BatchPlan bp) {
  const FramePlan &fp = bp.frames[blockIdx.x];
  FrameState *st = fp.st;
  __shared__ int32_t s_status;
  if (threadIdx.x == 0) s_status = load_status(st);
  __syncthreads();
  if (s_status != RSZ_OK) {
    if (threadIdx.x == 0) {
      *fp.res_status = s_status;
      *fp.res_bytes = 0;
    }
    return;
  }
  const uint64_t T = st->T;
  const uint32_t n_out = st->n_out;
  const uint64_t nwords = (T + 31) / 32;
  // with the runs coded the bitstream is not in the stream
  const uint64_t off_oidx = fp.off_bits + (fp.run_coding ? 0 : 4 * nwords);
  const uint64_t off_ores = off_oidx + 4ull * n_out;
  // coded ROI: its section follows the outliers
  const uint64_t Troi = fp.roi_coding ? st->Troi : 0;
  const uint64_t off_rsec = off_ores + 4ull * n_out;
  const uint64_t off_rbits = off_rsec + kRoiLens + 4ull * fp.npeaks;
  const uint64_t end_roi = fp.roi_coding ? off_rbits + 4 * ((Troi + 31) / 32) : off_rsec;
  // run section: parameters, offsets, run bits -- the end of the stream
  const uint64_t Trun = fp.run_coding ? fp.run_off[fp.nchunks] : 0;
  const uint64_t off_runoffs = end_roi + align_up(fp.nchunks, 4);
  const uint64_t off_runbits = off_runoffs + 4ull * (fp.nchunks + 1);
  const uint64_t total = fp.run_coding ? off_runbits + 4 * ((Trun + 31) / 32) : end_roi;
  const bool fits = total <= fp.out_cap;
  __syncthreads();
  if (threadIdx.x == 0) {
    st->total = total;
    st->off_runbits = off_runbits;
    if (!fits) st->status = RSZ_ERR_CAPACITY;
    *fp.res_status = fits ? RSZ_OK : RSZ_ERR_CAPACITY;
    *fp.res_bytes = total;
  }
  if (!fits) return;
  uint8_t *o = fp.out;
  if (threadIdx.x == 0) {
    put_u32(o, 0, 0x315A5352u);  // "RSZ1"
    // version 1; flags: bit 0 bin_mode, bits 1-2 the Lorenzo dimension (0 for
    // 2), bit 3 the ROI coded, bit 4 the runs coded
    const uint32_t flags = (fp.mode & 1u) | ((fp.dim == 2 ? 0u : fp.dim) << 1) |
                           ((fp.roi_coding & 1u) << 3) | ((fp.run_coding & 1u) << 4);
    put_u32(o, 4, 1u | (flags << 16));
    put_u32(o, 8, fp.P);
    put_u32(o, 12, fp.H);
    put_u32(o, 16, fp.W);
    put_u32(o, 20, fp.w);
    put_u32(o, 24, fp.b);
    put_u32(o, 28, (uint32_t)kRadius);
    const uint64_t ebits = __double_as_longlong(fp.eb);
    put_u32(o, 32, (uint32_t)ebits);
    put_u32(o, 36, (uint32_t)(ebits >> 32));
    put_u32(o, 40, fp.npeaks);
    put_u32(o, 44, n_out);
    put_u32(o, 48, kChunk);
    put_u32(o, 52, fp.nchunks);
    put_u32(o, 56, (uint32_t)T);
    put_u32(o, 60, (uint32_t)(T >> 32));
    put_u32(o, 64, (uint32_t)total);
    put_u32(o, 68, (uint32_t)(total >> 32));
    put_u32(o, 72, (uint32_t)Troi);
    put_u32(o, 76, (uint32_t)(Troi >> 32));
  }
  if (fp.roi_coding) {
    // class code lengths (padded), window bit offsets, zeroed ROI words that
    // k_roi_pack ORs the codes into
    for (uint32_t c = threadIdx.x; c < kRoiLens; c += 256)
      o[off_rsec + c] = c < (uint32_t)kRoiClasses ? fp.roi_lens[c] : 0;
    uint32_t *roffs = (uint32_t *)(o + off_rsec + kRoiLens);
    for (uint32_t k = threadIdx.x; k < fp.npeaks; k += 256) roffs[k] = fp.roi_bits[k];
    uint32_t *rw = (uint32_t *)(o + off_rbits);
    for (uint64_t t = threadIdx.x; t < (Troi + 31) / 32; t += 256) rw[t] = 0u;
  }
  // peaks as u16 triples, padded with zeros to 4 bytes
  uint16_t *pk = (uint16_t *)(o + kHeader);
  for (uint32_t e = threadIdx.x; e < 3 * fp.npeaks; e += 256) pk[e] = (uint16_t)fp.peaks[e];
  if (threadIdx.x == 0 && (3 * fp.npeaks) % 2) pk[3 * fp.npeaks] = 0;
  for (int s = threadIdx.x; s < kNumSym; s += 256) o[fp.off_lens + s] = st->lens[s];
  if (fp.run_coding) {
    // Rice parameters (padded with zeros to 4 bytes), chunk bit offsets and
    // the section's bits, zeroed run words that k_run_pack ORs the codes into
    for (uint32_t c = threadIdx.x; c < align_up(fp.nchunks, 4); c += 256)
      o[end_roi + c] = c < fp.nchunks ? fp.run_k[c] : 0;
    uint32_t *ro = (uint32_t *)(o + off_runoffs);
    for (uint32_t c = threadIdx.x; c <= fp.nchunks; c += 256) ro[c] = fp.run_off[c];
    uint32_t *rw = (uint32_t *)(o + off_runbits);
    for (uint64_t t = threadIdx.x; t < (Trun + 31) / 32; t += 256) rw[t] = 0u;
  } else {
    // chunk boundary words: previous chunk's bits (stored by it) | this chunk's
    uint32_t *bw = (uint32_t *)(o + fp.off_bits);
    for (uint32_t c = threadIdx.x; c < fp.nchunks; c += 256) {
      const uint32_t S0 = fp.chunk_off[c];
      if (S0 & 31) bw[S0 >> 5] |= fp.head[c];
    }
  }
  uint32_t *oidx = (uint32_t *)(o + off_oidx);
  int32_t *ores = (int32_t *)(o + off_ores);
  for (uint32_t k = threadIdx.x; k < n_out; k += 256) {
    const uint32_t g = fp.obuf[k];
    oidx[k] = g;
    ores[k] = fp.rbuf[g];
  }
}

// ------------------------------------------------------ coded ROI windows

// Lossless coding of the ROI windows (in place of the paper's fpzip, Sec.
// IV): a window's payload words b (0 outside the panel) map to
// order-preserving integers M (b | 2^31 for positive floats, ~b for
// negative), predicted by the 2D Lorenzo predictor over the window with M =
// 2^31 (mapped +0.0) outside it.  The zigzag residual z has class c = its bit
// length (0..32), Huffman coded per frame, then its c - 1 low bits.  Every
// value's residual depends only on the payload, so all are computed in
// parallel: k_roi_classes (class histogram), k_roi_book (the code, by the
// same block function as the main code), k_roi_count and k_roi_scan (window
// bit offsets), then, after k_tail has checked the size and zeroed the
// words, k_roi_pack.  One wave per window.
struct RoiWin {
  const float *src;
  int64_t r0, c0, H, W;
};

__device__ __forceinline__ uint32_t roi_fmap(uint32_t b) {
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ uint32_t roi_word(const RoiWin &rw, int64_t u, int64_t v) {
  const int64_t i = rw.r0 + u, j = rw.c0 + v;
  return (i >= 0 && i < rw.H && j >= 0 && j < rw.W) ? __float_as_uint(rw.src[i * rw.W + j]) : 0u;
}
__device__ __forceinline__ uint32_t roi_z(const RoiWin &rw, int64_t u, int64_t v) {
  const uint32_t zero = 0x80000000u;
  const uint32_t m = roi_fmap(roi_word(rw, u, v));
  const uint32_t up = u > 0 ? roi_fmap(roi_word(rw, u - 1, v)) : zero;
  const uint32_t left = v > 0 ? roi_fmap(roi_word(rw, u, v - 1)) : zero;
  const uint32_t ul = (u > 0 && v > 0) ? roi_fmap(roi_word(rw, u - 1, v - 1)) : zero;
  const int32_t r = (int32_t)(m - (up + left - ul));
  return ((uint32_t)r << 1) ^ (uint32_t)(r >> 31);
}
__device__ __forceinline__ uint32_t roi_class(uint32_t z) { return z ? 32u - __clz(z) : 0u; }

// Windows up to kRoiStageW pixels wide are staged in LDS, one wave per
// window: the mapped values at row stride w + 1 after a border row and column
// of mapped +0.0 (the predictor's value outside the window), loaded
// kRoiSlots per lane before any is stored.  A residual then takes four LDS
// reads instead of four global loads.  Wider windows read the frame directly.
constexpr uint32_t kRoiStageW = 31;
constexpr uint32_t kRoiStageWords = (kRoiStageW + 1) * (kRoiStageW + 1);
struct RoiVals {
  RoiWin rw;
  const uint32_t *s;   // the staged values, or null
  uint32_t st;         // their row stride
  __device__ uint32_t z(uint32_t u, uint32_t v) const {
    if (!s) return roi_z(rw, u, v);
    const uint32_t *p = s + (u + 1) * st + (v + 1);
    const int32_t r = (int32_t)(p[0] - (p[-(int)st] + p[-1] - p[-(int)st - 1]));
    return ((uint32_t)r << 1) ^ (uint32_t)(r >> 31);
  }
};

__device__ __forceinline__ void roi_stage(const RoiWin &rw, uint32_t w, uint32_t *buf,
                                          RoiVals &rv) {
  rv.rw = rw;
  rv.s = nullptr;
  if (w > kRoiStageW) return;
  const int lane = threadIdx.x & 63;
  const uint32_t st = w + 1, ww = w * w, M = 0xFFFFFFFFu / w + 1u;
  for (uint32_t e = lane; e < st; e += 64) {
    buf[e] = 0x80000000u;
    buf[e * st] = 0x80000000u;
  }
  for (uint32_t e0 = 0; e0 < ww; e0 += 64 * kRoiSlots) {
    uint32_t val[kRoiSlots];
#pragma unroll
    for (uint32_t t = 0; t < kRoiSlots; ++t) {
      const uint32_t e = e0 + 64 * t + lane;
      const uint32_t u = __umulhi(e, M), v = e - u * w;
      val[t] = e < ww ? roi_fmap(roi_word(rw, u, v)) : 0u;
    }
#pragma unroll
    for (uint32_t t = 0; t < kRoiSlots; ++t) {
      const uint32_t e = e0 + 64 * t + lane;
      const uint32_t u = __umulhi(e, M), v = e - u * w;
      if (e < ww) buf[(u + 1) * st + v + 1] = val[t];
    }
  }
  wave_sync();
  rv.s = buf;
  rv.st = st;
}

// The window of global peak kg if its frame codes the ROI and is still fine.
__device__ __forceinline__ bool roi_window(const BatchPlan &bp, uint32_t kg, uint32_t &f,
                                           uint32_t &k, RoiWin &rw) {
  f = bp.peak_frame[kg];
  const FramePlan &fp = bp.frames[f];
  if (!fp.roi_coding || load_status(fp.st) != RSZ_OK) return false;
  k = kg - bp.peak_prefix[f];
  const int64_t pa = fp.peaks[3 * k], h = fp.w / 2;
  if (pa < 0 || pa >= fp.P) return false;
  rw.src = fp.frame + (size_t)pa * fp.H * fp.W;
  rw.r0 = fp.peaks[3 * k + 1] - h;
  rw.c0 = fp.peaks[3 * k + 2] - h;
  rw.H = fp.H;
  rw.W = fp.W;
  return true;
}

__global__ __launch_bounds__(256) void k_roi_classes(BatchPlan bp) {
  __shared__ uint32_t s_h[kWaves][kRoiClasses];
  __shared__ uint32_t s_v[kWaves][kRoiStageWords];
  const int lane = threadIdx.x & 63;
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t kg = blockIdx.x * kWaves + wv;
  if (kg >= bp.total_peaks) return;
  uint32_t f, k;
  RoiWin rw;
  if (!roi_window(bp, kg, f, k, rw)) return;
  const FramePlan &fp = bp.frames[f];
  const uint32_t w = fp.w, ww = w * w, M = 0xFFFFFFFFu / w + 1u;
  for (int c = lane; c < kRoiClasses; c += 64) s_h[wv][c] = 0u;
  RoiVals rv;
  roi_stage(rw, w, s_v[wv], rv);
  wave_sync();
  for (uint32_t e = lane; e < ww; e += 64) {
    const uint32_t u = __umulhi(e, M), v = e - u * w;
    atomicAdd(&s_h[wv][roi_class(rv.z(u, v))], 1u);
  }
  wave_sync();
  for (int c = lane; c < kRoiClasses; c += 64)
    if (s_h[wv][c]) atomicAdd(&fp.roi_hist[c], s_h[wv][c]);
}

__global__ __launch_bounds__(256) void k_roi_book(BatchPlan bp) {
  const FramePlan &fp = bp.frames[blockIdx.x];
  if (!fp.roi_coding) return;   // the same frame for the whole workgroup
  build_code(fp.st, fp.roi_hist, fp.roi_lens, fp.roi_cw);
}

// Bits of each window (class codeword + raw bits of every value).
__global__ __launch_bounds__(256) void k_roi_count(BatchPlan bp) {
  __shared__ uint32_t s_v[kWaves][kRoiStageWords];
  const int lane = threadIdx.x & 63;
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t kg = blockIdx.x * kWaves + wv;
  if (kg >= bp.total_peaks) return;
  uint32_t f, k;
  RoiWin rw;
  if (!roi_window(bp, kg, f, k, rw)) return;
  const FramePlan &fp = bp.frames[f];
  const uint32_t w = fp.w, ww = w * w, M = 0xFFFFFFFFu / w + 1u;
  // class c costs its code length plus c - 1 raw bits; lane c holds it
  const uint32_t cost = lane < kRoiClasses ? fp.roi_lens[lane] + (lane >= 2 ? lane - 1 : 0) : 0u;
  RoiVals rv;
  roi_stage(rw, w, s_v[wv], rv);
  uint32_t bits = 0;
  for (uint32_t e0 = 0; e0 < ww; e0 += 64) {   // every lane takes part in the shuffle
    const uint32_t e = e0 + lane;
    uint32_t c = 0;
    if (e < ww) {
      const uint32_t u = __umulhi(e, M), v = e - u * w;
      c = roi_class(rv.z(u, v));
    }
    const uint32_t x = __shfl(cost, (int)c);
    if (e < ww) bits += x;
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) bits += __shfl_xor(bits, d);
  if (lane == 0) fp.roi_bits[k] = bits;   // < 2^26 * 63 / npeaks
}

// Window bits -> bit offsets (exclusive scan), and the frame's ROI bits.
__global__ __launch_bounds__(256) void k_roi_scan(BatchPlan bp) {
  __shared__ uint32_t s_tmp[4];
  const FramePlan &fp = bp.frames[blockIdx.x];
  if (!fp.roi_coding || load_status(fp.st) != RSZ_OK) return;   // uniform
  uint32_t carry = 0;   // npeaks * w^2 <= 2^26 bounds the total below 2^32
  for (uint32_t k0 = 0; k0 < fp.npeaks; k0 += 256) {
    const uint32_t k = k0 + threadIdx.x;
    const uint32_t v = k < fp.npeaks ? fp.roi_bits[k] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t>(v, s_tmp, tot);
    if (k < fp.npeaks) fp.roi_bits[k] = carry + ex;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) fp.st->Troi = carry;
}

// Writes the n-bit value (n <= 63) MSB-first at bit pos of words (zeroed).
__device__ __forceinline__ void or_bits(uint32_t *words, uint64_t pos, uint64_t value, uint32_t n) {
  uint64_t wi = pos >> 5;
  uint32_t s = (uint32_t)(pos & 31);
  int rem = (int)n;
  while (rem > 0) {
    const int take = min(rem, 32 - (int)s);
    const uint32_t piece = (uint32_t)((value >> (rem - take)) & ((1ull << take) - 1));
    if (piece) atomicOr(&words[wi], piece << (32 - s - take));
    rem -= take;
    wi++;
    s = 0;
  }
}

// The window's bits go to an LDS buffer of kRoiOutWords words when they fit
// (ORed in there, then stored as whole words: the first and last by atomicOr,
// shared with the neighbouring windows), else straight into the stream.
constexpr uint32_t kRoiOutWords = 512;
__global__ __launch_bounds__(256) void k_roi_pack(BatchPlan bp) {
  __shared__ uint32_t s_v[kWaves][kRoiStageWords];
  __shared__ uint32_t s_o[kWaves][kRoiOutWords];
  const int lane = threadIdx.x & 63;
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t kg = blockIdx.x * kWaves + wv;
  if (kg >= bp.total_peaks) return;
  uint32_t f, k;
  RoiWin rw;
  if (!roi_window(bp, kg, f, k, rw)) return;
  const FramePlan &fp = bp.frames[f];
  const FrameState *st = fp.st;
  const uint64_t off_ores =
      fp.off_bits + (fp.run_coding ? 0 : 4 * ((st->T + 31) / 32)) + 4ull * st->n_out;
  uint32_t *words =
      (uint32_t *)(fp.out + off_ores + 4ull * st->n_out + kRoiLens + 4ull * fp.npeaks);
  const uint32_t w = fp.w, ww = w * w, M = 0xFFFFFFFFu / w + 1u;
  const uint32_t len = lane < kRoiClasses ? fp.roi_lens[lane] : 0u;
  const uint32_t cwd = lane < kRoiClasses ? fp.roi_cw[lane] : 0u;
  const uint64_t start = fp.roi_bits[k];
  const uint64_t end = k + 1 < fp.npeaks ? fp.roi_bits[k + 1] : st->Troi;
  // the staging buffer's word 0 is stream word start / 32
  const uint64_t w0 = start >> 5;
  const bool staged = ((end + 31) >> 5) - w0 <= kRoiOutWords;
  uint32_t *ob = s_o[wv];
  if (staged)
    for (uint32_t i = lane; i < kRoiOutWords; i += 64) ob[i] = 0u;
  RoiVals rv;
  roi_stage(rw, w, s_v[wv], rv);
  uint32_t *dst = staged ? ob : words;
  uint64_t base = start - (staged ? 32 * w0 : 0);
  for (uint32_t e0 = 0; e0 < ww; e0 += 64) {
    const uint32_t e = e0 + lane;
    uint32_t z = 0, c = 0;
    if (e < ww) {
      const uint32_t u = __umulhi(e, M), v = e - u * w;
      z = rv.z(u, v);
      c = roi_class(z);
    }
    const uint32_t extra = c >= 2 ? c - 1 : 0u;
    const uint32_t cl = __shfl(len, (int)c), cc = __shfl(cwd, (int)c);
    const uint32_t n = e < ww ? cl + extra : 0u;
    const uint64_t value = ((uint64_t)cc << extra) | (extra ? (z & ((1u << extra) - 1u)) : 0u);
    uint64_t tot;
    const uint64_t ex = wave_exclusive_scan(n, tot);
    if (n) or_bits(dst, base + ex, value, n);
    base += tot;
  }
  if (staged) {
    wave_sync();
    const uint32_t nw = (uint32_t)(((end + 31) >> 5) - w0);
    for (uint32_t i = lane; i < nw; i += 64) {
      const uint32_t v = ob[i];
      if (i == 0 || i + 1 == nw) {
        if (v) atomicOr(&words[w0 + i], v);
      } else {
        words[w0 + i] = v;
      }
    }
  }
}

// ------------------------------------------------------------ run stage

// A lossless stage after the Huffman coder: per 4096-symbol chunk, the
// lengths r of the zero runs before each one bit of the chunk's Huffman bits
// are Rice coded with the chunk's parameter k (r >> k one bits, a zero, the
// k low bits of r, MSB-first); zeros after the last one are implied by the
// chunk's end.  k in 0..kRunKMax minimises the chunk's bits, the smallest on
// ties.  One wave per chunk, lanes on consecutive words of its bits.
constexpr uint32_t kRunKMax = 20;

// Word i of the Huffman bits as chunk c sees it: a chunk that starts
// mid-word has its share of that word in head[c] (the word in bw holds the
// previous chunk's bits); every other word of the chunk holds its bits only
// (a later chunk's bits in its last word go to that chunk's head).
__device__ __forceinline__ uint32_t chunk_word(const FramePlan &fp, uint32_t c, uint32_t S0,
                                               uint32_t i) {
  return (i == (S0 >> 5) && (S0 & 31)) ? fp.head[c] : fp.bw[i];
}

// Inclusive max over the lanes of a wave.
__device__ __forceinline__ uint32_t wave_max_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(v, d);
    if (lane >= d) v = max(v, y);
  }
  return v;
}

// A chunk's Huffman bits [S0, S1), words w0 .. w1 - 1, walked in blocks of
// 64 words (lane l on word base + l).  The first kRunPre blocks are loaded
// up front (their loads in flight together); later blocks, rare, load as
// they come.
constexpr int kRunPre = 4;
struct RunChunk {
  uint32_t S0, S1, w0, w1, nblk;
  uint32_t word[kRunPre];
};

__device__ __forceinline__ void run_chunk(const FramePlan &fp, const FrameState *st, uint32_t c,
                                          RunChunk &ch) {
  const int lane = threadIdx.x & 63;
  ch.S0 = fp.chunk_off[c];
  ch.S1 = c + 1 < fp.nchunks ? fp.chunk_off[c + 1] : (uint32_t)st->T;
  ch.w0 = ch.S0 >> 5;
  ch.w1 = (ch.S1 + 31) >> 5;
  ch.nblk = (ch.w1 - ch.w0 + 63) / 64;
#pragma unroll
  for (int b = 0; b < kRunPre; ++b) {
    const uint32_t i = ch.w0 + 64 * b + lane;
    ch.word[b] = i < ch.w1 ? chunk_word(fp, c, ch.S0, i) : 0u;
  }
}

// Calls g(base, word) for each block, base its first word's index.
template <class G>
__device__ __forceinline__ void for_each_word(const FramePlan &fp, uint32_t c, const RunChunk &ch,
                                              G &&g) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int b = 0; b < kRunPre; ++b)
    if (b < (int)ch.nblk) g(ch.w0 + 64 * b, ch.word[b]);
  for (uint32_t b = kRunPre; b < ch.nblk; ++b) {
    const uint32_t base = ch.w0 + 64 * b, i = base + lane;
    g(base, i < ch.w1 ? chunk_word(fp, c, ch.S0, i) : 0u);
  }
}

// Calls g(at, word, prev) for each block: at = the bit position of the
// lane's word, prev = the position after the last one bit before that word
// (the chunk start if none).  The runs of the lane's ones, in order, are
// one - prev, then one - (previous one + 1).
template <class G>
__device__ __forceinline__ void for_each_block(const FramePlan &fp, uint32_t c, const RunChunk &ch,
                                               G &&g) {
  const int lane = threadIdx.x & 63;
  uint32_t carry = ch.S0;   // after the last one of the earlier blocks
  for_each_word(fp, c, ch, [&](uint32_t base, uint32_t word) {
    const uint32_t i = base + lane;
    const uint32_t after = word ? 32 * i + (32 - __builtin_ctz(word)) : 0u;
    const uint32_t incl = wave_max_scan(after);
    const uint32_t excl = __shfl_up(incl, 1);
    const uint32_t prev = max(carry, lane ? excl : 0u);
    carry = max(carry, __shfl(incl, 63));
    g(32 * i, word, prev);
  });
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d));
  return v;
}

// The chunk's cost f(k) = sum(r >> k) + n (1 + k) is convex in k: f(k+1) -
// f(k) = n - sum(ceil((r >> k) / 2)), which never decreases.  While 3 n 2^k
// < S (S the sum of the runs) that difference is negative, and once n 2^k >=
// S it is >= 0, so the smallest minimiser lies in [kl, kl + 2] with kl the
// smallest k where 3 n 2^k >= S.  n is the popcount of the chunk's bits and
// S telescopes to (last one + 1) - S0 - n; one walk over the ones then
// gives the three costs.  A chunk holds at most 4096 * 32 bits, so every
// sum fits 32 bits.
__global__ __launch_bounds__(256) void k_run_count(BatchPlan bp) {
  const int lane = threadIdx.x & 63;
  const uint32_t item = blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (item >= bp.total_chunks) {
    // the ROI windows' payload, in the same launch (it needs only k_prep's
    // peak check, and this kernel leaves HBM bandwidth to spare)
    roi_copy(bp, item - bp.total_chunks);
    return;
  }
  const uint32_t f = find_frame(bp.chunk_prefix, bp.nframes, item);
  const FramePlan &fp = bp.frames[f];
  const FrameState *st = fp.st;
  if (!fp.run_coding || load_status(st) != RSZ_OK) return;
  const uint32_t c = item - bp.chunk_prefix[f];
  RunChunk ch;
  run_chunk(fp, st, c, ch);
  uint32_t n = 0, after = 0;
  for_each_word(fp, c, ch, [&](uint32_t base, uint32_t word) {
    n += __popc(word);
    if (word) after = max(after, 32 * (base + lane) + (32 - __builtin_ctz(word)));
  });
  n = wave_sum(n);
  after = wave_max(after);
  const uint32_t S = n ? after - ch.S0 - n : 0u;
  uint32_t kl = 0;
  while (kl < kRunKMax && 3ull * n * (1ull << kl) < S) kl++;
  uint32_t a0 = 0, a1 = 0, a2 = 0;
  for_each_block(fp, c, ch, [&](uint32_t at, uint32_t word, uint32_t prev) {
    while (word) {
      const uint32_t t = __builtin_clz(word);
      word &= ~(0x80000000u >> t);
      const uint32_t r = at + t - prev;
      prev = at + t + 1;
      a0 += r >> kl;
      a1 += r >> (kl + 1);
      a2 += r >> (kl + 2);
    }
  });
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  uint32_t best = kl, cost = a0 + n * (1 + kl);
  if (kl + 1 <= kRunKMax && a1 + n * (2 + kl) < cost) {
    best = kl + 1;
    cost = a1 + n * (2 + kl);
  }
  if (kl + 2 <= kRunKMax && a2 + n * (3 + kl) < cost) {
    best = kl + 2;
    cost = a2 + n * (3 + kl);
  }
  if (lane == 0) {
    fp.run_off[c] = cost;
    fp.run_k[c] = (uint8_t)best;
  }
}

// Chunk run bits -> bit offsets (exclusive scan), the section's bits last.
__global__ __launch_bounds__(256) void k_run_scan(BatchPlan bp) {
  __shared__ uint32_t s_tmp[4];
  const FramePlan &fp = bp.frames[blockIdx.x];
  if (!fp.run_coding || load_status(fp.st) != RSZ_OK) return;   // uniform
  uint32_t carry = 0;   // at most the bitstream's bits, below 2^32
  for (uint32_t c0 = 0; c0 < fp.nchunks; c0 += 256) {
    const uint32_t c = c0 + threadIdx.x;
    const uint32_t v = c < fp.nchunks ? fp.run_off[c] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t>(v, s_tmp, tot);
    if (c < fp.nchunks) fp.run_off[c] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) fp.run_off[fp.nchunks] = carry;
}

// A lane's codes occupy one contiguous range of bits: they are assembled in
// a 64-bit register and leave as whole words, aligned to the destination's
// words.  Only the range's first and last words can be shared with another
// lane (or chunk), so only they are ORed atomically; the words between are
// stored.
struct LaneBits {
  uint32_t *dst;
  uint64_t w;      // destination word of the next whole word
  uint64_t acc;    // pending bits in the low n bits (higher bits are stale)
  uint32_t n;
  bool first;
  __device__ void init(uint32_t *d, uint64_t pos) {
    dst = d;
    w = pos >> 5;
    acc = 0;
    n = (uint32_t)(pos & 31);   // zero bits that align the words
    first = true;
  }
  // appends the len (1..32) low bits of v, MSB-first
  __device__ void put(uint32_t v, uint32_t len) {
    acc = (acc << len) | v;
    n += len;
    if (n >= 32) {
      const uint32_t word = (uint32_t)(acc >> (n - 32));
      if (first) {
        if (word) atomicOr(&dst[w], word);
        first = false;
      } else {
        dst[w] = word;
      }
      w++;
      n -= 32;
    }
  }
  __device__ void finish() {
    if (n) {
      const uint32_t word = (uint32_t)(acc << (32 - n));
      if (word) atomicOr(&dst[w], word);
    }
  }
};

// Words [0, nw) of a wave's staging buffer to the stream words from word
// `wbase`: the first and last by atomicOr (a neighbouring chunk, or codes
// written directly, may share them), the rest by plain stores (this chunk's
// alone).
constexpr uint32_t kRunBufWords = 512;
__device__ __forceinline__ void run_flush(const uint32_t *buf, uint32_t *out, uint64_t wbase,
                                          uint32_t nw) {
  for (uint32_t i = threadIdx.x & 63; i < nw; i += 64) {
    const uint32_t v = buf[i];
    if (i == 0 || i + 1 == nw) {
      if (v) atomicOr(&out[wbase + i], v);
    } else {
      out[wbase + i] = v;
    }
  }
}

// The codes of each chunk at its offset in the run words k_tail zeroed.  A
// wave stages its chunk's codes in an LDS buffer of kRunBufWords words (ORed
// in by LDS atomics) and stores whole words; a block of 64 input words whose
// codes would overflow the buffer flushes it first, and if they still do not
// fit, ORs them straight into the stream.
__global__ __launch_bounds__(256) void k_run_pack(BatchPlan bp) {
  __shared__ uint32_t s_buf[kWaves][kRunBufWords];
  const int lane = threadIdx.x & 63;
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t item = blockIdx.x * kWaves + wv;
  if (item >= bp.total_chunks) {
    // the ROI windows' payload, in the same launch (it needs only k_prep's
    // peak check, and this kernel leaves HBM bandwidth to spare)
    roi_copy(bp, item - bp.total_chunks);
    return;
  }
  const uint32_t f = find_frame(bp.chunk_prefix, bp.nframes, item);
  const FramePlan &fp = bp.frames[f];
  const FrameState *st = fp.st;
  if (!fp.run_coding || load_status(st) != RSZ_OK) return;
  const uint32_t c = item - bp.chunk_prefix[f];
  uint32_t *out = (uint32_t *)(fp.out + st->off_runbits);
  uint32_t *buf = s_buf[wv];
  for (uint32_t i = lane; i < kRunBufWords; i += 64) buf[i] = 0u;
  wave_sync();
  const uint32_t k = fp.run_k[c];
  uint64_t base_bit = fp.run_off[c];
  uint64_t wbase = base_bit >> 5;   // stream word of buf[0]
  RunChunk ch;
  run_chunk(fp, st, c, ch);
  for_each_block(fp, c, ch, [&](uint32_t at, uint32_t word, uint32_t prev) {
    // this lane's code bits, placed by a wave scan
    uint32_t bits = 0, p = prev, w = word;
    while (w) {
      const uint32_t t = __builtin_clz(w);
      w &= ~(0x80000000u >> t);
      bits += ((at + t - p) >> k) + 1 + k;
      p = at + t + 1;
    }
    uint64_t tot;
    const uint64_t ex = wave_exclusive_scan(bits, tot);
    bool direct = false;
    if ((base_bit + tot + 31) / 32 - wbase > kRunBufWords) {
      // keep only the partial word at base_bit
      const uint32_t nw = (uint32_t)((base_bit >> 5) - wbase);
      run_flush(buf, out, wbase, nw);
      const uint32_t part = nw < kRunBufWords ? buf[nw] : 0u;
      wave_sync();
      for (uint32_t i = lane; i < kRunBufWords; i += 64) buf[i] = i == 0 ? part : 0u;
      wave_sync();
      wbase += nw;
      if ((base_bit + tot + 31) / 32 - wbase > kRunBufWords) {
        direct = true;
        if (lane == 0 && part) atomicOr(&out[wbase], part);
        wave_sync();
        if (lane == 0) buf[0] = 0u;
        wave_sync();
      }
    }
    LaneBits lb;
    lb.init(direct ? out : buf, base_bit + ex - (direct ? 0 : 32 * wbase));
    p = prev;
    w = word;
    while (w) {
      const uint32_t t = __builtin_clz(w);
      w &= ~(0x80000000u >> t);
      const uint32_t r = at + t - p;
      p = at + t + 1;
      uint32_t q = r >> k;
      for (; q >= 32; q -= 32) lb.put(0xFFFFFFFFu, 32);
      lb.put(((1u << q) - 1u) << 1, q + 1);   // q ones and the closing zero
      if (k) lb.put(r & ((1u << k) - 1u), k);
    }
    lb.finish();
    wave_sync();
    base_bit += tot;
    if (direct) wbase = base_bit >> 5;   // the buffer is empty again
  });
  run_flush(buf, out, wbase, (uint32_t)((base_bit + 31) / 32 - wbase));
}

// -------------------------------------------------------------- launchers

#define RSZ_LAUNCH_B(name, kern, grid, block, s, ...)             \
  do {                                                            \
    prof_begin(name, s);                                          \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, __VA_ARGS__); \
    prof_end(s);                                                  \
    hipError_t e_ = hipGetLastError();                            \
    if (e_ != hipSuccess) return e_;                              \
  } while (0)
#define RSZ_LAUNCH(name, kern, grid, s, ...) RSZ_LAUNCH_B(name, kern, grid, 256, s, __VA_ARGS__)

hipError_t launch_codebook(const BatchPlan &bp, hipStream_t s) {
  hipLaunchKernelGGL(k_codebook, dim3(bp.nframes), dim3(256), 0, s, bp);
  return hipGetLastError();
}

// Debug: the u16 codes of frame 0 of a plan, expanded from the code bytes.
__global__ __launch_bounds__(256) void k_debug_codes(BatchPlan bp, uint16_t *out) {
  const FramePlan &fp = bp.frames[0];
  for (uint32_t g = blockIdx.x * 256 + threadIdx.x; g < fp.nbins; g += gridDim.x * 256) {
    const uint4 v = code_group(fp, g & ~15u);
    const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
    const uint32_t b = (w4[(g >> 2) & 3] >> (8 * (g & 3))) & 0xFFu;
    out[g] = (uint16_t)(b ? b + (kRadius - 128) : code_from_residual(fp.rbuf[g]));
  }
}

// The outliers of frame 0 (bins whose residual has no code) in bin order:
// their count, indices and residuals, from the codes k_bin leaves (the
// outlier section of the stream holds the same list).  One workgroup.
__global__ __launch_bounds__(256) void k_debug_outliers(BatchPlan bp, uint32_t *n_out,
                                                        uint32_t *idx, int32_t *res) {
  const FramePlan &fp = bp.frames[0];
  __shared__ uint32_t s_tmp[4];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < fp.nbins; base += 256) {
    const uint32_t g = base + threadIdx.x;
    uint32_t o = 0;
    int32_t r = 0;
    if (g < fp.nbins) {
      const uint4 v = code_group(fp, g & ~15u);
      const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
      if (((w4[(g >> 2) & 3] >> (8 * (g & 3))) & 0xFFu) == 0) {
        r = fp.rbuf[g];
        o = code_from_residual(r) == 0;
      }
    }
    uint32_t tot;
    const uint32_t at = carry + block_exclusive_scan<uint32_t>(o, s_tmp, tot);
    if (o) {
      if (idx) idx[at] = g;
      if (res) res[at] = r;
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && n_out) *n_out = carry;
}

hipError_t launch_debug_outliers(const BatchPlan &bp, uint32_t *n_out, uint32_t *idx,
                                 int32_t *res, hipStream_t s) {
  hipLaunchKernelGGL(k_debug_outliers, dim3(1), dim3(256), 0, s, bp, n_out, idx, res);
  return hipGetLastError();
}

hipError_t launch_debug_codes(const BatchPlan &bp, uint32_t nbins, uint16_t *out, hipStream_t s) {
  const uint32_t grid = std::max(1u, std::min(4096u, (nbins + 255) / 256));
  hipLaunchKernelGGL(k_debug_codes, dim3(grid), dim3(256), 0, s, bp, out);
  return hipGetLastError();
}

// `b`: the common bin factor of the batch, or 0 (mixed or not 1, 2, 4).
template <bool DEBUG, int DIM>
static hipError_t launch_bin(const BatchPlan &bp, uint32_t b, hipStream_t s) {
  if (bp.total_tiles == 0) return hipSuccess;
  const uint32_t grid = bp.total_tiles;
  switch (b) {
    case 1: RSZ_LAUNCH_B("k_bin", (k_bin<1, DEBUG, DIM>), grid, 64 * bp.bin_waves, s, bp); break;
    case 2:
      if (!DEBUG && bp.all_vec) RSZ_LAUNCH_B("k_bin", (k_bin_vec<2, DIM>), grid, 64 * bp.bin_waves, s, bp);
      else RSZ_LAUNCH_B("k_bin", (k_bin<2, DEBUG, DIM>), grid, 64 * bp.bin_waves, s, bp);
      break;
    case 4:
      if (!DEBUG && bp.all_vec) RSZ_LAUNCH_B("k_bin", (k_bin_vec<4, DIM>), grid, 64 * bp.bin_waves, s, bp);
      else RSZ_LAUNCH_B("k_bin", (k_bin<4, DEBUG, DIM>), grid, 64 * bp.bin_waves, s, bp);
      break;
    default: RSZ_LAUNCH_B("k_bin", (k_bin<0, DEBUG, DIM>), grid, 64 * bp.bin_waves, s, bp); break;
  }
  return hipSuccess;
}

// prep + bin + codebook; `b` and `dim` are the common bin factor and Lorenzo
// dimension of the batch, or 0.  The debug build reads the dimension per frame.
hipError_t launch_compress_front_b(const BatchPlan &bp, uint32_t b, uint32_t dim, hipStream_t s,
                                   bool debug) {
  RSZ_LAUNCH("k_prep", k_prep, bp.nframes, s, bp);
  hipError_t e;
  if (debug) e = launch_bin<true, 0>(bp, b, s);
  else if (dim == 2) e = launch_bin<false, 2>(bp, b, s);
  else if (dim == 1) e = launch_bin<false, 1>(bp, b, s);
  else if (dim == 3) e = launch_bin<false, 3>(bp, b, s);
  else e = launch_bin<false, 0>(bp, b, s);
  if (e != hipSuccess) return e;
  if (bp.total_fix) RSZ_LAUNCH("k_lorenzo_dims", k_lorenzo_dims, bp.total_fix, s, bp);
  RSZ_LAUNCH("k_codebook", k_codebook, bp.nframes, s, bp);
  return hipSuccess;
}

hipError_t launch_compress_back(const BatchPlan &bp, hipStream_t s) {
  // k_count's items: the chunks, then the peaks (ROI payload)
  const uint32_t cgrid = (bp.total_chunks + bp.total_peaks + kWaves - 1) / kWaves;
  if (cgrid) {
    if (bp.all_sparse) RSZ_LAUNCH("k_count", k_count<true>, cgrid, s, bp);
    else RSZ_LAUNCH("k_count", k_count<false>, cgrid, s, bp);
  }
  RSZ_LAUNCH("k_scan", k_scan, bp.nframes, s, bp);
  if (bp.total_units) {
    RSZ_LAUNCH("k_encode", k_encode, bp.total_units, s, bp);
  }
  const uint32_t roi_grid = (bp.total_peaks + kWaves - 1) / kWaves;   // a wave per window
  if (bp.roi_coding) {
    if (bp.total_peaks) RSZ_LAUNCH("k_roi_classes", k_roi_classes, roi_grid, s, bp);
    RSZ_LAUNCH("k_roi_book", k_roi_book, bp.nframes, s, bp);
    if (bp.total_peaks) RSZ_LAUNCH("k_roi_count", k_roi_count, roi_grid, s, bp);
    RSZ_LAUNCH("k_roi_scan", k_roi_scan, bp.nframes, s, bp);
  }
  const uint32_t run_grid = (bp.total_chunks + kWaves - 1) / kWaves;
  if (bp.run_coding) {
    if (bp.total_chunks) RSZ_LAUNCH("k_run_count", k_run_count, run_grid, s, bp);
    RSZ_LAUNCH("k_run_scan", k_run_scan, bp.nframes, s, bp);
  }
  RSZ_LAUNCH("k_tail", k_tail, bp.nframes, s, bp);
  if (bp.total_peaks && bp.roi_coding) RSZ_LAUNCH("k_roi_pack", k_roi_pack, roi_grid, s, bp);
  if (bp.run_coding && bp.total_chunks) RSZ_LAUNCH("k_run_pack", k_run_pack, run_grid, s, bp);
  return hipSuccess;
}

}  // namespace rsz
