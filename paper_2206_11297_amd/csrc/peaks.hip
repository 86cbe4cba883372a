// peaks.hip -- peak finding on the GPU: the step before the compression path,
// producing the peak list whose windows form the ROI mask (Sec. IV-B names
// peak_finder_v3 and its parameters; non-hit rejection, Sec. IV, counts
// these peaks).
//
// k_peaks_init  zeroes each frame's peak counter.
// k_peaks_find  streams every frame once, 16 float4 loads per lane.  The
//               rare pixels at or above amax_min are taken by their wave in
//               rounds: the wave stages the round's neighbourhoods in LDS
//               with all loads in flight, then one lane per candidate decides
//               (window maximum, background ring, peak pixels, cuts);
//               accepted peaks are appended as (panel, row, col) keys.  (A
//               lane that fetched its neighbourhood itself, one load after
//               another, spent most of the kernel waiting on them.)
// k_peaks_sort  one workgroup per frame: bitonic sort of the keys in LDS, so
//               the list comes out in raster order whatever the append order.
//
// The arithmetic of a decision follows one fixed order on every lane: fp64
// sums in raster order, a correctly rounded divide, products compared instead
// of square roots.  Compiled with -ffp-contract=off.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "rsz_internal.h"

namespace rsz {

namespace {

__device__ __forceinline__ int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }
__device__ __forceinline__ int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t iabs(int64_t a) { return a < 0 ? -a : a; }

__device__ __forceinline__ uint32_t peak_frame_of(const uint32_t *prefix, uint32_t nframes,
                                                  uint32_t item) {
  uint32_t lo = 0, hi = nframes;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (prefix[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

// LDS per wave for staged neighbourhoods ((2 * ring_out + 1)^2 pixels each,
// ring_out <= 15): 1024 floats hold 8 neighbourhoods of the default ring
// (11 x 11), one of the largest (31 x 31).  Twice that halved the workgroups
// a CU holds and slowed the streaming part of the kernel by half.
constexpr int kNbFloats = 1024;
static_assert(kNbFloats >= 31 * 31, "a neighbourhood must fit");

// The decision for pixel (i, j) of a panel of H x W, from its neighbourhood
// staged in nb: pixel (u, v) at nb[(u - i + R) * (2R + 1) + (v - j + R)],
// R = ring_out (only in-panel pixels are staged and read).  One lane runs it,
// in the oracle's order: window maximum (ties to the first pixel in raster
// order), background ring mean and squared deviations, the cut, the
// 4-connected component of the maximum, its sum, the cuts.
__device__ bool peak_decide(const rsz_peak_params &q, const float *nb, int64_t H, int64_t W,
                            int64_t i, int64_t j) {
  const int64_t h = q.rank, ww = 2 * h + 1, ro = q.ring_out, ri = q.ring_in, side = 2 * ro + 1;
  auto at = [&](int64_t u, int64_t v) { return nb[(u - i + ro) * side + (v - j + ro)]; };
  const float c = at(i, j);
  for (int64_t u = imax(i - h, 0); u <= imin(i + h, H - 1); ++u)
    for (int64_t v = imax(j - h, 0); v <= imin(j + h, W - 1); ++v) {
      if (u == i && v == j) continue;
      const float o = at(u, v);
      // earlier pixels must be smaller, later ones not larger (NaN fails both)
      const bool before = u < i || (u == i && v < j);
      if (before ? !(o < c) : !(o <= c)) return false;
    }
  const int64_t u0 = imax(i - ro, 0), u1 = imin(i + ro, H - 1);
  const int64_t v0 = imax(j - ro, 0), v1 = imin(j + ro, W - 1);
  // background ring: mean, then the sum of squared deviations
  double sum = 0.0;
  int64_t m = 0;
  for (int64_t u = u0; u <= u1; ++u)
    for (int64_t v = v0; v <= v1; ++v) {
      if (imax(iabs(u - i), iabs(v - j)) < ri) continue;
      sum += (double)at(u, v);
      m++;
    }
  if (m == 0) return false;
  const double mu = sum / (double)m;
  double V = 0.0;
  for (int64_t u = u0; u <= u1; ++u)
    for (int64_t v = v0; v <= v1; ++v) {
      if (imax(iabs(u - i), iabs(v - j)) < ri) continue;
      const double e = (double)at(u, v) - mu;
      V += e * e;
    }
  const double k2V = q.pix_nsigma * q.pix_nsigma * V;
  // window pixels above the cut, as bits a*ww + b of the (2h+1)^2 window
  uint64_t above = 0;
  for (int64_t a = 0; a < ww; ++a)
    for (int64_t b = 0; b < ww; ++b) {
      const int64_t u = i - h + a, v = j - h + b;
      if (u < 0 || u >= H || v < 0 || v >= W) continue;
      const double d = (double)at(u, v) - mu;
      if (d > 0.0 && d * d * (double)m > k2V) above |= 1ull << (a * ww + b);
    }
  // the 4-connected component of the maximum: grow by one step in each of the
  // four directions until nothing changes (shifts by 1 must not wrap rows)
  uint64_t first_col = 0, last_col = 0;
  for (int64_t a = 0; a < ww; ++a) {
    first_col |= 1ull << (a * ww);
    last_col |= 1ull << (a * ww + ww - 1);
  }
  uint64_t comp = above & (1ull << (h * ww + h));
  for (;;) {
    const uint64_t grown = (comp | ((comp << 1) & ~first_col) | ((comp >> 1) & ~last_col) |
                            (comp << ww) | (comp >> ww)) & above;
    if (grown == comp) break;
    comp = grown;
  }
  double S = 0.0;
  int64_t n = 0;
  for (int64_t a = 0; a < ww; ++a)
    for (int64_t b = 0; b < ww; ++b)
      if ((comp >> (a * ww + b)) & 1u) {
        S += (double)at(i - h + a, j - h + b);
        n++;
      }
  if (n < (int64_t)q.npix_min || n > (int64_t)q.npix_max) return false;
  if (!(S > q.atot_min)) return false;
  const double num = S - (double)n * mu;
  return num > 0.0 && num * num * (double)m > q.snr_min * q.snr_min * (double)n * V;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(256) void k_peaks_init(PeakBatchPlan pp) {
  const uint32_t f = blockIdx.x * 256 + threadIdx.x;
  if (f < pp.nframes) *pp.frames[f].count = 0u;
}

__global__ __launch_bounds__(256) void k_peaks_find(PeakBatchPlan pp) {
  const uint32_t f = peak_frame_of(pp.tile_prefix, pp.nframes, blockIdx.x);
  const PeakFramePlan &fp = pp.frames[f];
  if (fp.init_status != RSZ_OK) return;
  const uint64_t npix = (uint64_t)fp.P * fp.H * fp.W;
  const uint64_t base = (uint64_t)(blockIdx.x - pp.tile_prefix[f]) * kPeakTile;
  const float *x = fp.frame;
  constexpr int K = (int)(kPeakTile / 1024);   // float4 loads per lane
  float v[K][4];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t e0 = base + (uint64_t)(k * 256 + threadIdx.x) * 4;
    if (e0 + 4 <= npix) {
      const float4 w = *(const float4 *)(x + e0);   // the frame is 16-byte aligned
      v[k][0] = w.x;
      v[k][1] = w.y;
      v[k][2] = w.z;
      v[k][3] = w.w;
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) v[k][t] = e0 + t < npix ? x[e0 + t] : -INFINITY;
    }
  }
  // candidates: pixels at or above amax_min (amax_f is the smallest float
  // >= amax_min, so a float compare decides exactly as the fp64 one)
  const float amax_f = pp.amax_f;
  uint64_t cand = 0;   // bit 4k + t: pixel t of load k
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int t = 0; t < 4; ++t) cand |= (uint64_t)(v[k][t] >= amax_f) << (4 * k + t);
  // The wave takes its candidates in rounds of up to kNbFloats / side^2: every
  // lane loads part of the round's neighbourhoods into the wave's LDS slice
  // (all loads in flight together), then one lane per candidate decides.
  uint64_t pending = __builtin_amdgcn_uicmp((uint32_t)(cand | (cand >> 32)), 0u, 33 /* ne */);
  if (!pending) return;
  __shared__ float s_nb[4][kNbFloats];
  __shared__ int32_t s_pij[4][64][3];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float *nb = s_nb[wv];
  int32_t(*pij)[3] = s_pij[wv];
  const rsz_peak_params q = pp.q;
  // a frame has < 2^31 pixels: 32-bit index arithmetic
  const int32_t H = (int32_t)fp.H, W = (int32_t)fp.W, ro = (int32_t)q.ring_out;
  const int32_t side = 2 * ro + 1, area = side * side;
  const int per_round = min(64, kNbFloats / area);
  uint64_t cm = 0;   // the lane's candidates not yet queued
  int L = -1;        // the lane whose candidates are being queued
  for (;;) {
    // queue up to per_round candidates (uniform): their (panel, row, col)
    int nq = 0;
    while (nq < per_round) {
      if (!cm) {
        if (!pending) break;
        L = __builtin_ctzll(pending);
        pending &= pending - 1;
        cm = ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(cand >> 32), L) << 32) |
             __builtin_amdgcn_readlane((uint32_t)cand, L);
      }
      const int b = __builtin_ctzll(cm);
      cm &= cm - 1;
      const uint32_t e = (uint32_t)(base + (uint64_t)((b >> 2) * 256 + wv * 64 + L) * 4 + (b & 3));
      if (lane == 0) {
        const uint32_t r = e / (uint32_t)W;
        pij[nq][0] = (int32_t)(r / (uint32_t)H);
        pij[nq][1] = (int32_t)(r % (uint32_t)H);
        pij[nq][2] = (int32_t)(e % (uint32_t)W);
      }
      nq++;
    }
    if (nq == 0) break;
    wave_sync();
    // stage: candidate c's neighbourhood at nb[c * area, (c + 1) * area)
    for (int c = 0; c < nq; ++c) {
      const int32_t p = pij[c][0], i = pij[c][1], j = pij[c][2];
      const float *xp = x + ((uint64_t)p * H) * W;
      for (int32_t o = lane; o < area; o += 64) {
        const int32_t du = o / side, u = i - ro + du, w = j - ro + (o - du * side);
        if (u >= 0 && u < H && w >= 0 && w < W) nb[c * area + o] = xp[(uint32_t)u * W + w];
      }
    }
    wave_sync();
    if (lane < nq) {
      const int32_t p = pij[lane][0], i = pij[lane][1], j = pij[lane][2];
      if (peak_decide(q, nb + lane * area, H, W, i, j)) {
        const uint32_t slot = atomicAdd(fp.count, 1u);
        if (slot < fp.cap) fp.keys[slot] = ((uint64_t)p << 32) | ((uint64_t)i << 16) | (uint64_t)j;
      }
    }
    wave_sync();
  }
}

__global__ __launch_bounds__(256) void k_peaks_sort(PeakBatchPlan pp) {
  __shared__ uint64_t s_key[kPeakCapMax];
  const PeakFramePlan &fp = pp.frames[blockIdx.x];
  if (fp.init_status != RSZ_OK) {
    if (threadIdx.x == 0) {
      *fp.res_count = 0u;
      *fp.res_status = fp.init_status;
    }
    return;
  }
  const uint32_t n = *fp.count;
  if (n > fp.cap) {
    if (threadIdx.x == 0) {
      *fp.res_count = n;
      *fp.res_status = RSZ_ERR_CAPACITY;
    }
    return;
  }
  uint32_t n2 = 1;
  while (n2 < n) n2 <<= 1;
  for (uint32_t k = threadIdx.x; k < n2; k += 256) s_key[k] = k < n ? fp.keys[k] : ~0ull;
  __syncthreads();
  // ascending bitonic sort of s_key[0, n2) (keys are unique within a frame)
  for (uint32_t size = 2; size <= n2; size <<= 1)
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t t = threadIdx.x; t < n2 / 2; t += 256) {
        const uint32_t a = 2 * t - (t & (stride - 1)), b = a + stride;
        const bool up = (a & size) == 0;
        const uint64_t ka = s_key[a], kb = s_key[b];
        if ((ka > kb) == up) {
          s_key[a] = kb;
          s_key[b] = ka;
        }
      }
      __syncthreads();
    }
  for (uint32_t k = threadIdx.x; k < n; k += 256) {
    const uint64_t key = s_key[k];
    fp.out[k].panel = (int32_t)(key >> 32);
    fp.out[k].row = (int32_t)((key >> 16) & 0xFFFFu);
    fp.out[k].col = (int32_t)(key & 0xFFFFu);
  }
  if (threadIdx.x == 0) {
    *fp.res_count = n;
    *fp.res_status = RSZ_OK;
  }
}

}  // namespace

#define RSZ_PLAUNCH(name, kern, grid, s)                              \
  do {                                                                \
    prof_begin(name, s);                                              \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, pp);        \
    prof_end(s);                                                      \
    hipError_t e_ = hipGetLastError();                                \
    if (e_ != hipSuccess) return e_;                                  \
  } while (0)

hipError_t launch_find_peaks(const PeakBatchPlan &pp, hipStream_t s) {
  RSZ_PLAUNCH("k_peaks_init", k_peaks_init, (pp.nframes + 255) / 256, s);
  if (pp.total_tiles) RSZ_PLAUNCH("k_peaks_find", k_peaks_find, pp.total_tiles, s);
  RSZ_PLAUNCH("k_peaks_sort", k_peaks_sort, pp.nframes, s);
  return hipSuccess;
}

}  // namespace rsz
