// decompress.hip -- HIP kernels that decode a ROIBIN-SZ stream on gfx950.
//
//   k_dec_tables    one workgroup: check code lengths (<= 32, complete prefix
//                   code), peaks and chunk offsets; build canonical decode
//                   tables (11-bit lookup table + per-length first codes).
//   k_dec_chunks    one lane per 4096-symbol chunk: Huffman decode to
//                   residuals; each chunk must end exactly at the next offset.
//   k_dec_outliers  scatter outlier residuals onto the code-0 positions.
//   k_dec_rows      inclusive prefix sum along each bin row (wrapping int32).
//   k_dec_cols      inclusive prefix sum down each bin column -> q.
//   k_dec_expand    every pixel gets float(q * 2eb) of its bin.
//   k_dec_roi       ROI windows restored from the payload bits.
//   k_dec_roi_check overlapping windows must agree on their shared pixels.
// The inverse Lorenzo step is the 2D prefix sum of the residuals per panel.
#include <algorithm>

#include "rsz_internal.h"

namespace rsz {

constexpr int kLutBits = 11;
constexpr int32_t kMark = INT32_MIN;  // residual slot waiting for its outlier

// tables: [0,2048) lut (sym | len << 16, 0 = slow path), then first[33],
// count[33], offs[33], sorted[1024]
constexpr int kTabLut = 0, kTabFirst = 1 << kLutBits, kTabCount = kTabFirst + 33,
              kTabOffs = kTabCount + 33, kTabSorted = kTabOffs + 33,
              kTabWords = kTabSorted + kNumSym;

__device__ __forceinline__ void corrupt(int32_t *status) {
  atomicCAS(status, (int32_t)RSZ_OK, (int32_t)RSZ_ERR_CORRUPT);
}

__device__ __forceinline__ bool dec_ok(const int32_t *status) {
  return __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == RSZ_OK;
}

__device__ __forceinline__ uint32_t rd32(const uint8_t *p, uint64_t off) {
  return *(const uint32_t *)(p + off);
}

__global__ __launch_bounds__(256) void k_dec_tables(DecodePlan dp) {
  __shared__ uint8_t s_len[kNumSym];
  __shared__ uint32_t s_count[kMaxLen + 1];
  __shared__ unsigned long long s_kraft;
  __shared__ int s_used, s_bad;
  if (threadIdx.x == 0) {
    s_kraft = 0;
    s_used = 0;
    s_bad = 0;
    *dp.status = RSZ_OK;
  }
  if (threadIdx.x <= kMaxLen) s_count[threadIdx.x] = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < kNumSym; s += 256) {
    const uint32_t L = dp.in[dp.off_lens + s];
    s_len[s] = (uint8_t)L;
    if (L > kMaxLen) {
      s_bad = 1;
    } else if (L) {
      atomicAdd(&s_kraft, 1ull << (kMaxLen - L));
      atomicAdd(&s_used, 1);
      atomicAdd(&s_count[L], 1u);
    }
  }
  for (uint32_t k = threadIdx.x; k < dp.npeaks; k += 256) {
    const uint16_t *pk = (const uint16_t *)(dp.in + dp.off_peaks) + 3 * k;
    if (pk[0] >= dp.P || pk[1] >= dp.H || pk[2] >= dp.W) s_bad = 1;
  }
  const uint32_t *co = (const uint32_t *)(dp.in + dp.off_chunks);
  for (uint32_t c = threadIdx.x; c < dp.nchunks; c += 256) {
    const uint32_t o = co[c];
    if (o > dp.T || (c == 0 && o != 0) || (c > 0 && o < co[c - 1])) s_bad = 1;
  }
  __syncthreads();
  const bool complete = s_kraft == (1ull << kMaxLen);
  const bool single = s_used == 1 && s_kraft == (1ull << (kMaxLen - 1));
  if (s_bad || !(complete || single)) {
    if (threadIdx.x == 0) *dp.status = RSZ_ERR_CORRUPT;
    return;
  }
  uint32_t *tab = dp.tables;
  if (threadIdx.x == 0) {
    // canonical first code, symbol count and sorted offset per length
    uint64_t code = 0;
    uint32_t start = 0, prev = 0;
    for (int L = 1; L <= kMaxLen; ++L) {
      code = (code + prev) << 1;
      tab[kTabFirst + L] = (uint32_t)code;
      tab[kTabCount + L] = s_count[L];
      tab[kTabOffs + L] = start;
      start += s_count[L];
      prev = s_count[L];
    }
    // symbols in (length, symbol) order
    uint32_t fill[kMaxLen + 1];
    for (int L = 0; L <= kMaxLen; ++L) fill[L] = 0;
    for (int s = 0; s < kNumSym; ++s) {
      const uint32_t L = s_len[s];
      if (L) tab[kTabSorted + tab[kTabOffs + L] + fill[L]++] = (uint32_t)s;
    }
  }
  for (int i = threadIdx.x; i < (1 << kLutBits); i += 256) tab[kTabLut + i] = 0u;
  __syncthreads();
  // lookup entries for codewords of at most kLutBits bits
  for (int s = threadIdx.x; s < kNumSym; s += 256) {
    const uint32_t L = s_len[s];
    if (!L || L > (uint32_t)kLutBits) continue;
    // rank of s among the symbols of length L
    uint32_t rank = 0;
    for (int t = 0; t < s; ++t) rank += s_len[t] == L;
    const uint32_t code = tab[kTabFirst + L] + rank;
    const uint32_t lo = code << (kLutBits - L), n = 1u << (kLutBits - L);
    for (uint32_t e = 0; e < n; ++e) tab[kTabLut + lo + e] = (uint32_t)s | (L << 16);
  }
}

// Peek 32 stream bits starting at bit `pos`; bits past the stream read 0.
__device__ __forceinline__ uint32_t peek32(const uint32_t *bw, uint64_t nwords, uint64_t pos) {
  const uint64_t w = pos >> 5;
  const uint64_t a = w < nwords ? bw[w] : 0u;
  const uint64_t b = w + 1 < nwords ? bw[w + 1] : 0u;
  return (uint32_t)((((a << 32) | b) << (pos & 31)) >> 32);
}

__global__ __launch_bounds__(64) void k_dec_chunks(DecodePlan dp) {
  __shared__ uint32_t s_lut[1 << kLutBits];
  __shared__ uint32_t s_first[kMaxLen + 1], s_count[kMaxLen + 1], s_offs[kMaxLen + 1];
  __shared__ uint16_t s_sorted[kNumSym];
  for (int i = threadIdx.x; i < (1 << kLutBits); i += 64) s_lut[i] = dp.tables[kTabLut + i];
  for (int i = threadIdx.x; i < kNumSym; i += 64) s_sorted[i] = (uint16_t)dp.tables[kTabSorted + i];
  if (threadIdx.x <= kMaxLen) {
    s_first[threadIdx.x] = dp.tables[kTabFirst + threadIdx.x];
    s_count[threadIdx.x] = dp.tables[kTabCount + threadIdx.x];
    s_offs[threadIdx.x] = dp.tables[kTabOffs + threadIdx.x];
  }
  __syncthreads();
  const uint32_t c = blockIdx.x * 64 + threadIdx.x;
  if (c >= dp.nchunks || !dec_ok(dp.status)) return;
  const uint32_t *co = (const uint32_t *)(dp.in + dp.off_chunks);
  const uint32_t *bw = (const uint32_t *)(dp.in + dp.off_bits);
  const uint64_t nwords = (dp.T + 31) / 32;
  uint64_t pos = co[c];
  const uint64_t end = c + 1 < dp.nchunks ? co[c + 1] : dp.T;
  const uint32_t g0 = c * kChunk;
  const uint32_t nsym = min(kChunk, dp.nbins - g0);
  uint32_t zeros = 0;
  bool bad = false;
  for (uint32_t k = 0; k < nsym; ++k) {
    const uint32_t v = peek32(bw, nwords, pos);
    const uint32_t e = s_lut[v >> (32 - kLutBits)];
    uint32_t sym, L;
    if (e) {
      sym = e & 0xFFFFu;
      L = e >> 16;
    } else {
      L = 0;
      sym = 0;
      for (uint32_t l = kLutBits + 1; l <= (uint32_t)kMaxLen; ++l) {
        const uint32_t cd = v >> (32 - l);
        if (s_count[l] && cd >= s_first[l] && cd - s_first[l] < s_count[l]) {
          L = l;
          sym = s_sorted[s_offs[l] + cd - s_first[l]];
          break;
        }
      }
      if (L == 0) {
        bad = true;
        break;
      }
    }
    if (pos + L > end) {
      bad = true;
      break;
    }
    pos += L;
    dp.res[g0 + k] = sym ? (int32_t)sym - kRadius : kMark;
    zeros += sym == 0;
  }
  if (bad || pos != end) corrupt(dp.status);
  dp.zcount[c] = zeros;
}

__global__ __launch_bounds__(256) void k_dec_outliers(DecodePlan dp) {
  const uint32_t k = blockIdx.x * 256 + threadIdx.x;
  if (k >= dp.n_out || !dec_ok(dp.status)) return;
  const uint32_t *oi = (const uint32_t *)(dp.in + dp.off_oidx);
  const int32_t *orr = (const int32_t *)(dp.in + dp.off_ores);
  const uint32_t g = oi[k];
  const int32_t r = orr[k];
  // |q| < 2^28 bounds every residual below 2^30 in magnitude
  if (g >= dp.nbins || (k > 0 && g <= oi[k - 1]) || (r > -kRadius && r < kRadius) ||
      r <= -(1 << 30) || r >= (1 << 30) || dp.res[g] != kMark) {
    corrupt(dp.status);
    return;
  }
  dp.res[g] = r;
}

// One wave per bin row: inclusive prefix sum along the row.
__global__ __launch_bounds__(256) void k_dec_rows(DecodePlan dp) {
  const uint32_t row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= dp.P * dp.Hb || !dec_ok(dp.status)) return;
  int32_t *r = dp.res + (size_t)row * dp.Wb;
  uint32_t carry = 0;
  bool bad = false;
  for (uint32_t j0 = 0; j0 < dp.Wb; j0 += 64) {
    const uint32_t j = j0 + lane;
    uint32_t x = 0;
    if (j < dp.Wb) {
      const int32_t v = r[j];
      bad |= v == kMark;
      x = (uint32_t)v;
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    x += carry;
    if (j < dp.Wb) r[j] = (int32_t)x;
    carry = __shfl(x, 63);
  }
  if (bad) corrupt(dp.status);
}

// One lane per bin column: inclusive prefix sum down the column.
__global__ __launch_bounds__(256) void k_dec_cols(DecodePlan dp) {
  const uint32_t col = blockIdx.x * 256 + threadIdx.x;
  if (col >= dp.P * dp.Wb || !dec_ok(dp.status)) return;
  const uint32_t p = col / dp.Wb, J = col - p * dp.Wb;
  int32_t *r = dp.res + (size_t)p * dp.Hb * dp.Wb + J;
  uint32_t acc = 0;
  for (uint32_t I = 0; I < dp.Hb; ++I) {
    acc += (uint32_t)r[(size_t)I * dp.Wb];
    r[(size_t)I * dp.Wb] = (int32_t)acc;
  }
}

__global__ __launch_bounds__(256) void k_dec_expand(DecodePlan dp) {
  if (!dec_ok(dp.status)) return;
  const uint64_t npix = (uint64_t)dp.P * dp.H * dp.W;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < npix; e += stride) {
    const uint64_t j = e % dp.W, t = e / dp.W;
    const uint64_t i = t % dp.H, p = t / dp.H;
    const uint64_t g = (p * dp.Hb + i / dp.b) * dp.Wb + j / dp.b;
    dp.frame[e] = (float)((double)dp.res[g] * dp.step);
  }
}

__global__ __launch_bounds__(256) void k_dec_roi(DecodePlan dp) {
  if (!dec_ok(dp.status)) return;
  const uint64_t ww = (uint64_t)dp.w * dp.w;
  const uint64_t n = (uint64_t)dp.npeaks * ww;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  const uint16_t *pk = (const uint16_t *)(dp.in + dp.off_peaks);
  const uint32_t *pay = (const uint32_t *)(dp.in + dp.off_roi);
  const int64_t h = dp.w / 2;
  for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += stride) {
    const uint64_t k = e / ww, rem = e - k * ww;
    const int64_t u = rem / dp.w, v = rem - u * dp.w;
    const int64_t pa = pk[3 * k], i = (int64_t)pk[3 * k + 1] - h + u,
                  j = (int64_t)pk[3 * k + 2] - h + v;
    if (pa < dp.P && i >= 0 && i < dp.H && j >= 0 && j < dp.W)
      ((uint32_t *)dp.frame)[((uint64_t)pa * dp.H + i) * dp.W + j] = pay[e];
  }
}

// Overlapping windows copy the same frame pixel: every payload entry must
// match what was restored at its pixel, else the stream is malformed.
__global__ __launch_bounds__(256) void k_dec_roi_check(DecodePlan dp) {
  if (!dec_ok(dp.status)) return;
  const uint64_t ww = (uint64_t)dp.w * dp.w;
  const uint64_t n = (uint64_t)dp.npeaks * ww;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  const uint16_t *pk = (const uint16_t *)(dp.in + dp.off_peaks);
  const uint32_t *pay = (const uint32_t *)(dp.in + dp.off_roi);
  const int64_t h = dp.w / 2;
  bool bad = false;
  for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += stride) {
    const uint64_t k = e / ww, rem = e - k * ww;
    const int64_t u = rem / dp.w, v = rem - u * dp.w;
    const int64_t pa = pk[3 * k], i = (int64_t)pk[3 * k + 1] - h + u,
                  j = (int64_t)pk[3 * k + 2] - h + v;
    if (pa < dp.P && i >= 0 && i < dp.H && j >= 0 && j < dp.W)
      bad |= ((const uint32_t *)dp.frame)[((uint64_t)pa * dp.H + i) * dp.W + j] != pay[e];
  }
  if (bad) corrupt(dp.status);
}

#define RSZ_DLAUNCH(name, kern, grid, block, s)                      \
  do {                                                               \
    prof_begin(name, s);                                             \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, dp);     \
    prof_end(s);                                                     \
    hipError_t e_ = hipGetLastError();                               \
    if (e_ != hipSuccess) return e_;                                 \
  } while (0)

hipError_t launch_decompress(const DecodePlan &dp, hipStream_t s) {
  RSZ_DLAUNCH("k_dec_tables", k_dec_tables, 1, 256, s);
  RSZ_DLAUNCH("k_dec_chunks", k_dec_chunks, (dp.nchunks + 63) / 64, 64, s);
  if (dp.n_out) RSZ_DLAUNCH("k_dec_outliers", k_dec_outliers, (dp.n_out + 255) / 256, 256, s);
  RSZ_DLAUNCH("k_dec_rows", k_dec_rows, (dp.P * dp.Hb + 3) / 4, 256, s);
  RSZ_DLAUNCH("k_dec_cols", k_dec_cols, (dp.P * dp.Wb + 255) / 256, 256, s);
  const uint64_t npix = (uint64_t)dp.P * dp.H * dp.W;
  RSZ_DLAUNCH("k_dec_expand", k_dec_expand, (uint32_t)std::min<uint64_t>((npix + 255) / 256, 1u << 20),
              256, s);
  const uint64_t nroi = (uint64_t)dp.npeaks * dp.w * dp.w;
  if (nroi) {
    const uint32_t g = (uint32_t)std::min<uint64_t>((nroi + 255) / 256, 1u << 20);
    RSZ_DLAUNCH("k_dec_roi", k_dec_roi, g, 256, s);
    RSZ_DLAUNCH("k_dec_roi_check", k_dec_roi_check, g, 256, s);
  }
  return hipSuccess;
}

uint64_t decode_tables_bytes() { return 4ull * kTabWords; }

}  // namespace rsz
