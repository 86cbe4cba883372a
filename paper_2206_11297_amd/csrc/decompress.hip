// decompress.hip -- HIP kernels that decode ROIBIN-SZ streams on gfx950.
//
// Each kernel is launched once for all the streams of a call: its workgroups
// are numbered across the streams (per-kernel prefixes of per-stream
// counts), and a workgroup works on one stream's plan.
//   k_dec_tables    one workgroup per stream: check code lengths (<= 32,
//                   complete prefix code), peaks and chunk offsets; build
//                   canonical decode tables (11-bit single- and multi-symbol
//                   lookup tables + per-length first codes); write the
//                   status of a stream the host rejected.
//   k_dec_run_zero  runs coded: clear the words the runs expand into.
//   k_dec_runs      runs coded: one thread per chunk expands its Rice-coded
//                   zero runs back into the Huffman bits (a word at a time),
//                   checking parameters, offsets and that every one bit stays
//                   inside its chunk.
//   k_dec_chunks    one wave per 4096-symbol chunk, lanes on slices of its
//                   bits (self-synchronising starts): Huffman decode to
//                   residuals (runs of the one-bit residual-0 codeword 32 at
//                   a time; the chunk zeroed with whole-row stores first, then
//                   only nonzero residuals stored); each chunk must end
//                   exactly at the next offset.
//   k_dec_outliers  scatter outlier residuals onto the code-0 positions.
//   k_dec_rows      inclusive prefix sum along each bin row (wrapping int32),
//                   four rows per wave.
//   k_dec_carry, k_dec_rowadd  dimension 1: carries across the rows.
//   k_dec_cols      inclusive prefix sum down each bin column -> q; for
//                   dimension 2 it also writes every pixel float(q * 2eb)
//                   of its bin.
//   k_dec_panel     dimension 2 with a panel's bins in LDS (instead of
//                   k_dec_rows and k_dec_cols): one workgroup per panel, row
//                   sums, column sums and pixels.
//   k_dec_panels    dimension 3: prefix sum across the panels.
//   k_dec_expand    dimensions 1 and 3, one wave per bin row: every pixel
//                   gets float(q * 2eb) of its bin.
//   k_dec_roi_tables, k_dec_roi_decode, k_dec_roi_unpred  coded ROI: class
//                   tables, per-window decode, inverse prediction.
//   k_dec_roi       ROI windows restored from the payload bits, one wave
//                   per window.
//   k_dec_roi_check overlapping windows must agree on their shared pixels
//                   (one wave per window).
// The inverse Lorenzo step is the prefix sum of the residuals along each
// axis the predictor spans.
#include <algorithm>

#include "rsz_internal.h"

namespace rsz {

constexpr int kLutBits = 11;
constexpr int32_t kMark = INT32_MIN;  // residual slot waiting for its outlier

// Dimension 2 where a panel's bins fit in LDS (and a bin row in one
// workgroup's threads): one workgroup per panel takes the row sums, the
// column sums and the pixel writes, so the residuals make one trip from HBM.
constexpr uint32_t kPanelBins = 19200;
constexpr uint32_t kPanelThreads = 1024;
__host__ __device__ inline bool panel_in_lds(const DecodePlan &dp) {
  return dp.dim == 2 && (uint64_t)dp.Hb * dp.Wb <= kPanelBins && dp.Wb <= kPanelThreads;
}


// tables: [0,2048) lut (sym | len << 16, 0 = longer code), then first[33],
// count[33], offs[33], sorted[1024], then the multi-symbol table: per 11-bit
// window two words, (up to 3 whole codewords' symbols, 10 bits each) | count
// << 30 and the bit position after each of them (4 bits each)
constexpr int kTabLut = 0, kTabFirst = 1 << kLutBits, kTabCount = kTabFirst + 33,
              kTabOffs = kTabCount + 33, kTabSorted = kTabOffs + 33,
              kTabMulti = kTabSorted + kNumSym, kTabWords = kTabMulti + 2 * (1 << kLutBits);

__device__ __forceinline__ void corrupt(int32_t *status) {
  atomicCAS(status, (int32_t)RSZ_OK, (int32_t)RSZ_ERR_CORRUPT);
}

__device__ __forceinline__ bool dec_ok(const int32_t *status) {
  return __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == RSZ_OK;
}

__device__ __forceinline__ uint32_t rd32(const uint8_t *p, uint64_t off) {
  return *(const uint32_t *)(p + off);
}

// A batch of streams: each kernel's workgroups are numbered across the
// frames, kernel K's per-frame counts in the prefix pre[K * (n + 1) ...]; a
// workgroup finds its frame (the last with prefix <= its index) and works on
// that frame's plan with its index and count inside the frame.
__device__ __forceinline__ uint32_t dec_frame(const uint32_t *pre, uint32_t n, uint32_t b) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}
#define RSZ_DEC_FRAME(K)                                                   \
  const uint32_t *pre_ = db.pre + (size_t)(K) * (db.n + 1);                \
  const uint32_t f_ = dec_frame(pre_, db.n, blockIdx.x);                   \
  const uint32_t bid = blockIdx.x - pre_[f_];                              \
  const uint32_t nblk = pre_[f_ + 1] - pre_[f_];                           \
  (void)bid;                                                               \
  (void)nblk;                                                              \
  const DecodePlan &dp = db.plans[f_]

__global__ __launch_bounds__(256) void k_dec_tables(DecBatch db) {
  RSZ_DEC_FRAME(0);
  __shared__ uint8_t s_len[kNumSym];
  __shared__ uint32_t s_count[kMaxLen + 1], s_first[kMaxLen + 1], s_offs[kMaxLen + 1],
      s_fill[kMaxLen + 1];
  __shared__ uint16_t s_sorted[kNumSym];
  __shared__ uint32_t s_lut[1 << kLutBits];
  __shared__ unsigned long long s_kraft;
  __shared__ int s_used, s_bad;
  // a stream the host already rejected gets its status and no other work
  if (dp.init_status != RSZ_OK) {
    if (threadIdx.x == 0) *dp.status = dp.init_status;
    return;
  }
  if (threadIdx.x == 0) {
    s_kraft = 0;
    s_used = 0;
    s_bad = 0;
    *dp.status = RSZ_OK;
  }
  if (threadIdx.x <= kMaxLen) {
    s_count[threadIdx.x] = 0;
    s_fill[threadIdx.x] = 0;
  }
  for (int i = threadIdx.x; i < kNumSym; i += 256) s_sorted[i] = 0;
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
      s_first[L] = (uint32_t)code;
      s_offs[L] = start;
      start += s_count[L];
      prev = s_count[L];
    }
  }
  __syncthreads();
  if (threadIdx.x <= kMaxLen && threadIdx.x > 0) {
    tab[kTabFirst + threadIdx.x] = s_first[threadIdx.x];
    tab[kTabCount + threadIdx.x] = s_count[threadIdx.x];
    tab[kTabOffs + threadIdx.x] = s_offs[threadIdx.x];
  }
  // symbols in (length, symbol) order: wave 0 walks the symbols 64 at a
  // time; a symbol's rank among its length is the count of earlier ones
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    for (int i = 0; i < kNumSym / 64; ++i) {
      const uint32_t sym = i * 64 + lane, L = s_len[sym];
      uint64_t pending = __builtin_amdgcn_uicmp(L, 0u, 33 /* ne */);
      while (pending) {
        const int leader = __builtin_ctzll(pending);
        const uint32_t Lc = __builtin_amdgcn_readlane(L, leader);
        const uint64_t same = __builtin_amdgcn_uicmp(L, Lc, 32 /* eq */) & pending;
        if ((same >> lane) & 1ull)
          s_sorted[s_offs[Lc] + s_fill[Lc] + __builtin_popcountll(same & ((1ull << lane) - 1))] =
              (uint16_t)sym;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane == leader) s_fill[Lc] += (uint32_t)__builtin_popcountll(same);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        pending &= ~same;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kNumSym; i += 256) tab[kTabSorted + i] = s_sorted[i];
  // lookup entry of an 11-bit window: the codeword (at most 11 bits) that is
  // its prefix, if any (the code is prefix-free: at most one)
  for (uint32_t x = threadIdx.x; x < (1u << kLutBits); x += 256) {
    uint32_t e = 0;
    for (uint32_t L = 1; L <= (uint32_t)kLutBits; ++L) {
      const uint32_t n = s_count[L];
      const uint32_t cd = x >> (kLutBits - L);
      if (n && cd - s_first[L] < n) {
        e = (uint32_t)s_sorted[s_offs[L] + cd - s_first[L]] | (L << 16);
        break;
      }
    }
    s_lut[x] = e;
    tab[kTabLut + x] = e;
  }
  __syncthreads();
  // multi-symbol entry: the whole codewords (at most 3) that the window
  // holds one after the other
  for (uint32_t x = threadIdx.x; x < (1u << kLutBits); x += 256) {
    uint32_t syms = 0, n = 0, pos = 0, ends = 0;
    while (n < 3) {
      const uint32_t e = s_lut[(x << pos) & ((1u << kLutBits) - 1)];
      const uint32_t L = e >> 16;
      if (!e || pos + L > (uint32_t)kLutBits) break;
      syms |= (e & 0x3FFu) << (10 * n);
      pos += L;
      ends |= pos << (4 * n);
      ++n;
    }
    tab[kTabMulti + 2 * x] = syms | n << 30;
    tab[kTabMulti + 2 * x + 1] = ends;
  }
}

// Four stream words from word index w (0 past the stream's end).
__device__ __forceinline__ uint4 ld4(const uint32_t *bw_, uint64_t nwords, uint64_t w) {
  const RSZ_G uint32_t *bw = gm(bw_);
  uint4 r;
  r.x = w < nwords ? bw[w] : 0u;
  r.y = w + 1 < nwords ? bw[w + 1] : 0u;
  r.z = w + 2 < nwords ? bw[w + 2] : 0u;
  r.w = w + 3 < nwords ? bw[w + 3] : 0u;
  return r;
}

// Exclusive prefix sum of v over the lanes of a wave; total of all lanes.
__device__ __forceinline__ uint64_t wave_exclusive_scan_u64(uint64_t v, uint64_t &total) {
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

__device__ __forceinline__ uint32_t pick8(const uint4 &a, const uint4 &b, uint32_t i) {
  const uint32_t lo = (i & 3) == 0 ? a.x : (i & 3) == 1 ? a.y : (i & 3) == 2 ? a.z : a.w;
  const uint32_t hi = (i & 3) == 0 ? b.x : (i & 3) == 1 ? b.y : (i & 3) == 2 ? b.z : b.w;
  return i < 4 ? lo : hi;
}

// Decoder state of one lane: its stream bits come through a window of three
// 4-word blocks (the third loading while the first two are decoded).
struct BitWindow {
  const uint32_t *bw;
  uint64_t nwords, wb;   // wb: word index of block A
  uint4 A, B, C;
  __device__ void init(const uint32_t *words, uint64_t n, uint64_t pos) {
    bw = words;
    nwords = n;
    wb = pos >> 5;
    A = ld4(bw, nwords, wb);
    B = ld4(bw, nwords, wb + 4);
    C = ld4(bw, nwords, wb + 8);
  }
  // the 32 stream bits from bit `pos` (pos never moves back)
  __device__ uint32_t peek(uint64_t pos) {
    uint32_t r = (uint32_t)((pos >> 5) - wb);
    while (r >= 4) {
      A = B;
      B = C;
      wb += 4;
      C = ld4(bw, nwords, wb + 8);
      r -= 4;
    }
    const uint64_t two = ((uint64_t)pick8(A, B, r) << 32) | pick8(A, B, r + 1);
    return (uint32_t)((two << (pos & 31)) >> 32);
  }
};

// Decodes codewords from `pos` while pos < lim: returns the count and leaves
// pos at the first boundary >= lim; with WRITE, writes each nonzero residual
// (kMark for code 0) at out[k] for k < cap (out holds zeros already).
// `inval` reports a bit pattern that is no codeword.  With `zrun` (residual
// 0's codeword is the single bit 0), a run of z zero bits is z residual-0
// symbols, taken at once up to lim.
// One decoded symbol other than residual 0 into slot k: a residual, or the
// outlier mark for code 0; with out8 (k_dec_panel's streams) a code byte,
// and the residual in out only when the byte is 0.
__device__ __forceinline__ void put_sym(int32_t *out, uint8_t *out8, uint32_t k, uint32_t sym) {
  const int32_t r = sym ? (int32_t)sym - kRadius : kMark;
  if (out8) {
    const bool small = sym && (uint32_t)(r + 127) < 255u;
    *gm(out8 + k) = small ? (uint8_t)(r + 128) : (uint8_t)0;
    if (!small) *gm(out + k) = r;
  } else {
    *gm(out + k) = r;
  }
}

template <bool WRITE>
__device__ __forceinline__ uint32_t decode_run(BitWindow &win, uint64_t &pos, uint64_t lim,
                                               const uint2 *s_multi, const uint32_t *s_first,
                                               const uint32_t *s_count, const uint32_t *s_offs,
                                               const uint16_t *s_sorted, int32_t *out,
                                               uint32_t cap, uint32_t &zeros, bool &inval,
                                               bool zrun, uint8_t *out8 = nullptr) {
  uint32_t m = 0;
  while (pos < lim) {
    const uint32_t v = win.peek(pos);
    if (zrun && !(v >> 31)) {
      const uint32_t z = v ? (uint32_t)__builtin_clz(v) : 32u;
      const uint32_t take = (uint32_t)min<uint64_t>(z, lim - pos);
      pos += take;
      m += take;
      continue;
    }
    const uint2 e = s_multi[v >> (32 - kLutBits)];
    const uint32_t n = e.x >> 30;
    if (n) {
      // up to n symbols, stopping after the first that reaches lim
      uint32_t take = 1;
      while (take < n && pos + ((e.y >> (4 * (take - 1))) & 0xFu) < lim) ++take;
      for (uint32_t j = 0; j < take; ++j) {
        const uint32_t sym = (e.x >> (10 * j)) & 0x3FFu;
        zeros += sym == 0;
        if (WRITE && m + j < cap && sym != kRadius) put_sym(out, out8, m + j, sym);
      }
      pos += (e.y >> (4 * (take - 1))) & 0xFu;
      m += take;
    } else {
      uint32_t L = 0, sym = 0;
      for (uint32_t l = kLutBits + 1; l <= (uint32_t)kMaxLen; ++l) {
        const uint32_t cd = v >> (32 - l);
        if (s_count[l] && cd >= s_first[l] && cd - s_first[l] < s_count[l]) {
          L = l;
          sym = s_sorted[s_offs[l] + cd - s_first[l]];
          break;
        }
      }
      if (L == 0) {
        inval = true;
        break;
      }
      zeros += sym == 0;
      if (WRITE && m < cap && sym != kRadius) put_sym(out, out8, m, sym);
      pos += L;
      ++m;
    }
  }
  return m;
}

// ------------------------------------------------------------ run stage

constexpr uint32_t kRunKMax = 20;

__global__ __launch_bounds__(256) void k_dec_run_zero(DecBatch db) {
  RSZ_DEC_FRAME(1);
  const uint64_t n = (dp.T + 31) / 32 + 2;
  for (uint64_t i = bid * 256ull + threadIdx.x; i < n; i += nblk * 256ull)
    dp.hbits[i] = 0u;
}

// The 32 bits of words (n of them, zero beyond) from bit pos, MSB-first.
__device__ __forceinline__ uint32_t peek_bits(const uint32_t *w, uint64_t n, uint64_t pos) {
  const uint64_t i = pos >> 5;
  const uint32_t s = (uint32_t)(pos & 31);
  const uint32_t hi = i < n ? w[i] : 0u, lo = i + 1 < n ? w[i + 1] : 0u;
  return s ? (hi << s) | (lo >> (32 - s)) : hi;
}

// Chunk c's codes occupy run bits [runoffs[c], runoffs[c + 1]): each is a
// unary quotient q (ones closed by a zero) and k low bits, giving the zero
// run before the chunk's next one bit.  A valid section has parameters <= 20
// (zero padding), offsets from 0 that never decrease, a last offset whose
// words end the stream exactly, codes that end exactly at the next offset,
// and every one bit inside its chunk [chunk_off[c], chunk_off[c + 1]).
// Reads stay inside the section once its size is checked; the loop ends
// after at most one step per run bit.
__global__ __launch_bounds__(256) void k_dec_runs(DecBatch db) {
  RSZ_DEC_FRAME(2);
  const uint32_t c = bid * 256 + threadIdx.x;
  if (c >= dp.nchunks || !dec_ok(dp.status)) return;
  const uint8_t *kpar = dp.in + dp.off_run;
  const uint32_t *ro = (const uint32_t *)(dp.in + dp.off_runoffs);
  const uint64_t Trun = ro[dp.nchunks];
  const uint64_t nrw = (Trun + 31) / 32;
  bool bad = dp.off_runbits + 4 * nrw != dp.total || ro[0] != 0 || kpar[c] > kRunKMax;
  if (c + 1 == dp.nchunks)   // padding of the parameters
    for (uint64_t t = dp.nchunks; t < align_up(dp.nchunks, 4); ++t) bad |= kpar[t] != 0;
  const uint32_t *co = (const uint32_t *)(dp.in + dp.off_chunks);
  const uint64_t start = co[c], end = c + 1 < dp.nchunks ? co[c + 1] : dp.T;
  uint64_t pos = ro[c];
  const uint64_t rend = ro[c + 1];
  bad |= start > end || end > dp.T || rend < pos || rend > Trun;
  if (bad) {
    corrupt(dp.status);
    return;
  }
  const uint32_t *rw = (const uint32_t *)(dp.in + dp.off_runbits);
  const uint32_t k = kpar[c];
  uint64_t b = start;   // next Huffman bit position
  // the one bits of the current word gather in acc; a word wholly inside
  // the chunk is this thread's alone (a plain store), the two it may share
  // with the chunks beside it take an atomic OR
  uint64_t cw = 0;
  uint32_t acc = 0;
  auto flush = [&]() {
    if (!acc) return;
    if (cw * 32 >= start && cw * 32 + 32 <= end) dp.hbits[cw] = acc;
    else atomicOr(&dp.hbits[cw], acc);
  };
  while (pos < rend) {
    uint64_t q = 0;
    for (;;) {   // the unary part, up to 32 bits a step
      const uint32_t x = peek_bits(rw, nrw, pos);
      const uint64_t avail = min<uint64_t>(32, rend - pos);
      const uint64_t n = ~x ? (uint64_t)__builtin_clz(~x) : 32;   // leading ones
      if (n < avail) {
        q += n;
        pos += n + 1;   // and the closing zero
        break;
      }
      q += avail;
      pos += avail;
      // no closing zero before the chunk's end, or a run past the chunk
      if (pos >= rend || b + (q << k) >= end) bad = true;
      if (bad) break;
    }
    if (bad || pos + k > rend) {
      bad = true;
      break;
    }
    const uint64_t low = k ? peek_bits(rw, nrw, pos) >> (32 - k) : 0;
    pos += k;
    b += (q << k) | low;
    if (b >= end) {
      bad = true;
      break;
    }
    if ((b >> 5) != cw) {
      flush();
      cw = b >> 5;
      acc = 0;
    }
    acc |= 0x80000000u >> (b & 31);
    b++;
  }
  if (bad) corrupt(dp.status);
  else flush();
}

// One wave per chunk.  The chunk's bits split into 64 equal slices; lane i
// decodes from a start s_i until the first codeword boundary at or past the
// next slice.  Lane 0 starts at the chunk offset, a true boundary; every
// other lane starts at its slice's first bit, then again at the boundary the
// lane before it stopped at, until no start changes: then every start is a
// true boundary (by induction from lane 0).  Huffman decoding
// resynchronises within a few codewords, so this takes one or two rounds
// (64 at most).  A scan of the lanes' symbol counts places their outputs, and
// a last pass writes them.  A valid chunk decodes to exactly its symbol count
// and ends exactly at the next chunk offset.
__global__ __launch_bounds__(256) void k_dec_chunks(DecBatch db) {
  RSZ_DEC_FRAME(3);
  __shared__ uint2 s_multi[1 << kLutBits];
  __shared__ uint32_t s_first[kMaxLen + 1], s_count[kMaxLen + 1], s_offs[kMaxLen + 1];
  __shared__ uint16_t s_sorted[kNumSym];
  for (int i = threadIdx.x; i < (1 << kLutBits); i += 256)
    s_multi[i] = make_uint2(dp.tables[kTabMulti + 2 * i], dp.tables[kTabMulti + 2 * i + 1]);
  for (int i = threadIdx.x; i < kNumSym; i += 256) s_sorted[i] = (uint16_t)dp.tables[kTabSorted + i];
  if (threadIdx.x <= kMaxLen) {
    s_first[threadIdx.x] = dp.tables[kTabFirst + threadIdx.x];
    s_count[threadIdx.x] = dp.tables[kTabCount + threadIdx.x];
    s_offs[threadIdx.x] = dp.tables[kTabOffs + threadIdx.x];
  }
  __syncthreads();
  // residual 0 (symbol 512) coded as the single bit 0: the only length-1
  // code, canonical code 0
  const bool zrun = s_count[1] == 1 && s_first[1] == 0 && s_sorted[s_offs[1]] == kRadius;
  const int lane = threadIdx.x & 63;
  const uint32_t c = bid * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (c >= dp.nchunks || !dec_ok(dp.status)) return;
  const RSZ_G uint32_t *co = gm((const uint32_t *)(dp.in + dp.off_chunks));
  const uint32_t *bw = dp.bits;   // the stream's bitstream, or the expanded runs
  const uint64_t nwords = (dp.T + 31) / 32;
  const uint64_t S = co[c], E = c + 1 < dp.nchunks ? co[c + 1] : dp.T;
  const uint32_t g0 = c * kChunk;
  const uint32_t nsym = min(kChunk, dp.nbins - g0);
  const uint64_t len = E > S ? E - S : 0;
  const uint64_t lim = lane == 63 ? E : S + len * (uint64_t)(lane + 1) / 64;
  uint64_t start = lane == 0 ? S : S + len * (uint64_t)lane / 64;
  uint64_t stop = start;
  uint32_t m = 0;
  bool converged = false, inv = false;
  for (int round = 0; round <= 64 && !converged; ++round) {
    BitWindow win;
    win.init(bw, nwords, start);
    uint64_t pos = start;
    uint32_t z = 0;
    inv = false;
    m = decode_run<false>(win, pos, lim, s_multi, s_first, s_count, s_offs, s_sorted, nullptr, 0,
                          z, inv, zrun);
    stop = inv ? ~0ull : pos;   // a lane stuck on a non-codeword hands on no boundary
    // the boundary the lane before stopped at is this lane's next start
    const uint64_t prev = __shfl_up(stop, 1);
    const uint64_t next = lane == 0 ? S : prev;
    const bool changed = lane > 0 && next != start;
    converged = __builtin_amdgcn_uicmp((uint32_t)changed, 0u, 33 /* ne */) == 0;
    if (!converged) start = next == ~0ull ? lim : next;
  }
  uint64_t tot;
  const uint32_t off = (uint32_t)wave_exclusive_scan_u64(m, tot);
  const uint64_t last = __shfl(stop, 63);
  // a valid chunk converges (64 rounds at most) with no non-codeword on its path
  bool bad = !converged || __builtin_amdgcn_uicmp((uint32_t)inv, 0u, 33 /* ne */) != 0 ||
             tot != nsym || last != E;
  inv = false;
  // the output pass, from the true starts: the wave zeroes the chunk's
  // residuals with whole-row stores, waits for them to complete, and the
  // lanes then store only their nonzero residuals (most are 0)
  // (code bytes: 128, residual 0, in 16-byte stores; the region holds 64
  // bytes past the last chunk)
  const bool bytes = panel_in_lds(dp);
  if (!bad) {
    if (bytes) {
      RSZ_G uint8_t *rc = gm(dp.res8 + g0);
      for (uint32_t i = 16 * lane; i < nsym; i += 1024)
        *(RSZ_G u32x4 *)(rc + i) = u32x4{0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u};
    } else {
      RSZ_G int32_t *rc = gm(dp.res + g0);
      for (uint32_t i = 4 * lane; i < nsym; i += 256) {
        if (i + 4 <= nsym) {
          *(RSZ_G u32x4 *)(rc + i) = u32x4{0u, 0u, 0u, 0u};
        } else {
          for (uint32_t k = i; k < nsym; ++k) rc[k] = 0;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  }
  BitWindow win;
  win.init(bw, nwords, start);
  uint64_t pos = start;
  uint32_t zeros = 0;
  if (!bad)
    decode_run<true>(win, pos, lim, s_multi, s_first, s_count, s_offs, s_sorted, dp.res + g0 + off,
                     off < nsym ? nsym - off : 0u, zeros, inv, zrun,
                     bytes ? dp.res8 + g0 + off : nullptr);
  bad |= __builtin_amdgcn_uicmp((uint32_t)inv, 0u, 33 /* ne */) != 0;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) zeros += __shfl_xor(zeros, d);
  if (lane == 0) {
    if (bad) corrupt(dp.status);
    *gm(dp.zcount + c) = zeros;
  }
}

// The outliers into their bins' residual slots; the frame's workgroups take
// every nblk-th block of 256 (a verification plan launches a fixed number
// per frame, the outlier count being known only on the device).
__global__ __launch_bounds__(256) void k_dec_outliers(DecBatch db) {
  RSZ_DEC_FRAME(4);
  if (!dec_ok(dp.status)) return;
  const uint32_t *oi = (const uint32_t *)(dp.in + dp.off_oidx);
  const int32_t *orr = (const int32_t *)(dp.in + dp.off_ores);
  // |q| < 2^28 bounds a residual of dimension d below 2^(28+d) in magnitude
  const int64_t lim = (int64_t)1 << (28 + dp.dim);
  for (uint32_t k = bid * 256 + threadIdx.x; k < dp.n_out; k += nblk * 256) {
    const uint32_t g = oi[k];
    const int32_t r = orr[k];
    // the bin must have decoded as code 0 (its code byte 0 and the mark in res)
    if (g >= dp.nbins || (k > 0 && g <= oi[k - 1]) || (r > -kRadius && r < kRadius) ||
        (int64_t)r <= -lim || (int64_t)r >= lim || (panel_in_lds(dp) && dp.res8[g] != 0) ||
        dp.res[g] != kMark) {
      corrupt(dp.status);
      return;
    }
    dp.res[g] = r;
  }
}

// One wave per bin row: inclusive prefix sum along the row.
constexpr uint32_t kDecRowsPerWave = 4;   // bin rows per wave of k_dec_rows
__global__ __launch_bounds__(256) void k_dec_rows(DecBatch db) {
  RSZ_DEC_FRAME(5);
  const uint32_t row0 = (bid * 4 + (threadIdx.x >> 6)) * kDecRowsPerWave;
  const int lane = threadIdx.x & 63;
  const uint32_t nrows = dp.P * dp.Hb;
  if (row0 >= nrows || !dec_ok(dp.status)) return;
  const uint32_t Wb = dp.Wb;
  if (Wb <= 256) {
    // four consecutive bins per lane, the wave's rows all loaded first; per
    // row the lanes' prefixes and one wave scan of their totals
    int32_t v[kDecRowsPerWave][4];
#pragma unroll
    for (uint32_t rr = 0; rr < kDecRowsPerWave; ++rr)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint32_t j = 4 * lane + t;
        v[rr][t] = row0 + rr < nrows && j < Wb ? dp.res[(size_t)(row0 + rr) * Wb + j] : 0;
      }
    bool bad = false;
#pragma unroll
    for (uint32_t rr = 0; rr < kDecRowsPerWave; ++rr) {
      if (row0 + rr >= nrows) break;
      uint32_t x[4], sum = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        bad |= v[rr][t] == kMark;
        sum += (uint32_t)v[rr][t];
        x[t] = sum;
      }
      const uint32_t incl = wave_inclusive_sum(sum);
      const uint32_t before = incl - sum;
      int32_t *r = dp.res + (size_t)(row0 + rr) * Wb;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint32_t j = 4 * lane + t;
        if (j < Wb) r[j] = (int32_t)(x[t] + before);
      }
    }
    if (bad) corrupt(dp.status);
    return;
  }
  bool bad = false;
  for (uint32_t row = row0; row < min(row0 + kDecRowsPerWave, nrows); ++row) {
    int32_t *r = dp.res + (size_t)row * Wb;
    uint32_t carry = 0;
    for (uint32_t j0 = 0; j0 < Wb; j0 += 64) {
      const uint32_t j = j0 + lane;
      uint32_t x = 0;
      if (j < Wb) {
        const int32_t v = r[j];
        bad |= v == kMark;
        x = (uint32_t)v;
      }
      x = wave_inclusive_sum(x) + carry;
      if (j < Wb) r[j] = (int32_t)x;
      carry = __builtin_amdgcn_readlane(x, 63);
    }
  }
  if (bad) corrupt(dp.status);
}

// One lane per bin column: inclusive prefix sum down the column.
// The pixels of bin (I, J) of a panel whose first pixel is out get v:
// rows [I*b, min(I*b + b, H)), columns [J*b, min(J*b + b, W)).  For b = 2 or 4
// with W a multiple of b a bin's pixels of one row are an aligned float2 /
// float4 (the frame is 16-byte aligned).
__device__ __forceinline__ void fill_bin(float *out_, uint32_t H, uint32_t W, uint32_t b,
                                         uint32_t I, uint32_t J, float v) {
  RSZ_G float *out = gm(out_);
  const uint32_t i0 = I * b, i1 = min(i0 + b, H), j0 = J * b;
  if (b == 2 && W % 2 == 0) {
    for (uint32_t i = i0; i < i1; ++i) *(RSZ_G f32x2 *)(out + (size_t)i * W + j0) = f32x2{v, v};
  } else if (b == 4 && W % 4 == 0) {
    for (uint32_t i = i0; i < i1; ++i)
      *(RSZ_G f32x4 *)(out + (size_t)i * W + j0) = f32x4{v, v, v, v};
  } else {
    const uint32_t j1 = min(j0 + b, W);
    for (uint32_t i = i0; i < i1; ++i)
      for (uint32_t j = j0; j < j1; ++j) out[(size_t)i * W + j] = v;
  }
}

__global__ __launch_bounds__(256) void k_dec_cols(DecBatch db) {
  RSZ_DEC_FRAME(8);
  const uint32_t col = bid * 256 + threadIdx.x;
  if (col >= dp.P * dp.Wb || !dec_ok(dp.status)) return;
  const uint32_t p = col / dp.Wb, J = col - p * dp.Wb;
  int32_t *r = dp.res + (size_t)p * dp.Hb * dp.Wb + J;
  const size_t Wb = dp.Wb;
  // dimension 2: q is final here, so its pixels are written at once (no
  // expansion pass re-reads the residuals); dimension 3 stores q for the
  // sum across the panels
  const bool fill = dp.dim == 2;
  float *out = dp.frame + (size_t)p * dp.H * dp.W;
  const uint32_t H = dp.H, W = dp.W, b = dp.b;
  const double step = dp.step;
  auto put = [&](uint32_t I, uint32_t acc) {
    if (fill) fill_bin(out, H, W, b, I, J, (float)((double)(int32_t)acc * step));
    else r[I * Wb] = (int32_t)acc;
  };
  uint32_t acc = 0;
  uint32_t I = 0;
  // eight rows loaded before any is stored (a store would otherwise hold
  // back the next load: the compiler cannot reorder them)
  for (; I + 8 <= dp.Hb; I += 8) {
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = (uint32_t)r[(I + k) * Wb];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      acc += v[k];
      put(I + k, acc);
    }
  }
  for (; I < dp.Hb; ++I) {
    acc += (uint32_t)r[I * Wb];
    put(I, acc);
  }
}

// Dimension 1: the raster sequence continues across rows, so each row adds
// the sum of every row before it.  One workgroup scans the row totals (the
// last element of each row-scanned row) into exclusive carries.
__global__ __launch_bounds__(256) void k_dec_carry(DecBatch db) {
  RSZ_DEC_FRAME(6);
  __shared__ uint32_t s_w[4];
  if (!dec_ok(dp.status)) return;
  const uint32_t rows = dp.P * dp.Hb;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t run = 0;
  for (uint32_t r0 = 0; r0 < rows; r0 += 256) {
    const uint32_t row = r0 + threadIdx.x;
    uint32_t x = row < rows ? (uint32_t)dp.res[(size_t)row * dp.Wb + dp.Wb - 1] : 0u;
    const uint32_t v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    if (lane == 63) s_w[wv] = x;
    __syncthreads();
    uint32_t before = run;
    for (int i = 0; i < wv; ++i) before += s_w[i];
    if (row < rows) dp.carry[row] = before + x - v;
    run += s_w[0] + s_w[1] + s_w[2] + s_w[3];
    __syncthreads();
  }
}

// Dimension 1: adds each row's carry (one lane per bin).
__global__ __launch_bounds__(256) void k_dec_rowadd(DecBatch db) {
  RSZ_DEC_FRAME(7);
  if (!dec_ok(dp.status)) return;
  const uint64_t stride = (uint64_t)nblk * 256;
  for (uint64_t g = (uint64_t)bid * 256 + threadIdx.x; g < dp.nbins; g += stride)
    dp.res[g] = (int32_t)((uint32_t)dp.res[g] + dp.carry[g / dp.Wb]);
}

// Dimension 3: inclusive prefix sum across the panels (one lane per bin
// position of the panel plane), after the 2D sums of each panel.
__global__ __launch_bounds__(256) void k_dec_panels(DecBatch db) {
  RSZ_DEC_FRAME(9);
  const uint32_t plane = dp.Hb * dp.Wb;
  const uint32_t c = bid * 256 + threadIdx.x;
  if (c >= plane || !dec_ok(dp.status)) return;
  int32_t *r = dp.res + c;
  uint32_t acc = 0;
  for (uint32_t p = 0; p < dp.P; ++p) {
    acc += (uint32_t)r[(size_t)p * plane];
    r[(size_t)p * plane] = (int32_t)acc;
  }
}

// One wave per bin row: each lane takes a bin, computes its value once and
// writes it to the bin's b x b pixels (clipped at the panel edges), a raw
// row at a time, so the wave's stores of a row are contiguous.
__global__ __launch_bounds__(1024) void k_dec_panel(DecBatch db) {
  RSZ_DEC_FRAME(16);
  // s_v[lead + i]: residual i of the panel, lead = the panel's byte offset
  // in its 16-byte line (the loads below are whole aligned lines)
  __shared__ __align__(16) uint32_t s_v[kPanelBins + 32];
  __shared__ uint32_t s_part[kPanelThreads];
  __shared__ int s_ok, s_bad;
  const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
  // one read of the status for the whole workgroup (another panel may
  // change it meanwhile), so every thread takes the same branch
  if (t == 0) {
    s_ok = dec_ok(dp.status);
    s_bad = 0;
  }
  __syncthreads();
  if (!s_ok) return;
  const uint32_t Hb = dp.Hb, Wb = dp.Wb, n = Hb * Wb;
  const RSZ_G int32_t *r = gm(dp.res + (size_t)bid * n);
  // The panel's code bytes into LDS as residuals: aligned 16-byte loads, all
  // of a thread's in flight at once (res8 is 256-byte aligned with 64 bytes
  // to spare past the last bin, so the lines cover the panel and stay in
  // the buffer).  A byte 0 (its residual in res) is marked and filled in a
  // second pass, so that no load waits on another.
  const uint8_t *p8 = dp.res8 + (size_t)bid * n;
  const uint8_t *a8 = (const uint8_t *)((uintptr_t)p8 & ~(uintptr_t)15);
  const uint32_t lead = (uint32_t)(p8 - a8), nw = (lead + n + 15) / 16;
  uint32_t *sv = s_v + lead;
  bool bad = false;
  for (uint32_t w0 = 0; w0 < nw; w0 += 2 * kPanelThreads) {
    uint4 v[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const uint32_t w = w0 + k * kPanelThreads + t;
      v[k] = w < nw ? ld16(a8 + 16 * (size_t)w) : make_uint4(0x80808080u, 0x80808080u,
                                                               0x80808080u, 0x80808080u);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const uint32_t w = w0 + k * kPanelThreads + t;
      if (w < nw) {
        // bytes of this line inside the panel: [lo, hi)
        const int32_t lo = max((int32_t)lead - (int32_t)(16 * w), 0);
        const int32_t hi = min((int32_t)(lead + n) - (int32_t)(16 * w), 16);
        const uint32_t inr = hi > lo ? ((hi == 16 ? 0xFFFFu : (1u << hi) - 1u) & ~((1u << lo) - 1u))
                                     : 0u;
        const uint32_t e[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
        uint32_t zm = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint32_t o[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const uint32_t by = (e[q] >> (8 * j)) & 0xFFu;
            zm |= (by == 0 ? 1u : 0u) << (4 * q + j);
            o[j] = by ? (uint32_t)((int32_t)by - 128) : (uint32_t)kMark;
          }
          *(uint4 *)(s_v + 16 * w + 4 * q) = make_uint4(o[0], o[1], o[2], o[3]);
        }
        // escapes (byte 0): the residual (or the outlier mark) from res,
        // by the thread that holds the byte (rare; no other thread reads
        // these entries before the barrier below)
        for (uint32_t zb = zm & inr; zb; zb &= zb - 1) {
          const uint32_t e16 = (uint32_t)__builtin_ctz(zb);
          const int32_t x = r[16 * w + e16 - lead];
          bad |= x == kMark;
          s_v[16 * w + e16] = (uint32_t)x;
        }
      }
    }
  }
  if (bad) s_bad = 1;
  __syncthreads();
  if (s_bad) {
    if (t == 0) corrupt(dp.status);
    return;
  }
  // row sums: wave w takes rows w, w + 16, ...
  for (uint32_t I = wave; I < Hb; I += kPanelThreads / 64) {
    uint32_t carry = 0;
    for (uint32_t j0 = 0; j0 < Wb; j0 += 64) {
      const uint32_t j = j0 + lane;
      uint32_t x = j < Wb ? sv[I * Wb + j] : 0u;
      x = wave_inclusive_sum(x) + carry;
      if (j < Wb) sv[I * Wb + j] = x;
      carry = __builtin_amdgcn_readlane(x, 63);
    }
  }
  __syncthreads();
  // column sums: thread (g, J) = (t / Wb, t % Wb) takes bin column J over
  // the g-th block of rows; the blocks' totals give each its carry
  const uint32_t G = min(kPanelThreads / Wb, Hb), per = (Hb + G - 1) / G;
  const uint32_t g = t / Wb, J = t - g * Wb;
  const uint32_t I0 = min(g * per, Hb), I1 = min(I0 + per, Hb);
  uint32_t part = 0;
  if (g < G)
    for (uint32_t I = I0; I < I1; ++I) part += sv[I * Wb + J];
  s_part[t] = part;
  __syncthreads();
  float *out = dp.frame + (size_t)bid * dp.H * dp.W;
  const uint32_t H = dp.H, W = dp.W, b = dp.b;
  const double step = dp.step;
  // Linear output (b = 1, 2 or 4 with rows of whole 16-byte groups and the
  // frame 16-byte aligned, so the panel is a run of aligned float4): the
  // bins' values go back into LDS, then the workgroup writes the panel's
  // pixels in order, one float4 per thread and step, so that every store
  // of a wave fills whole cache lines (stores by bin leave a line's pieces
  // to different waves and times).  Otherwise each thread writes its bins'
  // pixels.
  const bool lin = (b == 1 || b == 2 || b == 4) && W % 4 == 0 && ((uintptr_t)out & 15) == 0;
  if (g < G) {
    uint32_t acc = 0;
    for (uint32_t h = 0; h < g; ++h) acc += s_part[h * Wb + J];
    for (uint32_t I = I0; I < I1; ++I) {
      acc += sv[I * Wb + J];
      const float v = (float)((double)(int32_t)acc * step);
      if (lin) sv[I * Wb + J] = __float_as_uint(v);
      else fill_bin(out, H, W, b, I, J, v);
    }
  }
  if (!lin) return;
  __syncthreads();
  const uint32_t sh = b == 1 ? 0u : (b == 2 ? 1u : 2u), W4 = W / 4;
  RSZ_G f32x4 *o4 = gm((f32x4 *)out);
  auto pix4 = [&](const uint32_t *rowv) {
    f32x4 v;
    if (b == 4) {
      v.x = v.y = v.z = v.w = __uint_as_float(rowv[0]);
    } else if (b == 2) {
      v.x = v.y = __uint_as_float(rowv[0]);
      v.z = v.w = __uint_as_float(rowv[1]);
    } else {
      v = f32x4{__uint_as_float(rowv[0]), __uint_as_float(rowv[1]), __uint_as_float(rowv[2]),
                __uint_as_float(rowv[3])};
    }
    return v;
  };
  // A pass covers R whole pixel rows (R a multiple of b), thread t the
  // float4 (t mod W4) of row t / W4: from pass to pass its LDS bin row and
  // its output move by fixed steps, with no division per store.
  uint32_t R = kPanelThreads / W4;
  R -= R % b;
  if (R > 0) {
    const uint32_t r0 = t / W4, c4 = t - r0 * W4;
    if (r0 < R) {
      const uint32_t dv = (R >> sh) * Wb;
      const size_t dO = (size_t)R * W4;
      const uint32_t *rowv = sv + (r0 >> sh) * Wb + ((4 * c4) >> sh);
      RSZ_G f32x4 *o = o4 + (size_t)r0 * W4 + c4;
      for (uint32_t i = r0; i < H; i += R, rowv += dv, o += dO) *o = pix4(rowv);
    }
  } else {
    const FastDiv fW = fast_div(W);
    for (uint32_t c = t; c < H * W4; c += kPanelThreads) {
      const uint32_t i = fdiv(fW, 4 * c), j = 4 * c - i * W;
      o4[c] = pix4(sv + (i >> sh) * Wb + (j >> sh));
    }
  }
}

__global__ __launch_bounds__(256) void k_dec_expand(DecBatch db) {
  RSZ_DEC_FRAME(10);
  const uint32_t brow = bid * 4 + (threadIdx.x >> 6);
  if (brow >= dp.P * dp.Hb || !dec_ok(dp.status)) return;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t p = brow / dp.Hb, I = brow - p * dp.Hb;
  const int32_t *rb = dp.res + (size_t)brow * dp.Wb;
  float *out = dp.frame + (size_t)p * dp.H * dp.W;
  const double step = dp.step;
  for (uint32_t J = lane; J < dp.Wb; J += 64)
    fill_bin(out, dp.H, dp.W, dp.b, I, J, (float)((double)rb[J] * step));
}

// ------------------------------------------------------- coded ROI windows

// Tables of the ROI class code: per length L the first canonical code, the
// number of classes and where they start in the (length, class) order, then
// that order.  The lengths must be a complete prefix code (or one class of
// length 1), padding zero; no class at all when there is no window.
constexpr int kRoiTabFirst = 0, kRoiTabCount = 33, kRoiTabBase = 66, kRoiTabSym = 99;
constexpr int kRoiTabWords = 132;
constexpr int kRoiLutBits = 10;   // k_dec_roi_decode: codes this short by one lookup

__global__ __launch_bounds__(64) void k_dec_roi_tables(DecBatch db) {
  RSZ_DEC_FRAME(11);
  if (threadIdx.x != 0 || !dec_ok(dp.status)) return;
  const uint8_t *lens = dp.in + dp.off_rsec;
  uint32_t *t = dp.roi_tables;
  uint64_t kraft = 0;
  int used = 0;
  bool bad = false;
  for (int c = 0; c < (int)kRoiLens; ++c) {
    const uint32_t L = lens[c];
    if (c >= kRoiClasses ? L != 0 : L > (uint32_t)kMaxLen) bad = true;
    if (c < kRoiClasses && L && L <= (uint32_t)kMaxLen) {
      kraft += 1ull << (kMaxLen - L);
      used++;
    }
  }
  if (dp.npeaks == 0) bad |= used != 0;
  else bad |= !(kraft == (1ull << kMaxLen) || (used == 1 && kraft == (1ull << (kMaxLen - 1))));
  if (bad) {
    corrupt(dp.status);
    return;
  }
  uint32_t code = 0, n = 0, prev_count = 0;
  for (int L = 1; L <= kMaxLen; ++L) {
    code = (code + prev_count) << 1;
    uint32_t cnt = 0;
    t[kRoiTabBase + L - 1] = n;
    for (int c = 0; c < kRoiClasses; ++c)
      if (lens[c] == L) t[kRoiTabSym + n + cnt++] = (uint32_t)c;
    t[kRoiTabFirst + L - 1] = code;
    t[kRoiTabCount + L - 1] = cnt;
    n += cnt;
    prev_count = cnt;
  }
}

// One lane per window: decode its classes and raw bits into the zigzag
// residuals, written as r (mod 2^32) to roi_payload.  A window must start at
// its offset (the first at 0) and end exactly at the next offset, the last
// at Troi.
__global__ __launch_bounds__(256) void k_dec_roi_decode(DecBatch db) {
  RSZ_DEC_FRAME(12);
  // the frame's class tables in LDS, and a lookup of every code of at most
  // kRoiLutBits bits by the stream's next kRoiLutBits bits: class | L << 8
  // (0: a longer code, or none)
  __shared__ uint32_t s_t[kRoiTabWords];
  __shared__ uint16_t s_lut[1 << kRoiLutBits];
  __shared__ int s_ok;
  // one read of the status for the workgroup (a window may set it
  // meanwhile), so that every thread takes the same branch
  if (threadIdx.x == 0) s_ok = dec_ok(dp.status);
  for (uint32_t x = threadIdx.x; x < (uint32_t)kRoiTabWords; x += 256) s_t[x] = dp.roi_tables[x];
  __syncthreads();
  if (!s_ok) return;
  for (uint32_t x = threadIdx.x; x < (1u << kRoiLutBits); x += 256) {
    uint16_t e = 0;
    for (int L = 1; L <= kRoiLutBits; ++L) {
      const uint32_t code = x >> (kRoiLutBits - L);
      const uint32_t cnt = s_t[kRoiTabCount + L - 1], first = s_t[kRoiTabFirst + L - 1];
      if (cnt && code - first < cnt) {
        e = (uint16_t)(s_t[kRoiTabSym + s_t[kRoiTabBase + L - 1] + (code - first)] | (L << 8));
        break;
      }
    }
    s_lut[x] = e;
  }
  __syncthreads();
  const uint32_t k = bid * 256 + threadIdx.x;
  if (k >= dp.npeaks) return;
  const uint32_t *offs = (const uint32_t *)(dp.in + dp.off_roffs);
  const uint32_t *words = (const uint32_t *)(dp.in + dp.off_rbits);
  const uint64_t nwords = (dp.Troi + 31) / 32;
  const uint64_t start = offs[k], end = k + 1 < dp.npeaks ? offs[k + 1] : dp.Troi;
  if ((k == 0 && start != 0) || end < start || end > dp.Troi) {
    corrupt(dp.status);
    return;
  }
  const uint64_t ww = (uint64_t)dp.w * dp.w;
  uint32_t *out = dp.roi_payload + k * ww;
  uint64_t pos = start;
  BitWindow win;   // the window's bits through registers, 4 words a load
  win.init(words, nwords, start);
  for (uint64_t e = 0; e < ww; ++e) {
    const uint32_t peek = win.peek(pos);
    const uint32_t hit = s_lut[peek >> (32 - kRoiLutBits)];
    int cls = -1, L = 1;
    if (hit) {
      cls = (int)(hit & 0xFFu);
      L = (int)(hit >> 8);
    } else {
      for (L = kRoiLutBits + 1; L <= kMaxLen; ++L) {
        const uint32_t code = peek >> (32 - L);
        const uint32_t cnt = s_t[kRoiTabCount + L - 1], first = s_t[kRoiTabFirst + L - 1];
        if (cnt && code - first < cnt) {
          cls = (int)s_t[kRoiTabSym + s_t[kRoiTabBase + L - 1] + (code - first)];
          break;
        }
      }
    }
    if (cls < 0 || pos + L > end) {
      corrupt(dp.status);
      return;
    }
    pos += L;
    uint32_t z = cls == 0 ? 0u : 1u;
    if (cls >= 2) {
      const uint32_t extra = (uint32_t)cls - 1;
      if (pos + extra > end) {
        corrupt(dp.status);
        return;
      }
      z = (1u << extra) | (win.peek(pos) >> (32 - extra));
      pos += extra;
    }
    out[e] = (z >> 1) ^ (0u - (z & 1u));
  }
  if (pos != end) corrupt(dp.status);
}

// One wave per window: undo the prediction.  With D = M - 2^31 (zero outside
// the window), D(u, v) = r + D(u-1, v) + D(u, v-1) - D(u-1, v-1), so D is the
// 2D prefix sum of r: a wave scan along each row plus the column sums kept
// per lane.  Then M = D + 2^31 maps back to the float bits.
constexpr int kRoiMaxChunks = 16;   // w <= 1023: 16 chunks of 64 columns
__global__ __launch_bounds__(256) void k_dec_roi_unpred(DecBatch db) {
  RSZ_DEC_FRAME(13);
  const uint32_t k = bid * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= dp.npeaks || !dec_ok(dp.status)) return;
  const uint32_t w = dp.w;
  uint32_t *win = dp.roi_payload + (uint64_t)k * w * w;
  uint32_t col[kRoiMaxChunks];
#pragma unroll
  for (int c = 0; c < kRoiMaxChunks; ++c) col[c] = 0u;
  for (uint32_t u = 0; u < w; ++u) {
    uint32_t carry = 0;
#pragma unroll
    for (int c = 0; c < kRoiMaxChunks; ++c) {
      if (c * 64 < (int)w) {   // uniform
        const uint32_t v = c * 64 + lane;
        uint32_t x = v < w ? win[u * w + v] : 0u;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t y = __shfl_up(x, d);
          if (lane >= d) x += y;
        }
        x += carry;
        carry = __shfl(x, 63);
        col[c] += x;   // D(u, v) = row prefix of row u + D(u - 1, v)
        if (v < w) {
          const uint32_t m = col[c] + 0x80000000u;
          win[u * w + v] = (m & 0x80000000u) ? (m & 0x7FFFFFFFu) : ~m;
        }
      }
    }
  }
}

// Window k of a frame, one wave: lane l starts at window element l and steps
// 64 elements at a time, its (row, column) in the window advanced without a
// division.  Pixels outside the frame are not part of the window.  CHECK
// compares the frame with the payload instead of writing it.
template <bool CHECK>
__device__ __forceinline__ bool roi_window(const DecodePlan &dp, uint32_t k, uint32_t lane) {
  const uint32_t w = dp.w, ww = w * w;
  const uint16_t *pk = (const uint16_t *)(dp.in + dp.off_peaks);
  const uint32_t *pay =
      (dp.roi_coding ? dp.roi_payload : (const uint32_t *)(dp.in + dp.off_roi)) + (size_t)k * ww;
  const uint32_t pa = pk[3 * k];
  if (pa >= dp.P) return false;
  const int32_t h = (int32_t)(w / 2), H = (int32_t)dp.H, W = (int32_t)dp.W;
  const int32_t i0 = (int32_t)pk[3 * k + 1] - h, j0 = (int32_t)pk[3 * k + 2] - h;
  uint32_t *fr = (uint32_t *)dp.frame + (size_t)pa * dp.H * dp.W;
  const uint32_t du = 64 / w, dv = 64 % w;
  uint32_t u = lane / w, v = lane - u * w;
  bool bad = false;
  for (uint32_t e = lane; e < ww; e += 64) {
    const int32_t i = i0 + (int32_t)u, j = j0 + (int32_t)v;
    if (i >= 0 && i < H && j >= 0 && j < W) {
      uint32_t *px = fr + (size_t)i * dp.W + j;
      if (CHECK) bad |= *px != pay[e];
      else *px = pay[e];
    }
    u += du;
    v += dv;
    if (v >= w) {
      v -= w;
      ++u;
    }
  }
  return bad;
}

__global__ __launch_bounds__(256) void k_dec_roi(DecBatch db) {
  RSZ_DEC_FRAME(14);
  const uint32_t k = bid * 4 + (threadIdx.x >> 6);
  if (k >= dp.npeaks || !dec_ok(dp.status)) return;
  roi_window<false>(dp, k, threadIdx.x & 63);
}
__global__ __launch_bounds__(256) void k_dec_roi_check(DecBatch db) {
  RSZ_DEC_FRAME(15);
  const uint32_t k = bid * 4 + (threadIdx.x >> 6);
  if (k >= dp.npeaks || !dec_ok(dp.status)) return;
  if (roi_window<true>(dp, k, threadIdx.x & 63)) corrupt(dp.status);
}

void decode_blocks(const DecodePlan &dp, uint32_t *nb) {
  for (int k = 0; k < kDecKernels; ++k) nb[k] = 0;
  nb[0] = 1;   // k_dec_tables writes every frame's status
  if (dp.init_status != RSZ_OK) return;
  if (dp.run_coding) {
    nb[1] = (uint32_t)std::min<uint64_t>(((dp.T + 31) / 32 + 2 + 255) / 256, 1u << 16);
    nb[2] = (dp.nchunks + 255) / 256;
  }
  nb[3] = (dp.nchunks + 3) / 4;
  nb[4] = (dp.n_out + 255) / 256;
  // inverse Lorenzo: prefix sums along each axis the predictor spans
  if (panel_in_lds(dp)) {
    nb[16] = dp.P;   // k_dec_panel: rows, columns and pixels
  } else {
    nb[5] = (dp.P * dp.Hb + 4 * kDecRowsPerWave - 1) / (4 * kDecRowsPerWave);
    if (dp.dim == 1) {
      nb[6] = 1;
      nb[7] = std::min<uint32_t>((dp.nbins + 255) / 256, 1u << 16);
    } else {
      nb[8] = (dp.P * dp.Wb + 255) / 256;
      if (dp.dim == 3) nb[9] = (dp.Hb * dp.Wb + 255) / 256;
    }
  }
  if (dp.dim != 2) nb[10] = (dp.P * dp.Hb + 3) / 4;   // dimension 2: k_dec_cols
  if (dp.roi_coding) {
    nb[11] = 1;
    nb[12] = (dp.npeaks + 255) / 256;
    nb[13] = (dp.npeaks + 3) / 4;
  }
  nb[14] = nb[15] = (dp.npeaks + 3) / 4;   // a wave per window
}

#define RSZ_DLAUNCH(k, name, kern, block)                              \
  do {                                                                 \
    if (total[k]) {                                                    \
      prof_begin(name, s);                                             \
      hipLaunchKernelGGL(kern, dim3(total[k]), dim3(block), 0, s, db); \
      prof_end(s);                                                     \
      hipError_t e_ = hipGetLastError();                               \
      if (e_ != hipSuccess) return e_;                                 \
    }                                                                  \
  } while (0)

hipError_t launch_decompress(const DecBatch &db, const uint32_t *total, hipStream_t s) {
  RSZ_DLAUNCH(0, "k_dec_tables", k_dec_tables, 256);
  RSZ_DLAUNCH(1, "k_dec_run_zero", k_dec_run_zero, 256);
  RSZ_DLAUNCH(2, "k_dec_runs", k_dec_runs, 256);
  RSZ_DLAUNCH(3, "k_dec_chunks", k_dec_chunks, 256);
  RSZ_DLAUNCH(4, "k_dec_outliers", k_dec_outliers, 256);
  RSZ_DLAUNCH(5, "k_dec_rows", k_dec_rows, 256);
  RSZ_DLAUNCH(6, "k_dec_carry", k_dec_carry, 256);
  RSZ_DLAUNCH(7, "k_dec_rowadd", k_dec_rowadd, 256);
  RSZ_DLAUNCH(8, "k_dec_cols", k_dec_cols, 256);
  RSZ_DLAUNCH(9, "k_dec_panels", k_dec_panels, 256);
  RSZ_DLAUNCH(10, "k_dec_expand", k_dec_expand, 256);
  RSZ_DLAUNCH(16, "k_dec_panel", k_dec_panel, 1024);
  RSZ_DLAUNCH(11, "k_dec_roi_tables", k_dec_roi_tables, 64);
  RSZ_DLAUNCH(12, "k_dec_roi_decode", k_dec_roi_decode, 256);
  RSZ_DLAUNCH(13, "k_dec_roi_unpred", k_dec_roi_unpred, 256);
  RSZ_DLAUNCH(14, "k_dec_roi", k_dec_roi, 256);
  RSZ_DLAUNCH(15, "k_dec_roi_check", k_dec_roi_check, 256);
  return hipSuccess;
}

uint64_t decode_tables_bytes() { return 4ull * kTabWords; }
uint64_t decode_roi_tables_bytes() { return 4ull * kRoiTabWords; }

}  // namespace rsz
