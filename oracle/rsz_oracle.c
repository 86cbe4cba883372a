/*
 * rsz_oracle.c -- plain, slow, single-threaded CPU oracle for the ROIBIN-SZ
 * per-frame compression path (arXiv 2206.11297).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library) never calls it, links it or shares code, headers or tables with
 * it.
 *
 * What the paper fixes and what is a stated reading:
 *   - ROI windows around each Bragg peak are kept without error, with a
 *     constant fill outside the panel (Sec. IV, Sec. IV-A).
 *   - The background is binned as a b x b mean (Sec. VI) and compressed with an
 *     absolute error bound that holds on the *binned* values (Sec. V-C, "Our
 *     Approach", and the footnote of Sec. VI).
 *   - The SZ stage is a black box in the paper (Sec. V-C names Lorenzo +
 *     regression + linear quantization).  Here it is the dual-quantisation
 *     recipe: prequantise to integers at step 2*eb, Lorenzo on the integer
 *     field, outliers for residuals outside the radius, Huffman over 1024
 *     symbols.  The Lorenzo predictor works in the dimension of Sec. VI's
 *     grid search: 1 (the frame as one sequence of bins in raster order),
 *     2 (each panel as an image; the default) or 3 (the stack of panels as
 *     a volume).  Every constant the paper leaves open is a reading listed in the
 *     design notes (radius 512, chunk 4096, tie-breaks, container layout).
 *   - Compression ratio is relative to raw uint16 detector bytes (Sec. IV).
 *   - The peak list can also come from the peak finder at the end of this
 *     file (Sec. IV-B's peak_finder_v3 parameters), the step before the path.
 *
 * Arithmetic: fp64 sums in raster order, a correctly rounded divide and
 * rint() (round half to even).  Build with -ffp-contract=off and without
 * fast-math so that nothing is contracted or reordered.
 *
 * Parity pins (tests): brute-force masks, numpy sums, the closed-form
 * reconstruction, prefix-sum inverse of the Lorenzo step, an independent heap
 * Huffman cost, Kraft sums, brute-force optimality on tiny alphabets and
 * hand-derived stream fixtures.  The Huffman build's three stated rules
 * (equal counts taken in symbol order, a leaf winning a tie with an internal
 * node, floor-halving of the counts when a length exceeds 32) decide the code
 * lengths among several optimal ones; each has a hand-derived fixture that
 * fails when the rule is changed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RO_OK 0
#define RO_ERR_ARG (-1)
#define RO_ERR_PEAK (-2)
#define RO_ERR_RANGE (-3)
#define RO_ERR_CAPACITY (-4)
#define RO_ERR_CORRUPT (-5)

#define RO_RADIUS 512
#define RO_NSYM 1024
#define RO_MAXLEN 32
#define RO_CHUNK 4096
#define RO_QMAX 268435455.0 /* 2^28 - 1 */
#define RO_HEADER 80

typedef struct {
  uint32_t panels, height, width; /* frame is panels x height x width f32 */
  uint32_t window;                /* ROI window edge w                     */
  uint32_t bin;                   /* bin factor b                          */
  uint32_t bin_mode;              /* 0 = background pixels only, 1 = all   */
  double eb;                      /* absolute bound on binned values       */
  uint32_t dim;                   /* Lorenzo dimension 1, 2 or 3; 0 means 2 */
  uint32_t roi_coding;            /* 0: ROI payload verbatim, 1: coded    */
  uint32_t run_coding;            /* 0: Huffman bits as they are, 1: runs */
  uint32_t reserved;
} ro_params;

static uint32_t ro_dim(const ro_params *p) { return p->dim ? p->dim : 2u; }

/* ------------------------------------------------------------------ sizes */

static uint64_t ro_hb(const ro_params *p) { return (p->height + p->bin - 1) / p->bin; }
static uint64_t ro_wb(const ro_params *p) { return (p->width + p->bin - 1) / p->bin; }
static uint64_t ro_nbins(const ro_params *p) { return (uint64_t)p->panels * ro_hb(p) * ro_wb(p); }
static uint64_t ro_align4(uint64_t x) { return (x + 3u) & ~(uint64_t)3u; }

/* Argument validation.  Limits: each dimension 1..65535, window 1..1023,
 * bin 1..8, bin_mode 0/1, dim 0..3, roi_coding and run_coding 0/1, reserved 0,
 * eb finite and > 0, pixels < 2^31, bins < 2^27 (so T and Trun fit u32 offsets),
 * npeaks * w * w <= 2^28 payload words. */
int ro_check_params(const ro_params *p, uint32_t npeaks) {
  if (!p) return RO_ERR_ARG;
  if (p->panels < 1 || p->panels > 65535 || p->height < 1 || p->height > 65535 ||
      p->width < 1 || p->width > 65535)
    return RO_ERR_ARG;
  if (p->window < 1 || p->window > 1023) return RO_ERR_ARG;
  if (p->bin < 1 || p->bin > 8) return RO_ERR_ARG;
  if (p->bin_mode > 1 || p->dim > 3 || p->roi_coding > 1 || p->run_coding > 1 || p->reserved)
    return RO_ERR_ARG;
  if (!(p->eb > 0.0) || !isfinite(p->eb)) return RO_ERR_ARG;
  if ((uint64_t)p->panels * p->height * p->width >= (1ull << 31)) return RO_ERR_ARG;
  if (ro_nbins(p) >= (1ull << 27)) return RO_ERR_ARG;
  if ((uint64_t)npeaks * p->window * p->window > (1ull << 28)) return RO_ERR_ARG;
  /* coded ROI bits (at most 63 per value) must fit u32 offsets */
  if (p->roi_coding && (uint64_t)npeaks * p->window * p->window > (1ull << 26)) return RO_ERR_ARG;
  return RO_OK;
}

/* Every peak must name a pixel of the frame (panel, row, col). */
int ro_check_peaks(const ro_params *p, const int32_t *peaks, uint32_t npeaks) {
  for (uint32_t k = 0; k < npeaks; ++k) {
    int32_t pa = peaks[3 * k], r = peaks[3 * k + 1], c = peaks[3 * k + 2];
    if (pa < 0 || (uint32_t)pa >= p->panels || r < 0 || (uint32_t)r >= p->height || c < 0 ||
        (uint32_t)c >= p->width)
      return RO_ERR_PEAK;
  }
  return RO_OK;
}

/* ------------------------------------------------------- region of interest */

/* ROI mask (Sec. IV: the stream is split into the regions around each peak and
 * the background).  Window rows r-h .. r-h+w-1 and cols c-h .. c-h+w-1 with
 * h = floor(w/2), clipped to the panel; the mask is the union over peaks.
 * Bitmap: one u32 word per 32 columns of each (panel,row), LSB = lowest col. */
void ro_mask(const ro_params *p, const int32_t *peaks, uint32_t npeaks, uint32_t *bitmap) {
  const uint64_t wpr = (p->width + 31u) / 32u;
  memset(bitmap, 0, sizeof(uint32_t) * (size_t)(p->panels * (uint64_t)p->height * wpr));
  const int64_t h = p->window / 2;
  for (uint32_t k = 0; k < npeaks; ++k) {
    const int64_t pa = peaks[3 * k], r0 = peaks[3 * k + 1] - h, c0 = peaks[3 * k + 2] - h;
    for (int64_t i = r0; i < r0 + (int64_t)p->window; ++i) {
      if (i < 0 || i >= (int64_t)p->height) continue;
      for (int64_t j = c0; j < c0 + (int64_t)p->window; ++j) {
        if (j < 0 || j >= (int64_t)p->width) continue;
        bitmap[((uint64_t)pa * p->height + (uint64_t)i) * wpr + (uint64_t)j / 32u] |=
            1u << (j % 32);
      }
    }
  }
}

static int ro_mask_bit(const ro_params *p, const uint32_t *bitmap, uint64_t pa, uint64_t i,
                       uint64_t j) {
  const uint64_t wpr = (p->width + 31u) / 32u;
  return (bitmap[(pa * p->height + i) * wpr + j / 32u] >> (j % 32u)) & 1u;
}

/* ROI payload (Sec. IV-A: npeaks x window buffer, constant fill outside the
 * panel).  Entries are the raw 32-bit patterns of the frame, never touched as
 * floats, so the window round-trips bit-exactly; the fill is 0x00000000. */
void ro_roi(const ro_params *p, const float *frame, const int32_t *peaks, uint32_t npeaks,
            uint32_t *payload) {
  const int64_t h = p->window / 2, w = p->window;
  for (uint32_t k = 0; k < npeaks; ++k) {
    const int64_t pa = peaks[3 * k], r0 = peaks[3 * k + 1] - h, c0 = peaks[3 * k + 2] - h;
    for (int64_t u = 0; u < w; ++u)
      for (int64_t v = 0; v < w; ++v) {
        const int64_t i = r0 + u, j = c0 + v;
        uint32_t bits = 0u;
        if (i >= 0 && i < (int64_t)p->height && j >= 0 && j < (int64_t)p->width)
          memcpy(&bits, &frame[((uint64_t)pa * p->height + (uint64_t)i) * p->width + (uint64_t)j],
                 4);
        payload[((uint64_t)k * w + (uint64_t)u) * w + (uint64_t)v] = bits;
      }
  }
}

/* ---------------------------------------------------------------- binning */

/* b x b binning (Sec. VI: a bin combines b*b values into their mean).  Bin
 * (pa,I,J) covers rows [I*b, min(I*b+b,H)) and cols [J*b, min(J*b+b,W)).  The
 * included pixels are all of them (bin_mode 1) or those outside the ROI mask
 * (bin_mode 0).  S is the fp64 sum in raster order starting from +0.0, n the
 * number of included pixels; the mean is S/n. */
void ro_bin(const ro_params *p, const float *frame, const uint32_t *bitmap, double *S,
            uint32_t *n) {
  const uint64_t Hb = ro_hb(p), Wb = ro_wb(p), b = p->bin;
  for (uint64_t pa = 0; pa < p->panels; ++pa)
    for (uint64_t I = 0; I < Hb; ++I)
      for (uint64_t J = 0; J < Wb; ++J) {
        double s = 0.0;
        uint32_t cnt = 0;
        for (uint64_t i = I * b; i < I * b + b && i < p->height; ++i)
          for (uint64_t j = J * b; j < J * b + b && j < p->width; ++j) {
            if (p->bin_mode == 0 && ro_mask_bit(p, bitmap, pa, i, j)) continue;
            s = s + (double)frame[(pa * p->height + i) * p->width + j];
            cnt++;
          }
        const uint64_t g = (pa * Hb + I) * Wb + J;
        S[g] = s;
        n[g] = cnt;
      }
}

/* ------------------------------------------------------- error-bounded part */

/* Prequantisation at step 2*eb so that |q*2eb - S/n| <= eb (the absolute bound
 * on binned values, Sec. V-C "Our Approach").  q = rint(S / (n*2eb)), q = 0 for
 * an empty bin.  |q| must stay below 2^28 (this also rejects NaN/Inf). */
int ro_prequant(const ro_params *p, const double *S, const uint32_t *n, int32_t *q) {
  const uint64_t nb = ro_nbins(p);
  const double step = 2.0 * p->eb;
  int status = RO_OK;
  for (uint64_t g = 0; g < nb; ++g) {
    if (n[g] == 0) {
      q[g] = 0;
      continue;
    }
    const double den = (double)n[g] * step;
    const double t = rint(S[g] / den);
    if (!(fabs(t) <= RO_QMAX)) {
      status = RO_ERR_RANGE;
      q[g] = 0;
      continue;
    }
    q[g] = (int32_t)t;
  }
  return status;
}

/* Lorenzo predictor on the integer field (the SZ predictor of Sec. V-C, in
 * the dimension of Sec. VI).  The residual is q minus its prediction from the
 * neighbours that precede it along each axis the predictor spans, with zeros
 * outside the domain:
 *   dim 1: the frame is one sequence of bins in raster order (panel, row,
 *          column); r[g] = q[g] - q[g-1], and the first bin of a row follows
 *          the last bin of the row before it, across panels too;
 *   dim 2: each panel is an image; r = q - q_up - q_left + q_upleft;
 *   dim 3: the panels form a volume; r is the signed sum over the eight
 *          corners (p-a, I-c, J-e), a, c, e in {0,1}, of q with sign
 *          (-1)^(a+c+e). */
void ro_lorenzo(const ro_params *p, const int32_t *q, int32_t *r) {
  const uint64_t Hb = ro_hb(p), Wb = ro_wb(p), nb = ro_nbins(p);
  const uint32_t dim = ro_dim(p);
  if (dim == 1) {
    for (uint64_t g = 0; g < nb; ++g)
      r[g] = (int32_t)((int64_t)q[g] - (g > 0 ? (int64_t)q[g - 1] : 0));
    return;
  }
  for (uint64_t pa = 0; pa < p->panels; ++pa)
    for (uint64_t I = 0; I < Hb; ++I)
      for (uint64_t J = 0; J < Wb; ++J) {
        int64_t acc = 0;
        for (int a = 0; a <= (dim == 3 ? 1 : 0); ++a)
          for (int c = 0; c <= 1; ++c)
            for (int e = 0; e <= 1; ++e) {
              if ((uint64_t)a > pa || (uint64_t)c > I || (uint64_t)e > J) continue;
              const int64_t v = q[((pa - a) * Hb + (I - c)) * Wb + (J - e)];
              acc += ((a + c + e) & 1) ? -v : v;
            }
        r[(pa * Hb + I) * Wb + J] = (int32_t)acc;
      }
}

/* Quantisation codes: code = r + 512 when |r| < 512, else code 0 and the pair
 * (bin index, r) goes to the outlier list in ascending bin order. */
uint32_t ro_codes(uint64_t nbins, const int32_t *r, uint16_t *codes, uint32_t *out_idx,
                  int32_t *out_res) {
  uint32_t n_out = 0;
  for (uint64_t g = 0; g < nbins; ++g) {
    if (r[g] > -RO_RADIUS && r[g] < RO_RADIUS) {
      codes[g] = (uint16_t)(r[g] + RO_RADIUS);
    } else {
      codes[g] = 0;
      if (out_idx) out_idx[n_out] = (uint32_t)g;
      if (out_res) out_res[n_out] = r[g];
      n_out++;
    }
  }
  return n_out;
}

void ro_histogram(uint64_t nbins, const uint16_t *codes, uint32_t *hist) {
  memset(hist, 0, sizeof(uint32_t) * RO_NSYM);
  for (uint64_t g = 0; g < nbins; ++g) hist[codes[g]]++;
}

/* ------------------------------------------------------------------ Huffman */

typedef struct {
  uint64_t w;
  uint32_t sym;
} ro_leaf;

static int ro_leaf_cmp(const void *a, const void *b) {
  const ro_leaf *x = (const ro_leaf *)a, *y = (const ro_leaf *)b;
  if (x->w != y->w) return x->w < y->w ? -1 : 1;
  return x->sym < y->sym ? -1 : (x->sym > y->sym ? 1 : 0);
}

/* One Huffman build with the two-queue method: leaves sorted by (weight,
 * symbol); internal nodes in a FIFO; each pick takes the leaf when the leaf
 * weight is <= the front internal weight.  Returns the longest length. */
static int ro_huffman_once(const uint64_t *weight, uint8_t *len) {
  ro_leaf leaf[RO_NSYM];
  int nl = 0;
  memset(len, 0, RO_NSYM);
  for (int s = 0; s < RO_NSYM; ++s)
    if (weight[s] > 0) {
      leaf[nl].w = weight[s];
      leaf[nl].sym = (uint32_t)s;
      nl++;
    }
  if (nl == 0) return 0;
  if (nl == 1) {
    len[leaf[0].sym] = 1;
    return 1;
  }
  qsort(leaf, (size_t)nl, sizeof(ro_leaf), ro_leaf_cmp);
  /* node ids: 0..nl-1 leaves (sorted order), nl..2nl-2 internal in creation order */
  uint64_t nw[2 * RO_NSYM];
  int parent[2 * RO_NSYM];
  for (int i = 0; i < nl; ++i) nw[i] = leaf[i].w;
  int lf = 0, nf = nl, nend = nl; /* leaf front, internal front, next internal id */
  for (int m = 0; m < nl - 1; ++m) {
    int pick[2];
    for (int t = 0; t < 2; ++t) {
      if (nf == nend || (lf < nl && nw[lf] <= nw[nf]))
        pick[t] = lf++;
      else
        pick[t] = nf++;
    }
    nw[nend] = nw[pick[0]] + nw[pick[1]];
    parent[pick[0]] = nend;
    parent[pick[1]] = nend;
    nend++;
  }
  int depth[2 * RO_NSYM];
  const int root = nend - 1;
  depth[root] = 0;
  for (int v = root - 1; v >= 0; --v) depth[v] = depth[parent[v]] + 1;
  int maxlen = 0;
  for (int i = 0; i < nl; ++i) {
    len[leaf[i].sym] = (uint8_t)(depth[i] > 255 ? 255 : depth[i]);
    if (depth[i] > maxlen) maxlen = depth[i];
  }
  return maxlen;
}

/* Huffman code lengths for the 1024-symbol histogram.  A single used symbol
 * gets length 1.  If a length exceeds 32 the weights are halved (kept >= 1)
 * and the build repeats. */
void ro_huffman_lengths(const uint32_t *hist, uint8_t *len) {
  uint64_t w[RO_NSYM];
  for (int s = 0; s < RO_NSYM; ++s) w[s] = hist[s];
  for (;;) {
    if (ro_huffman_once(w, len) <= RO_MAXLEN) return;
    for (int s = 0; s < RO_NSYM; ++s)
      if (w[s] > 0) w[s] = (w[s] >> 1) > 0 ? (w[s] >> 1) : 1;
  }
}

/* Canonical codes: symbols ordered by (length, symbol); the first gets 0, each
 * next one (previous + 1) shifted left by the length increase (the canonical
 * assignment of RFC 1951 sec. 3.2.2). */
void ro_canonical(const uint8_t *len, uint32_t *code) {
  memset(code, 0, sizeof(uint32_t) * RO_NSYM);
  uint64_t c = 0;
  int prev = 0, first = 1;
  for (int L = 1; L <= RO_MAXLEN; ++L)
    for (int s = 0; s < RO_NSYM; ++s) {
      if (len[s] != L) continue;
      if (first) {
        c = 0;
        first = 0;
      } else {
        c = (c + 1) << (L - prev);
      }
      code[s] = (uint32_t)c;
      prev = L;
    }
}

/* Bitstream: codewords of code[0..nbins) concatenated MSB-first; stream bit k
 * is bit 31-(k%32) of word k/32; trailing bits of the last word are zero.
 * chunk_off[c] = bit offset of symbol c*4096.  Returns the total bit count T.
 * words may be NULL to only count. */
uint64_t ro_bitstream(uint64_t nbins, const uint16_t *codes, const uint8_t *len,
                      const uint32_t *cw, uint32_t *words, uint32_t *chunk_off) {
  uint64_t T = 0;
  for (uint64_t g = 0; g < nbins; ++g) {
    if (g % RO_CHUNK == 0 && chunk_off) chunk_off[g / RO_CHUNK] = (uint32_t)T;
    const unsigned L = len[codes[g]];
    const uint32_t c = cw[codes[g]];
    if (words)
      for (unsigned t = 0; t < L; ++t) {
        const uint64_t k = T + t;
        const uint32_t bit = (c >> (L - 1 - t)) & 1u;
        if (k % 32 == 0) words[k / 32] = 0;
        words[k / 32] |= bit << (31 - k % 32);
      }
    T += L;
  }
  return T;
}

/* ---------------------------------------------------------------- container */

/* Section order: header, peaks, ROI payload, code lengths, chunk offsets,
 * bitstream, outlier indices, outlier residuals.  With the ROI coded the
 * verbatim payload is absent and the coded ROI section follows the outliers:
 * 33 class code lengths (u8, padded to 36 bytes), one u32 bit offset per
 * window, then the ROI bitstream (Troi bits in u32 words).  With the runs
 * coded the bitstream is absent and the run section closes the stream: one
 * Rice parameter per chunk (u8, padded to 4 bytes), nchunks + 1 u32 bit
 * offsets (the last one the section's bits, Trun), then Trun bits. */
#define RO_ROI_CLASSES 33
#define RO_ROI_LENS 36
#define RO_RUN_KMAX 20
typedef struct {
  uint64_t peaks, roi, lens, chunks, bits, oidx, ores, rsec, roffs, rbits, run, runoffs, runbits,
      total;
} ro_layout;

static ro_layout ro_sections(const ro_params *p, uint32_t npeaks, uint64_t n_out,
                             uint64_t n_chunks, uint64_t T, uint64_t Troi, uint64_t Trun) {
  ro_layout L;
  L.peaks = RO_HEADER;
  L.roi = L.peaks + ro_align4(6ull * npeaks);
  L.lens = L.roi + (p->roi_coding ? 0 : 4ull * npeaks * p->window * p->window);
  L.chunks = L.lens + RO_NSYM;
  L.bits = L.chunks + 4ull * n_chunks;
  L.oidx = L.bits + (p->run_coding ? 0 : 4ull * ((T + 31) / 32));
  L.ores = L.oidx + 4ull * n_out;
  L.rsec = L.ores + 4ull * n_out;
  L.roffs = L.rsec + RO_ROI_LENS;
  L.rbits = L.roffs + 4ull * npeaks;
  L.run = p->roi_coding ? L.rbits + 4ull * ((Troi + 31) / 32) : L.rsec;
  L.runoffs = L.run + ro_align4(n_chunks);
  L.runbits = L.runoffs + 4ull * (n_chunks + 1);
  L.total = p->run_coding ? L.runbits + 4ull * ((Trun + 31) / 32) : L.run;
  return L;
}

/* ------------------------------------------------- lossless run stage */

/* A lossless stage after the Huffman coder (SZ follows its Huffman stage with
 * a lossless compressor; here one written for these bits).  The most common
 * code (residual 0) is the all-zero codeword, so the Huffman bits are mostly
 * zeros.  Per 4096-symbol chunk, the chunk's bits [off_c, off_c+1) are coded
 * as the lengths r of the zero runs before each 1 bit, Rice coded with the
 * chunk's parameter k: r >> k one bits, a zero bit, then the k low bits of r,
 * MSB-first.  Zeros after the chunk's last 1 are implied by its length.  k
 * (0..20) minimises the chunk's coded bits, the smallest k on ties. */
static uint32_t ro_getbit(const uint32_t *words, uint64_t k) {
  return (words[k / 32] >> (31 - k % 32)) & 1u;
}

/* Codes T Huffman bits in chunks starting at chunk_off[0..nc); writes the
 * parameters kpar[nc], offsets runoffs[nc + 1] and, if out is not NULL
 * (zeroed), the run bits; returns Trun. */
uint64_t ro_run_code(const uint32_t *words, uint64_t T, const uint32_t *chunk_off, uint64_t nc,
                     uint8_t *kpar, uint32_t *runoffs, uint32_t *out) {
  uint64_t pos = 0;
  for (uint64_t c = 0; c < nc; ++c) {
    const uint64_t start = chunk_off[c], end = c + 1 < nc ? chunk_off[c + 1] : T;
    uint64_t cost[RO_RUN_KMAX + 1];
    memset(cost, 0, sizeof cost);
    uint64_t prev = start;   /* first position after the previous 1 */
    for (uint64_t b = start; b < end; ++b)
      if (ro_getbit(words, b)) {
        for (uint32_t k = 0; k <= RO_RUN_KMAX; ++k) cost[k] += ((b - prev) >> k) + 1 + k;
        prev = b + 1;
      }
    uint32_t best = 0;
    for (uint32_t k = 1; k <= RO_RUN_KMAX; ++k)
      if (cost[k] < cost[best]) best = k;
    kpar[c] = (uint8_t)best;
    runoffs[c] = (uint32_t)pos;
    if (out) {
      prev = start;
      for (uint64_t b = start; b < end; ++b)
        if (ro_getbit(words, b)) {
          const uint64_t r = b - prev;
          for (uint64_t q = 0; q < (r >> best); ++q) {
            out[pos / 32] |= 1u << (31 - pos % 32);
            pos++;
          }
          pos++;   /* the zero that ends the unary part */
          for (uint32_t t = 0; t < best; ++t) {
            if ((r >> (best - 1 - t)) & 1u) out[pos / 32] |= 1u << (31 - pos % 32);
            pos++;
          }
          prev = b + 1;
        }
    } else {
      pos += cost[best];
    }
  }
  runoffs[nc] = (uint32_t)pos;
  return pos;
}

/* ---------------------------------------------------- lossless ROI coding */

/* Predictive lossless coding of the ROI windows (the paper codes them with
 * fpzip, Sec. IV; this is a coder of the same class written here).  Each
 * window's w*w payload words b (fill 0 outside the panel) are mapped to
 * order-preserving integers M (positive floats: b | 2^31, negative: ~b), so
 * that near values are near integers.  M is predicted in raster order by the
 * 2D Lorenzo predictor over the window, M[u-1][v] + M[u][v-1] - M[u-1][v-1]
 * with M = 2^31 (mapped +0.0) outside it, all mod 2^32.  The residual r is
 * zigzag-mapped to z = (r << 1) ^ (r >> 31); its class c = bit length of z
 * (0..32) is Huffman coded (per frame, the two-queue rule and canonical
 * codes of the main code) and followed by the low c - 1 bits of z (c >= 2;
 * the leading 1 is implied), MSB-first. */
static uint32_t ro_fmap(uint32_t b) { return (b & 0x80000000u) ? ~b : (b | 0x80000000u); }
static uint32_t ro_funmap(uint32_t m) { return (m & 0x80000000u) ? (m & 0x7FFFFFFFu) : ~m; }
static uint32_t ro_zclass(uint32_t z) {
  uint32_t c = 0;
  while (z) {
    c++;
    z >>= 1;
  }
  return c;
}

/* Zigzag residual of value (u, v) of a w x w window of mapped words M. */
static uint32_t ro_roi_z(const uint32_t *M, int64_t w, int64_t u, int64_t v) {
  const uint32_t zero = 0x80000000u;
  const uint32_t up = u > 0 ? M[(u - 1) * w + v] : zero;
  const uint32_t left = v > 0 ? M[u * w + v - 1] : zero;
  const uint32_t ul = (u > 0 && v > 0) ? M[(u - 1) * w + v - 1] : zero;
  const uint32_t pred = up + left - ul;
  const int32_t r = (int32_t)(M[u * w + v] - pred);
  return ((uint32_t)r << 1) ^ (uint32_t)(r >> 31);
}

static void ro_putbits(uint32_t *words, uint64_t *pos, uint32_t value, uint32_t nbits) {
  for (uint32_t i = 0; i < nbits; ++i) {
    const uint32_t bit = (value >> (nbits - 1 - i)) & 1u;
    if (bit) words[*pos / 32] |= 1u << (31 - *pos % 32);
    (*pos)++;
  }
}

/* Codes the payload of npeaks windows: class lengths (33), window bit offsets
 * and, if words is not NULL, the bitstream (words must be zeroed).  Returns
 * the number of bits. */
uint64_t ro_roi_code(const ro_params *p, const uint32_t *payload, uint32_t npeaks, uint8_t *lens33,
                     uint32_t *offsets, uint32_t *words) {
  const int64_t w = p->window, ww = w * w;
  uint32_t *M = (uint32_t *)malloc(4 * (size_t)ww);
  uint32_t hist[RO_NSYM];
  memset(hist, 0, sizeof hist);
  for (uint32_t k = 0; k < npeaks; ++k) {
    for (int64_t t = 0; t < ww; ++t) M[t] = ro_fmap(payload[(uint64_t)k * ww + t]);
    for (int64_t u = 0; u < w; ++u)
      for (int64_t v = 0; v < w; ++v) hist[ro_zclass(ro_roi_z(M, w, u, v))]++;
  }
  uint8_t len[RO_NSYM];
  uint32_t cw[RO_NSYM];
  memset(len, 0, sizeof len);
  if (npeaks) ro_huffman_lengths(hist, len);
  ro_canonical(len, cw);
  memcpy(lens33, len, RO_ROI_CLASSES);
  uint64_t pos = 0;
  for (uint32_t k = 0; k < npeaks; ++k) {
    offsets[k] = (uint32_t)pos;
    for (int64_t t = 0; t < ww; ++t) M[t] = ro_fmap(payload[(uint64_t)k * ww + t]);
    for (int64_t u = 0; u < w; ++u)
      for (int64_t v = 0; v < w; ++v) {
        const uint32_t z = ro_roi_z(M, w, u, v), c = ro_zclass(z);
        if (words) {
          ro_putbits(words, &pos, cw[c], len[c]);
          if (c >= 2) ro_putbits(words, &pos, z, c - 1);
        } else {
          pos += len[c] + (c >= 2 ? c - 1 : 0);
        }
      }
  }
  free(M);
  return pos;
}

static void put16(uint8_t *b, uint64_t o, uint16_t v) { memcpy(b + o, &v, 2); }
static void put32(uint8_t *b, uint64_t o, uint32_t v) { memcpy(b + o, &v, 4); }
static void put64(uint8_t *b, uint64_t o, uint64_t v) { memcpy(b + o, &v, 8); }
static uint16_t get16(const uint8_t *b, uint64_t o) { uint16_t v; memcpy(&v, b + o, 2); return v; }
static uint32_t get32(const uint8_t *b, uint64_t o) { uint32_t v; memcpy(&v, b + o, 4); return v; }
static uint64_t get64(const uint8_t *b, uint64_t o) { uint64_t v; memcpy(&v, b + o, 8); return v; }

/* Worst-case stream size: every bin an outlier and every codeword 32 bits. */
int ro_max_bytes(const ro_params *p, uint32_t npeaks, uint64_t *bytes) {
  int st = ro_check_params(p, npeaks);
  if (st) return st;
  const uint64_t nb = ro_nbins(p), nc = (nb + RO_CHUNK - 1) / RO_CHUNK;
  /* worst case: every code 32 bits, every bin an outlier, every ROI value 63
   * bits; the run section never exceeds the bits it codes */
  *bytes = ro_sections(p, npeaks, nb, nc, 32ull * nb, 63ull * npeaks * p->window * p->window,
                       32ull * nb).total;
  return RO_OK;
}

/* Everything the compressor computes, for parity tests.  Any pointer may be
 * NULL.  Returns the status of compression (OK / ARG / PEAK / RANGE). */
int ro_intermediates(const ro_params *p, const float *frame, const int32_t *peaks,
                     uint32_t npeaks, uint32_t *mask, uint32_t *payload, double *S, uint32_t *n,
                     int32_t *q, int32_t *r, uint16_t *codes, uint32_t *out_idx, int32_t *out_res,
                     uint32_t *n_out_p, uint32_t *hist, uint8_t *lens, uint32_t *cw,
                     uint32_t *chunk_off, uint64_t *T_p) {
  int st = ro_check_params(p, npeaks);
  if (st) return st;
  st = ro_check_peaks(p, peaks, npeaks);
  if (st) return st;
  const uint64_t nb = ro_nbins(p), nc = (nb + RO_CHUNK - 1) / RO_CHUNK;
  const uint64_t wpr = (p->width + 31u) / 32u;
  uint32_t *m = (uint32_t *)malloc(4 * (size_t)(p->panels * (uint64_t)p->height * wpr));
  double *s = (double *)malloc(8 * (size_t)nb);
  uint32_t *cnt = (uint32_t *)malloc(4 * (size_t)nb);
  int32_t *qq = (int32_t *)malloc(4 * (size_t)nb);
  int32_t *rr = (int32_t *)malloc(4 * (size_t)nb);
  uint16_t *cd = (uint16_t *)malloc(2 * (size_t)nb);
  ro_mask(p, peaks, npeaks, m);
  if (payload) ro_roi(p, frame, peaks, npeaks, payload);
  ro_bin(p, frame, m, s, cnt);
  st = ro_prequant(p, s, cnt, qq);
  ro_lorenzo(p, qq, rr);
  const uint32_t n_out = ro_codes(nb, rr, cd, out_idx, out_res);
  uint32_t h[RO_NSYM];
  uint8_t l[RO_NSYM];
  uint32_t c[RO_NSYM];
  ro_histogram(nb, cd, h);
  ro_huffman_lengths(h, l);
  ro_canonical(l, c);
  uint32_t *co = (uint32_t *)malloc(4 * (size_t)nc);
  const uint64_t T = ro_bitstream(nb, cd, l, c, NULL, co);
  if (mask) memcpy(mask, m, 4 * (size_t)(p->panels * (uint64_t)p->height * wpr));
  if (S) memcpy(S, s, 8 * (size_t)nb);
  if (n) memcpy(n, cnt, 4 * (size_t)nb);
  if (q) memcpy(q, qq, 4 * (size_t)nb);
  if (r) memcpy(r, rr, 4 * (size_t)nb);
  if (codes) memcpy(codes, cd, 2 * (size_t)nb);
  if (n_out_p) *n_out_p = n_out;
  if (hist) memcpy(hist, h, sizeof h);
  if (lens) memcpy(lens, l, sizeof l);
  if (cw) memcpy(cw, c, sizeof c);
  if (chunk_off) memcpy(chunk_off, co, 4 * (size_t)nc);
  if (T_p) *T_p = T;
  free(m); free(s); free(cnt); free(qq); free(rr); free(cd); free(co);
  return st;
}

/* Compress one frame into the self-contained stream (header, peaks, ROI
 * payload, code lengths, chunk offsets, bitstream, outliers).  On
 * RO_ERR_CAPACITY *out_bytes holds the required size. */
int ro_compress(const ro_params *p, const float *frame, const int32_t *peaks, uint32_t npeaks,
                uint8_t *out, uint64_t out_cap, uint64_t *out_bytes) {
  int st = ro_check_params(p, npeaks);
  if (st) return st;
  st = ro_check_peaks(p, peaks, npeaks);
  if (st) return st;
  const uint64_t nb = ro_nbins(p), nc = (nb + RO_CHUNK - 1) / RO_CHUNK;
  const uint64_t wpr = (p->width + 31u) / 32u;
  uint32_t *m = (uint32_t *)malloc(4 * (size_t)(p->panels * (uint64_t)p->height * wpr));
  double *s = (double *)malloc(8 * (size_t)nb);
  uint32_t *cnt = (uint32_t *)malloc(4 * (size_t)nb);
  int32_t *qq = (int32_t *)malloc(4 * (size_t)nb);
  int32_t *rr = (int32_t *)malloc(4 * (size_t)nb);
  uint16_t *cd = (uint16_t *)malloc(2 * (size_t)nb);
  uint32_t *oi = (uint32_t *)malloc(4 * (size_t)nb);
  int32_t *orr = (int32_t *)malloc(4 * (size_t)nb);
  uint32_t *co = (uint32_t *)malloc(4 * (size_t)nc);
  ro_mask(p, peaks, npeaks, m);
  ro_bin(p, frame, m, s, cnt);
  st = ro_prequant(p, s, cnt, qq);
  if (st == RO_OK) {
    ro_lorenzo(p, qq, rr);
    const uint32_t n_out = ro_codes(nb, rr, cd, oi, orr);
    uint32_t h[RO_NSYM];
    uint8_t l[RO_NSYM];
    uint32_t c[RO_NSYM];
    ro_histogram(nb, cd, h);
    ro_huffman_lengths(h, l);
    ro_canonical(l, c);
    const uint64_t T = ro_bitstream(nb, cd, l, c, NULL, co);
    /* the ROI payload, and its coded form when asked for */
    const uint64_t nroi = (uint64_t)npeaks * p->window * p->window;
    uint32_t *pay = (uint32_t *)malloc(4 * (size_t)(nroi ? nroi : 1));
    uint32_t *roffs = (uint32_t *)malloc(4 * (size_t)(npeaks ? npeaks : 1));
    uint8_t rl[RO_ROI_CLASSES];
    ro_roi(p, frame, peaks, npeaks, pay);
    const uint64_t Troi = p->roi_coding ? ro_roi_code(p, pay, npeaks, rl, roffs, NULL) : 0;
    /* the Huffman bits, and their run coding when asked for */
    uint32_t *hw = (uint32_t *)calloc((size_t)((T + 31) / 32 + 1), 4);
    uint8_t *kpar = (uint8_t *)malloc((size_t)nc + 1);
    uint32_t *runoffs = (uint32_t *)malloc(4 * (size_t)(nc + 1));
    ro_bitstream(nb, cd, l, c, hw, NULL);
    const uint64_t Trun = p->run_coding ? ro_run_code(hw, T, co, nc, kpar, runoffs, NULL) : 0;
    const ro_layout L = ro_sections(p, npeaks, n_out, nc, T, Troi, Trun);
    *out_bytes = L.total;
    if (L.total > out_cap) {
      st = RO_ERR_CAPACITY;
    } else {
      memset(out, 0, (size_t)L.total);
      memcpy(out, "RSZ1", 4);
      put16(out, 4, 1);
      /* flags: bit 0 bin_mode, bits 1-2 the Lorenzo dimension (0 for the
       * default 2, else 1 or 3), bit 3 the ROI coded, bit 4 the runs coded */
      put16(out, 6, (uint16_t)((p->bin_mode & 1u) | ((ro_dim(p) == 2 ? 0u : ro_dim(p)) << 1) |
                               ((p->roi_coding & 1u) << 3) | ((p->run_coding & 1u) << 4)));
      put32(out, 8, p->panels);
      put32(out, 12, p->height);
      put32(out, 16, p->width);
      put32(out, 20, p->window);
      put32(out, 24, p->bin);
      put32(out, 28, RO_RADIUS);
      memcpy(out + 32, &p->eb, 8);
      put32(out, 40, npeaks);
      put32(out, 44, n_out);
      put32(out, 48, RO_CHUNK);
      put32(out, 52, (uint32_t)nc);
      put64(out, 56, T);
      put64(out, 64, L.total);
      put64(out, 72, Troi);   /* ROI bits (0 with the payload verbatim) */
      for (uint32_t k = 0; k < npeaks; ++k)
        for (int t = 0; t < 3; ++t) put16(out, L.peaks + 6ull * k + 2 * t, (uint16_t)peaks[3 * k + t]);
      if (p->roi_coding) {
        ro_roi_code(p, pay, npeaks, out + L.rsec, roffs, (uint32_t *)(out + L.rbits));
        for (uint32_t k = 0; k < npeaks; ++k) put32(out, L.roffs + 4ull * k, roffs[k]);
      } else {
        memcpy(out + L.roi, pay, 4 * (size_t)nroi);
      }
      memcpy(out + L.lens, l, RO_NSYM);
      for (uint32_t k = 0; k < n_out; ++k) {
        put32(out, L.oidx + 4ull * k, oi[k]);
        put32(out, L.ores + 4ull * k, (uint32_t)orr[k]);
      }
      for (uint64_t k = 0; k < nc; ++k) put32(out, L.chunks + 4 * k, co[k]);
      if (p->run_coding) {
        ro_run_code(hw, T, co, nc, out + L.run, runoffs, (uint32_t *)(out + L.runbits));
        for (uint64_t k = 0; k <= nc; ++k) put32(out, L.runoffs + 4 * k, runoffs[k]);
      } else {
        ro_bitstream(nb, cd, l, c, (uint32_t *)(out + L.bits), NULL);
      }
    }
    free(pay); free(roffs); free(hw); free(kpar); free(runoffs);
  }
  free(m); free(s); free(cnt); free(qq); free(rr); free(cd); free(oi); free(orr); free(co);
  return st;
}

/* ---------------------------------------------------------------- decoding */

/* Parse the header of a stream and check it against the buffer size. */
int ro_stream_info(const uint8_t *in, uint64_t in_bytes, ro_params *p, uint32_t *npeaks,
                   uint64_t *stream_bytes) {
  if (in_bytes < RO_HEADER || memcmp(in, "RSZ1", 4) != 0 || get16(in, 4) != 1)
    return RO_ERR_CORRUPT;
  ro_params q;
  const uint32_t flags = get16(in, 6), dcode = (flags >> 1) & 3u;
  if ((flags >> 5) != 0 || dcode == 2) return RO_ERR_CORRUPT;
  memset(&q, 0, sizeof q);
  q.bin_mode = flags & 1u;
  q.dim = dcode == 0 ? 2u : dcode;
  q.roi_coding = (flags >> 3) & 1u;
  q.run_coding = (flags >> 4) & 1u;
  q.panels = get32(in, 8);
  q.height = get32(in, 12);
  q.width = get32(in, 16);
  q.window = get32(in, 20);
  q.bin = get32(in, 24);
  memcpy(&q.eb, in + 32, 8);
  const uint32_t np = get32(in, 40);
  if (ro_check_params(&q, np) != RO_OK) return RO_ERR_CORRUPT;
  /* offset 72: the coded ROI bits, 0 when the payload is verbatim */
  const uint64_t Troi = get64(in, 72);
  if (get32(in, 28) != RO_RADIUS || get32(in, 48) != RO_CHUNK || (!q.roi_coding && Troi != 0) ||
      Troi > 63ull * np * q.window * q.window)
    return RO_ERR_CORRUPT;
  const uint64_t nb = ro_nbins(&q), nc = (nb + RO_CHUNK - 1) / RO_CHUNK;
  const uint64_t n_out = get32(in, 44), T = get64(in, 56), total = get64(in, 64);
  if (get32(in, 52) != nc || n_out > nb || T > 32ull * nb) return RO_ERR_CORRUPT;
  /* the run section's size comes from its last offset: the header fixes its
   * start, and the total must leave room for the offsets */
  const ro_layout L0 = ro_sections(&q, np, n_out, nc, T, Troi, 0);
  if (q.run_coding ? (total < L0.total || (total - L0.total) % 4 != 0) : L0.total != total)
    return RO_ERR_CORRUPT;
  if (total > in_bytes) return RO_ERR_CORRUPT;
  if (p) *p = q;
  if (npeaks) *npeaks = np;
  if (stream_bytes) *stream_bytes = total;
  return RO_OK;
}

/* Decodes the coded ROI section (see ro_roi_code) into payload (npeaks * w
 * * w words).  The class lengths must form a complete prefix code (or one
 * class of length 1; none when there is no window), padding bytes zero;
 * window k starts at its offset (the first at 0, offsets non-decreasing) and
 * ends exactly where window k + 1 starts, the last at Troi.  Anything else is
 * RO_ERR_CORRUPT. */
static int ro_roi_decode(const ro_params *p, const uint8_t *in, const ro_layout *L, uint32_t np,
                         uint64_t Troi, uint32_t *payload) {
  const uint8_t *lens = in + L->rsec;
  uint64_t kraft = 0;
  int used = 0;
  for (int c = 0; c < RO_ROI_LENS; ++c) {
    if (c >= RO_ROI_CLASSES ? lens[c] != 0 : lens[c] > RO_MAXLEN) return RO_ERR_CORRUPT;
    if (c < RO_ROI_CLASSES && lens[c]) {
      kraft += 1ull << (RO_MAXLEN - lens[c]);
      used++;
    }
  }
  if (np == 0) return (used == 0 && Troi == 0) ? RO_OK : RO_ERR_CORRUPT;
  if (!(kraft == (1ull << RO_MAXLEN) || (used == 1 && kraft == (1ull << (RO_MAXLEN - 1)))))
    return RO_ERR_CORRUPT;
  uint8_t len[RO_NSYM];
  uint32_t cw[RO_NSYM];
  memset(len, 0, sizeof len);
  memcpy(len, lens, RO_ROI_CLASSES);
  ro_canonical(len, cw);
  const uint32_t *words = (const uint32_t *)(in + L->rbits);
  const int64_t w = p->window, ww = w * w;
  uint32_t *M = (uint32_t *)malloc(4 * (size_t)ww);
  int bad = 0;
  uint64_t pos = 0;
  for (uint32_t k = 0; k < np && !bad; ++k) {
    const uint64_t start = get32(in, L->roffs + 4ull * k);
    const uint64_t end = k + 1 < np ? get32(in, L->roffs + 4ull * (k + 1)) : Troi;
    if (start != pos || end < start || end > Troi) {
      bad = 1;
      break;
    }
    for (int64_t u = 0; u < w && !bad; ++u)
      for (int64_t v = 0; v < w && !bad; ++v) {
        /* class: the codeword whose length and value match, read bit by bit */
        uint64_t code = 0;
        int cls = -1;
        for (int n = 1; n <= RO_MAXLEN && cls < 0; ++n) {
          if (pos >= end) { bad = 1; break; }
          code = (code << 1) | ((words[pos / 32] >> (31 - pos % 32)) & 1u);
          pos++;
          for (int c = 0; c < RO_ROI_CLASSES; ++c)
            if (len[c] == n && cw[c] == code) { cls = c; break; }
        }
        if (bad || cls < 0) { bad = 1; break; }
        uint32_t z = cls == 0 ? 0u : 1u;
        for (int b = 0; b + 1 < cls; ++b) {
          if (pos >= end) { bad = 1; break; }
          z = (z << 1) | ((words[pos / 32] >> (31 - pos % 32)) & 1u);
          pos++;
        }
        if (bad) break;
        const uint32_t r = (z >> 1) ^ (0u - (z & 1u));
        const uint32_t zero = 0x80000000u;
        const uint32_t up = u > 0 ? M[(u - 1) * w + v] : zero;
        const uint32_t left = v > 0 ? M[u * w + v - 1] : zero;
        const uint32_t ul = (u > 0 && v > 0) ? M[(u - 1) * w + v - 1] : zero;
        M[u * w + v] = up + left - ul + r;
        payload[(uint64_t)k * ww + u * w + v] = ro_funmap(M[u * w + v]);
      }
    if (!bad && pos != end) bad = 1;
  }
  free(M);
  return bad ? RO_ERR_CORRUPT : RO_OK;
}

/* Expands the run section back into the T Huffman bits (words, zeroed,
 * (T + 31) / 32 of them).  Offsets start at 0 and never decrease, the last
 * one is the section's bits (which fill its words exactly); parameters are
 * <= 20 and the padding is zero; each chunk's codes end exactly at the next
 * chunk's offset and place their 1 bits inside the chunk.  Anything else is
 * RO_ERR_CORRUPT. */
static int ro_run_decode(const uint8_t *in, uint64_t total, const ro_layout *L, uint64_t nc,
                         uint64_t T, const uint32_t *chunk_off, uint32_t *words) {
  const uint8_t *kpar = in + L->run;
  for (uint64_t c = 0; c < ro_align4(nc); ++c)
    if (c < nc ? kpar[c] > RO_RUN_KMAX : kpar[c] != 0) return RO_ERR_CORRUPT;
  const uint64_t Trun = get32(in, L->runoffs + 4 * nc);
  if (L->runbits + 4 * ((Trun + 31) / 32) != total || get32(in, L->runoffs) != 0)
    return RO_ERR_CORRUPT;
  const uint32_t *rw = (const uint32_t *)(in + L->runbits);
  for (uint64_t c = 0; c < nc; ++c) {
    uint64_t pos = get32(in, L->runoffs + 4 * c);
    const uint64_t rend = get32(in, L->runoffs + 4 * (c + 1));
    const uint64_t start = chunk_off[c], end = c + 1 < nc ? chunk_off[c + 1] : T;
    if (rend < pos || rend > Trun) return RO_ERR_CORRUPT;
    const uint32_t k = kpar[c];
    uint64_t b = start;   /* next Huffman bit position */
    while (pos < rend) {
      uint64_t q = 0;
      while (pos < rend && ro_getbit(rw, pos)) {
        q++;
        pos++;
      }
      if (pos >= rend) return RO_ERR_CORRUPT;   /* no zero closing the unary part */
      pos++;
      if (pos + k > rend) return RO_ERR_CORRUPT;
      uint64_t low = 0;
      for (uint32_t t = 0; t < k; ++t) low = (low << 1) | ro_getbit(rw, pos++);
      b += (q << k) | low;   /* the run of zeros */
      if (b >= end) return RO_ERR_CORRUPT;
      words[b / 32] |= 1u << (31 - b % 32);
      b++;
    }
  }
  return RO_OK;
}

/* Decompress a stream into a panels x height x width float frame.
 * Structural validation first (any failure -> RO_ERR_CORRUPT); then
 * codes -> residuals -> q by prefix sums -> bin value q*2eb replicated over
 * the bin -> ROI windows restored bit-exactly from the payload.  Overlapping
 * windows must carry identical bits for their shared pixels. */
int ro_decompress(const uint8_t *in, uint64_t in_bytes, float *frame, uint64_t frame_elems) {
  ro_params p;
  uint32_t np;
  uint64_t total;
  int st = ro_stream_info(in, in_bytes, &p, &np, &total);
  if (st) return st;
  const uint64_t pix = (uint64_t)p.panels * p.height * p.width;
  if (frame_elems < pix) return RO_ERR_ARG;
  const uint64_t nb = ro_nbins(&p), nc = (nb + RO_CHUNK - 1) / RO_CHUNK;
  const uint64_t n_out = get32(in, 44), T = get64(in, 56), Troi = get64(in, 72);
  const ro_layout L0 = ro_sections(&p, np, n_out, nc, T, Troi, 0);
  const uint64_t Trun = p.run_coding ? get32(in, L0.runoffs + 4 * nc) : 0;
  const ro_layout L = ro_sections(&p, np, n_out, nc, T, Troi, Trun);
  /* the Huffman bits: in the stream, or expanded from the run section */
  uint32_t *hw = NULL;
  const uint8_t *bits = in + L.bits;
  if (p.run_coding) {
    uint32_t *co = (uint32_t *)malloc(4 * (size_t)(nc + 1));
    for (uint64_t c = 0; c < nc; ++c) co[c] = get32(in, L.chunks + 4 * c);
    hw = (uint32_t *)calloc((size_t)((T + 31) / 32 + 1), 4);
    int okc = 1;
    for (uint64_t c = 0; c < nc && okc; ++c)
      okc = co[c] <= T && (c == 0 || co[c] >= co[c - 1]);
    const int rs = okc ? ro_run_decode(in, total, &L, nc, T, co, hw) : RO_ERR_CORRUPT;
    free(co);
    if (rs != RO_OK) {
      free(hw);
      return RO_ERR_CORRUPT;
    }
    bits = (const uint8_t *)hw;
  }
  /* peaks */
  int32_t *pk = (int32_t *)malloc(12 * (size_t)(np ? np : 1));
  for (uint32_t k = 0; k < np; ++k)
    for (int t = 0; t < 3; ++t) pk[3 * k + t] = get16(in, L.peaks + 6ull * k + 2 * t);
  if (ro_check_peaks(&p, pk, np) != RO_OK) {
    free(pk); free(hw);
    return RO_ERR_CORRUPT;
  }
  /* code lengths: each <= 32 and a complete prefix code (Kraft sum 1), or one
   * symbol of length 1 */
  uint8_t len[RO_NSYM];
  memcpy(len, in + L.lens, RO_NSYM);
  uint64_t kraft = 0;
  int used = 0;
  for (int s = 0; s < RO_NSYM; ++s) {
    if (len[s] > RO_MAXLEN) { free(pk); free(hw); return RO_ERR_CORRUPT; }
    if (len[s]) { kraft += 1ull << (RO_MAXLEN - len[s]); used++; }
  }
  if (!(kraft == (1ull << RO_MAXLEN) || (used == 1 && kraft == (1ull << (RO_MAXLEN - 1))))) {
    free(pk); free(hw);
    return RO_ERR_CORRUPT;
  }
  /* canonical decoding tables: per length, first code, count and offset into
   * the (length, symbol)-ordered symbol list */
  uint32_t cw[RO_NSYM];
  ro_canonical(len, cw);
  uint64_t first[RO_MAXLEN + 2];
  uint32_t count[RO_MAXLEN + 2], offs[RO_MAXLEN + 2], sorted[RO_NSYM];
  uint32_t ns = 0;
  for (int Lx = 1; Lx <= RO_MAXLEN; ++Lx) {
    count[Lx] = 0;
    offs[Lx] = ns;
    first[Lx] = 0;
    for (int s = 0; s < RO_NSYM; ++s)
      if (len[s] == Lx) {
        if (count[Lx] == 0) first[Lx] = cw[s];
        sorted[ns++] = (uint32_t)s;
        count[Lx]++;
      }
  }
  /* decode every symbol sequentially, checking the chunk offsets */
  int32_t *res = (int32_t *)malloc(4 * (size_t)nb);
  uint16_t *cd = (uint16_t *)malloc(2 * (size_t)nb);
  uint64_t pos = 0, prev_off = 0;
  int bad = 0;
  for (uint64_t g = 0; g < nb && !bad; ++g) {
    if (g % RO_CHUNK == 0) {
      const uint64_t off = get32(in, L.chunks + 4 * (g / RO_CHUNK));
      if (off != pos || off < prev_off || off > T) { bad = 1; break; }
      prev_off = off;
    }
    uint64_t c = 0;
    int Lx = 0, found = -1;
    while (Lx < RO_MAXLEN) {
      if (pos >= T) { bad = 1; break; }
      const uint32_t word = get32(bits, 4 * (pos / 32));
      c = (c << 1) | ((word >> (31 - pos % 32)) & 1u);
      pos++;
      Lx++;
      if (count[Lx] && c >= first[Lx] && c - first[Lx] < count[Lx]) {
        found = (int)sorted[offs[Lx] + (uint32_t)(c - first[Lx])];
        break;
      }
    }
    if (found < 0) { bad = 1; break; }
    cd[g] = (uint16_t)found;
  }
  if (!bad && pos != T) bad = 1;
  /* outliers: strictly increasing indices at the code-0 positions, |r| >= 512 */
  const int64_t rlim = (int64_t)1 << (28 + ro_dim(&p));
  if (!bad) {
    uint64_t k = 0;
    for (uint64_t g = 0; g < nb && !bad; ++g) {
      if (cd[g] != 0) {
        res[g] = (int32_t)cd[g] - RO_RADIUS;
        continue;
      }
      if (k >= n_out) { bad = 1; break; }
      const uint32_t idx = get32(in, L.oidx + 4 * k);
      const int32_t rv = (int32_t)get32(in, L.ores + 4 * k);
      /* |q| < 2^28 bounds a residual of dimension d below 2^(28+d) */
      if (idx != g || (rv > -RO_RADIUS && rv < RO_RADIUS) || (int64_t)rv <= -rlim ||
          (int64_t)rv >= rlim) {
        bad = 1;
        break;
      }
      res[g] = rv;
      k++;
    }
    if (k != n_out) bad = 1;
  }
  if (bad) {
    free(pk); free(hw); free(res); free(cd);
    return RO_ERR_CORRUPT;
  }
  /* inverse Lorenzo: q is the inclusive prefix sum of r along each axis the
   * predictor spans -- the whole raster sequence (dim 1), the rows and
   * columns of each panel (dim 2), and in addition the panel axis (dim 3) --
   * with two's-complement wrap-around, as int32 */
  const uint64_t Hb = ro_hb(&p), Wb = ro_wb(&p), b = p.bin;
  if (ro_dim(&p) == 1) {
    for (uint64_t g = 1; g < nb; ++g) res[g] = (int32_t)((uint32_t)res[g] + (uint32_t)res[g - 1]);
  } else {
    for (uint64_t pa = 0; pa < p.panels; ++pa) {
      for (uint64_t I = 0; I < Hb; ++I)
        for (uint64_t J = 1; J < Wb; ++J) {
          const uint64_t g = (pa * Hb + I) * Wb + J;
          res[g] = (int32_t)((uint32_t)res[g] + (uint32_t)res[g - 1]);
        }
      for (uint64_t I = 1; I < Hb; ++I)
        for (uint64_t J = 0; J < Wb; ++J) {
          const uint64_t g = (pa * Hb + I) * Wb + J;
          res[g] = (int32_t)((uint32_t)res[g] + (uint32_t)res[g - Wb]);
        }
    }
    if (ro_dim(&p) == 3)
      for (uint64_t g = Hb * Wb; g < nb; ++g)
        res[g] = (int32_t)((uint32_t)res[g] + (uint32_t)res[g - Hb * Wb]);
  }
  /* background: the bin value replicated over the bin */
  const double step = 2.0 * p.eb;
  for (uint64_t pa = 0; pa < p.panels; ++pa)
    for (uint64_t i = 0; i < p.height; ++i)
      for (uint64_t j = 0; j < p.width; ++j) {
        const uint64_t g = (pa * Hb + i / b) * Wb + j / b;
        frame[(pa * p.height + i) * p.width + j] = (float)((double)res[g] * step);
      }
  /* ROI windows, bit-exact from the payload (verbatim, or decoded) */
  const int64_t h = p.window / 2, w = p.window;
  const uint64_t nroi = (uint64_t)np * w * w;
  uint32_t *dec = NULL;
  const uint8_t *payload = in + L.roi;
  if (p.roi_coding) {
    dec = (uint32_t *)malloc(4 * (size_t)(nroi ? nroi : 1));
    if (ro_roi_decode(&p, in, &L, np, Troi, dec) != RO_OK) {
      free(pk); free(hw); free(res); free(cd); free(dec);
      return RO_ERR_CORRUPT;
    }
    payload = (const uint8_t *)dec;
  }
  for (uint32_t k = 0; k < np; ++k) {
    const int64_t pa = pk[3 * k], r0 = pk[3 * k + 1] - h, c0 = pk[3 * k + 2] - h;
    for (int64_t u = 0; u < w; ++u)
      for (int64_t v = 0; v < w; ++v) {
        const int64_t i = r0 + u, j = c0 + v;
        if (i < 0 || i >= (int64_t)p.height || j < 0 || j >= (int64_t)p.width) continue;
        memcpy(&frame[((uint64_t)pa * p.height + (uint64_t)i) * p.width + (uint64_t)j],
               payload + 4 * (((uint64_t)k * w + (uint64_t)u) * w + (uint64_t)v), 4);
      }
  }
  /* windows that overlap copy the same frame pixel, so every payload entry
   * must agree with what was restored there; a stream where they differ is
   * malformed */
  for (uint32_t k = 0; k < np && !bad; ++k) {
    const int64_t pa = pk[3 * k], r0 = pk[3 * k + 1] - h, c0 = pk[3 * k + 2] - h;
    for (int64_t u = 0; u < w && !bad; ++u)
      for (int64_t v = 0; v < w; ++v) {
        const int64_t i = r0 + u, j = c0 + v;
        if (i < 0 || i >= (int64_t)p.height || j < 0 || j >= (int64_t)p.width) continue;
        if (memcmp(&frame[((uint64_t)pa * p.height + (uint64_t)i) * p.width + (uint64_t)j],
                   payload + 4 * (((uint64_t)k * w + (uint64_t)u) * w + (uint64_t)v), 4) != 0) {
          bad = 1;
          break;
        }
      }
  }
  free(pk); free(hw); free(res); free(cd); free(dec);
  return bad ? RO_ERR_CORRUPT : RO_OK;
}

/* ------------------------------------------------------------ peak finding */

/* Peak finder feeding the ROI mask (the step before the path: Sec. IV-B names
 * the algorithm and its parameters; Sec. II and Sec. IV the non-hit
 * rejection that counts its peaks).  Readings where the text is loose:
 *   - local maximum: the pixel is >= every pixel of its (2h+1)^2 window
 *     (clipped to the panel) and > every one before it in raster order, so
 *     a plateau yields its first pixel;
 *   - background: mean mu and population variance V/m of the m pixels whose
 *     Chebyshev distance from the maximum lies in [ring_in, ring_out],
 *     clipped to the panel (two passes, raster order); no such pixel, no
 *     peak;
 *   - peak pixels ("neighbouring pixels above 0 ADU"): the pixels of the
 *     window 4-connected to the maximum through pixels x with x - mu >
 *     pix_nsigma * sigma (pix_nsigma = 0 is the text taken relative to the
 *     background; on noisy frames half of the background would then count);
 *   - total intensity: the sum S of the peak pixels (raster order); signal
 *     to noise: (S - n mu) / (sigma sqrt(n)).
 * Square roots are avoided by comparing squares of non-negative sides:
 * d > k sigma  <=>  d > 0 and d*d*m > k*k*V  (and the same for the SNR). */
typedef struct {
  uint32_t rank;                /* h: window (2h+1) x (2h+1), 1..3 (3: 7x7)   */
  uint32_t ring_in, ring_out;   /* background ring, h < ring_in <= ring_out <= 15 */
  uint32_t npix_min, npix_max;  /* peak pixel count bounds (2, 30)           */
  uint32_t reserved;
  double amax_min;              /* maximum >= amax_min (300 ADU)            */
  double atot_min;              /* total intensity > atot_min (600 ADU)     */
  double snr_min;               /* signal to noise > snr_min (10)           */
  double pix_nsigma;            /* peak pixel cut above the background (3)  */
} ro_peak_params;

int ro_check_peak_params(const ro_peak_params *q) {
  if (!q || q->rank < 1 || q->rank > 3 || q->ring_in <= q->rank || q->ring_out < q->ring_in ||
      q->ring_out > 15 || q->npix_min > q->npix_max || q->reserved != 0)
    return RO_ERR_ARG;
  if (!isfinite(q->amax_min) || !isfinite(q->atot_min) || !isfinite(q->snr_min) ||
      !(q->snr_min >= 0.0) || !isfinite(q->pix_nsigma) || !(q->pix_nsigma >= 0.0))
    return RO_ERR_ARG;
  return RO_OK;
}

/* Decision for the local maximum at (i, j) of panel x (H x W). */
static int ro_peak_accept(const ro_peak_params *q, const float *x, int64_t H, int64_t W,
                          int64_t i, int64_t j) {
  const int64_t h = q->rank, ww = 2 * h + 1;
  /* background ring */
  double sum = 0.0;
  int64_t m = 0;
  for (int64_t u = i - (int64_t)q->ring_out; u <= i + (int64_t)q->ring_out; ++u)
    for (int64_t v = j - (int64_t)q->ring_out; v <= j + (int64_t)q->ring_out; ++v) {
      const int64_t d = llabs(u - i) > llabs(v - j) ? llabs(u - i) : llabs(v - j);
      if (u < 0 || u >= H || v < 0 || v >= W || d < (int64_t)q->ring_in) continue;
      sum += (double)x[u * W + v];
      m++;
    }
  if (m == 0) return 0;
  const double mu = sum / (double)m;
  double V = 0.0;
  for (int64_t u = i - (int64_t)q->ring_out; u <= i + (int64_t)q->ring_out; ++u)
    for (int64_t v = j - (int64_t)q->ring_out; v <= j + (int64_t)q->ring_out; ++v) {
      const int64_t d = llabs(u - i) > llabs(v - j) ? llabs(u - i) : llabs(v - j);
      if (u < 0 || u >= H || v < 0 || v >= W || d < (int64_t)q->ring_in) continue;
      const double e = (double)x[u * W + v] - mu;
      V += e * e;
    }
  const double k2V = q->pix_nsigma * q->pix_nsigma * V;
  /* window pixels above the cut, then the 4-connected component of the
   * maximum by repeated growth over the 7x7 (at most) grid */
  int above[7][7], comp[7][7];
  for (int64_t a = 0; a < ww; ++a)
    for (int64_t b = 0; b < ww; ++b) {
      const int64_t u = i - h + a, v = j - h + b;
      above[a][b] = 0;
      comp[a][b] = 0;
      if (u < 0 || u >= H || v < 0 || v >= W) continue;
      const double d = (double)x[u * W + v] - mu;
      above[a][b] = d > 0.0 && d * d * (double)m > k2V;
    }
  comp[h][h] = above[h][h];
  for (int changed = 1; changed;) {
    changed = 0;
    for (int64_t a = 0; a < ww; ++a)
      for (int64_t b = 0; b < ww; ++b) {
        if (comp[a][b] || !above[a][b]) continue;
        if ((a > 0 && comp[a - 1][b]) || (a + 1 < ww && comp[a + 1][b]) ||
            (b > 0 && comp[a][b - 1]) || (b + 1 < ww && comp[a][b + 1])) {
          comp[a][b] = 1;
          changed = 1;
        }
      }
  }
  double S = 0.0;
  int64_t n = 0;
  for (int64_t a = 0; a < ww; ++a)
    for (int64_t b = 0; b < ww; ++b)
      if (comp[a][b]) {
        S += (double)x[(i - h + a) * W + (j - h + b)];
        n++;
      }
  if (n < (int64_t)q->npix_min || n > (int64_t)q->npix_max) return 0;
  if (!(S > q->atot_min)) return 0;
  const double num = S - (double)n * mu;
  return num > 0.0 && num * num * (double)m > q->snr_min * q->snr_min * (double)n * V;
}

/* Peaks of a panels x height x width frame, in raster order (panel, row,
 * col), as int32 triples in peaks[0 .. min(count, cap)); returns the count
 * (which may exceed cap). */
uint64_t ro_find_peaks(const ro_peak_params *q, uint32_t P, uint32_t H, uint32_t W,
                       const float *frame, int32_t *peaks, uint64_t cap) {
  const int64_t h = q->rank;
  uint64_t cnt = 0;
  for (int64_t p = 0; p < P; ++p) {
    const float *x = frame + (uint64_t)p * H * W;
    for (int64_t i = 0; i < H; ++i)
      for (int64_t j = 0; j < W; ++j) {
        const float c = x[i * W + j];
        if (!((double)c >= q->amax_min)) continue;
        int ismax = 1;
        for (int64_t u = i - h; u <= i + h && ismax; ++u)
          for (int64_t v = j - h; v <= j + h; ++v) {
            if (u < 0 || u >= H || v < 0 || v >= W || (u == i && v == j)) continue;
            const float o = x[u * W + v];
            const int before = u < i || (u == i && v < j);
            if (before ? !(o < c) : !(o <= c)) {
              ismax = 0;
              break;
            }
          }
        if (!ismax || !ro_peak_accept(q, x, H, W, i, j)) continue;
        if (cnt < cap) {
          peaks[3 * cnt] = (int32_t)p;
          peaks[3 * cnt + 1] = (int32_t)i;
          peaks[3 * cnt + 2] = (int32_t)j;
        }
        cnt++;
      }
  }
  return cnt;
}
