/* Test infrastructure, not part of the product path: runs the oracle over
 * cases read from a file, outside Python, so that the oracle can be built
 * with AddressSanitizer and UndefinedBehaviorSanitizer and its results
 * compared with those of the normal build.  The oracle's source is included
 * so that one build instruments all of it.
 *
 * Usage: sanitize_driver <cases> <results>.  Records, little endian, until
 * the end of <cases>; each writes one result record:
 *   1 compress and decompress: ro_params, u32 npeaks, f32 frame[P*H*W],
 *     i32 peaks[3*npeaks]  ->  i32 status, u64 nbytes, u8 stream[nbytes],
 *     and when status is 0: i32 status of the decompression, f32 frame[P*H*W]
 *   2 decompress: u64 n, u64 frame_elems, u8 stream[n]  ->  i32 status,
 *     f32 frame[frame_elems]
 *   3 find peaks: ro_peak_params, u32 P, H, W, u64 cap, f32 frame[P*H*W]
 *     ->  u64 count, i32 peaks[3*min(count, cap)]
 *   4 Huffman code: u32 hist[1024]  ->  u8 lengths[1024], u32 codewords[1024]
 * Every buffer is allocated to its exact size, so that a read or write past
 * it is reported. */
#include "rsz_oracle.c"

#include <stdio.h>

static FILE *g_in, *g_out;

static void *take(size_t n) {
  void *p = malloc(n ? n : 1);
  if (!p || (n && fread(p, 1, n, g_in) != n)) {
    fprintf(stderr, "sanitize_driver: short read\n");
    exit(2);
  }
  return p;
}

static void put(const void *p, size_t n) {
  if (n && fwrite(p, 1, n, g_out) != n) {
    fprintf(stderr, "sanitize_driver: short write\n");
    exit(2);
  }
}

static void compress_case(void) {
  ro_params *p = (ro_params *)take(sizeof(ro_params));
  uint32_t *np = (uint32_t *)take(4);
  const uint64_t elems = (uint64_t)p->panels * p->height * p->width;
  float *frame = (float *)take(4 * elems);
  int32_t *peaks = (int32_t *)take(12ull * *np);
  uint64_t cap = 0, nbytes = 0;
  int32_t st = ro_max_bytes(p, *np, &cap);
  uint8_t *out = (uint8_t *)malloc(cap ? cap : 1);
  if (st == 0) st = ro_compress(p, frame, *np ? peaks : NULL, *np, out, cap, &nbytes);
  put(&st, 4);
  put(&nbytes, 8);
  if (st == 0) {
    /* the stream in a buffer of exactly its size */
    uint8_t *s = (uint8_t *)malloc(nbytes);
    memcpy(s, out, nbytes);
    put(s, nbytes);
    float *y = (float *)malloc(4 * elems);
    const int32_t ds = ro_decompress(s, nbytes, y, elems);
    put(&ds, 4);
    put(y, 4 * elems);
    free(y);
    free(s);
  }
  free(out);
  free(peaks);
  free(frame);
  free(np);
  free(p);
}

static void decompress_case(void) {
  uint64_t *n = (uint64_t *)take(8), *elems = (uint64_t *)take(8);
  uint8_t *s = (uint8_t *)take(*n);
  float *y = (float *)calloc(*elems ? *elems : 1, 4);
  const int32_t st = ro_decompress(s, *n, y, *elems);
  put(&st, 4);
  put(y, 4 * *elems);
  free(y);
  free(s);
  free(elems);
  free(n);
}

static void peaks_case(void) {
  ro_peak_params *q = (ro_peak_params *)take(sizeof(ro_peak_params));
  uint32_t *dims = (uint32_t *)take(12);
  uint64_t *cap = (uint64_t *)take(8);
  float *frame = (float *)take(4ull * dims[0] * dims[1] * dims[2]);
  int32_t *peaks = (int32_t *)malloc(12 * (*cap ? *cap : 1));
  const uint64_t cnt = ro_find_peaks(q, dims[0], dims[1], dims[2], frame, peaks, *cap);
  put(&cnt, 8);
  put(peaks, 12 * (cnt < *cap ? cnt : *cap));
  free(peaks);
  free(frame);
  free(cap);
  free(dims);
  free(q);
}

static void huffman_case(void) {
  uint32_t *hist = (uint32_t *)take(4 * RO_NSYM);
  uint8_t *len = (uint8_t *)malloc(RO_NSYM);
  uint32_t *cw = (uint32_t *)malloc(4 * RO_NSYM);
  ro_huffman_lengths(hist, len);
  ro_canonical(len, cw);
  put(len, RO_NSYM);
  put(cw, 4 * RO_NSYM);
  free(cw);
  free(len);
  free(hist);
}

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: sanitize_driver <cases> <results>\n");
    return 2;
  }
  g_in = fopen(argv[1], "rb");
  g_out = fopen(argv[2], "wb");
  if (!g_in || !g_out) return 2;
  uint32_t kind;
  while (fread(&kind, 4, 1, g_in) == 1) {
    switch (kind) {
      case 1: compress_case(); break;
      case 2: decompress_case(); break;
      case 3: peaks_case(); break;
      case 4: huffman_case(); break;
      default: fprintf(stderr, "sanitize_driver: unknown record %u\n", kind); return 2;
    }
  }
  fclose(g_in);
  return fclose(g_out) == 0 ? 0 : 2;
}
