// rsz_internal.h -- plan structures shared by the host side and the HIP
// kernels of librsz.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rsz.h"

namespace rsz {

constexpr int kRadius = 512;          // residuals in (-512, 512) get a code
constexpr int kNumSym = 1024;         // code alphabet; code 0 marks an outlier
constexpr int kMaxLen = 32;           // longest Huffman codeword
constexpr uint32_t kChunk = 4096;     // symbols between bitstream sync offsets
constexpr double kQMax = 268435455.0; // |q| <= 2^28 - 1
constexpr uint64_t kHeader = 80;
constexpr int kRoiClasses = 33;       // coded ROI: bit lengths 0..32 of the zigzag residual
constexpr uint64_t kRoiLens = 36;     // their code lengths, padded

// Binning kernel geometry: up to 4 independent waves per workgroup, each
// owning a tile of one panel: a segment of up to kMaxTH bin rows x a column
// group of up to group_strips(b) strips of 64 bin columns.
constexpr int kWaves = 4;
constexpr int kMaxTH = 32;
constexpr int kMaskWords = 1024;      // per wave: (TH+1)*b rows x (2b*strips+1) words
constexpr uint64_t kTargetWaves = 8192;         // default tiling: binning waves per batch
constexpr uint32_t kFixBins3 = 16384;           // k_lorenzo_dims, dim 3: bins per workgroup
constexpr uint32_t kTileEntries = kMaxTH * 4;   // sparse codes: entries per binning tile

// Strips per column group for bin factor b as compiled in the binning kernel
// (0: any b, and batches mixing bin factors).
__host__ __device__ constexpr int group_strips(int b) {
  return b == 1 || b == 2 ? 4 : (b == 4 ? 2 : 1);
}

inline __host__ __device__ uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// The plans' pointers are generic; the path's buffers are all device (global)
// memory, and accesses through an address_space(1) pointer compile to global
// loads and stores.  Generic (flat) ones would also count against the LDS
// wait counter, so every LDS wait would wait for the HBM accesses in flight
// too.
#define RSZ_G __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ RSZ_G T *gm(T *p) {
  return (RSZ_G T *)p;
}
// Plain vector types for such accesses (loads and stores of 8 and 16 bytes).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld16(const void *p) {
  const u32x4 v = *gm((const u32x4 *)p);
  return make_uint4(v.x, v.y, v.z, v.w);
}

// Inclusive prefix sum (wrapping) of x over the 64 lanes of a wave, on DPP
// lane moves: shifts by 1, 2, 4 and 8 lanes within each row of 16, then
// lane 15 of a row added into the next row and lane 31 into the upper
// half.  A lane with no source lane, or outside the rows a move writes,
// adds 0.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false); // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false); // row_bcast:31
  return x;
}

// Division by a run-time constant d (1 <= d < 2^16) through a multiply: with
// l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1, n / d = (hi32(n m) +
// n) >> l for every n < 2^31 (Granlund and Montgomery, "Division by invariant
// integers using multiplication", 1994: the round-up multiplier; the sum
// stays below 2^32 because hi32(n m) < n).
struct FastDiv {
  uint32_t m, l;
};
__host__ __device__ inline FastDiv fast_div(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  return FastDiv{(uint32_t)((((1ull << l) - d) << 32) / d + 1), l};
}
__host__ __device__ __forceinline__ uint32_t fdiv(FastDiv f, uint32_t n) {
  return (uint32_t)((((uint64_t)n * f.m) >> 32) + n) >> f.l;
}

// Per-frame mutable state in the workspace.
struct FrameState {
  int32_t status;
  uint32_t n_out;
  uint64_t T;          // bitstream bits
  uint64_t total;      // stream bytes
  uint64_t Troi;       // coded ROI bits
  uint64_t off_runbits;  // run coding: stream offset of the run bits
  uint32_t hist[kNumSym];
  uint32_t cw[kNumSym];
  uint8_t lens[kNumSym];
  double inv[65];      // inv[n] = 1 / (n * 2eb), correctly rounded (k_prep)
};

// Per-frame constant plan, built on the host and copied to the workspace.
struct FramePlan {
  uint32_t P, H, W, w, b, mode;
  uint32_t dim;             // Lorenzo dimension: 1, 2 or 3
  uint32_t roi_coding;      // ROI windows coded (1) or verbatim (0)
  uint32_t run_coding;      // Huffman bits run coded (1) or verbatim (0)
  double eb, step;          // step = 2*eb
  uint32_t Hb, Wb, nbins, nchunks;
  uint32_t npeaks, TH, segs, groups;   // segments per panel, workgroups per panel
  uint32_t nstrips, gstrips, cgs;   // strips per panel row, per column group; groups
  int32_t init_status;      // RSZ_OK or RSZ_ERR_ARG
  uint32_t vec;             // rows load as float2/float4 (W % b == 0, aligned)
  const float *frame;
  const int32_t *peaks;     // npeaks x (panel,row,col)
  uint8_t *out;
  uint64_t out_cap;
  // stream sections before the bitstream have fixed offsets
  uint64_t off_roi, off_lens, off_chunks, off_bits;
  uint8_t *codes;           // nbins code bytes (r + 128, or 0: see rbuf), dense
                            // (dimension 3), then the chunk form's bytes
  int32_t *rbuf;            // nbins, residual of bins whose code byte is 0
  uint64_t *cmask;          // nchunks * 64: the chunk form's masks (k_count)
  uint32_t *lanecnt;        // nchunks * 64: per 64 bins of a chunk, their bits
                            // (low 16) and outliers (high 16) (k_count)
  // Sparse codes (frames of Lorenzo dimension 1 or 2; dimension 3 keeps the
  // dense bytes above): per binning tile (index (panel * cgs + cg) * segs +
  // seg), kTileEntries entries, entry s * 32 + i for strip s of the column
  // group and tile row i: zm, bit k set where column 64 * strip + k carries a
  // code byte other than 128 (residual 0); zp, how many such bytes the tile
  // holds before the entry.  The bytes themselves, in tile order (row,
  // strip, column), at zb + tile * tile_cap.
  uint32_t sparse;
  uint32_t tile_cap;
  FastDiv fd_Wb, fd_Hb, fd_TH, fd_gs;
  uint64_t *zm;
  uint16_t *zp;
  uint8_t *zb;
  uint8_t *codes2;          // where k_bin writes its code bytes and residuals:
  int32_t *rbuf2;           // codes / rbuf, except for dim 3 (own buffers of
                            // the 2D residuals, differenced by k_lorenzo_dims)
  uint32_t *obuf;           // nbins, outlier bin indices in stream order
  uint32_t *chunk_off;      // nchunks: bit count, then bit offset of each chunk
  uint32_t *chunk_oo;       // nchunks: outlier count, then outlier offset
  uint32_t *head;           // nchunks: bits of a chunk in its shared first word
  uint32_t *bstart;         // P*segs+1 starts of the peak bands: band k =
                            // (panel k / segs, raw rows [(k % segs)*TH*b, +TH*b))
  uint32_t *bucket;         // npeaks peaks as (row << 16 | col), grouped by band
  // coded ROI (else null): class histogram, code lengths and codewords (over
  // kNumSym entries, the first kRoiClasses used), window bits then offsets
  uint32_t *roi_hist;
  uint8_t *roi_lens;
  uint32_t *roi_cw;
  uint32_t *roi_bits;
  int32_t *qedge;           // dim 1: q of the last bin of each of the P*Hb bin
                            // rows (those k_lorenzo_dims reads), else null
  // where k_encode writes the Huffman words: the stream's bitstream section
  // (bw_cap = the words the output buffer holds there), or with the runs
  // coded a workspace buffer of nbins + 2 words
  uint32_t *bw;
  uint64_t bw_cap;
  // run coding (else null): per chunk the run bits, then their bit offsets
  // (nchunks + 1, the last the section's bits), and the Rice parameters
  uint32_t *run_off;
  uint8_t *run_k;
  FrameState *st;
  uint64_t *res_bytes;      // where to report the size (device)
  int32_t *res_status;      // where to report the status (device)
  // debug outputs (device, may be null)
  uint32_t *dbg_mask;
  double *dbg_S;
  uint32_t *dbg_n;
  int32_t *dbg_q;
};

// Prefix sums over the frames of a batch, for mapping flat work items.
struct BatchPlan {
  uint32_t nframes;
  uint32_t total_tiles, total_units, total_peaks, total_chunks;
  uint32_t cpw;                  // chunks encoded by one k_encode workgroup
  uint32_t all_vec;              // every frame's rows load as float2/float4 (k_bin)
  uint32_t bin_waves;            // waves per k_bin workgroup (1..kWaves)
  uint32_t total_fix;            // workgroups of k_lorenzo_dims (0: every frame is 2D)
  uint32_t roi_coding;           // some frame codes its ROI windows
  uint32_t run_coding;           // some frame codes its Huffman bits' runs
  const FramePlan *frames;
  const uint32_t *tile_prefix;   // nframes + 1
  const uint32_t *unit_prefix;   // nframes + 1 (units of cpw chunks)
  const uint32_t *peak_prefix;   // nframes + 1
  const uint32_t *chunk_prefix;  // nframes + 1
  const uint32_t *fix_prefix;    // nframes + 1 (k_lorenzo_dims workgroups)
  // frame tables, written by k_prep (every frame's workgroup writes its own
  // entries): per k_count workgroup (frame, chunk) of its first chunk; the
  // frame of each k_bin workgroup, k_encode workgroup and peak
  uint2 *count_frame;
  uint32_t *tile_frame;
  uint32_t *unit_frame;
  uint32_t *peak_frame;
  uint32_t all_sparse;           // every frame has sparse codes (no dimension 3)
};

// Launchers (compress.hip).
// k_prep + k_bin (+ k_lorenzo_dims) + k_codebook; b and dim: the common bin
// factor and Lorenzo dimension of the batch, or 0 when its frames differ.
hipError_t launch_compress_front_b(const BatchPlan &bp, uint32_t b, uint32_t dim, hipStream_t s,
                                   bool debug);
hipError_t launch_debug_codes(const BatchPlan &bp, uint32_t nbins, uint16_t *out, hipStream_t s);
hipError_t launch_debug_outliers(const BatchPlan &bp, uint32_t *n_out, uint32_t *idx,
                                 int32_t *res, hipStream_t s);
hipError_t launch_codebook(const BatchPlan &bp, hipStream_t s);
// k_count + k_scan + k_encode + k_tail + k_roi.
hipError_t launch_compress_back(const BatchPlan &bp, hipStream_t s);

// Decompression plan and launchers (decompress.hip).
struct DecodePlan {
  uint32_t P, H, W, w, b, npeaks, dim, roi_coding;
  uint64_t Troi;
  uint64_t off_rsec, off_roffs, off_rbits;   // coded ROI section
  uint32_t *roi_payload;                      // coded ROI: npeaks*w*w decoded words
  uint32_t *roi_tables;                       // coded ROI: decode tables
  uint32_t run_coding;                        // run section instead of the bitstream:
  uint64_t off_run, off_runoffs, off_runbits; // parameters, offsets, run bits
  const uint32_t *bits;                       // the Huffman words (stream or hbits)
  uint32_t *hbits;                            // runs coded: ceil(T/32) + 2 expanded words
  double step;
  uint32_t Hb, Wb, nbins, nchunks, n_out;
  uint64_t T, total;
  uint64_t off_peaks, off_roi, off_lens, off_oidx, off_ores, off_chunks, off_bits;
  const uint8_t *in;
  float *frame;
  int32_t *res;         // nbins: residuals; for k_dec_panel's streams only those
                        // whose code byte (res8) is 0
  uint8_t *res8;        // nbins (+64): k_dec_panel's streams, r + 128 for
                        // |r| <= 127, else 0 with r (or the outlier mark) in res
  uint32_t *zcount;     // nchunks code-0 counts
  uint32_t *carry;      // dim 1: P*Hb row carries
  int32_t *status;      // one word
  uint32_t *tables;     // decode tables
  int32_t init_status;  // RSZ_OK, or the host's verdict on the stream (no other work)
};

// Streams decoded together: every decoder kernel is launched once for all of
// them, its workgroups numbered across the frames.  pre holds kDecKernels
// prefix arrays of n + 1 entries, kernel K's per-frame workgroup counts.
constexpr int kDecKernels = 17;
struct DecBatch {
  uint32_t n;
  const DecodePlan *plans;
  const uint32_t *pre;
};
// Workgroups of each decoder kernel for one frame (0: not launched for it).
void decode_blocks(const DecodePlan &dp, uint32_t *nb);
// Launches the kernels with total[K] workgroups (the prefixes' last entries).
hipError_t launch_decompress(const DecBatch &db, const uint32_t *total, hipStream_t s);

// On-device verification of a compressed batch (verify.hip): the batch's
// streams decoded by the decoder kernels (their plans completed on the
// device from the compression's totals), then every pixel checked against
// the frame it came from.
constexpr uint32_t kVerifyMaskWords = 8192;   // LDS ROI bitmap of a workgroup's rows
constexpr uint32_t kVerifyOutlierBlocks = 16; // k_dec_outliers workgroups per frame
struct VerifyFrame {
  const float *x;           // the frame
  const float *y;           // its decoding
  const int32_t *peaks;
  uint32_t npeaks, P, H, W, w, b, mode;
  double eb;
  uint32_t rows;            // raw rows per k_verify workgroup (a multiple of b)
  uint32_t chunks;          // k_verify workgroups per panel
  int32_t valid;            // the descriptor was valid
  const FramePlan *cplan;   // the compression's plan of the frame (device)
  DecodePlan *dplan;        // the decoder's plan (device; k_vplan completes it)
  uint32_t *bad;            // device: violations, or 0xFFFFFFFF when a stage failed
};
struct VerifyBatch {
  uint32_t n;
  const VerifyFrame *frames;  // device
  const uint32_t *wg_prefix;  // device, n + 1: k_verify workgroups per frame
  uint32_t total_wgs;
};
hipError_t launch_verify_plan(const VerifyBatch &vb, hipStream_t s);
hipError_t launch_verify_check(const VerifyBatch &vb, hipStream_t s);

// Peak finding (peaks.hip).
constexpr uint32_t kPeakTile = 16384;     // pixels per k_peaks_find workgroup
constexpr uint32_t kPeakCapMax = 8192;    // most peaks a frame's list may hold

struct PeakFramePlan {
  uint32_t P, H, W, cap;
  int32_t init_status;       // RSZ_OK or RSZ_ERR_ARG
  const float *frame;
  rsz_peak *out;             // cap entries (caller's)
  uint64_t *keys;            // cap keys (p << 32 | i << 16 | j), unordered
  uint32_t *count;           // peaks found (may exceed cap)
  uint32_t *res_count;       // caller's count
  int32_t *res_status;       // caller's status
};

struct PeakBatchPlan {
  uint32_t nframes, total_tiles;
  float amax_f;                  // smallest float >= q.amax_min
  rsz_peak_params q;
  const PeakFramePlan *frames;
  const uint32_t *tile_prefix;   // nframes + 1
};
hipError_t launch_find_peaks(const PeakBatchPlan &pp, hipStream_t s);

// Kernel timing hooks (api.hip).
void prof_begin(const char *name, hipStream_t s);
void prof_end(hipStream_t s);

}  // namespace rsz
