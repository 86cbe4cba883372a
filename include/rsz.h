/*
 * rsz.h -- C ABI of librsz: ROIBIN-SZ per-frame compression of serial
 * crystallography detector frames on an AMD MI355X (gfx950) GPU.
 *
 * Method (arXiv 2206.11297): each frame is split into the regions of interest
 * around its Bragg peaks, kept without error, and the background (Sec. IV).
 * The background is binned b x b by its mean (Sec. VI) and compressed with an
 * absolute error bound that holds on the binned values (Sec. V-C, "Our
 * Approach").  Here the background compressor is prequantisation at step 2*eb,
 * a Lorenzo predictor over the integer field (in one, two or three
 * dimensions, the "dimension" of Sec. VI), outlier capture outside a radius
 * of 512, and Huffman coding over 1024 symbols.
 *
 * Conventions for every entry point:
 *   - Pointers prefixed d_ are device memory (e.g. torch tensors on the GPU),
 *     h_ are host memory.  The caller owns every buffer; the library allocates
 *     no device memory and keeps no pointer after a call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   - Functions return an rsz_status value and never throw.  After an error
 *     the contents of output buffers are unspecified.
 *   - Calls on different streams with different workspaces may run
 *     concurrently; calls sharing a workspace must be ordered by the caller.
 *   - Device buffers must be 16-byte aligned (frames, outputs, workspaces).
 *
 * Frame layout: panels x height x width float32, C-contiguous.  Stream
 * layout (little-endian, sections 4-byte aligned): 80-byte header (flags:
 * bit 0 bin_mode, bits 1-2 the Lorenzo dimension, 0 for 2, bit 3 the ROI
 * coded, bit 4 the runs coded; bytes 72-79 the coded ROI bits, else 0), peaks
 * (u16 panel,row,col), ROI payload (npeaks*w*w u32 bit patterns, 0 outside
 * the panel), code lengths (1024 u8), chunk bit offsets (u32, one per 4096
 * symbols), bitstream (u32 words, codewords MSB-first), outlier bin indices
 * (u32), outlier residuals (i32).  With the ROI coded, the verbatim payload is
 * absent and the coded ROI section ends the stream: 33 class code lengths
 * (u8, padded to 36 bytes), one u32 bit offset per window, the ROI bitstream.
 * With the runs coded, the bitstream is absent and a run section ends the
 * stream: one Rice parameter per chunk (u8, padded to 4 bytes), one u32 bit
 * offset per chunk plus the section's total bits, then the run bits.
 */
#ifndef RSZ_H
#define RSZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A Bragg peak: integer pixel position (Sec. IV-B: the peak list is an array
 * of coordinates). */
typedef struct {
  int32_t panel, row, col;
} rsz_peak;

/* Compression parameters.
 *   panels, height, width: frame shape, each 1..65535, pixels < 2^31, and
 *     panels*ceil(height/bin)*ceil(width/bin) < 2^27 bins.
 *   window: ROI edge w in pixels, 1..1023 (17 in the paper, Sec. IV); the
 *     window of a peak at (r,c) covers rows r-w/2 .. r-w/2+w-1 (integer
 *     division), same for columns, clipped to the panel.
 *   bin: bin factor b, 1..8 (2 in the paper's chosen setting, Sec. VI).
 *   bin_mode: RSZ_BIN_BACKGROUND averages only pixels outside every ROI
 *     window; RSZ_BIN_ALL averages every pixel of the bin.
 *   eb: absolute error bound on binned values, finite and > 0.
 *   dim: dimension of the Lorenzo predictor (Sec. VI): 1 reads the binned
 *     frame as one sequence in raster order (panel, row, column), 2 reads
 *     each panel as an image (0 also means 2, the default), 3 reads the
 *     stack of panels as a volume.  Residuals take zeros outside the domain.
 *   roi_coding: 0 stores the ROI windows verbatim; 1 codes them losslessly
 *     (the paper uses fpzip, Sec. IV): each window's float bits are mapped to
 *     order-preserving integers, predicted by a 2D Lorenzo predictor over the
 *     window, and the zigzag residual's bit length is Huffman coded and
 *     followed by its remaining bits.  Needs npeaks*window^2 <= 2^26.
 *   run_coding: 0 stores the Huffman bitstream as it is; 1 passes it through
 *     a lossless stage of this library's own (the paper does not describe
 *     one; SZ-family coders follow their Huffman coder with a general
 *     lossless pass): in each 4096-symbol chunk the lengths of the zero runs
 *     before each one bit are Rice coded (a unary quotient, then k low bits)
 *     with the chunk's cheapest parameter k in 0..20.  Never more bits than
 *     the bitstream; it pays off where residual 0 dominates, as its codeword
 *     is the all-zero one.
 *   reserved: set to 0. */
typedef struct {
  uint32_t panels, height, width;
  uint32_t window;
  uint32_t bin;
  uint32_t bin_mode;
  double eb;
  uint32_t dim;
  uint32_t roi_coding;
  uint32_t run_coding;
  uint32_t reserved;
} rsz_params;

enum { RSZ_BIN_BACKGROUND = 0, RSZ_BIN_ALL = 1 };

typedef enum {
  RSZ_OK = 0,
  RSZ_ERR_ARG = -1,       /* invalid parameter, pointer, size or alignment */
  RSZ_ERR_PEAK = -2,      /* a peak lies outside the frame                 */
  RSZ_ERR_RANGE = -3,     /* a background bin is non-finite or |q| >= 2^28 */
  RSZ_ERR_CAPACITY = -4,  /* output buffer too small (size reported)       */
  RSZ_ERR_CORRUPT = -5,   /* malformed compressed stream                   */
  RSZ_ERR_WORKSPACE = -6, /* workspace too small                           */
  RSZ_ERR_HIP = -7        /* HIP runtime error                             */
} rsz_status;

/* Human-readable name of a status value (static string).  A diagnostic of
 * this library's status codes; no passage of the paper defines it. */
const char *rsz_status_string(int status);

/* Upper bound of the compressed size of one frame with npeaks peaks (every
 * bin an outlier and every codeword 32 bits).  Host-only.  With the workspace
 * query below it lets the caller preallocate every buffer, so compression
 * itself allocates nothing (the zero-allocation compression into
 * preallocated buffers of Sec. IV-A). */
int rsz_max_compressed_bytes(const rsz_params *p, uint32_t npeaks, uint64_t *bytes);

/* Device workspace needed by rsz_compress for one frame (preallocated by the
 * caller, Sec. IV-A).  Host-only. */
int rsz_workspace_bytes(const rsz_params *p, uint32_t npeaks, uint64_t *bytes);

/* Compress one device-resident frame (Sec. IV: ROI extraction, binning,
 * error-bounded compression of the binned background).
 *   d_frame: panels*height*width float32.  d_peaks: npeaks peaks (may be NULL
 *   when npeaks is 0).  d_out/out_cap: output buffer.  h_out_bytes: receives
 *   the stream size (also on RSZ_ERR_CAPACITY, where it is the size needed).
 *   d_ws/ws_bytes: workspace of at least rsz_workspace_bytes().
 * Work is queued on `stream`; the call returns after the stream has finished
 * it (it reads back the size).  Peaks outside the frame give RSZ_ERR_PEAK,
 * a non-finite or out-of-range background bin RSZ_ERR_RANGE. */
int rsz_compress(const rsz_params *p, const float *d_frame, const rsz_peak *d_peaks,
                 uint32_t npeaks, void *d_out, uint64_t out_cap, uint64_t *h_out_bytes,
                 void *d_ws, uint64_t ws_bytes, void *stream);

/* rsz_compress without a workspace argument, for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): it calls no hipMalloc, hipFree, hipHostMalloc or other
 * allocating routine.  Its workspace is a static device array of
 * RSZ_NOALLOC_SCRATCH_BYTES in the library's code object, one per GPU the
 * library runs on, held until the process ends; a frame whose
 * rsz_workspace_bytes exceeds it gives RSZ_ERR_WORKSPACE before any work is
 * queued (64 MiB covers e.g. a 32x512x1024 frame at bin 2).  The array keeps
 * the last call's contents, which the path never reads before writing.
 * Every call on a GPU shares that GPU's array, so two calls overlapping on
 * one GPU would race: the library holds a per-GPU lock for the whole call,
 * which (like rsz_compress) returns only after `stream` has finished its
 * work.  Other arguments, results and errors as rsz_compress; the stream
 * must belong to the current device.  Not for use under stream capture (the
 * call synchronizes). */
#define RSZ_NOALLOC_SCRATCH_BYTES (64ull << 20)
int rsz_compress_noalloc(const rsz_params *p, const float *d_frame, const rsz_peak *d_peaks,
                         uint32_t npeaks, void *d_out, uint64_t out_cap, uint64_t *h_out_bytes,
                         void *stream);

/* One frame of a batch.  out/out_cap: that frame's own output buffer
 * (device); the frames of a batch may have different shapes, parameters and
 * peak counts.  tile_rows, tile_strips: tuning knobs of the binning kernel's
 * tiles, the most bin rows and 64-column strips one wave walks (0 = library
 * default: the coarsest tiles that give a batch about 8192 waves;
 * clamped to what the kernel's LDS and registers hold).  tile_waves: waves
 * (tiles of consecutive row segments) per binning workgroup, 1..4 (0 = 4;
 * the batch takes its first valid frame's value).  These knobs change speed
 * only: the output bytes never depend on them (the autotuning of thread
 * counts in Sec. V-C, "Autotuning Configuration", likewise leaves the
 * output unchanged). */
typedef struct {
  rsz_params params;
  const float *frame;
  const rsz_peak *peaks;
  uint32_t npeaks;
  uint32_t tile_rows;
  uint32_t tile_strips;
  uint32_t tile_waves;
  void *out;
  uint64_t out_cap;
} rsz_frame_desc;

/* Device workspace for rsz_compress_batch over these descriptors (preallocated
 * by the caller, Sec. IV-A).  Host-only.  Descriptors with invalid parameters
 * are sized as empty. */
int rsz_batch_workspace_bytes(uint32_t nframes, const rsz_frame_desc *h_descs,
                              uint64_t *bytes);

/* Compress nframes frames in one batched launch sequence (every step of the
 * path is one kernel launch over all frames): the GPU form of compressing a
 * chunk of several events per compressor invocation (Sec. V-C, "Choice of
 * Chunk Size"), where each frame keeps its own self-contained stream so that
 * single events stay accessible.  h_descs is host memory and may
 * be reused once the call returns.  Per-frame results go to device arrays:
 * d_out_bytes[i] (stream size, or the size needed on RSZ_ERR_CAPACITY) and
 * d_status[i] (an rsz_status).  Asynchronous: returns after queueing; the
 * results are valid once `stream` has finished.  The return value reports only
 * errors of the call itself (ARG, WORKSPACE, HIP); a frame with invalid
 * parameters reports RSZ_ERR_ARG in d_status. */
int rsz_compress_batch(uint32_t nframes, const rsz_frame_desc *h_descs, uint64_t *d_out_bytes,
                       int32_t *d_status, void *d_ws, uint64_t ws_bytes, void *stream);

/* The same batch split in two, for callers that replay it (e.g. from a HIP
 * graph): rsz_batch_prepare copies the plan of the batch into d_ws (queued on
 * `stream`) and fills *h_plan, a caller-owned host record; rsz_batch_launch
 * queues only the kernels of the path, reading the plan from d_ws, and makes
 * no copy, memset or allocation, so it can be captured and replayed.  Every
 * replay recomputes all outputs from the frames' current contents; the
 * descriptors (pointers, shapes, peak counts) are fixed at prepare time. */
typedef struct {
  uint64_t opaque[32];
} rsz_batch_plan;

int rsz_batch_prepare(uint32_t nframes, const rsz_frame_desc *h_descs, uint64_t *d_out_bytes,
                      int32_t *d_status, void *d_ws, uint64_t ws_bytes, void *stream,
                      rsz_batch_plan *h_plan);
int rsz_batch_launch(const rsz_batch_plan *h_plan, void *stream);

/* Captures rsz_batch_launch of a prepared plan into a HIP graph on `stream`
 * (which must not be capturing already) and instantiates it: *h_graph_exec
 * receives a hipGraphExec_t (as void*).  rsz_graph_launch replays it on a
 * stream; rsz_graph_destroy frees it. */
int rsz_batch_graph_create(const rsz_batch_plan *h_plan, void *stream, void **h_graph_exec);
int rsz_graph_launch(void *graph_exec, void *stream);

/* On-device verification of a prepared batch, the decompress-and-check stage
 * of a graph-captured pipeline: every stream the batch writes is decoded on
 * the device (the decoder kernels of rsz_decompress_batch, their plans
 * completed on the device from the totals the compression left there) into
 * h_frames_out[i] (device, panels*height*width float32), and every pixel is
 * checked against the frame it came from: a pixel of an ROI window must
 * carry the frame's bits (Sec. IV), any other pixel must lie within eb of
 * the mean of its bin's pixels (Sec. V-C, the absolute bound on binned
 * values; Sec. IV-A, the bin value restored to each pixel), with the
 * float32 rounding of the stored value and a 2^-40 relative slack for the
 * fp64 sums.  d_bad[i] (device) receives frame i's count of pixels that
 * fail, 0xFFFFFFFF when its compression or decoding failed or it is not
 * verified (only frames with the ROI verbatim and no run stage are).
 * h_plan: from rsz_batch_prepare over the same descriptors; the plan,
 * descriptors and buffers are fixed at prepare time, and every launch
 * decodes and checks the batch's current streams.  rsz_verify_launch
 * queues kernels only (capturable); rsz_verify_graph_create captures the
 * batch's launch followed by the verification into one HIP graph (replay
 * with rsz_graph_launch, free with rsz_graph_destroy).  The workspace is
 * the caller's, separate from the batch's. */
typedef struct {
  uint64_t opaque[32];
} rsz_verify_plan;

int rsz_verify_workspace_bytes(const rsz_batch_plan *h_plan, uint32_t nframes,
                               const rsz_frame_desc *h_descs, uint64_t *bytes);
int rsz_verify_prepare(const rsz_batch_plan *h_plan, uint32_t nframes,
                       const rsz_frame_desc *h_descs, float *const *h_frames_out, uint32_t *d_bad,
                       void *d_ws, uint64_t ws_bytes, void *stream, rsz_verify_plan *h_vplan);
int rsz_verify_launch(const rsz_verify_plan *h_vplan, void *stream);
int rsz_verify_graph_create(const rsz_batch_plan *h_plan, const rsz_verify_plan *h_vplan,
                            void *stream, void **h_graph_exec);
int rsz_graph_destroy(void *graph_exec);

/* Parse and check the 80-byte header of a stream held in host memory
 * (h_stream, n >= 80 bytes).  The container is this library's own format (the
 * paper composes its stages through LibPressio, Sec. IV, and fixes no byte
 * layout).  Fills *p, *npeaks and *stream_bytes.
 * Returns RSZ_ERR_CORRUPT for a malformed header.  Host-only. */
int rsz_stream_info(const void *h_stream, uint64_t n, rsz_params *p, uint32_t *npeaks,
                    uint64_t *stream_bytes);

/* Device workspace for rsz_decompress of the stream whose header is given
 * (host copy of at least its first 80 bytes).  Host-only. */
int rsz_decompress_workspace_bytes(const void *h_header, uint64_t n, uint64_t *bytes);

/* Decompress one device-resident stream into d_frame (panels*height*width
 * float32, frame_elems >= that).  Background pixels get their bin value
 * q*2*eb (Sec. VI "binning", bound of Sec. V-C); ROI pixels get their exact
 * bits back (Sec. IV).  Structurally invalid streams give RSZ_ERR_CORRUPT.
 * Synchronous with respect to `stream` (reads the header and the status). */
int rsz_decompress(const void *d_in, uint64_t in_bytes, float *d_frame, uint64_t frame_elems,
                   void *d_ws, uint64_t ws_bytes, void *stream);

/* One stream of a batched decompression.
 *   in/in_bytes: the stream (device).  header: a host copy of its first 80
 *   bytes (the call plans from it without reading device memory).
 *   frame/frame_elems: the output frame (device, panels*height*width float32
 *   at least). */
typedef struct {
  const void *in;
  uint64_t in_bytes;
  const void *header;
  float *frame;
  uint64_t frame_elems;
} rsz_decode_desc;

/* Device workspace for rsz_decompress_batch of these streams.  Host-only. */
int rsz_decompress_batch_workspace_bytes(uint32_t n, const rsz_decode_desc *h_descs,
                                         uint64_t *bytes);

/* Decompress n streams (the decompression of Sec. IV-A, as rsz_decompress)
 * with one launch of each decoder kernel for all of them: a kernel's
 * workgroups are numbered across the streams.  d_status[i] (device) receives
 * stream i's status: RSZ_OK, RSZ_ERR_CORRUPT for a malformed stream (also a
 * header the host rejects), RSZ_ERR_ARG for a frame buffer that is null,
 * misaligned or too small.  Asynchronous: queued on `stream`, no host
 * synchronisation.  Returns RSZ_ERR_ARG for n == 0 or a null pointer,
 * RSZ_ERR_WORKSPACE for a workspace below
 * rsz_decompress_batch_workspace_bytes. */
int rsz_decompress_batch(uint32_t n, const rsz_decode_desc *h_descs, int32_t *d_status,
                         void *d_ws, uint64_t ws_bytes, void *stream);

/* ---- Peak finding: the step before the path, feeding the peak list ---- */

/* Peak-finder parameters (Sec. IV-B: local maxima of a 7x7 window, maxima
 * below 300 ADU rejected, the peak's pixels above 0 ADU, total intensity
 * above 600 ADU, signal to noise above 10, 2 to 30 peak pixels).  A pixel is
 * a peak when:
 *   - it is >= amax_min and the maximum of its (2*rank+1)^2 window clipped to
 *     the panel (ties: the first pixel in raster order wins);
 *   - the background ring, pixels at Chebyshev distance ring_in..ring_out
 *     from it inside the panel, is not empty; mu and sigma are its mean and
 *     population standard deviation;
 *   - its peak pixels, the window pixels 4-connected to it through pixels with
 *     x - mu > pix_nsigma * sigma, number npix_min..npix_max;
 *   - their sum S is > atot_min, and (S - n*mu) / (sigma*sqrt(n)) > snr_min.
 * pix_nsigma reads the paper's "above 0 ADU" as above the background's noise
 * (0 takes it as above the background).  Limits: rank 1..3, rank < ring_in
 * <= ring_out <= 15, npix_min <= npix_max, thresholds finite, snr_min and
 * pix_nsigma >= 0, reserved 0.  rsz_peak_params_default fills the paper's
 * values (rank 3, ring 4..5, 2..30 pixels, 300, 600, 10) and pix_nsigma 3. */
typedef struct {
  uint32_t rank, ring_in, ring_out;
  uint32_t npix_min, npix_max;
  uint32_t reserved;
  double amax_min, atot_min, snr_min, pix_nsigma;
} rsz_peak_params;

void rsz_peak_params_default(rsz_peak_params *q);

/* One frame of a peak-finding batch.  frame: panels x height x width float32
 * (device, 16-byte aligned; shape limits as in rsz_params).  peaks: device
 * array of max_peaks entries (1..8192) that receives the frame's peaks in
 * raster order (panel, row, col). */
typedef struct {
  uint32_t panels, height, width;
  uint32_t max_peaks;
  const float *frame;
  rsz_peak *peaks;
} rsz_peak_desc;

/* Device workspace for rsz_find_peaks_batch.  Host-only. */
int rsz_find_peaks_workspace_bytes(uint32_t nframes, const rsz_peak_desc *h_descs,
                                   uint64_t *bytes);

/* Finds the peaks of nframes frames in one batched launch sequence.
 * d_counts[i] receives the number of peaks of frame i and d_status[i] its
 * status: RSZ_OK, RSZ_ERR_ARG (invalid descriptor) or RSZ_ERR_CAPACITY (more
 * than max_peaks peaks; the count is still reported and the list is
 * unspecified).  Non-hit rejection (Sec. IV: fewer than 10 peaks) is the
 * caller's comparison of d_counts.  Asynchronous like rsz_compress_batch;
 * the return value reports errors of the call itself (ARG, WORKSPACE, HIP). */
int rsz_find_peaks_batch(const rsz_peak_params *q, uint32_t nframes, const rsz_peak_desc *h_descs,
                         uint32_t *d_counts, int32_t *d_status, void *d_ws, uint64_t ws_bytes,
                         void *stream);

/* Intermediates of compressing one frame, for parity checks.  Every pointer
 * is device memory and may be NULL to skip that output.
 *   mask: panels*height*ceil(width/32) u32, bit j%32 of word j/32 = ROI pixel.
 *   S: nbins f64 sums, n: nbins u32 counts, q: nbins i32 quantised bins,
 *   codes: nbins u16, hist: 1024 u32, lens: 1024 u8, cw: 1024 u32 canonical
 *   codewords; n_out: 1 u32, the number of outliers (bins whose Lorenzo
 *   residual lies outside the codes' range, Sec. V-C), out_idx: up to nbins
 *   u32 their bin indices in increasing order, out_res: up to nbins i32 their
 *   residuals.  Bins are ordered (panel, bin row, bin column). */
typedef struct {
  uint32_t *mask;
  double *S;
  uint32_t *n;
  int32_t *q;
  uint16_t *codes;
  uint32_t *hist;
  uint8_t *lens;
  uint32_t *cw;
  uint32_t *n_out;
  uint32_t *out_idx;
  int32_t *out_res;
} rsz_debug_bufs;

/* Runs the compression kernels of one frame up to the codebook and copies the
 * intermediates out.  Same workspace as rsz_compress.  Synchronous. */
int rsz_debug_intermediates(const rsz_params *p, const float *d_frame, const rsz_peak *d_peaks,
                            uint32_t npeaks, const rsz_debug_bufs *bufs, void *d_ws,
                            uint64_t ws_bytes, void *stream);

/* Huffman code lengths and canonical codewords of one 1024-symbol histogram,
 * computed by the kernel of the compression path (the Huffman stage of the
 * SZ compressor, Sec. V-C: two-queue construction over leaves sorted by
 * (count, symbol), a leaf first on equal weights, lengths limited to 32 by
 * halving the counts, canonical codewords in (length, symbol) order).  For
 * parity checks.  h_hist: 1024 counts (host), at least one nonzero, sum below
 * 2^27; h_lens (1024 u8) and h_cw (1024 u32) receive the results (host).
 * d_ws: device workspace of at least 16 KiB, 256-byte aligned.  Synchronous
 * with respect to `stream`. */
int rsz_debug_codebook(const uint32_t *h_hist, uint8_t *h_lens, uint32_t *h_cw, void *d_ws,
                       uint64_t ws_bytes, void *stream);

/* Measurement helper: the rate of a plain streaming read of d_buf on this
 * GPU, the measured reference that the binning kernel's read rate is compared
 * with beside the HBM peak.  d_buf: `bytes` of device memory, 16-byte
 * aligned (bytes / 16 16-byte loads per pass); d_sink: device scratch of at
 * least 4 KiB (normally left untouched); reps passes are timed with HIP events
 * after one untimed pass; *h_gbps receives 10^9 bytes per second.
 * Synchronous with respect to `stream`. */
int rsz_measure_read(const void *d_buf, uint64_t bytes, void *d_sink, int reps, double *h_gbps,
                     void *stream);

/* Kernel timing with HIP events recorded around every launch, on the stream
 * the kernel runs on.  rsz_profile_enable(1) clears and starts recording;
 * rsz_profile_read waits for the recorded events and returns, per kernel
 * name, the number of launches and the summed milliseconds (up to max
 * entries; *n receives the count). */
typedef struct {
  char name[48];
  uint32_t launches;
  double total_ms;
} rsz_kernel_time;

int rsz_profile_enable(int enable);
int rsz_profile_read(rsz_kernel_time *h_out, int max, int *n);
/* Record only the launches of the kernel with this name (NULL or "": every
 * kernel), so that a timed region carries the events of one kernel only. */
int rsz_profile_only(const char *name);

#ifdef __cplusplus
}
#endif

#endif /* RSZ_H */
