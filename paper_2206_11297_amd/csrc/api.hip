// api.hip -- host side of librsz: argument checks, batch planning, workspace
// layout, the exported C ABI, and kernel timing.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "rsz_internal.h"

namespace rsz {

// ----------------------------------------------------------------- timing

namespace {
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::string g_prof_only;   // record only this kernel's launches (empty: all)
std::vector<ProfRec> g_prof;
thread_local ProfRec *g_open = nullptr;
}  // namespace

void prof_begin(const char *name, hipStream_t s) {
  if (!g_prof_on) return;
  g_open = nullptr;
  if (!g_prof_only.empty() && g_prof_only != name) return;
  ProfRec r;
  r.name = name;
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
  (void)hipEventRecord(r.a, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.push_back(r);
  g_open = &g_prof.back();
}

void prof_end(hipStream_t s) {
  if (!g_prof_on) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (g_open) (void)hipEventRecord(g_open->b, s);
  g_open = nullptr;
}

// --------------------------------------------------------------- planning

static uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

static int check_params(const rsz_params *p, uint32_t npeaks) {
  if (!p) return RSZ_ERR_ARG;
  if (p->panels < 1 || p->panels > 65535 || p->height < 1 || p->height > 65535 ||
      p->width < 1 || p->width > 65535)
    return RSZ_ERR_ARG;
  if (p->window < 1 || p->window > 1023 || p->bin < 1 || p->bin > 8 || p->bin_mode > 1 ||
      p->dim > 3 || p->roi_coding > 1 || p->run_coding > 1 || p->reserved != 0)
    return RSZ_ERR_ARG;
  if (!(p->eb > 0.0) || !std::isfinite(p->eb)) return RSZ_ERR_ARG;
  const uint64_t pix = (uint64_t)p->panels * p->height * p->width;
  const uint64_t nb = (uint64_t)p->panels * div_up(p->height, p->bin) * div_up(p->width, p->bin);
  // (bins < 2^27 keeps the bitstream's and the run section's bits below 2^32)
  if (pix >= (1ull << 31) || nb >= (1ull << 27)) return RSZ_ERR_ARG;
  if ((uint64_t)npeaks * p->window * p->window > (1ull << 28)) return RSZ_ERR_ARG;
  // coded ROI bits (at most 63 per value) must fit u32 offsets
  if (p->roi_coding && (uint64_t)npeaks * p->window * p->window > (1ull << 26))
    return RSZ_ERR_ARG;
  return RSZ_OK;
}

struct Geom {
  uint32_t Hb, Wb, nbins, nchunks, TH, segs, groups, nstrips, gstrips, cgs;
  uint64_t off_roi, off_lens, off_chunks, off_bits;
  uint64_t max_bytes;
};

// Binning tiles: column groups of at most `gs` strips (the kernel's compiled
// width for this batch) and segments of at most kMaxTH bin rows whose LDS
// mask, (TH+1)*b raw rows of wpr words, fits kMaskWords; segments are
// balanced in groups of wpg (waves per workgroup).
static Geom geometry(const rsz_params *p, uint32_t npeaks, uint32_t th_cap, uint32_t gs,
                     uint32_t wpg = kWaves) {
  Geom g;
  g.Hb = (uint32_t)div_up(p->height, p->bin);
  g.Wb = (uint32_t)div_up(p->width, p->bin);
  g.nbins = p->panels * g.Hb * g.Wb;
  g.nchunks = (uint32_t)div_up(g.nbins, kChunk);
  g.nstrips = (uint32_t)div_up(g.Wb, 64);
  g.gstrips = std::max<uint32_t>(1, std::min(gs, g.nstrips));
  g.cgs = (uint32_t)div_up(g.nstrips, g.gstrips);
  // one extra word left of a group for its halo column
  const uint32_t wpr = 2 * p->bin * g.gstrips + (g.cgs > 1 ? 1 : 0);
  uint32_t thmax = (uint32_t)kMaskWords / (p->bin * wpr);
  thmax = thmax > 1 ? thmax - 1 : 1;
  thmax = std::max<uint32_t>(1, std::min({thmax, (uint32_t)kMaxTH, th_cap}));
  const uint32_t nseg = wpg * (uint32_t)div_up(g.Hb, (uint64_t)wpg * thmax);
  g.TH = (uint32_t)div_up(g.Hb, nseg);
  g.segs = (uint32_t)div_up(g.Hb, g.TH);
  g.groups = (uint32_t)div_up(g.segs, wpg);
  g.off_roi = kHeader + align_up(6ull * npeaks, 4);
  const uint64_t nroi = (uint64_t)npeaks * p->window * p->window;
  g.off_lens = g.off_roi + (p->roi_coding ? 0 : 4ull * nroi);
  g.off_chunks = g.off_lens + kNumSym;
  g.off_bits = g.off_chunks + 4ull * g.nchunks;
  // worst case: every codeword 32 bits and every bin an outlier (and every
  // coded ROI value 63 bits; the run section codes at most the bitstream's
  // bits, plus its parameters and offsets)
  g.max_bytes = g.off_bits + 4ull * g.nbins + 8ull * g.nbins +
                (p->roi_coding ? kRoiLens + 4ull * npeaks + 4 * div_up(63 * nroi, 32) : 0) +
                (p->run_coding ? align_up(g.nchunks, 4) + 4ull * (g.nchunks + 1) : 0);
  return g;
}

struct Layout {
  // plans and prefixes are copied from the host; the frame tables after
  // them are written by k_prep
  uint64_t plans, prefix, tables, tile_frame, unit_frame, peak_frame, states, frames_begin, total;
  std::vector<uint64_t> frame_off;  // per frame start of its private region
};

// Bytes of one binning tile's region of sparse code bytes: room for every
// bin of the tile, in whole 128-byte lines.
static uint32_t tile_cap(const Geom &g) {
  return (uint32_t)align_up(64ull * g.TH * g.gstrips, 128);
}

static uint64_t frame_region_bytes(const rsz_params *p, uint32_t npeaks, const Geom &g) {
  uint64_t b = 0;
  b += align_up(4ull * ((uint64_t)p->panels * g.segs + 1), 256);  // bstart
  b += align_up(4ull * npeaks, 256);                              // bucket
  // code bytes (dense, then the chunk form), whole chunks and 32 bytes past the
  // last; the chunk form's masks
  b += align_up(1ull * kChunk * g.nchunks + 32, 256) + align_up(512ull * g.nchunks, 256) +
       align_up(256ull * g.nchunks, 256);   // and the lanes' bit and outlier counts
  if (p->dim != 3) {   // sparse codes: zero-map words, counts, bytes per binning tile
    const uint64_t nt = (uint64_t)p->panels * g.cgs * g.segs, ne = nt * kTileEntries;
    b += align_up(8ull * ne, 256) + align_up(2ull * ne, 256) + align_up(nt * tile_cap(g), 256);
  }
  b += align_up(4ull * g.nbins, 256);          // rbuf
  b += align_up(4ull * g.nbins, 256);          // obuf
  b += 3 * align_up(4ull * g.nchunks, 256);    // chunk_off, chunk_oo, head
  if (p->dim == 1) b += align_up(4ull * p->panels * g.Hb, 256);   // qedge
  if (p->dim == 3)   // 2D code bytes and residuals
    b += align_up(1ull * kChunk * g.nchunks, 256) + align_up(4ull * g.nbins, 256);
  if (p->roi_coding)   // class histogram, lengths, codewords, window bits
    b += 4 * kNumSym + kNumSym + 4 * kNumSym + align_up(4ull * npeaks, 256);
  if (p->run_coding)   // Huffman words, chunk run bits then offsets, parameters
    b += align_up(4ull * (g.nbins + 2), 256) + align_up(4ull * (g.nchunks + 1), 256) +
         align_up(g.nchunks, 256);
  return b;
}

// Chunks per encode workgroup (its waves take every kWaves-th chunk): a
// multiple of kWaves, about 8192 workgroups for large batches (a workgroup
// first copies the code tables to LDS; one chunk per wave measured slower).
static uint32_t encode_cpw(uint64_t all_chunks) {
  return kWaves * (uint32_t)std::min<uint64_t>(8, std::max<uint64_t>(1, all_chunks / (8192 * kWaves)));
}

static Layout layout(uint32_t nframes, const std::vector<const rsz_params *> &ps,
                     const std::vector<uint32_t> &np, const std::vector<Geom> &gs,
                     const std::vector<int> &valid) {
  Layout L;
  L.plans = 0;
  L.prefix = align_up(sizeof(FramePlan) * nframes, 256);
  // the frame tables: (frame, chunk) of each k_count workgroup's first
  // chunk, the frame of each k_bin and k_encode workgroup and of each peak
  uint64_t chunks = 0, tiles = 0, units = 0, peaks = 0;
  for (uint32_t f = 0; f < nframes; ++f)
    if (valid[f]) chunks += gs[f].nchunks;
  const uint32_t cpw = encode_cpw(chunks);
  for (uint32_t f = 0; f < nframes; ++f)
    if (valid[f]) {
      tiles += (uint64_t)ps[f]->panels * gs[f].cgs * gs[f].groups;
      units += div_up(gs[f].nchunks, cpw);
      peaks += np[f];
    }
  L.tables = L.prefix + align_up(5 * 4ull * (nframes + 1), 256);
  L.tile_frame = L.tables + align_up(8 * div_up(chunks, kWaves) + 8, 256);
  L.unit_frame = L.tile_frame + align_up(4 * tiles + 4, 256);
  L.peak_frame = L.unit_frame + align_up(4 * units + 4, 256);
  L.states = L.peak_frame + align_up(4 * peaks + 4, 256);
  L.frames_begin = L.states + align_up(sizeof(FrameState) * nframes, 256);
  uint64_t off = L.frames_begin;
  L.frame_off.resize(nframes);
  for (uint32_t f = 0; f < nframes; ++f) {
    L.frame_off[f] = off;
    if (valid[f]) off += frame_region_bytes(ps[f], np[f], gs[f]);
  }
  L.total = off;
  return L;
}

// Host image of the plan, copied to the head of the workspace.
struct HostPlan {
  std::vector<uint8_t> bytes;
  BatchPlan bp;
  uint32_t common_b;    // bin factor of every valid frame, or 0 when they differ
  uint32_t common_dim;  // Lorenzo dimension of every valid frame, or 0
};

static int build_plan(uint32_t nframes, const rsz_frame_desc *d, uint64_t *res_bytes,
                      int32_t *res_status, uint8_t *ws, uint64_t ws_bytes, uint32_t th_cap,
                      HostPlan &hp, uint64_t *need, const rsz_debug_bufs *dbg) {
  std::vector<const rsz_params *> ps(nframes);
  std::vector<uint32_t> np(nframes);
  std::vector<Geom> gs(nframes);
  std::vector<int> valid(nframes);
  for (uint32_t f = 0; f < nframes; ++f) {
    ps[f] = &d[f].params;
    np[f] = d[f].npeaks;
    valid[f] = check_params(ps[f], np[f]) == RSZ_OK && d[f].frame && d[f].out &&
               (np[f] == 0 || d[f].peaks) && ((uintptr_t)d[f].frame % 16 == 0) &&
               ((uintptr_t)d[f].out % 16 == 0);
  }
  // the binning kernel is compiled for the common bin factor of the batch
  hp.common_b = 0;
  hp.common_dim = 2;
  bool first = true;
  for (uint32_t f = 0; f < nframes; ++f) {
    if (!valid[f]) continue;
    const uint32_t dim = ps[f]->dim ? ps[f]->dim : 2u;
    if (first) {
      hp.common_b = ps[f]->bin;
      hp.common_dim = dim;
    } else {
      if (hp.common_b != ps[f]->bin) hp.common_b = 0;
      if (hp.common_dim != dim) hp.common_dim = 0;
    }
    first = false;
  }
  const uint32_t gsw = (uint32_t)group_strips((int)hp.common_b);
  // waves per binning workgroup: the first valid frame's tile_waves
  uint32_t wpg = kWaves;
  for (uint32_t f = 0; f < nframes; ++f)
    if (valid[f]) {
      if (d[f].tile_waves) wpg = std::min<uint32_t>(d[f].tile_waves, kWaves);
      break;
    }
  // tile shape of each frame: the caller's tile_rows / tile_strips, else the
  // coarsest shape of the ladder below that gives the batch kTargetWaves
  // binning waves, down to 8-row single-strip tiles (shorter tiles re-read
  // too many halo rows; measured on MI355X across 1..1000-frame batches)
  static const uint32_t ladder[][2] = {{kMaxTH, 0}, {16, 0}, {8, 0}, {8, 1}};
  auto shape_of = [&](uint32_t f, uint32_t rung, uint32_t &rows, uint32_t &strips) {
    rows = d[f].tile_rows ? d[f].tile_rows : (th_cap ? th_cap : ladder[rung][0]);
    const uint32_t sd = th_cap ? 0 : ladder[rung][1];
    strips = d[f].tile_strips ? std::min(d[f].tile_strips, gsw) : (sd ? std::min(sd, gsw) : gsw);
  };
  uint32_t rung = 0;
  for (; rung + 1 < sizeof ladder / sizeof ladder[0]; ++rung) {
    uint64_t waves = 0;
    for (uint32_t f = 0; f < nframes; ++f) {
      if (!valid[f]) continue;
      uint32_t rows, strips;
      shape_of(f, rung, rows, strips);
      const Geom g = geometry(ps[f], np[f], rows, strips, wpg);
      waves += (uint64_t)ps[f]->panels * g.cgs * g.groups * wpg;
    }
    if (waves >= kTargetWaves) break;
  }
  for (uint32_t f = 0; f < nframes; ++f)
    if (valid[f]) {
      uint32_t rows, strips;
      shape_of(f, rung, rows, strips);
      gs[f] = geometry(ps[f], np[f], rows, strips, wpg);
    }
  Layout L = layout(nframes, ps, np, gs, valid);
  if (need) *need = L.total;
  if (!ws) return RSZ_OK;
  if (ws_bytes < L.total) return RSZ_ERR_WORKSPACE;
  hp.bytes.assign(L.tables, 0);
  memset(&hp.bp, 0, sizeof hp.bp);
  FramePlan *fpl = (FramePlan *)hp.bytes.data();
  uint32_t *tp = (uint32_t *)(hp.bytes.data() + L.prefix);
  uint32_t *cp = tp + (nframes + 1);
  uint32_t *rp = cp + (nframes + 1);
  uint32_t *kp = rp + (nframes + 1);
  uint32_t *xp = kp + (nframes + 1);
  uint64_t tiles = 0, units = 0, npk_total = 0, chunks_done = 0, fixes = 0;
  bool all_vec = true;
  uint64_t all_chunks = 0;
  for (uint32_t f = 0; f < nframes; ++f)
    if (valid[f]) all_chunks += gs[f].nchunks;
  const uint32_t cpw = encode_cpw(all_chunks);
  for (uint32_t f = 0; f < nframes; ++f) {
    FramePlan &fp = fpl[f];
    memset(&fp, 0, sizeof fp);
    tp[f] = (uint32_t)tiles;
    cp[f] = (uint32_t)units;
    rp[f] = (uint32_t)npk_total;
    kp[f] = (uint32_t)chunks_done;
    xp[f] = (uint32_t)fixes;
    fp.st = (FrameState *)(ws + L.states) + f;
    fp.res_bytes = res_bytes + f;
    fp.res_status = res_status + f;
    if (!valid[f]) {
      fp.init_status = RSZ_ERR_ARG;
      continue;
    }
    const rsz_params *p = ps[f];
    const Geom &g = gs[f];
    fp.P = p->panels;
    fp.H = p->height;
    fp.W = p->width;
    fp.w = p->window;
    fp.b = p->bin;
    fp.mode = p->bin_mode;
    fp.dim = p->dim ? p->dim : 2u;
    fp.roi_coding = p->roi_coding;
    fp.eb = p->eb;
    fp.step = 2.0 * p->eb;
    fp.Hb = g.Hb;
    fp.Wb = g.Wb;
    fp.nbins = g.nbins;
    fp.nchunks = g.nchunks;
    fp.npeaks = np[f];
    fp.TH = g.TH;
    fp.segs = g.segs;
    fp.groups = g.groups;
    fp.nstrips = g.nstrips;
    fp.gstrips = g.gstrips;
    fp.cgs = g.cgs;
    fp.init_status = RSZ_OK;
    fp.vec = (p->bin == 2 || p->bin == 4) && p->width % p->bin == 0 &&
             (uintptr_t)d[f].frame % (4 * p->bin) == 0;
    all_vec = all_vec && fp.vec;
    fp.frame = d[f].frame;
    fp.peaks = (const int32_t *)d[f].peaks;
    fp.out = (uint8_t *)d[f].out;
    fp.out_cap = d[f].out_cap;
    fp.off_roi = g.off_roi;
    fp.off_lens = g.off_lens;
    fp.off_chunks = g.off_chunks;
    fp.off_bits = g.off_bits;
    uint8_t *base = ws + L.frame_off[f];
    fp.bstart = (uint32_t *)base;
    base += align_up(4ull * ((uint64_t)p->panels * g.segs + 1), 256);
    fp.bucket = (uint32_t *)base;
    base += align_up(4ull * np[f], 256);
    fp.sparse = fp.dim != 3;
    if (fp.sparse) {
      const uint64_t nt = (uint64_t)p->panels * g.cgs * g.segs, ne = nt * kTileEntries;
      fp.tile_cap = tile_cap(g);
      fp.fd_Wb = fast_div(g.Wb);
      fp.fd_Hb = fast_div(g.Hb);
      fp.fd_TH = fast_div(g.TH);
      fp.fd_gs = fast_div(g.gstrips);
      fp.zm = (uint64_t *)base;
      base += align_up(8ull * ne, 256);
      fp.zp = (uint16_t *)base;
      base += align_up(2ull * ne, 256);
      fp.zb = base;
      base += align_up(nt * fp.tile_cap, 256);
    }
    fp.codes = base;
    base += align_up(1ull * kChunk * g.nchunks + 32, 256);
    fp.cmask = (uint64_t *)base;
    base += align_up(512ull * g.nchunks, 256);
    fp.lanecnt = (uint32_t *)base;
    base += align_up(256ull * g.nchunks, 256);
    fp.rbuf = (int32_t *)base;
    base += align_up(4ull * g.nbins, 256);
    fp.obuf = (uint32_t *)base;
    base += align_up(4ull * g.nbins, 256);
    fp.chunk_off = (uint32_t *)base;
    base += align_up(4ull * g.nchunks, 256);
    fp.chunk_oo = (uint32_t *)base;
    base += align_up(4ull * g.nchunks, 256);
    fp.head = (uint32_t *)base;
    base += align_up(4ull * g.nchunks, 256);
    fp.codes2 = fp.codes;
    fp.rbuf2 = fp.rbuf;
    if (fp.dim == 1) {
      fp.qedge = (int32_t *)base;
      base += align_up(4ull * p->panels * g.Hb, 256);
    }
    if (fp.dim == 3) {
      fp.codes2 = base;
      base += align_up(1ull * kChunk * g.nchunks, 256);
      fp.rbuf2 = (int32_t *)base;
      base += align_up(4ull * g.nbins, 256);
    }
    if (fp.roi_coding) {
      fp.roi_hist = (uint32_t *)base;
      base += 4 * kNumSym;
      fp.roi_cw = (uint32_t *)base;
      base += 4 * kNumSym;
      fp.roi_lens = base;
      base += kNumSym;
      fp.roi_bits = (uint32_t *)base;
      base += align_up(4ull * np[f], 256);
      hp.bp.roi_coding = 1;
    }
    // the bitstream's words: in the stream, or in the workspace when the run
    // stage codes them
    fp.run_coding = p->run_coding;
    fp.bw = (uint32_t *)(fp.out + g.off_bits);
    fp.bw_cap = fp.out_cap >= g.off_bits ? (fp.out_cap - g.off_bits) / 4 : 0;
    if (fp.run_coding) {
      fp.bw = (uint32_t *)base;
      fp.bw_cap = g.nbins + 2;   // T <= 32 * nbins
      base += align_up(4ull * (g.nbins + 2), 256);
      fp.run_off = (uint32_t *)base;
      base += align_up(4ull * (g.nchunks + 1), 256);
      fp.run_k = base;
      base += align_up(g.nchunks, 256);
      hp.bp.run_coding = 1;
    }
    if (dbg) {
      fp.dbg_mask = dbg->mask;
      fp.dbg_S = dbg->S;
      fp.dbg_n = dbg->n;
      fp.dbg_q = dbg->q;
    }
    tiles += (uint64_t)p->panels * g.cgs * g.groups;
    units += div_up(g.nchunks, cpw);
    chunks_done += g.nchunks;
    npk_total += np[f];
    // k_lorenzo_dims: 256 bin rows to correct (dim 1: the first row of each
    // panel, or every row when a panel row spans column groups) or kFixBins3
    // bins (dim 3) per workgroup
    if (fp.dim == 1) fixes += div_up((uint64_t)p->panels * (g.cgs == 1 ? 1 : g.Hb), 256);
    else if (fp.dim == 3) fixes += div_up(g.nbins, kFixBins3);
  }
  if (tiles >= (1ull << 31) || units >= (1ull << 31) || npk_total >= (1ull << 31) ||
      chunks_done >= (1ull << 31) || fixes >= (1ull << 31))
    return RSZ_ERR_ARG;
  tp[nframes] = (uint32_t)tiles;
  cp[nframes] = (uint32_t)units;
  rp[nframes] = (uint32_t)npk_total;
  kp[nframes] = (uint32_t)chunks_done;
  xp[nframes] = (uint32_t)fixes;
  hp.bp.nframes = nframes;
  hp.bp.total_chunks = (uint32_t)chunks_done;
  hp.bp.total_tiles = (uint32_t)tiles;
  hp.bp.total_units = (uint32_t)units;
  hp.bp.total_peaks = (uint32_t)npk_total;
  hp.bp.cpw = cpw;
  hp.bp.all_vec = all_vec ? 1u : 0u;
  hp.bp.bin_waves = wpg;
  hp.bp.frames = (const FramePlan *)(ws + L.plans);
  hp.bp.tile_prefix = (const uint32_t *)(ws + L.prefix);
  hp.bp.unit_prefix = hp.bp.tile_prefix + (nframes + 1);
  hp.bp.peak_prefix = hp.bp.unit_prefix + (nframes + 1);
  hp.bp.chunk_prefix = hp.bp.peak_prefix + (nframes + 1);
  hp.bp.fix_prefix = hp.bp.chunk_prefix + (nframes + 1);
  hp.bp.total_fix = (uint32_t)fixes;
  hp.bp.count_frame = (uint2 *)(ws + L.tables);
  hp.bp.tile_frame = (uint32_t *)(ws + L.tile_frame);
  hp.bp.unit_frame = (uint32_t *)(ws + L.unit_frame);
  hp.bp.peak_frame = (uint32_t *)(ws + L.peak_frame);
  bool all_sparse = true;
  for (uint32_t f = 0; f < nframes; ++f)
    if (valid[f] && fpl[f].dim == 3) all_sparse = false;
  hp.bp.all_sparse = all_sparse ? 1u : 0u;
  return RSZ_OK;
}


// Plans reach the device through a ring of pinned host buffers: a slot is
// reused only after the event recorded behind its previous copy has fired, so
// an asynchronous call never reads host memory that has been overwritten.
namespace {
struct StageSlot {
  void *ptr = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
};
std::mutex g_stage_mu;
StageSlot g_stage[8];
unsigned g_stage_next = 0;
}  // namespace

static int stage_to_device(void *dst, const void *src, size_t n, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  StageSlot &sl = g_stage[g_stage_next++ % 8];
  if (sl.ev && hipEventSynchronize(sl.ev) != hipSuccess) return RSZ_ERR_HIP;
  if (sl.cap < n) {
    if (sl.ptr) (void)hipHostFree(sl.ptr);
    sl.ptr = nullptr;
    sl.cap = 0;
    const size_t cap = std::max<size_t>(align_up(n, 1 << 16), 1 << 16);
    if (hipHostMalloc(&sl.ptr, cap, hipHostMallocDefault) != hipSuccess) return RSZ_ERR_HIP;
    sl.cap = cap;
  }
  memcpy(sl.ptr, src, n);
  if (hipMemcpyAsync(dst, sl.ptr, n, hipMemcpyHostToDevice, s) != hipSuccess) return RSZ_ERR_HIP;
  if (!sl.ev && hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess)
    return RSZ_ERR_HIP;
  if (hipEventRecord(sl.ev, s) != hipSuccess) return RSZ_ERR_HIP;
  return RSZ_OK;
}

// Host record of a prepared batch (the public rsz_batch_plan is its storage).
struct PlanRecord {
  BatchPlan bp;
  uint32_t common_b;
  uint32_t common_dim;
};
static_assert(sizeof(PlanRecord) <= sizeof(rsz_batch_plan), "plan record too large");

// Queue the whole path for a batch; results land in res_bytes/res_status.
static int enqueue(uint32_t nframes, const rsz_frame_desc *d, uint64_t *res_bytes,
                   int32_t *res_status, void *ws, uint64_t ws_bytes, hipStream_t s,
                   const rsz_debug_bufs *dbg, bool front_only, HostPlan &hp,
                   bool direct_copy = false) {
  const int st = build_plan(nframes, d, res_bytes, res_status, (uint8_t *)ws, ws_bytes,
                            0, hp, nullptr, dbg);
  if (st) return st;
  // direct_copy: the plan goes straight from hp (which the caller keeps
  // until the stream has finished) instead of through the pinned staging
  // slots, which may grow
  if (direct_copy ? hipMemcpyAsync(ws, hp.bytes.data(), hp.bytes.size(), hipMemcpyHostToDevice,
                                   s) != hipSuccess
                  : stage_to_device(ws, hp.bytes.data(), hp.bytes.size(), s) != RSZ_OK)
    return RSZ_ERR_HIP;
  if (launch_compress_front_b(hp.bp, hp.common_b, hp.common_dim, s, dbg != nullptr) !=
      hipSuccess)
    return RSZ_ERR_HIP;
  if (!front_only && launch_compress_back(hp.bp, s) != hipSuccess) return RSZ_ERR_HIP;
  return RSZ_OK;
}

uint64_t decode_tables_bytes();

// Host parse of a stream header; fills the decode plan geometry.
static int parse_header(const uint8_t *h, uint64_t n, uint64_t in_bytes, rsz_params *p,
                        uint32_t *npeaks, DecodePlan *dp) {
  if (!h || n < kHeader) return RSZ_ERR_CORRUPT;
  uint32_t u[20];
  memcpy(u, h, 80);
  if (memcmp(h, "RSZ1", 4) != 0 || (u[1] & 0xFFFFu) != 1u) return RSZ_ERR_CORRUPT;
  rsz_params q;
  memset(&q, 0, sizeof q);
  // flags: bit 0 bin_mode, bits 1-2 the Lorenzo dimension (0 for 2, else 1
  // or 3), bit 3 the ROI coded, bit 4 the runs coded; every other bit zero
  const uint32_t flags = u[1] >> 16, dcode = (flags >> 1) & 3u;
  if ((flags >> 5) != 0 || dcode == 2) return RSZ_ERR_CORRUPT;
  q.bin_mode = flags & 1u;
  q.dim = dcode == 0 ? 2u : dcode;
  q.roi_coding = (flags >> 3) & 1u;
  q.run_coding = (flags >> 4) & 1u;
  q.panels = u[2];
  q.height = u[3];
  q.width = u[4];
  q.window = u[5];
  q.bin = u[6];
  memcpy(&q.eb, h + 32, 8);
  const uint32_t np = u[10];
  if (check_params(&q, np) != RSZ_OK) return RSZ_ERR_CORRUPT;
  uint64_t T, total, Troi;   // Troi: coded ROI bits, 0 with the payload verbatim
  memcpy(&T, h + 56, 8);
  memcpy(&total, h + 64, 8);
  memcpy(&Troi, h + 72, 8);
  if (u[7] != (uint32_t)kRadius || u[12] != kChunk || (!q.roi_coding && Troi != 0) ||
      Troi > 63ull * np * q.window * q.window)
    return RSZ_ERR_CORRUPT;
  const Geom g = geometry(&q, np, kMaxTH, 1);
  const uint64_t n_out = u[11];
  if (u[13] != g.nchunks || n_out > g.nbins || T > 32ull * g.nbins) return RSZ_ERR_CORRUPT;
  const uint64_t off_oidx = g.off_bits + (q.run_coding ? 0 : 4 * ((T + 31) / 32));
  const uint64_t off_ores = off_oidx + 4 * n_out;
  const uint64_t off_rsec = off_ores + 4 * n_out;
  const uint64_t off_rbits = off_rsec + kRoiLens + 4ull * np;
  const uint64_t end = q.roi_coding ? off_rbits + 4 * ((Troi + 31) / 32) : off_rsec;
  // run section: its size comes from its last offset, checked on the device;
  // the total must leave room for the offsets and end on a whole word
  const uint64_t off_runoffs = end + align_up(g.nchunks, 4);
  const uint64_t off_runbits = off_runoffs + 4ull * (g.nchunks + 1);
  if (q.run_coding ? (total < off_runbits || (total - off_runbits) % 4 != 0) : end != total)
    return RSZ_ERR_CORRUPT;
  if (total > in_bytes) return RSZ_ERR_CORRUPT;
  if (p) *p = q;
  if (npeaks) *npeaks = np;
  if (dp) {
    memset(dp, 0, sizeof *dp);
    dp->P = q.panels;
    dp->H = q.height;
    dp->W = q.width;
    dp->w = q.window;
    dp->b = q.bin;
    dp->npeaks = np;
    dp->dim = q.dim;
    dp->roi_coding = q.roi_coding;
    dp->Troi = Troi;
    dp->off_rsec = off_rsec;
    dp->off_roffs = off_rsec + kRoiLens;
    dp->off_rbits = off_rbits;
    dp->step = 2.0 * q.eb;
    dp->Hb = g.Hb;
    dp->Wb = g.Wb;
    dp->nbins = g.nbins;
    dp->nchunks = g.nchunks;
    dp->n_out = (uint32_t)n_out;
    dp->T = T;
    dp->total = total;
    dp->off_peaks = kHeader;
    dp->off_roi = g.off_roi;
    dp->off_lens = g.off_lens;
    dp->off_chunks = g.off_chunks;
    dp->off_bits = g.off_bits;
    dp->off_oidx = off_oidx;
    dp->off_ores = off_ores;
    dp->run_coding = q.run_coding;
    dp->off_run = end;
    dp->off_runoffs = off_runoffs;
    dp->off_runbits = off_runbits;
  }
  return RSZ_OK;
}

uint64_t decode_roi_tables_bytes();

static uint64_t decode_ws_bytes(const DecodePlan &dp) {
  return align_up(4ull * dp.nbins, 256) + align_up(dp.nbins + 64ull, 256) +
         align_up(4ull * dp.nchunks, 256) + 256 +
         align_up(decode_tables_bytes(), 256) +
         (dp.dim == 1 ? align_up(4ull * dp.P * dp.Hb, 256) : 0) +
         (dp.roi_coding ? align_up(4ull * dp.npeaks * dp.w * dp.w, 256) +
                              align_up(decode_roi_tables_bytes(), 256)
                        : 0) +
         (dp.run_coding ? align_up(4 * ((dp.T + 31) / 32 + 2), 256) : 0);
}

// Results of a single-frame call live in the workspace tail.
static uint64_t single_extra() { return 256; }

// Decoder workspace: the plans and the per-kernel workgroup prefixes of the n
// streams, then each valid stream's region (decode_ws_bytes).
static uint64_t decode_head_bytes(uint32_t n) {
  return align_up((uint64_t)sizeof(DecodePlan) * n, 256) +
         align_up(4ull * kDecKernels * (n + 1), 256);
}

// One stream to decode: its device bytes, a host copy of its header, the
// output frame and where its status goes (device).
struct DecodeItem {
  const void *in;
  uint64_t in_bytes;
  const uint8_t *header;
  float *frame;
  uint64_t frame_elems;
  int32_t *status;   // null: the status word of the stream's region
};

// Plans the streams (a stream the host rejects gets RSZ_ERR_CORRUPT or
// RSZ_ERR_ARG as its status and no other work), and with a workspace lays
// out the regions, uploads the plans and launches the decoder.  *need: the
// workspace bytes.
static int decode_streams(uint32_t n, const DecodeItem *it, uint8_t *ws, uint64_t ws_bytes,
                          hipStream_t s, uint64_t *need, int32_t **status_words) {
  const uint64_t head = decode_head_bytes(n);
  std::vector<DecodePlan> dps(n);
  std::vector<uint64_t> region(n, 0);
  uint64_t total = head;
  for (uint32_t f = 0; f < n; ++f) {
    DecodePlan &dp = dps[f];
    int st = parse_header(it[f].header, kHeader, it[f].in_bytes, nullptr, nullptr, &dp);
    if (st == RSZ_OK) {
      if (!it[f].in || (uintptr_t)it[f].in % 16 || !it[f].frame || (uintptr_t)it[f].frame % 16 ||
          it[f].frame_elems < (uint64_t)dp.P * dp.H * dp.W)
        st = RSZ_ERR_ARG;
    }
    if (st != RSZ_OK) {
      memset(&dp, 0, sizeof dp);
      dp.init_status = st;
      continue;
    }
    dp.init_status = RSZ_OK;
    region[f] = decode_ws_bytes(dp);
    total += region[f];
  }
  if (need) *need = total;
  if (!ws) return RSZ_OK;
  if (ws_bytes < total) return RSZ_ERR_WORKSPACE;
  // regions
  uint64_t off = head;
  for (uint32_t f = 0; f < n; ++f) {
    DecodePlan &dp = dps[f];
    uint8_t *w = ws + off;
    off += region[f];
    if (dp.init_status == RSZ_OK) {
      dp.in = (const uint8_t *)it[f].in;
      dp.frame = it[f].frame;
      dp.res = (int32_t *)w;
      w += align_up(4ull * dp.nbins, 256);
      dp.res8 = w;
      w += align_up(dp.nbins + 64ull, 256);
      dp.zcount = (uint32_t *)w;
      w += align_up(4ull * dp.nchunks, 256);
      dp.status = (int32_t *)w;
      w += 256;
      dp.tables = (uint32_t *)w;
      w += align_up(decode_tables_bytes(), 256);
      if (dp.dim == 1) {
        dp.carry = (uint32_t *)w;
        w += align_up(4ull * dp.P * dp.Hb, 256);
      }
      if (dp.roi_coding) {
        dp.roi_payload = (uint32_t *)w;
        w += align_up(4ull * dp.npeaks * dp.w * dp.w, 256);
        dp.roi_tables = (uint32_t *)w;
        w += align_up(decode_roi_tables_bytes(), 256);
      }
      // the Huffman words: in the stream, or expanded from the run section
      dp.bits = (const uint32_t *)(dp.in + dp.off_bits);
      if (dp.run_coding) {
        dp.hbits = (uint32_t *)w;
        dp.bits = dp.hbits;
      }
    }
    if (it[f].status) dp.status = it[f].status;
    if (!dp.status) return RSZ_ERR_ARG;   // a rejected stream needs a status word
    if (status_words) status_words[f] = dp.status;
  }
  // plans and prefixes, one upload
  std::vector<uint8_t> host(head, 0);
  memcpy(host.data(), dps.data(), sizeof(DecodePlan) * n);
  uint32_t *pre = (uint32_t *)(host.data() + align_up((uint64_t)sizeof(DecodePlan) * n, 256));
  uint32_t total_blocks[kDecKernels] = {0};
  for (uint32_t f = 0; f < n; ++f) {
    uint32_t nb[kDecKernels];
    decode_blocks(dps[f], nb);
    for (int k = 0; k < kDecKernels; ++k) {
      pre[(size_t)k * (n + 1) + f] = total_blocks[k];
      if ((uint64_t)total_blocks[k] + nb[k] > 0x7FFFFFFFull) return RSZ_ERR_ARG;
      total_blocks[k] += nb[k];
    }
  }
  for (int k = 0; k < kDecKernels; ++k) pre[(size_t)k * (n + 1) + n] = total_blocks[k];
  const int st = stage_to_device(ws, host.data(), head, s);
  if (st) return st;
  DecBatch db;
  db.n = n;
  db.plans = (const DecodePlan *)ws;
  db.pre = (const uint32_t *)(ws + align_up((uint64_t)sizeof(DecodePlan) * n, 256));
  if (launch_decompress(db, total_blocks, s) != hipSuccess) return RSZ_ERR_HIP;
  return RSZ_OK;
}

}  // namespace rsz

using namespace rsz;

// The workspace of rsz_compress_noalloc: one array per GPU, in the code
// object, so that the call allocates nothing.  Host code never passes the
// array's name to a kernel or a copy (on the host it is only a stand-in);
// it uses the device address that hipGetSymbolAddress returns for the
// current GPU, looked up once per device.
static __device__ __align__(256) uint8_t scratch[RSZ_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_init_mu;
std::mutex g_scratch_mu[kMaxDevices];
void *g_scratch_ptr[kMaxDevices];
}  // namespace

// The current GPU's address of `scratch` (dev is the current device).
static int scratch_address(int dev, void **ptr) {
  std::lock_guard<std::mutex> lk(g_scratch_init_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RSZ_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return RSZ_OK;
}

extern "C" {

const char *rsz_status_string(int s) {
  switch (s) {
    case RSZ_OK: return "ok";
    case RSZ_ERR_ARG: return "invalid argument";
    case RSZ_ERR_PEAK: return "peak outside the frame";
    case RSZ_ERR_RANGE: return "background value out of range";
    case RSZ_ERR_CAPACITY: return "output buffer too small";
    case RSZ_ERR_CORRUPT: return "corrupt stream";
    case RSZ_ERR_WORKSPACE: return "workspace too small";
    case RSZ_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

int rsz_max_compressed_bytes(const rsz_params *p, uint32_t npeaks, uint64_t *bytes) {
  const int st = check_params(p, npeaks);
  if (st) return st;
  if (!bytes) return RSZ_ERR_ARG;
  *bytes = geometry(p, npeaks, kMaxTH, 1).max_bytes;
  return RSZ_OK;
}

static rsz_frame_desc one_desc(const rsz_params *p, const float *frame, const rsz_peak *peaks,
                               uint32_t npeaks, void *out, uint64_t cap) {
  rsz_frame_desc d;
  memset(&d, 0, sizeof d);
  d.params = *p;
  d.frame = frame;
  d.peaks = peaks;
  d.npeaks = npeaks;
  d.out = out;
  d.out_cap = cap;
  return d;
}

int rsz_workspace_bytes(const rsz_params *p, uint32_t npeaks, uint64_t *bytes) {
  const int st = check_params(p, npeaks);
  if (st) return st;
  if (!bytes) return RSZ_ERR_ARG;
  // shapes only: use aligned placeholder pointers
  rsz_frame_desc d = one_desc(p, (const float *)256, npeaks ? (const rsz_peak *)256 : nullptr,
                              npeaks, (void *)256, 0);
  HostPlan hp;
  uint64_t need = 0;
  build_plan(1, &d, nullptr, nullptr, nullptr, 0, 0, hp, &need, nullptr);
  *bytes = need + single_extra();
  return RSZ_OK;
}

int rsz_batch_workspace_bytes(uint32_t nframes, const rsz_frame_desc *h_descs, uint64_t *bytes) {
  if (!bytes || nframes == 0 || !h_descs) return RSZ_ERR_ARG;
  HostPlan hp;
  uint64_t need = 0;
  build_plan(nframes, h_descs, nullptr, nullptr, nullptr, 0, 0, hp, &need,
             nullptr);
  *bytes = need;
  return RSZ_OK;
}

static int single_frame(const rsz_params *p, const float *d_frame, const rsz_peak *d_peaks,
                        uint32_t npeaks, void *d_out, uint64_t out_cap, uint64_t *h_out_bytes,
                        void *d_ws, uint64_t ws_bytes, hipStream_t s, const rsz_debug_bufs *dbg,
                        bool direct_copy = false) {
  int st = check_params(p, npeaks);
  if (st) return st;
  if (!d_frame || !d_ws || (npeaks && !d_peaks) || (!dbg && (!d_out || !h_out_bytes)))
    return RSZ_ERR_ARG;
  if ((uintptr_t)d_frame % 16 || (uintptr_t)d_ws % 256 || (d_out && (uintptr_t)d_out % 16))
    return RSZ_ERR_ARG;
  uint64_t need = 0;
  rsz_workspace_bytes(p, npeaks, &need);
  if (ws_bytes < need) return RSZ_ERR_WORKSPACE;
  // result slots at the workspace tail
  uint8_t *tail = (uint8_t *)d_ws + (need - single_extra());
  uint64_t *res_bytes = (uint64_t *)tail;
  int32_t *res_status = (int32_t *)(tail + 8);
  rsz_frame_desc d = one_desc(p, d_frame, d_peaks, npeaks, d_out ? d_out : (void *)d_ws, out_cap);
  HostPlan hp;
  st = enqueue(1, &d, res_bytes, res_status, d_ws, need - single_extra(), s, dbg, dbg != nullptr,
               hp, direct_copy);
  if (st) return st;
  if (dbg) {
    // the codebook intermediates sit in the frame's state and region
    const FramePlan *fp = (const FramePlan *)hp.bytes.data();
    const FrameState *fs = fp->st;
    if (dbg->codes && launch_debug_codes(hp.bp, fp->nbins, dbg->codes, s) != hipSuccess)
      return RSZ_ERR_HIP;
    if ((dbg->n_out || dbg->out_idx || dbg->out_res) &&
        launch_debug_outliers(hp.bp, dbg->n_out, dbg->out_idx, dbg->out_res, s) != hipSuccess)
      return RSZ_ERR_HIP;
    if (dbg->hist && hipMemcpyAsync(dbg->hist, fs->hist, 4 * kNumSym, hipMemcpyDeviceToDevice, s))
      return RSZ_ERR_HIP;
    if (dbg->lens && hipMemcpyAsync(dbg->lens, fs->lens, kNumSym, hipMemcpyDeviceToDevice, s))
      return RSZ_ERR_HIP;
    if (dbg->cw && hipMemcpyAsync(dbg->cw, fs->cw, 4 * kNumSym, hipMemcpyDeviceToDevice, s))
      return RSZ_ERR_HIP;
    int32_t status = 0;
    if (hipMemcpyAsync(&status, &fs->status, 4, hipMemcpyDeviceToHost, s) != hipSuccess)
      return RSZ_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return RSZ_ERR_HIP;
    return status;
  }
  uint64_t res[2] = {0, 0};
  if (hipMemcpyAsync(res, tail, 16, hipMemcpyDeviceToHost, s) != hipSuccess) return RSZ_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return RSZ_ERR_HIP;
  const int32_t status = (int32_t)(uint32_t)res[1];
  if (status == RSZ_OK || status == RSZ_ERR_CAPACITY) *h_out_bytes = res[0];
  return status;
}

int rsz_compress(const rsz_params *p, const float *d_frame, const rsz_peak *d_peaks,
                 uint32_t npeaks, void *d_out, uint64_t out_cap, uint64_t *h_out_bytes,
                 void *d_ws, uint64_t ws_bytes, void *stream) {
  return single_frame(p, d_frame, d_peaks, npeaks, d_out, out_cap, h_out_bytes, d_ws, ws_bytes,
                      (hipStream_t)stream, nullptr);
}

int rsz_compress_noalloc(const rsz_params *p, const float *d_frame, const rsz_peak *d_peaks,
                         uint32_t npeaks, void *d_out, uint64_t out_cap, uint64_t *h_out_bytes,
                         void *stream) {
  int st = check_params(p, npeaks);
  if (st) return st;
  uint64_t need = 0;
  rsz_workspace_bytes(p, npeaks, &need);
  if (need > RSZ_NOALLOC_SCRATCH_BYTES) return RSZ_ERR_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RSZ_ERR_HIP;
  void *ws = nullptr;
  st = scratch_address(dev, &ws);
  if (st) return st;
  // the call waits for its own kernels, so holding the device's lock keeps
  // calls from several host threads off each other's scratch
  std::lock_guard<std::mutex> lk(g_scratch_mu[dev]);
  return single_frame(p, d_frame, d_peaks, npeaks, d_out, out_cap, h_out_bytes, ws,
                      RSZ_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream, nullptr, true);
}

int rsz_debug_intermediates(const rsz_params *p, const float *d_frame, const rsz_peak *d_peaks,
                            uint32_t npeaks, const rsz_debug_bufs *bufs, void *d_ws,
                            uint64_t ws_bytes, void *stream) {
  if (!bufs) return RSZ_ERR_ARG;
  return single_frame(p, d_frame, d_peaks, npeaks, nullptr, 0, nullptr, d_ws, ws_bytes,
                      (hipStream_t)stream, bufs);
}

int rsz_compress_batch(uint32_t nframes, const rsz_frame_desc *h_descs, uint64_t *d_out_bytes,
                       int32_t *d_status, void *d_ws, uint64_t ws_bytes, void *stream) {
  if (nframes == 0 || !h_descs || !d_out_bytes || !d_status || !d_ws) return RSZ_ERR_ARG;
  if ((uintptr_t)d_ws % 256) return RSZ_ERR_ARG;
  HostPlan hp;
  return enqueue(nframes, h_descs, d_out_bytes, d_status, d_ws, ws_bytes, (hipStream_t)stream,
                 nullptr, false, hp);
}

int rsz_stream_info(const void *h_stream, uint64_t n, rsz_params *p, uint32_t *npeaks,
                    uint64_t *stream_bytes) {
  DecodePlan dp;
  const int st = parse_header((const uint8_t *)h_stream, n, ~0ull, p, npeaks, &dp);
  if (st) return st;
  if (dp.total > n && n > kHeader) {
    // a caller that passes more than the header must pass the whole stream
    return RSZ_ERR_CORRUPT;
  }
  if (stream_bytes) *stream_bytes = dp.total;
  return RSZ_OK;
}

int rsz_decompress_workspace_bytes(const void *h_header, uint64_t n, uint64_t *bytes) {
  DecodePlan dp;
  const int st = parse_header((const uint8_t *)h_header, n, ~0ull, nullptr, nullptr, &dp);
  if (st) return st;
  if (!bytes) return RSZ_ERR_ARG;
  *bytes = decode_head_bytes(1) + decode_ws_bytes(dp);
  return RSZ_OK;
}

int rsz_decompress(const void *d_in, uint64_t in_bytes, float *d_frame, uint64_t frame_elems,
                   void *d_ws, uint64_t ws_bytes, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  if (!d_in || !d_frame || !d_ws || (uintptr_t)d_in % 16 || (uintptr_t)d_frame % 16 ||
      (uintptr_t)d_ws % 256)
    return RSZ_ERR_ARG;
  if (in_bytes < kHeader) return RSZ_ERR_CORRUPT;
  uint8_t hdr[80];
  if (hipMemcpyAsync(hdr, d_in, 80, hipMemcpyDeviceToHost, s) != hipSuccess) return RSZ_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return RSZ_ERR_HIP;
  DecodePlan dp;
  int st = parse_header(hdr, 80, in_bytes, nullptr, nullptr, &dp);
  if (st) return st;
  if (frame_elems < (uint64_t)dp.P * dp.H * dp.W) return RSZ_ERR_ARG;
  // a batch of one stream
  DecodeItem it{d_in, in_bytes, hdr, d_frame, frame_elems, nullptr};
  int32_t *status_word = nullptr;
  st = decode_streams(1, &it, (uint8_t *)d_ws, ws_bytes, s, nullptr, &status_word);
  if (st) return st;
  int32_t status = 0;
  if (hipMemcpyAsync(&status, status_word, 4, hipMemcpyDeviceToHost, s) != hipSuccess)
    return RSZ_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return RSZ_ERR_HIP;
  return status;
}

static int decode_items(uint32_t n, const rsz_decode_desc *d, int32_t *d_status,
                        std::vector<DecodeItem> &items) {
  if (n == 0 || !d) return RSZ_ERR_ARG;
  items.resize(n);
  for (uint32_t f = 0; f < n; ++f) {
    if (!d[f].header) return RSZ_ERR_ARG;
    items[f] = DecodeItem{d[f].in, d[f].in_bytes, (const uint8_t *)d[f].header, d[f].frame,
                          d[f].frame_elems, d_status ? d_status + f : nullptr};
  }
  return RSZ_OK;
}

int rsz_decompress_batch_workspace_bytes(uint32_t n, const rsz_decode_desc *h_descs,
                                         uint64_t *bytes) {
  std::vector<DecodeItem> items;
  const int st = decode_items(n, h_descs, nullptr, items);
  if (st) return st;
  if (!bytes) return RSZ_ERR_ARG;
  return decode_streams(n, items.data(), nullptr, 0, nullptr, bytes, nullptr);
}

int rsz_decompress_batch(uint32_t n, const rsz_decode_desc *h_descs, int32_t *d_status,
                         void *d_ws, uint64_t ws_bytes, void *stream) {
  if (!d_status || !d_ws || (uintptr_t)d_ws % 256) return RSZ_ERR_ARG;
  std::vector<DecodeItem> items;
  const int st = decode_items(n, h_descs, d_status, items);
  if (st) return st;
  return decode_streams(n, items.data(), (uint8_t *)d_ws, ws_bytes, (hipStream_t)stream, nullptr,
                        nullptr);
}

int rsz_batch_prepare(uint32_t nframes, const rsz_frame_desc *h_descs, uint64_t *d_out_bytes,
                      int32_t *d_status, void *d_ws, uint64_t ws_bytes, void *stream,
                      rsz_batch_plan *h_plan) {
  if (nframes == 0 || !h_descs || !d_out_bytes || !d_status || !d_ws || !h_plan) return RSZ_ERR_ARG;
  if ((uintptr_t)d_ws % 256) return RSZ_ERR_ARG;
  HostPlan hp;
  const int st = build_plan(nframes, h_descs, d_out_bytes, d_status, (uint8_t *)d_ws, ws_bytes,
                            0, hp, nullptr, nullptr);
  if (st) return st;
  if (stage_to_device(d_ws, hp.bytes.data(), hp.bytes.size(), (hipStream_t)stream) != RSZ_OK)
    return RSZ_ERR_HIP;
  PlanRecord rec;
  rec.bp = hp.bp;
  rec.common_b = hp.common_b;
  rec.common_dim = hp.common_dim;
  memset(h_plan, 0, sizeof *h_plan);
  memcpy(h_plan, &rec, sizeof rec);
  return RSZ_OK;
}

int rsz_batch_launch(const rsz_batch_plan *h_plan, void *stream) {
  if (!h_plan) return RSZ_ERR_ARG;
  PlanRecord rec;
  memcpy(&rec, h_plan, sizeof rec);
  if (rec.bp.nframes == 0 || !rec.bp.frames) return RSZ_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (launch_compress_front_b(rec.bp, rec.common_b, rec.common_dim, s, false) != hipSuccess)
    return RSZ_ERR_HIP;
  if (launch_compress_back(rec.bp, s) != hipSuccess) return RSZ_ERR_HIP;
  return RSZ_OK;
}

int rsz_batch_graph_create(const rsz_batch_plan *h_plan, void *stream, void **h_graph_exec) {
  if (!h_plan || !h_graph_exec) return RSZ_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  hipGraph_t g = nullptr;
  // timing events are not recorded into graphs
  const bool prof = g_prof_on;
  g_prof_on = false;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    g_prof_on = prof;
    return RSZ_ERR_HIP;
  }
  const int st = rsz_batch_launch(h_plan, stream);
  const hipError_t e = hipStreamEndCapture(s, &g);
  g_prof_on = prof;
  if (st != RSZ_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st != RSZ_OK ? st : RSZ_ERR_HIP;
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return RSZ_ERR_HIP;
  *h_graph_exec = (void *)ex;
  return RSZ_OK;
}

// ------------------------------------------------------------ verification

}  // extern "C"

namespace rsz {
// Host record of a prepared verification (the public rsz_verify_plan is its
// storage): the verification batch, the decoder batch and its grid sizes.
struct VerifyRecord {
  VerifyBatch vb;
  DecBatch db;
  uint32_t dec_total[kDecKernels];
};
static_assert(sizeof(VerifyRecord) <= sizeof(rsz_verify_plan), "verify record too large");

// Plans the verification of a prepared batch: per frame a decoder plan whose
// geometry and pointers are fixed here (k_vplan fills in the totals on the
// device), its workspace region, and the k_verify blocks.  With ws, uploads
// it all and fills *vr; *need: the workspace bytes.
static int verify_plan(const PlanRecord &rec, uint32_t n, const rsz_frame_desc *d,
                       float *const *frames_out, uint32_t *d_bad, uint8_t *ws, uint64_t ws_bytes,
                       hipStream_t s, uint64_t *need, VerifyRecord *vr) {
  if (n == 0 || !d || n != rec.bp.nframes || !rec.bp.frames) return RSZ_ERR_ARG;
  std::vector<DecodePlan> dps(n);
  std::vector<VerifyFrame> vfs(n);
  std::vector<uint64_t> region(n, 0);
  const uint64_t h_dp = align_up((uint64_t)sizeof(DecodePlan) * n, 256);
  const uint64_t h_pre = align_up(4ull * kDecKernels * (n + 1), 256);
  const uint64_t h_vf = align_up((uint64_t)sizeof(VerifyFrame) * n, 256);
  const uint64_t h_vp = align_up(4ull * (n + 1), 256);
  const uint64_t head = h_dp + h_pre + h_vf + h_vp;
  uint64_t total = head;
  for (uint32_t f = 0; f < n; ++f) {
    DecodePlan &dp = dps[f];
    VerifyFrame &vf = vfs[f];
    memset(&dp, 0, sizeof dp);
    memset(&vf, 0, sizeof vf);
    const rsz_params *p = &d[f].params;
    // (the sizing pass has no output frames yet; the prepare pass needs them)
    bool ok = check_params(p, d[f].npeaks) == RSZ_OK && !p->roi_coding && !p->run_coding &&
              d[f].frame && d[f].out && (d[f].npeaks == 0 || d[f].peaks);
    if (ok && ws && !(frames_out && frames_out[f])) return RSZ_ERR_ARG;
    uint32_t rows = 0;
    if (ok) {
      const uint32_t wpr = (p->width + 31) / 32;
      rows = (kVerifyMaskWords / wpr) / p->bin * p->bin;
      ok = rows > 0;
    }
    if (!ok) {
      dp.init_status = RSZ_ERR_ARG;
      region[f] = 256;   // its status word
      total += region[f];
      continue;
    }
    const Geom g = geometry(p, d[f].npeaks, kMaxTH, 1);
    dp.P = p->panels;
    dp.H = p->height;
    dp.W = p->width;
    dp.w = p->window;
    dp.b = p->bin;
    dp.npeaks = d[f].npeaks;
    dp.dim = p->dim ? p->dim : 2u;
    dp.step = 2.0 * p->eb;
    dp.Hb = g.Hb;
    dp.Wb = g.Wb;
    dp.nbins = g.nbins;
    dp.nchunks = g.nchunks;
    dp.off_peaks = kHeader;
    dp.off_roi = g.off_roi;
    dp.off_lens = g.off_lens;
    dp.off_chunks = g.off_chunks;
    dp.off_bits = g.off_bits;
    dp.init_status = RSZ_OK;
    region[f] = decode_ws_bytes(dp);
    total += region[f];
    rows = std::min<uint32_t>(rows, (uint32_t)align_up(p->height, p->bin));
    vf.x = d[f].frame;
    vf.y = frames_out ? frames_out[f] : nullptr;
    vf.peaks = (const int32_t *)d[f].peaks;
    vf.npeaks = d[f].npeaks;
    vf.P = p->panels;
    vf.H = p->height;
    vf.W = p->width;
    vf.w = p->window;
    vf.b = p->bin;
    vf.mode = p->bin_mode;
    vf.eb = p->eb;
    vf.rows = rows;
    vf.chunks = (p->height + rows - 1) / rows;
    vf.valid = 1;
  }
  if (need) *need = total;
  if (!ws) return RSZ_OK;
  if (!d_bad || (uintptr_t)ws % 256) return RSZ_ERR_ARG;
  if (ws_bytes < total) return RSZ_ERR_WORKSPACE;
  std::vector<uint8_t> host(head, 0);
  uint32_t *pre = (uint32_t *)(host.data() + h_dp);
  uint32_t *vpre = (uint32_t *)(host.data() + h_dp + h_pre + h_vf);
  uint64_t off = head;
  uint32_t dec_total[kDecKernels] = {0};
  uint64_t wgs = 0;
  for (uint32_t f = 0; f < n; ++f) {
    DecodePlan &dp = dps[f];
    VerifyFrame &vf = vfs[f];
    uint8_t *w = ws + off;
    off += region[f];
    if (vf.valid) {
      dp.in = (const uint8_t *)d[f].out;
      dp.frame = frames_out[f];
      dp.res = (int32_t *)w;
      w += align_up(4ull * dp.nbins, 256);
      dp.res8 = w;
      w += align_up(dp.nbins + 64ull, 256);
      dp.zcount = (uint32_t *)w;
      w += align_up(4ull * dp.nchunks, 256);
      dp.status = (int32_t *)w;
      w += 256;
      dp.tables = (uint32_t *)w;
      w += align_up(decode_tables_bytes(), 256);
      if (dp.dim == 1) dp.carry = (uint32_t *)w;
      dp.bits = (const uint32_t *)(dp.in + dp.off_bits);
    } else {
      dp.status = (int32_t *)w;
    }
    vf.cplan = rec.bp.frames + f;
    vf.dplan = (DecodePlan *)ws + f;
    vf.bad = d_bad + f;
    uint32_t nb[kDecKernels];
    decode_blocks(dp, nb);
    // the outliers: a fixed number of workgroups (their count is known only
    // on the device), each striding over them
    if (vf.valid) nb[4] = std::min<uint32_t>(kVerifyOutlierBlocks, (dp.nbins + 255) / 256);
    for (int k = 0; k < kDecKernels; ++k) {
      pre[(size_t)k * (n + 1) + f] = dec_total[k];
      if ((uint64_t)dec_total[k] + nb[k] > 0x7FFFFFFFull) return RSZ_ERR_ARG;
      dec_total[k] += nb[k];
    }
    vpre[f] = (uint32_t)wgs;
    if (vf.valid) wgs += (uint64_t)vf.P * vf.chunks;
    if (wgs > 0x7FFFFFFFull) return RSZ_ERR_ARG;
  }
  for (int k = 0; k < kDecKernels; ++k) pre[(size_t)k * (n + 1) + n] = dec_total[k];
  vpre[n] = (uint32_t)wgs;
  memcpy(host.data(), dps.data(), sizeof(DecodePlan) * n);
  memcpy(host.data() + h_dp + h_pre, vfs.data(), sizeof(VerifyFrame) * n);
  const int st = stage_to_device(ws, host.data(), head, s);
  if (st) return st;
  memset(vr, 0, sizeof *vr);
  vr->vb.n = n;
  vr->vb.frames = (const VerifyFrame *)(ws + h_dp + h_pre);
  vr->vb.wg_prefix = (const uint32_t *)(ws + h_dp + h_pre + h_vf);
  vr->vb.total_wgs = (uint32_t)wgs;
  vr->db.n = n;
  vr->db.plans = (const DecodePlan *)ws;
  vr->db.pre = (const uint32_t *)(ws + h_dp);
  memcpy(vr->dec_total, dec_total, sizeof dec_total);
  return RSZ_OK;
}
}  // namespace rsz

extern "C" {

int rsz_verify_workspace_bytes(const rsz_batch_plan *h_plan, uint32_t nframes,
                               const rsz_frame_desc *h_descs, uint64_t *bytes) {
  if (!h_plan || !bytes) return RSZ_ERR_ARG;
  PlanRecord rec;
  memcpy(&rec, h_plan, sizeof rec);
  return verify_plan(rec, nframes, h_descs, nullptr, nullptr, nullptr, 0, nullptr, bytes,
                     nullptr);
}

int rsz_verify_prepare(const rsz_batch_plan *h_plan, uint32_t nframes,
                       const rsz_frame_desc *h_descs, float *const *h_frames_out, uint32_t *d_bad,
                       void *d_ws, uint64_t ws_bytes, void *stream, rsz_verify_plan *h_vplan) {
  if (!h_plan || !h_vplan || !d_ws || !h_frames_out) return RSZ_ERR_ARG;
  PlanRecord rec;
  memcpy(&rec, h_plan, sizeof rec);
  VerifyRecord vr;
  const int st = verify_plan(rec, nframes, h_descs, h_frames_out, d_bad, (uint8_t *)d_ws,
                             ws_bytes, (hipStream_t)stream, nullptr, &vr);
  if (st) return st;
  memset(h_vplan, 0, sizeof *h_vplan);
  memcpy(h_vplan, &vr, sizeof vr);
  return RSZ_OK;
}

int rsz_verify_launch(const rsz_verify_plan *h_vplan, void *stream) {
  if (!h_vplan) return RSZ_ERR_ARG;
  VerifyRecord vr;
  memcpy(&vr, h_vplan, sizeof vr);
  if (vr.vb.n == 0 || !vr.vb.frames) return RSZ_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (launch_verify_plan(vr.vb, s) != hipSuccess) return RSZ_ERR_HIP;
  if (launch_decompress(vr.db, vr.dec_total, s) != hipSuccess) return RSZ_ERR_HIP;
  if (launch_verify_check(vr.vb, s) != hipSuccess) return RSZ_ERR_HIP;
  return RSZ_OK;
}

int rsz_verify_graph_create(const rsz_batch_plan *h_plan, const rsz_verify_plan *h_vplan,
                            void *stream, void **h_graph_exec) {
  if (!h_plan || !h_vplan || !h_graph_exec) return RSZ_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  hipGraph_t g = nullptr;
  const bool prof = g_prof_on;
  g_prof_on = false;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    g_prof_on = prof;
    return RSZ_ERR_HIP;
  }
  int st = rsz_batch_launch(h_plan, stream);
  if (st == RSZ_OK) st = rsz_verify_launch(h_vplan, stream);
  const hipError_t e = hipStreamEndCapture(s, &g);
  g_prof_on = prof;
  if (st != RSZ_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st != RSZ_OK ? st : RSZ_ERR_HIP;
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return RSZ_ERR_HIP;
  *h_graph_exec = (void *)ex;
  return RSZ_OK;
}

int rsz_graph_launch(void *graph_exec, void *stream) {
  if (!graph_exec) return RSZ_ERR_ARG;
  return hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream) == hipSuccess
             ? RSZ_OK
             : RSZ_ERR_HIP;
}

int rsz_graph_destroy(void *graph_exec) {
  if (!graph_exec) return RSZ_ERR_ARG;
  return hipGraphExecDestroy((hipGraphExec_t)graph_exec) == hipSuccess ? RSZ_OK : RSZ_ERR_HIP;
}

int rsz_debug_codebook(const uint32_t *h_hist, uint8_t *h_lens, uint32_t *h_cw, void *d_ws,
                       uint64_t ws_bytes, void *stream) {
  if (!h_hist || !h_lens || !h_cw || !d_ws || (uintptr_t)d_ws % 256) return RSZ_ERR_ARG;
  uint64_t total = 0;
  for (int i = 0; i < kNumSym; ++i) total += h_hist[i];
  if (total == 0 || total >= (1ull << 27)) return RSZ_ERR_ARG;
  const uint64_t off_state = align_up(sizeof(FramePlan), 256);
  if (ws_bytes < off_state + sizeof(FrameState)) return RSZ_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  uint8_t *ws = (uint8_t *)d_ws;
  FramePlan fp;
  memset(&fp, 0, sizeof fp);
  fp.st = (FrameState *)(ws + off_state);
  FrameState fs;
  memset(&fs, 0, sizeof fs);
  fs.status = RSZ_OK;
  memcpy(fs.hist, h_hist, sizeof fs.hist);
  BatchPlan bp;
  memset(&bp, 0, sizeof bp);
  bp.nframes = 1;
  bp.frames = (const FramePlan *)ws;
  if (hipMemcpyAsync(ws, &fp, sizeof fp, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(ws + off_state, &fs, sizeof fs, hipMemcpyHostToDevice, s) != hipSuccess ||
      launch_codebook(bp, s) != hipSuccess ||
      hipMemcpyAsync(h_lens, ((FrameState *)(ws + off_state))->lens, kNumSym,
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(h_cw, ((FrameState *)(ws + off_state))->cw, 4 * kNumSym,
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return RSZ_ERR_HIP;
  return RSZ_OK;
}

// Plain streaming read: grid-stride 16-byte loads, folded so the loads stay.
__global__ __launch_bounds__(256) void k_measure_read(const uint4 *x, uint64_t n16,
                                                      uint32_t *sink) {
  uint32_t acc = 0;
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * 256) {
    const uint4 v = x[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x9E3779B9u) sink[blockIdx.x & 1023] = acc;
}

int rsz_measure_read(const void *d_buf, uint64_t bytes, void *d_sink, int reps, double *h_gbps,
                     void *stream) {
  if (!d_buf || !d_sink || !h_gbps || reps < 1 || bytes < 16 || (uintptr_t)d_buf % 16 ||
      (uintptr_t)d_sink % 4)
    return RSZ_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  const uint64_t n16 = bytes / 16;
  const uint32_t grid = 8192;
  hipEvent_t a, e;
  if (hipEventCreate(&a) != hipSuccess) return RSZ_ERR_HIP;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipEventDestroy(a);
    return RSZ_ERR_HIP;
  }
  int st = RSZ_OK;
  hipLaunchKernelGGL(k_measure_read, dim3(grid), dim3(256), 0, s, (const uint4 *)d_buf, n16,
                     (uint32_t *)d_sink);
  const hipError_t ea = hipEventRecord(a, s);
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL(k_measure_read, dim3(grid), dim3(256), 0, s, (const uint4 *)d_buf, n16,
                       (uint32_t *)d_sink);
  const hipError_t ee = hipEventRecord(e, s);
  float ms = 0.f;
  if (ea != hipSuccess || ee != hipSuccess || hipGetLastError() != hipSuccess ||
      hipEventSynchronize(e) != hipSuccess ||
      hipEventElapsedTime(&ms, a, e) != hipSuccess || ms <= 0.f)
    st = RSZ_ERR_HIP;
  else
    *h_gbps = (double)reps * (double)(n16 * 16) / ((double)ms * 1e6);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(e);
  return st;
}

int rsz_profile_enable(int enable) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto &r : g_prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  g_prof.reserve(1 << 16);
  g_prof_on = enable != 0;
  return RSZ_OK;
}

int rsz_profile_only(const char *name) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_only = name ? name : "";
  return RSZ_OK;
}

int rsz_profile_read(rsz_kernel_time *out, int max, int *n) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  std::vector<rsz_kernel_time> acc;
  for (auto &r : g_prof) {
    if (hipEventSynchronize(r.b) != hipSuccess) return RSZ_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return RSZ_ERR_HIP;
    auto it = std::find_if(acc.begin(), acc.end(),
                           [&](const rsz_kernel_time &k) { return r.name == k.name; });
    if (it == acc.end()) {
      rsz_kernel_time k;
      memset(&k, 0, sizeof k);
      strncpy(k.name, r.name.c_str(), sizeof k.name - 1);
      acc.push_back(k);
      it = acc.end() - 1;
    }
    it->launches++;
    it->total_ms += ms;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  const int m = std::min<int>((int)acc.size(), max);
  for (int i = 0; i < m; ++i) out[i] = acc[i];
  if (n) *n = (int)acc.size();
  return RSZ_OK;
}

// ------------------------------------------------------------ peak finding

void rsz_peak_params_default(rsz_peak_params *q) {
  if (!q) return;
  memset(q, 0, sizeof *q);
  q->rank = 3;          // 7x7 window
  q->ring_in = 4;       // background ring just outside the window
  q->ring_out = 5;
  q->npix_min = 2;
  q->npix_max = 30;
  q->amax_min = 300.0;
  q->atot_min = 600.0;
  q->snr_min = 10.0;
  q->pix_nsigma = 3.0;
}

static int check_peak_params(const rsz_peak_params *q) {
  if (!q || q->rank < 1 || q->rank > 3 || q->ring_in <= q->rank || q->ring_out < q->ring_in ||
      q->ring_out > 15 || q->npix_min > q->npix_max || q->reserved != 0)
    return RSZ_ERR_ARG;
  if (!std::isfinite(q->amax_min) || !std::isfinite(q->atot_min) || !std::isfinite(q->snr_min) ||
      !(q->snr_min >= 0.0) || !std::isfinite(q->pix_nsigma) || !(q->pix_nsigma >= 0.0))
    return RSZ_ERR_ARG;
  return RSZ_OK;
}

static bool peak_desc_ok(const rsz_peak_desc &d) {
  if (d.panels < 1 || d.panels > 65535 || d.height < 1 || d.height > 65535 || d.width < 1 ||
      d.width > 65535)
    return false;
  if ((uint64_t)d.panels * d.height * d.width >= (1ull << 31)) return false;
  if (d.max_peaks < 1 || d.max_peaks > kPeakCapMax || !d.frame || !d.peaks) return false;
  return (uintptr_t)d.frame % 16 == 0 && (uintptr_t)d.peaks % 4 == 0;
}

// Workspace: frame plans, tile prefix, then per frame a counter and its keys.
static uint64_t peak_layout(uint32_t nframes, const rsz_peak_desc *d, std::vector<uint64_t> *off,
                            uint64_t *prefix_off) {
  uint64_t o = align_up(sizeof(PeakFramePlan) * nframes, 256);
  *prefix_off = o;
  o += align_up(4ull * (nframes + 1), 256);
  if (off) off->resize(nframes);
  for (uint32_t f = 0; f < nframes; ++f) {
    if (off) (*off)[f] = o;
    o += 256 + align_up(8ull * (peak_desc_ok(d[f]) ? d[f].max_peaks : 0), 256);
  }
  return o;
}

int rsz_find_peaks_workspace_bytes(uint32_t nframes, const rsz_peak_desc *h_descs,
                                   uint64_t *bytes) {
  if (nframes == 0 || !h_descs || !bytes) return RSZ_ERR_ARG;
  uint64_t po;
  *bytes = peak_layout(nframes, h_descs, nullptr, &po);
  return RSZ_OK;
}

int rsz_find_peaks_batch(const rsz_peak_params *q, uint32_t nframes, const rsz_peak_desc *h_descs,
                         uint32_t *d_counts, int32_t *d_status, void *d_ws, uint64_t ws_bytes,
                         void *stream) {
  if (check_peak_params(q) != RSZ_OK || nframes == 0 || !h_descs || !d_counts || !d_status ||
      !d_ws || (uintptr_t)d_ws % 256)
    return RSZ_ERR_ARG;
  std::vector<uint64_t> off;
  uint64_t prefix_off;
  const uint64_t need = peak_layout(nframes, h_descs, &off, &prefix_off);
  if (ws_bytes < need) return RSZ_ERR_WORKSPACE;
  uint8_t *ws = (uint8_t *)d_ws;
  std::vector<uint8_t> host(align_up(prefix_off + 4ull * (nframes + 1), 256), 0);
  PeakFramePlan *fpl = (PeakFramePlan *)host.data();
  uint32_t *tp = (uint32_t *)(host.data() + prefix_off);
  uint64_t tiles = 0;
  for (uint32_t f = 0; f < nframes; ++f) {
    const rsz_peak_desc &d = h_descs[f];
    PeakFramePlan &fp = fpl[f];
    tp[f] = (uint32_t)tiles;
    fp.count = (uint32_t *)(ws + off[f]);
    fp.keys = (uint64_t *)(ws + off[f] + 256);
    fp.res_count = d_counts + f;
    fp.res_status = d_status + f;
    if (!peak_desc_ok(d)) {
      fp.init_status = RSZ_ERR_ARG;
      continue;
    }
    fp.init_status = RSZ_OK;
    fp.P = d.panels;
    fp.H = d.height;
    fp.W = d.width;
    fp.cap = d.max_peaks;
    fp.frame = d.frame;
    fp.out = d.peaks;
    tiles += div_up((uint64_t)d.panels * d.height * d.width, kPeakTile);
  }
  if (tiles >= (1ull << 31)) return RSZ_ERR_ARG;
  tp[nframes] = (uint32_t)tiles;
  hipStream_t s = (hipStream_t)stream;
  if (stage_to_device(ws, host.data(), host.size(), s) != RSZ_OK) return RSZ_ERR_HIP;
  PeakBatchPlan pp;
  memset(&pp, 0, sizeof pp);
  pp.nframes = nframes;
  pp.total_tiles = (uint32_t)tiles;
  pp.q = *q;
  // float x >= amax_min (in fp64) exactly when x >= the smallest float at or
  // above amax_min
  float af = (float)q->amax_min;
  if ((double)af < q->amax_min) af = std::nextafter(af, INFINITY);
  pp.amax_f = af;
  pp.frames = (const PeakFramePlan *)ws;
  pp.tile_prefix = (const uint32_t *)(ws + prefix_off);
  return launch_find_peaks(pp, s) == hipSuccess ? RSZ_OK : RSZ_ERR_HIP;
}

}  // extern "C"
