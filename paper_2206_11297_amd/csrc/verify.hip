// On-device verification of a compressed batch: the decompress-and-check
// stage that a graph-captured pipeline appends to compression.  The batch's
// own streams are decoded by the decoder kernels (decompress.hip), whose
// plans are completed here from the totals the compression left on the
// device, and every pixel of every decoding is checked against the frame
// it came from: ROI pixels bit for bit (Sec. IV: the windows are kept
// losslessly), every other pixel within the error bound of its bin's mean
// (Sec. V-C: the bound is absolute on the binned values; Sec. IV-A: the
// bin value is restored to each of its pixels).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsz_internal.h"

namespace rsz {

// The data-dependent fields of each frame's decoder plan, from the totals
// the compression wrote (only frames with the ROI verbatim and no run stage
// are verified); a frame whose compression failed decodes nothing.  The
// violation counts start at zero.
__global__ __launch_bounds__(256) void k_vplan(VerifyBatch vb) {
  const uint32_t f = blockIdx.x * 256 + threadIdx.x;
  if (f >= vb.n) return;
  const VerifyFrame &vf = vb.frames[f];
  *vf.bad = 0u;
  if (!vf.valid) return;
  DecodePlan *dp = vf.dplan;
  const FrameState *st = vf.cplan->st;
  const int32_t status = __hip_atomic_load(&st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (status != RSZ_OK) {
    dp->init_status = RSZ_ERR_ARG;
    return;
  }
  const uint64_t T = st->T;
  const uint32_t n_out = st->n_out;
  dp->T = T;
  dp->n_out = n_out;
  dp->total = st->total;
  dp->off_oidx = dp->off_bits + 4 * ((T + 31) / 32);
  dp->off_ores = dp->off_oidx + 4ull * n_out;
  dp->init_status = RSZ_OK;
}

// One workgroup per block of `rows` raw rows of a panel: the block's ROI
// bitmap in LDS from the frame's peaks (the windows of Sec. IV, clipped to
// the panel), then one thread per bin: the mean of the bin's pixels that
// enter it (all of them, or those outside every window) in fp64, and each
// pixel's check.  A background pixel passes when |y - mean| <= eb + |y|
// 2^-23 + |mean| 2^-40: the bound, plus the float32 rounding of the stored
// value and the rounding of the fp64 sums (taken here in another order than
// the compressor's).
__global__ __launch_bounds__(256) void k_verify(VerifyBatch vb) {
  __shared__ uint32_t s_mask[kVerifyMaskWords];
  __shared__ uint32_t s_f;
  if (threadIdx.x == 0) {
    uint32_t lo = 0, hi = vb.n;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (vb.wg_prefix[mid] <= blockIdx.x) lo = mid; else hi = mid;
    }
    s_f = lo;
  }
  __syncthreads();
  const uint32_t f = s_f;
  const VerifyFrame &vf = vb.frames[f];
  // both stages of this frame finished without an error (else k_vdone
  // reports it)
  if (!vf.valid || vf.cplan->st->status != RSZ_OK || *vf.dplan->status != RSZ_OK) return;
  const uint32_t blk = blockIdx.x - vb.wg_prefix[f];
  const uint32_t p = blk / vf.chunks, r0 = (blk - p * vf.chunks) * vf.rows;
  const uint32_t H = vf.H, W = vf.W, b = vf.b;
  const uint32_t r1 = min(r0 + vf.rows, H), nr = r1 - r0, wpr = (W + 31) / 32;
  for (uint32_t i = threadIdx.x; i < nr * wpr; i += 256) s_mask[i] = 0u;
  __syncthreads();
  const int32_t h = (int32_t)(vf.w / 2);
  for (uint32_t k = threadIdx.x; k < vf.npeaks; k += 256) {
    if ((uint32_t)vf.peaks[3 * k] != p) continue;
    const int32_t pr = vf.peaks[3 * k + 1] - h, pc = vf.peaks[3 * k + 2] - h;
    const int32_t ra = max(pr, (int32_t)r0), rb = min(pr + (int32_t)vf.w, (int32_t)r1);
    const int32_t ca = max(pc, 0), cb = min(pc + (int32_t)vf.w, (int32_t)W);
    for (int32_t r = ra; r < rb; ++r)
      for (int32_t c = ca; c < cb;) {
        const int32_t e = min(cb, (c & ~31) + 32);
        const uint32_t bits = (e - c == 32 ? ~0u : ((1u << (e - c)) - 1u)) << (c & 31);
        atomicOr(&s_mask[(uint32_t)(r - (int32_t)r0) * wpr + (uint32_t)c / 32], bits);
        c = e;
      }
  }
  __syncthreads();
  const uint32_t Wb = (W + b - 1) / b, Ib0 = r0 / b, Ib1 = (r1 + b - 1) / b;
  const float *x = vf.x + (size_t)p * H * W, *y = vf.y + (size_t)p * H * W;
  const double eb = vf.eb;
  uint32_t bad = 0;
  for (uint32_t i = threadIdx.x; i < (Ib1 - Ib0) * Wb; i += 256) {
    const uint32_t I = Ib0 + i / Wb, J = i % Wb;
    const uint32_t ia = I * b, ie = min(ia + b, H), ja = J * b, je = min(ja + b, W);
    double S = 0.0;
    uint32_t n = 0;
    for (uint32_t r = ia; r < ie; ++r)
      for (uint32_t c = ja; c < je; ++c) {
        const bool roi = (s_mask[(r - r0) * wpr + c / 32] >> (c & 31)) & 1u;
        if (vf.mode || !roi) {
          S += (double)x[(size_t)r * W + c];
          ++n;
        }
      }
    const double mean = n ? S / (double)n : 0.0;
    for (uint32_t r = ia; r < ie; ++r)
      for (uint32_t c = ja; c < je; ++c) {
        const size_t g = (size_t)r * W + c;
        const bool roi = (s_mask[(r - r0) * wpr + c / 32] >> (c & 31)) & 1u;
        if (roi) {
          bad += __float_as_uint(y[g]) != __float_as_uint(x[g]);
        } else {
          const double yv = (double)y[g];
          const double tol = eb + fabs(yv) * 0x1p-23 + fabs(mean) * 0x1p-40;
          bad += !(fabs(yv - mean) <= tol);
        }
      }
  }
  if (bad) atomicAdd(vf.bad, bad);
}

// A frame whose compression or decoding failed reports 0xFFFFFFFF.
__global__ __launch_bounds__(256) void k_vdone(VerifyBatch vb) {
  const uint32_t f = blockIdx.x * 256 + threadIdx.x;
  if (f >= vb.n) return;
  const VerifyFrame &vf = vb.frames[f];
  if (!vf.valid || vf.cplan->st->status != RSZ_OK || *vf.dplan->status != RSZ_OK)
    *vf.bad = 0xFFFFFFFFu;
}

hipError_t launch_verify_plan(const VerifyBatch &vb, hipStream_t s) {
  prof_begin("k_vplan", s);
  hipLaunchKernelGGL(k_vplan, dim3((vb.n + 255) / 256), dim3(256), 0, s, vb);
  prof_end(s);
  return hipGetLastError();
}

hipError_t launch_verify_check(const VerifyBatch &vb, hipStream_t s) {
  if (vb.total_wgs) {
    prof_begin("k_verify", s);
    hipLaunchKernelGGL(k_verify, dim3(vb.total_wgs), dim3(256), 0, s, vb);
    prof_end(s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  prof_begin("k_vdone", s);
  hipLaunchKernelGGL(k_vdone, dim3((vb.n + 255) / 256), dim3(256), 0, s, vb);
  prof_end(s);
  return hipGetLastError();
}

}  // namespace rsz
