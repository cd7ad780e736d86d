// xcorr_tri.hip -- gfx950 correlation kernel for arrays of at most 256
// elements: one workgroup computes the whole upper triangle of a channel.
//
// Same contraction as the other kernels (paper Sec. II-A, Eq. 1 and 2):
//   Re V_ij = P_i . P_j,  Im V_ij = Q_i . P_j,   P_e = [Re e, Im e],
//   Q_e = [Im e, -Re e]  over the time axis,
// on v_mfma_i32_32x32x32_i8, over the triangle of 32x32 blocks that Sec. II-C
// and Fig. 1 draw (36 blocks for 256 elements). Shape, chosen for gfx950:
//   * 8 waves, two per SIMD. SIMD s owns block rows s and 7-s: (8-s) + (s+1)
//     = 9 blocks, so the four SIMDs carry equal MFMA work. The SIMD's first
//     wave takes row s, columns s..s+4; its second wave the other four blocks.
//   * the matrix cores multiply the Excess-8 fields themselves, u = x + 8 in
//     [0, 15] (the offset arithmetic of Sec. III-A, Eq. 3), not the signed
//     values: with a, b the fields (Re, Im) of element i and c, d those of j,
//       Re V_ij = sum(a c + b d) - 8 (SR_i + SI_i) - 8 (SR_j + SI_j) + 128 T
//       Im V_ij = sum(b c + a' d) + 8 SR_i - 8 SI_i - 8 SR_j - 7 SI_j,
//     a' = 15 - a, SR_e and SI_e the sums of element e's fields, T the number
//     of samples. On realistic data int8 MFMA throughput is power-limited, and
//     operands whose upper four bits never toggle run about 13 % faster than
//     sign-extended ones. The byte 0x00 (the padding the loads produce past
//     the end of the data) then adds nothing to any sum, so no sample masks
//     are needed; the uncorrected sums may wrap in int32, but the arithmetic
//     is exact modulo 2^32 and the corrected result fits.
//   * every operand, row or column, is decoded once per workgroup into LDS
//     slabs P = [a g, a g+1, b g, b g+1] (each dword = 4 consecutive samples
//     of one field). Q = [b g, b g+1, a' g, a' g+1] is formed from P in
//     registers (a' = a XOR 15: one op per dword).
//   * packed bytes go from HBM straight into LDS (buffer_load ... lds), two
//     stages ahead of use. Each wave loads 8 sample rows per stage and is the
//     only reader of them: it waits for its own loads only, and the stage
//     barrier never waits for memory.
//   * a wave decodes its 8 samples with ds_read_b64_tr_b8, whose 8x8 byte
//     transpose hands each lane 8 consecutive samples of one element.
//
// Blocks of the triangle that lie past n (n < 256) are computed from padding
// and never stored; entries below the diagonal of a diagonal block likewise
// (Sec. II-C computes and ignores them).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "xcorr_device.h"
#include "xcorr_launch.h"
#include "xcorr_tri_common.h"
#include "xcorr_tri_run.h"

namespace xeng {

namespace {

using namespace tri;
// Delay compensation (per-element integer sample delays applied while
// staging); the input holds max_delay halo samples before the frame.
__global__ __launch_bounds__(kThreads, 1) void xcorr_tri_delay_kernel(TriParams p, TriDelays d) {
  // the gather slots; after the stage loop the raw buffers of the corrections
  // live in the same memory
  __shared__ __attribute__((aligned(16))) uint8_t gath0[kGathGroup];
  __shared__ __attribute__((aligned(16))) uint8_t gath1[kGathGroup];
  __shared__ __attribute__((aligned(16))) uint8_t gath2[kGathGroup];
  __shared__ __attribute__((aligned(16))) uint8_t gath3[kGathGroup];
  __shared__ __attribute__((aligned(16))) uint8_t dec_p[kGroups * kPGroup];
  // partial sums of the corrections (16 KiB) and the corrections (3 KiB)
  uint8_t* const raw0 = gath0;
  uint8_t* const raw1 = gath1;
  const int ch = blockIdx.x, part = blockIdx.y;
  const int sb = part * p.stages_per_split;
  const int se = min(sb + p.stages_per_split, p.total_stages);
  if (sb >= se) return;
  tri_channel_t<kGather>(p, ch, sb, se, raw0, raw1, dec_p, &d,
                         GathSlots{{gath0, gath1, gath2, gath3}});
}

// Delay compensation for delay spreads up to kRingSpread samples: the sample
// window of each stage is loaded whole into an LDS ring and gathered there.
__global__ __launch_bounds__(kThreads, 1) void xcorr_tri_window_kernel(TriParams p, TriDelays d) {
  __shared__ __attribute__((aligned(16))) uint8_t ring[kRingBytes];
  __shared__ __attribute__((aligned(16))) uint8_t dec_p[kGroups * kPGroup];
  const int ch = blockIdx.x, part = blockIdx.y;
  const int sb = part * p.stages_per_split;
  const int se = min(sb + p.stages_per_split, p.total_stages);
  if (sb >= se) return;
  // after the stage loop the ring holds the corrections' partial sums (raw0)
  // and the corrections (raw1)
  tri_channel_t<kWindow>(p, ch, sb, se, ring, ring + 2 * 8 * kElems * 4, dec_p, &d, GathSlots{});
}

// Several sample segments of each channel summed into one result (the runs of
// one gate of a gated correlation): the same kernel, with the stage loop
// running over the segments' stages.
__global__ __launch_bounds__(kThreads, 1) void xcorr_tri_segments_kernel(TriParams p,
                                                                         TriSegments sg) {
  __shared__ __attribute__((aligned(16))) uint8_t raw0[kRawBytes];
  __shared__ __attribute__((aligned(16))) uint8_t raw1[kRawBytes];
  __shared__ __attribute__((aligned(16))) uint8_t dec_p[kGroups * kPGroup];
  const int ch = blockIdx.x, part = blockIdx.y;
  const int sb = part * p.stages_per_split;
  const int se = min(sb + p.stages_per_split, p.total_stages);
  if (sb >= se) return;
  tri_channel_t<kSegments>(p, ch, sb, se, raw0, raw1, dec_p, nullptr, GathSlots{}, &sg);
}

__global__ __launch_bounds__(kThreads, 1) void xcorr_tri_kernel(TriParams p) {
  // Each raw buffer is its own variable: the compiler then tracks the loads
  // into one separately from reads of the other and waits only for those.
  __shared__ __attribute__((aligned(16))) uint8_t raw0[kRawBytes];
  __shared__ __attribute__((aligned(16))) uint8_t raw1[kRawBytes];
  __shared__ __attribute__((aligned(16))) uint8_t dec_p[kGroups * kPGroup];  // 64 KiB
  // Two waves per SIMD: 256 registers per wave. The accumulators (up to 160)
  // stay in ordinary VGPRs; the compiler's default split when AGPRs are in
  // use (128 + 128) could not hold them.
  // grid x = channel, y = part of the time axis: no integer division, so
  // every index below stays in scalar registers
  const int ch = blockIdx.x, part = blockIdx.y;
  const int sb = part * p.stages_per_split;
  const int se = min(sb + p.stages_per_split, p.total_stages);
  if (sb >= se) return;
  tri_channel(p, ch, sb, se, raw0, raw1, dec_p);
}

}  // namespace

int tri_max_elements() { return kElems; }

hipError_t launch_tri_delayed(const uint8_t* in, int32_t* vis, int n, int f, int t,
                              const int32_t* delays, int max_delay, int accumulate, int split,
                              hipStream_t stream) {
  if (n < 1 || n > kElems || t < kStage || t % kStage != 0) return hipErrorInvalidValue;
  if (max_delay < 0 || max_delay > 65535) return hipErrorInvalidValue;
  TriDelays d;
  d.max_delay = max_delay;
  int dmin = max_delay, dmax = 0;
  for (int e = 0; e < kElems; ++e) {
    const int v = e < n ? delays[e] : 0;
    if (v < 0 || v > max_delay) return hipErrorInvalidValue;
    d.delay[e] = (uint16_t)v;
    if (e < n) {
      dmin = v < dmin ? v : dmin;
      dmax = v > dmax ? v : dmax;
    }
  }
  d.lo = max_delay - dmax;
  d.hi = max_delay - dmin;
  // Dword loads (the dense kernel and the ring) need n % 4 == 0 and a 4-byte
  // aligned input; otherwise every element is gathered bytewise.
  const bool dwords = n % 4 == 0 && reinterpret_cast<uintptr_t>(in) % 4 == 0;
  // One common delay shifts every stream alike: the plain correlation of the
  // samples [max_delay - delay, max_delay - delay + t) of each channel.
  if (dwords && dmin == dmax)
    return launch_tri(in, vis, n, f, t + max_delay, n, (int64_t)(t + max_delay) * n,
                      max_delay - dmin, t, accumulate, split, stream);
  const bool window = d.hi - d.lo <= kRingSpread && dwords;
  TriParams p;
  p.in = in;
  p.vis = vis;
  p.n = n;
  p.e0 = 0;
  p.n_total = p.n;
  p.f = f;
  p.t = t + max_delay;
  p.ss = n;
  p.cs = (int64_t)(t + max_delay) * n;
  p.t0 = 0;
  p.t_end = t;
  p.total_stages = t / kStage;
  if (split < 1) split = 1;
  if (split > p.total_stages) split = p.total_stages;
  p.split = split;
  p.stages_per_split = (p.total_stages + split - 1) / split;
  p.accumulate = accumulate;
  p.atomic_out = split > 1;
  if (f <= 0 || split > 65535) return hipErrorInvalidConfiguration;
  if (window)
    xcorr_tri_window_kernel<<<dim3((unsigned)f, (unsigned)split), dim3(kThreads), 0, stream>>>(p,
                                                                                            d);
  else
    xcorr_tri_delay_kernel<<<dim3((unsigned)f, (unsigned)split), dim3(kThreads), 0, stream>>>(p,
                                                                                           d);
  return hipGetLastError();
}

int tri_max_segments() { return kMaxSegments; }

hipError_t launch_tri_segments(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                               int64_t cs, const int32_t* seg_t0, const int32_t* seg_t_end,
                               int count, int accumulate, int split, hipStream_t stream) {
  if (n < 1 || n > kElems || n % 4 != 0) return hipErrorInvalidValue;
  if (count < 1 || count > kMaxSegments) return hipErrorInvalidValue;
  TriSegments sg;
  sg.count = count;
  int stages = 0;
  for (int k = 0; k < count; ++k) {
    if (seg_t0[k] < 0 || seg_t_end[k] <= seg_t0[k] || seg_t_end[k] > t)
      return hipErrorInvalidValue;
    sg.t0[k] = seg_t0[k];
    sg.t_end[k] = seg_t_end[k];
    sg.stage0[k] = stages;
    stages += (seg_t_end[k] - seg_t0[k] + kStage - 1) / kStage;
  }
  sg.stage0[count] = stages;
  for (int k = count; k < kMaxSegments; ++k) sg.t0[k] = sg.t_end[k] = 0;
  TriParams p;
  p.in = in;
  p.vis = vis;
  p.n = n;
  p.e0 = 0;
  p.n_total = p.n;
  p.f = f;
  p.t = t;
  p.ss = ss;
  p.cs = cs;
  p.t0 = 0;
  p.t_end = t;
  p.total_stages = stages;
  if (split < 1) split = 1;
  if (split > stages) split = stages;
  p.split = split;
  p.stages_per_split = (stages + split - 1) / split;
  p.accumulate = accumulate;
  p.atomic_out = split > 1;
  if (f <= 0 || split > 65535) return hipErrorInvalidConfiguration;
  xcorr_tri_segments_kernel<<<dim3((unsigned)f, (unsigned)split), dim3(kThreads), 0, stream>>>(
      p, sg);
  return hipGetLastError();
}

int tri_stage_samples() { return kStage; }

hipError_t launch_tri(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                      int64_t cs, int t0, int t_count, int accumulate, int split,
                      hipStream_t stream) {
  if (n < 1 || n > kElems || n % 4 != 0) return hipErrorInvalidValue;
  if (t_count <= 0 || t0 < 0 || (int64_t)t0 + t_count > t) return hipErrorInvalidValue;
  TriParams p;
  p.in = in;
  p.vis = vis;
  p.n = n;
  p.e0 = 0;
  p.n_total = p.n;
  p.f = f;
  p.t = t;
  p.ss = ss;
  p.cs = cs;
  p.t0 = t0;
  p.t_end = t0 + t_count;
  p.total_stages = (t_count + kStage - 1) / kStage;
  if (split < 1) split = 1;
  if (split > p.total_stages) split = p.total_stages;
  p.split = split;
  p.stages_per_split = (p.total_stages + split - 1) / split;
  p.accumulate = accumulate;
  p.atomic_out = split > 1;
  if (f <= 0 || split > 65535) return hipErrorInvalidConfiguration;
  xcorr_tri_kernel<<<dim3((unsigned)f, (unsigned)split), dim3(kThreads), 0, stream>>>(p);
  return hipGetLastError();
}

}  // namespace xeng
