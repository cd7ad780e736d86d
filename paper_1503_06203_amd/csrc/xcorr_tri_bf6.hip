// xcorr_tri_bf6.hip -- the triangle kernel (N <= 256, one workgroup per
// channel) on the f8f6f4 matrix cores with bf6 operands.
//
// The 4-bit values x in [-8, 7] (Sec. III) are integers of at most four
// significant bits, so the 6-bit float format E3M2 (bf6: sign, 3 exponent bits
// with bias 3, 2 mantissa bits) holds each of them exactly, and
// v_mfma_scale_f32_32x32x64_f8f6f4 multiplies them exactly. Its fp32
// accumulators stay exact while every partial sum is an integer below 2^24:
// one sample adds at most |Re| = 128 (or |Im| = 128), so a workgroup sums at
// most kMaxStagesPerPart stages (131 008 samples) and longer runs are split
// along time. The result, converted to int32 at the end, is the same Eq. 1
// sum the int8 kernels produce, bit for bit.
//
// One bf6 step takes 64 values per output element pair and lane-pair: 32
// samples of (Re, Im), twice the samples of an int8 step, at the same issue
// cost, and needs no offset corrections because the signed values are
// multiplied directly (Eq. 2 form):
//   Re V_ij = P_i . P_j,  Im V_ij = Q_i . P_j,
//   P = [Re s0..s7, Im s0..s7] per 8-sample slot, Q = [Im s0..s7, -Re s0..s7].
//
// Shape: as the int8 triangle kernel (8 waves, two per SIMD, the same block
// programs, HBM -> LDS loads two stages ahead, ds_read_b64_tr_b8 transposes).
// Decode: a wave turns its 8 samples of an element into f16 values with one
// mask-and-insert and one packed f16 add per pair of values, and the hardware
// packs 32 of them (two elements) into 6 dwords of bf6 codes
// (v_cvt_scalef32_pk32_bf6_f16). A fragment of one element for one lane half
// and step is 6 dwords = two 3-dword slots, one per wave: slot w & 1 of step
// w >> 2, lane half (w >> 1) & 1; slot s of all elements is a plane of
// 16-byte cells, so a slot is written with one 12-byte store per element and
// a lane reads its operand with two 12-byte loads, both at a 16-byte lane
// stride. Q is formed from P in registers: three
// funnel shifts and two sign flips per slot.
//
// Padding: sample rows past the end of the data load as 0x00, which decodes
// to (-8, -8); each such sample adds 128 to Re and 0 to Im of every pair and
// is subtracted at the end.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "xcorr_device.h"
#include "xcorr_launch.h"
#include "xcorr_tri_common.h"
#include "xcorr_tri_bf6_run.h"

namespace xeng {

namespace {

using namespace tri;

__global__ __launch_bounds__(kThreads, 1) void xcorr_tri_bf6_kernel(TriParams p) {
  __shared__ __attribute__((aligned(16))) uint8_t raw0[kRawBytes];
  __shared__ __attribute__((aligned(16))) uint8_t raw1[kRawBytes];
  __shared__ __attribute__((aligned(16))) uint8_t dec[kDecBytes];
  const int ch = blockIdx.x, part = blockIdx.y;
  const int sb = part * p.stages_per_split;
  const int se = min(sb + p.stages_per_split, p.total_stages);
  if (sb >= se) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int simd = wave & 3;
  if (wave < 4) {
    tri_run_bf6<ProgA>(p, ch, simd, sb, se, raw0, raw1, dec);
  } else {
    switch (simd) {
      case 0: tri_run_bf6<ProgB<0>>(p, ch, 0, sb, se, raw0, raw1, dec); break;
      case 1: tri_run_bf6<ProgB<1>>(p, ch, 0, sb, se, raw0, raw1, dec); break;
      case 2: tri_run_bf6<ProgB<2>>(p, ch, 0, sb, se, raw0, raw1, dec); break;
      default: tri_run_bf6<ProgB<3>>(p, ch, 0, sb, se, raw0, raw1, dec); break;
    }
  }
}

}  // namespace

int tri_bf6_min_split(int64_t t_count) {
  const int64_t stages = (t_count + kStage - 1) / kStage;
  return (int)((stages + kMaxStagesPerPart - 1) / kMaxStagesPerPart);
}

hipError_t launch_tri_bf6(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
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
  // the caller sizes split so that no part exceeds the exact fp32 range
  if (p.stages_per_split > kMaxStagesPerPart) return hipErrorInvalidValue;
  p.accumulate = accumulate;
  p.atomic_out = split > 1;
  if (f <= 0 || split > 65535) return hipErrorInvalidConfiguration;
  xcorr_tri_bf6_kernel<<<dim3((unsigned)f, (unsigned)split), dim3(kThreads), 0, stream>>>(p);
  return hipGetLastError();
}

}  // namespace xeng
