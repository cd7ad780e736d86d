// xcorr_tri_bf6_run.h -- the bf6 triangle kernel's per-wave routine (internal):
// the 8 x 8 block triangle of 256 elements (e0 .. e0 + 255 of an array of
// n_total elements) on the f8f6f4 matrix cores with bf6 operands. Used by the
// bf6 triangle kernel (e0 = 0) and by the bf6 form of the rect kernel's
// diagonal squares.
//
// The 4-bit values x in [-8, 7] (Sec. III) are integers of at most four
// significant bits, so the 6-bit float format E3M2 (bf6: sign, 3 exponent bits
// with bias 3, 2 mantissa bits) holds each of them exactly, and
// v_mfma_scale_f32_32x32x64_f8f6f4 multiplies them exactly. Its fp32
// accumulators stay exact while every partial sum is an integer below 2^24:
// one sample adds at most |Re| = 128 (or |Im| = 128), so a workgroup sums at
// most kMaxStagesPerPart stages (131 008 samples).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "xcorr_device.h"
#include "xcorr_tri_common.h"

namespace xeng {
namespace tri {

typedef int v3i __attribute__((ext_vector_type(3)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef unsigned int v16u __attribute__((ext_vector_type(16)));
typedef unsigned int v6u __attribute__((ext_vector_type(6)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef _Float16 v32h __attribute__((ext_vector_type(32)));

constexpr int kStepSamples = 32;                     // samples per bf6 MFMA step
constexpr int kSteps = kStage / kStepSamples;        // 2 steps per stage
constexpr int kCell = 16;                            // LDS bytes per element and slot
constexpr int kPlane = kElems * kCell;               // one slot of all elements (4 KiB)
constexpr int kDHalf = 2 * kPlane;                   // one lane half of one step (8 KiB)
constexpr int kDStep = 2 * kDHalf;
constexpr int kDBuf = kSteps * kDStep;               // one stage (32 KiB)
constexpr int kDecBytes = 2 * kDBuf;                 // double-buffered (64 KiB)
// at most 128 * 64 * 2047 < 2^24 in any fp32 accumulator
constexpr int kMaxStagesPerPart = 2047;
// E8M0 scale exponent 127: scale factor 1
constexpr int kScaleOne = 127;
constexpr int kFmtBf6 = 3;

__device__ inline uint32_t f16_pair(uint32_t t, uint32_t mask, uint32_t bits, _Float16 off) {
  // (t & mask) | bits is the f16 pair 2^E + u (u the field); adding -(2^E + 8)
  // gives u - 8 exactly
  h2 v = __builtin_bit_cast(h2, (t & mask) | bits);
  v = v + h2{off, off};
  return __builtin_bit_cast(uint32_t, v);
}

// Q of a bf6 operand (for Im = Q . P): per 3-dword slot (d0, d1, d2) =
// [Re 48 bits | Im 48 bits] it is [Im | -Re], the sign bit (bit 5 of each
// 6-bit code) of the Re codes flipped.
__device__ __forceinline__ v8i bf6_q(const v8i& pa) {
  const uint32_t p0 = pa[0], p1 = pa[1], p2 = pa[2], p3 = pa[3], p4 = pa[4], p5 = pa[5];
  return v8i{(int)__builtin_amdgcn_alignbit(p2, p1, 16),
             (int)(__builtin_amdgcn_alignbit(p0, p2, 16) ^ 0x08200000u),
             (int)(__builtin_amdgcn_alignbit(p1, p0, 16) ^ 0x82082082u),
             (int)__builtin_amdgcn_alignbit(p5, p4, 16),
             (int)(__builtin_amdgcn_alignbit(p3, p5, 16) ^ 0x08200000u),
             (int)(__builtin_amdgcn_alignbit(p4, p3, 16) ^ 0x82082082u),
             (int)p5,
             (int)p5};   // dwords 6, 7 are not read for bf6
}

template <class Prog>
__device__ __forceinline__ void tri_run_bf6(const TriParams& p, int ch, int base, int sb, int se,
                                            uint8_t* raw0, uint8_t* raw1, uint8_t* dec) {
  constexpr int kNP = Prog::kNP, kNS = Prog::kNS;
  // The five-block program (row block 0 against blocks 0..4, 160
  // accumulators) only multiplies; the four-block wave of the same SIMD loads
  // and decodes the sample rows of both (rows of waves s and s + 4).
  constexpr bool kMultiplyOnly = kNS > 4;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int vw0 = wave & 3, vw1 = vw0 + 4;   // the two row groups a four-block wave serves
  const int half = lane >> 5, l32 = lane & 31;
  const int n = p.n;
  const uint8_t* chan = p.in + (int64_t)ch * p.cs;
  const int64_t ss = p.ss;

  // ---- loads (as in the int8 triangle kernel): rows 8*vw .. 8*vw+7 of a
  // stage, four elements per lane, 8 loads per row group and stage; rows past
  // the end of this workgroup's samples read 0x00
  const uint32_t voff = (4 * lane < n) ? (uint32_t)(p.e0 + 4 * lane) : kOob;
  const int t_stop = min(p.t_end, p.t0 + se * kStage);
  auto fetch = [&](uint8_t* raw, int st, int vw) {
    const int first = __builtin_amdgcn_readfirstlane(p.t0 + st * kStage + 8 * vw);
    const int64_t bytes = t_stop > first ? (int64_t)(t_stop - first - 1) * ss + p.e0 + n : 0;
    const int records = bytes <= 0 ? 0 : (bytes > 0x7fffffff ? 0x7fffffff : (int)bytes);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(chan + (int64_t)first * ss), 0, records, 0x00020000);
#pragma unroll
    for (int r = 0; r < 8; ++r)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rs, (lds_void_ptr)(raw + (8 * vw + r) * kRawStride), 4, voff + (uint32_t)(r * ss), 0,
          0, 0);
  };
  // both row groups: 16 loads per stage
  auto fetch2 = [&](uint8_t* raw, int st) {
    fetch(raw, st, vw0);
    fetch(raw, st, vw1);
  };
  // transposing read i of row group vw: lane gets element 64*i + lane, byte
  // m = sample m of the group's 8 rows
  const int lq = lane & 15;
  const int tr_off = (lq >> 1) * kRawStride + 16 * ((lane >> 4) & 3) + 8 * (lq & 1);
  auto tr_read = [&](const uint8_t* raw, int vw, int i) {
    return __builtin_amdgcn_ds_read_tr8_b64_v2i32(
        (lds_v2i_ptr)(raw + 8 * vw * kRawStride + tr_off + 64 * i));
  };

  // ---- decode: row group vw fills slot vw & 1 of step vw >> 2, lane half
  // (vw >> 1) & 1; element groups i0 and i0 + 1 (elements 64*i + lane) are
  // converted together. Slot s of element e: 12 bytes at 16 e of plane s (a
  // 16-byte lane stride: no bank conflicts for the 12-byte stores and loads).
  // Addresses into dec are formed as one offset from the array
  // (not a chain of pointer steps): the compiler then keeps each access's link
  // to its LDS array and does not make these stores wait for the loads into
  // the raw buffers.
  auto wr_off = [&](int vw) {
    return (vw >> 2) * kDStep + ((vw >> 1) & 1) * kDHalf + (vw & 1) * kPlane + lane * kCell;
  };
  // A word holds samples 0..3 (x) or 4..7 (y) of an element, one per byte;
  // the word and the word shifted right by 8 hold samples (0, 2) and (1, 3) in
  // the low bytes of their two halves (the sample order inside a slot is the
  // same for every element, so any fixed order will do). Re is then 64 + u as
  // f16, Im 1024 + u. One of the two constants of each mask-and-insert lives
  // in a register, so that it is a single v_and_or_b32 (an instruction with
  // three operands takes at most one constant).
  uint32_t re_bits = 0x54005400u, im_bits = 0x64006400u;
  asm volatile("; f16 exponent bits held in registers" : "+v"(re_bits), "+v"(im_bits));
  auto re16 = [&](uint32_t t) { return f16_pair(t, 0x00F000F0u, re_bits, (_Float16)-72.0f); };
  auto im16 = [&](uint32_t t) { return f16_pair(t, 0x000F000Fu, im_bits, (_Float16)-1032.0f); };
  auto decode_pair = [&](int vw, v2i wa, v2i wb, int buf, int i0) {
    const uint32_t a0 = (uint32_t)wa.x, a1 = (uint32_t)wa.x >> 8;
    const uint32_t a2 = (uint32_t)wa.y, a3 = (uint32_t)wa.y >> 8;
    const uint32_t b0 = (uint32_t)wb.x, b1 = (uint32_t)wb.x >> 8;
    const uint32_t b2 = (uint32_t)wb.y, b3 = (uint32_t)wb.y >> 8;
    const v16u u = {re16(a0), re16(a1), re16(a2), re16(a3), im16(a0), im16(a1), im16(a2), im16(a3),
                    re16(b0), re16(b1), re16(b2), re16(b3), im16(b0), im16(b1), im16(b2), im16(b3)};
    const v6u b = __builtin_amdgcn_cvt_scalef32_pk32_bf6_f16(__builtin_bit_cast(v32h, u), 1.0f);
    const int o = wr_off(vw) + buf * kDBuf;
    *reinterpret_cast<v3i*>(dec + (o + 64 * i0 * kCell)) = v3i{(int)b[0], (int)b[1], (int)b[2]};
    *reinterpret_cast<v3i*>(dec + (o + 64 * (i0 + 1) * kCell)) =
        v3i{(int)b[3], (int)b[4], (int)b[5]};
  };

  // ---- MFMA operands: lane half h reads its 6 dwords of element 32*block + l32
  const int rd_off = half * kDHalf + (32 * base + l32) * kCell;
  // one operand per block: dwords 0..5 hold the 32 bf6 codes (6 and 7 unused)
  struct Frags {
    v8i f[kNP];
  };
  auto load_frags = [&](Frags& fr, int buf, int step) {
#pragma unroll
    for (int k = 0; k < kNP; ++k) {
      const int o = buf * kDBuf + step * kDStep;
      const v3i x = *reinterpret_cast<const v3i*>(dec + (rd_off + o + Prog::p[k] * 32 * kCell));
      const v3i y =
          *reinterpret_cast<const v3i*>(dec + (rd_off + o + Prog::p[k] * 32 * kCell + kPlane));
      fr.f[k] = __builtin_shufflevector(x, y, 0, 1, 2, 3, 4, 5, -1, -1);
    }
  };
  v16f acc_re[kNS], acc_im[kNS];
#pragma unroll
  for (int s = 0; s < kNS; ++s) {
    acc_re[s] = v16f{};
    acc_im[s] = v16f{};
  }
  auto q_of = [](const v8i& pa) { return bf6_q(pa); };
  auto mfma_pair = [&](const v8i& pa, const v8i& qa, const v8i& pb, int s) {
    acc_re[s] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
        pa, pb, acc_re[s], kFmtBf6, kFmtBf6, 0, kScaleOne, 0, kScaleOne);
    acc_im[s] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
        qa, pb, acc_im[s], kFmtBf6, kFmtBf6, 0, kScaleOne, 0, kScaleOne);
  };
  auto mfma_step = [&](const Frags& fr) {
#pragma unroll
    for (int s = 0; s < kNS; ++s) {
      const v8i pa = fr.f[Prog::sa[s]];
      mfma_pair(pa, q_of(pa), fr.f[Prog::sb[s]], s);
    }
  };
  // The five-block program (row block 0 against blocks 0..4): column operands
  // are read one block ahead of their MFMAs instead of all at once, so that
  // only three operands and Q are held next to the 160 accumulators.
  auto load_frag = [&](int buf, int step, int k) {
    const int o = rd_off + buf * kDBuf + step * kDStep + Prog::p[k] * 32 * kCell;
    const v3i x = *reinterpret_cast<const v3i*>(dec + o);
    const v3i y = *reinterpret_cast<const v3i*>(dec + (o + kPlane));
    return v8i(__builtin_shufflevector(x, y, 0, 1, 2, 3, 4, 5, -1, -1));
  };
  auto stream_step = [&](int buf, int step) {
    const v8i f0 = load_frag(buf, step, 0);
    v8i nxt = load_frag(buf, step, 1);
    const v8i q = q_of(f0);
    mfma_pair(f0, q, f0, 0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 1; c < kNS; ++c) {
      const v8i cur = nxt;
      if (c + 1 < kNS) nxt = load_frag(buf, step, c + 1);
      mfma_pair(f0, q, cur, c);
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  // One stage st. Four-block waves: load both row groups of st+2, then two
  // steps, each reading one row group of st+1 back transposed, decoding it
  // into the other buffer and multiplying one step of st. Five-block waves:
  // the two MFMA steps only. Stages past se are loaded and
  // decoded but never multiplied.
  auto body = [&](auto par, int st) {
    constexpr int kPar = decltype(par)::value;
    uint8_t* const raw_ld = kPar ? raw1 : raw0;
    const uint8_t* const raw_dc = kPar ? raw0 : raw1;
    if (kMultiplyOnly) {
      stream_step(kPar, 0);
      stream_step(kPar, 1);
    } else {
      fetch2(raw_ld, st + 2);
      vm_wait<16>();   // all but the 16 loads just issued are done: rows of st+1 are in LDS
      // step g multiplies step g of st while it decodes row group g of st+1
      // into the other buffer: the decode's VALU work fills the MFMA issue gaps
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int vw = g ? vw1 : vw0;
        const v2i a0 = tr_read(raw_dc, vw, 0), a1 = tr_read(raw_dc, vw, 1);
        const v2i a2 = tr_read(raw_dc, vw, 2), a3 = tr_read(raw_dc, vw, 3);
        Frags fr;
        load_frags(fr, kPar, g);
        decode_pair(vw, a0, a1, kPar ^ 1, 0);
        decode_pair(vw, a2, a3, kPar ^ 1, 2);
        mfma_step(fr);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    lds_barrier();
  };

  if (!kMultiplyOnly) {
    fetch2(raw0, sb);
    fetch2(raw1, sb + 1);
    vm_wait<16>();
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int vw = g ? vw1 : vw0;
      decode_pair(vw, tr_read(raw0, vw, 0), tr_read(raw0, vw, 1), 0, 0);
      decode_pair(vw, tr_read(raw0, vw, 2), tr_read(raw0, vw, 3), 0, 2);
    }
  }
  lds_barrier();
  int st = sb;
  for (; st + 1 < se; st += 2) {
    body(std::integral_constant<int, 0>{}, st);
    body(std::integral_constant<int, 1>{}, st + 1);
  }
  if (st < se) body(std::integral_constant<int, 0>{}, st);
  // the loads of the two stages past se may still be writing LDS: let them
  // land before the workgroup ends and releases its LDS
  vm_wait<0>();
  lds_barrier();

  // samples summed, and the padding samples among the stages multiplied
  const int t_sum = max(0, t_stop - (p.t0 + sb * kStage));
  const int pad = (se - sb) * kStage - t_sum;
  const int re_pad = 128 * pad;

  // ---- epilogue: masked writes of i <= j < n into the packed triangle;
  // entries are indexed in the whole array (p.n_total elements), this
  // triangle covers elements p.e0 .. p.e0 + n - 1
  const int64_t n64 = p.n_total;
  const int64_t entries = n64 * (n64 + 1) / 2;
  int32_t* out = p.vis + (int64_t)ch * entries * 2;
  auto store_all = [&](auto mode) {
    constexpr int kMode = decltype(mode)::value;   // 0 store, 1 add, 2 atomic add
#pragma unroll
    for (int s = 0; s < kNS; ++s) {
      const int rb = base + Prog::p[Prog::sa[s]], cb = base + Prog::p[Prog::sb[s]];
      const int j = 32 * cb + l32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = 32 * rb + 8 * (r >> 2) + 4 * half + (r & 3);
        if (i <= j && j < n) {
          int32_t* o = out + 2 * tri_index(n64, p.e0 + i, p.e0 + j);
          // integers below 2^24 in magnitude: the conversion is exact
          const int re = (int)acc_re[s][r] - re_pad;
          const int im = (int)acc_im[s][r];
          if (kMode == 2) {
            atomicAdd(o, re);
            atomicAdd(o + 1, im);
          } else if (kMode == 1) {
            const v2i old = *reinterpret_cast<const v2i*>(o);
            *reinterpret_cast<v2i*>(o) = v2i{old.x + re, old.y + im};
          } else {
            *reinterpret_cast<v2i*>(o) = v2i{re, im};
          }
        }
      }
    }
  };
  if (p.atomic_out)
    store_all(std::integral_constant<int, 2>{});
  else if (p.accumulate)
    store_all(std::integral_constant<int, 1>{});
  else
    store_all(std::integral_constant<int, 0>{});
}


}  // namespace tri
}  // namespace xeng
