// xcorr_tri_run.h -- one wave's share of the triangle kernel (paper Sec. II-C,
// Fig. 1: the 8 x 8 triangle of 32 x 32 blocks of 256 elements), its staging
// pipeline, decode, offset corrections (Sec. III-A, Eq. 3) and masked epilogue.
// Shared by the triangle kernels (n <= 256) and by the kernel for larger
// arrays, whose diagonal 256-element squares are such triangles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "xcorr_device.h"
#include "xcorr_tri_common.h"

namespace xeng {
namespace tri {

constexpr int kPBuf = kElems * 16;              // P slabs of one 8-sample group, one buffer
constexpr int kPGroup = 2 * kPBuf;              // a group's slabs in both buffers
constexpr int kGroups = kStage / 8;             // 8-sample groups per stage (= waves)
// delay compensation: a 256-byte slot per (element group, row) and wave, one
// LDS array per element group
constexpr int kGathSlot = 64 * 4;
constexpr int kGathWave = 8 * kGathSlot;
constexpr int kGathGroup = 8 * kGathWave;           // 16 KiB per element group
// after the stage loop the corrections reuse two groups: the per-wave partial
// field sums (2 x 8 waves x 256 words) and the three correction rows
static_assert(kGathGroup >= 2 * 8 * kElems * 4 && kGathGroup >= 3 * kElems * 4,
              "the corrections fit the gather slots");
struct GathSlots {
  uint8_t* g[4];
};
// Per-element sample delays (delay compensation): element e at output sample t
// reads input sample t + max_delay - delay[e]; the input holds max_delay halo
// samples before the first output sample.
struct TriDelays {
  int max_delay;
  int lo, hi;   // smallest and largest max_delay - delay[e] over the elements
  uint16_t delay[kElems];
};
// Delay compensation with a bounded spread (hi - lo <= kRingSpread): the
// sample rows an output stage needs, [st*64 + lo, st*64 + 64 + hi), are loaded
// whole (coalesced, like the dense form) into a ring of kRingRows rows in LDS,
// and each lane gathers its elements' bytes from there. Slot k of the ring
// holds rows congruent to k modulo kRingRows; the first kRingGuard slots are
// also written after the last one, so the 8 consecutive rows a gather reads
// never wrap. A row stride of 65 dwords spreads the bytes of different rows
// over the LDS banks.
constexpr int kRingRows = 256;
constexpr int kRingGuard = 7;
constexpr int kRingStride = kElems + 4;
constexpr int kRingBytes = ((kRingRows + kRingGuard) * kRingStride + 15) / 16 * 16;
constexpr int kRingSpread = kRingRows - 2 * kStage;   // the window and the rows loaded ahead
static_assert(kRingBytes >= 2 * 8 * kElems * 4 + 4096, "the corrections fit the ring");
// Sample segments (gated correlation): the workgroup sums the samples
// [t0[k], t_end[k]) of every segment k; segment k covers the stages
// [stage0[k], stage0[k+1]) of the stage loop, each stage 64 samples of one
// segment (the last one of a segment may be partial).
constexpr int kMaxSegments = 32;
struct TriSegments {
  int count;
  int t0[kMaxSegments];
  int t_end[kMaxSegments];
  int stage0[kMaxSegments + 1];
};
// modes of the triangle kernel: dense, the two delay forms, sample segments
constexpr int kDense = 0, kGather = 1, kWindow = 2, kSegments = 3;


// The block programs of the two waves of a SIMD, balanced: ProgA's 5 blocks
// and ProgB's 4 (the 9 blocks of SIMD s), except that block (s, s + 4) is
// split along the time axis, the first wave multiplying it over the first
// two MFMA steps of each stage (kHalfKs = 0) and the second over the last two
// (kHalfKs = 2). The second wave hands its partial sums to the first before
// the output is written (kSend). Each wave then issues 36 MFMAs per stage
// instead of 40 and 32, so neither waits at the stage barrier while the
// other still multiplies (about 2 % faster at N = 256).
struct BalancedA {
  static constexpr int kNP = 5, kNS = 5;
  static constexpr int p[kNP] = {0, 1, 2, 3, 4};
  static constexpr int sa[kNS] = {0, 0, 0, 0, 0};
  static constexpr int sb[kNS] = {0, 1, 2, 3, 4};
  static constexpr int kHalf = 4, kHalfKs = 0;
  static constexpr bool kSend = false;
};
template <int S>
struct BalancedB;
template <>
struct BalancedB<0> {  // (0,5) (0,6) (0,7) (7,7) + (0,4) late half
  static constexpr int kNP = 5, kNS = 5;
  static constexpr int p[kNP] = {0, 5, 6, 7, 4};
  static constexpr int sa[kNS] = {0, 0, 0, 3, 0};
  static constexpr int sb[kNS] = {1, 2, 3, 3, 4};
  static constexpr int kHalf = 4, kHalfKs = 2;
  static constexpr bool kSend = true;
};
template <>
struct BalancedB<1> {  // (1,6) (1,7) (6,6) (6,7) + (1,5) late half
  static constexpr int kNP = 4, kNS = 5;
  static constexpr int p[kNP] = {1, 6, 7, 5};
  static constexpr int sa[kNS] = {0, 0, 1, 1, 0};
  static constexpr int sb[kNS] = {1, 2, 1, 2, 3};
  static constexpr int kHalf = 4, kHalfKs = 2;
  static constexpr bool kSend = true;
};
template <>
struct BalancedB<2> {  // (2,7) (5,5) (5,6) (5,7) + (2,6) late half
  static constexpr int kNP = 4, kNS = 5;
  static constexpr int p[kNP] = {2, 5, 6, 7};
  static constexpr int sa[kNS] = {0, 1, 1, 1, 0};
  static constexpr int sb[kNS] = {3, 1, 2, 3, 2};
  static constexpr int kHalf = 4, kHalfKs = 2;
  static constexpr bool kSend = true;
};
template <>
struct BalancedB<3> {  // (4,4) (4,5) (4,6) (4,7) + (3,7) late half
  static constexpr int kNP = 5, kNS = 5;
  static constexpr int p[kNP] = {4, 5, 6, 7, 3};
  static constexpr int sa[kNS] = {0, 0, 0, 0, 4};
  static constexpr int sb[kNS] = {0, 1, 2, 3, 3};
  static constexpr int kHalf = 4, kHalfKs = 2;
  static constexpr bool kSend = true;
};

template <class Prog, int kMode = kDense>
__device__ __forceinline__ void tri_run(const TriParams& p, int ch, int base, int sb, int se,
                                        uint8_t* raw0, uint8_t* raw1, uint8_t* dec_p,
                                        const TriDelays* dl = nullptr, GathSlots gs = {},
                                        const TriSegments* sg = nullptr) {
  constexpr int kNP = Prog::kNP, kNS = Prog::kNS;
  constexpr bool kDelay = kMode == kGather;
  const int tid = opaque_tid();
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int half = lane >> 5, l32 = lane & 31;
  const int n = p.n;
  const uint8_t* chan = p.in + (int64_t)ch * p.cs;
  const int64_t ss = p.ss;

  // ---- loads: this wave fetches sample rows 8*wave .. 8*wave+7 of a stage; a
  // lane carries four elements. Every stage issues exactly 8 loads per wave
  // (the waits below count on it): the buffer descriptor's record count ends
  // at the end of this workgroup's samples (t_end, or the end of stage se), so
  // rows past it read nothing and stay 0x00, which adds nothing; lanes past n
  // use an offset beyond every record.
  const uint32_t voff = (4 * lane < n) ? (uint32_t)(p.e0 + 4 * lane) : kOob;
  const int t_stop = min(p.t_end, p.t0 + se * kStage);   // samples [t0 + sb*64, t_stop)
  // first sample of stage st and the end of its samples; in the segment mode
  // stages past se (loaded ahead, never multiplied) are empty. The stage loop
  // fetches stages in increasing order, so the segment of the next one is
  // found by moving on from the last one found.
  int seg = 0;
  auto stage_span = [&](int st, int& row0, int& stop) {
    if (kMode == kSegments) {
      int k = seg;
      while (k + 1 < sg->count && sg->stage0[k + 1] <= st) ++k;
      seg = k;
      row0 = sg->t0[k] + (st - sg->stage0[k]) * kStage;
      stop = st < se ? sg->t_end[k] : row0;
    } else {
      row0 = p.t0 + st * kStage;
      stop = t_stop;
    }
  };
  auto fetch = [&](uint8_t* raw, int st) {
    int row0, stop;
    stage_span(st, row0, stop);
    // a sample index (< 2^25) that is uniform across the wave; saying so keeps
    // the buffer descriptor in scalar registers
    const int first = __builtin_amdgcn_readfirstlane(row0 + 8 * wave);
    // up to the end of the last sample row before the stop
    const int64_t bytes = stop > first ? (int64_t)(stop - first - 1) * ss + p.e0 + n : 0;
    const int records = bytes <= 0 ? 0 : (bytes > 0x7fffffff ? 0x7fffffff : (int)bytes);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(chan + (int64_t)first * ss), 0, records, 0x00020000);
#pragma unroll
    for (int r = 0; r < 8; ++r)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rs, (lds_void_ptr)(raw + (8 * wave + r) * kRawStride), 4, voff + (uint32_t)(r * ss), 0,
          0, 0);
  };
  // Delay compensation: each lane gathers the bytes of its own elements
  // e = 64*q + lane, row r of this wave's 8 from input row
  // (row + max_delay - delay[e]), with one-byte loads into LDS. Such a load
  // writes each lane's byte as a zero-extended dword at 4*lane, so every
  // (q, r) pair has a 256-byte slot private to the wave (element group q in
  // LDS array gs.g[q]: the compiler then tracks the loads into one group apart
  // from reads of another), and the lane reads its 8 dwords of group q back and
  // packs their low bytes into the two words a transposing read yields in the
  // dense form. Stages inside [sb, se) are full (the caller guarantees
  // t % 64 == 0); for stages past se every lane uses an offset beyond every
  // record, so the loads write zero bytes, which add nothing.
  uint32_t voff_d[4];
  if (kDelay) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = 64 * q + lane;
      voff_d[q] = e < n ? (uint32_t)((dl->max_delay - (int)dl->delay[e]) * ss + p.e0 + e) : kOob;
    }
  }

  // the 8 loads of element group q of stage st
  auto gather_q = [&](int st, int q) {
    const bool in_range = st < se;
    const int first = __builtin_amdgcn_readfirstlane(p.t0 + (in_range ? st : sb) * kStage + 8 * wave);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(chan + (int64_t)first * ss), 0, 0x7fffffff, 0x00020000);
#pragma unroll
    for (int r = 0; r < 8; ++r)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rs, (lds_void_ptr)(gs.g[q] + wave * kGathWave + r * kGathSlot), 1,
          in_range ? voff_d[q] : kOob,
          (int)(r * ss), 0, 0);
  };
  auto gather_read = [&](int q) {
    uint32_t d[8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
      d[r] = *reinterpret_cast<const uint32_t*>(gs.g[q] + wave * kGathWave + r * kGathSlot +
                                                4 * lane);
    return v2i{(int)(d[0] | (d[1] << 8) | (d[2] << 16) | (d[3] << 24)),
               (int)(d[4] | (d[5] << 8) | (d[6] << 16) | (d[7] << 24))};
  };

  // Window form (kWindow): raw0 is the ring. ring_load(r0, r1) loads rows
  // [r0, r1) of the channel, 8 per wave per round (row r0 + 8*w + r of each
  // round of 64); the descriptor ends at the channel's last row (t rows,
  // halo included), so rows past it read zeros.
  auto ring_load = [&](int r0, int r1) {
    for (int rb = r0; rb < r1; rb += kStage) {
      const int first = __builtin_amdgcn_readfirstlane(rb + 8 * wave);
      const int64_t bytes = (int64_t)(p.t - first) * ss;
      const int records = bytes <= 0 ? 0 : (bytes > 0x7fffffff ? 0x7fffffff : (int)bytes);
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<uint8_t*>(chan + (int64_t)first * ss), 0, records, 0x00020000);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int row = first + r;
        // Rows past the channel's last sample are never gathered by a live
        // stage (the last one reads up to row t - 1), so they are not loaded:
        // every load stays inside the input, whatever the range check makes
        // of the scalar row offset.
        if (row < r1 && row < p.t) {
          const int slot = row & (kRingRows - 1);
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_ptr)(raw0 + slot * kRingStride),
                                                   4, voff, r * (int)ss, 0, 0);
          if (slot < kRingGuard)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rs, (lds_void_ptr)(raw0 + (kRingRows + slot) * kRingStride), 4, voff,
                r * (int)ss, 0, 0);
        }
      }
    }
  };
  // the 8 bytes of element 64*q + lane at this wave's rows of stage st, packed
  // as a transposing read would give them; ring_off[q] = max_delay - delay[e]
  int ring_off[4];
  if (kMode == kWindow) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = 64 * q + lane;
      ring_off[q] = e < n ? dl->max_delay - (int)dl->delay[e] : dl->lo;
    }
  }
  auto ring_gather = [&](int st, int q) {
    const int row0 = st * kStage + 8 * wave + ring_off[q];
    const uint8_t* const a = raw0 + (row0 & (kRingRows - 1)) * kRingStride + 64 * q + lane;
    uint32_t d[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) d[r] = a[r * kRingStride];
    return v2i{(int)(d[0] | (d[1] << 8) | (d[2] << 16) | (d[3] << 24)),
               (int)(d[4] | (d[5] << 8) | (d[6] << 16) | (d[7] << 24))};
  };

  // ---- decode: ds_read_b64_tr_b8 over the wave's 8 rows. In each 16-lane
  // group the even lanes name the rows of elements e0..e0+7 and the odd lanes
  // those of e0+8..e0+15; lane k of the group receives element e0+k, byte m =
  // sample m. Read i covers elements 64*i .. 64*i+63 (lane = element - 64*i).
  const int lq = lane & 15;
  const int tr_off = (8 * wave + (lq >> 1)) * kRawStride + 16 * ((lane >> 4) & 3) + 8 * (lq & 1);
  // stores into dec_p use one offset from the array (not a chain of pointer
  // steps): the compiler then keeps their link to dec_p and does not make
  // them wait for loads into other LDS arrays
  const int wr_off = wave * kPGroup + lane * 16;
  auto tr_read = [&](const uint8_t* raw, int i) {
    return __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i_ptr)(raw + tr_off + 64 * i));
  };
  // Field sums of the lane's elements 64*i + lane over this wave's samples.
  uint32_t sum_re[4] = {0, 0, 0, 0}, sum_im[4] = {0, 0, 0, 0};
  auto decode = [&](v2i w, int buf, int i) {
    const uint32_t ra = fields_hi((uint32_t)w.x), rb = fields_hi((uint32_t)w.y);
    const uint32_t ia = fields_lo((uint32_t)w.x), ib = fields_lo((uint32_t)w.y);
    const v4i ps = {(int)ra, (int)rb, (int)ia, (int)ib};
    *reinterpret_cast<v4i*>(dec_p + (wr_off + buf * kPBuf + i * 1024)) = ps;
    // v_sad_u8 against zero adds the four bytes of a word
    sum_re[i] = __builtin_amdgcn_sad_u8(rb, 0u, __builtin_amdgcn_sad_u8(ra, 0u, sum_re[i]));
    sum_im[i] = __builtin_amdgcn_sad_u8(ib, 0u, __builtin_amdgcn_sad_u8(ia, 0u, sum_im[i]));
  };

  // ---- MFMA operands: lane half h reads group 2*ks + h, element 32*block + l32
  const int rd_off = half * kPGroup + (32 * base + l32) * 16;
  v16i acc_re[kNS], acc_im[kNS];
#pragma unroll
  for (int s = 0; s < kNS; ++s) {
    acc_re[s] = v16i{};
    acc_im[s] = v16i{};
  }
  // Operand fragments of one 16-sample MFMA step.
  struct Frags {
    v4i pf[kNP];
  };
  auto load_frags = [&](Frags& fr, int buf, int ks) {
#pragma unroll
    for (int k = 0; k < kNP; ++k)
      fr.pf[k] = *reinterpret_cast<const v4i*>(
          dec_p + (rd_off + ks * 2 * kPGroup + buf * kPBuf + Prog::p[k] * 512));
  };
  auto mfma_step = [&](const Frags& fr, int ks) {
#pragma unroll
    for (int s = 0; s < kNS; ++s) {
      if (s == Prog::kHalf && (ks < Prog::kHalfKs || ks >= Prog::kHalfKs + 2)) continue;
      const v4i a = fr.pf[Prog::sa[s]];
      const v4i q = {a.z, a.w, (int)((uint32_t)a.x ^ 0x0F0F0F0Fu),
                     (int)((uint32_t)a.y ^ 0x0F0F0F0Fu)};
      const v4i b = fr.pf[Prog::sb[s]];
      acc_re[s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc_re[s], 0, 0, 0);
      acc_im[s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(q, b, acc_im[s], 0, 0, 0);
    }
  };

  // One stage st, software-pipelined: the step-0 fragments are requested
  // first, then (once this wave's loads of st+1, issued a stage earlier, are
  // in) the transposing reads of its rows of st+1; each MFMA step then
  // requests the next step's fragments and overlaps its MFMAs with the decode
  // of one quarter of the elements of st+1 (written to the other operand
  // buffer). The loads of st+2 go out after the first MFMA step, so that the
  // matrix cores start first (about 1 % faster than issuing them before the
  // MFMAs). kPar = (st - sb) & 1 selects the static buffers. Stages past se are fetched and decoded as well (their rows
  // read nothing: zero bytes, which add nothing to the products or the field
  // sums): every stage is the same straight-line code.
  auto body = [&](auto par, int st) {
    constexpr int kPar = decltype(par)::value;
    uint8_t* const raw_ld = kPar ? raw1 : raw0;
    const uint8_t* const raw_dc = kPar ? raw0 : raw1;
    Frags fr[2];
    load_frags(fr[0], kPar, 0);
    vm_wait<0>();   // this wave's loads of st+1 are in LDS
    v2i rawv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) rawv[i] = tr_read(raw_dc, i);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      if (ks < 3) load_frags(fr[(ks + 1) & 1], kPar, ks + 1);
      decode(rawv[ks], kPar ^ 1, ks);
      mfma_step(fr[ks & 1], ks);
      __builtin_amdgcn_sched_barrier(0);
      if (ks == 0) {
        fetch(raw_ld, st + 2);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    lds_barrier();
  };
  // The delayed form: at step ks the wave reads its bytes of element group ks
  // of st+1 (loaded one stage earlier), decodes them and then reuses their
  // slots for the loads of group ks of st+2. Between issuing the loads of a
  // group and reading it back, three groups (24 loads) are issued: the wait
  // count is the same at every step.
  auto body_delayed = [&](auto par, int st) {
    constexpr int kPar = decltype(par)::value;
    Frags fr[2];
    load_frags(fr[0], kPar, 0);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      vm_wait<24>();
      const v2i w = gather_read(ks);
      if (ks < 3) load_frags(fr[(ks + 1) & 1], kPar, ks + 1);
      decode(w, kPar ^ 1, ks);
      // the reads of the slots returned (decode used them): they may be refilled
      __builtin_amdgcn_sched_barrier(0);
      gather_q(st + 2, ks);
      mfma_step(fr[ks & 1], ks);
      __builtin_amdgcn_sched_barrier(0);
    }
    lds_barrier();
  };

  // The window form: at stage st the rows of st+1 are gathered (they were
  // loaded, and every wave waited for its loads, before the previous stage
  // barrier), then the rows that st+2 adds to the window are requested, and
  // every wave waits for its own requests before this stage's barrier. The
  // ring then holds [(st+1)*64 + lo, (st+3)*64 + hi): 128 + hi - lo rows.
  // Stages past se are gathered as zeros (their field sums must stay out).
  auto body_window = [&](auto par, int st) {
    constexpr int kPar = decltype(par)::value;
    Frags fr[2];
    load_frags(fr[0], kPar, 0);
    v2i rawv[4];
    const bool live = st + 1 < se;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const v2i g = ring_gather(st + 1, q);
      rawv[q] = live ? g : v2i{0, 0};
    }
    __builtin_amdgcn_sched_barrier(0);
    ring_load((st + 2) * kStage + dl->hi, (st + 3) * kStage + dl->hi);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      if (ks < 3) load_frags(fr[(ks + 1) & 1], kPar, ks + 1);
      decode(rawv[ks], kPar ^ 1, ks);
      mfma_step(fr[ks & 1], ks);
      __builtin_amdgcn_sched_barrier(0);
    }
    vm_wait<0>();
    lds_barrier();
  };

  if (kMode == kWindow) {
    // the rows of stages sb and sb+1: [sb*64 + lo, (sb+2)*64 + hi)
    ring_load(sb * kStage + dl->lo, (sb + 2) * kStage + dl->hi);
    vm_wait<0>();
    lds_barrier();
#pragma unroll
    for (int q = 0; q < 4; ++q) decode(ring_gather(sb, q), 0, q);
    lds_barrier();
    int st = sb;
    for (; st + 1 < se; st += 2) {
      body_window(std::integral_constant<int, 0>{}, st);
      body_window(std::integral_constant<int, 1>{}, st + 1);
    }
    if (st < se) body_window(std::integral_constant<int, 0>{}, st);
  } else if (!kDelay) {
    // ---- prologue: fetch sb and sb+1, decode sb ----------------------------------
    fetch(raw0, sb);
    fetch(raw1, sb + 1);
    vm_wait<8>();
#pragma unroll
    for (int i = 0; i < 4; ++i) decode(tr_read(raw0, i), 0, i);
    lds_barrier();

    int st = sb;
    for (; st + 1 < se; st += 2) {
      body(std::integral_constant<int, 0>{}, st);
      body(std::integral_constant<int, 1>{}, st + 1);
    }
    if (st < se) body(std::integral_constant<int, 0>{}, st);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) gather_q(sb, q);
    vm_wait<0>();
#pragma unroll
    for (int q = 0; q < 4; ++q) decode(gather_read(q), 0, q);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) gather_q(sb + 1, q);
    lds_barrier();
    int st = sb;
    for (; st + 1 < se; st += 2) {
      body_delayed(std::integral_constant<int, 0>{}, st);
      body_delayed(std::integral_constant<int, 1>{}, st + 1);
    }
    if (st < se) body_delayed(std::integral_constant<int, 0>{}, st);
  }
  // loads issued for the two stages past se may still be writing LDS: let
  // them land (in every wave) before the raw buffers are reused below and
  // before the workgroup moves on or ends and releases its LDS
  vm_wait<0>();
  lds_barrier();
  // the second wave of a SIMD hands its partial sums of the shared block over
  uint32_t* const xch = reinterpret_cast<uint32_t*>(dec_p) + (wave & 3) * (32 * 64);
  if constexpr (Prog::kSend) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      xch[r * 64 + lane] = (uint32_t)acc_re[Prog::kHalf][r];
      xch[(16 + r) * 64 + lane] = (uint32_t)acc_im[Prog::kHalf][r];
    }
  }

  // ---- offset corrections: per element e, from the field sums of all waves,
  // cr_e = 8 (SR_e + SI_e), ci_row_e = 8 (SR_e - SI_e), ci_col_e = 8 SR_e + 7 SI_e
  {
    uint32_t* part = reinterpret_cast<uint32_t*>(raw0);   // [wave][re, im][element]
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      part[(2 * wave) * kElems + 64 * i + lane] = sum_re[i];
      part[(2 * wave + 1) * kElems + 64 * i + lane] = sum_im[i];
    }
  }
  lds_barrier();
  if constexpr (!Prog::kSend) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      acc_re[Prog::kHalf][r] = (int)((uint32_t)acc_re[Prog::kHalf][r] + xch[r * 64 + lane]);
      acc_im[Prog::kHalf][r] = (int)((uint32_t)acc_im[Prog::kHalf][r] + xch[(16 + r) * 64 + lane]);
    }
  }
  int32_t* const corr = reinterpret_cast<int32_t*>(raw1);   // [cr, ci_row, ci_col][element]
  if (tid < kElems) {
    const uint32_t* part = reinterpret_cast<const uint32_t*>(raw0);
    uint32_t sr = 0, si = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
      sr += part[(2 * w) * kElems + tid];
      si += part[(2 * w + 1) * kElems + tid];
    }
    corr[tid] = (int32_t)(8u * (sr + si));
    corr[kElems + tid] = (int32_t)(8u * (sr - si));
    corr[2 * kElems + tid] = (int32_t)(8u * sr + 7u * si);
  }
  lds_barrier();
  // samples this workgroup summed (stages sb..se-1 within t_end)
  int t_sum = max(0, t_stop - (p.t0 + sb * kStage));
  if (kMode == kSegments) {
    // the samples of each segment that fall into stages [sb, se)
    t_sum = 0;
    for (int k = 0; k < sg->count; ++k) {
      const int lo = max(sb, sg->stage0[k]), hi = min(se, sg->stage0[k + 1]);
      if (lo < hi)
        t_sum += min(sg->t_end[k], sg->t0[k] + (hi - sg->stage0[k]) * kStage) -
                 (sg->t0[k] + (lo - sg->stage0[k]) * kStage);
    }
  }
  const uint32_t re_const = 128u * (uint32_t)t_sum;

  // ---- epilogue: masked writes of i <= j < n into the packed triangle ------------
  // entries are indexed in the whole array (p.n_total elements); this
  // triangle covers elements p.e0 .. p.e0 + n - 1
  const int64_t n64 = p.n_total;
  const int64_t entries = n64 * (n64 + 1) / 2;
  int32_t* out = p.vis + (int64_t)ch * entries * 2;
  auto store_all = [&](auto mode) {
    constexpr int kStore = decltype(mode)::value;   // 0 store, 1 add, 2 atomic add
#pragma unroll
    for (int s = 0; s < kNS; ++s) {
      if (Prog::kSend && s == Prog::kHalf) continue;   // added into the partner's sums
      const int rb = base + Prog::p[Prog::sa[s]], cb = base + Prog::p[Prog::sb[s]];
      const int j = 32 * cb + l32;
      const uint32_t re_j = re_const - (uint32_t)corr[j];
      const uint32_t ci_col_j = (uint32_t)corr[2 * kElems + j];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = 32 * rb + 8 * (r >> 2) + 4 * half + (r & 3);
        if (i <= j && j < n) {
          int32_t* o = out + 2 * tri_index(n64, p.e0 + i, p.e0 + j);
          // int32 arithmetic modulo 2^32 (unsigned): exact for the result
          const int re = (int)((uint32_t)acc_re[s][r] + re_j - (uint32_t)corr[i]);
          const int im =
              (int)((uint32_t)acc_im[s][r] + (uint32_t)corr[kElems + i] - ci_col_j);
          if (kStore == 2) {
            atomicAdd(o, re);
            atomicAdd(o + 1, im);
          } else if (kStore == 1) {
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

// The 8 waves of a workgroup each run their share of the triangle.
__device__ __forceinline__ void tri_channel(const TriParams& p, int ch, int sb, int se,
                                            uint8_t* raw0, uint8_t* raw1, uint8_t* dec_p) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int simd = wave & 3;
  if (wave < 4) {
    tri_run<BalancedA>(p, ch, simd, sb, se, raw0, raw1, dec_p);
  } else {
    switch (simd) {
      case 0: tri_run<BalancedB<0>>(p, ch, 0, sb, se, raw0, raw1, dec_p); break;
      case 1: tri_run<BalancedB<1>>(p, ch, 0, sb, se, raw0, raw1, dec_p); break;
      case 2: tri_run<BalancedB<2>>(p, ch, 0, sb, se, raw0, raw1, dec_p); break;
      default: tri_run<BalancedB<3>>(p, ch, 0, sb, se, raw0, raw1, dec_p); break;
    }
  }
}

template <int kMode>
__device__ __forceinline__ void tri_channel_t(const TriParams& p, int ch, int sb, int se,
                                              uint8_t* raw0, uint8_t* raw1, uint8_t* dec_p,
                                              const TriDelays* dl, GathSlots gs,
                                              const TriSegments* sg = nullptr) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int simd = wave & 3;
  if (wave < 4) {
    tri_run<BalancedA, kMode>(p, ch, simd, sb, se, raw0, raw1, dec_p, dl, gs, sg);
  } else {
    switch (simd) {
      case 0: tri_run<BalancedB<0>, kMode>(p, ch, 0, sb, se, raw0, raw1, dec_p, dl, gs, sg); break;
      case 1: tri_run<BalancedB<1>, kMode>(p, ch, 0, sb, se, raw0, raw1, dec_p, dl, gs, sg); break;
      case 2: tri_run<BalancedB<2>, kMode>(p, ch, 0, sb, se, raw0, raw1, dec_p, dl, gs, sg); break;
      default: tri_run<BalancedB<3>, kMode>(p, ch, 0, sb, se, raw0, raw1, dec_p, dl, gs, sg); break;
    }
  }
}

}  // namespace tri
}  // namespace xeng
