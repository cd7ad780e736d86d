// xcorr_rect_bf6.hip -- the kernel of 256-element diagonal squares and 128 x 256
// off-diagonal tiles (the cover of xcorr_rect.hip, for arrays of more than
// 256 elements) on the f8f6f4 matrix cores with bf6 operands.
//
// As in the bf6 triangle kernel, the 4-bit values of Sec. III are exact in
// the 6-bit float E3M2 and v_mfma_scale_f32_32x32x64_f8f6f4 multiplies them
// exactly; its fp32 sums stay exact while they are integers below 2^24, so a
// workgroup sums at most kMaxStagesPerPart stages (131 008 samples) and longer
// runs are split along time. The signed values are multiplied directly
// (Sec. II-A, Eq. 1 and 2: Re V_ij = P_i . P_j, Im V_ij = Q_i . P_j with
// P = [Re, Im], Q = [Im, -Re]), so no offset corrections are needed; sample
// rows past the end of the data load as 0x00, which decodes to (-8, -8) and
// adds 128 to Re and 0 to Im of every pair, subtracted at the end.
//
// Diagonal squares run the bf6 triangle kernel's per-wave routine. A tile is
// staged like the int8 tile (packed bytes HBM -> LDS with buffer_load ... lds,
// two stages ahead; wave w loads sample rows 8w .. 8w+7 of both panels, reads
// them back transposed with ds_read_b64_tr_b8), but a wave decodes its
// 8-sample group of all 384 elements into bf6 cells: per element 12 bytes,
// [Re of the 8 samples | Im of the 8 samples], in a 16-byte cell of the
// group's plane. One bf6 MFMA step takes 32 samples: lane half h of step s
// reads the cells of groups 4s + 2h and 4s + 2h + 1, two 12-byte reads per
// operand. Wave w owns the 64 x 64 sub-tile (rows 64 (w >> 2), columns
// 64 (w & 3)): 2 x 2 blocks, Re and Im, 128 fp32 accumulators.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "xcorr_device.h"
#include "xcorr_launch.h"
#include "xcorr_tri_bf6_run.h"
#include "xcorr_tri_common.h"

namespace xeng {

namespace {

using tri::bf6_q;
using tri::f16_pair;
using tri::lds_barrier;
using tri::lds_v2i_ptr;
using tri::lds_void_ptr;
using tri::v16f;
using tri::v16u;
using tri::v32h;
using tri::v3i;
using tri::v6u;
using tri::v8i;
using tri::vm_wait;

constexpr int kThreads = 512;                   // 8 waves, two per SIMD
constexpr int kRows = 128;                      // tile rows (i)
constexpr int kCols = 256;                      // tile columns (j); also the square's edge
constexpr int kStage = 64;                      // samples per stage
constexpr int kSlots = kCols + kRows;           // decoded elements: columns, then rows
constexpr int kColStride = kCols + 32;          // raw column panel, bytes per sample row
constexpr int kColRaw = kStage * kColStride;    // 18 KiB
// raw row panel: one load instruction fills 256 bytes, two sample rows of the
// 128 row elements (lanes 0-31 the even row, lanes 32-63 the odd one)
constexpr int kPairStride = 2 * kRows + 32;
constexpr int kRowRaw = (kStage / 2) * kPairStride;   // 9 KiB
constexpr int kCell = 16;                       // one element's 8-sample group (12 bytes used)
constexpr int kGPlane = kSlots * kCell;         // one group of all elements: 6 KiB
constexpr int kDBuf = 8 * kGPlane;              // one stage: 48 KiB
constexpr int kDecBytes = 2 * kDBuf;            // double-buffered: 96 KiB
constexpr int kLoads = 8 + 4;                   // load instructions per wave and stage
constexpr uint32_t kOob = 0x80000000u;          // offset past every record: the load returns 0

static_assert(kColRaw == tri::kRawBytes, "the diagonal squares use the column raw buffers");
static_assert(kDecBytes >= tri::kDecBytes, "the diagonal squares' cells fit");
static_assert(2 * kColRaw + 2 * kRowRaw + kDecBytes <= 160 * 1024, "LDS of one compute unit");

struct RectBf6Params {
  const uint8_t* in;
  int32_t* vis;
  int n, f;
  int t;                 // samples per channel
  int64_t ss, cs;        // bytes from one sample to the next, and from one channel to the next
  int t0, t_end;         // this launch sums samples [t0, t_end)
  int nbc;               // 256-element blocks, ceil(n / 256)
  int units;             // pieces per channel: nbc squares, then nbc (nbc - 1) tiles
  int split;             // workgroups along time per piece
  int stages_per_split;
  int total_stages;
  int accumulate;
  int atomic_out;
};

// Tile rows row0 .. row0+127, columns col0 .. col0+255, row0 < col0.
__device__ __forceinline__ void rect_run_bf6(const RectBf6Params& p, int ch, int row0, int col0,
                                             int sb, int se, uint8_t* craw0, uint8_t* craw1,
                                             uint8_t* rraw0, uint8_t* rraw1, uint8_t* dec) {
  const int tid = tri::opaque_tid();
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int half = lane >> 5, l32 = lane & 31;
  const int n = p.n;
  const uint8_t* chan = p.in + (int64_t)ch * p.cs;
  const int64_t ss = p.ss;

  // ---- loads, as in the int8 tile: sample rows 8*wave .. 8*wave+7 of a stage;
  // elements past n and rows past this workgroup's samples read 0x00
  const uint32_t voff_c = (col0 + 4 * lane < n) ? (uint32_t)(col0 + 4 * lane) : kOob;
  const uint32_t voff_r =
      (row0 + 4 * l32 < n) ? (uint32_t)(row0 + 4 * l32) + (uint32_t)(half * ss) : kOob;
  const int t_stop = min(p.t_end, p.t0 + se * kStage);   // samples [t0 + sb*64, t_stop)
  auto fetch = [&](uint8_t* craw, uint8_t* rraw, int st) {
    const int first = __builtin_amdgcn_readfirstlane(p.t0 + st * kStage + 8 * wave);
    const int64_t bytes = t_stop > first ? (int64_t)(t_stop - first - 1) * ss + n : 0;
    const int records = bytes <= 0 ? 0 : (bytes > 0x7fffffff ? 0x7fffffff : (int)bytes);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(chan + (int64_t)first * ss), 0, records, 0x00020000);
#pragma unroll
    for (int r = 0; r < 8; ++r)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rs, (lds_void_ptr)(craw + (8 * wave + r) * kColStride), 4,
          voff_c + (uint32_t)(r * ss), 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rs, (lds_void_ptr)(rraw + (4 * wave + q) * kPairStride), 4,
          voff_r + (uint32_t)(2 * q * ss), 0, 0, 0);
  };

  // ---- transposing reads: 0-3 cover columns 64i .. 64i+63, 4-5 rows
  // 64(i-4) .. 64(i-4)+63; lane k of a 16-lane group receives element
  // 64i + lane, byte m = sample m of the wave's 8 rows
  const int lq = lane & 15, grp = (lane >> 4) & 3;
  const int trc_off = (8 * wave + (lq >> 1)) * kColStride + 16 * grp + 8 * (lq & 1);
  const int trr_off =
      (4 * wave + (lq >> 2)) * kPairStride + ((lq >> 1) & 1) * kRows + 16 * grp + 8 * (lq & 1);
  auto tr_read = [&](const uint8_t* craw, const uint8_t* rraw, int i) {
    return i < 4 ? __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i_ptr)(craw + trc_off + 64 * i))
                 : __builtin_amdgcn_ds_read_tr8_b64_v2i32(
                       (lds_v2i_ptr)(rraw + trr_off + 64 * (i - 4)));
  };

  // ---- decode: the wave's group (plane `wave`) of element slots 64 i0 + lane
  // and 64 (i0 + 1) + lane. A word holds samples 0..3 (x) or 4..7 (y) of an
  // element, one per byte; the word and the word shifted right by 8 hold two
  // samples each in the low bytes of their halves (the order of samples
  // inside a cell is the same for every element, which is all the dot
  // product needs). Re becomes the f16 value 64 + u, Im 1024 + u; adding
  // -(64 + 8) or -(1024 + 8) gives u - 8 exactly, and the hardware packs 32
  // such values (two elements' cells) into 6 dwords of bf6 codes.
  uint32_t re_bits = 0x54005400u, im_bits = 0x64006400u;
  asm volatile("; f16 exponent bits held in registers" : "+v"(re_bits), "+v"(im_bits));
  auto re16 = [&](uint32_t t) { return f16_pair(t, 0x00F000F0u, re_bits, (_Float16)-72.0f); };
  auto im16 = [&](uint32_t t) { return f16_pair(t, 0x000F000Fu, im_bits, (_Float16)-1032.0f); };
  // stores into dec use one offset from the array, which keeps the compiler's
  // link between them and dec (it then does not wait for the loads into the
  // raw arrays before them)
  const int wr_off = wave * kGPlane + lane * kCell;
  auto decode_pair = [&](v2i wa, v2i wb, int buf, int i0) {
    const uint32_t a0 = (uint32_t)wa.x, a1 = (uint32_t)wa.x >> 8;
    const uint32_t a2 = (uint32_t)wa.y, a3 = (uint32_t)wa.y >> 8;
    const uint32_t b0 = (uint32_t)wb.x, b1 = (uint32_t)wb.x >> 8;
    const uint32_t b2 = (uint32_t)wb.y, b3 = (uint32_t)wb.y >> 8;
    const v16u u = {re16(a0), re16(a1), re16(a2), re16(a3), im16(a0), im16(a1), im16(a2), im16(a3),
                    re16(b0), re16(b1), re16(b2), re16(b3), im16(b0), im16(b1), im16(b2), im16(b3)};
    const v6u b = __builtin_amdgcn_cvt_scalef32_pk32_bf6_f16(__builtin_bit_cast(v32h, u), 1.0f);
    const int o = wr_off + buf * kDBuf + 64 * i0 * kCell;
    *reinterpret_cast<v3i*>(dec + o) = v3i{(int)b[0], (int)b[1], (int)b[2]};
    *reinterpret_cast<v3i*>(dec + (o + 64 * kCell)) = v3i{(int)b[3], (int)b[4], (int)b[5]};
  };

  // ---- MFMA operands: lane half h of step s reads groups 4s + 2h, 4s + 2h + 1
  // of its element; rows are slots kCols + 64 wr + 32 rb + l32, columns
  // 64 wc + 32 cb + l32
  const int wr = wave >> 2, wc = wave & 3;
  int a_off[2], b_off[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    a_off[k] = 2 * half * kGPlane + (kCols + 64 * wr + 32 * k + l32) * kCell;
    b_off[k] = 2 * half * kGPlane + (64 * wc + 32 * k + l32) * kCell;
  }
  auto operand = [&](int buf, int step, int off) {
    const uint8_t* base = dec + (buf * kDBuf + 4 * step * kGPlane + off);
    const v3i x = *reinterpret_cast<const v3i*>(base);
    const v3i y = *reinterpret_cast<const v3i*>(base + kGPlane);
    return v8i(__builtin_shufflevector(x, y, 0, 1, 2, 3, 4, 5, -1, -1));
  };
  struct Frags {
    v8i a[2], b[2];
  };
  auto load_frags = [&](Frags& fr, int buf, int step) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      fr.a[k] = operand(buf, step, a_off[k]);
      fr.b[k] = operand(buf, step, b_off[k]);
    }
  };
  v16f acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      acc_re[rb][cb] = v16f{};
      acc_im[rb][cb] = v16f{};
    }
  auto mfma_step = [&](const Frags& fr) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const v8i a = fr.a[rb];
      const v8i q = bf6_q(a);
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        acc_re[rb][cb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
            a, fr.b[cb], acc_re[rb][cb], tri::kFmtBf6, tri::kFmtBf6, 0, tri::kScaleOne, 0,
            tri::kScaleOne);
        acc_im[rb][cb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
            q, fr.b[cb], acc_im[rb][cb], tri::kFmtBf6, tri::kFmtBf6, 0, tri::kScaleOne, 0,
            tri::kScaleOne);
      }
    }
  };

  // One stage st: the step-0 operands are requested first, then this wave's
  // loads for st+2, a wait for its loads of st+1 and their transposing reads;
  // each of the two MFMA steps then overlaps its MFMAs with part of the decode
  // of st+1 (into the other buffer). kPar = (st - sb) & 1 selects the static
  // buffers. Stages past se are fetched and decoded as well; their rows read
  // nothing.
  auto body = [&](auto par, int st) {
    constexpr int kPar = decltype(par)::value;
    uint8_t* const c_ld = kPar ? craw1 : craw0;
    uint8_t* const r_ld = kPar ? rraw1 : rraw0;
    const uint8_t* const c_dc = kPar ? craw0 : craw1;
    const uint8_t* const r_dc = kPar ? rraw0 : rraw1;
    fetch(c_ld, r_ld, st + 2);
    vm_wait<kLoads>();   // all but the loads just issued are done: st+1 is in LDS
    // Each half of the stage decodes part of st+1 (into the other buffer),
    // then reads one step's operands and multiplies. The segments are kept
    // apart: the decode's temporaries, the operands and the 128 accumulators
    // do not all fit at once (the other wave of the SIMD fills one's decode
    // with its MFMAs). The transposed words are read just before their decode.
    Frags fr;
    decode_pair(tr_read(c_dc, r_dc, 0), tr_read(c_dc, r_dc, 1), kPar ^ 1, 0);
    __builtin_amdgcn_sched_barrier(0);
    load_frags(fr, kPar, 0);
    mfma_step(fr);
    __builtin_amdgcn_sched_barrier(0);
    decode_pair(tr_read(c_dc, r_dc, 2), tr_read(c_dc, r_dc, 3), kPar ^ 1, 2);
    __builtin_amdgcn_sched_barrier(0);
    decode_pair(tr_read(c_dc, r_dc, 4), tr_read(c_dc, r_dc, 5), kPar ^ 1, 4);
    __builtin_amdgcn_sched_barrier(0);
    load_frags(fr, kPar, 1);
    mfma_step(fr);
    __builtin_amdgcn_sched_barrier(0);
    lds_barrier();
  };

  // ---- prologue: fetch sb and sb+1, decode sb ----------------------------------
  fetch(craw0, rraw0, sb);
  fetch(craw1, rraw1, sb + 1);
  vm_wait<kLoads>();
  decode_pair(tr_read(craw0, rraw0, 0), tr_read(craw0, rraw0, 1), 0, 0);
  decode_pair(tr_read(craw0, rraw0, 2), tr_read(craw0, rraw0, 3), 0, 2);
  decode_pair(tr_read(craw0, rraw0, 4), tr_read(craw0, rraw0, 5), 0, 4);
  lds_barrier();
  int st = sb;
  for (; st + 1 < se; st += 2) {
    body(std::integral_constant<int, 0>{}, st);
    body(std::integral_constant<int, 1>{}, st + 1);
  }
  if (st < se) body(std::integral_constant<int, 0>{}, st);
  // loads of the two stages past se may still be writing LDS
  vm_wait<0>();
  lds_barrier();

  // samples summed, and the padding samples among the stages multiplied
  const int t_sum = max(0, t_stop - (p.t0 + sb * kStage));
  const int re_pad = 128 * ((se - sb) * kStage - t_sum);

  // ---- epilogue: masked writes of i <= j < n into the packed triangle ------------
  const int64_t n64 = n;
  const int64_t entries = n64 * (n64 + 1) / 2;
  int32_t* out = p.vis + (int64_t)ch * entries * 2;
  auto store_all = [&](auto mode) {
    constexpr int kStore = decltype(mode)::value;   // 0 store, 1 add, 2 atomic add
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int j = col0 + 64 * wc + 32 * cb + l32;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = row0 + 64 * wr + 32 * rb + 8 * (r >> 2) + 4 * half + (r & 3);
          if (i <= j && j < n) {
            int32_t* o = out + 2 * tri_index(n64, i, j);
            // integers below 2^24 in magnitude: the conversions are exact
            const int re = (int)acc_re[rb][cb][r] - re_pad;
            const int im = (int)acc_im[rb][cb][r];
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
    }
  };
  if (p.atomic_out)
    store_all(std::integral_constant<int, 2>{});
  else if (p.accumulate)
    store_all(std::integral_constant<int, 1>{});
  else
    store_all(std::integral_constant<int, 0>{});
}

__global__ __launch_bounds__(kThreads, 1) void xcorr_rect_bf6_kernel(RectBf6Params p) {
  // Each buffer is its own variable: the compiler then tracks the loads into
  // one separately from reads of the others and waits only for those.
  __shared__ __attribute__((aligned(16))) uint8_t craw0[kColRaw];
  __shared__ __attribute__((aligned(16))) uint8_t craw1[kColRaw];
  __shared__ __attribute__((aligned(16))) uint8_t rraw0[kRowRaw];
  __shared__ __attribute__((aligned(16))) uint8_t rraw1[kRowRaw];
  __shared__ __attribute__((aligned(16))) uint8_t dec[kDecBytes];
  // logical workgroup -> (channel, piece, part of the time axis); consecutive
  // logical ids run on one XCD, so the pieces of a channel share its L2
  const int logical = xcd_logical_id(blockIdx.x, gridDim.x);
  const int per_ch = p.units * p.split;
  const int ch = __builtin_amdgcn_readfirstlane(logical / per_ch);
  const int rest = logical - ch * per_ch;
  const int u = __builtin_amdgcn_readfirstlane(rest / p.split);
  const int part = rest - u * p.split;
  const int sb = part * p.stages_per_split;
  const int se = min(sb + p.stages_per_split, p.total_stages);
  if (sb >= se) return;
  if (u < p.nbc) {
    // diagonal square u: elements 256u .. 256u+255, the bf6 triangle routine
    tri::TriParams tp;
    tp.in = p.in;
    tp.vis = p.vis;
    tp.e0 = kCols * u;
    tp.n = min(kCols, p.n - tp.e0);
    tp.n_total = p.n;
    tp.f = p.f;
    tp.t = p.t;
    tp.ss = p.ss;
    tp.cs = p.cs;
    tp.t0 = p.t0;
    tp.t_end = p.t_end;
    tp.split = p.split;
    tp.stages_per_split = p.stages_per_split;
    tp.total_stages = p.total_stages;
    tp.accumulate = p.accumulate;
    tp.atomic_out = p.atomic_out;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int simd = wave & 3;
    if (wave < 4) {
      tri::tri_run_bf6<tri::ProgA>(tp, ch, simd, sb, se, craw0, craw1, dec);
    } else {
      switch (simd) {
        case 0: tri::tri_run_bf6<tri::ProgB<0>>(tp, ch, 0, sb, se, craw0, craw1, dec); break;
        case 1: tri::tri_run_bf6<tri::ProgB<1>>(tp, ch, 0, sb, se, craw0, craw1, dec); break;
        case 2: tri::tri_run_bf6<tri::ProgB<2>>(tp, ch, 0, sb, se, craw0, craw1, dec); break;
        default: tri::tri_run_bf6<tri::ProgB<3>>(tp, ch, 0, sb, se, craw0, craw1, dec); break;
      }
    }
  } else {
    // tiles column block by column block: block J >= 1 holds the 2J row
    // blocks above its square, J (J - 1) tiles come before it
    const int r = u - p.nbc;
    int J = 1;
    while ((J + 1) * J <= r) ++J;
    const int I = r - J * (J - 1);
    rect_run_bf6(p, ch, kRows * I, kCols * J, sb, se, craw0, craw1, rraw0, rraw1, dec);
  }
}

}  // namespace

hipError_t launch_rect_bf6(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                           int64_t cs, int t0, int t_count, int accumulate, int split,
                           hipStream_t stream) {
  if (n < 1 || n % 4 != 0) return hipErrorInvalidValue;
  if (t_count <= 0 || t0 < 0 || (int64_t)t0 + t_count > t) return hipErrorInvalidValue;
  RectBf6Params p;
  p.in = in;
  p.vis = vis;
  p.n = n;
  p.f = f;
  p.t = t;
  p.ss = ss;
  p.cs = cs;
  p.t0 = t0;
  p.t_end = t0 + t_count;
  p.nbc = (n + kCols - 1) / kCols;
  p.units = p.nbc * p.nbc;
  p.total_stages = (t_count + kStage - 1) / kStage;
  if (split < 1) split = 1;
  if (split > p.total_stages) split = p.total_stages;
  p.split = split;
  p.stages_per_split = (p.total_stages + split - 1) / split;
  // the caller sizes split so that no part exceeds the exact fp32 range
  if (p.stages_per_split > tri::kMaxStagesPerPart) return hipErrorInvalidValue;
  p.accumulate = accumulate;
  p.atomic_out = split > 1;
  const int64_t grid = (int64_t)f * p.units * split;
  if (f <= 0 || grid <= 0 || grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  xcorr_rect_bf6_kernel<<<dim3((unsigned)grid), dim3(kThreads), 0, stream>>>(p);
  return hipGetLastError();
}

}  // namespace xeng
