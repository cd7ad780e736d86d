// xcorr_rect.hip -- gfx950 correlation kernel for arrays of more than 256
// elements: the upper triangle cut into 256-element diagonal squares and
// 128 x 256 off-diagonal tiles, one workgroup of 8 waves per piece.
//
// Same contraction as the other kernels (paper Sec. II-A, Eq. 1 and 2):
//   Re V_ij = P_i . P_j,  Im V_ij = Q_i . P_j,   P_e = [Re e, Im e],
//   Q_e = [Im e, -Re e]  over the time axis,
// on v_mfma_i32_32x32x32_i8, with the offset arithmetic of Sec. III-A (Eq. 3):
// the matrix cores multiply the Excess-8 fields and per-element field sums
// correct the products in the epilogue (see xcorr_tri.hip for the identities).
//
// How the triangle is covered (Sec. II-C tiles the upper triangle and computes
// only tiles that reach it):
//   * diagonal square J (elements 256J .. 256J+255) is the 8 x 8 block triangle
//     of Fig. 1; it runs the triangle kernel's block programs, which give each
//     SIMD 9 of the 36 blocks. Only 36 of its 64 blocks are multiplied.
//   * above the diagonal squares, rows 128I .. 128I+127 and columns
//     256J .. 256J+255 with 128I < 256J form a 128 x 256 tile that lies wholly
//     in the upper triangle: 8 waves, wave w owns the 64 x 64 sub-tile (rows
//     64 (w >> 2), columns 64 (w & 3)): 2 x 2 blocks, Re and Im, 128 int32
//     accumulators in ordinary registers. The two waves of a SIMD (w, w + 4)
//     share their columns.
// At N = 2048 a channel is 8 squares (9 blocks per SIMD) and 56 tiles (8 per
// SIMD), so the MFMA work per SIMD is 1.5 % above the 2049 blocks the entries
// need; tiles that straddle the diagonal would cost 12 %.
//
// Staging of a tile, per 64-sample stage, as in the triangle kernel: packed
// bytes go from HBM into LDS with buffer_load ... lds (no registers), two
// stages ahead; wave w loads sample rows 8w .. 8w+7 of both panels and is the
// only reader of them, so it waits for its own loads only. It transposes them
// with ds_read_b64_tr_b8 (each lane receives 8 consecutive samples of one
// element), decodes the fields and writes 16-byte slabs
// [uRe g, uRe g+1, uIm g, uIm g+1] for its 8-sample group of all 384 elements
// (256 columns, 128 rows); every wave then reads ready operands for its
// MFMA steps. The field sums are taken with v_sad_u8 during the decode.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "xcorr_device.h"
#include "xcorr_launch.h"
#include "xcorr_tri_common.h"
#include "xcorr_tri_run.h"

namespace xeng {

namespace {

using tri::lds_barrier;
using tri::lds_v2i_ptr;
using tri::lds_void_ptr;
using tri::vm_wait;

constexpr int kThreads = 512;                   // 8 waves, two per SIMD
constexpr int kRows = 128;                      // tile rows (i)
constexpr int kCols = 256;                      // tile columns (j); also the square's edge
constexpr int kStage = 64;                      // samples per stage
constexpr int kSlots = kCols + kRows;           // decoded elements: columns, then rows
constexpr int kColStride = kCols + 32;          // raw column panel, bytes per sample row
constexpr int kColRaw = kStage * kColStride;    // 18 KiB
// Raw row panel: one load instruction fills 256 bytes, so each line holds two
// sample rows of the 128 row elements (lanes 0-31 the even row, lanes 32-63
// the odd one), and lines are padded so the 8 rows one transposing read
// touches fall on distinct banks.
constexpr int kPairStride = 2 * kRows + 32;
constexpr int kRowRaw = (kStage / 2) * kPairStride;   // 9 KiB
constexpr int kPBuf = kSlots * 16;              // slabs of one 8-sample group, one buffer
constexpr int kPGroup = 2 * kPBuf;              // a group's slabs in both buffers
constexpr int kDecBytes = 8 * kPGroup;          // 96 KiB
constexpr int kLoads = 8 + 4;                   // load instructions per wave and stage
constexpr uint32_t kOob = 0x80000000u;          // offset past every record: the load returns 0

static_assert(kColRaw == tri::kRawBytes, "the diagonal squares use the column raw buffers");
static_assert(kDecBytes >= tri::kGroups * tri::kPGroup, "the diagonal squares' slabs fit");
static_assert(8 * 2 * kSlots * 4 <= kDecBytes && 3 * kSlots * 4 <= kColRaw,
              "the corrections fit the operand and raw buffers");
static_assert(2 * kColRaw + 2 * kRowRaw + kDecBytes <= 160 * 1024, "LDS of one compute unit");

struct RectParams {
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

using tri::kDense;
using tri::kSegments;
using tri::TriSegments;

// Tile rows 128I .. 128I+127, columns 256J .. 256J+255, 128I < 256J.
// kMode: kDense sums samples [t0, t_end); kSegments sums the sample segments
// of *sg (the runs of one gate), stage by stage as the triangle kernel does.
template <int kMode>
__device__ __forceinline__ void rect_run(const RectParams& p, int ch, int row0, int col0, int sb,
                                         int se, uint8_t* craw0, uint8_t* craw1, uint8_t* rraw0,
                                         uint8_t* rraw1, uint8_t* dec,
                                         const TriSegments* sg = nullptr) {
  const int tid = tri::opaque_tid();
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int half = lane >> 5, l32 = lane & 31;
  const int n = p.n;
  const uint8_t* chan = p.in + (int64_t)ch * p.cs;
  const int64_t ss = p.ss;

  // ---- loads: sample rows 8*wave .. 8*wave+7 of a stage. Column panel: one
  // instruction per row, a lane carries 4 elements. Row panel: one
  // instruction per two rows (lanes 32-63 one row further). Elements past n
  // use an offset past every record; rows past the end of this workgroup's
  // samples lie past the descriptor's record count. Both read 0x00 bytes,
  // whose fields are 0 and add nothing to any product or field sum.
  const uint32_t voff_c = (col0 + 4 * lane < n) ? (uint32_t)(col0 + 4 * lane) : kOob;
  const uint32_t voff_r =
      (row0 + 4 * l32 < n) ? (uint32_t)(row0 + 4 * l32) + (uint32_t)(half * ss) : kOob;
  const int t_stop = min(p.t_end, p.t0 + se * kStage);   // samples [t0 + sb*64, t_stop)
  // first sample of stage st and the end of its samples; in the segment mode
  // stages past se (loaded ahead, never multiplied) are empty. The stage loop
  // fetches stages in increasing order, so the segment of the next one is
  // found by moving on from the last one found.
  int seg = 0;
  auto stage_span = [&](int st, int& first_row, int& stop) {
    if (kMode == kSegments) {
      int k = seg;
      while (k + 1 < sg->count && sg->stage0[k + 1] <= st) ++k;
      seg = k;
      first_row = sg->t0[k] + (st - sg->stage0[k]) * kStage;
      stop = st < se ? sg->t_end[k] : first_row;
    } else {
      first_row = p.t0 + st * kStage;
      stop = t_stop;
    }
  };
  // kPanels: 1 loads the column panel, 2 the row panel, 3 both
  auto fetch = [&](uint8_t* craw, uint8_t* rraw, int st, auto panels) {
    constexpr int kPanels = decltype(panels)::value;
    int row0_st, stop;
    stage_span(st, row0_st, stop);
    const int first = __builtin_amdgcn_readfirstlane(row0_st + 8 * wave);
    const int64_t bytes = stop > first ? (int64_t)(stop - first - 1) * ss + n : 0;
    const int records = bytes <= 0 ? 0 : (bytes > 0x7fffffff ? 0x7fffffff : (int)bytes);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(chan + (int64_t)first * ss), 0, records, 0x00020000);
    if constexpr ((kPanels & 1) != 0) {
#pragma unroll
      for (int r = 0; r < 8; ++r)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (lds_void_ptr)(craw + (8 * wave + r) * kColStride), 4,
            voff_c + (uint32_t)(r * ss), 0, 0, 0);
    }
    if constexpr ((kPanels & 2) != 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (lds_void_ptr)(rraw + (4 * wave + q) * kPairStride), 4,
            voff_r + (uint32_t)(2 * q * ss), 0, 0, 0);
    }
  };
  const std::integral_constant<int, 1> kColPanel;
  const std::integral_constant<int, 2> kRowPanel;
  const std::integral_constant<int, 3> kBothPanels;

  // ---- decode: ds_read_b64_tr_b8 over the wave's 8 rows. In each 16-lane
  // group the even lanes name the rows of elements e0..e0+7 and the odd lanes
  // those of e0+8..e0+15; lane k of the group receives element e0+k, byte m =
  // sample m. Reads 0-3 cover columns 64i .. 64i+63, reads 4-5 rows
  // 64(i-4) .. 64(i-4)+63: slot 64i + lane either way.
  const int lq = lane & 15, grp = (lane >> 4) & 3;
  const int trc_off = (8 * wave + (lq >> 1)) * kColStride + 16 * grp + 8 * (lq & 1);
  const int trr_off =
      (4 * wave + (lq >> 2)) * kPairStride + ((lq >> 1) & 1) * kRows + 16 * grp + 8 * (lq & 1);
  auto tr_read = [&](const uint8_t* craw, const uint8_t* rraw, int i) {
    return i < 4 ? __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_v2i_ptr)(craw + trc_off + 64 * i))
                 : __builtin_amdgcn_ds_read_tr8_b64_v2i32(
                       (lds_v2i_ptr)(rraw + trr_off + 64 * (i - 4)));
  };
  // stores into dec use one offset from the array, which keeps the compiler's
  // link between them and dec (it then does not wait for the loads into the
  // raw arrays before them)
  const int wr_off = wave * kPGroup + lane * 16;
  uint32_t sum_re[6] = {0, 0, 0, 0, 0, 0}, sum_im[6] = {0, 0, 0, 0, 0, 0};
  auto decode = [&](v2i w, int buf, int i) {
    const uint32_t ra = fields_hi((uint32_t)w.x), rb = fields_hi((uint32_t)w.y);
    const uint32_t ia = fields_lo((uint32_t)w.x), ib = fields_lo((uint32_t)w.y);
    *reinterpret_cast<v4i*>(dec + (wr_off + buf * kPBuf + i * 1024)) =
        v4i{(int)ra, (int)rb, (int)ia, (int)ib};
    // v_sad_u8 against zero adds the four bytes of a word
    sum_re[i] = __builtin_amdgcn_sad_u8(rb, 0u, __builtin_amdgcn_sad_u8(ra, 0u, sum_re[i]));
    sum_im[i] = __builtin_amdgcn_sad_u8(ib, 0u, __builtin_amdgcn_sad_u8(ia, 0u, sum_im[i]));
  };

  // ---- MFMA operands: lane half h reads group 2*ks + h; the wave's rows are
  // slots kCols + 64*wr + 32*rb + l32, its columns 64*wc + 32*cb + l32
  const int wr = wave >> 2, wc = wave & 3;
  int a_off[2], b_off[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    a_off[k] = half * kPGroup + (kCols + 64 * wr + 32 * k + l32) * 16;
    b_off[k] = half * kPGroup + (64 * wc + 32 * k + l32) * 16;
  }
  v16i acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      acc_re[rb][cb] = v16i{};
      acc_im[rb][cb] = v16i{};
    }
  struct Frags {
    v4i a[2], b[2];
  };
  auto load_frags = [&](Frags& fr, int buf, int ks) {
    const uint8_t* const base = dec + ks * 2 * kPGroup + buf * kPBuf;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      fr.a[k] = *reinterpret_cast<const v4i*>(base + a_off[k]);
      fr.b[k] = *reinterpret_cast<const v4i*>(base + b_off[k]);
    }
  };
  // P = [uRe, uIm] on both sides, Q = [uIm, 15 - uRe] on the row side
  auto mfma_step = [&](const Frags& fr) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const v4i a = fr.a[rb];
      const v4i q = {a.z, a.w, (int)((uint32_t)a.x ^ 0x0F0F0F0Fu),
                     (int)((uint32_t)a.y ^ 0x0F0F0F0Fu)};
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        acc_re[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, fr.b[cb], acc_re[rb][cb], 0, 0, 0);
        acc_im[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(q, fr.b[cb], acc_im[rb][cb], 0, 0, 0);
      }
    }
  };

  // One stage st: the step-0 operands are requested first, then a wait for
  // this wave's loads of st+1 (issued a stage earlier) and their transposing
  // reads; each MFMA step then requests the next step's operands and overlaps
  // its MFMAs with part of the decode of st+1 (into the other operand buffer).
  // The loads of st+2 go out after the first MFMA step (the column panel) and
  // the second (the row panel), so that the matrix cores start before the
  // load instructions are issued (about 2 % faster than issuing them all
  // first). kPar = (st - sb) & 1 selects the static
  // buffers. Stages past se are fetched and decoded as well; their rows read
  // nothing.
  auto body = [&](auto par, int st) {
    constexpr int kPar = decltype(par)::value;
    uint8_t* const c_ld = kPar ? craw1 : craw0;
    uint8_t* const r_ld = kPar ? rraw1 : rraw0;
    const uint8_t* const c_dc = kPar ? craw0 : craw1;
    const uint8_t* const r_dc = kPar ? rraw0 : rraw1;
    Frags fr[2];
    load_frags(fr[0], kPar, 0);
    vm_wait<0>();   // this wave's loads of st+1 are in LDS
    v2i rawv[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) rawv[i] = tr_read(c_dc, r_dc, i);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      if (ks < 3) load_frags(fr[(ks + 1) & 1], kPar, ks + 1);
      if (ks < 2) {
        decode(rawv[2 * ks], kPar ^ 1, 2 * ks);
        decode(rawv[2 * ks + 1], kPar ^ 1, 2 * ks + 1);
      } else {
        decode(rawv[ks + 2], kPar ^ 1, ks + 2);
      }
      mfma_step(fr[ks & 1]);
      __builtin_amdgcn_sched_barrier(0);
      if (ks == 0) {
        fetch(c_ld, r_ld, st + 2, kColPanel);
        __builtin_amdgcn_sched_barrier(0);
      } else if (ks == 1) {
        fetch(c_ld, r_ld, st + 2, kRowPanel);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    lds_barrier();
  };

  // ---- prologue: fetch sb and sb+1, decode sb -------------------------------------
  fetch(craw0, rraw0, sb, kBothPanels);
  fetch(craw1, rraw1, sb + 1, kBothPanels);
  vm_wait<kLoads>();
#pragma unroll
  for (int i = 0; i < 6; ++i) decode(tr_read(craw0, rraw0, i), 0, i);
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

  // ---- offset corrections: per element (slot) s, from the field sums of all
  // waves, cr = 8 (SR + SI), ci_row = 8 (SR - SI), ci_col = 8 SR + 7 SI
  {
    uint32_t* part = reinterpret_cast<uint32_t*>(dec);   // [wave][re, im][slot]
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      part[(2 * wave) * kSlots + 64 * i + lane] = sum_re[i];
      part[(2 * wave + 1) * kSlots + 64 * i + lane] = sum_im[i];
    }
  }
  lds_barrier();
  int32_t* const corr = reinterpret_cast<int32_t*>(craw0);   // [cr, ci_row, ci_col][slot]
  if (tid < kSlots) {
    const uint32_t* part = reinterpret_cast<const uint32_t*>(dec);
    uint32_t sr = 0, si = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
      sr += part[(2 * w) * kSlots + tid];
      si += part[(2 * w + 1) * kSlots + tid];
    }
    corr[tid] = (int32_t)(8u * (sr + si));
    corr[kSlots + tid] = (int32_t)(8u * (sr - si));
    corr[2 * kSlots + tid] = (int32_t)(8u * sr + 7u * si);
  }
  lds_barrier();
  // samples this workgroup summed
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
  const int64_t n64 = n;
  const int64_t entries = n64 * (n64 + 1) / 2;
  int32_t* out = p.vis + (int64_t)ch * entries * 2;
  auto store_all = [&](auto mode) {
    constexpr int kStore = decltype(mode)::value;   // 0 store, 1 add, 2 atomic add
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int jl = 64 * wc + 32 * cb + l32;
      const int j = col0 + jl;
      const uint32_t re_j = re_const - (uint32_t)corr[jl];
      const uint32_t ci_col_j = (uint32_t)corr[2 * kSlots + jl];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int il = 64 * wr + 32 * rb + 8 * (r >> 2) + 4 * half + (r & 3);
          const int i = row0 + il;
          if (i <= j && j < n) {
            int32_t* o = out + 2 * tri_index(n64, i, j);
            // int32 arithmetic modulo 2^32 (unsigned): exact for the result
            const int re =
                (int)((uint32_t)acc_re[rb][cb][r] + re_j - (uint32_t)corr[kCols + il]);
            const int im = (int)((uint32_t)acc_im[rb][cb][r] +
                                 (uint32_t)corr[kSlots + kCols + il] - ci_col_j);
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

// Piece u of a channel: u < nbc is diagonal square u; the others are tiles,
// column block by column block (column block J >= 1 holds the 2J row blocks
// above its square, J (J - 1) tiles come before it).
template <int kMode = kDense>
__device__ __forceinline__ void rect_piece(const RectParams& p, int ch, int u, int sb, int se,
                                           uint8_t* craw0, uint8_t* craw1, uint8_t* rraw0,
                                           uint8_t* rraw1, uint8_t* dec,
                                           const TriSegments* sg = nullptr) {
  if (u < p.nbc) {
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
    if (kMode == kSegments)
      tri::tri_channel_t<kSegments>(tp, ch, sb, se, craw0, craw1, dec, nullptr, tri::GathSlots{},
                                    sg);
    else
      tri::tri_channel(tp, ch, sb, se, craw0, craw1, dec);
  } else {
    const int r = u - p.nbc;
    int J = 1;
    while ((J + 1) * J <= r) ++J;
    const int I = r - J * (J - 1);
    rect_run<kMode>(p, ch, kRows * I, kCols * J, sb, se, craw0, craw1, rraw0, rraw1, dec, sg);
  }
}

__global__ __launch_bounds__(kThreads, 1) void xcorr_rect_kernel(RectParams p) {
  // Each buffer is its own variable: the compiler then tracks the loads into
  // one separately from reads of the others and waits only for those.
  __shared__ __attribute__((aligned(16))) uint8_t craw0[kColRaw];
  __shared__ __attribute__((aligned(16))) uint8_t craw1[kColRaw];
  __shared__ __attribute__((aligned(16))) uint8_t rraw0[kRowRaw];
  __shared__ __attribute__((aligned(16))) uint8_t rraw1[kRowRaw];
  __shared__ __attribute__((aligned(16))) uint8_t dec[kDecBytes];
  // logical workgroup -> (channel, piece, part of the time axis); consecutive
  // logical ids run on one XCD, so the pieces of a channel share its L2
  // (the divisions run on the vector ALU; their results are uniform, and
  // saying so keeps the buffer descriptors built from them in scalar registers)
  const int logical = xcd_logical_id(blockIdx.x, gridDim.x);
  const int per_ch = p.units * p.split;
  const int ch = __builtin_amdgcn_readfirstlane(logical / per_ch);
  const int rest = logical - ch * per_ch;
  const int u = __builtin_amdgcn_readfirstlane(rest / p.split);
  const int part = rest - u * p.split;
  const int sb = part * p.stages_per_split;
  const int se = min(sb + p.stages_per_split, p.total_stages);
  if (sb >= se) return;
  rect_piece(p, ch, u, sb, se, craw0, craw1, rraw0, rraw1, dec);
}

// The same pieces over several sample segments of each channel summed into
// one result (the runs of one gate of a gated correlation): the stage loop
// runs over the segments' stages.
__global__ __launch_bounds__(kThreads, 1) void xcorr_rect_segments_kernel(RectParams p,
                                                                          TriSegments sg) {
  __shared__ __attribute__((aligned(16))) uint8_t craw0[kColRaw];
  __shared__ __attribute__((aligned(16))) uint8_t craw1[kColRaw];
  __shared__ __attribute__((aligned(16))) uint8_t rraw0[kRowRaw];
  __shared__ __attribute__((aligned(16))) uint8_t rraw1[kRowRaw];
  __shared__ __attribute__((aligned(16))) uint8_t dec[kDecBytes];
  const int logical = xcd_logical_id(blockIdx.x, gridDim.x);
  const int per_ch = p.units * p.split;
  const int ch = __builtin_amdgcn_readfirstlane(logical / per_ch);
  const int rest = logical - ch * per_ch;
  const int u = __builtin_amdgcn_readfirstlane(rest / p.split);
  const int part = rest - u * p.split;
  const int sb = part * p.stages_per_split;
  const int se = min(sb + p.stages_per_split, p.total_stages);
  if (sb >= se) return;
  rect_piece<kSegments>(p, ch, u, sb, se, craw0, craw1, rraw0, rraw1, dec, &sg);
}

// Persistent workgroups over a queue of pieces of many jobs (batched mode and
// the server). Workgroup w serves sub-queue w % 8 (the XCD it runs on, so
// neighbouring pieces of a channel share that XCD's L2) and then steals from
// the others. Queue state that only thread 0 touches lives in LDS; the header,
// job and item are read through the constant address space per item, so none
// of it occupies registers while a piece is computed. Every workgroup leaves
// once all sub-queues are empty; the last one out resets the counters, so the
// workspace is ready for the next launch (no memset, which keeps the launch
// capturable in a graph).
struct QueueCursor {
  int next_item;
  int part;    // sub-queue being served
  int tried;   // sub-queues found empty so far
};

__global__ __launch_bounds__(kThreads, 1) void xcorr_queue_kernel(uint8_t* ws) {
  __shared__ __attribute__((aligned(16))) uint8_t craw0[kColRaw];
  __shared__ __attribute__((aligned(16))) uint8_t craw1[kColRaw];
  __shared__ __attribute__((aligned(16))) uint8_t rraw0[kRowRaw];
  __shared__ __attribute__((aligned(16))) uint8_t rraw1[kRowRaw];
  __shared__ __attribute__((aligned(16))) uint8_t dec[kDecBytes];
  __shared__ QueueCursor qc;
  if (threadIdx.x == 0) {
    qc.part = blockIdx.x % kQueueParts;
    qc.tried = 0;
  }
  while (true) {
    if (threadIdx.x == 0) {
      QueueHeader* hdr = reinterpret_cast<QueueHeader*>(ws);
      const QueueHeaderC hdr_c = (QueueHeaderC)ws;
      int part = qc.part, tried = qc.tried, it = -1;
      while (tried < kQueueParts) {
        const int b = hdr_c->part_begin[part], e = hdr_c->part_begin[part + 1];
        if (b < e) {
          const unsigned k = atomicAdd(&hdr->cursor[part], 1u);
          if ((int)k < e - b) {
            it = b + (int)k;
            break;
          }
        }
        part = (part + 1) % kQueueParts;
        ++tried;
      }
      qc.part = part;
      qc.tried = tried;
      qc.next_item = it;
    }
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(qc.next_item);
    __syncthreads();
    if (it < 0) break;
    const QueueHeaderC hdr_c = (QueueHeaderC)ws;
    const QueueItemC items = (QueueItemC)(ws + hdr_c->items_offset);
    const QueueJobC jobs = (QueueJobC)(ws + hdr_c->jobs_offset);
    const int jb = items[it].job;
    RectParams p;
    p.in = jobs[jb].in;
    p.vis = jobs[jb].vis;
    p.n = jobs[jb].n;
    p.f = jobs[jb].f;
    p.t = jobs[jb].t;
    p.ss = jobs[jb].ss;
    p.cs = jobs[jb].cs;
    p.t0 = jobs[jb].t0;
    p.t_end = jobs[jb].t_end;
    p.nbc = jobs[jb].nbc;
    p.units = jobs[jb].units;
    p.split = 1;
    p.stages_per_split = jobs[jb].total_stages;
    p.total_stages = jobs[jb].total_stages;
    p.accumulate = jobs[jb].accumulate;
    p.atomic_out = jobs[jb].atomic_out;
    rect_piece(p, items[it].ch, items[it].unit, items[it].stage_begin, items[it].stage_end, craw0,
               craw1, rraw0, rraw1, dec);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    QueueHeader* hdr = reinterpret_cast<QueueHeader*>(ws);
    __threadfence();
    const unsigned d = atomicAdd(&hdr->done, 1u);
    if (d == gridDim.x - 1) {
      for (int k = 0; k < kQueueParts; ++k) hdr->cursor[k] = 0u;
      hdr->done = 0u;
      __threadfence();
    }
  }
}

}  // namespace

int queue_stage_samples() { return kStage; }

hipError_t launch_queue(void* d_ws, int64_t items, int grid, hipStream_t stream) {
  if (items <= 0) return hipSuccess;
  if (grid <= 0) return hipErrorInvalidConfiguration;
  xcorr_queue_kernel<<<dim3((unsigned)grid), dim3(kThreads), 0, stream>>>(
      reinterpret_cast<uint8_t*>(d_ws));
  return hipGetLastError();
}

int64_t rect_units_per_channel(int n) {
  const int64_t nbc = (n + kCols - 1) / kCols;
  return nbc * nbc;
}

hipError_t launch_rect_segments(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                                int64_t cs, const int32_t* seg_t0, const int32_t* seg_t_end,
                                int count, int accumulate, int split, hipStream_t stream) {
  if (n < 1 || n % 4 != 0) return hipErrorInvalidValue;
  if (count < 1 || count > tri::kMaxSegments) return hipErrorInvalidValue;
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
  for (int k = count; k < tri::kMaxSegments; ++k) sg.t0[k] = sg.t_end[k] = 0;
  RectParams p;
  p.in = in;
  p.vis = vis;
  p.n = n;
  p.f = f;
  p.t = t;
  p.ss = ss;
  p.cs = cs;
  p.t0 = 0;
  p.t_end = t;
  p.nbc = (n + kCols - 1) / kCols;
  p.units = p.nbc * p.nbc;
  p.total_stages = stages;
  if (split < 1) split = 1;
  if (split > stages) split = stages;
  p.split = split;
  p.stages_per_split = (stages + split - 1) / split;
  p.accumulate = accumulate;
  p.atomic_out = split > 1;
  const int64_t grid = (int64_t)f * p.units * split;
  if (f <= 0 || grid <= 0 || grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  xcorr_rect_segments_kernel<<<dim3((unsigned)grid), dim3(kThreads), 0, stream>>>(p, sg);
  return hipGetLastError();
}

hipError_t launch_rect(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                       int64_t cs, int t0, int t_count, int accumulate, int split,
                       hipStream_t stream) {
  if (n < 1 || n % 4 != 0) return hipErrorInvalidValue;
  if (t_count <= 0 || t0 < 0 || (int64_t)t0 + t_count > t) return hipErrorInvalidValue;
  RectParams p;
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
  p.accumulate = accumulate;
  p.atomic_out = split > 1;
  const int64_t grid = (int64_t)f * p.units * split;
  if (f <= 0 || grid <= 0 || grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  xcorr_rect_kernel<<<dim3((unsigned)grid), dim3(kThreads), 0, stream>>>(p);
  return hipGetLastError();
}

}  // namespace xeng
