// xcorr_wide.hip -- the main gfx950 correlation kernel: 128x256 tiles, one
// workgroup per CU, accumulators held across the whole time axis.
//
// Same contraction as the 128x128 kernel (paper Sec. II-A, Eq. 1 and 2):
//   Re V_ij = P_i . P_j,  Im V_ij = Q_i . P_j,   P_e = [Re e, Im e],
//   Q_e = [Im e, -Re e]  over the time axis,
// on v_mfma_i32_32x32x32_i8. The shape is chosen for gfx950:
//   * a workgroup owns a 128 (rows, i) x 256 (columns, j) tile; each of the 4
//     waves owns 64 x 128 = 2 x 4 blocks of 32x32, Re and Im: 256 int32
//     accumulators per lane, one wave per SIMD.
//   * packed bytes are fetched with buffer loads whose row offset is a scalar
//     register (no vector ALU work per load), two stages ahead of use.
//   * LDS traffic is the scarce resource (writes run at about half the read
//     rate), so the two panels are staged differently:
//       rows (A side, needs -Re): transposed and decoded once per workgroup
//         into int8 slabs [Re g, Re g+1, Im g, Im g+1];
//       columns (B side): stored raw, one byte per sample in the input's own
//         [sample][element] order, and read with ds_read_b64_tr_b8, whose 8x8
//         byte transpose hands each lane 8 consecutive samples of its own
//         element; the lane then decodes them to 16 x [Re, Re', Im, Im'].
//   * the decode of stage s+1 is interleaved with the MFMA work of stage s,
//     and operand fragments are read one MFMA step ahead.
//
// K layout of one 16-sample step for element e, lane half h (0/1): the slab
// [Re g, Re g+1, Im g, Im g+1] with g = 2h (each dword = 4 consecutive samples
// of one component). Q is [Im g, Im g+1, -Re g, -Re g+1], which pairs sample by
// sample with P_j. The B side carries 16x the sample values; every sum is an
// exact multiple of 16 and the epilogue divides it out.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "xcorr_device.h"
#include "xcorr_launch.h"

namespace xeng {

namespace {

constexpr int kRows = 128;            // tile rows (i, the Q/P "A" side)
constexpr int kCols = 256;            // tile columns (j, the P "B" side)
constexpr int kThreads = 256;         // 4 waves, one per SIMD
constexpr int kStage = 64;            // samples per LDS stage
constexpr int kSteps = 4;             // 16-sample MFMA K steps per stage (= waves)
// Raw column panel: one row of kCols bytes per sample, padded so the eight
// rows read by one 16-lane ds_read_b64_tr_b8 group fall on distinct banks.
constexpr int kColRowStride = kCols + 32;
constexpr int kColRawBytes = kStage * kColRowStride;                // 18 KiB
constexpr int kRowPBytes = kSteps * 2 * kRows * 16;                 // 16 KiB
constexpr int kBufBytes = kColRawBytes + kRowPBytes;
constexpr uint32_t kOob = 0x80000000u;  // buffer offset past every record: load returns 0
// The B operand carries 16x the sample value and one sample adds at most 128
// to |Re|, so 16 * 128 * samples must stay below 2^31 within one launch.
constexpr int kMaxSamplesPerLaunch = (1 << 20) - kStage;

struct WideParams {
  const uint8_t* in;
  int32_t* vis;
  int n, f;
  int t;                    // samples per channel
  int64_t ss, cs;           // bytes from one sample to the next, and from one channel to the next
  int t0, t_end;            // this launch sums samples [t0, t_end)
  int nbr;                  // 128-row blocks: ceil(n / 128)
  int nbc;                  // 256-column blocks: ceil(n / 256)
  int ntiles;               // tiles per channel
  int split;                // workgroups along time per tile
  int stages_per_split;
  int total_stages;
  int accumulate;
  int atomic_out;
  int full_panels;          // n % 256 == 0: no element of any panel is out of range
};

// Raw packed dwords of one stage held by one lane: 16 rows of its column
// quad (its wave's K step) and 8 rows of its row quad (half of that step).
struct Raw {
  uint32_t col[16];
  uint32_t row[8];
};

__device__ inline __amdgpu_buffer_rsrc_t stage_rsrc(const uint8_t* chan, int64_t first_row,
                                                    int64_t ss) {
  // every valid offset used below is < 2^31; kOob is out of range
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(chan + first_row * ss), 0,
                                           0x7fffffff, 0x00020000);
}

// Fetch one stage. kChecked handles the last stage of the time axis and
// panels that run past n: rows or elements out of range become decoded zeros.
template <bool kChecked>
__device__ inline void load_stage(Raw& raw, const uint8_t* chan, int ss, int t0, int t_end,
                                  int stage, int wave, uint32_t voff_col, uint32_t voff_row,
                                  bool col_ok, bool row_ok, int half) {
  const int64_t first = t0 + (int64_t)stage * kStage + wave * 16;   // first row of this wave's step
  const __amdgpu_buffer_rsrc_t rs = stage_rsrc(chan, first, ss);
  if (!kChecked) {
#pragma unroll
    for (int r = 0; r < 16; ++r) raw.col[r] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff_col, r * ss, 0);
#pragma unroll
    for (int r = 0; r < 8; ++r) raw.row[r] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff_row, r * ss, 0);
  } else {
    const int valid = t_end - (int)first;   // rows of this step that exist
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const bool ok = col_ok && r < valid;
      const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(rs, ok ? voff_col : kOob, r * ss, 0);
      raw.col[r] = ok ? v : kZeroSamples;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const bool ok = row_ok && r + 8 * half < valid;
      const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(rs, ok ? voff_row : kOob, r * ss, 0);
      raw.row[r] = ok ? v : kZeroSamples;
    }
  }
}

// Row (A) side: transpose 8 raw rows (two 4-sample groups) of one quad and
// write, per element, the unscaled slab [Re g, Re g+1, Im g, Im g+1]. Split in
// two halves (elements 0-1, 2-3) so the work spreads over two MFMA steps.
__device__ inline void transpose_rows(const uint32_t* rows8, uint32_t x0[4], uint32_t x1[4]) {
  transpose_4x4(rows8, x0);
  transpose_4x4(rows8 + 4, x1);
}
__device__ inline void decode_rows_half(const uint32_t x0[4], const uint32_t x1[4], int part,
                                        uint8_t* pslab, int quad_base) {
#pragma unroll
  for (int kq = 0; kq < 2; ++kq) {
    const int k = 2 * part + kq;
    const int slot = slot_swizzle(quad_base + k);
    const v4i s = {(int)fields_to_s8(fields_hi(x0[k])), (int)fields_to_s8(fields_hi(x1[k])),
                   (int)fields_to_s8(fields_lo(x0[k])), (int)fields_to_s8(fields_lo(x1[k]))};
    *reinterpret_cast<v4i*>(pslab + slot * 16) = s;
  }
}

// Offset form of the row slabs (8-wave kernel): the Excess-8 fields
// themselves, [uRe g, uRe g+1, uIm g, uIm g+1]. The per-element field sums
// are added into sr[k] (Re) and si[k] (Im) for the lane's 4 row elements;
// the caller folds them into LDS once, after the last stage.
__device__ inline void decode_rows_fields(const uint32_t x0[4], const uint32_t x1[4], int part,
                                          uint8_t* pslab, int quad_base, uint32_t sr[4],
                                          uint32_t si[4]) {
#pragma unroll
  for (int kq = 0; kq < 2; ++kq) {
    const int k = 2 * part + kq;
    const int slot = slot_swizzle(quad_base + k);
    const uint32_t r0 = fields_hi(x0[k]), r1 = fields_hi(x1[k]);
    const uint32_t i0 = fields_lo(x0[k]), i1 = fields_lo(x1[k]);
    *reinterpret_cast<v4i*>(pslab + slot * 16) = v4i{(int)r0, (int)r1, (int)i0, (int)i1};
    sr[k] = __builtin_amdgcn_sad_u8(r1, 0u, __builtin_amdgcn_sad_u8(r0, 0u, sr[k]));
    si[k] = __builtin_amdgcn_sad_u8(i1, 0u, __builtin_amdgcn_sad_u8(i0, 0u, si[k]));
  }
}

// Column (B) side: 16 raw rows of the lane's quad go to LDS unchanged.
__device__ inline void write_cols_raw(const uint32_t* rows16, uint8_t* dst) {
#pragma unroll
  for (int r = 0; r < 16; ++r)
    *reinterpret_cast<uint32_t*>(dst + r * kColRowStride) = rows16[r];
}

// 16 x [Re, Im] of four samples from four raw bytes. With u = w ^ 0x88 per
// byte, u's high nibble is the 4-bit two's complement of Re, so u & 0xF0 is
// exactly 16*Re as a signed byte, and (u << 4) & 0xF0 is 16*Im.
__device__ inline uint32_t re16(uint32_t w) { return (w ^ kZeroSamples) & 0xF0F0F0F0u; }
__device__ inline uint32_t im16(uint32_t w) { return ((w ^ kZeroSamples) << 4) & 0xF0F0F0F0u; }

// Negated signed bytes in [-8, 7]: x ^ 0x7F + 1 stays below 0x100 per byte
// (no carry), and flipping bit 7 turns the biased result back into -x.
__device__ inline uint32_t neg_s8(uint32_t x) {
  return ((x ^ 0x7F7F7F7Fu) + 0x01010101u) ^ 0x80808080u;
}

// Tile t of a channel -> (row block bi of 128, column block bj of 256). Tiles
// are ordered column block by column block; column block J holds the row
// blocks I <= 2J+1, the ones that reach the upper triangle.
__device__ inline void tile_coords(int tile, int nbr, int* bi_out, int* bj_out) {
  int bj = 0, bi = tile;
  while (true) {
    const int cnt = min(2 * bj + 2, nbr);
    if (bi < cnt) break;
    bi -= cnt;
    ++bj;
  }
  *bi_out = bi;
  *bj_out = bj;
}

__global__ __launch_bounds__(kThreads, 1) void xcorr_wide_kernel(WideParams p) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[2 * kBufBytes];

  // ---- tile, channel and time range of this workgroup --------------------------
  const int logical = xcd_logical_id(blockIdx.x, gridDim.x);
  const int tile = logical % p.ntiles;
  const int rest = logical / p.ntiles;
  const int split_idx = rest % p.split;
  const int ch = rest / p.split;
  // tiles are ordered column block by column block; column block J holds the
  // row blocks I <= 2J+1 (those that reach the upper triangle)
  int bj = 0, bi = tile;
  while (true) {
    const int cnt = min(2 * bj + 2, p.nbr);
    if (bi < cnt) break;
    bi -= cnt;
    ++bj;
  }
  const int row0 = bi * kRows, col0 = bj * kCols;
  const int stage_begin = split_idx * p.stages_per_split;
  const int stage_end = min(stage_begin + p.stages_per_split, p.total_stages);
  if (stage_begin >= stage_end) return;

  const int tid = threadIdx.x;
  // the wave index is uniform across the wave; say so, so that the buffer
  // descriptors built from it stay in scalar registers
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int half = lane >> 5, l32 = lane & 31;
  const int n = p.n;
  const uint8_t* chan = p.in + (int64_t)ch * p.cs;
  const int ss = (int)p.ss;

  // ---- staging roles: column quad = lane, row quad = l32 (rows 8*half..) --------
  const int col_e = col0 + 4 * lane;
  const int row_e = row0 + 4 * l32;
  const bool col_ok = col_e < n, row_ok = row_e < n;
  const uint32_t voff_col = (uint32_t)col_e;
  const uint32_t voff_row = (uint32_t)row_e + (uint32_t)(8 * half) * (uint32_t)ss;
  const bool panels_full = p.full_panels != 0;

  // LDS destinations of this lane's staged data: its 16 raw column rows
  // (samples 16*wave.. of the stage, elements 4*lane..) and its row slabs
  auto col_raw = [&](int buf) {
    return lds + buf * kBufBytes + (wave * 16) * kColRowStride + 4 * lane;
  };
  auto row_slab = [&](int buf) {
    return lds + buf * kBufBytes + kColRawBytes + ((wave * 2 + half) * kRows) * 16;
  };

  auto fetch = [&](Raw& raw, int stage) {
    const bool tail = p.t0 + (int64_t)stage * kStage + wave * 16 + 16 > p.t_end;
    if (panels_full && !tail)
      load_stage<false>(raw, chan, ss, p.t0, p.t_end, stage, wave, voff_col, voff_row, col_ok,
                        row_ok, half);
    else
      load_stage<true>(raw, chan, ss, p.t0, p.t_end, stage, wave, voff_col, voff_row, col_ok,
                       row_ok, half);
  };

  // ---- MFMA roles ------------------------------------------------------------------
  const int wr = wave >> 1, wc = wave & 1;
  bool active[2][4];
  bool wave_active = false;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int rs = row0 + wr * 64 + rb * 32, cs = col0 + wc * 128 + cb * 32;
      active[rb][cb] = rs <= cs + 31 && rs < n && cs < n;
      wave_active |= active[rb][cb];
    }
  int a_off[2];   // slot index of this lane's A slabs within one K step
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
    a_off[rb] = (half * kRows + slot_swizzle(wr * 64 + rb * 32 + l32));
  // ds_read_b64_tr_b8 addressing: in each 16-lane group the even lanes name
  // the 8 sample rows of elements e0..e0+7 and the odd lanes those of
  // e0+8..e0+15; lane k of the group receives element e0+k, 8 samples. Group
  // g = (lane/16) covers elements 16*(g&1).. of the block, samples 8*(g>>1)..
  const int grp = (lane >> 4) & 3;
  const int b_off = ((grp >> 1) * 8 + ((lane & 15) >> 1)) * kColRowStride + wc * 128 +
                    16 * (grp & 1) + 8 * (lane & 1);

  v16i acc_re[2][4], acc_im[2][4];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      acc_re[rb][cb] = v16i{};
      acc_im[rb][cb] = v16i{};
    }

  // Operand fragments of one 16-sample MFMA step: A slabs (decoded) and B raw
  // bytes (8 samples of this lane's column element per block).
  struct Frags {
    v4i pa[2];
    v2i rb[4];
  };
  auto load_frags = [&](Frags& fr, const uint8_t* base, int kk) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
      fr.pa[rb] = *reinterpret_cast<const v4i*>(base + kColRawBytes +
                                                (kk * 2 * kRows + a_off[rb]) * 16);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
      fr.rb[cb] = __builtin_amdgcn_ds_read_tr8_b64_v2i32(
          (__attribute__((address_space(3))) v2i*)(base + b_off + kk * 16 * kColRowStride +
                                                   cb * 32));
  };
  // All 8 blocks of the wave. Blocks lying below the diagonal are computed and
  // never stored: the busiest wave of the tile sets the stage time anyway.
  auto mfma_step = [&](const Frags& fr) {
    v4i pb[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const uint32_t lo = (uint32_t)fr.rb[cb].x, hi = (uint32_t)fr.rb[cb].y;
      pb[cb] = v4i{(int)re16(lo), (int)re16(hi), (int)im16(lo), (int)im16(hi)};
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const v4i qa = {fr.pa[rb].z, fr.pa[rb].w, (int)neg_s8((uint32_t)fr.pa[rb].x),
                      (int)neg_s8((uint32_t)fr.pa[rb].y)};
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        acc_re[rb][cb] =
            __builtin_amdgcn_mfma_i32_32x32x32_i8(fr.pa[rb], pb[cb], acc_re[rb][cb], 0, 0, 0);
        acc_im[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(qa, pb[cb], acc_im[rb][cb], 0, 0, 0);
      }
    }
  };

  // One stage: MFMA over buffer `cur` with the operands of step k+1 loaded
  // while step k multiplies; meanwhile decode `dec` (the next stage) into
  // buffer cur^1 in four slices, and fetch stage `ld_stage` into `ld`.
  // kFast: the fetched stage lies wholly inside the time window and the
  // panels, so the fetch is unchecked and the body is one straight block.
  // Otherwise do_dec / do_ld say what this (late) stage still has to do.
  auto body = [&](auto fast_tag, int cur, Raw& dec, Raw& ld, int ld_stage, bool do_dec,
                  bool do_ld) {
    constexpr bool kFast = decltype(fast_tag)::value;
    const uint8_t* base = lds + cur * kBufBytes;
    Frags f0, f1;
    uint32_t tx0[4], tx1[4];
    // Order inside one MFMA step: the next step's LDS reads go out first, then
    // each MFMA is followed by a few VALU ops (decode work), and the LDS
    // writes of the decoded data come last.
    auto pattern = []() {
      __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);    // DS reads
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);  // VALU
      }
      __builtin_amdgcn_sched_group_barrier(0x200, 16, 0);   // DS writes
    };
    __builtin_amdgcn_sched_barrier(0);
    load_frags(f0, base, 0);
    if (kFast)
      load_stage<false>(ld, chan, ss, p.t0, p.t_end, ld_stage, wave, voff_col, voff_row, col_ok,
                        row_ok, half);
    else if (do_ld)
      load_stage<true>(ld, chan, ss, p.t0, p.t_end, ld_stage, wave, voff_col, voff_row, col_ok,
                       row_ok, half);
    __builtin_amdgcn_sched_barrier(0);
    load_frags(f1, base, 1);
    if (kFast || do_dec) write_cols_raw(dec.col, col_raw(cur ^ 1));
    mfma_step(f0);
    if (kFast) pattern();
    __builtin_amdgcn_sched_barrier(0);
    load_frags(f0, base, 2);
    if (kFast || do_dec) transpose_rows(dec.row, tx0, tx1);
    mfma_step(f1);
    if (kFast) pattern();
    __builtin_amdgcn_sched_barrier(0);
    load_frags(f1, base, 3);
    if (kFast || do_dec) decode_rows_half(tx0, tx1, 0, row_slab(cur ^ 1), 4 * l32);
    mfma_step(f0);
    if (kFast) pattern();
    __builtin_amdgcn_sched_barrier(0);
    if (kFast || do_dec) decode_rows_half(tx0, tx1, 1, row_slab(cur ^ 1), 4 * l32);
    mfma_step(f1);
    if (kFast) pattern();
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
  };

  Raw ra, rb_;
  fetch(ra, stage_begin);
  if (stage_begin + 1 < stage_end) fetch(rb_, stage_begin + 1);
  {
    uint32_t tx0[4], tx1[4];
    write_cols_raw(ra.col, col_raw(0));
    transpose_rows(ra.row, tx0, tx1);
    decode_rows_half(tx0, tx1, 0, row_slab(0), 4 * l32);
    decode_rows_half(tx0, tx1, 1, row_slab(0), 4 * l32);
  }
  __syncthreads();
  // Steady state, two stages per trip (buffers 0 and 1, register sets in
  // fixed roles): every stage fetched here is wholly in range.
  const int full_stages = panels_full ? (p.t_end - p.t0) / kStage : 0;
  const int fast_end = min(stage_end, full_stages);
  int s = stage_begin;
  for (; s + 3 < fast_end; s += 2) {
    body(std::true_type{}, 0, rb_, ra, s + 2, true, true);
    body(std::true_type{}, 1, ra, rb_, s + 3, true, true);
  }
  // The remaining stages one at a time; the buffer parity continues from s.
  // Each parity names its register sets statically (a run-time choice between
  // the two would force them into memory).
  for (; s < stage_end; ++s) {
    const bool do_dec = s + 1 < stage_end, do_ld = s + 2 < stage_end;
    if (((s - stage_begin) & 1) == 0)
      body(std::false_type{}, 0, rb_, ra, s + 2, do_dec, do_ld);
    else
      body(std::false_type{}, 1, ra, rb_, s + 2, do_dec, do_ld);
  }

  // ---- epilogue: masked writes of i <= j into the packed triangle ---------------
  if (!wave_active) return;
  const int64_t n64 = n;
  const int64_t entries = n64 * (n64 + 1) / 2;
  int32_t* out = p.vis + (int64_t)ch * entries * 2;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      if (!active[rb][cb]) continue;
      const int j = col0 + wc * 128 + cb * 32 + l32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = row0 + wr * 64 + rb * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        if (i <= j && j < n) {
          int32_t* o = out + 2 * tri_index(n64, i, j);
          // the B operand is scaled by 16: every sum is an exact multiple of 16
          const int re = acc_re[rb][cb][r] >> 4, im = acc_im[rb][cb][r] >> 4;
          if (p.atomic_out) {
            atomicAdd(o, re);
            atomicAdd(o + 1, im);
          } else if (p.accumulate) {
            const v2i old = *reinterpret_cast<const v2i*>(o);
            *reinterpret_cast<v2i*>(o) = v2i{old.x + re, old.y + im};
          } else {
            *reinterpret_cast<v2i*>(o) = v2i{re, im};
          }
        }
      }
    }
}


// ---------------------------------------------------------------------------
// Two waves per SIMD: the same 128x256 tile and stage length, but 8 waves of
// 64x64 (2x2 blocks, 128 accumulators each). The two waves that share a SIMD
// own the same 64 columns and complementary staging duties (waves 0-3 decode
// the row panel of K step `wave`, waves 4-7 the column panel of K step
// `wave-4`), so while one waits on memory or LDS the other keeps the SIMD's
// matrix core busy. Both panels are decoded once per workgroup into 16-byte
// slabs, so the MFMA steps read both operands ready to use.
constexpr int kThreads8 = 512;
// LDS of the 8-wave kernel, per stage buffer: the column panel decoded into
// 16-byte slabs [uRe g, uRe g+1, uIm g, uIm g+1] per (K step, lane half,
// column), then the row slabs in the same format; after both buffers the
// row and column field sums.
constexpr int kColSlabBytes = kSteps * 2 * kCols * 16;                // 32 KiB
constexpr int kBufBytes8 = kColSlabBytes + kRowPBytes;

struct Raw16 {
  uint32_t w[16];
};

// One tile of one channel over stages [stage_begin, stage_end) of the launch
// window in p.
__device__ __forceinline__ void wide8_tile(const WideParams& p, uint8_t* lds, int ch, int bi,
                                           int bj, int stage_begin, int stage_end) {
  const int row0 = bi * kRows, col0 = bj * kCols;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int half = lane >> 5, l32 = lane & 31;
  const int n = p.n;
  const uint8_t* chan = p.in + (int64_t)ch * p.cs;
  const int ss = (int)p.ss;
  const bool panels_full = p.full_panels != 0;
  const int ks = wave & 3;               // K step this wave stages
  const bool row_role = wave < 4;

  // staging addresses
  const int col_e = col0 + 4 * lane;
  const int row_e = row0 + 4 * l32;
  const bool col_ok = col_e < n, row_ok = row_e < n;
  const uint32_t voff_col = (uint32_t)col_e;
  const uint32_t voff_row = (uint32_t)row_e + (uint32_t)(8 * half) * (uint32_t)ss;
  uint8_t* const col_dst0 = lds + ((ks * 2) * kCols) * 16;     // lane half 0; half 1 follows
  uint8_t* const row_dst0 = lds + kColSlabBytes + ((ks * 2 + half) * kRows) * 16;

  // MFMA roles: rows 64*wr.., columns 64*wc..
  const int wr = wave >> 2, wc = wave & 3;
  bool wave_active = false;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int rs = row0 + wr * 64 + rb * 32, cs = col0 + wc * 64 + cb * 32;
      wave_active |= rs <= cs + 31 && rs < n && cs < n;
    }
  int a_off[2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
    a_off[rb] = (half * kRows + slot_swizzle(wr * 64 + rb * 32 + l32));
  int b_off[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
    b_off[cb] = (half * kCols + slot_swizzle(wc * 64 + cb * 32 + l32));

  v16i acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      acc_re[rb][cb] = v16i{};
      acc_im[rb][cb] = v16i{};
    }

  // Field sums for the offset corrections, kept in registers by the staging
  // waves as they decode (row waves for their 4 row elements, column waves
  // for their 4 columns) and added into row_sums / col_sums in LDS after the
  // last stage.
  uint32_t* const row_sums = reinterpret_cast<uint32_t*>(lds + 2 * kBufBytes8);   // [re, im][128]
  uint32_t* const col_sums = row_sums + 2 * kRows;                               // [re, im][256]
  uint32_t csum_re[4] = {0, 0, 0, 0}, csum_im[4] = {0, 0, 0, 0};
  uint32_t rsum_re[4] = {0, 0, 0, 0}, rsum_im[4] = {0, 0, 0, 0};
  for (int e = tid; e < 2 * kRows + 2 * kCols; e += kThreads8) row_sums[e] = 0u;
  __syncthreads();

  struct Frags {
    v4i pa[2];
    v4i pb[2];
  };
  auto load_frags = [&](Frags& fr, const uint8_t* base, int kk) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
      fr.pa[rb] = *reinterpret_cast<const v4i*>(base + kColSlabBytes +
                                                (kk * 2 * kRows + a_off[rb]) * 16);
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
      fr.pb[cb] = *reinterpret_cast<const v4i*>(base + (kk * 2 * kCols + b_off[cb]) * 16);
  };
  // Offset arithmetic (Sec. III-A, Eq. 3) on the Excess-8 fields u in [0, 15]:
  // P = [uRe, uIm] both sides, Q = [uIm, 15 - uRe] on the row side; the field
  // sums correct the products in the epilogue.
  auto mfma_step = [&](const Frags& fr) {
    const v4i* const pb = fr.pb;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const v4i qa = {fr.pa[rb].z, fr.pa[rb].w, (int)((uint32_t)fr.pa[rb].x ^ 0x0F0F0F0Fu),
                      (int)((uint32_t)fr.pa[rb].y ^ 0x0F0F0F0Fu)};
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        acc_re[rb][cb] =
            __builtin_amdgcn_mfma_i32_32x32x32_i8(fr.pa[rb], pb[cb], acc_re[rb][cb], 0, 0, 0);
        acc_im[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(qa, pb[cb], acc_im[rb][cb], 0, 0, 0);
      }
    }
  };

  // Fetch this wave's share of one stage: row waves 8 rows of their row quad
  // (half of K step ks), column waves 16 rows of their column quad.
  auto fetch = [&](auto row_tag, Raw16& raw, int stage, bool checked) {
    constexpr bool kRow = decltype(row_tag)::value;
    const int64_t first = p.t0 + (int64_t)stage * kStage + ks * 16;
    const __amdgpu_buffer_rsrc_t rs = stage_rsrc(chan, first, ss);
    const int valid = p.t_end - (int)first;
    if (kRow) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        if (!checked) {
          raw.w[r] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff_row, r * ss, 0);
        } else {
          const bool ok = row_ok && r + 8 * half < valid;
          const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(rs, ok ? voff_row : kOob, r * ss, 0);
          raw.w[r] = ok ? v : 0u;
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if (!checked) {
          raw.w[r] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff_col, r * ss, 0);
        } else {
          const bool ok = col_ok && r < valid;
          const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(rs, ok ? voff_col : kOob, r * ss, 0);
          raw.w[r] = ok ? v : 0u;
        }
      }
    }
  };
  auto stage_checked = [&](int stage) {
    return !panels_full || p.t0 + (int64_t)stage * kStage + ks * 16 + 16 > p.t_end;
  };

  auto run = [&](auto row_tag, auto mfma_tag) {
    constexpr bool kRow = decltype(row_tag)::value;
    constexpr bool kMfma = decltype(mfma_tag)::value;
    // staging slices, spread over the four MFMA steps of a stage
    auto slice = [&](int seg, Raw16& dec, int buf, uint32_t* tx0, uint32_t* tx1) {
      if (kRow) {
        if (seg == 1) transpose_rows(dec.w, tx0, tx1);
        if (seg == 2)
          decode_rows_fields(tx0, tx1, 0, row_dst0 + buf * kBufBytes8, 4 * l32, rsum_re, rsum_im);
        if (seg == 3)
          decode_rows_fields(tx0, tx1, 1, row_dst0 + buf * kBufBytes8, 4 * l32, rsum_re, rsum_im);
      } else {
        // the lane's 4 columns: samples 0-7 (lane half 0 of the MFMA
        // operands) in slices 1-2, samples 8-15 in slices 2-3
        uint8_t* const dst = col_dst0 + buf * kBufBytes8;
        if (seg == 1) {
          transpose_rows(dec.w, tx0, tx1);
          decode_rows_fields(tx0, tx1, 0, dst, 4 * lane, csum_re, csum_im);
          decode_rows_fields(tx0, tx1, 1, dst, 4 * lane, csum_re, csum_im);
        }
        if (seg == 2) {
          transpose_rows(dec.w + 8, tx0, tx1);
          decode_rows_fields(tx0, tx1, 0, dst + kCols * 16, 4 * lane, csum_re, csum_im);
        }
        if (seg == 3) decode_rows_fields(tx0, tx1, 1, dst + kCols * 16, 4 * lane, csum_re, csum_im);
      }
    };
    auto body = [&](auto fast_tag, int cur, Raw16& dec, Raw16& ld, int ld_stage, bool do_dec,
                    bool do_ld) {
      constexpr bool kFast = decltype(fast_tag)::value;
      const uint8_t* base = lds + cur * kBufBytes8;
      Frags f0, f1;
      uint32_t tx0[4], tx1[4];
      __builtin_amdgcn_sched_barrier(0);
      if (kMfma) load_frags(f0, base, 0);
      if (kFast) fetch(row_tag, ld, ld_stage, false);
      else if (do_ld) fetch(row_tag, ld, ld_stage, stage_checked(ld_stage));
      __builtin_amdgcn_sched_barrier(0);
      if (kMfma) load_frags(f1, base, 1);
      if (kFast || do_dec) slice(1, dec, cur ^ 1, tx0, tx1);
      if (kMfma) mfma_step(f0);
      __builtin_amdgcn_sched_barrier(0);
      if (kMfma) load_frags(f0, base, 2);
      if (kFast || do_dec) slice(2, dec, cur ^ 1, tx0, tx1);
      if (kMfma) mfma_step(f1);
      __builtin_amdgcn_sched_barrier(0);
      if (kMfma) load_frags(f1, base, 3);
      if (kFast || do_dec) slice(3, dec, cur ^ 1, tx0, tx1);
      if (kMfma) mfma_step(f0);
      __builtin_amdgcn_sched_barrier(0);
      if (kMfma) mfma_step(f1);
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();
    };

    Raw16 ra, rb_;
    fetch(row_tag, ra, stage_begin, stage_checked(stage_begin));
    if (stage_begin + 1 < stage_end)
      fetch(row_tag, rb_, stage_begin + 1, stage_checked(stage_begin + 1));
    {
      uint32_t tx0[4], tx1[4];
      slice(1, ra, 0, tx0, tx1);
      slice(2, ra, 0, tx0, tx1);
      slice(3, ra, 0, tx0, tx1);
    }
    __syncthreads();
    const int full_stages = panels_full ? (p.t_end - p.t0) / kStage : 0;
    const int fast_end = min(stage_end, full_stages);
    int s = stage_begin;
    for (; s + 3 < fast_end; s += 2) {
      body(std::true_type{}, 0, rb_, ra, s + 2, true, true);
      body(std::true_type{}, 1, ra, rb_, s + 3, true, true);
    }
    for (; s < stage_end; ++s) {
      const bool do_dec = s + 1 < stage_end, do_ld = s + 2 < stage_end;
      if (((s - stage_begin) & 1) == 0)
        body(std::false_type{}, 0, rb_, ra, s + 2, do_dec, do_ld);
      else
        body(std::false_type{}, 1, ra, rb_, s + 2, do_dec, do_ld);
    }
  };
  if (row_role) {
    if (wave_active) run(std::true_type{}, std::true_type{});
    else run(std::true_type{}, std::false_type{});
  } else {
    if (wave_active) run(std::false_type{}, std::true_type{});
    else run(std::false_type{}, std::false_type{});
  }

  // ---- offset corrections -------------------------------------------------------
  // per row element of the tile: 8 (SR + SI) and 8 (SR - SI), from row_sums;
  // per column: 8 (SR + SI) and 8 SR + 7 SI, from this wave's column sums.
  // The staging waves add their field sums now (every wave reaches the
  // barrier below).
  if (!row_role) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      atomicAdd(col_sums + 4 * lane + k, csum_re[k]);
      atomicAdd(col_sums + kCols + 4 * lane + k, csum_im[k]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      atomicAdd(row_sums + 4 * l32 + k, rsum_re[k]);
      atomicAdd(row_sums + kRows + 4 * l32 + k, rsum_im[k]);
    }
  }
  __syncthreads();
  if (!wave_active) return;
  // samples this tile summed: stages [stage_begin, stage_end) within t_end
  const int64_t t_first = p.t0 + (int64_t)stage_begin * kStage;
  const int64_t t_last = min((int64_t)p.t_end, p.t0 + (int64_t)stage_end * kStage);
  const uint32_t re_const = 128u * (uint32_t)max((int64_t)0, t_last - t_first);
  const int64_t n64 = n;
  const int64_t entries = n64 * (n64 + 1) / 2;
  int32_t* out = p.vis + (int64_t)ch * entries * 2;
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int jl = wc * 64 + cb * 32 + l32;
    const uint32_t csr = col_sums[jl], csi = col_sums[kCols + jl];
    const uint32_t re_j = re_const - 8u * (csr + csi);
    const uint32_t ci_j = 8u * csr + 7u * csi;
    const int j = col0 + wc * 64 + cb * 32 + l32;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int il = wr * 64 + rb * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        const int i = row0 + il;
        if (i <= j && j < n) {
          int32_t* o = out + 2 * tri_index(n64, i, j);
          // int32 arithmetic modulo 2^32: the uncorrected sums may wrap
          const uint32_t sr = row_sums[il], si = row_sums[kRows + il];
          const int re = (int)((uint32_t)acc_re[rb][cb][r] + re_j - 8u * (sr + si));
          const int im = (int)((uint32_t)acc_im[rb][cb][r] + 8u * (sr - si) - ci_j);
          if (p.atomic_out) {
            atomicAdd(o, re);
            atomicAdd(o + 1, im);
          } else if (p.accumulate) {
            const v2i old = *reinterpret_cast<const v2i*>(o);
            *reinterpret_cast<v2i*>(o) = v2i{old.x + re, old.y + im};
          } else {
            *reinterpret_cast<v2i*>(o) = v2i{re, im};
          }
        }
      }
    }
  }
}
__global__ __launch_bounds__(kThreads8, 1) void xcorr_wide8_kernel(WideParams p) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[2 * kBufBytes8 + 2 * kRows * 4 + 2 * kCols * 4];
  // With two waves per SIMD each wave has 256 registers. An AGPR operand here
  // tells the compiler the kernel uses accumulation registers, so it splits
  // them 128 VGPR + 128 AGPR and keeps the 128 accumulators out of the VGPRs.
  asm volatile("; accumulators live in AGPRs" ::"a"(0));
  const int logical = xcd_logical_id(blockIdx.x, gridDim.x);
  const int tile = logical % p.ntiles;
  const int rest = logical / p.ntiles;
  const int split_idx = rest % p.split;
  const int ch = rest / p.split;
  int bi, bj;
  tile_coords(tile, p.nbr, &bi, &bj);
  const int stage_begin = split_idx * p.stages_per_split;
  const int stage_end = min(stage_begin + p.stages_per_split, p.total_stages);
  if (stage_begin >= stage_end) return;
  wide8_tile(p, lds, ch, bi, bj, stage_begin, stage_end);
}


}  // namespace

int64_t wide_tiles_per_channel(int n) {
  const int nbr = (n + kRows - 1) / kRows, nbc = (n + kCols - 1) / kCols;
  int64_t cnt = 0;
  for (int j = 0; j < nbc; ++j) cnt += (2 * j + 2 < nbr) ? 2 * j + 2 : nbr;
  return cnt;
}

int64_t wide_max_samples_per_launch() { return kMaxSamplesPerLaunch; }


hipError_t launch_wide(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                       int64_t cs, int t0, int t_count, int accumulate, int split, int waves,
                       hipStream_t stream) {
  if (t_count <= 0 || t_count > kMaxSamplesPerLaunch || t0 < 0 || t0 + t_count > t)
    return hipErrorInvalidValue;
  WideParams p;
  p.in = in;
  p.vis = vis;
  p.n = n;
  p.f = f;
  p.t = t;
  p.ss = ss;
  p.cs = cs;
  p.t0 = t0;
  p.t_end = t0 + t_count;
  p.nbr = (n + kRows - 1) / kRows;
  p.nbc = (n + kCols - 1) / kCols;
  p.ntiles = (int)wide_tiles_per_channel(n);
  p.total_stages = (t_count + kStage - 1) / kStage;
  if (split < 1) split = 1;
  if (split > p.total_stages) split = p.total_stages;
  p.split = split;
  p.stages_per_split = (p.total_stages + split - 1) / split;
  p.accumulate = accumulate;
  p.atomic_out = split > 1;
  p.full_panels = (n % kCols) == 0;
  const int64_t grid = (int64_t)p.ntiles * f * split;
  if (grid <= 0 || grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  if (waves == 8)
    xcorr_wide8_kernel<<<dim3((unsigned)grid), dim3(kThreads8), 0, stream>>>(p);
  else
    xcorr_wide_kernel<<<dim3((unsigned)grid), dim3(kThreads), 0, stream>>>(p);
  return hipGetLastError();
}

}  // namespace xeng
