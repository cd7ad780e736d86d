// xcorr_wide.hip -- the main gfx950 correlation kernel: 128x256 tiles, one
// workgroup per CU, accumulators held across the whole time axis.
//
// Same contraction as the 128x128 kernel (paper Sec. II-A, Eq. 1 and 2):
//   Re V_ij = P_i . P_j,  Im V_ij = Q_i . P_j,   P_e = [Re e, Im e],
//   Q_e = [Im e, -Re e]  over the time axis,
// on v_mfma_i32_32x32x32_i8. What changes is the shape, chosen for gfx950:
//   * a workgroup owns a 128 (rows, i) x 256 (columns, j) tile; each of the 4
//     waves owns 64 x 128 = 2 x 4 blocks of 32x32, Re and Im: 256 int32
//     accumulators per lane, one wave per SIMD. Larger tiles amortise the
//     nibble decode (done once per staged byte) over more MFMA work.
//   * packed bytes are fetched with buffer loads whose row offset is a scalar
//     register, so a load costs no vector ALU work; each wave fetches its own
//     16-sample MFMA step of both panels, two stages ahead of use.
//   * the decode of stage s+1 (transpose, Excess-8 -> int8, LDS write) is
//     interleaved with the MFMA work of stage s.
//
// K layout of one 16-sample step for element e, lane half h (0/1): the slab
// [Re g, Re g+1, Im g, Im g+1] (g = 2h; each dword = 4 samples of one
// component), plus a plane [-Re g, -Re g+1]. The Q operand is then
// [Im g, Im g+1, -Re g, -Re g+1]: the slab's upper half followed by the plane,
// which pairs sample by sample with P_j = [Re g, Re g+1, Im g, Im g+1].
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
constexpr int kColPBytes = kSteps * 2 * kCols * 16;
constexpr int kRowPBytes = kSteps * 2 * kRows * 16;
constexpr int kRowNaBytes = kSteps * 2 * kRows * 8;
constexpr int kBufBytes = kColPBytes + kRowPBytes + kRowNaBytes;   // 56 KiB
constexpr uint32_t kOob = 0x80000000u;  // buffer offset past every record: load returns 0
// The B operand carries 16x the sample value and one sample adds at most 128
// to |Re|, so 16 * 128 * samples must stay below 2^31 within one launch.
constexpr int kMaxSamplesPerLaunch = (1 << 20) - kStage;

struct WideParams {
  const uint8_t* in;
  int32_t* vis;
  int n, f;
  int t;                    // samples per channel (channel stride is t * n bytes)
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
                                                    int64_t n) {
  // every valid offset used below is < 2^31; kOob is out of range
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(chan + first_row * n), 0,
                                           0x7fffffff, 0x00020000);
}

// Fetch one stage. kChecked handles the last stage of the time axis and
// panels that run past n: rows or elements out of range become decoded zeros.
template <bool kChecked>
__device__ inline void load_stage(Raw& raw, const uint8_t* chan, int n, int t0, int t_end,
                                  int stage, int wave, uint32_t voff_col, uint32_t voff_row,
                                  bool col_ok, bool row_ok, int half) {
  const int64_t first = t0 + (int64_t)stage * kStage + wave * 16;   // first row of this wave's step
  const __amdgpu_buffer_rsrc_t rs = stage_rsrc(chan, first, n);
  if (!kChecked) {
#pragma unroll
    for (int r = 0; r < 16; ++r) raw.col[r] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff_col, r * n, 0);
#pragma unroll
    for (int r = 0; r < 8; ++r) raw.row[r] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff_row, r * n, 0);
  } else {
    const int valid = t_end - (int)first;   // rows of this step that exist
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const bool ok = col_ok && r < valid;
      const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(rs, ok ? voff_col : kOob, r * n, 0);
      raw.col[r] = ok ? v : kZeroSamples;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const bool ok = row_ok && r + 8 * half < valid;
      const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(rs, ok ? voff_row : kOob, r * n, 0);
      raw.row[r] = ok ? v : kZeroSamples;
    }
  }
}

// Column (B) side: decode 8 raw rows (two 4-sample groups) of one quad and
// write, per element, the slab [16 Re g, 16 Re g+1, 16 Im g, 16 Im g+1].
// Scaling by 16 makes the decode two operations per dword: with u = w ^ 0x88
// per nibble, u's high nibble is the 4-bit two's complement of Re, so
// (u & 0xF0) is exactly 16*Re as a signed byte, and (u << 4) & 0xF0 is 16*Im.
// Every product on the B side is then 16x; the epilogue divides exactly.
__device__ inline void decode_cols(const uint32_t* rows8, uint8_t* pslab, int quad_base) {
  uint32_t x0[4], x1[4];
  transpose_4x4(rows8, x0);        // group g:   element k at samples 0..3
  transpose_4x4(rows8 + 4, x1);    // group g+1
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int slot = slot_swizzle(quad_base + k);
    const uint32_t u0 = x0[k] ^ kZeroSamples, u1 = x1[k] ^ kZeroSamples;
    const v4i s = {(int)(u0 & 0xF0F0F0F0u), (int)(u1 & 0xF0F0F0F0u),
                   (int)((u0 << 4) & 0xF0F0F0F0u), (int)((u1 << 4) & 0xF0F0F0F0u)};
    *reinterpret_cast<v4i*>(pslab + slot * 16) = s;
  }
}

// Row (A) side, unscaled: per element the slab [Re g, Re g+1, Im g, Im g+1]
// and the plane [-Re g, -Re g+1]. Split in two halves (elements 0-1, 2-3) so
// the work can be spread over two MFMA steps; x0/x1 carry the transposes.
__device__ inline void transpose_rows(const uint32_t* rows8, uint32_t x0[4], uint32_t x1[4]) {
  transpose_4x4(rows8, x0);
  transpose_4x4(rows8 + 4, x1);
}
__device__ inline void decode_rows_half(const uint32_t x0[4], const uint32_t x1[4], int part,
                                        uint8_t* pslab, uint8_t* naslab, int quad_base) {
#pragma unroll
  for (int kq = 0; kq < 2; ++kq) {
    const int k = 2 * part + kq;
    const int slot = slot_swizzle(quad_base + k);
    const uint32_t h0 = fields_hi(x0[k]), h1 = fields_hi(x1[k]);
    const v4i s = {(int)fields_to_s8(h0), (int)fields_to_s8(h1),
                   (int)fields_to_s8(fields_lo(x0[k])), (int)fields_to_s8(fields_lo(x1[k]))};
    *reinterpret_cast<v4i*>(pslab + slot * 16) = s;
    const v2i na = {(int)fields_to_neg_s8(h0), (int)fields_to_neg_s8(h1)};
    *reinterpret_cast<v2i*>(naslab + slot * 8) = na;
  }
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
  const uint8_t* chan = p.in + (int64_t)ch * p.t * (int64_t)n;

  // ---- staging roles: column quad = lane, row quad = l32 (rows 8*half..) --------
  const int col_e = col0 + 4 * lane;
  const int row_e = row0 + 4 * l32;
  const bool col_ok = col_e < n, row_ok = row_e < n;
  const uint32_t voff_col = (uint32_t)col_e;
  const uint32_t voff_row = (uint32_t)row_e + (uint32_t)(8 * half) * (uint32_t)n;
  const bool panels_full = p.full_panels != 0;

  // LDS destinations of this lane's decoded data
  auto col_slab = [&](int buf, int h) {
    return lds + buf * kBufBytes + ((wave * 2 + h) * kCols) * 16;
  };
  auto row_slab = [&](int buf) {
    return lds + buf * kBufBytes + kColPBytes + ((wave * 2 + half) * kRows) * 16;
  };
  auto row_na = [&](int buf) {
    return lds + buf * kBufBytes + kColPBytes + kRowPBytes + ((wave * 2 + half) * kRows) * 8;
  };

  auto fetch = [&](Raw& raw, int stage) {
    const bool tail = p.t0 + (int64_t)stage * kStage + wave * 16 + 16 > p.t_end;
    if (panels_full && !tail)
      load_stage<false>(raw, chan, n, p.t0, p.t_end, stage, wave, voff_col, voff_row, col_ok,
                        row_ok, half);
    else
      load_stage<true>(raw, chan, n, p.t0, p.t_end, stage, wave, voff_col, voff_row, col_ok,
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
  int a_off[2], b_off[4];   // byte offsets of this lane's operand slots in a stage buffer
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
    a_off[rb] = (half * kRows + slot_swizzle(wr * 64 + rb * 32 + l32));
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
    b_off[cb] = (half * kCols + slot_swizzle(wc * 128 + cb * 32 + l32));

  v16i acc_re[2][4], acc_im[2][4];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      acc_re[rb][cb] = v16i{};
      acc_im[rb][cb] = v16i{};
    }

  // Operand fragments of one 16-sample MFMA step.
  struct Frags {
    v4i pa[2];
    v2i na[2];
    v4i pb[4];
  };
  auto load_frags = [&](Frags& fr, const uint8_t* base, int kk) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      fr.pa[rb] = *reinterpret_cast<const v4i*>(base + kColPBytes + (kk * 2 * kRows + a_off[rb]) * 16);
      fr.na[rb] = *reinterpret_cast<const v2i*>(base + kColPBytes + kRowPBytes +
                                                (kk * 2 * kRows + a_off[rb]) * 8);
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
      fr.pb[cb] = *reinterpret_cast<const v4i*>(base + (kk * 2 * kCols + b_off[cb]) * 16);
  };
  // All 8 blocks of the wave. Blocks lying below the diagonal are computed and
  // never stored: the busiest wave of the tile sets the stage time anyway.
  auto mfma_step = [&](const Frags& fr) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const v4i qa = {fr.pa[rb].z, fr.pa[rb].w, fr.na[rb].x, fr.na[rb].y};
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        acc_re[rb][cb] =
            __builtin_amdgcn_mfma_i32_32x32x32_i8(fr.pa[rb], fr.pb[cb], acc_re[rb][cb], 0, 0, 0);
        acc_im[rb][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(qa, fr.pb[cb], acc_im[rb][cb], 0, 0, 0);
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
    __builtin_amdgcn_sched_barrier(0);
    load_frags(f0, base, 0);
    if (kFast)
      load_stage<false>(ld, chan, n, p.t0, p.t_end, ld_stage, wave, voff_col, voff_row, col_ok,
                        row_ok, half);
    else if (do_ld)
      load_stage<true>(ld, chan, n, p.t0, p.t_end, ld_stage, wave, voff_col, voff_row, col_ok,
                       row_ok, half);
    __builtin_amdgcn_sched_barrier(0);
    load_frags(f1, base, 1);
    if (kFast || do_dec) decode_cols(dec.col, col_slab(cur ^ 1, 0), 4 * lane);
    mfma_step(f0);
    __builtin_amdgcn_sched_barrier(0);
    load_frags(f0, base, 2);
    if (kFast || do_dec) decode_cols(dec.col + 8, col_slab(cur ^ 1, 1), 4 * lane);
    mfma_step(f1);
    __builtin_amdgcn_sched_barrier(0);
    load_frags(f1, base, 3);
    if (kFast || do_dec) {
      transpose_rows(dec.row, tx0, tx1);
      decode_rows_half(tx0, tx1, 0, row_slab(cur ^ 1), row_na(cur ^ 1), 4 * l32);
    }
    mfma_step(f0);
    __builtin_amdgcn_sched_barrier(0);
    if (kFast || do_dec) decode_rows_half(tx0, tx1, 1, row_slab(cur ^ 1), row_na(cur ^ 1), 4 * l32);
    mfma_step(f1);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
  };

  Raw ra, rb_;
  fetch(ra, stage_begin);
  if (stage_begin + 1 < stage_end) fetch(rb_, stage_begin + 1);
  {
    uint32_t tx0[4], tx1[4];
    decode_cols(ra.col, col_slab(0, 0), 4 * lane);
    decode_cols(ra.col + 8, col_slab(0, 1), 4 * lane);
    transpose_rows(ra.row, tx0, tx1);
    decode_rows_half(tx0, tx1, 0, row_slab(0), row_na(0), 4 * l32);
    decode_rows_half(tx0, tx1, 1, row_slab(0), row_na(0), 4 * l32);
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

}  // namespace

int64_t wide_tiles_per_channel(int n) {
  const int nbr = (n + kRows - 1) / kRows, nbc = (n + kCols - 1) / kCols;
  int64_t cnt = 0;
  for (int j = 0; j < nbc; ++j) cnt += (2 * j + 2 < nbr) ? 2 * j + 2 : nbr;
  return cnt;
}

int64_t wide_max_samples_per_launch() { return kMaxSamplesPerLaunch; }

hipError_t launch_wide(const uint8_t* in, int32_t* vis, int n, int f, int t, int t0, int t_count,
                       int accumulate, int split, hipStream_t stream) {
  if (t_count <= 0 || t_count > kMaxSamplesPerLaunch || t0 < 0 || t0 + t_count > t)
    return hipErrorInvalidValue;
  WideParams p;
  p.in = in;
  p.vis = vis;
  p.n = n;
  p.f = f;
  p.t = t;
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
  xcorr_wide_kernel<<<dim3((unsigned)grid), dim3(kThreads), 0, stream>>>(p);
  return hipGetLastError();
}

}  // namespace xeng
