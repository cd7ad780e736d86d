// xcorr_tile.hip -- the gfx950 correlation kernel.
//
// Computes, per channel, the upper triangle of V = sum_t x(t) x(t)^H for 4-bit
// Excess-8 complex samples (paper Sec. II-A, Eq. 1 and Eq. 2; Sec. III). The
// correlation is the dense contraction it is: with, for each element e, the
// int8 vectors over K = 2T
//     P_e = [Re e(t), Im e(t)]_t   and   Q_e = [Im e(t), -Re e(t)]_t
// one has Re V_ij = P_i . P_j and Im V_ij = Q_i . P_j, two real GEMMs over the
// time axis. They run on v_mfma_i32_32x32x32_i8 with int32 accumulation.
//
// One workgroup owns one 128x128 tile of the upper triangle of one channel
// (paper Sec. II-C, Fig. 1: tiles that are computed independently, only the
// diagonal tiles hold redundant products). It walks the time axis in stages of
// KC samples:
//   stage : coalesced dword loads of the packed bytes of both element panels,
//           a 4x4 byte transpose (time-major -> element-major), nibble decode
//           to signed int8 and a write of the MFMA operand slabs to LDS (double
//           buffered; the next stage's global loads are in flight while the
//           current stage is multiplied);
//   MFMA  : 4 waves in a 2x2 grid, each 64x64 = 2x2 blocks of 32x32, Re and Im.
//           32x32 blocks lying wholly below the diagonal are skipped.
//   store : masked i <= j writes into the packed triangle, optionally adding to
//           the previous sums, or int32 atomic adds when the time axis is split
//           among several workgroups (exact: integer addition is associative).
//
// K layout of one 16-sample MFMA step for element e: lane half h (0/1) holds
// the 16-byte slab [Re g, Im g, Re g+1, Im g+1] for the 4-sample groups
// g = 2h, 2h+1 (each dword = 4 samples of one component). The Q operand is
// then [Im g, -Re g, Im g+1, -Re g+1]: it reuses the slab's Im dwords plus a
// separate plane of negated real parts. A and B operands use the same K
// layout, so the product sums exactly the intended sample pairs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xcorr_device.h"
#include "xcorr_launch.h"

namespace xeng {

namespace {

constexpr int kTile = 128;          // tile edge in elements
constexpr int kThreads = 256;       // 4 waves
constexpr int kStepSamples = 16;    // samples per MFMA K step (32 int8 of K)

struct TileParams {
  const uint8_t* in;
  int32_t* vis;
  int n, f, t;
  int nb;                 // tile rows = ceil(n / kTile)
  int ntiles;             // nb (nb + 1) / 2
  int split;              // workgroups along time per tile
  int stages_per_split;
  int total_stages;
  int accumulate;         // add to previous sums (plain stores)
  int atomic_out;         // int32 atomic adds (time split)
};

template <int KC, bool kAligned>
__global__ __launch_bounds__(kThreads, 2) void xcorr_tile128_kernel(TileParams p) {
  constexpr int kSteps = KC / kStepSamples;
  constexpr int kPBytes = kSteps * 2 * kTile * 16;   // one panel's P slabs
  constexpr int kNaBytes = kSteps * 2 * kTile * 8;   // row panel's -Re plane
  constexpr int kBufBytes = 2 * kPBytes + kNaBytes;
  __shared__ __attribute__((aligned(16))) uint8_t lds[2 * kBufBytes];

  // ---- which tile, channel and time range ------------------------------------
  const int logical = xcd_logical_id(blockIdx.x, gridDim.x);
  const int tile = logical % p.ntiles;
  const int rest = logical / p.ntiles;
  const int split_idx = rest % p.split;
  const int ch = rest / p.split;
  int bi = 0, rem = tile;
  while (rem >= p.nb - bi) {
    rem -= p.nb - bi;
    ++bi;
  }
  const int bj = bi + rem;
  const bool diag = (bi == bj);
  const int row0 = bi * kTile, col0 = bj * kTile;
  const int stage_begin = split_idx * p.stages_per_split;
  const int stage_end = min(stage_begin + p.stages_per_split, p.total_stages);

  // ---- staging roles: threads 0..127 the row panel, 128..255 the column panel.
  // Each unit loads 4 elements x 16 samples (one MFMA K step).
  const int tid = threadIdx.x;
  const bool is_row = tid < 128;
  const bool stager = is_row || !diag;   // a diagonal tile stages one panel
  const int unit = tid & 127;
  const int eg = unit & 31;               // element quad within the panel
  const int kstep = unit >> 5;            // K step within the stage (KC = 64)
  const int e_local = 4 * eg;
  const int e_glob = (is_row ? row0 : col0) + e_local;
  const int64_t n64 = p.n;
  const uint8_t* chan = p.in + (int64_t)ch * p.t * n64;
  static_assert(KC == 4 * kStepSamples, "staging map assumes 4 K steps per stage");

  uint32_t raw[16];
  auto load_stage = [&](int stage) {
    const int t0 = stage * KC + kstep * kStepSamples;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int t = t0 + r;
      if (kAligned) {
        raw[r] = (t < p.t && e_glob < p.n)
                     ? *reinterpret_cast<const uint32_t*>(chan + (int64_t)t * n64 + e_glob)
                     : kZeroSamples;
      } else {
        uint32_t w = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint32_t byte = (t < p.t && e_glob + b < p.n)
                                    ? (uint32_t)chan[(int64_t)t * n64 + e_glob + b]
                                    : 0x88u;
          w |= byte << (8 * b);
        }
        raw[r] = w;
      }
    }
  };

  auto store_stage = [&](int buf) {
    uint8_t* base = lds + buf * kBufBytes;
    uint8_t* pslab = base + (is_row ? 0 : kPBytes);
    uint8_t* naslab = base + 2 * kPBytes;
    uint32_t x[4][4];
#pragma unroll
    for (int g = 0; g < 4; ++g) transpose_4x4(&raw[4 * g], x[g]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int slot = slot_swizzle(e_local + k);
      uint32_t re[4], im[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        re[g] = fields_to_s8(fields_hi(x[g][k]));
        im[g] = fields_to_s8(fields_lo(x[g][k]));
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        v4i s = {(int)re[2 * h], (int)im[2 * h], (int)re[2 * h + 1], (int)im[2 * h + 1]};
        *reinterpret_cast<v4i*>(pslab + ((kstep * 2 + h) * kTile + slot) * 16) = s;
      }
      if (is_row) {
        uint32_t nre[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) nre[g] = fields_to_neg_s8(fields_hi(x[g][k]));
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          v2i s = {(int)nre[2 * h], (int)nre[2 * h + 1]};
          *reinterpret_cast<v2i*>(naslab + ((kstep * 2 + h) * kTile + slot) * 8) = s;
        }
      }
    }
  };

  // ---- MFMA roles ---------------------------------------------------------------
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int half = lane >> 5, l32 = lane & 31;
  bool active[2][2];
  bool wave_active = false;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      active[rb][cb] = !diag || (wr * 2 + rb <= wc * 2 + cb);
      wave_active |= active[rb][cb];
    }

  v16i acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      acc_re[rb][cb] = v16i{};
      acc_im[rb][cb] = v16i{};
    }

  if (stage_begin < stage_end) {
    if (stager) {
      load_stage(stage_begin);
      store_stage(0);
    }
    __syncthreads();
    for (int st = stage_begin; st < stage_end; ++st) {
      const int buf = (st - stage_begin) & 1;
      const bool more = st + 1 < stage_end;
      if (more && stager) load_stage(st + 1);
      if (wave_active) {
        const uint8_t* base = lds + buf * kBufBytes;
        const uint8_t* prow = base;
        const uint8_t* pcol = diag ? base : base + kPBytes;
        const uint8_t* narow = base + 2 * kPBytes;
#pragma unroll
        for (int kk = 0; kk < kSteps; ++kk) {
          v4i pr[2], qr[2], pc[2];
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) {
            const int slot = slot_swizzle(wr * 64 + rb * 32 + l32);
            pr[rb] = *reinterpret_cast<const v4i*>(prow + ((kk * 2 + half) * kTile + slot) * 16);
            const v2i na =
                *reinterpret_cast<const v2i*>(narow + ((kk * 2 + half) * kTile + slot) * 8);
            qr[rb] = v4i{pr[rb].y, na.x, pr[rb].w, na.y};
          }
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) {
            const int slot = slot_swizzle(wc * 64 + cb * 32 + l32);
            pc[cb] = *reinterpret_cast<const v4i*>(pcol + ((kk * 2 + half) * kTile + slot) * 16);
          }
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
              if (active[rb][cb]) {
                acc_re[rb][cb] =
                    __builtin_amdgcn_mfma_i32_32x32x32_i8(pr[rb], pc[cb], acc_re[rb][cb], 0, 0, 0);
                acc_im[rb][cb] =
                    __builtin_amdgcn_mfma_i32_32x32x32_i8(qr[rb], pc[cb], acc_im[rb][cb], 0, 0, 0);
              }
            }
        }
      }
      if (more && stager) store_stage(buf ^ 1);
      __syncthreads();
    }
  }

  // ---- epilogue: masked writes of i <= j into the packed triangle -------------
  // 32x32 MFMA result layout: lane l, register r holds row
  // 8*(r/4) + 4*(l/32) + r%4 and column l%32 of the block.
  if (!wave_active || stage_begin >= stage_end) return;
  const int64_t entries = n64 * (n64 + 1) / 2;
  int32_t* out = p.vis + (int64_t)ch * entries * 2;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      if (!active[rb][cb]) continue;
      const int j = col0 + wc * 64 + cb * 32 + l32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = row0 + wr * 64 + rb * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        if (i <= j && j < p.n) {
          int32_t* o = out + 2 * tri_index(n64, i, j);
          const int re = acc_re[rb][cb][r], im = acc_im[rb][cb][r];
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

__global__ void fill_zero_kernel(v2i* out, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride)
    out[k] = v2i{0, 0};
}

}  // namespace

hipError_t launch_fill_zero(int32_t* vis, int64_t pairs, hipStream_t stream) {
  if (pairs <= 0) return hipSuccess;
  int64_t blocks = (pairs + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  fill_zero_kernel<<<dim3((unsigned)blocks), dim3(256), 0, stream>>>(
      reinterpret_cast<v2i*>(vis), pairs);
  return hipGetLastError();
}

int tile128_stage_samples() { return 64; }

hipError_t launch_tile128(const uint8_t* in, int32_t* vis, int n, int f, int t, int accumulate,
                          int split, bool aligned, hipStream_t stream) {
  constexpr int KC = 64;
  TileParams p;
  p.in = in;
  p.vis = vis;
  p.n = n;
  p.f = f;
  p.t = t;
  p.nb = (n + kTile - 1) / kTile;
  p.ntiles = p.nb * (p.nb + 1) / 2;
  p.total_stages = (t + KC - 1) / KC;
  if (split < 1) split = 1;
  if (split > p.total_stages) split = p.total_stages > 0 ? p.total_stages : 1;
  p.split = split;
  p.stages_per_split = (p.total_stages + split - 1) / split;
  p.accumulate = accumulate;
  p.atomic_out = split > 1;
  const int64_t grid = (int64_t)p.ntiles * f * split;
  if (grid <= 0 || grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  if (aligned)
    xcorr_tile128_kernel<KC, true><<<dim3((unsigned)grid), dim3(kThreads), 0, stream>>>(p);
  else
    xcorr_tile128_kernel<KC, false><<<dim3((unsigned)grid), dim3(kThreads), 0, stream>>>(p);
  return hipGetLastError();
}

}  // namespace xeng
