// xcorr_small.hip -- gfx950 correlation kernel for arrays of at most 64
// elements, where the input stream, not the matrix cores, sets the pace: one
// byte of input carries 4 (N + 1) effective operations (Sec. II-A, Eq. 2), 260
// at N = 64, under the ~625 op/B ridge of the int8 MFMA peak against 8 TB/s.
//
// Same contraction as the other kernels (Sec. II-A, Eq. 1 and 2) with the
// offset arithmetic of Sec. III-A (Eq. 3): the matrix cores multiply the
// Excess-8 fields u = x + 8, P = [uRe, uIm] on both sides and
// Q = [uIm, 15 - uRe] on the row side, and per-element field sums correct the
// products in the epilogue (see xcorr_tri.hip for the identities). The
// triangle of an array of at most 64 elements is at most the three 32 x 32
// blocks (0,0), (0,1), (1,1) of Sec. II-C's tiling.
//
// Every wave works alone on one channel over one part of its time axis, so the
// stage loop has no barrier:
//   * the wave's sample rows stream from HBM into its own ring of 16 steps of
//     16 samples in LDS (4 dword loads per step straight into LDS, 64 bytes
//     per sample row), 15 steps ahead of use: 120 KiB of loads in flight per
//     compute unit, enough to cover HBM latency at the full stream rate. A
//     step waits for its own loads only (the loads retire in order).
//   * one ds_read_b64_tr_b8 per block and step hands each lane the 8 samples of
//     one element that its MFMA operand needs: lanes 0-31 elements 32b .. 32b+31
//     at samples 0-7 of the step, lanes 32-63 the same elements at samples 8-15.
//     The lane decodes them in registers into the operand itself
//     [uRe g, uRe g+1, uIm g, uIm g+1]; nothing decoded goes back to LDS.
//     These reads are written as inline assembly that waits for its own
//     results: the compiler cannot tell which ring slot an LDS read touches
//     and would otherwise wait for every load in flight before each one.
// A workgroup of 8 waves holds C channels x S parts of the time axis
// (C x S = 8, chosen so the launch fills the compute units). The parts of one
// channel combine in order: part 0 writes (or adds to) the output, then after a
// workgroup barrier the other parts add theirs with int32 atomics, so no zero
// fill is needed.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "xcorr_device.h"
#include "xcorr_launch.h"
#include "xcorr_tri_common.h"

namespace xeng {

namespace {

using tri::lds_v2i_ptr;
using tri::vm_wait;

constexpr int kThreads = 512;                  // 8 waves
constexpr int kWaves = kThreads / 64;
constexpr int kMaxElems = 64;
constexpr int kStep = 16;                      // samples per MFMA step
constexpr int kRow = 64;                       // LDS bytes per staged sample row
constexpr int kStepBytes = kStep * kRow;       // 1 KiB
constexpr int kRing = 16;                      // steps in a wave's LDS ring
constexpr int kLoadsPerStep = kStepBytes / 256;   // one dword per lane fills 256 bytes
constexpr int kWaveBytes = kRing * kStepBytes; // the wave's LDS ring: 16 KiB
constexpr uint32_t kOob = 0x80000000u;         // offset past every record: the load returns 0
static_assert(kLoadsPerStep * (kRing - 1) <= 63, "outstanding loads fit the vmcnt field");
static_assert(kWaves * kWaveBytes <= 160 * 1024, "LDS of one compute unit");

struct SmallParams {
  const uint8_t* in;
  int32_t* vis;
  int n, f;
  int64_t ss, cs;        // bytes from one sample to the next, and from one channel to the next
  int t0, t_end;         // this launch sums samples [t0, t_end)
  int chans;             // channels per workgroup (C); parts per channel S = 8 / C
  int steps_per_part;    // 16-sample steps per part
  int accumulate;
};

// kNB = 32-element blocks per side (1 for n <= 32, else 2).
template <int kNB>
__device__ __forceinline__ void small_run(const SmallParams& p, uint8_t* ring_all) {
  constexpr int kPairs = kNB * (kNB + 1) / 2;   // blocks (0,0) [, (0,1), (1,1)]
  const int tid = (int)threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int half = lane >> 5, l32 = lane & 31;
  const int C = p.chans, S = kWaves / p.chans;
  const int cw = wave % C, part = wave / C;     // channel slot and time part of this wave
  const int ch = blockIdx.x * C + cw;
  const bool live = ch < p.f;
  const int n = p.n;
  const int64_t ss = p.ss;
  const uint8_t* chan = p.in + (int64_t)(live ? ch : 0) * p.cs;
  uint8_t* const ring = ring_all + wave * kWaveBytes;

  // this part's samples [s0, s1) and steps
  const int total = p.t_end - p.t0;
  const int s0 = min(total, part * p.steps_per_part * kStep);
  const int s1 = min(total, s0 + p.steps_per_part * kStep);
  const int nsteps = live ? (s1 - s0 + kStep - 1) / kStep : 0;

  // ---- loads: the k-th step a wave takes is rows [s0 + 16k', s0 + 16k' + 16)
  // of the part, k' = (k + rot) mod nsteps, four instructions of four rows
  // each (lane l: row l / 16, elements 4 (l % 16)), into ring slot k % kRing
  // at 256 bytes per instruction. Rows past s1 lie past the descriptor's
  // record count and elements past n use an offset past every record; both
  // read 0x00, whose fields add nothing. The fetches for k >= nsteps (issued
  // so that every step has the same count of loads after it) have no
  // records and read nothing from memory.
  const uint32_t voff = (4 * (lane & 15) < n) ? (uint32_t)((lane >> 4) * ss + 4 * (lane & 15)) : kOob;
  // Each wave walks its steps from a starting step of its own and wraps
  // around (the sums do not depend on the order). Channels and parts start on
  // large power-of-two strides; walked in lockstep from their first steps,
  // all the streams of the launch would hit the same HBM channels at once.
  const int rot =
      nsteps > 0 ? (int)(((unsigned)(ch * kWaves + part) * 2654435761u >> 8) % (unsigned)nsteps)
                 : 0;
  auto fetch = [&](int k) {
    int kk = k + rot;                             // the step's place in the part
    if (kk >= nsteps) kk -= nsteps;
    const int first = k < nsteps ? p.t0 + s0 + kk * kStep : p.t0 + s1;   // uniform
    const int stop = p.t0 + s1;
    const int64_t bytes = stop > first ? (int64_t)(stop - first - 1) * ss + n : 0;
    const int records = bytes <= 0 ? 0 : (bytes > 0x7fffffff ? 0x7fffffff : (int)bytes);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(chan + (int64_t)(stop > first ? first : 0) * ss), 0, records,
        0x00020000);
    uint8_t* const slot = ring + (k % kRing) * kStepBytes;
#pragma unroll
    for (int q = 0; q < kLoadsPerStep; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (tri::lds_void_ptr)(slot + q * 256), 4,
                                               voff + (uint32_t)(4 * q * ss), 0, 0, 0);
  };

  // ---- operands: lane (l32, half) reads 8 rows (samples 8 half ..) of its
  // element 32 b + l32. In a 16-lane group the even lanes name the rows of the
  // first 8 elements and the odd lanes those of the next 8.
  const int lq = lane & 15, grp = lane >> 4;
  const int tr_off = (8 * (grp >> 1) + (lq >> 1)) * kRow + 16 * (grp & 1) + 8 * (lq & 1);
  // the transposing reads of step k's slot, complete on return
  auto tr_read = [&](int k, v2i* raw) {
    const uint32_t a = (uint32_t)(uintptr_t)(tri::lds_void_ptr)(ring + (k % kRing) * kStepBytes +
                                                                  tr_off);
    if constexpr (kNB == 1) {
      asm volatile("ds_read_b64_tr_b8 %0, %1\n\ts_waitcnt lgkmcnt(0)"
                   : "=&v"(raw[0])
                   : "v"(a)
                   : "memory");
    } else {
      asm volatile(
          "ds_read_b64_tr_b8 %0, %2\n\tds_read_b64_tr_b8 %1, %2 offset:32\n\ts_waitcnt lgkmcnt(0)"
          : "=&v"(raw[0]), "=&v"(raw[kNB - 1])
          : "v"(a)
          : "memory");
    }
  };
  uint32_t sum_re[kNB], sum_im[kNB];
  v16i acc_re[kPairs], acc_im[kPairs];
#pragma unroll
  for (int b = 0; b < kNB; ++b) sum_re[b] = sum_im[b] = 0u;
#pragma unroll
  for (int q = 0; q < kPairs; ++q) {
    acc_re[q] = v16i{};
    acc_im[q] = v16i{};
  }
  auto step = [&](const v2i* raw) {
    v4i pv[kNB], qv[kNB];
#pragma unroll
    for (int b = 0; b < kNB; ++b) {
      const uint32_t ra = fields_hi((uint32_t)raw[b].x), rb = fields_hi((uint32_t)raw[b].y);
      const uint32_t ia = fields_lo((uint32_t)raw[b].x), ib = fields_lo((uint32_t)raw[b].y);
      pv[b] = v4i{(int)ra, (int)rb, (int)ia, (int)ib};
      qv[b] = v4i{(int)ia, (int)ib, (int)(ra ^ 0x0F0F0F0Fu), (int)(rb ^ 0x0F0F0F0Fu)};
      sum_re[b] = __builtin_amdgcn_sad_u8(rb, 0u, __builtin_amdgcn_sad_u8(ra, 0u, sum_re[b]));
      sum_im[b] = __builtin_amdgcn_sad_u8(ib, 0u, __builtin_amdgcn_sad_u8(ia, 0u, sum_im[b]));
    }
    int q = 0;
#pragma unroll
    for (int bi = 0; bi < kNB; ++bi)
#pragma unroll
      for (int bj = bi; bj < kNB; ++bj, ++q) {
        acc_re[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(pv[bi], pv[bj], acc_re[q], 0, 0, 0);
        acc_im[q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(qv[bi], pv[bj], acc_im[q], 0, 0, 0);
      }
  };

  // ---- stream: every step first issues the loads of step k + kRing - 1 into
  // the slot step k - 1 has vacated, then waits until only the loads issued
  // after step k's are in flight, reads its slot and multiplies.
  if (nsteps > 0) {
    for (int k = 0; k < kRing - 1; ++k) fetch(k);
#pragma unroll 1
    for (int k = 0; k < nsteps; ++k) {
      fetch(k + kRing - 1);
      vm_wait<kLoadsPerStep * (kRing - 1)>();
      v2i raw[kNB];
      tr_read(k, raw);
      step(raw);
    }
  }
  // no load into LDS may land after the ring is reused or the workgroup ends
  vm_wait<0>();

  // ---- offset corrections: the two lane halves hold the field sums of the
  // same element over complementary samples
  uint32_t* const cor = reinterpret_cast<uint32_t*>(ring);   // [cr, ci_row, ci_col][64]
#pragma unroll
  for (int b = 0; b < kNB; ++b) {
    const uint32_t sr = sum_re[b] + (uint32_t)__shfl_xor((int)sum_re[b], 32);
    const uint32_t si = sum_im[b] + (uint32_t)__shfl_xor((int)sum_im[b], 32);
    if (half == 0) {
      cor[32 * b + l32] = 8u * (sr + si);
      cor[kMaxElems + 32 * b + l32] = 8u * (sr - si);
      cor[2 * kMaxElems + 32 * b + l32] = 8u * sr + 7u * si;
    }
  }
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_wave_barrier();
  const uint32_t re_const = 128u * (uint32_t)max(0, s1 - s0);

  // ---- epilogue: part 0 of each channel writes (or adds to) the triangle,
  // then, after a barrier, the other parts add theirs atomically
  const int64_t n64 = n;
  const int64_t entries = n64 * (n64 + 1) / 2;
  int32_t* out = p.vis + (int64_t)(live ? ch : 0) * entries * 2;
  auto store_all = [&](auto mode) {
    constexpr int kStore = decltype(mode)::value;   // 0 store, 1 add, 2 atomic add
    int q = 0;
#pragma unroll
    for (int bi = 0; bi < kNB; ++bi)
#pragma unroll
      for (int bj = bi; bj < kNB; ++bj, ++q) {
        const int j = 32 * bj + l32;
        const uint32_t re_j = re_const - cor[j];
        const uint32_t ci_col_j = cor[2 * kMaxElems + j];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = 32 * bi + 8 * (r >> 2) + 4 * half + (r & 3);
          if (i <= j && j < n) {
            int32_t* o = out + 2 * tri_index(n64, i, j);
            // int32 arithmetic modulo 2^32 (unsigned): exact for the result
            const int re = (int)((uint32_t)acc_re[q][r] + re_j - cor[i]);
            const int im = (int)((uint32_t)acc_im[q][r] + cor[kMaxElems + i] - ci_col_j);
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
  if (live && part == 0) {
    if (p.accumulate)
      store_all(std::integral_constant<int, 1>{});
    else
      store_all(std::integral_constant<int, 0>{});
  }
  if (S > 1) {
    __threadfence();
    __syncthreads();
    if (live && part > 0) store_all(std::integral_constant<int, 2>{});
  }
}

__global__ __launch_bounds__(kThreads, 1) void xcorr_small_kernel(SmallParams p) {
  __shared__ __attribute__((aligned(16))) uint8_t ring[kWaves * kWaveBytes];
  if (p.n <= 32)
    small_run<1>(p, ring);
  else
    small_run<2>(p, ring);
}

}  // namespace

int small_max_elements() { return kMaxElems; }

hipError_t launch_small(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                        int64_t cs, int t0, int t_count, int accumulate, int cus,
                        hipStream_t stream) {
  if (n < 1 || n > kMaxElems || n % 4 != 0 || f < 1) return hipErrorInvalidValue;
  if (t_count <= 0 || t0 < 0 || (int64_t)t0 + t_count > t) return hipErrorInvalidValue;
  SmallParams p;
  p.in = in;
  p.vis = vis;
  p.n = n;
  p.f = f;
  p.ss = ss;
  p.cs = cs;
  p.t0 = t0;
  p.t_end = t0 + t_count;
  p.accumulate = accumulate;
  // channels per workgroup: the most that still leaves a workgroup per
  // compute unit (more channels per workgroup = fewer parts per channel)
  int c = kWaves;
  while (c > 1 && ((int64_t)f + c - 1) / c < cus) c /= 2;
  p.chans = c;
  const int parts = kWaves / c;
  const int64_t steps = ((int64_t)t_count + kStep - 1) / kStep;
  p.steps_per_part = (int)((steps + parts - 1) / parts);
  const int64_t grid = ((int64_t)f + c - 1) / c;
  if (grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  xcorr_small_kernel<<<dim3((unsigned)grid), dim3(kThreads), 0, stream>>>(p);
  return hipGetLastError();
}

}  // namespace xeng
