// xcorr_device.h -- device-side building blocks of the gfx950 correlator:
// Excess-8 nibble decode, 4x4 byte transposes, LDS slot swizzle and the
// upper-triangle index.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xeng {

typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// A raw word whose four bytes all decode to 0 + 0i: both fields hold 8.
constexpr uint32_t kZeroSamples = 0x88888888u;

// ---- Excess-8 decode, four fields (one per byte) at a time -----------------
// Paper Sec. III: a 4-bit field holds value + 8, value in [-8, 7]; the real
// part is the high nibble of the sample byte.
__host__ __device__ inline uint32_t fields_hi(uint32_t w) { return (w >> 4) & 0x0F0F0F0Fu; }
__host__ __device__ inline uint32_t fields_lo(uint32_t w) { return w & 0x0F0F0F0Fu; }

// u in [0,15] per byte -> signed byte u - 8. u + 0x78 lies in [0x78, 0x87], so
// no carry leaves a byte; flipping bit 7 then gives the two's complement value.
__host__ __device__ inline uint32_t fields_to_s8(uint32_t u) {
  return (u + 0x78787878u) ^ 0x80808080u;
}
// u in [0,15] per byte -> signed byte 8 - u, the negated value (in [-7, 8]).
// 0x88 - u lies in [0x79, 0x88], again without borrows between bytes.
__host__ __device__ inline uint32_t fields_to_neg_s8(uint32_t u) {
  return (0x88888888u - u) ^ 0x80808080u;
}

// ---- 4x4 byte transpose ------------------------------------------------------
// w[r] holds four consecutive elements at sample r (byte k = element k);
// x[k] receives element k at samples 0..3 (byte r = sample r).
__device__ inline void transpose_4x4(const uint32_t w[4], uint32_t x[4]) {
  // v_perm_b32 picks bytes of {hi:lo} = {src0:src1}; selector byte s picks
  // byte s of that 8-byte pair.
  const uint32_t lo01 = __builtin_amdgcn_perm(w[1], w[0], 0x05010400u);  // w0.0 w1.0 w0.1 w1.1
  const uint32_t hi01 = __builtin_amdgcn_perm(w[1], w[0], 0x07030602u);  // w0.2 w1.2 w0.3 w1.3
  const uint32_t lo23 = __builtin_amdgcn_perm(w[3], w[2], 0x05010400u);
  const uint32_t hi23 = __builtin_amdgcn_perm(w[3], w[2], 0x07030602u);
  x[0] = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
  x[1] = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
  x[2] = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
  x[3] = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
}

// ---- LDS slot swizzle ----------------------------------------------------------
// Operand slabs are 16-byte slots indexed by element. Writers touch elements
// 4 apart per lane, readers consecutive elements; XOR-ing bits 4..5 of the
// element into bits 0..1 keeps both patterns free of bank conflicts.
__host__ __device__ inline int slot_swizzle(int e) { return e ^ ((e >> 4) & 3); }

// ---- packed upper-triangle index ----------------------------------------------
// Row-major packing: row i holds j = i..n-1, so k(i,j) = i*(2n-i+1)/2 + (j-i).
__host__ __device__ inline int64_t tri_index(int64_t n, int64_t i, int64_t j) {
  return i * (2 * n - i + 1) / 2 + (j - i);
}

// ---- workgroup -> XCD-local logical id ----------------------------------------
// The dispatcher hands consecutive workgroup ids to the 8 XCDs in turn. Remap
// so that each XCD receives one contiguous range of logical ids: neighbouring
// tiles (which share input panels) then share that XCD's L2.
__device__ inline int xcd_logical_id(int wg, int grid) {
  constexpr int kXcds = 8;
  const int xcd = wg % kXcds, slot = wg / kXcds;
  const int per = grid / kXcds, extra = grid % kXcds;
  return xcd * per + (xcd < extra ? xcd : extra) + slot;
}

}  // namespace xeng
