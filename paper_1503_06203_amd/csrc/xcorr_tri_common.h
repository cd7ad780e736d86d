// xcorr_tri_common.h -- pieces shared by the triangle kernels (N <= 256, one
// workgroup per channel): launch shape, stage geometry, parameters, the block
// programs that split the 8x8 block triangle of Sec. II-C over the waves, and
// the LDS and vector-memory waits of the staging pipeline.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xcorr_device.h"

namespace xeng {
namespace tri {

constexpr int kThreads = 512;                   // 8 waves, two per SIMD
constexpr int kElems = 256;                     // elements one workgroup covers
constexpr int kStage = 64;                      // samples per stage
constexpr int kRawStride = kElems + 32;         // LDS bytes per raw sample row (bank spread)
constexpr int kRawBytes = kStage * kRawStride;  // 18 KiB per raw buffer
constexpr uint32_t kOob = 0x80000000u;          // buffer offset past every record: load returns 0

struct TriParams {
  const uint8_t* in;
  int32_t* vis;
  int n, f;              // elements of this triangle, channels
  int e0;                // first element of the triangle (a multiple of 4)
  int n_total;           // elements of the whole array (output indexing)
  int t;                 // samples per channel
  int64_t ss, cs;        // bytes from one sample to the next, and from one channel to the next
  int t0, t_end;         // this launch sums samples [t0, t_end)
  int split;             // workgroups along time per channel
  int stages_per_split;
  int total_stages;
  int accumulate;
  int atomic_out;
};

// ---- block programs ---------------------------------------------------------------
// A wave's share of the 8x8 block triangle, relative to its base block (the
// SIMD index for the first wave of a SIMD, 0 for the second):
//   p[]  blocks whose P slabs the wave reads each MFMA step (A and B sides)
//   slot k computes block (p[sa[k]], p[sb[k]]).
struct ProgA {  // row s, columns s..s+4
  static constexpr int kNP = 5, kNS = 5;
  static constexpr int p[kNP] = {0, 1, 2, 3, 4};
  static constexpr int sa[kNS] = {0, 0, 0, 0, 0};
  static constexpr int sb[kNS] = {0, 1, 2, 3, 4};
};
template <int S>
struct ProgB;
template <>
struct ProgB<0> {  // (0,5) (0,6) (0,7) (7,7)
  static constexpr int kNP = 4, kNS = 4;
  static constexpr int p[kNP] = {0, 5, 6, 7};
  static constexpr int sa[kNS] = {0, 0, 0, 3};
  static constexpr int sb[kNS] = {1, 2, 3, 3};
};
template <>
struct ProgB<1> {  // (1,6) (1,7) (6,6) (6,7)
  static constexpr int kNP = 3, kNS = 4;
  static constexpr int p[kNP] = {1, 6, 7};
  static constexpr int sa[kNS] = {0, 0, 1, 1};
  static constexpr int sb[kNS] = {1, 2, 1, 2};
};
template <>
struct ProgB<2> {  // (2,7) (5,5) (5,6) (5,7)
  static constexpr int kNP = 4, kNS = 4;
  static constexpr int p[kNP] = {2, 5, 6, 7};
  static constexpr int sa[kNS] = {0, 1, 1, 1};
  static constexpr int sb[kNS] = {3, 1, 2, 3};
};
template <>
struct ProgB<3> {  // (4,4) (4,5) (4,6) (4,7)
  static constexpr int kNP = 4, kNS = 4;
  static constexpr int p[kNP] = {4, 5, 6, 7};
  static constexpr int sa[kNS] = {0, 0, 0, 0};
  static constexpr int sb[kNS] = {0, 1, 2, 3};
};

// The thread index, through an empty asm statement the compiler cannot see
// through or move: values derived from it are then computed where they are
// used. In a persistent kernel, which runs this code once per queue item,
// the compiler would otherwise compute every lane offset of every code path
// once, before the item loop, and hold them all in registers for its whole
// length.
__device__ inline int opaque_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

typedef __attribute__((address_space(3))) void* lds_void_ptr;
typedef __attribute__((address_space(3))) v2i* lds_v2i_ptr;

// Stage barrier for LDS traffic only: this wave's LDS reads and writes are
// complete, then all waves meet. Loads still in flight into the raw buffers
// are not waited for (each wave waits for its own before reading them).
__device__ inline void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt left at their maximum
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Wait until at most kLeft of this wave's vector-memory operations are in
// flight. They retire in issue order, so issuing a stage's 8 loads and then
// waiting for kLeft = 8 means every operation issued before them (the loads of
// the previous stage among them) is complete. The compiler's own tracking of
// loads into LDS is not relied on: it does not carry across loop back-edges.
// The empty asm statements keep memory operations from moving across the wait.
template <int kLeft>
__device__ inline void vm_wait() {
  static_assert(kLeft >= 0 && kLeft < 64, "vmcnt field");
  asm volatile("" ::: "memory");
  // vmcnt(kLeft) (bits 3:0 and 15:14); lgkmcnt and expcnt at their maximum
  __builtin_amdgcn_s_waitcnt(0x0F70 | (kLeft & 15) | ((kLeft >> 4) << 14));
  asm volatile("" ::: "memory");
}

}  // namespace tri
}  // namespace xeng
