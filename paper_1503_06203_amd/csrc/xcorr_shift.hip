// xcorr_shift.hip -- delay compensation ahead of correlation for arrays of any
// size (Sec. IV: a kernel that moves single elements by whole time steps
// before they are correlated, to create or remove lags such as those of
// unequal cable lengths).
//
// The kernel writes the delay-aligned samples of a window of frame samples
// into a dense buffer that the correlation kernels then read like any frame:
//   out[c][s][e] = in[c][max_delay + t0 + s - delay[e]][e],   0 <= s < tc,
// where the input holds max_delay halo samples before the frame's t. It is
// bound by HBM (one byte read and one written per sample and element, plus the
// rows its window re-reads), which at large N is small next to the
// correlation's matrix-core time.
//
// One workgroup covers 256 elements of one channel over a strip of 2048
// output rows. When the delays of its elements differ by at most kMaxSpread,
// it slides down the strip through a ring of input rows in LDS: each input
// row its output needs is loaded once, whole and coalesced (LDS-DMA, one
// dword of 4 elements per lane, no registers), one chunk of 128 rows ahead of
// use (by four loader waves), and each lane of the four gather waves collects
// its 4 elements' bytes of a chunk from the rows their delays name and writes
// them as one dword. Otherwise (a wider spread,
// or an input that dword loads cannot read) every byte is read from HBM.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xcorr_launch.h"

namespace xeng {

namespace {

constexpr int kThreads = 512;                   // 8 waves
constexpr int kWaves = kThreads / 64;
constexpr int kBlockElems = 256;                // elements per workgroup, 4 per lane
constexpr int kStripRows = 2048;                // output rows per workgroup
constexpr int kChunk = 128;                     // output rows gathered per ring step
constexpr int kMaxSpread = 128;                 // ring form: largest delay spread
// The ring: three arrays of kChunk input rows. A chunk of output rows reads
// two of them (its rows and up to kMaxSpread more), the third is loaded
// meanwhile.
constexpr int kRowStride = kBlockElems + 4;     // 65 dwords: rows start on different banks
constexpr uint32_t kOob = 0x80000000u;          // buffer offset past every record: reads 0
static_assert(kMaxSpread <= kChunk && (kChunk & (kChunk - 1)) == 0, "ring geometry");
static_assert(3 * kChunk * kRowStride <= 160 * 1024, "LDS of one compute unit");

typedef __attribute__((address_space(3))) void* lds_void_ptr;

struct ShiftParams {
  const uint8_t* in;
  uint8_t* out;
  int n;
  int t_in;               // samples per input channel (halo included)
  int64_t in_cs;          // bytes per input channel: t_in * n
  int64_t out_cs;         // bytes per output channel: tc * n
  int max_delay, t0, tc;
  int e_begin, e_count;   // the elements whose delays this launch carries
  int strips;             // row strips per channel
  int blocks;             // 256-element blocks of this launch
  int aligned;            // n % 4 == 0 and 4-byte aligned in and out: dword access
  uint16_t delay[kShiftGroupElems];
};

// This wave's LDS reads and writes are complete, then all waves meet.
__device__ inline void ring_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// All of this wave's vector-memory operations (ring loads and output stores)
// are complete.
__device__ inline void vm_wait_all() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0); lgkmcnt and expcnt at their maximum
  asm volatile("" ::: "memory");
}

__global__ __launch_bounds__(kThreads) void xcorr_shift_kernel(ShiftParams p) {
  __shared__ __attribute__((aligned(16))) uint8_t ring0[kChunk * kRowStride];
  __shared__ __attribute__((aligned(16))) uint8_t ring1[kChunk * kRowStride];
  __shared__ __attribute__((aligned(16))) uint8_t ring2[kChunk * kRowStride];
  __shared__ int bounds[2];
  const int tid = (int)threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int b = (int)(blockIdx.x % (unsigned)p.blocks);
  const int rest = (int)(blockIdx.x / (unsigned)p.blocks);
  const int strip = rest % p.strips, c = rest / p.strips;
  const int eb = b * kBlockElems;                      // first element, within the launch
  const int ne = min(kBlockElems, p.e_count - eb);     // elements of this block
  const int s0 = strip * kStripRows, ns = min(kStripRows, p.tc - s0);
  const uint8_t* src = p.in + (int64_t)c * p.in_cs;
  uint8_t* dst = p.out + (int64_t)c * p.out_cs;
  const int64_t n = p.n;
  const int first_row = p.max_delay + p.t0 + s0;       // input row of output row s0, delay 0

  // spread of this block's delays
  if (tid == 0) {
    bounds[0] = 0x7fffffff;
    bounds[1] = -1;
  }
  __syncthreads();
  if (tid < ne) {
    atomicMin(&bounds[0], (int)p.delay[eb + tid]);
    atomicMax(&bounds[1], (int)p.delay[eb + tid]);
  }
  __syncthreads();
  const int dmin = bounds[0], dmax = bounds[1];
  const int spread = dmax - dmin;
  const int e4 = eb + 4 * lane;                        // this lane's first element (launch-relative)
  const bool quad = 4 * lane < ne;                     // the lane has elements in this block
  int back[4];                                         // input row of output row s: s + back[k]
#pragma unroll
  for (int k = 0; k < 4; ++k) back[k] = (4 * lane + k < ne) ? dmax - (int)p.delay[e4 + k] : 0;

  if (p.aligned && spread <= kMaxSpread) {
    // relative input row r is input row base_row + r of the channel, for
    // r in [0, ns + spread); segment r / kChunk of the strip lives in ring
    // array (r / kChunk) % 3
    const int base_row = first_row - dmax;
    const int rows = ns + spread;
    const int64_t col0 = p.e_begin + eb;               // absolute element of the block
    const int64_t bytes = (int64_t)(p.t_in - base_row) * n - col0;   // to the channel's end
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(src + (int64_t)base_row * n + col0), 0,
        bytes > 0x7fffffff ? 0x7fffffff : (int)bytes, 0x00020000);
    const uint32_t voff = quad ? (uint32_t)(4 * lane) : kOob;
    // Waves 0-3 load the ring, waves 4-7 gather from it and store. Loads and
    // stores share one counter of outstanding vector-memory operations, so a
    // wave that did both would wait for its stores whenever it waits for its
    // loads; split this way the loaders wait for loads only and the
    // gatherers never wait on memory.
    const bool loader = wave < kWaves / 2;
    const int rw = loader ? wave : wave - kWaves / 2;   // index within the role
    constexpr int kRole = kWaves / 2;
    // segment k's rows [k * kChunk, (k + 1) * kChunk) that the strip uses;
    // loader wave rw loads rows rw, rw + 4, ... of it
    auto load_seg = [&](uint8_t* seg, int k) {
      const int lo = k * kChunk, hi = min(lo + kChunk, rows);
      for (int r = lo + rw; r < hi; r += kRole)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_ptr)(seg + (r - lo) * kRowStride),
                                                 4, voff + (uint32_t)r * (uint32_t)n, 0, 0, 0);
    };
    uint32_t* out = reinterpret_cast<uint32_t*>(dst + (int64_t)s0 * n + p.e_begin + e4);
    // output rows of chunk k read input rows [k * kChunk, (k + 1) * kChunk +
    // spread): segments k (cur) and k + 1 (nxt)
    // Element q's byte of output row s sits in input row rr = s - k * kChunk +
    // back[q] of the two segments, in [0, 2 * kChunk). Both arrays are read at
    // the same offset and the value is selected afterwards: a read through a
    // pointer chosen at run time carries no alias scope, and the compiler
    // would then wait for the loads into the third array before it. The empty
    // asm statements keep the compiler from folding the two reads back into
    // one; they cover four rows at a time, so 32 reads are in flight before
    // the wave waits for them.
    constexpr int kRows = 4;
    auto gather = [&](const uint8_t* cur, const uint8_t* nxt, int k) {
      if (!quad) return;
      const int end = min(ns, (k + 1) * kChunk);
      for (int s = k * kChunk + rw; s < end; s += kRows * kRole) {
        uint32_t a[kRows][4], b[kRows][4];
#pragma unroll
        for (int j = 0; j < kRows; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int rr = s + j * kRole - k * kChunk + back[q];
            const int at = (rr & (kChunk - 1)) * kRowStride + 4 * lane + q;
            a[j][q] = cur[at];
            b[j][q] = nxt[at];
          }
        asm volatile("" : "+v"(a[0][0]), "+v"(a[0][1]), "+v"(a[0][2]), "+v"(a[0][3]),
                     "+v"(a[1][0]), "+v"(a[1][1]), "+v"(a[1][2]), "+v"(a[1][3]),
                     "+v"(a[2][0]), "+v"(a[2][1]), "+v"(a[2][2]), "+v"(a[2][3]),
                     "+v"(a[3][0]), "+v"(a[3][1]), "+v"(a[3][2]), "+v"(a[3][3]));
        asm volatile("" : "+v"(b[0][0]), "+v"(b[0][1]), "+v"(b[0][2]), "+v"(b[0][3]),
                     "+v"(b[1][0]), "+v"(b[1][1]), "+v"(b[1][2]), "+v"(b[1][3]),
                     "+v"(b[2][0]), "+v"(b[2][1]), "+v"(b[2][2]), "+v"(b[2][3]),
                     "+v"(b[3][0]), "+v"(b[3][1]), "+v"(b[3][2]), "+v"(b[3][3]));
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
          const int sj = s + j * kRole;
          if (sj >= end) break;
          uint32_t w = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            w |= (sj - k * kChunk + back[q] < kChunk ? a[j][q] : b[j][q]) << (8 * q);
          *reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(out) + (int64_t)sj * n) = w;
        }
      }
    };
    // Step k: the loaders' rows so far (segments up to k + 1) are in, then
    // at the barrier everyone's are and chunk k - 1 is read; the loaders load
    // segment k + 2 into the array chunk k - 1 read while the gatherers
    // gather chunk k. Each array is its own variable and every step names its
    // arrays statically, so the compiler sees that the gather's reads cannot
    // touch the array being loaded and does not wait for those loads.
    auto step = [&](const uint8_t* cur, const uint8_t* nxt, uint8_t* ld, int k) {
      if (loader) vm_wait_all();
      ring_barrier();
      if (loader)
        load_seg(ld, k + 2);
      else
        gather(cur, nxt, k);
    };
    if (loader) {
      load_seg(ring0, 0);
      load_seg(ring1, 1);
    }
    const int nchunks = (ns + kChunk - 1) / kChunk;
    for (int k = 0; k < nchunks; k += 3) {
      step(ring0, ring1, ring2, k);
      if (k + 1 < nchunks) step(ring1, ring2, ring0, k + 1);
      if (k + 2 < nchunks) step(ring2, ring0, ring1, k + 2);
    }
    // no load into LDS may land after the workgroup ends
    if (loader) vm_wait_all();
    return;
  }
  // direct form: every byte from HBM
  if (!quad) return;
  for (int s = wave; s < ns; s += kWaves) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = e4 + k;
      if (e >= eb + ne) break;
      const int64_t col = p.e_begin + e;
      dst[(int64_t)(s0 + s) * n + col] = src[(int64_t)(first_row + s - p.delay[e]) * n + col];
    }
  }
}

}  // namespace

int shift_tile_rows() { return kChunk; }

hipError_t launch_shift(const uint8_t* in, uint8_t* out, int n, int f, int t_in, int max_delay,
                        int t0, int tc, int e_begin, int e_count, const int32_t* delays,
                        hipStream_t stream) {
  if (n < 1 || f < 1 || tc < 1 || t0 < 0 || max_delay < 0) return hipErrorInvalidValue;
  if ((int64_t)max_delay + t0 + tc > t_in) return hipErrorInvalidValue;
  if (e_begin < 0 || e_count < 1 || e_count > kShiftGroupElems || e_begin + e_count > n)
    return hipErrorInvalidValue;
  ShiftParams p;
  p.in = in;
  p.out = out;
  p.n = n;
  p.t_in = t_in;
  p.in_cs = (int64_t)t_in * n;
  p.out_cs = (int64_t)tc * n;
  p.max_delay = max_delay;
  p.t0 = t0;
  p.tc = tc;
  p.e_begin = e_begin;
  p.e_count = e_count;
  p.strips = (tc + kStripRows - 1) / kStripRows;
  p.blocks = (e_count + kBlockElems - 1) / kBlockElems;
  // the ring form addresses a strip's rows with 32-bit offsets
  p.aligned = n % 4 == 0 && reinterpret_cast<uintptr_t>(in) % 4 == 0 &&
              reinterpret_cast<uintptr_t>(out) % 4 == 0 &&
              (int64_t)(kStripRows + kMaxSpread + kChunk) * n < ((int64_t)1 << 31);
  for (int k = 0; k < kShiftGroupElems; ++k) {
    const int d = k < e_count ? delays[e_begin + k] : 0;
    if (d < 0 || d > max_delay) return hipErrorInvalidValue;
    p.delay[k] = (uint16_t)d;
  }
  const int64_t grid = (int64_t)f * p.strips * p.blocks;
  if (grid <= 0 || grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  xcorr_shift_kernel<<<dim3((unsigned)grid), dim3(kThreads), 0, stream>>>(p);
  return hipGetLastError();
}

}  // namespace xeng
