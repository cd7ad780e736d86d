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
// output rows. When the delays of its elements differ by at most kMaxSpread
// (and every row of the block starts on a 16-byte boundary), it slides down
// the strip through a ring of five LDS arrays of 128 input rows: each input
// row its output needs is loaded once, whole and coalesced (16-byte LDS-DMA,
// four rows per instruction), three chunks ahead of use by four loader
// waves; each lane of the four gather waves collects its 4 elements' bytes of
// a chunk from the rows their delays name and writes them as one dword.
// Otherwise (a wider spread, or rows that such loads cannot read) every byte
// is read from HBM.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "xcorr_launch.h"

namespace xeng {

namespace {

constexpr int kThreads = 512;                   // 8 waves
constexpr int kWaves = kThreads / 64;
constexpr int kBlockElems = 256;                // elements per workgroup, 4 per lane
constexpr int kStripRows = 2048;                // output rows per workgroup
constexpr int kChunk = 128;                     // output rows gathered per ring step
constexpr int kMaxSpread = 128;                 // ring form: largest delay spread
// The ring: kArrays arrays of kChunk input rows of 256 bytes. A chunk of
// output rows reads two of them (its rows and up to kMaxSpread more) while the
// next three are loaded. With 256-byte rows every lane reads only its own
// dword column of any row, so the gathers meet no bank conflicts.
constexpr int kArrays = 5;
constexpr int kRowBytes = kBlockElems;
constexpr int kArrayBytes = kChunk * kRowBytes;   // 32 KiB
constexpr int kRowsPerLoad = 1024 / kRowBytes;    // a 16-byte LDS-DMA load fills 1 KiB
constexpr int kLoaders = kWaves / 2;
constexpr int kLoadsPerChunk = kChunk / kRowsPerLoad / kLoaders;   // per loader wave
constexpr uint32_t kOob = 0x80000000u;          // buffer offset past every record: reads 0
static_assert(kMaxSpread <= kChunk && (kChunk & (kChunk - 1)) == 0, "ring geometry");
static_assert(kArrays * kArrayBytes <= 160 * 1024, "LDS of one compute unit");
static_assert(kLoadsPerChunk * (kArrays - 1) <= 63, "loads in flight fit the vmcnt field");

typedef __attribute__((address_space(3))) void* lds_void_ptr;

// f(std::integral_constant<int, c>) for c = 0, 1, ...: one copy of the body
// per value, so c is a constant in each.
template <class F, int... c>
__device__ __forceinline__ void for_each_c(F&& f, std::integer_sequence<int, c...>) {
  (f(std::integral_constant<int, c>{}), ...);
}

// Wait until at most kLeft of this wave's vector-memory operations are in
// flight (they retire in issue order).
template <int kLeft>
__device__ inline void vm_wait() {
  static_assert(kLeft >= 0 && kLeft < 64, "vmcnt field");
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0x0F70 | (kLeft & 15) | ((kLeft >> 4) << 14));
  asm volatile("" ::: "memory");
}

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
  int aligned;            // ring form possible: 16-byte rows, dword stores
  uint16_t delay[kShiftGroupElems];
};

// This wave's LDS reads and writes are complete, then all waves meet.
__device__ inline void ring_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

__global__ __launch_bounds__(kThreads) void xcorr_shift_kernel(ShiftParams p) {
  __shared__ __attribute__((aligned(16))) uint8_t ring[kArrays * kArrayBytes];
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

  // spread of this block's delays: each wave reduces all 256 (4 per lane)
  // across its lanes, so every wave holds the same bounds without LDS
  int dmin = 0x7fffffff, dmax = -1;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (4 * lane + k < ne) {
      dmin = min(dmin, (int)p.delay[eb + 4 * lane + k]);
      dmax = max(dmax, (int)p.delay[eb + 4 * lane + k]);
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    dmin = min(dmin, __shfl_xor(dmin, m));
    dmax = max(dmax, __shfl_xor(dmax, m));
  }
  dmin = __builtin_amdgcn_readfirstlane(dmin);
  dmax = __builtin_amdgcn_readfirstlane(dmax);
  const int spread = dmax - dmin;
  const int e4 = eb + 4 * lane;                        // this lane's first element (launch-relative)
  const bool quad = 4 * lane < ne;                     // the lane has elements in this block
  int back[4];                                         // input row of output row s: s + back[k]
#pragma unroll
  for (int k = 0; k < 4; ++k) back[k] = (4 * lane + k < ne) ? dmax - (int)p.delay[e4 + k] : 0;

  if (p.aligned && spread <= kMaxSpread) {
    // relative input row r is input row base_row + r of the channel, for
    // r in [0, ns + spread); segment r / kChunk of the strip lives in ring
    // array (r / kChunk) % kArrays
    const int base_row = first_row - dmax;
    const int rows = ns + spread;
    const int64_t col0 = p.e_begin + eb;               // absolute element of the block
    const int64_t bytes = (int64_t)(p.t_in - base_row) * n - col0;   // to the channel's end
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(src + (int64_t)base_row * n + col0), 0,
        bytes > 0x7fffffff ? 0x7fffffff : (int)bytes, 0x00020000);
    // Waves 0-3 load the ring, waves 4-7 gather from it and store. Loads and
    // stores share one counter of outstanding vector-memory operations, so a
    // wave that did both would wait for its stores whenever it waits for its
    // loads; split this way the loaders wait for loads only and the
    // gatherers never wait on memory.
    const bool loader = wave < kLoaders;
    const int rw = loader ? wave : wave - kLoaders;     // index within the role
    // a 16-byte load: lane l carries row r0 + l / 16, bytes 16 (l % 16) ..
    const int lr = lane >> 4, lc = 16 * (lane & 15);
    const uint32_t voff = lc < ne ? (uint32_t)(lr * n + lc) : kOob;
    // segment k: rows [k * kChunk, (k + 1) * kChunk); loader wave rw loads
    // rows 4 (rw + 4 i) .. 4 (rw + 4 i) + 3. Every wave issues the same number
    // of loads per segment, so a count of loads in flight names the segments
    // still arriving: a load of rows the strip does not use reads past the
    // record (nothing from HBM).
    auto load_seg = [&](uint8_t* seg, int k) {
      const int lo = k * kChunk;
#pragma unroll
      for (int i = 0; i < kLoadsPerChunk; ++i) {
        const int r0 = lo + kRowsPerLoad * (rw + kLoaders * i);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (lds_void_ptr)(seg + (r0 - lo) * kRowBytes), 16,
            r0 < rows ? voff + (uint32_t)r0 * (uint32_t)n : kOob, 0, 0, 0);
      }
    };
    uint32_t* out = reinterpret_cast<uint32_t*>(dst + (int64_t)s0 * n + p.e_begin + e4);
    // Element q's byte of output row s sits in relative input row
    // rr = s - k * kChunk + back[q] of segments k and k + 1, in [0, 2 * kChunk):
    // array (c + rr / kChunk) % kArrays, row rr % kChunk, for c = k % kArrays.
    // The arrays are consecutive in the ring, so for c < kArrays - 1 both
    // segments form one run of rows and the byte sits at
    //   ring + c * kArrayBytes + rr * kRowBytes + 4 * lane + q:
    // a per-lane base (delay and column) plus the row, whose part common to
    // the wave's four rows goes into the reads' immediate offsets. Only for
    // c = kArrays - 1 does segment k + 1 wrap to array 0. A wave gathers rows
    // rw, rw + 4, rw + 8, rw + 12 of every 16 (as the loaders load them), so
    // its rows lie at most 127 rows into the chunk and rr < 2 * kChunk.
    // The reads are inline assembly that waits for its own results (16 reads
    // per wait): the compiler cannot tell which array a read touches and would
    // otherwise wait for every load in flight before each.
    const uint32_t lds0 = (uint32_t)(uintptr_t)(lds_void_ptr)ring + 4 * lane;
    uint32_t col[4];                                   // lane's byte q, delay included
#pragma unroll
    for (int q = 0; q < 4; ++q) col[q] = lds0 + (uint32_t)(back[q] * kRowBytes + q);
    auto gather = [&](auto cc, int k) {
      constexpr int c = decltype(cc)::value;
      if (!quad) return;
      const int end = min(ns, (k + 1) * kChunk);
      for (int s = k * kChunk + rw; s < end; s += 4 * kLoaders) {
        const uint32_t row = (uint32_t)(c * kArrayBytes + (s - k * kChunk) * kRowBytes);
        uint32_t v[4][4];
        if constexpr (c < kArrays - 1) {
          const uint32_t a0 = col[0] + row, a1 = col[1] + row, a2 = col[2] + row,
                         a3 = col[3] + row;
          asm volatile(
              "ds_read_u8 %0, %16\n\tds_read_u8 %1, %17\n\tds_read_u8 %2, %18\n\t"
              "ds_read_u8 %3, %19\n\tds_read_u8 %4, %16 offset:1024\n\t"
              "ds_read_u8 %5, %17 offset:1024\n\tds_read_u8 %6, %18 offset:1024\n\t"
              "ds_read_u8 %7, %19 offset:1024\n\tds_read_u8 %8, %16 offset:2048\n\t"
              "ds_read_u8 %9, %17 offset:2048\n\tds_read_u8 %10, %18 offset:2048\n\t"
              "ds_read_u8 %11, %19 offset:2048\n\tds_read_u8 %12, %16 offset:3072\n\t"
              "ds_read_u8 %13, %17 offset:3072\n\tds_read_u8 %14, %18 offset:3072\n\t"
              "ds_read_u8 %15, %19 offset:3072\n\ts_waitcnt lgkmcnt(0)"
              : "=&v"(v[0][0]), "=&v"(v[0][1]), "=&v"(v[0][2]), "=&v"(v[0][3]), "=&v"(v[1][0]),
                "=&v"(v[1][1]), "=&v"(v[1][2]), "=&v"(v[1][3]), "=&v"(v[2][0]), "=&v"(v[2][1]),
                "=&v"(v[2][2]), "=&v"(v[2][3]), "=&v"(v[3][0]), "=&v"(v[3][1]), "=&v"(v[3][2]),
                "=&v"(v[3][3])
              : "v"(a0), "v"(a1), "v"(a2), "v"(a3)
              : "memory");
        } else {
          // segment k + 1 is array 0: rows past the chunk's end move back by
          // the whole ring
          uint32_t at[4][4];
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int rr = s + j * kLoaders - k * kChunk + back[q];
              at[j][q] = col[q] + row + (uint32_t)(j * kLoaders * kRowBytes) -
                         (rr >= kChunk ? (uint32_t)(kArrays * kArrayBytes) : 0u);
            }
          asm volatile(
              "ds_read_u8 %0, %16\n\tds_read_u8 %1, %17\n\tds_read_u8 %2, %18\n\t"
              "ds_read_u8 %3, %19\n\tds_read_u8 %4, %20\n\tds_read_u8 %5, %21\n\t"
              "ds_read_u8 %6, %22\n\tds_read_u8 %7, %23\n\tds_read_u8 %8, %24\n\t"
              "ds_read_u8 %9, %25\n\tds_read_u8 %10, %26\n\tds_read_u8 %11, %27\n\t"
              "ds_read_u8 %12, %28\n\tds_read_u8 %13, %29\n\tds_read_u8 %14, %30\n\t"
              "ds_read_u8 %15, %31\n\ts_waitcnt lgkmcnt(0)"
              : "=&v"(v[0][0]), "=&v"(v[0][1]), "=&v"(v[0][2]), "=&v"(v[0][3]), "=&v"(v[1][0]),
                "=&v"(v[1][1]), "=&v"(v[1][2]), "=&v"(v[1][3]), "=&v"(v[2][0]), "=&v"(v[2][1]),
                "=&v"(v[2][2]), "=&v"(v[2][3]), "=&v"(v[3][0]), "=&v"(v[3][1]), "=&v"(v[3][2]),
                "=&v"(v[3][3])
              : "v"(at[0][0]), "v"(at[0][1]), "v"(at[0][2]), "v"(at[0][3]), "v"(at[1][0]),
                "v"(at[1][1]), "v"(at[1][2]), "v"(at[1][3]), "v"(at[2][0]), "v"(at[2][1]),
                "v"(at[2][2]), "v"(at[2][3]), "v"(at[3][0]), "v"(at[3][1]), "v"(at[3][2]),
                "v"(at[3][3])
              : "memory");
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int sj = s + j * kLoaders;
          if (sj >= end) break;
          const uint32_t w = v[j][0] | (v[j][1] << 8) | (v[j][2] << 16) | (v[j][3] << 24);
          *reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(out) + (int64_t)sj * n) = w;
        }
      }
    };
    // Step k: the loaders' segments up to k + 1 are in (at most the loads of
    // segments k + 2 and k + 3 in flight), then at the barrier everyone's are
    // and chunk k - 1 is read; the loaders load segment k + 4 into the array
    // chunk k - 1 read first while the gatherers gather chunk k.
    const int nchunks = (ns + kChunk - 1) / kChunk;
    if (loader)
      for (int k = 0; k < kArrays - 1; ++k) load_seg(ring + k * kArrayBytes, k);
    for (int k0 = 0; k0 < nchunks; k0 += kArrays) {
      for_each_c(
          [&](auto cc) {
            constexpr int c = decltype(cc)::value;
            const int k = k0 + c;
            if (k >= nchunks) return;
            if (loader) vm_wait<2 * kLoadsPerChunk>();
            ring_barrier();
            if (loader)
              load_seg(ring + ((c + kArrays - 1) % kArrays) * kArrayBytes, k + kArrays - 1);
            else
              gather(cc, k);
          },
          std::make_integer_sequence<int, kArrays>{});
    }
    // no load into LDS may land after the workgroup ends
    if (loader) vm_wait<0>();
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
  // the ring form loads 16-byte pieces of rows (every row of a block must
  // start on a 16-byte boundary), stores dwords and addresses a strip's rows
  // with 32-bit offsets
  p.aligned = n % 16 == 0 && e_begin % 16 == 0 && reinterpret_cast<uintptr_t>(in) % 16 == 0 &&
              reinterpret_cast<uintptr_t>(out) % 4 == 0 &&
              (int64_t)(kStripRows + kMaxSpread + kArrays * kChunk) * n < ((int64_t)1 << 31);
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
