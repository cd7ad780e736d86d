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
// One workgroup covers 256 elements and 128 output rows of one channel. When
// the delays of its elements differ by at most kMaxSpread, it loads the input
// rows its output rows need, [lo, lo + 128 + spread), whole and coalesced into
// LDS (one dword of 4 elements per lane and row), and each lane then gathers
// its 4 elements' bytes from the rows their delays name and writes them as
// one dword. Otherwise (a wider spread, or an input that dword loads cannot
// read) every byte is read from HBM directly.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xcorr_launch.h"

namespace xeng {

namespace {

constexpr int kThreads = 512;                   // 8 waves
constexpr int kBlockElems = 256;                // elements per workgroup, 4 per lane
constexpr int kTileRows = 128;                  // output rows per workgroup
constexpr int kMaxSpread = 128;                 // staged form: largest delay spread
constexpr int kStageRows = kTileRows + kMaxSpread;
constexpr int kRowStride = kBlockElems + 4;     // 65 dwords: rows start on different banks
constexpr int kBatch = 8;                       // staging loads in flight per lane
static_assert(kStageRows * kRowStride <= 80 * 1024, "two workgroups per compute unit");

struct ShiftParams {
  const uint8_t* in;
  uint8_t* out;
  int n;
  int64_t in_cs;          // bytes per input channel: (t + max_delay) * n
  int64_t out_cs;         // bytes per output channel: tc * n
  int max_delay, t0, tc;
  int e_begin, e_count;   // the elements whose delays this launch carries
  int tiles;              // row tiles per channel
  int blocks;             // 256-element blocks of this launch
  int aligned;            // n % 4 == 0 and 4-byte aligned in and out: dword access
  uint16_t delay[kShiftGroupElems];
};

__global__ __launch_bounds__(kThreads) void xcorr_shift_kernel(ShiftParams p) {
  __shared__ __attribute__((aligned(16))) uint8_t rows[kStageRows * kRowStride];
  __shared__ int bounds[2];
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b = (int)(blockIdx.x % (unsigned)p.blocks);
  const int rest = (int)(blockIdx.x / (unsigned)p.blocks);
  const int tile = rest % p.tiles, c = rest / p.tiles;
  const int eb = b * kBlockElems;                      // first element, within the launch
  const int ne = min(kBlockElems, p.e_count - eb);     // elements of this block
  const int s0 = tile * kTileRows, ns = min(kTileRows, p.tc - s0);
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
  const int need = ns + dmax - dmin;                   // input rows the tile reads
  const int e4 = eb + 4 * lane;                        // this lane's first element (launch-relative)
  const bool quad = e4 < ne + eb;                      // the lane has elements in this block
  int back[4];                                         // rows behind the latest row a lane's element uses
#pragma unroll
  for (int k = 0; k < 4; ++k) back[k] = (e4 + k < eb + ne) ? dmax - (int)p.delay[e4 + k] : 0;

  if (p.aligned && need <= kStageRows) {
    // stage input rows [first_row - dmax, first_row - dmax + need) of the block
    const int64_t col = p.e_begin + e4;                // absolute element of the lane's dword
    const uint8_t* base = src + (int64_t)(first_row - dmax) * n + col;
    for (int r0 = wave; r0 < need; r0 += kBatch * (kThreads / 64)) {
      uint32_t v[kBatch];
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int r = r0 + k * (kThreads / 64);
        v[k] = (quad && r < need) ? *reinterpret_cast<const uint32_t*>(base + r * n) : 0u;
      }
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int r = r0 + k * (kThreads / 64);
        if (r < need) *reinterpret_cast<uint32_t*>(rows + r * kRowStride + 4 * lane) = v[k];
      }
    }
    __syncthreads();
    if (!quad) return;
    // output row s, element e: input row first_row + s - delay[e], staged row
    // s + dmax - delay[e]
    uint32_t* out = reinterpret_cast<uint32_t*>(dst + (int64_t)s0 * n + p.e_begin + e4);
    for (int s = wave; s < ns; s += kThreads / 64) {
      uint32_t w = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        w |= (uint32_t)rows[(s + back[k]) * kRowStride + 4 * lane + k] << (8 * k);
      *reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(out) + (int64_t)s * n) = w;
    }
    return;
  }
  // direct form: every byte from HBM
  if (!quad) return;
  for (int s = wave; s < ns; s += kThreads / 64) {
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

int shift_tile_rows() { return kTileRows; }

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
  p.in_cs = (int64_t)t_in * n;
  p.out_cs = (int64_t)tc * n;
  p.max_delay = max_delay;
  p.t0 = t0;
  p.tc = tc;
  p.e_begin = e_begin;
  p.e_count = e_count;
  p.tiles = (tc + kTileRows - 1) / kTileRows;
  p.blocks = (e_count + kBlockElems - 1) / kBlockElems;
  p.aligned = n % 4 == 0 && reinterpret_cast<uintptr_t>(in) % 4 == 0 &&
              reinterpret_cast<uintptr_t>(out) % 4 == 0;
  for (int k = 0; k < kShiftGroupElems; ++k) {
    const int d = k < e_count ? delays[e_begin + k] : 0;
    if (d < 0 || d > max_delay) return hipErrorInvalidValue;
    p.delay[k] = (uint16_t)d;
  }
  const int64_t grid = (int64_t)f * p.tiles * p.blocks;
  if (grid <= 0 || grid > 0x7fffffff) return hipErrorInvalidConfiguration;
  xcorr_shift_kernel<<<dim3((unsigned)grid), dim3(kThreads), 0, stream>>>(p);
  return hipGetLastError();
}

}  // namespace xeng
