// xcorr_launch.h -- host-side launchers of the correlation kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xeng {

// Zero `pairs` int32 pairs starting at vis (a fill kernel, so it is also safe
// to record into a captured graph).
hipError_t launch_fill_zero(int32_t* vis, int64_t pairs, hipStream_t stream);

// 128x128-tile MFMA kernel. split > 1 divides the time axis among that many
// workgroups per tile and combines them with int32 atomic adds; the caller
// zero-fills vis first when not accumulating. aligned = (n % 4 == 0 and the
// input base is 4-byte aligned), which enables dword loads.
hipError_t launch_tile128(const uint8_t* in, int32_t* vis, int n, int f, int t, int accumulate,
                          int split, bool aligned, hipStream_t stream);
int tile128_stage_samples();

// Kernel for arrays of any size (n % 4 == 0, 4-byte aligned input; meant for
// n > 256): each channel is cut into rect_units_per_channel(n) pieces, the
// 256-element diagonal squares (the triangle kernel's block programs) and the
// 128x256 tiles above them. Sums samples [t0, t0 + t_count); sums are
// unscaled, so one launch may cover any t_count. split > 1 divides the time
// axis and combines with int32 atomic adds (the caller zero-fills vis first
// when not accumulating).
hipError_t launch_rect(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                       int64_t cs, int t0, int t_count, int accumulate, int split,
                       hipStream_t stream);
int64_t rect_units_per_channel(int n);
// launch_rect on bf6 operands (exact for 4-bit values): same arguments and
// limits; split must keep every part within tri_bf6_min_split's bound
// (returns hipErrorInvalidValue otherwise).
hipError_t launch_rect_bf6(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                           int64_t cs, int t0, int t_count, int accumulate, int split,
                           hipStream_t stream);
// launch_rect over several sample segments [seg_t0[k], seg_t_end[k]) of each
// channel (host arrays, 1 <= count <= tri_max_segments()), summed into one
// result; otherwise as launch_rect with t0 = 0, t_count = t.
hipError_t launch_rect_segments(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                                int64_t cs, const int32_t* seg_t0, const int32_t* seg_t_end,
                                int count, int accumulate, int split, hipStream_t stream);

// Kernel for arrays of at most small_max_elements() elements (n % 4 == 0,
// 4-byte aligned input), bound by the input stream: each wave correlates one
// channel over a part of the time axis from a private ring of staged samples.
// Sums samples [t0, t0 + t_count) of each channel (any t_count); cus = compute
// units to fill. Overwrites vis unless accumulate (no zero fill needed).
hipError_t launch_small(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                        int64_t cs, int t0, int t_count, int accumulate, int cus,
                        hipStream_t stream);
int small_max_elements();

// Delay compensation ahead of correlation (any n): writes the delay-aligned
// window of tc frame samples starting at frame sample t0 as a dense
// uint8[f][tc][n] buffer,
//   out[c][s][e] = in[c][max_delay + t0 + s - delays[e]][e],
// for the elements [e_begin, e_begin + e_count) (e_count <= kShiftGroupElems;
// their delays travel as kernel arguments). in is uint8[f][t_in][n] with
// t_in >= max_delay + t0 + tc; delays is a host array of n values in
// [0, max_delay]. Returns hipErrorInvalidValue for arguments out of range.
constexpr int kShiftGroupElems = 1024;
hipError_t launch_shift(const uint8_t* in, uint8_t* out, int n, int f, int t_in, int max_delay,
                        int t0, int tc, int e_begin, int e_count, const int32_t* delays,
                        hipStream_t stream);
int shift_tile_rows();

// Triangle kernel for n <= tri_max_elements() (n % 4 == 0, 4-byte aligned
// input): one workgroup per channel (times split) computes the channel's whole
// upper triangle. Sums samples [t0, t0 + t_count) of each channel; sums are
// unscaled, so one launch may cover any t_count. split > 1 divides the time
// axis and combines with int32 atomic adds (the caller zero-fills vis first
// when not accumulating).
hipError_t launch_tri(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                      int64_t cs, int t0, int t_count, int accumulate, int split,
                      hipStream_t stream);
// Delay compensation on the triangle kernel: in is uint8[f][t + max_delay][n]
// (max_delay halo samples first); output sample s of element e is input
// sample s + max_delay - delays[e] (host array of n values in [0, max_delay]).
// Needs n <= tri_max_elements(), t % tri_stage_samples() == 0, t > 0.
// Picks the form from the delays: one common delay runs launch_tri on the
// shifted window, a spread up to 128 the ring (window) form, anything else or
// a misaligned input the bytewise gather form.
hipError_t launch_tri_delayed(const uint8_t* in, int32_t* vis, int n, int f, int t,
                              const int32_t* delays, int max_delay, int accumulate, int split,
                              hipStream_t stream);
// The triangle kernel on bf6 operands (exact for 4-bit values): same
// arguments and limits as launch_tri; split must keep every part within
// tri_bf6_min_split's bound (returns hipErrorInvalidValue otherwise).
hipError_t launch_tri_bf6(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                          int64_t cs, int t0, int t_count, int accumulate, int split,
                          hipStream_t stream);
// Smallest time split that keeps every part's fp32 sums exact.
int tri_bf6_min_split(int64_t t_count);
// The triangle kernel over several sample segments [seg_t0[k], seg_t_end[k])
// of each channel (host arrays, 1 <= count <= tri_max_segments()), summed
// into one result; otherwise as launch_tri.
hipError_t launch_tri_segments(const uint8_t* in, int32_t* vis, int n, int f, int t, int64_t ss,
                               int64_t cs, const int32_t* seg_t0, const int32_t* seg_t_end,
                               int count, int accumulate, int split, hipStream_t stream);
int tri_max_segments();
int tri_max_elements();
int tri_stage_samples();

// ---- batched mode: persistent launches over a queue of work items -------------
// Device-side image written by the host (plans, the server) into the caller's
// workspace: [header][job table][items]. Every job is cut into the pieces of
// launch_rect (one diagonal square per 256 elements and the tiles above
// them; a job of at most 256 elements is one square, the triangle kernel's
// work); one item = one piece of one channel over a range of stages.
struct QueueJob {            // one correlation job (one window of its samples)
  const uint8_t* in;
  int32_t* vis;
  int n, f, t;               // elements, channels, samples per channel
  int64_t ss, cs;            // bytes from one sample to the next, one channel to the next
  int t0, t_end;             // window of samples this job sums
  int nbc, units, total_stages;   // 256-element blocks, pieces per channel, stages
  int accumulate, atomic_out;
  int zero_first;            // zero vis before the queue runs (atomic sums, not accumulating)
};
struct QueueItem {           // one piece of one channel over a range of stages
  int job, ch, unit, stage_begin, stage_end, pad[3];
};
constexpr int kQueueParts = 8;   // one sub-queue per XCD
constexpr int kQueueHeaderStride = 256;
struct QueueHeader {
  unsigned cursor[kQueueParts];  // next item of each sub-queue (self-resetting)
  unsigned done;                 // workgroups that have finished (self-resetting)
  int part_begin[kQueueParts + 1];  // items of sub-queue k: [part_begin[k], part_begin[k+1])
  int jobs_offset;               // byte offset of the QueueJob array
  int items_offset;              // byte offset of the QueueItem array
  int pad[5];
};
static_assert(sizeof(QueueHeader) <= kQueueHeaderStride, "queue header size");
// Byte offsets of the job table and of the item array in a queue image.
__host__ __device__ inline size_t queue_jobs_offset() { return (size_t)kQueueHeaderStride; }
__host__ __device__ inline size_t queue_items_offset(int njobs) {
  return (queue_jobs_offset() + sizeof(QueueJob) * (size_t)njobs + 255) / 256 * 256;
}
// The header's offsets and item ranges, the item list and the job table are
// not written while a queue kernel runs (only cursor and done are, by atomics),
// so kernels read them through the constant address space: scalar loads, whose
// results stay in scalar registers and keep buffer descriptors scalar.
typedef const __attribute__((address_space(4))) QueueHeader* QueueHeaderC;
typedef const __attribute__((address_space(4))) QueueItem* QueueItemC;
typedef const __attribute__((address_space(4))) QueueJob* QueueJobC;

int queue_stage_samples();
// Build the image for job table `table` with `split` stage ranges per piece
// (*items_out receives the item count). The job table must already hold n, f,
// t0, t_end, total_stages, nbc and units.
void build_queue_image(const QueueJob* table, int njobs, int split, uint8_t** image_out,
                       size_t* bytes_out, int64_t* items_out);
// One persistent launch over the image's items (nothing if items == 0), on
// `stream`; grid = workgroups (one per compute unit).
hipError_t launch_queue(void* d_ws, int64_t items, int grid, hipStream_t stream);

}  // namespace xeng
