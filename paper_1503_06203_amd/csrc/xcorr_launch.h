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

// 128x256-tile MFMA kernel, one workgroup per CU. Needs n % 4 == 0 and a
// 4-byte aligned input (dword buffer loads). Sums samples [t0, t0 + t_count)
// of each channel (t = samples per channel); t_count is limited to
// wide_max_samples_per_launch() so the scaled int32 sums cannot overflow.
// waves = 4 (one wave of 64x128 per SIMD) or 8 (two waves of 64x64 per SIMD).
hipError_t launch_wide(const uint8_t* in, int32_t* vis, int n, int f, int t, int t0, int t_count,
                       int accumulate, int split, int waves, hipStream_t stream);
int64_t wide_max_samples_per_launch();
int64_t wide_tiles_per_channel(int n);

// Triangle kernel for n <= tri_max_elements() (n % 4 == 0, 4-byte aligned
// input): one workgroup per channel (times split) computes the channel's whole
// upper triangle. Sums samples [t0, t0 + t_count) of each channel; sums are
// unscaled, so one launch may cover any t_count. split > 1 divides the time
// axis and combines with int32 atomic adds (the caller zero-fills vis first
// when not accumulating).
hipError_t launch_tri(const uint8_t* in, int32_t* vis, int n, int f, int t, int t0, int t_count,
                      int accumulate, int split, hipStream_t stream);
int tri_max_elements();
int tri_stage_samples();

// ---- batched mode: one persistent launch over a queue of tiles --------------
// Device-side images written by the host plan into the caller's workspace.
struct QueueJob {            // one correlation job (one launch window of it)
  const uint8_t* in;
  int32_t* vis;
  int n, f, t;               // elements, channels, samples per channel
  int t0, t_end;             // window of samples this job sums
  int nbr, ntiles, total_stages;
  int accumulate, atomic_out, full_panels;
  int zero_first;            // zero vis before the queue runs (atomic sums, not accumulating)
};
struct QueueItem {           // one tile of one channel over a range of stages
  int job, ch, tile, stage_begin, stage_end, pad[3];
};
constexpr int kQueueParts = 8;   // one sub-queue per XCD
struct QueueHeader {
  unsigned cursor[kQueueParts];  // next item of each sub-queue (self-resetting)
  unsigned done;                 // workgroups that have finished (self-resetting)
  int part_begin[kQueueParts + 1];  // items of sub-queue k: [part_begin[k], part_begin[k+1])
  int jobs_offset;               // byte offset of the QueueJob array
  int items_offset;              // byte offset of the QueueItem array
  int pad[5];
};
// Byte offsets of the job and item arrays in a queue workspace.
__host__ __device__ inline size_t queue_jobs_offset() {
  return (sizeof(QueueHeader) + 255) / 256 * 256;
}
__host__ __device__ inline size_t queue_items_offset(int njobs) {
  return (queue_jobs_offset() + sizeof(QueueJob) * (size_t)njobs + 255) / 256 * 256;
}
// Launch the persistent kernel over a queue workspace prepared by the host.
hipError_t launch_queue(void* d_ws, int grid, hipStream_t stream);
int queue_stage_samples();
int64_t queue_tiles_per_channel(int n);

}  // namespace xeng
