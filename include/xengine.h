/*
 * xengine.h -- C ABI of the MI355X (gfx950) 4-bit X-engine correlator.
 *
 * The operation (Klages et al., "GPU Kernels for High-Speed 4-Bit
 * Astrophysical Data Processing"):
 *   For every frequency channel f and every element pair i <= j,
 *     V_f[i][j] = sum over t of x_i(t) * conj(x_j(t))
 *   with the complex product written out in Eq. 1 (Sec. II-A):
 *     Re = xRe*yRe + xIm*yIm,   Im = xIm*yRe - xRe*yIm.
 *   Only the upper triangle is produced: the matrix is Hermitian (Sec. II-A,
 *   Eq. 2 counts N(N+1)/2 entries).
 *
 * Input samples (Sec. III, Excess-8): one byte per complex sample; the high
 * nibble holds Re + 8 and the low nibble Im + 8, each value in [-8, 7].
 *
 * Layouts (all row-major, no padding):
 *   input   uint8_t  in[F][T][N]          channel, time sample, element
 *   output  int32_t  vis[F][N(N+1)/2][2]  (re, im) per entry; entry (i, j),
 *           i <= j, sits at k(i,j) = i*(2N-i+1)/2 + (j-i), so each row i of the
 *           triangle is contiguous.
 *
 * Accumulation (Sec. III-A: new sums are added to the results already held):
 *   accumulate = 0 overwrites vis; accumulate = 1 adds to it. t_prev is the
 *   number of samples already summed into vis (0 when overwriting). Sums are
 *   exact in int32 while t_prev + t <= XENG_MAX_SAMPLES, since one sample
 *   contributes at most 128 in magnitude; beyond that the call is refused.
 *
 * Memory and streams: every d_ pointer is device memory owned by the caller
 * (typically allocated through PyTorch). The library never allocates or frees
 * device memory, and keeps none apart from one static array per device that
 * only xeng_plan_run_static uses (XENG_STATIC_SCRATCH_BYTES). All GPU work is
 * enqueued on the caller's hipStream_t (passed as void*, NULL = the null
 * stream) and returns without waiting; buffers must stay valid until that work
 * completes.
 *
 * Errors: every call returns an xeng_status; nothing throws or aborts across
 * this boundary. xeng_last_error() returns a message for the calling thread's
 * last failed call.
 */
#ifndef XENGINE_H
#define XENGINE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XENG_MAX_SAMPLES 16777215LL
/* Size of the device array that xeng_plan_run_static uses on each GPU. */
#define XENG_STATIC_SCRATCH_BYTES (8LL << 20)

typedef enum xeng_status {
  XENG_OK = 0,
  XENG_EINVAL = -1,    /* bad pointer, size, alignment or overlap */
  XENG_ERANGE = -2,    /* t_prev + t would leave the exact int32 range */
  XENG_ENOMEM = -3,    /* host allocation failed, or workspace too small */
  XENG_EDEVICE = -4,   /* a HIP runtime call failed; see xeng_last_error() */
  XENG_EBUSY = -5,     /* admission refused: no memory or slot free now */
  XENG_ENOTFOUND = -6  /* unknown job, ticket or variant */
} xeng_status;

/* Message for the calling thread's most recent failed call ("" if none).
 * The pointer stays valid until the thread's next call into the library. */
const char* xeng_last_error(void);

/* Library version string. */
const char* xeng_version(void);

/* Entries of the packed upper triangle, n(n+1)/2 (Eq. 2); -1 if n < 0. */
int64_t xeng_vis_entries(int n);

/* Packed index k(i,j) = i*(2n-i+1)/2 + (j-i) for 0 <= i <= j < n, else -1. */
int64_t xeng_tri_index(int n, int i, int j);

/* Number of square tiles of edge `tile` that cover the upper triangle of an
 * n x n matrix (Sec. II-C, Fig. 1: 36 tiles of 32 for n = 256); -1 if invalid. */
int64_t xeng_tile_count(int n, int tile);

/*
 * Plain correlation of one job (Sec. II-A, Eq. 1 summed over t; upper
 * triangle per Eq. 2).
 *   d_in   device uint8_t[f][t][n], read only; any alignment.
 *   d_vis  device int32_t[f][n(n+1)/2][2], 8-byte aligned; must not overlap d_in.
 *   n >= 1 elements, f >= 1 channels, t >= 0 samples.
 *   t == 0: zero-fills vis when accumulate == 0, does nothing otherwise.
 * Returns XENG_EINVAL, XENG_ERANGE or XENG_EDEVICE on failure, in which case
 * nothing was enqueued.
 */
xeng_status xeng_correlate(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t,
                           int64_t t_prev, int accumulate, void* hip_stream);

/*
 * Kernel variants, for the autotuner and for tests that compare variants.
 * A variant fixes the tile shape and the samples staged per step; split_t >= 1
 * divides the time axis among that many workgroups per tile (partial sums are
 * combined with exact int32 atomic adds). Every variant gives bit-identical
 * results. variant = -1 lets the library choose (same as xeng_correlate).
 *   0 tile128_kc64_mfma32x32x32         any n, any input alignment
 *   1, 2 retired (128 x 256 tiles with 4 or 8 waves, superseded by 5):
 *     xeng_correlate_variant returns XENG_ENOTFOUND for them
 *   3 tri256_w8_kc64_mfma32x32x32       n <= 256, n % 4 == 0, aligned input
 *   4 tri256_w8_bf6_mfma32x32x64        as 3, on the f8f6f4 matrix cores: the
 *     4-bit values (Sec. III) are exact in the 6-bit float E3M2 and partial
 *     sums are exact in fp32 below 2^24, so each workgroup sums at most
 *     131 008 samples; split_t is raised to that bound where needed.
 *   5 rect128x256_tri256_w8_kc64_mfma32x32x32  n % 4 == 0, aligned input: the
 *     triangle cut into 256-element diagonal squares (the blocks of variant 3)
 *     and 128 x 256 tiles wholly above them (Sec. II-C: only tiles that reach
 *     the upper triangle are computed); the default for n > 256.
 *   6 small64_w8_ring16_mfma32x32x32   n <= 64, n % 4 == 0, aligned input: each
 *     wave streams one channel (or a part of its time axis) through a private
 *     ring in LDS; bound by HBM rather than the matrix cores at these sizes;
 *     the default for n <= 64. split_t is ignored (the kernel combines its
 *     time parts itself).
 *   7 rect128x256_tri256_w8_bf6_mfma32x32x64  as 5 on the f8f6f4 matrix
 *     cores with bf6 (E3M2) operands, exact as variant 4 is; split_t is
 *     raised so that no workgroup sums more than 131 008 samples.
 */
int xeng_variant_count(void);
const char* xeng_variant_name(int variant);   /* NULL if out of range */
xeng_status xeng_correlate_variant(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t,
                                   int64_t t_prev, int accumulate, int variant, int split_t,
                                   void* hip_stream);

/*
 * Correlation of a strided input, as for xeng_correlate otherwise. Element e
 * of channel c at sample s is the byte d_in[s * sample_stride +
 * c * channel_stride + e]; elements of one sample are contiguous. The dense
 * layout is sample_stride = n, channel_stride = t * n; the time-major packet
 * stream of Sec. III (Fig. 2: samples, then channels, then elements) is
 * sample_stride = f * n, channel_stride = n, read in place with no transpose.
 * Needs n % 4 == 0, a 4-byte aligned d_in, both strides multiples of 4,
 * sample_stride >= n and sample_stride <= (2^31 - n) / 32; the overlap check
 * uses the strided extent. Errors as for xeng_correlate.
 */
xeng_status xeng_correlate_strided(const uint8_t* d_in, int64_t sample_stride,
                                   int64_t channel_stride, int32_t* d_vis, int n, int f, int t,
                                   int64_t t_prev, int accumulate, void* hip_stream);

/*
 * Gated correlation: G accumulator sets, each time sample summed into the set
 * of its gate. The time axis is cut into blocks of `block` samples (the last
 * may be shorter); gate_of_block[k] (host array of ceil(t / block) bytes)
 * names the gate of block k, 0 <= gate < gates, or 0xFF to leave the block out
 * (flagged data). Each gate g gets V_g[i][j] = sum over its samples of
 * x_i(t) * conj(x_j(t)) (Sec. II-A, Eq. 1), the same packed triangle as
 * xeng_correlate.
 *   d_in   device uint8_t[f][t][n] (dense layout), read only.
 *   d_vis  device int32_t[gates][f][n(n+1)/2][2].
 *   t_prev host int64_t[gates]: samples already summed per gate (used when
 *          accumulate == 1, may be NULL when accumulate == 0).
 *   accumulate 0 overwrites every gate's set (gates without samples become
 *          zero), 1 adds to them; each gate's total must stay within
 *          XENG_MAX_SAMPLES (XENG_ERANGE otherwise).
 * All runs of one gate (consecutive blocks of that gate) are summed in one
 * launch per gate (up to 32 runs each), on the triangle kernel for n <= 256
 * and on the kernel of diagonal squares and tiles above that. Runs are read
 * in place as sub-ranges, so n % 4 == 0 and a 4-byte aligned d_in are
 * required. Errors as for xeng_correlate, XENG_EINVAL for gates < 1 or > 255,
 * block < 1, or a gate index out of range.
 */
xeng_status xeng_correlate_gated(const uint8_t* d_in, int32_t* d_vis, int gates, int n, int f,
                                 int t, int block, const uint8_t* gate_of_block,
                                 const int64_t* t_prev, int accumulate, void* hip_stream);

/*
 * Delay compensation (Sec. IV: single elements shifted by whole time steps
 * before correlation): an integer sample delay per element, applied while
 * the samples are staged, so each element's stream is aligned before the
 * products of Eq. 1 are summed:
 *   V_ij = sum_{s<t} x_i(s - delays[i]) * conj(x_j(s - delays[j])).
 *   d_in    device uint8_t[f][t + max_delay][n]: the first max_delay samples of
 *           each channel are the halo (the end of the previous frame), sample
 *           s of the frame is d_in[.][max_delay + s][.].
 *   delays  host int32_t[n], each in [0, max_delay]; max_delay <= 65535.
 *   d_vis, t_prev, accumulate as for xeng_correlate (t counts frame samples).
 * Runs on the triangle kernel: n <= 256, and t % 64 == 0. With n % 4 == 0
 * and a 4-byte aligned d_in, one delay common to all elements is the plain
 * correlation of a shifted sample window, and a delay spread of at most 128
 * samples stages whole rows; otherwise each element's samples are gathered
 * bytewise (slower, any alignment). Errors as for xeng_correlate; XENG_EINVAL
 * for a delay out of range, n > 256 or t % 64 != 0 (xeng_correlate_delayed_ws
 * takes those).
 */
xeng_status xeng_correlate_delayed(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t,
                                   const int32_t* delays, int max_delay, int64_t t_prev,
                                   int accumulate, void* hip_stream);

/*
 * Delay compensation for any n and t (Sec. IV, as the paper lays it out: a
 * kernel shifts each element's samples by its delay ahead of correlation).
 * Arguments as for xeng_correlate_delayed, plus a caller workspace:
 *   d_workspace  device memory of ws_bytes bytes, not overlapping d_in or d_vis.
 * Where xeng_correlate_delayed applies (n <= 256, t % 64 == 0) the same fused
 * kernels run and the workspace is not touched. Otherwise windows of frame
 * samples are written delay-aligned into the workspace as dense
 * uint8_t[f][window][n] frames (an HBM-bound copy) and correlated by the
 * kernel xeng_correlate would use, each window after the first adding to the
 * sums; the window is as long as ws_bytes allows (a multiple of 128 samples),
 * so a workspace of xeng_delayed_workspace_bytes(n, f, t) runs in one pass.
 * Results are the same integers as xeng_correlate_delayed gives. Errors as
 * for xeng_correlate_delayed, and XENG_EINVAL for a workspace shorter than
 * f * n * min(t, 128) bytes or one that overlaps d_in or d_vis.
 */
size_t xeng_delayed_workspace_bytes(int n, int f, int t);   /* 0: none needed */
xeng_status xeng_correlate_delayed_ws(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t,
                                      const int32_t* delays, int max_delay, int64_t t_prev,
                                      int accumulate, void* d_workspace, size_t ws_bytes,
                                      void* hip_stream);

/*
 * The variant and time split xeng_correlate would use for a job of this shape
 * (host only, no device work). input_aligned: the input pointer is 4-byte
 * aligned. Kernels: small64 (n <= 64, n % 4 == 0, aligned input: a wave per
 * channel or part of one), tri256 (n <= 256 likewise: one workgroup per
 * channel covers the whole triangle), rect128x256_tri256 (other aligned
 * n % 4 == 0 jobs), tile128 (everything else). Returns XENG_EINVAL for n < 1, f < 1
 * or t < 0, or a NULL output pointer.
 */
xeng_status xeng_choose_variant(int n, int f, int t, int input_aligned, int* variant,
                                int* split_t);

/*
 * Autotuner of plain calls. For one job class it times every kernel variant
 * that can run the job (each with time splits 0 = its own choice, 1, 2, 4 and
 * 8; reps timed runs after one untimed), keeps the fastest and records it in
 * a process-wide table that xeng_correlate, xeng_correlate_strided and
 * xeng_choose_variant consult for jobs of the same class where that variant
 * can run them (otherwise the default rule applies). Every variant gives the
 * same integers, so tuning changes speed only. A class is (device
 * architecture, n, f, floor(log2 t)).
 *   d_in, d_vis  a job as for xeng_correlate (overwritten: on success d_vis
 *                holds the correlation of d_in)
 *   tune_cache_path  may be NULL; otherwise one line per tuned class is
 *                appended ("xeng-tune arch n f log2t variant split ms")
 *   variant, split_t, best_ms  may be NULL; receive the choice
 * XENG_EINVAL for an invalid job or t < 1, or an unwritable cache file.
 * xeng_tune_load reads such a file (lines of other architectures and
 * malformed lines are skipped, later lines replace earlier ones; entries may
 * be NULL) and returns XENG_ENOTFOUND if it cannot be read; xeng_tune_clear
 * forgets every choice.
 */
xeng_status xeng_autotune(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t, int reps,
                          const char* tune_cache_path, int* variant, int* split_t,
                          float* best_ms, void* hip_stream);
xeng_status xeng_tune_load(const char* tune_cache_path, int* entries);
void xeng_tune_clear(void);

/* ---- Batched mode: many jobs in one persistent launch ------------------------
 * A plan holds a list of independent correlation jobs (each as for
 * xeng_correlate) of mixed n, f and t and runs them all with one launch of a
 * persistent kernel that pulls pieces (channel, 256-element diagonal square
 * or 128x256 tile above the squares, range of time stages) from a queue in
 * device memory. Results are bit-identical to one
 * xeng_correlate per job. Jobs need n % 4 == 0 and 4-byte aligned inputs; the
 * outputs of different jobs must not overlap.
 *
 * The plan's device image (job table, piece queue, counters) lives in a
 * workspace of xeng_plan_workspace_bytes() bytes that the caller allocates and
 * passes in; the library keeps no device memory. Order of calls:
 *   xeng_plan_create -> xeng_plan_upload (copies the image, stream-ordered)
 *   -> xeng_plan_run (kernel launches only; may be captured in a graph)
 *   -> per new frame: xeng_plan_set_frame (rewrites the job table) -> run.
 * A run leaves its counters reset, so runs can follow each other or be
 * replayed from a graph without re-uploading. Runs on one workspace must not
 * overlap in time.
 */
typedef struct xeng_plan xeng_plan;
typedef struct xeng_job {
  const uint8_t* d_in;   /* device uint8_t[f][t][n] */
  int32_t* d_vis;        /* device int32_t[f][n(n+1)/2][2] */
  int n, f, t;
  int64_t t_prev;        /* samples already summed in d_vis (0 unless accumulating) */
  int accumulate;        /* 0 overwrite, 1 add */
} xeng_job;

/* Build a plan (host only). tune_cache_path (may be NULL) names a text file
 * written by xeng_plan_autotune; a tuned time split for the same job shapes is
 * applied. */
xeng_status xeng_plan_create(xeng_plan** out, const xeng_job* jobs, int njobs,
                             const char* tune_cache_path);
/* Workspace bytes for the plan; enough for every time split the autotuner may
 * choose, so one allocation serves the plan for its whole life. */
size_t xeng_plan_workspace_bytes(const xeng_plan* plan);
int64_t xeng_plan_items(const xeng_plan* plan);   /* pieces in the queue; -1 if plan is NULL */
int xeng_plan_split(const xeng_plan* plan);       /* stages are split this many ways per tile */
xeng_status xeng_plan_upload(xeng_plan* plan, void* d_workspace, void* hip_stream);
/* Rebind every job to a new frame: d_in[k] (NULL keeps the inputs) and
 * accumulate (1: add to the sums, subject to the int32 range guard). The job
 * table is copied into d_workspace on hip_stream; with d_workspace NULL only
 * the plan's host copy changes (for xeng_plan_run_static, which uploads the
 * whole image on every call). */
xeng_status xeng_plan_set_frame(xeng_plan* plan, const uint8_t* const* d_in, int accumulate,
                                void* d_workspace, void* hip_stream);
xeng_status xeng_plan_run(xeng_plan* plan, void* d_workspace, void* hip_stream);
/* xeng_plan_run for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * plan's image lives in a static device array of XENG_STATIC_SCRATCH_BYTES
 * that the library holds on each GPU it runs on until the process ends, so no
 * workspace is passed and nothing is allocated. Each call copies the plan's
 * whole image (its queue counters start at zero) into that array on
 * hip_stream and then launches the same kernels as xeng_plan_run; results are
 * bit-identical to it. No earlier xeng_plan_upload is needed; rebind frames
 * with xeng_plan_set_frame(plan, d_in, accumulate, NULL, stream). Every call
 * on one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (other streams, other threads) race and must be ordered by the caller.
 * XENG_EINVAL for a NULL plan or a plan whose image exceeds the array (about
 * 260 000 pieces); XENG_EDEVICE for a HIP error. */
xeng_status xeng_plan_run_static(xeng_plan* plan, void* hip_stream);
/* Capture one run into a HIP graph owned by the plan (uses a private stream),
 * and replay it on hip_stream. The graph reads the workspace captured with it. */
xeng_status xeng_plan_graph_capture(xeng_plan* plan, void* d_workspace);
xeng_status xeng_plan_graph_launch(xeng_plan* plan, void* hip_stream);
/* Time the plan with several time splits per tile (running it reps times
 * each), keep the fastest, re-upload, and append the choice to tune_cache_path
 * (may be NULL). best_ms may be NULL. Every timed run overwrites the jobs'
 * outputs with the correlation of their current inputs, so the plan's jobs
 * must all overwrite (accumulate = 0): a plan with an accumulating job is
 * refused with XENG_EINVAL and nothing runs. On success the outputs hold one
 * frame's sums, as after one xeng_plan_run. */
xeng_status xeng_plan_autotune(xeng_plan* plan, void* d_workspace, void* hip_stream, int reps,
                               const char* tune_cache_path, float* best_ms);
void xeng_plan_destroy(xeng_plan* plan);

/* ---- Serving mode: continuous batching of streamed frames --------------------
 * A server accepts correlation frames as they arrive. Each job (one stream of
 * frames of one (n, f) shape) owns a device accumulator int32[f][n(n+1)/2][2]
 * that its frames add into; the job's first frame overwrites it. A call of
 * xeng_server_step() retires finished work and then launches, on each free
 * slot, one persistent-kernel step holding the oldest pending frames of every
 * job that has nothing in flight (up to 16 of a job whose accumulator already
 * holds sums, added with int32 atomic adds; only its first frame, which
 * overwrites, runs alone); frames that arrive meanwhile join later steps, and
 * up to max_inflight steps run concurrently on the device (each on a stream of
 * its own, ordered after the work queued so far on hip_stream, the stream the
 * frames are produced on). Results are bit-identical to
 * xeng_correlate over each job's frames in order.
 *
 * Admission by memory: xeng_job_open refuses (XENG_EBUSY) an accumulator that
 * would push the open accumulators past hbm_budget bytes; a frame is launched
 * only while accumulators plus frames in flight stay within hbm_budget, and
 * otherwise waits. The workspace (ws_bytes of caller device memory, split in
 * max_inflight slots) holds the per-step queues. Served jobs need n % 4 == 0;
 * frames need 4-byte aligned input and t >= 1 (a job's samples stay within
 * XENG_MAX_SAMPLES).
 * Frame buffers must stay valid until their ticket is done. Latency is
 * measured from xeng_submit to the device-side completion of the frame's step.
 */
typedef struct xeng_server xeng_server;
xeng_status xeng_server_create(xeng_server** out, size_t hbm_budget, int max_inflight,
                               void* d_workspace, size_t ws_bytes, void* hip_stream);
xeng_status xeng_job_open(xeng_server* srv, int n, int f, int32_t* d_vis, int64_t* job_id);
xeng_status xeng_submit(xeng_server* srv, int64_t job_id, const uint8_t* d_frame, int t,
                        uint64_t* ticket);
/* launched (may be NULL) receives the number of frames started by this call. */
xeng_status xeng_server_step(xeng_server* srv, int* launched);
/* done = 1 once the frame's sums are in the accumulator; latency_us is then
 * the submit-to-completion time (else -1). */
xeng_status xeng_poll(xeng_server* srv, uint64_t ticket, int* done, double* latency_us);
/* Run until every submitted frame is done (blocks). */
xeng_status xeng_server_drain(xeng_server* srv);
/* XENG_EBUSY while the job has frames queued or in flight. */
xeng_status xeng_job_close(xeng_server* srv, int64_t job_id);
xeng_status xeng_server_stats(xeng_server* srv, int64_t* open_jobs, int64_t* pending_frames,
                              int64_t* inflight_steps, size_t* bytes_in_use);
void xeng_server_destroy(xeng_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* XENGINE_H */
