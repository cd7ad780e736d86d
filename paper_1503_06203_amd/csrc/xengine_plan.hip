// xengine_plan.cpp -- batched mode: many correlation jobs of mixed size in one
// persistent launch over a flattened queue of tiles (the xeng_plan_* ABI).
//
// A plan turns each job into items (channel, piece, range of stages): the
// pieces are the 256-element diagonal squares and the 128 x 256 tiles above
// them (a job of at most 256 elements is one square). Items are ordered
// largest first, job by job and channel by channel (so pieces that share
// input panels stay together), and cut into kQueueParts contiguous sub-queues
// of about equal cost, one per XCD. The host builds the device
// image once; uploading it into the caller's workspace is the only copy. A run
// is then pure kernel launches (an optional zero fill, the queue kernel), so it
// can be captured in a HIP graph and replayed frame after frame; a new frame
// only rewrites the small job table (inputs, accumulate flags).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "xcorr_launch.h"
#include "xengine.h"
#include "xengine_internal.h"

namespace xeng {

namespace {

__global__ void queue_fill_kernel(const uint8_t* ws) {
  const QueueHeader* hdr = reinterpret_cast<const QueueHeader*>(ws);
  const QueueJob& J = reinterpret_cast<const QueueJob*>(ws + hdr->jobs_offset)[blockIdx.y];
  if (!J.zero_first) return;
  const int64_t pairs = (int64_t)J.f * ((int64_t)J.n * (J.n + 1) / 2);
  int2* out = reinterpret_cast<int2*>(J.vis);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < pairs; k += stride)
    out[k] = make_int2(0, 0);
}

constexpr int kMaxSplit = 8;   // largest per-tile time split the autotuner tries

}  // namespace

struct PlanWindow {
  int job;          // index into the user's job list
  int t0, t_end;
  bool first;       // first window of its job
};

}  // namespace xeng

struct xeng_plan {
  std::vector<xeng_job> jobs;
  std::vector<int64_t> held;       // samples each job's sums hold after the configured frame
  std::vector<xeng::PlanWindow> windows;
  int64_t items = 0;               // queue items
  std::vector<uint8_t> image;      // headers + job table + items, as uploaded
  int split = 1;                   // stage split per item (autotuned)
  size_t ws_bytes = 0;             // workspace for the largest split the tuner tries
  int grid = 0;
  // Some window combines partial sums with atomic adds. Such windows need a
  // zero fill whenever their job overwrites; the fill kernel is then part of
  // every run (and of a captured graph), and it reads each job's zero_first
  // flag on the device, so a later xeng_plan_set_frame that switches a job
  // between accumulating and overwriting needs no new capture.
  bool any_atomic = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  void* graph_ws = nullptr;
};

namespace xeng {
namespace {

// The job table (one entry per window) for the plan's current jobs.
std::vector<QueueJob> job_table(xeng_plan* pl) {
  const int stage = queue_stage_samples();
  std::vector<QueueJob> table;
  pl->any_atomic = false;
  for (size_t w = 0; w < pl->windows.size(); ++w) {
    const auto& win = pl->windows[w];
    const xeng_job& job = pl->jobs[win.job];
    const int nwin = (int)std::count_if(pl->windows.begin(), pl->windows.end(),
                                        [&](const PlanWindow& x) { return x.job == win.job; });
    QueueJob J{};
    J.in = job.d_in;
    J.vis = job.d_vis;
    J.n = job.n;
    J.f = job.f;
    J.t = job.t;
    J.ss = job.n;
    J.cs = (int64_t)job.t * job.n;
    J.t0 = win.t0;
    J.t_end = win.t_end;
    J.nbc = (job.n + 255) / 256;
    J.units = J.nbc * J.nbc;
    J.total_stages = (win.t_end - win.t0 + stage - 1) / stage;
    J.atomic_out = (nwin > 1 || pl->split > 1) ? 1 : 0;
    J.accumulate = job.accumulate;
    J.zero_first = (J.atomic_out && !job.accumulate && win.first) ? 1 : 0;
    pl->any_atomic |= J.atomic_out != 0;
    table.push_back(J);
  }
  return table;
}

// Rebuild the items and the device image for the current split.
bool build_items(xeng_plan* pl) {
  const std::vector<QueueJob> table = job_table(pl);
  uint8_t* image = nullptr;
  size_t bytes = 0;
  build_queue_image(table.data(), (int)table.size(), pl->split, &image, &bytes, &pl->items);
  if (image == nullptr) return false;
  pl->image.assign(image, image + bytes);
  std::free(image);
  return true;
}

// Write the job table (inputs, flags) into the image.
void write_jobs(xeng_plan* pl) {
  const std::vector<QueueJob> table = job_table(pl);
  std::memcpy(pl->image.data() + queue_jobs_offset(), table.data(),
              sizeof(QueueJob) * table.size());
}

xeng_status upload(xeng_plan* pl, void* d_ws, hipStream_t stream) {
  hipError_t e = hipMemcpyAsync(d_ws, pl->image.data(), pl->image.size(), hipMemcpyHostToDevice,
                                stream);
  return e == hipSuccess ? XENG_OK : device_error(e, "plan upload");
}

xeng_status launch(xeng_plan* pl, void* d_ws, hipStream_t stream) {
  if (pl->any_atomic) {
    queue_fill_kernel<<<dim3(64, (unsigned)pl->windows.size()), dim3(256), 0, stream>>>(
        reinterpret_cast<const uint8_t*>(d_ws));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return device_error(e, "plan zero fill");
  }
  hipError_t e = launch_queue(d_ws, pl->items, pl->grid, stream);
  return e == hipSuccess ? XENG_OK : device_error(e, "plan queue launch");
}

void drop_graph(xeng_plan* pl) {
  if (pl->graph_exec) (void)hipGraphExecDestroy(pl->graph_exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  pl->graph_exec = nullptr;
  pl->graph = nullptr;
  pl->graph_ws = nullptr;
}

std::string plan_key(const xeng_plan* pl) {
  std::ostringstream os;
  os << "plan";
  for (const auto& j : pl->jobs) os << ":" << j.n << "x" << j.f << "x" << j.t;
  return os.str();
}

}  // namespace
}  // namespace xeng

extern "C" {

xeng_status xeng_plan_create(xeng_plan** out, const xeng_job* jobs, int njobs,
                             const char* tune_cache_path) {
  using namespace xeng;
  if (out == nullptr || jobs == nullptr || njobs < 1)
    return fail(XENG_EINVAL, "need an output handle and at least one job");
  *out = nullptr;
  // one window per job: the queue kernel's sums are unscaled, so an item may
  // cover any sample count the int32 range guard admits
  const int64_t win = XENG_MAX_SAMPLES;
  auto pl = new (std::nothrow) xeng_plan();
  if (pl == nullptr) return fail(XENG_ENOMEM, "plan allocation failed");
  for (int k = 0; k < njobs; ++k) {
    const xeng_job& j = jobs[k];
    size_t ib = 0, vb = 0;
    xeng_status st = check_job(j.d_in, j.d_vis, j.n, j.f, j.t, j.t_prev, j.accumulate, &ib, &vb);
    if (st != XENG_OK) {
      delete pl;
      return fail(st, "job %d: %s", k, xeng_last_error());
    }
    if (j.n % 4 != 0 || (uintptr_t)j.d_in % 4 != 0 || (int64_t)j.n * 32 >= ((int64_t)1 << 31)) {
      delete pl;
      return fail(XENG_EINVAL,
                  "job %d: batched mode needs n %% 4 == 0, n < 2^26 and a 4-byte aligned input",
                  k);
    }
    pl->jobs.push_back(j);
    pl->held.push_back(j.t_prev + j.t);
    for (int64_t t0 = 0; t0 < j.t; t0 += win)
      pl->windows.push_back({k, (int)t0, (int)std::min<int64_t>(j.t, t0 + win), t0 == 0});
  }
  pl->grid = device_cu_count();
  // a tuned split for this set of job shapes, if the cache has one
  if (tune_cache_path != nullptr) {
    std::ifstream in(tune_cache_path);
    std::string key, line;
    const std::string want = plan_key(pl);
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      int split = 0;
      if (ls >> key >> split && key == want && split >= 1 && split <= kMaxSplit)
        pl->split = split;
    }
  }
  // size the workspace for the largest split the autotuner may choose
  const int chosen = pl->split;
  pl->split = kMaxSplit;
  bool ok = build_items(pl);
  pl->ws_bytes = pl->image.size();
  pl->split = chosen;
  ok = ok && build_items(pl);
  if (!ok) {
    delete pl;
    return fail(XENG_ENOMEM, "plan image allocation failed");
  }
  *out = pl;
  return XENG_OK;
}

size_t xeng_plan_workspace_bytes(const xeng_plan* plan) {
  return plan == nullptr ? 0 : plan->ws_bytes;
}

int64_t xeng_plan_items(const xeng_plan* plan) {
  return plan == nullptr ? -1 : plan->items;
}

int xeng_plan_split(const xeng_plan* plan) { return plan == nullptr ? -1 : plan->split; }

xeng_status xeng_plan_upload(xeng_plan* plan, void* d_workspace, void* hip_stream) {
  using namespace xeng;
  if (plan == nullptr || d_workspace == nullptr) return fail(XENG_EINVAL, "null plan or workspace");
  return upload(plan, d_workspace, reinterpret_cast<hipStream_t>(hip_stream));
}

xeng_status xeng_plan_set_frame(xeng_plan* plan, const uint8_t* const* d_in, int accumulate,
                                void* d_workspace, void* hip_stream) {
  using namespace xeng;
  if (plan == nullptr) return fail(XENG_EINVAL, "null plan");
  if (accumulate != 0 && accumulate != 1) return fail(XENG_EINVAL, "accumulate must be 0 or 1");
  for (size_t k = 0; k < plan->jobs.size(); ++k) {
    if (d_in != nullptr && (d_in[k] == nullptr || (uintptr_t)d_in[k] % 4 != 0))
      return fail(XENG_EINVAL, "job %zu: input must be non-null and 4-byte aligned", k);
    const xeng_job& j = plan->jobs[k];
    if (accumulate && plan->held[k] + j.t > XENG_MAX_SAMPLES)
      return fail(XENG_ERANGE, "job %zu: %lld samples would leave the exact int32 range", k,
                  (long long)(plan->held[k] + j.t));
  }
  for (size_t k = 0; k < plan->jobs.size(); ++k) {
    xeng_job& j = plan->jobs[k];
    // samples the sums hold once this frame has run
    plan->held[k] = accumulate ? plan->held[k] + j.t : j.t;
    j.t_prev = plan->held[k] - j.t;
    j.accumulate = accumulate;
    if (d_in != nullptr) j.d_in = d_in[k];
  }
  write_jobs(plan);
  if (d_workspace == nullptr) return XENG_OK;   // the plan's own copy only
  const size_t nj = queue_items_offset((int)plan->windows.size()) - queue_jobs_offset();
  hipError_t e = hipMemcpyAsync(static_cast<uint8_t*>(d_workspace) + queue_jobs_offset(),
                                plan->image.data() + queue_jobs_offset(), nj,
                                hipMemcpyHostToDevice, reinterpret_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? XENG_OK : device_error(e, "plan job table upload");
}

xeng_status xeng_plan_run(xeng_plan* plan, void* d_workspace, void* hip_stream) {
  using namespace xeng;
  if (plan == nullptr || d_workspace == nullptr) return fail(XENG_EINVAL, "null plan or workspace");
  return launch(plan, d_workspace, reinterpret_cast<hipStream_t>(hip_stream));
}

xeng_status xeng_plan_graph_capture(xeng_plan* plan, void* d_workspace) {
  using namespace xeng;
  if (plan == nullptr || d_workspace == nullptr) return fail(XENG_EINVAL, "null plan or workspace");
  drop_graph(plan);
  hipStream_t cap = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) return device_error(e, "capture stream");
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  xeng_status st = XENG_OK;
  if (e == hipSuccess) {
    st = launch(plan, d_workspace, cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (st == XENG_OK && e2 != hipSuccess) st = device_error(e2, "end capture");
    if (st == XENG_OK) {
      plan->graph = g;
      e2 = hipGraphInstantiate(&plan->graph_exec, g, nullptr, nullptr, 0);
      if (e2 != hipSuccess) st = device_error(e2, "graph instantiate");
      plan->graph_ws = d_workspace;
    } else if (g != nullptr) {
      (void)hipGraphDestroy(g);
    }
  } else {
    st = device_error(e, "begin capture");
  }
  (void)hipStreamDestroy(cap);
  if (st != XENG_OK) drop_graph(plan);
  return st;
}

xeng_status xeng_plan_graph_launch(xeng_plan* plan, void* hip_stream) {
  using namespace xeng;
  if (plan == nullptr || plan->graph_exec == nullptr)
    return fail(XENG_EINVAL, "plan has no captured graph");
  hipError_t e = hipGraphLaunch(plan->graph_exec, reinterpret_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? XENG_OK : device_error(e, "graph launch");
}

xeng_status xeng_plan_autotune(xeng_plan* plan, void* d_workspace, void* hip_stream, int reps,
                               const char* tune_cache_path, float* best_ms) {
  using namespace xeng;
  if (plan == nullptr || d_workspace == nullptr) return fail(XENG_EINVAL, "null plan or workspace");
  // Every candidate run writes the jobs' outputs. Timing them on jobs that
  // add into held sums would add the frame into those sums many times over.
  for (size_t k = 0; k < plan->jobs.size(); ++k)
    if (plan->jobs[k].accumulate)
      return fail(XENG_EINVAL,
                  "job %zu accumulates: autotune overwrites the outputs, so it needs a plan "
                  "whose jobs all overwrite (xeng_plan_set_frame with accumulate = 0)", k);
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (reps < 1) reps = 1;
  drop_graph(plan);
  const int candidates[] = {1, 2, 3, 4, 6, kMaxSplit};
  int best = plan->split;
  float best_t = -1.f;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(XENG_EDEVICE, "event creation failed");
  xeng_status st = XENG_OK;
  for (int cand : candidates) {
    plan->split = cand;
    if (!build_items(plan)) {
      st = fail(XENG_ENOMEM, "plan image allocation failed");
      break;
    }
    if ((st = upload(plan, d_workspace, stream)) != XENG_OK) break;
    if ((st = launch(plan, d_workspace, stream)) != XENG_OK) break;   // warm-up
    (void)hipEventRecord(e0, stream);
    for (int r = 0; r < reps && st == XENG_OK; ++r) st = launch(plan, d_workspace, stream);
    (void)hipEventRecord(e1, stream);
    if (st != XENG_OK) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      st = fail(XENG_EDEVICE, "event wait failed");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)reps;
    if (best_t < 0.f || ms < best_t) {
      best_t = ms;
      best = cand;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  plan->split = best;
  if (!build_items(plan) && st == XENG_OK) st = fail(XENG_ENOMEM, "plan image allocation failed");
  if (st == XENG_OK) st = upload(plan, d_workspace, stream);
  if (st == XENG_OK && tune_cache_path != nullptr) {
    std::ofstream outf(tune_cache_path, std::ios::app);
    outf << plan_key(plan) << " " << best << "\n";
  }
  if (best_ms != nullptr) *best_ms = best_t;
  return st;
}

void xeng_plan_destroy(xeng_plan* plan) {
  if (plan == nullptr) return;
  xeng::drop_graph(plan);
  delete plan;
}

}  // extern "C"

// ---- plan runs that allocate nothing ---------------------------------------------
// xeng_plan_run_static keeps the plan's device image (header, job table, piece
// queue) in one file-scope device array instead of a caller workspace. In host
// code the array's name is only a stand-in for the symbol; its device address
// comes from hipGetSymbolAddress, once per device with that device current, and
// only that address is ever handed to copies and kernels.
namespace xeng {
namespace {

__device__ __align__(256) uint8_t scratch[XENG_STATIC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// The current device's copy of scratch.
xeng_status static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_error(e, "static scratch: current device");
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(XENG_EDEVICE, "static scratch: device %d beyond the %d supported", dev,
                kMaxScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return device_error(e, "static scratch: symbol address");
    if (ptr == nullptr) return fail(XENG_EDEVICE, "static scratch: no device address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return XENG_OK;
}

}  // namespace
}  // namespace xeng

extern "C" xeng_status xeng_plan_run_static(xeng_plan* plan, void* hip_stream) {
  using namespace xeng;
  if (plan == nullptr) return fail(XENG_EINVAL, "null plan");
  if (plan->image.size() > (size_t)XENG_STATIC_SCRATCH_BYTES)
    return fail(XENG_EINVAL,
                "plan image of %zu bytes exceeds the static scratch of %lld bytes (%lld pieces "
                "queued); use xeng_plan_run with a workspace",
                plan->image.size(), (long long)XENG_STATIC_SCRATCH_BYTES, (long long)plan->items);
  void* ws = nullptr;
  xeng_status st = static_scratch(&ws);
  if (st != XENG_OK) return st;
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  // the whole image, header included: its queue cursors and counters start at
  // zero whatever an earlier call left in the array
  if ((st = upload(plan, ws, stream)) != XENG_OK) return st;
  return launch(plan, ws, stream);
}
