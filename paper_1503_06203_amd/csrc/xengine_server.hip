// xengine_server.hip -- serving mode: a request loop that takes correlation
// frames as they arrive and runs them with continuous batching (the
// xeng_server / xeng_job / xeng_submit ABI).
//
// Each open job owns a device-resident int32 accumulator that frames add into
// (paper Sec. III-A: new sums are added to the results already held). Frames
// wait in a FIFO per job. A scheduling step first retires finished work, then,
// while a workspace slot is free, takes the oldest pending frames of every job
// that has nothing in flight (several of a job whose accumulator already holds
// sums, combined with int32 atomic adds), merges all their pieces into one
// queue image in that slot and launches the persistent queue kernel on the
// slot's stream. Frames that arrive while earlier steps run join the next
// step, and steps on different slots overlap on the device; a job is in at
// most one step at a time, so its accumulator is only ever updated by one
// launch at a time.
// Admission is by memory: a job's accumulator must fit the HBM budget when it
// is opened, and a frame is launched only while the bytes of frames in flight
// plus all accumulators stay within the budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "xcorr_launch.h"
#include "xengine.h"
#include "xengine_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

// Frames of one job that one step may hold.
constexpr size_t kMaxFramesPerJob = 16;

struct Frame {
  uint64_t ticket;
  const uint8_t* d_in;
  int t;
  double submit_us;
};

struct ServerJob {
  int n, f;
  int32_t* d_vis;
  size_t acc_bytes;
  int64_t held = 0;        // samples in the accumulator once queued frames run
  bool busy = false;       // a frame of this job is in flight
  bool summed = false;     // the accumulator holds sums (first frame overwrites)
  std::deque<Frame> pending;
};

struct TicketState {
  double submit_us = 0, done_us = 0;
  bool done = false;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr, end = nullptr;
  bool busy = false;
  std::vector<uint64_t> tickets;
  std::vector<int64_t> jobs;
  size_t frame_bytes = 0;
  std::vector<uint8_t> image;
  int64_t items = 0;               // items in the image
};

}  // namespace

struct xeng_server {
  size_t budget = 0;
  uint8_t* d_ws = nullptr;
  size_t slot_bytes = 0;
  hipStream_t caller = nullptr;
  hipEvent_t caller_ready = nullptr;
  hipEvent_t ref = nullptr;        // device time origin
  double ref_us = 0;               // host time of the origin
  std::vector<Slot> slots;
  std::map<int64_t, ServerJob> jobs;
  std::map<uint64_t, TicketState> tickets;
  int64_t next_job = 1;
  uint64_t next_ticket = 1;
  size_t acc_total = 0, inflight_bytes = 0;
  int grid = 256;
  size_t max_pending = 1 << 20;
};

namespace {

using xeng::device_error;
using xeng::fail;

double host_us() {
  return std::chrono::duration<double, std::micro>(Clock::now().time_since_epoch()).count();
}

// Retire slots whose launch has finished: completion time comes from the
// device event (relative to the reference event recorded at creation).
xeng_status retire(xeng_server* s) {
  for (auto& sl : s->slots) {
    if (!sl.busy) continue;
    hipError_t q = hipEventQuery(sl.end);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return device_error(q, "step completion");
    float ms = 0.f;
    double done_us = host_us();
    if (hipEventElapsedTime(&ms, s->ref, sl.end) == hipSuccess) done_us = s->ref_us + 1e3 * ms;
    for (uint64_t tk : sl.tickets) {
      auto it = s->tickets.find(tk);
      if (it != s->tickets.end()) {
        it->second.done = true;
        it->second.done_us = std::max(done_us, it->second.submit_us);
      }
    }
    for (int64_t jid : sl.jobs) {
      auto it = s->jobs.find(jid);
      if (it != s->jobs.end()) it->second.busy = false;
    }
    s->inflight_bytes -= sl.frame_bytes;
    sl.busy = false;
    sl.tickets.clear();
    sl.jobs.clear();
    sl.frame_bytes = 0;
  }
  return XENG_OK;
}

// Build the queue image for the chosen frames into slot.image; returns false
// if it would not fit the slot (or the host allocation failed). A job with
// several frames in the step adds each of them into its sums with int32
// atomic adds (any order gives the same integers); a job with one frame
// stores or adds it directly.
bool build_image(xeng_server* s, Slot& sl, const std::vector<std::pair<int64_t, Frame>>& picks) {
  using namespace xeng;
  const int stage = queue_stage_samples();
  const int nw = (int)picks.size();
  std::map<int64_t, int> frames_of;
  for (const auto& pk : picks) ++frames_of[pk.first];
  std::vector<QueueJob> table(nw);
  for (int w = 0; w < nw; ++w) {
    const ServerJob& J = s->jobs[picks[w].first];
    const Frame& fr = picks[w].second;
    QueueJob& q = table[w];
    q.in = fr.d_in;
    q.vis = J.d_vis;
    q.n = J.n;
    q.f = J.f;
    q.t = fr.t;
    q.ss = J.n;
    q.cs = (int64_t)fr.t * J.n;
    q.t0 = 0;
    q.t_end = fr.t;
    q.nbc = (J.n + 255) / 256;
    q.units = q.nbc * q.nbc;
    q.total_stages = (fr.t + stage - 1) / stage;
    q.accumulate = J.summed ? 1 : 0;
    q.atomic_out = frames_of[picks[w].first] > 1 ? 1 : 0;   // only for jobs already summed
    q.zero_first = 0;
  }
  uint8_t* image = nullptr;
  size_t bytes = 0;
  build_queue_image(table.data(), nw, 1, &image, &bytes, &sl.items);
  const bool fits = image != nullptr && bytes <= s->slot_bytes;
  if (fits) sl.image.assign(image, image + bytes);
  std::free(image);
  return fits;
}

}  // namespace

extern "C" {

xeng_status xeng_server_create(xeng_server** out, size_t hbm_budget, int max_inflight,
                               void* d_workspace, size_t ws_bytes, void* hip_stream) {
  if (out == nullptr) return fail(XENG_EINVAL, "null output handle");
  *out = nullptr;
  if (max_inflight < 1 || max_inflight > 8)
    return fail(XENG_EINVAL, "max_inflight must be in [1, 8]");
  if (d_workspace == nullptr || ws_bytes < (size_t)max_inflight * 4096)
    return fail(XENG_ENOMEM, "workspace must hold at least 4 KiB per in-flight step");
  auto s = new (std::nothrow) xeng_server();
  if (s == nullptr) return fail(XENG_ENOMEM, "server allocation failed");
  s->budget = hbm_budget;
  s->d_ws = static_cast<uint8_t*>(d_workspace);
  s->slot_bytes = ws_bytes / (size_t)max_inflight / 256 * 256;
  s->caller = reinterpret_cast<hipStream_t>(hip_stream);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      cus > 0)
    s->grid = cus;
  hipError_t e = hipEventCreate(&s->ref);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->caller_ready, hipEventDisableTiming);
  s->slots.resize(max_inflight);
  for (auto& sl : s->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&sl.start);
    if (e == hipSuccess) e = hipEventCreate(&sl.end);
  }
  if (e == hipSuccess) {
    // time origin: an event on the caller's stream, synchronised once
    e = hipEventRecord(s->ref, s->caller);
    if (e == hipSuccess) e = hipEventSynchronize(s->ref);
    s->ref_us = host_us();
  }
  if (e != hipSuccess) {
    xeng_server_destroy(s);
    return device_error(e, "server setup");
  }
  *out = s;
  return XENG_OK;
}

xeng_status xeng_job_open(xeng_server* s, int n, int f, int32_t* d_vis, int64_t* job_id) {
  if (s == nullptr || job_id == nullptr || d_vis == nullptr)
    return fail(XENG_EINVAL, "null server, output or accumulator");
  if (n < 4 || n % 4 != 0 || f < 1 || (int64_t)n * 32 >= ((int64_t)1 << 31))
    return fail(XENG_EINVAL, "served jobs need n %% 4 == 0 (n >= 4, n < 2^26) and f >= 1");
  if ((uintptr_t)d_vis % 8 != 0) return fail(XENG_EINVAL, "accumulator must be 8-byte aligned");
  const size_t acc = (size_t)f * ((size_t)n * (n + 1) / 2) * 8;
  if (s->acc_total + acc > s->budget)
    return fail(XENG_EBUSY, "accumulator of %zu bytes does not fit the HBM budget (%zu of %zu used)",
                acc, s->acc_total, s->budget);
  ServerJob J;
  J.n = n;
  J.f = f;
  J.d_vis = d_vis;
  J.acc_bytes = acc;
  const int64_t id = s->next_job++;
  s->jobs.emplace(id, std::move(J));
  s->acc_total += acc;
  *job_id = id;
  return XENG_OK;
}

xeng_status xeng_submit(xeng_server* s, int64_t job_id, const uint8_t* d_frame, int t,
                        uint64_t* ticket) {
  if (s == nullptr || ticket == nullptr) return fail(XENG_EINVAL, "null server or ticket");
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return fail(XENG_ENOTFOUND, "unknown job %lld", (long long)job_id);
  ServerJob& J = it->second;
  if (d_frame == nullptr || (uintptr_t)d_frame % 4 != 0 || t < 1)
    return fail(XENG_EINVAL, "frame must be non-null, 4-byte aligned, with t >= 1");
  if (J.held + t > XENG_MAX_SAMPLES)
    return fail(XENG_ERANGE, "job %lld would hold %lld samples, beyond the exact int32 range",
                (long long)job_id, (long long)(J.held + t));
  if (J.pending.size() >= s->max_pending) return fail(XENG_EBUSY, "job queue full");
  const uint64_t tk = s->next_ticket++;
  Frame fr{tk, d_frame, t, host_us()};
  J.pending.push_back(fr);
  J.held += t;
  s->tickets[tk].submit_us = fr.submit_us;
  *ticket = tk;
  return XENG_OK;
}

xeng_status xeng_server_step(xeng_server* s, int* launched) {
  if (s == nullptr) return fail(XENG_EINVAL, "null server");
  if (launched) *launched = 0;
  xeng_status st = retire(s);
  if (st != XENG_OK) return st;
  for (auto& sl : s->slots) {
    if (sl.busy) continue;
    // The pending frames of every idle job, oldest first, within the budget:
    // up to kMaxFramesPerJob of a job whose accumulator already holds sums
    // (they add with atomics), one for a job whose first frame overwrites.
    // A job's frames stay in order: a later frame is only taken after every
    // earlier one of the same job.
    std::vector<std::pair<int64_t, Frame>> picks;
    for (auto& kv : s->jobs) {
      const ServerJob& J = kv.second;
      if (J.busy) continue;
      const size_t take = J.summed ? std::min(J.pending.size(), kMaxFramesPerJob)
                                   : std::min<size_t>(J.pending.size(), 1);
      for (size_t k = 0; k < take; ++k) picks.emplace_back(kv.first, J.pending[k]);
    }
    if (picks.empty()) break;
    std::stable_sort(picks.begin(), picks.end(), [](const auto& a, const auto& b) {
      return a.second.submit_us < b.second.submit_us;
    });
    std::vector<std::pair<int64_t, Frame>> chosen;
    std::map<int64_t, size_t> skipped;
    size_t bytes = 0;
    for (const auto& pk : picks) {
      const ServerJob& J = s->jobs[pk.first];
      const size_t fb = (size_t)J.f * pk.second.t * J.n;
      if (skipped.count(pk.first) ||
          s->acc_total + s->inflight_bytes + bytes + fb > s->budget) {
        ++skipped[pk.first];     // this job's later frames wait as well
        continue;
      }
      chosen.push_back(pk);
      bytes += fb;
    }
    if (chosen.empty()) break;   // admission: wait for memory to free up
    // drop newest frames until the image fits the slot
    while (!chosen.empty() && !build_image(s, sl, chosen)) chosen.pop_back();
    if (chosen.empty()) return fail(XENG_ENOMEM, "workspace slot too small for one frame");
    // the frames were produced on the caller's stream: order after that work
    hipError_t e = hipEventRecord(s->caller_ready, s->caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(sl.stream, s->caller_ready, 0);
    uint8_t* ws = s->d_ws + (&sl - s->slots.data()) * s->slot_bytes;
    if (e == hipSuccess)
      e = hipMemcpyAsync(ws, sl.image.data(), sl.image.size(), hipMemcpyHostToDevice, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.start, sl.stream);
    if (e == hipSuccess) e = xeng::launch_queue(ws, sl.items, s->grid, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.end, sl.stream);
    if (e != hipSuccess) return device_error(e, "step launch");
    sl.busy = true;
    sl.frame_bytes = 0;
    for (const auto& pk : chosen) {
      ServerJob& J = s->jobs[pk.first];
      J.pending.pop_front();     // chosen frames are each job's oldest, in order
      J.busy = true;
      J.summed = true;
      sl.tickets.push_back(pk.second.ticket);
      sl.jobs.push_back(pk.first);
      sl.frame_bytes += (size_t)J.f * pk.second.t * J.n;
    }
    s->inflight_bytes += sl.frame_bytes;
    if (launched) *launched += (int)chosen.size();
  }
  return XENG_OK;
}

xeng_status xeng_poll(xeng_server* s, uint64_t ticket, int* done, double* latency_us) {
  if (s == nullptr || done == nullptr) return fail(XENG_EINVAL, "null server or output");
  xeng_status st = retire(s);
  if (st != XENG_OK) return st;
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(XENG_ENOTFOUND, "unknown ticket %llu",
                                          (unsigned long long)ticket);
  *done = it->second.done ? 1 : 0;
  if (latency_us) *latency_us = it->second.done ? it->second.done_us - it->second.submit_us : -1.0;
  return XENG_OK;
}

xeng_status xeng_server_drain(xeng_server* s) {
  if (s == nullptr) return fail(XENG_EINVAL, "null server");
  while (true) {
    int launched = 0;
    xeng_status st = xeng_server_step(s, &launched);
    if (st != XENG_OK) return st;
    bool any = false;
    for (auto& sl : s->slots)
      if (sl.busy) {
        any = true;
        hipError_t e = hipEventSynchronize(sl.end);
        if (e != hipSuccess) return device_error(e, "drain");
      }
    bool pending = false;
    for (auto& kv : s->jobs) pending |= !kv.second.pending.empty();
    if (!any && !pending) break;
    if (!any && pending && launched == 0)
      return fail(XENG_EBUSY, "pending frames do not fit the HBM budget");
  }
  return retire(s);
}

xeng_status xeng_job_close(xeng_server* s, int64_t job_id) {
  if (s == nullptr) return fail(XENG_EINVAL, "null server");
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return fail(XENG_ENOTFOUND, "unknown job %lld", (long long)job_id);
  if (it->second.busy || !it->second.pending.empty())
    return fail(XENG_EBUSY, "job %lld still has frames queued or in flight", (long long)job_id);
  s->acc_total -= it->second.acc_bytes;
  s->jobs.erase(it);
  return XENG_OK;
}

xeng_status xeng_server_stats(xeng_server* s, int64_t* open_jobs, int64_t* pending_frames,
                              int64_t* inflight_steps, size_t* bytes_in_use) {
  if (s == nullptr) return fail(XENG_EINVAL, "null server");
  int64_t pend = 0, fl = 0;
  for (auto& kv : s->jobs) pend += (int64_t)kv.second.pending.size();
  for (auto& sl : s->slots) fl += sl.busy ? 1 : 0;
  if (open_jobs) *open_jobs = (int64_t)s->jobs.size();
  if (pending_frames) *pending_frames = pend;
  if (inflight_steps) *inflight_steps = fl;
  if (bytes_in_use) *bytes_in_use = s->acc_total + s->inflight_bytes;
  return XENG_OK;
}

void xeng_server_destroy(xeng_server* s) {
  if (s == nullptr) return;
  for (auto& sl : s->slots) {
    if (sl.end) (void)hipEventSynchronize(sl.end);
    if (sl.start) (void)hipEventDestroy(sl.start);
    if (sl.end) (void)hipEventDestroy(sl.end);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  if (s->ref) (void)hipEventDestroy(s->ref);
  if (s->caller_ready) (void)hipEventDestroy(s->caller_ready);
  delete s;
}

}  // extern "C"
