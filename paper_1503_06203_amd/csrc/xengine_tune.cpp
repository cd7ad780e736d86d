// xengine_tune.cpp -- the autotuner of plain correlation calls: for one job
// class it times every kernel variant that can run the job, with a few time
// splits each, and keeps the fastest. Choices live in a process-wide table
// that xeng_correlate and xeng_choose_variant consult, and in a cache file
// (one line per class) that a later process loads with xeng_tune_load.
//
// A class is (device architecture, n, f, floor(log2 t)): the kernels' cost
// depends on n and f through the tiling and on t only through how many rounds
// of the compute units the time axis fills, so one choice serves frames whose
// length is within a factor of two.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "xengine.h"
#include "xengine_internal.h"

namespace xeng {
namespace {

struct TuneKey {
  std::string arch;
  int n, f, tb;
  bool operator<(const TuneKey& o) const {
    return std::tie(arch, n, f, tb) < std::tie(o.arch, o.n, o.f, o.tb);
  }
};
struct TuneChoice {
  int variant, split;
  float ms;
};

std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tune;
std::atomic<int> g_tune_size{0};   // entries in g_tune: plain calls skip the lookup at 0

int t_bucket(int t) {
  int b = 0;
  while (b < 31 && ((int64_t)1 << (b + 1)) <= (int64_t)t) ++b;
  return b;
}

// The current device's architecture name without its feature suffix
// ("gfx950"); "none" when no device is usable. Queried once per device (the
// property query costs tens of microseconds).
std::string device_arch() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static std::string cache[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "none";
  std::lock_guard<std::mutex> lock(mu);
  if (dev >= 0 && dev < kMaxDevices && !cache[dev].empty()) return cache[dev];
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "none";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  if (colon != std::string::npos) a.resize(colon);
  if (a.empty()) a = "none";
  if (dev >= 0 && dev < kMaxDevices) cache[dev] = a;
  return a;
}

}  // namespace

bool tuned_choice(int n, int f, int t, int* variant, int* split) {
  if (t < 1 || g_tune_size.load(std::memory_order_relaxed) == 0) return false;
  const TuneKey key{device_arch(), n, f, t_bucket(t)};
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *variant = it->second.variant;
  *split = it->second.split;
  return true;
}

}  // namespace xeng

extern "C" {

xeng_status xeng_autotune(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t, int reps,
                          const char* tune_cache_path, int* variant, int* split_t,
                          float* best_ms, void* hip_stream) {
  using namespace xeng;
  size_t in_bytes = 0, vis_bytes = 0;
  xeng_status st = check_job(d_in, d_vis, n, f, t, 0, 0, &in_bytes, &vis_bytes);
  if (st != XENG_OK) return st;
  if (t < 1) return fail(XENG_EINVAL, "autotune needs t >= 1");
  if (reps < 1) reps = 1;
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  const int splits[] = {0, 1, 2, 4, 8};     // 0: the variant's own choice
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(XENG_EDEVICE, "event creation failed");
  }
  int best_v = -1, best_s = 0;
  float best_t = -1.f;
  st = XENG_OK;
  const int nv = xeng_variant_count();
  for (int v = 0; v < nv && st == XENG_OK; ++v) {
    for (int sp : splits) {
      if (v == variant_ids::kVariantSmall && sp != 0) continue;   // it takes no split
      // a variant that cannot run this job says so without enqueuing anything
      xeng_status s1 = xeng_correlate_variant(d_in, d_vis, n, f, t, 0, 0, v, sp, hip_stream);
      if (s1 == XENG_EINVAL || s1 == XENG_ENOTFOUND) break;
      if (s1 != XENG_OK) {
        st = s1;
        break;
      }
      (void)hipEventRecord(e0, stream);
      for (int r = 0; r < reps && st == XENG_OK; ++r)
        st = xeng_correlate_variant(d_in, d_vis, n, f, t, 0, 0, v, sp, hip_stream);
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
        best_v = v;
        best_s = sp;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != XENG_OK) return st;
  if (best_v < 0) return fail(XENG_EINVAL, "no kernel variant can run this job");
  const TuneKey key{device_arch(), n, f, t_bucket(t)};
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[key] = TuneChoice{best_v, best_s, best_t};
    g_tune_size.store((int)g_tune.size());
  }
  if (tune_cache_path != nullptr) {
    std::ofstream out(tune_cache_path, std::ios::app);
    if (!out) return fail(XENG_EINVAL, "cannot append to %s", tune_cache_path);
    out << "xeng-tune " << key.arch << " " << n << " " << f << " " << key.tb << " " << best_v
        << " " << best_s << " " << best_t << "\n";
  }
  if (variant) *variant = best_v;
  if (split_t) *split_t = best_s;
  if (best_ms) *best_ms = best_t;
  return XENG_OK;
}

xeng_status xeng_tune_load(const char* tune_cache_path, int* entries) {
  using namespace xeng;
  if (tune_cache_path == nullptr) return fail(XENG_EINVAL, "null path");
  std::ifstream in(tune_cache_path);
  if (!in) return fail(XENG_ENOTFOUND, "cannot read %s", tune_cache_path);
  const std::string arch = device_arch();
  int loaded = 0;
  std::string line;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string tag, a;
    TuneKey key;
    TuneChoice ch{};
    if (!(ls >> tag >> a >> key.n >> key.f >> key.tb >> ch.variant >> ch.split >> ch.ms)) continue;
    if (tag != "xeng-tune" || a != arch) continue;   // other devices' choices stay out
    if (key.n < 1 || key.f < 1 || key.tb < 0 || key.tb > 31) continue;
    if (ch.variant < 0 || ch.variant >= xeng_variant_count() || ch.split < 0 || ch.split > 64)
      continue;
    key.arch = a;
    g_tune[key] = ch;                                // later lines replace earlier ones
    ++loaded;
  }
  g_tune_size.store((int)g_tune.size());
  if (entries) *entries = loaded;
  return XENG_OK;
}

void xeng_tune_clear(void) {
  std::lock_guard<std::mutex> lock(xeng::g_tune_mu);
  xeng::g_tune.clear();
  xeng::g_tune_size.store(0);
}

}  // extern "C"
