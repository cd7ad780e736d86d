// xengine.cpp -- the C ABI declared in include/xengine.h: argument checks,
// error reporting and dispatch to the gfx950 kernels.
#include "xengine.h"

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "xcorr_launch.h"
#include "xengine_internal.h"

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace xeng {

xeng_status fail(xeng_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

xeng_status device_error(hipError_t err, const char* what) {
  return fail(XENG_EDEVICE, "%s: %s", what, hipGetErrorString(err));
}

int device_cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 256;
  return cus > 0 ? cus : 256;
}

int auto_split(int64_t units, int64_t stages, int cus) {
  // Cost model in stage times: rounds of workgroups x (stages per workgroup +
  // a fixed cost for the prologue and the output writes, larger when the
  // time axis is split: atomic adds and the zero fill). A split keeps at
  // least 16 stages per workgroup.
  if (cus < 1) cus = 1;
  int best = 1;
  double best_cost = 0.0;
  for (int split = 1; split <= 64; ++split) {
    if (split > 1 && stages / split < 16) break;
    const int64_t wgs = units * split;
    const int64_t rounds = (wgs + cus - 1) / cus;
    const double per_wg = (double)((stages + split - 1) / split) + (split > 1 ? 8.0 : 4.0);
    const double cost = (double)rounds * per_wg;
    if (split == 1 || cost < best_cost * 0.97) {
      best = split;
      best_cost = cost;
    }
  }
  return best;
}

int tri_auto_split(int f, int64_t t_count, int cus) {
  const int64_t stage = tri_stage_samples();
  return auto_split(f, (t_count + stage - 1) / stage, cus);
}

int rect_auto_split(int n, int f, int64_t t_count, int cus) {
  const int64_t stage = tri_stage_samples();
  return auto_split(rect_units_per_channel(n) * f, (t_count + stage - 1) / stage, cus);
}

}  // namespace xeng

namespace {
using xeng::check_job;
using xeng::device_error;
using xeng::fail;

struct Variant {
  const char* name;
};

// Index = variant id.
const Variant kVariants[] = {
    {"tile128_kc64_mfma32x32x32"},        // any n, any input alignment
    {"retired_wide128x256_w4"},           // superseded by 5; refused
    {"retired_wide128x256_w8"},           // superseded by 5; refused
    {"tri256_w8_kc64_mfma32x32x32"},      // n <= 256, n % 4 == 0, 4-byte aligned input
    {"tri256_w8_bf6_mfma32x32x64"},       // as above, on bf6 operands (exact)
    {"rect128x256_tri256_w8_kc64_mfma32x32x32"},  // n % 4 == 0, 4-byte aligned input
    {"small64_w8_ring16_mfma32x32x32"},   // n <= 64, n % 4 == 0, 4-byte aligned input
    {"rect128x256_tri256_w8_bf6_mfma32x32x64"},  // as 5, on bf6 operands (exact)
};
using namespace xeng::variant_ids;
constexpr int kVariantCount = sizeof(kVariants) / sizeof(kVariants[0]);
static_assert(kVariantCount == kVariantRectBf6 + 1, "one table entry per variant id");

// The kernel xeng_correlate uses: the triangle kernel where it applies (it
// wastes the least MFMA work on small arrays), else the kernel of diagonal
// squares and off-diagonal tiles for dword-loadable inputs, else the general
// one.
int default_variant(int n, bool aligned) {
  if (aligned && n <= xeng::small_max_elements()) return kVariantSmall;
  if (aligned && n <= xeng::tri_max_elements()) return kVariantTri;
  return aligned ? kVariantRect : kVariantTile128;
}

// Whether a variant can run a job (the rules correlate_impl enforces).
bool variant_fits(int v, int n, bool aligned, bool dense) {
  switch (v) {
    case kVariantTile128: return dense;
    case kVariantRect:
    case kVariantRectBf6: return aligned;
    case kVariantTri:
    case kVariantTriBf6: return aligned && n <= xeng::tri_max_elements();
    case kVariantSmall: return aligned && n <= xeng::small_max_elements();
    default: return false;
  }
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return na && nb && a0 < b0 + nb && b0 < a0 + na;
}

}  // namespace

namespace xeng {
// Shared validation of one correlation job; fills byte counts on success.
xeng_status check_job(const uint8_t* d_in, const int32_t* d_vis, int n, int f, int t,
                      int64_t t_prev, int accumulate, size_t* in_bytes, size_t* vis_bytes,
                      int64_t ss, int64_t cs) {
  if (n < 1 || f < 1 || t < 0)
    return fail(XENG_EINVAL, "need n >= 1, f >= 1, t >= 0 (got n=%d f=%d t=%d)", n, f, t);
  if (accumulate != 0 && accumulate != 1)
    return fail(XENG_EINVAL, "accumulate must be 0 or 1 (got %d)", accumulate);
  if (t_prev < 0 || (!accumulate && t_prev != 0))
    return fail(XENG_EINVAL, "t_prev must be >= 0, and 0 when not accumulating (got %lld)",
                (long long)t_prev);
  if (t_prev + (int64_t)t > XENG_MAX_SAMPLES)
    return fail(XENG_ERANGE, "t_prev + t = %lld exceeds %lld samples: int32 sums could overflow",
                (long long)(t_prev + t), (long long)XENG_MAX_SAMPLES);
  // bytes the input spans: dense [F][T][N], or the strided extent
  unsigned __int128 ib = (unsigned __int128)f * (unsigned)t * (unsigned)n;
  if (ss > 0 && t > 0)
    ib = (unsigned __int128)(t - 1) * (uint64_t)ss + (unsigned __int128)(f - 1) * (uint64_t)cs +
         (unsigned)n;
  const unsigned __int128 entries = (unsigned __int128)n * (n + 1) / 2;
  const unsigned __int128 vb = entries * (unsigned)f * 8u;
  if (ib > ((unsigned __int128)1 << 62) || vb > ((unsigned __int128)1 << 62))
    return fail(XENG_EINVAL, "problem size overflows the address space");
  if (d_vis == nullptr) return fail(XENG_EINVAL, "d_vis is NULL");
  if (t > 0 && d_in == nullptr) return fail(XENG_EINVAL, "d_in is NULL");
  if (((uintptr_t)d_vis) % 8 != 0) return fail(XENG_EINVAL, "d_vis must be 8-byte aligned");
  *in_bytes = (size_t)ib;
  *vis_bytes = (size_t)vb;
  if (t > 0 && ranges_overlap(d_in, *in_bytes, d_vis, *vis_bytes))
    return fail(XENG_EINVAL, "d_in and d_vis overlap");
  return XENG_OK;
}
}  // namespace xeng

extern "C" {

const char* xeng_last_error(void) { return g_last_error.c_str(); }

const char* xeng_version(void) { return "xengine-gfx950 0.1.0"; }

int64_t xeng_vis_entries(int n) { return n < 0 ? -1 : (int64_t)n * (n + 1) / 2; }

int64_t xeng_tri_index(int n, int i, int j) {
  if (n < 1 || i < 0 || j < i || j >= n) return -1;
  return (int64_t)i * (2 * (int64_t)n - i + 1) / 2 + (j - i);
}

int64_t xeng_tile_count(int n, int tile) {
  if (n < 1 || tile < 1) return -1;
  const int64_t nb = ((int64_t)n + tile - 1) / tile;
  return nb * (nb + 1) / 2;
}

int xeng_variant_count(void) { return kVariantCount; }

const char* xeng_variant_name(int variant) {
  return (variant >= 0 && variant < kVariantCount) ? kVariants[variant].name : nullptr;
}

namespace {

// Shared by the dense and strided entry points. ss, cs: bytes from one sample
// to the next and from one channel to the next (dense: n and t * n).
xeng_status correlate_impl(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t, int64_t ss,
                           int64_t cs, int64_t t_prev, int accumulate, int variant, int split_t,
                           void* hip_stream) {
  const bool dense = ss == (int64_t)n && cs == (int64_t)t * n;
  if (!dense) {
    if (ss < n || cs < 0 || ss % 4 != 0 || cs % 4 != 0 || n % 4 != 0 ||
        (uintptr_t)d_in % 4 != 0)
      return fail(XENG_EINVAL,
                  "strided input needs n %% 4 == 0, a 4-byte aligned base and strides that are "
                  "multiples of 4 with sample stride >= n (got n=%d, strides %lld, %lld)",
                  n, (long long)ss, (long long)cs);
    if (ss > (((int64_t)1 << 31) - n) / 32)
      return fail(XENG_EINVAL, "sample stride %lld too large (limit %lld bytes)", (long long)ss,
                  (long long)((((int64_t)1 << 31) - n) / 32));
  }
  size_t in_bytes = 0, vis_bytes = 0;
  xeng_status st = check_job(d_in, d_vis, n, f, t, t_prev, accumulate, &in_bytes, &vis_bytes,
                             dense ? 0 : ss, dense ? 0 : cs);
  if (st != XENG_OK) return st;
  if (variant < -1 || variant >= kVariantCount)
    return fail(XENG_ENOTFOUND, "unknown kernel variant %d", variant);
  if (split_t < 0) return fail(XENG_EINVAL, "split_t must be >= 0 (0 = choose)");
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  const int64_t pairs = (int64_t)(vis_bytes / 8);
  if (t == 0) {
    if (accumulate) return XENG_OK;
    hipError_t e = xeng::launch_fill_zero(d_vis, pairs, stream);
    return e == hipSuccess ? XENG_OK : device_error(e, "zero fill");
  }
  const bool aligned = (n % 4 == 0) && ((uintptr_t)d_in % 4 == 0);
  const bool tri_ok = aligned && n <= xeng::tri_max_elements();
  if (variant == -1 && split_t == 0) {
    // a choice the autotuner made for this job class, where it can run
    int tv = -1, ts = 0;
    if (xeng::tuned_choice(n, f, t, &tv, &ts) && variant_fits(tv, n, aligned, dense)) {
      variant = tv;
      split_t = ts;
    }
  }
  if (variant == -1) variant = default_variant(n, aligned);
  if (!dense && variant == kVariantTile128)
    return fail(XENG_EINVAL, "variant %s reads the dense [F][T][N] layout only",
                kVariants[variant].name);
  if (variant == kVariantRetired1 || variant == kVariantRetired2)
    return fail(XENG_ENOTFOUND, "variant %d (%s) is retired; variant %d covers its jobs", variant,
                kVariants[variant].name, kVariantRect);
  const bool rect = variant == kVariantRect || variant == kVariantRectBf6;
  if (rect && !aligned)
    return fail(XENG_EINVAL, "variant %s needs n %% 4 == 0 and a 4-byte aligned input",
                kVariants[variant].name);
  const bool small = variant == kVariantSmall;
  if (small && !(aligned && n <= xeng::small_max_elements()))
    return fail(XENG_EINVAL, "variant %s needs n <= %d, n %% 4 == 0 and a 4-byte aligned input",
                kVariants[variant].name, xeng::small_max_elements());
  const bool tri = variant == kVariantTri || variant == kVariantTriBf6;
  if (tri && !tri_ok)
    return fail(XENG_EINVAL, "variant %s needs n <= %d, n %% 4 == 0 and a 4-byte aligned input",
                kVariants[variant].name, xeng::tri_max_elements());
  int split = split_t > 0 ? split_t : 1;
  if (tri && split_t == 0) split = xeng::tri_auto_split(f, t, xeng::device_cu_count());
  if (rect && split_t == 0) split = xeng::rect_auto_split(n, f, t, xeng::device_cu_count());
  // the bf6 kernels' fp32 sums are exact up to a bounded number of samples per part
  if (variant == kVariantTriBf6 || variant == kVariantRectBf6)
    split = std::max(split, xeng::tri_bf6_min_split(t));
  // the small kernel combines its time parts itself: no split, no fill
  if (small) split = 1;
  if (split > 1 && !accumulate) {
    hipError_t e = xeng::launch_fill_zero(d_vis, pairs, stream);
    if (e != hipSuccess) return device_error(e, "zero fill");
  }
  hipError_t e = hipSuccess;
  if (small) {
    e = xeng::launch_small(d_in, d_vis, n, f, t, ss, cs, 0, t, accumulate,
                           xeng::device_cu_count(), stream);
  } else if (variant == kVariantTri) {
    e = xeng::launch_tri(d_in, d_vis, n, f, t, ss, cs, 0, t, accumulate, split, stream);
  } else if (variant == kVariantRectBf6) {
    e = xeng::launch_rect_bf6(d_in, d_vis, n, f, t, ss, cs, 0, t, accumulate, split, stream);
  } else if (rect) {
    e = xeng::launch_rect(d_in, d_vis, n, f, t, ss, cs, 0, t, accumulate, split, stream);
  } else if (variant == kVariantTriBf6) {
    e = xeng::launch_tri_bf6(d_in, d_vis, n, f, t, ss, cs, 0, t, accumulate, split, stream);
  } else {
    e = xeng::launch_tile128(d_in, d_vis, n, f, t, accumulate, split, aligned, stream);
  }
  if (e != hipSuccess) return device_error(e, "correlation kernel launch");
  return XENG_OK;
}

}  // namespace

xeng_status xeng_correlate_variant(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t,
                                   int64_t t_prev, int accumulate, int variant, int split_t,
                                   void* hip_stream) {
  return correlate_impl(d_in, d_vis, n, f, t, n, (int64_t)t * n, t_prev, accumulate, variant,
                        split_t, hip_stream);
}

xeng_status xeng_correlate_strided(const uint8_t* d_in, int64_t sample_stride,
                                   int64_t channel_stride, int32_t* d_vis, int n, int f, int t,
                                   int64_t t_prev, int accumulate, void* hip_stream) {
  return correlate_impl(d_in, d_vis, n, f, t, sample_stride, channel_stride, t_prev, accumulate,
                        -1, 0, hip_stream);
}

xeng_status xeng_correlate_gated(const uint8_t* d_in, int32_t* d_vis, int gates, int n, int f,
                                 int t, int block, const uint8_t* gate_of_block,
                                 const int64_t* t_prev, int accumulate, void* hip_stream) {
  if (gates < 1 || gates > 255) return fail(XENG_EINVAL, "gates must be in [1, 255] (got %d)", gates);
  if (block < 1) return fail(XENG_EINVAL, "block must be >= 1 (got %d)", block);
  if (n % 4 != 0 || (uintptr_t)d_in % 4 != 0)
    return fail(XENG_EINVAL, "gated correlation needs n %% 4 == 0 and a 4-byte aligned input");
  if (accumulate != 0 && accumulate != 1)
    return fail(XENG_EINVAL, "accumulate must be 0 or 1 (got %d)", accumulate);
  if (accumulate && t_prev == nullptr) return fail(XENG_EINVAL, "t_prev is NULL");
  const int64_t nblocks = t > 0 ? ((int64_t)t + block - 1) / block : 0;
  if (nblocks > 0 && gate_of_block == nullptr) return fail(XENG_EINVAL, "gate_of_block is NULL");
  // per-gate sample counts and the range guard
  std::vector<int64_t> count(gates, 0);
  for (int64_t k = 0; k < nblocks; ++k) {
    const int g = gate_of_block[k];
    if (g == 0xFF) continue;
    if (g >= gates)
      return fail(XENG_EINVAL, "block %lld names gate %d of %d", (long long)k, g, gates);
    count[g] += std::min<int64_t>(block, t - k * (int64_t)block);
  }
  for (int g = 0; g < gates; ++g) {
    const int64_t prev = accumulate ? t_prev[g] : 0;
    if (prev < 0) return fail(XENG_EINVAL, "t_prev[%d] < 0", g);
    if (prev + count[g] > XENG_MAX_SAMPLES)
      return fail(XENG_ERANGE, "gate %d would hold %lld samples: int32 sums could overflow", g,
                  (long long)(prev + count[g]));
  }
  // validate the whole job once (shapes, pointers, overlap of input and all gate sets)
  size_t in_bytes = 0, vis_bytes = 0;
  xeng_status st = check_job(d_in, d_vis, n, f, t, 0, 0, &in_bytes, &vis_bytes);
  if (st != XENG_OK) return st;
  const int64_t set_pairs = (int64_t)(vis_bytes / 8);           // (re, im) pairs of one gate
  if ((unsigned __int128)vis_bytes * (unsigned)gates > ((unsigned __int128)1 << 62))
    return fail(XENG_EINVAL, "problem size overflows the address space");
  if (t > 0) {
    const uintptr_t a0 = (uintptr_t)d_in, b0 = (uintptr_t)d_vis;
    const uintptr_t b1 = b0 + vis_bytes * (size_t)gates;
    if (a0 < b1 && b0 < a0 + in_bytes) return fail(XENG_EINVAL, "d_in and d_vis overlap");
  }
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  std::vector<int64_t> held(gates, 0);                           // samples summed in this call
  if (t > 0) {
    // All runs of one gate in one launch (up to tri_max_segments() runs each):
    // the triangle kernel for n <= 256, else the kernel of diagonal squares and
    // tiles, so a gate's accumulators are read and written once per launch
    // instead of once per run.
    const bool tri = n <= xeng::tri_max_elements();
    std::vector<std::vector<int32_t>> run_t0(gates), run_t1(gates);
    for (int64_t k = 0; k < nblocks;) {
      const int g = gate_of_block[k];
      int64_t e = k + 1;
      while (e < nblocks && gate_of_block[e] == g) ++e;
      if (g != 0xFF) {
        run_t0[g].push_back((int32_t)(k * (int64_t)block));
        run_t1[g].push_back((int32_t)std::min<int64_t>((int64_t)t, e * (int64_t)block));
      }
      k = e;
    }
    const int max_seg = xeng::tri_max_segments();
    for (int g = 0; g < gates; ++g) {
      int32_t* vis_g = d_vis + (int64_t)g * set_pairs * 2;
      for (size_t c = 0; c < run_t0[g].size(); c += (size_t)max_seg) {
        const int cnt = (int)std::min<size_t>((size_t)max_seg, run_t0[g].size() - c);
        int64_t samples = 0;
        for (int r = 0; r < cnt; ++r) samples += run_t1[g][c + r] - run_t0[g][c + r];
        const bool first = !accumulate && held[g] == 0;
        const int cus = xeng::device_cu_count();
        const int split = tri ? xeng::tri_auto_split(f, samples, cus)
                              : xeng::rect_auto_split(n, f, samples, cus);
        if (first && split > 1) {
          hipError_t e = xeng::launch_fill_zero(vis_g, set_pairs, stream);
          if (e != hipSuccess) return device_error(e, "zero fill");
        }
        hipError_t e =
            tri ? xeng::launch_tri_segments(d_in, vis_g, n, f, t, n, (int64_t)t * n,
                                            run_t0[g].data() + c, run_t1[g].data() + c, cnt,
                                            first ? 0 : 1, split, stream)
                : xeng::launch_rect_segments(d_in, vis_g, n, f, t, n, (int64_t)t * n,
                                             run_t0[g].data() + c, run_t1[g].data() + c, cnt,
                                             first ? 0 : 1, split, stream);
        if (e != hipSuccess) return device_error(e, "gated correlation launch");
        held[g] += samples;
      }
    }
  }
  if (!accumulate) {
    // gates that received no samples are zero
    for (int g = 0; g < gates; ++g) {
      if (held[g] != 0) continue;
      hipError_t e = xeng::launch_fill_zero(d_vis + (int64_t)g * set_pairs * 2, set_pairs, stream);
      if (e != hipSuccess) return device_error(e, "zero fill");
    }
  }
  return XENG_OK;
}

}  // extern "C"

namespace {

// Checks shared by both delay entry points: delays, the input extent
// (t + max_delay samples per channel) and the int32 range.
xeng_status check_delayed(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t,
                          const int32_t* delays, int max_delay, int64_t t_prev, int accumulate,
                          size_t* in_bytes, size_t* vis_bytes) {
  if (n < 1) return fail(XENG_EINVAL, "need n >= 1 (got %d)", n);
  if (max_delay < 0 || max_delay > 65535)
    return fail(XENG_EINVAL, "max_delay must be in [0, 65535] (got %d)", max_delay);
  if (t < 0) return fail(XENG_EINVAL, "need t >= 0 (got %d)", t);
  if (delays == nullptr) return fail(XENG_EINVAL, "delays is NULL");
  for (int e = 0; e < n; ++e)
    if (delays[e] < 0 || delays[e] > max_delay)
      return fail(XENG_EINVAL, "delay of element %d is %d, outside [0, %d]", e, delays[e],
                  max_delay);
  if ((int64_t)t + max_delay > 0x7fffffff)
    return fail(XENG_EINVAL, "t + max_delay exceeds 2^31 - 1 samples");
  xeng_status st = check_job(d_in, d_vis, n, f, t + max_delay, t_prev, accumulate, in_bytes,
                             vis_bytes);
  if (st != XENG_OK) return st;
  if (t_prev + (int64_t)t > XENG_MAX_SAMPLES)
    return fail(XENG_ERANGE, "t_prev + t = %lld exceeds %lld samples", (long long)(t_prev + t),
                (long long)XENG_MAX_SAMPLES);
  return XENG_OK;
}

// The triangle kernel's fused forms: delays applied while staging (n <= 256,
// t % 64 == 0, t > 0).
bool delayed_fused_ok(int n, int t) {
  return n <= xeng::tri_max_elements() && t > 0 && t % xeng::tri_stage_samples() == 0;
}

xeng_status delayed_fused(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t,
                          const int32_t* delays, int max_delay, int accumulate, int64_t pairs,
                          hipStream_t stream) {
  const int split = xeng::tri_auto_split(f, t, xeng::device_cu_count());
  if (split > 1 && !accumulate) {
    hipError_t e = xeng::launch_fill_zero(d_vis, pairs, stream);
    if (e != hipSuccess) return device_error(e, "zero fill");
  }
  hipError_t e = xeng::launch_tri_delayed(d_in, d_vis, n, f, t, delays, max_delay, accumulate,
                                          split, stream);
  return e == hipSuccess ? XENG_OK : device_error(e, "delay-compensated correlation launch");
}

}  // namespace

extern "C" {

xeng_status xeng_correlate_delayed(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t,
                                   const int32_t* delays, int max_delay, int64_t t_prev,
                                   int accumulate, void* hip_stream) {
  if (n < 1 || n > xeng::tri_max_elements())
    return fail(XENG_EINVAL,
                "delay compensation without a workspace supports 1 <= n <= %d (got %d); "
                "xeng_correlate_delayed_ws takes any n",
                xeng::tri_max_elements(), n);
  if (t % xeng::tri_stage_samples() != 0)
    return fail(XENG_EINVAL,
                "delay compensation without a workspace needs t %% %d == 0 (got t=%d); "
                "xeng_correlate_delayed_ws takes any t",
                xeng::tri_stage_samples(), t);
  size_t in_bytes = 0, vis_bytes = 0;
  xeng_status st = check_delayed(d_in, d_vis, n, f, t, delays, max_delay, t_prev, accumulate,
                                 &in_bytes, &vis_bytes);
  if (st != XENG_OK) return st;
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  const int64_t pairs = (int64_t)(vis_bytes / 8);
  if (t == 0) {
    if (accumulate) return XENG_OK;
    hipError_t e = xeng::launch_fill_zero(d_vis, pairs, stream);
    return e == hipSuccess ? XENG_OK : device_error(e, "zero fill");
  }
  return delayed_fused(d_in, d_vis, n, f, t, delays, max_delay, accumulate, pairs, stream);
}

size_t xeng_delayed_workspace_bytes(int n, int f, int t) {
  if (n < 1 || f < 1 || t < 0) return 0;
  if (t == 0 || delayed_fused_ok(n, t)) return 0;
  return (size_t)f * (size_t)t * (size_t)n;
}

xeng_status xeng_correlate_delayed_ws(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t,
                                      const int32_t* delays, int max_delay, int64_t t_prev,
                                      int accumulate, void* d_workspace, size_t ws_bytes,
                                      void* hip_stream) {
  size_t in_bytes = 0, vis_bytes = 0;
  xeng_status st = check_delayed(d_in, d_vis, n, f, t, delays, max_delay, t_prev, accumulate,
                                 &in_bytes, &vis_bytes);
  if (st != XENG_OK) return st;
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  const int64_t pairs = (int64_t)(vis_bytes / 8);
  if (t == 0) {
    if (accumulate) return XENG_OK;
    hipError_t e = xeng::launch_fill_zero(d_vis, pairs, stream);
    return e == hipSuccess ? XENG_OK : device_error(e, "zero fill");
  }
  if (delayed_fused_ok(n, t))
    return delayed_fused(d_in, d_vis, n, f, t, delays, max_delay, accumulate, pairs, stream);
  // One delay common to all elements shifts every stream alike: the plain
  // correlation of a sample window, read in place (dword-loadable input).
  const bool common = std::all_of(delays, delays + n, [&](int32_t d) { return d == delays[0]; });
  if (common && n % 4 == 0 && (uintptr_t)d_in % 4 == 0)
    return correlate_impl(d_in + (int64_t)(max_delay - delays[0]) * n, d_vis, n, f, t, n,
                          (int64_t)(t + max_delay) * n, t_prev, accumulate, -1, 0, hip_stream);
  // Shift, then correlate: windows of `chunk` frame samples are written
  // delay-aligned into the workspace and correlated like plain frames, each
  // window after the first adding to the sums.
  const int64_t row = (int64_t)f * n;                 // workspace bytes per frame sample
  const int64_t min_rows = std::min<int64_t>(t, xeng::shift_tile_rows());
  if (d_workspace == nullptr || (int64_t)ws_bytes < min_rows * row)
    return fail(XENG_EINVAL,
                "workspace of %zu bytes is too small: at least %lld bytes (%lld frame samples); "
                "%zu bytes run in one pass",
                ws_bytes, (long long)(min_rows * row), (long long)min_rows,
                xeng_delayed_workspace_bytes(n, f, t));
  int64_t chunk = std::min<int64_t>(t, (int64_t)ws_bytes / row);
  if (chunk < t) chunk = chunk / xeng::shift_tile_rows() * xeng::shift_tile_rows();
  uint8_t* buf = static_cast<uint8_t*>(d_workspace);
  const size_t buf_bytes = (size_t)(chunk * row);
  if (ranges_overlap(buf, buf_bytes, d_in, in_bytes) ||
      ranges_overlap(buf, buf_bytes, d_vis, vis_bytes))
    return fail(XENG_EINVAL, "the workspace overlaps d_in or d_vis");
  for (int64_t t0 = 0; t0 < t; t0 += chunk) {
    const int tc = (int)std::min<int64_t>(chunk, t - t0);
    for (int e0 = 0; e0 < n; e0 += xeng::kShiftGroupElems) {
      const int cnt = std::min(xeng::kShiftGroupElems, n - e0);
      hipError_t e = xeng::launch_shift(d_in, buf, n, f, t + max_delay, max_delay, (int)t0, tc,
                                        e0, cnt, delays, stream);
      if (e != hipSuccess) return device_error(e, "delay shift launch");
    }
    const int acc = (accumulate || t0 > 0) ? 1 : 0;
    const int64_t prev = acc ? (accumulate ? t_prev : 0) + t0 : 0;
    st = correlate_impl(buf, d_vis, n, f, tc, n, (int64_t)tc * n, prev, acc, -1, 0, hip_stream);
    if (st != XENG_OK) return st;
  }
  return XENG_OK;
}

xeng_status xeng_choose_variant(int n, int f, int t, int input_aligned, int* variant,
                                int* split_t) {
  if (n < 1 || f < 1 || t < 0)
    return fail(XENG_EINVAL, "need n >= 1, f >= 1, t >= 0 (got n=%d f=%d t=%d)", n, f, t);
  if (variant == nullptr || split_t == nullptr) return fail(XENG_EINVAL, "NULL output pointer");
  const bool aligned = input_aligned != 0 && n % 4 == 0;
  // the autotuner's choice for this class where it can run, else the default
  int v = default_variant(n, aligned), tv = -1, ts = 0;
  if (xeng::tuned_choice(n, f, t, &tv, &ts) && variant_fits(tv, n, aligned, true))
    v = tv;
  else
    ts = 0;
  // the split correlate_impl then uses (ts = 0: the variant's own choice)
  const int cus = xeng::device_cu_count();
  int split = 1;
  if (t > 0 && (v == kVariantTri || v == kVariantTriBf6)) split = xeng::tri_auto_split(f, t, cus);
  if (t > 0 && (v == kVariantRect || v == kVariantRectBf6))
    split = xeng::rect_auto_split(n, f, t, cus);
  if (ts > 0) split = ts;
  if ((v == kVariantTriBf6 || v == kVariantRectBf6) && t > 0)
    split = std::max(split, xeng::tri_bf6_min_split(t));
  if (v == kVariantSmall) split = 1;
  *variant = v;
  *split_t = split;
  return XENG_OK;
}

xeng_status xeng_correlate(const uint8_t* d_in, int32_t* d_vis, int n, int f, int t,
                           int64_t t_prev, int accumulate, void* hip_stream) {
  return xeng_correlate_variant(d_in, d_vis, n, f, t, t_prev, accumulate, -1, 0, hip_stream);
}

}  // extern "C"
