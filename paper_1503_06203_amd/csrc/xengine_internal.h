// xengine_internal.h -- error reporting and argument checks shared by the
// C ABI translation units (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "xengine.h"

namespace xeng {

// Kernel variant ids, as xeng_correlate_variant takes them (the order of the
// name table in xengine.cpp).
namespace variant_ids {
constexpr int kVariantTile128 = 0;
constexpr int kVariantRetired1 = 1;   // 128 x 256 tiles, 4 waves: refused
constexpr int kVariantRetired2 = 2;   // 128 x 256 tiles, 8 waves: refused
constexpr int kVariantTri = 3;
constexpr int kVariantTriBf6 = 4;
constexpr int kVariantRect = 5;
constexpr int kVariantSmall = 6;
constexpr int kVariantRectBf6 = 7;
}  // namespace variant_ids

// Record a message for xeng_last_error() and return st.
xeng_status fail(xeng_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// XENG_EDEVICE with the HIP error string.
xeng_status device_error(hipError_t err, const char* what);
// Validate one correlation job; fills its input and output byte counts.
// ss, cs > 0: strided input (bytes between samples, between channels); the
// overlap check then uses the strided extent. 0: dense [F][T][N].
xeng_status check_job(const uint8_t* d_in, const int32_t* d_vis, int n, int f, int t,
                      int64_t t_prev, int accumulate, size_t* in_bytes, size_t* vis_bytes,
                      int64_t ss = 0, int64_t cs = 0);
// Compute units of the current device (256 if the query fails).
int device_cu_count();
// Time split: `units` workgroups per split step (channels, or tiles of all
// channels) over `stages` stages, chosen to fill `cus` compute units in whole
// rounds.
int auto_split(int64_t units, int64_t stages, int cus);
// The split for the triangle kernel and for the squares-and-tiles kernel.
int tri_auto_split(int f, int64_t t_count, int cus);
int rect_auto_split(int n, int f, int64_t t_count, int cus);
// The autotuner's choice for this job class on the current device, if any
// (variant id, split_t as xeng_correlate_variant takes it: 0 = the variant's own).
bool tuned_choice(int n, int f, int t, int* variant, int* split);

}  // namespace xeng
