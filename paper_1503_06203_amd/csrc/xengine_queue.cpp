// xengine_queue.cpp -- host side of the batched queues: builds the device
// image (two queue headers, the job table, the item lists) that the
// persistent kernels consume, and launches those kernels. Shared by plans and
// the server.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "xcorr_launch.h"

namespace xeng {

int queue_kind_of(int n) { return n <= tri_max_elements() ? kQueueTri : kQueueWide; }

void build_queue_image(const QueueJob* table, int njobs, int split, uint8_t** image_out,
                       size_t* bytes_out, int64_t items_out[kQueueKinds]) {
  if (split < 1) split = 1;
  // Windows in order of decreasing cost per item, so the queue hands out the
  // longest items first and the short ones fill the tail.
  struct JobCost {
    int w;
    int64_t per_item;
  };
  std::vector<JobCost> order;
  for (int w = 0; w < njobs; ++w) {
    const int stages = table[w].total_stages;
    order.push_back({w, (stages + split - 1) / split});
  }
  std::stable_sort(order.begin(), order.end(),
                   [](const JobCost& a, const JobCost& b) { return a.per_item > b.per_item; });
  std::vector<QueueItem> items[kQueueKinds];
  std::vector<int64_t> cost[kQueueKinds];
  for (const auto& jc : order) {
    const QueueJob& J = table[jc.w];
    const int kind = queue_kind_of(J.n);
    const int ntiles = kind == kQueueTri ? 1 : J.ntiles;
    const int stages = J.total_stages;
    const int per = (stages + split - 1) / split;
    for (int ch = 0; ch < J.f; ++ch)
      for (int tile = 0; tile < ntiles; ++tile)
        for (int sb = 0; sb < stages; sb += per) {
          QueueItem it{};
          it.job = jc.w;
          it.ch = ch;
          it.tile = tile;
          it.stage_begin = sb;
          it.stage_end = std::min(stages, sb + per);
          items[kind].push_back(it);
          cost[kind].push_back(it.stage_end - it.stage_begin);
        }
  }
  size_t offset[kQueueKinds];
  offset[0] = queue_items_offset(njobs);
  for (int k = 1; k < kQueueKinds; ++k)
    offset[k] = (offset[k - 1] + sizeof(QueueItem) * items[k - 1].size() + 255) / 256 * 256;
  const size_t bytes = offset[kQueueKinds - 1] + sizeof(QueueItem) * items[kQueueKinds - 1].size();
  uint8_t* image = static_cast<uint8_t*>(std::calloc(bytes, 1));
  *image_out = image;
  *bytes_out = image ? bytes : 0;
  if (image == nullptr) return;
  std::memcpy(image + queue_jobs_offset(), table, sizeof(QueueJob) * (size_t)njobs);
  for (int k = 0; k < kQueueKinds; ++k) {
    // cut this kind's items into kQueueParts contiguous parts of about equal cost
    QueueHeader hdr{};
    const int64_t total = std::accumulate(cost[k].begin(), cost[k].end(), (int64_t)0);
    int part = 0;
    int64_t acc = 0;
    for (size_t i = 0; i < cost[k].size() && part < kQueueParts - 1; ++i) {
      acc += cost[k][i];
      if (acc * kQueueParts >= total * (part + 1)) hdr.part_begin[++part] = (int)i + 1;
    }
    while (part < kQueueParts - 1) hdr.part_begin[++part] = (int)items[k].size();
    hdr.part_begin[kQueueParts] = (int)items[k].size();
    hdr.jobs_offset = (int)queue_jobs_offset();
    hdr.items_offset = (int)offset[k];
    std::memcpy(image + (size_t)k * kQueueHeaderStride, &hdr, sizeof hdr);
    if (!items[k].empty())
      std::memcpy(image + offset[k], items[k].data(), sizeof(QueueItem) * items[k].size());
    items_out[k] = (int64_t)items[k].size();
  }
}

hipError_t launch_queues(void* d_ws, const int64_t items[kQueueKinds], int grid,
                         hipStream_t stream) {
  hipError_t e = hipSuccess;
  if (items[kQueueTri] > 0)
    e = launch_queue_tri(d_ws, kQueueTri * kQueueHeaderStride, grid, stream);
  if (e == hipSuccess && items[kQueueWide] > 0)
    e = launch_queue_wide(d_ws, kQueueWide * kQueueHeaderStride, grid, stream);
  return e;
}

}  // namespace xeng
