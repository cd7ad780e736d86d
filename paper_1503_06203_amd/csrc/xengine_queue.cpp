// xengine_queue.cpp -- host side of the batched queue: builds the device image
// (header, job table, item list) that the persistent queue kernel consumes.
// Shared by plans and the server.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "xcorr_launch.h"

namespace xeng {

void build_queue_image(const QueueJob* table, int njobs, int split, uint8_t** image_out,
                       size_t* bytes_out, int64_t* items_out) {
  if (split < 1) split = 1;
  // Jobs in order of decreasing cost per item, so the queue hands out the
  // longest items first and the short ones fill the tail. A diagonal square
  // gives each SIMD 9 blocks of 32 x 32 per step, an off-diagonal tile 8.
  struct JobCost {
    int w;
    int64_t per_item;
  };
  std::vector<JobCost> order;
  for (int w = 0; w < njobs; ++w) {
    const int stages = table[w].total_stages;
    order.push_back({w, (int64_t)((stages + split - 1) / split) * 9});
  }
  std::stable_sort(order.begin(), order.end(),
                   [](const JobCost& a, const JobCost& b) { return a.per_item > b.per_item; });
  std::vector<QueueItem> items;
  std::vector<int64_t> cost;
  for (const auto& jc : order) {
    const QueueJob& J = table[jc.w];
    const int stages = J.total_stages;
    const int per = (stages + split - 1) / split;
    // channel by channel, so the pieces that share a channel's panels are
    // neighbours in the queue (and on one XCD)
    for (int ch = 0; ch < J.f; ++ch)
      for (int u = 0; u < J.units; ++u)
        for (int sb = 0; sb < stages; sb += per) {
          QueueItem it{};
          it.job = jc.w;
          it.ch = ch;
          it.unit = u;
          it.stage_begin = sb;
          it.stage_end = std::min(stages, sb + per);
          items.push_back(it);
          cost.push_back((int64_t)(it.stage_end - it.stage_begin) * (u < J.nbc ? 9 : 8));
        }
  }
  const size_t offset = queue_items_offset(njobs);
  const size_t bytes = offset + sizeof(QueueItem) * items.size();
  uint8_t* image = static_cast<uint8_t*>(std::calloc(bytes, 1));
  *image_out = image;
  *bytes_out = image ? bytes : 0;
  if (image == nullptr) return;
  std::memcpy(image + queue_jobs_offset(), table, sizeof(QueueJob) * (size_t)njobs);
  // cut the items into kQueueParts contiguous parts of about equal cost
  QueueHeader hdr{};
  const int64_t total = std::accumulate(cost.begin(), cost.end(), (int64_t)0);
  int part = 0;
  int64_t acc = 0;
  for (size_t i = 0; i < cost.size() && part < kQueueParts - 1; ++i) {
    acc += cost[i];
    if (acc * kQueueParts >= total * (part + 1)) hdr.part_begin[++part] = (int)i + 1;
  }
  while (part < kQueueParts - 1) hdr.part_begin[++part] = (int)items.size();
  hdr.part_begin[kQueueParts] = (int)items.size();
  hdr.jobs_offset = (int)queue_jobs_offset();
  hdr.items_offset = (int)offset;
  std::memcpy(image, &hdr, sizeof hdr);
  if (!items.empty()) std::memcpy(image + offset, items.data(), sizeof(QueueItem) * items.size());
  *items_out = (int64_t)items.size();
}

}  // namespace xeng
