// Admission decision of the serving loop's worker pool (host only, no HIP).
//
// An idle worker holding `hold` bytes of grow-only device buffers looks at
// the queue (oldest first) while `others` bytes are reserved by the running
// problems and the other idle workers' buffers.  It runs the first request
// whose footprint fits next to its own buffers; if the first request that
// does not fit would fit without them, it releases them and decides again;
// the oldest request may be passed over at most kMaxSkips times, after which
// nothing behind it is taken.  If nothing fits, a worker that holds memory
// releases it (it may be what is missing), and otherwise waits.  The caller
// holds the pool's lock and counts the passes over the oldest request.
#pragma once

#include <cstddef>

namespace hotrg {

constexpr int kMaxSkips = 8;

enum AdmitAction { ADMIT_RUN, ADMIT_RELEASE, ADMIT_WAIT };

struct AdmitChoice {
  AdmitAction action;
  size_t index;  // the request to run (ADMIT_RUN)
};

// Queue: indexable, size(); footprint(q[i]) -> bytes, skips(q[i]) -> passes
template <class Queue, class Footprint, class Skips>
AdmitChoice admit_choice(const Queue& q, Footprint footprint, Skips skips, size_t others,
                         size_t hold, size_t budget) {
  for (size_t i = 0; i < q.size(); ++i) {
    const size_t f = footprint(q[i]);
    if (others + hold + f <= budget) return {ADMIT_RUN, i};
    if (others + f <= budget) return {ADMIT_RELEASE, 0};
    if (i == 0 && skips(q[0]) >= kMaxSkips) break;
  }
  if (q.size() > 0 && hold > 0) return {ADMIT_RELEASE, 0};
  return {ADMIT_WAIT, 0};
}

}  // namespace hotrg
