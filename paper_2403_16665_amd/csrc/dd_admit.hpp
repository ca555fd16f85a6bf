// dd_admit.hpp -- which queued requests a free server slot takes (host only).
//
// The policy, separated from the server so that it can be checked without a
// GPU:
//   * a request the batch kernel does not serve (a plain execution: large,
//     FP64, or a length the kernel is not built for) takes a slot alone when
//     it reaches the head of the queue, so that its execution overlaps the
//     batches on the other slots;
//   * otherwise the slot gathers kernel requests in arrival order, stepping
//     over plain ones (the next free slot takes those), up to `cap`
//     requests, looking at most 4 * cap entries into the queue;
//   * it stops at the first kernel request that `reserve` refuses (the
//     memory budget or the scratch pool), so kernel requests keep their
//     order;
//   * in plain mode every request takes a slot alone;
//   * in batched mode, while no more than `solo_upto` requests are queued
//     (the server passes its number of free slots), the head takes the slot
//     alone too: a lightly loaded server runs each request as soon as a slot
//     frees, concurrently on separate slots, each at its solo latency (a
//     batch launch pays its staging and queue kernels; it wins once requests
//     outnumber the slots that could run them).
#pragma once

#include <vector>

namespace dd {

// pending: a std::deque (or list) of requests in arrival order; taken ones are
// removed and appended to `take`.  is_kernel(r): the batch kernel serves r.
// reserve(r): claims r's memory and returns true, or returns false (nothing
// claimed) when r does not fit now.
template <class Queue, class IsKernel, class Reserve>
void admit_requests(Queue& pending, int cap, bool plain_mode, IsKernel is_kernel, Reserve reserve,
                    std::vector<typename Queue::value_type>& take, int solo_upto = 0) {
  if (pending.empty() || cap < 1) return;
  if (plain_mode || !is_kernel(pending.front()) || (int)pending.size() <= solo_upto) {
    if (reserve(pending.front())) {
      take.push_back(pending.front());
      pending.pop_front();
    }
    return;
  }
  int scanned = 0;
  for (auto it = pending.begin(); it != pending.end() && (int)take.size() < cap && scanned < 4 * cap;
       ++scanned) {
    if (!is_kernel(*it)) {
      ++it;
      continue;
    }
    if (!reserve(*it)) break;
    take.push_back(*it);
    it = pending.erase(it);
  }
}

}  // namespace dd
