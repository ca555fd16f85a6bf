// Checks of the server's admission policy (dd_admit.hpp) on synthetic queues:
// plain requests at the head go alone, batches step over plain requests,
// kernel requests keep their order at the budget or pool limit, the batch
// size and the scan window bound a batch, plain mode takes one at a time.
#include <cstdio>
#include <deque>
#include <string>
#include <vector>

#include "../../paper_2403_16665_amd/csrc/dd_admit.hpp"
#include "../../paper_2403_16665_amd/csrc/dd_pool.hpp"

struct R {
  int id;
  bool kernel;
  size_t footprint, scratch;
};

static int failures = 0;

static void expect(bool ok, const std::string& what) {
  if (!ok) {
    std::printf("FAIL: %s\n", what.c_str());
    ++failures;
  }
}

static std::string ids(const std::vector<R*>& v) {
  std::string s;
  for (R* r : v) s += std::to_string(r->id) + " ";
  return s;
}

// One admission round with a byte budget and a scratch pool.
struct Server {
  size_t budget, used = 0;
  dd::RangeAlloc pool;
  Server(size_t b, size_t pool_bytes) : budget(b) { pool.reset(pool_bytes); }
  std::vector<R*> round(std::deque<R*>& q, int cap, bool plain, int solo_upto = 0) {
    std::vector<R*> take;
    auto reserve = [&](R* r) {
      if (used + r->footprint > budget) return false;
      size_t off = 0;
      if (r->scratch && !pool.alloc(r->scratch, &off)) return false;
      used += r->footprint;
      return true;
    };
    dd::admit_requests(q, cap, plain, [](const R* r) { return r->kernel; }, reserve, take, solo_upto);
    return take;
  }
};

int main() {
  std::vector<R> rs;
  for (int i = 0; i < 64; ++i) rs.push_back({i, true, 10, 0});
  auto queue = [&](std::initializer_list<int> order) {
    std::deque<R*> q;
    for (int i : order) q.push_back(&rs[i]);
    return q;
  };
  {  // a plain request at the head takes the slot alone
    rs[0].kernel = false;
    auto q = queue({0, 1, 2, 3});
    Server s(1000, 0);
    auto t = s.round(q, 8, false);
    expect(ids(t) == "0 " && q.size() == 3, "plain head alone: got " + ids(t));
    t = s.round(q, 8, false);
    expect(ids(t) == "1 2 3 " && q.empty(), "then the batch: got " + ids(t));
    rs[0].kernel = true;
  }
  {  // batches step over plain requests, which stay queued in order
    rs[3].kernel = rs[5].kernel = false;
    auto q = queue({1, 2, 3, 4, 5, 6});
    Server s(1000, 0);
    auto t = s.round(q, 8, false);
    expect(ids(t) == "1 2 4 6 ", "skip plain: got " + ids(t));
    expect(q.size() == 2 && q[0]->id == 3 && q[1]->id == 5, "plain requests remain in order");
    t = s.round(q, 8, false);
    expect(ids(t) == "3 ", "next slot takes the first plain: got " + ids(t));
    t = s.round(q, 8, false);
    expect(ids(t) == "5 " && q.empty(), "and then the second: got " + ids(t));
    rs[3].kernel = rs[5].kernel = true;
  }
  {  // the budget stops the batch at the first request that does not fit
    rs[2].footprint = 100;
    auto q = queue({1, 2, 3});
    Server s(50, 0);
    auto t = s.round(q, 8, false);
    expect(ids(t) == "1 " && q.size() == 2 && q[0]->id == 2, "budget keeps kernel order: got " + ids(t));
    rs[2].footprint = 10;
  }
  {  // the scratch pool does the same
    rs[1].scratch = rs[2].scratch = rs[3].scratch = 400;
    auto q = queue({1, 2, 3});
    Server s(1000, 1024);
    auto t = s.round(q, 8, false);
    expect(ids(t) == "1 2 " && q.size() == 1, "pool limit: got " + ids(t));
    rs[1].scratch = rs[2].scratch = rs[3].scratch = 0;
  }
  {  // a plain head that does not fit leaves the queue as it was
    rs[0].kernel = false;
    rs[0].footprint = 500;
    auto q = queue({0, 1});
    Server s(100, 0);
    auto t = s.round(q, 8, false);
    expect(t.empty() && q.size() == 2 && q[0]->id == 0, "plain head that does not fit");
    rs[0].kernel = true;
    rs[0].footprint = 10;
  }
  {  // the batch size bounds a batch
    auto q = queue({1, 2, 3, 4, 5, 6, 7, 8, 9, 10});
    Server s(1000, 0);
    auto t = s.round(q, 4, false);
    expect(ids(t) == "1 2 3 4 " && q.size() == 6, "cap: got " + ids(t));
  }
  {  // the scan window (4 * cap entries) bounds how far a batch looks
    for (int i = 11; i <= 20; ++i) rs[i].kernel = false;
    auto q = queue({1, 11, 12, 13, 14, 15, 16, 17, 18, 2});
    Server s(1000, 0);
    auto t = s.round(q, 2, false);
    expect(ids(t) == "1 ", "scan window: got " + ids(t));
    for (int i = 11; i <= 20; ++i) rs[i].kernel = true;
  }
  {  // plain mode: one request per slot, whatever it is
    auto q = queue({1, 2, 3});
    Server s(1000, 0);
    auto t = s.round(q, 8, true);
    expect(ids(t) == "1 " && q.size() == 2, "plain mode: got " + ids(t));
  }
  {  // light load: up to solo_upto queued requests go one per slot, more form a batch
    auto q = queue({1, 2});
    Server s(1000, 0);
    auto t = s.round(q, 8, false, 2);
    expect(ids(t) == "1 " && q.size() == 1, "solo at light load: got " + ids(t));
    t = s.round(q, 8, false, 2);
    expect(ids(t) == "2 " && q.empty(), "the second solo too: got " + ids(t));
    auto q3 = queue({3, 4, 5});
    t = s.round(q3, 8, false, 2);
    expect(ids(t) == "3 4 5 " && q3.empty(), "three queued form a batch: got " + ids(t));
    auto q1 = queue({6});
    t = s.round(q1, 8, false, 0);
    expect(ids(t) == "6 ", "solo_upto 0 keeps the batch path: got " + ids(t));
  }
  {  // nothing queued
    std::deque<R*> q;
    Server s(1000, 0);
    expect(s.round(q, 8, false).empty(), "empty queue");
  }
  if (failures == 0) std::printf("admission checks passed\n");
  return failures == 0 ? 0 : 1;
}
