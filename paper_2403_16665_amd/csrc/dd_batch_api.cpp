// dd_batch_api.cpp -- C ABI of the persistent batched execution (host code).
//
// A batch holds many signals of uneven N and alpha (each the problem of
// Section 2 of the paper).  Planning groups them by (N, alpha) schedule class
// for the twiddle tables, orders them largest first and lays out their task
// ranges; execution is two launches of the persistent queue kernel of
// dd_batch.hip (plus plain executions for signals it is not built for).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "../../include/dense_dft.h"
#include "dd_batch_host.hpp"
#include "dd_launch.hpp"

using namespace dd;

struct dd_batch {
  int device = 0;
  uint32_t flags = 0;
  std::vector<dd_desc> descs;
  std::vector<int> kitems;                 // descriptor index of each kernel item, queue order
  std::vector<int> fb;                     // descriptor index of each fallback signal
  std::vector<dd_plan_t> fb_plans;
  std::map<std::pair<int64_t, int>, ClassTables> classes;
  BatchTable tab;                          // descriptor table (queue order)
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  size_t lds1 = 0, lds2 = 0;
  int grid1 = 1, grid2 = 1;
};

namespace {

void batch_free(dd_batch* b) {
  for (dd_plan_t p : b->fb_plans)
    if (p) dense_dft_destroy(p);
  b->fb_plans.clear();
  for (auto& kv : b->classes) free_class_tables(kv.second);
  b->classes.clear();
  free_table(b->tab);
  if (b->scratch) (void)hipFree(b->scratch);
  b->scratch = nullptr;
}

}  // namespace

dd_status dd::batch_plan_forced(dd_batch_t* out, const dd_desc* descs, int32_t count, uint32_t flags,
                                const Sched* force) {
  if (!out) return DD_ERR_INVALID;
  *out = nullptr;
  if (!descs || count < 1) return DD_ERR_INVALID;
  if (flags & ~(uint32_t)DD_TWIDDLE_FP32) return DD_ERR_INVALID;
  for (int32_t i = 0; i < count; ++i) {
    const dd_status st = batch_check_desc(descs[i]);
    if (st != DD_OK) return st;
  }
  dd_batch* b = new (std::nothrow) dd_batch;
  if (!b) return DD_ERR_NOMEM;
  b->flags = flags;
  b->descs.assign(descs, descs + count);
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return DD_ERR_DEVICE;
  }
  const bool fp32tw = (flags & DD_TWIDDLE_FP32) != 0;
  hipStream_t s = nullptr;
  dd_status st = DD_OK;

  // schedules and per-class tables
  std::vector<Sched> sched(count);
  for (int32_t i = 0; i < count && st == DD_OK; ++i) {
    const dd_desc& d = descs[i];
    const bool kernel = force ? (d.dtype == DD_F32 || d.dtype == DD_C64) && batch_sched_valid(d.N, d.alpha, *force)
                              : batch_kernel_ok(d, &sched[i]);
    if (force) sched[i] = *force;
    if (kernel) {
      b->kitems.push_back(i);
      const auto key = std::make_pair(d.N, (int)d.alpha);
      if (!b->classes.count(key)) {
        ClassTables ct;
        st = make_class_tables(d.N, d.alpha, sched[i], fp32tw, s, &ct);
        if (st == DD_OK) b->classes[key] = ct;
      }
    } else {
      b->fb.push_back(i);
    }
  }

  // queue order: one-pass signals of 1024 samples and more first (each is
  // one long task, a block's whole transform; started late, one of them
  // outlasts the rest of the queue), then the largest spectra, so that their
  // many tasks start early and the small ones fill the tail
  const auto long_task = [&](int i) { return sched[i].single && descs[i].N >= 1024; };
  std::stable_sort(b->kitems.begin(), b->kitems.end(), [&](int a, int c) {
    if (long_task(a) != long_task(c)) return long_task(a);
    return (int64_t)descs[a].alpha * descs[a].N > (int64_t)descs[c].alpha * descs[c].N;
  });
  const int nk = (int)b->kitems.size();
  std::vector<BatchItem> items(nk);
  std::vector<int64_t> ysoff(nk, -1);
  int64_t scratch_elems = 0;
  for (int k = 0; k < nk; ++k) {
    const dd_desc& d = descs[b->kitems[k]];
    if (!sched[b->kitems[k]].single) {
      ysoff[k] = scratch_elems;
      scratch_elems += (int64_t)d.alpha * d.N;
    }
  }
  b->scratch_bytes = (size_t)scratch_elems * sizeof(cx<float>);
  if (st == DD_OK && nk > 0) {
    st = hip_status(hipMalloc(&b->scratch, b->scratch_bytes > 0 ? b->scratch_bytes : 8));
    for (int k = 0; k < nk && st == DD_OK; ++k) {
      const dd_desc& d = descs[b->kitems[k]];
      const ClassTables& ct = b->classes[std::make_pair(d.N, (int)d.alpha)];
      fill_item(items[k], d, ct, ysoff[k] >= 0 ? static_cast<cx<float>*>(b->scratch) + ysoff[k] : nullptr);
      b->lds1 = std::max(b->lds1, item_lds1(items[k]));
      b->lds2 = std::max(b->lds2, item_lds2(items[k]));
    }
    BatchMeta meta;
    assign_task_offsets(items.data(), nk, &meta);
    if (st == DD_OK) st = alloc_table(b->tab, nk);
    if (st == DD_OK) {
      std::memcpy(b->tab.items(), items.data(), sizeof(BatchItem) * nk);
      *b->tab.host = meta;
    }
    if (st == DD_OK) st = hip_status(batch_set_lds(b->lds1, b->lds2));
    if (st == DD_OK) {
      hipDeviceProp_t prop;
      st = hip_status(hipGetDeviceProperties(&prop, b->device));
      const int cus = prop.multiProcessorCount;
      b->grid1 = std::max(1, std::min(cus * batch_max_blocks_per_cu(0, b->lds1), meta.n_first));
      b->grid2 = std::max(1, std::min(cus * batch_max_blocks_per_cu(1, b->lds2), meta.n_second));
    }
  }
  // fallback signals: plain plans of one signal each
  for (size_t i = 0; i < b->fb.size() && st == DD_OK; ++i) {
    const dd_desc& d = descs[b->fb[i]];
    dd_plan_t p = nullptr;
    st = dense_dft_plan(&p, d.N, d.alpha, d.T, 1, d.dtype, flags);
    b->fb_plans.push_back(p);
  }
  if (st == DD_OK) st = hip_status(hipStreamSynchronize(s));
  if (st != DD_OK) {
    batch_free(b);
    delete b;
    return st;
  }
  *out = b;
  return DD_OK;
}

extern "C" {

dd_status dense_dft_batch_plan(dd_batch_t* out, const dd_desc* descs, int32_t count, uint32_t flags) {
  return batch_plan_forced(out, descs, count, flags, nullptr);
}

dd_status dense_dft_batch_plan_sched(dd_batch_t* out, const dd_desc* descs, int32_t count, uint32_t flags,
                                     const dd_sched* sched) {
  if (out) *out = nullptr;
  if (!sched || (sched->passes != 1 && sched->passes != 2)) return DD_ERR_INVALID;
  Sched sc;
  sc.single = sched->passes == 1;
  sc.N1 = (int)std::min<int64_t>(sched->N1, 1 << 30);
  sc.N2 = (int)std::min<int64_t>(sched->passes == 1 ? 1 : sched->N2, 1 << 30);
  for (int32_t i = 0; descs && i < count; ++i)
    if ((descs[i].dtype == DD_F32 || descs[i].dtype == DD_C64) && !batch_sched_valid(descs[i].N, descs[i].alpha, sc))
      return DD_ERR_UNSUPPORTED;
  return batch_plan_forced(out, descs, count, flags, &sc);
}

dd_status dense_dft_batch_sched_candidates(int64_t N, int32_t alpha, dd_sched* out, int32_t cap, int32_t* count) {
  if (!count || cap < 0 || (cap > 0 && !out)) return DD_ERR_INVALID;
  *count = 0;
  const dd_status st = batch_check_shape(N, alpha, 1.0, DD_C64);
  if (st != DD_OK) return st;
  Sched c[16];
  const int n = batch_candidates(N, alpha, c, 16);
  for (int i = 0; i < n && i < cap; ++i) {
    out[i] = dd_sched{};
    out[i].passes = c[i].single ? 1 : 2;
    out[i].N1 = c[i].N1;
    out[i].N2 = c[i].N2;
  }
  *count = n;
  return n > 0 ? DD_OK : DD_ERR_UNSUPPORTED;
}

dd_status dense_dft_batch_exec(dd_batch_t b, void* stream) {
  if (!b) return DD_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nk = (int)b->kitems.size();
  if (nk > 0) {
    const int g2 = b->tab.host->n_second > 0 ? b->grid2 : 0;
    const hipError_t e =
        launch_batch(b->tab.host_dev, b->tab.dev, b->tab.cap, b->tab.ctl, b->grid1, g2, b->lds1, b->lds2, s);
    if (e != hipSuccess) return hip_status(e);
  }
  for (size_t i = 0; i < b->fb.size(); ++i) {
    const dd_desc& d = b->descs[b->fb[i]];
    const dd_status st = dense_dft_exec(b->fb_plans[i], d.x, d.X, nullptr, stream);
    if (st != DD_OK) return st;
  }
  return DD_OK;
}

dd_status dense_dft_batch_set_buffers(dd_batch_t b, const dd_desc* descs, int32_t count) {
  if (!b || !descs || count != (int32_t)b->descs.size()) return DD_ERR_INVALID;
  for (int32_t i = 0; i < count; ++i) {
    const dd_desc &o = b->descs[i], &d = descs[i];
    if (d.N != o.N || d.alpha != o.alpha || d.T != o.T || d.dtype != o.dtype) return DD_ERR_INVALID;
    if (batch_check_desc(d) != DD_OK) return DD_ERR_INVALID;
  }
  for (int32_t i = 0; i < count; ++i) b->descs[i] = descs[i];
  for (size_t k = 0; k < b->kitems.size(); ++k) {
    b->tab.items()[k].x = descs[b->kitems[k]].x;
    b->tab.items()[k].X = static_cast<cx<float>*>(descs[b->kitems[k]].X);
  }
  return DD_OK;
}

dd_status dense_dft_batch_status(dd_batch_t b, uint32_t* flags) {
  if (!b || !flags) return DD_ERR_INVALID;
  *flags = 0;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(b->device);
  const hipError_t e = hipDeviceSynchronize();
  (void)hipSetDevice(cur);
  return hip_status(e);
}

dd_status dense_dft_batch_info(dd_batch_t b, int32_t* tasks, int32_t* grid, size_t* scratch_bytes,
                               int32_t* fallback) {
  if (!b) return DD_ERR_INVALID;
  if (tasks) *tasks = b->tab.host ? b->tab.host->n_first + b->tab.host->n_second : 0;
  if (grid) *grid = std::max(b->grid1, b->grid2);
  if (scratch_bytes) *scratch_bytes = b->scratch_bytes;
  if (fallback) *fallback = (int32_t)b->fb.size();
  return DD_OK;
}

dd_status dense_dft_batch_destroy(dd_batch_t b) {
  if (!b) return DD_ERR_INVALID;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  batch_free(b);
  (void)hipSetDevice(cur);
  delete b;
  return DD_OK;
}

dd_status dense_dft_exec_many(const dd_desc* descs, int32_t count, void* stream) {
  dd_batch_t b = nullptr;
  dd_status st = dense_dft_batch_plan(&b, descs, count, 0);
  if (st != DD_OK) return st;
  st = dense_dft_batch_exec(b, stream);
  if (st == DD_OK) st = hip_status(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  const dd_status st2 = dense_dft_batch_destroy(b);
  return st != DD_OK ? st : st2;
}

}  // extern "C"
