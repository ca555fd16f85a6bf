// dd_batch_api.cpp -- C ABI of the persistent batched execution (host code).
//
// A batch holds many signals of uneven N and alpha (each the problem of
// Section 2 of the paper).  Planning groups them by (N, alpha) schedule class
// for the twiddle tables, cuts every signal into block-sized tasks and orders
// the task queue; execution is two launches of the persistent queue kernel of
// dd_batch.hip (plus plain executions for signals it is not built for).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "../../include/dense_dft.h"
#include "dd_batch.hpp"
#include "dd_host.hpp"
#include "dd_launch.hpp"

using namespace dd;

namespace {

struct Sched {
  bool single = false;
  int N1 = 0, N2 = 1;
};

struct ClassTables {
  Sched sc;
  void* twL1 = nullptr;
  void* twPre = nullptr;
  void* twQ = nullptr;
  void* twPost = nullptr;
  void* twL2 = nullptr;
};

bool in_list_single(int L) { return batch_code(BK_SINGLE, L) >= 0; }
bool in_list_p1(int L) { return batch_code(BK_PASS1, L) >= 0; }
bool in_list_p2(int L) { return batch_code(BK_PASS2, L) >= 0; }

size_t lds_single_b(int L, int alpha) { return lds_single(L, 1, alpha, 4); }

// Schedule of one FP32 signal in the batch kernel: one pass when its
// spectrum fits one block's LDS, else the most balanced N1 x N2 of the
// compiled pass lengths (N1 <= N2 on ties).  False: not runnable there.
bool batch_schedule(int64_t N, int alpha, Sched* out) {
  if (N <= 4096 && in_list_single((int)N) && lds_single_b((int)N, alpha) <= (size_t)BATCH_LDS_MAX) {
    out->single = true;
    out->N1 = (int)N;
    out->N2 = 1;
    return true;
  }
  int best = 1 << 30;
  bool found = false;
  for (int n2 = 32; n2 <= 512; n2 *= 2) {
    if (N % n2 || !in_list_p2(n2)) continue;
    const int64_t n1 = N / n2;
    if (n1 > 512 || !in_list_p1((int)n1)) continue;
    const int score = std::abs(ilog2(n1) - ilog2(n2)) * 2 + (n1 > n2 ? 1 : 0);
    if (score < best) {
      best = score;
      out->single = false;
      out->N1 = (int)n1;
      out->N2 = n2;
      found = true;
    }
  }
  return found;
}

}  // namespace

struct dd_batch {
  int device = 0;
  uint32_t flags = 0;
  std::vector<dd_desc> descs;
  std::vector<int> kitems;                 // descriptor index of each kernel item
  std::vector<int> fb;                     // descriptor index of each fallback signal
  std::vector<dd_plan_t> fb_plans;
  std::map<std::pair<int64_t, int>, ClassTables> classes;
  BatchItem* h_items = nullptr;            // pinned host copy of the descriptor table
  BatchItem* d_items = nullptr;
  BatchTask* d_tasks = nullptr;
  unsigned* d_ctl = nullptr;
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  int ntasks = 0, n_first = 0;
  size_t lds = 0;
  int grid = 0, grid1 = 0, grid2 = 0;
};

namespace {

void batch_free(dd_batch* b) {
  for (dd_plan_t p : b->fb_plans)
    if (p) dense_dft_destroy(p);
  b->fb_plans.clear();
  for (auto& kv : b->classes) {
    void* ts[] = {kv.second.twL1, kv.second.twPre, kv.second.twQ, kv.second.twPost, kv.second.twL2};
    for (void* t : ts)
      if (t) (void)hipFree(t);
  }
  b->classes.clear();
  if (b->h_items) (void)hipHostFree(b->h_items);
  void* ds[] = {b->d_items, b->d_tasks, b->d_ctl, b->scratch};
  for (void* d : ds)
    if (d) (void)hipFree(d);
  b->h_items = nullptr;
  b->d_items = nullptr;
  b->d_tasks = nullptr;
  b->d_ctl = nullptr;
  b->scratch = nullptr;
}

size_t in_elem(dd_dtype t) { return t == DD_F32 ? 4 : t == DD_C128 ? 16 : 8; }
size_t out_elem(dd_dtype t) { return (t == DD_F64 || t == DD_C128) ? 16 : 8; }

dd_status check_desc(const dd_desc& d) {
  if (d.N < 1 || !(d.T > 0.0) || !std::isfinite(d.T)) return DD_ERR_INVALID;
  if (d.dtype != DD_F32 && d.dtype != DD_C64 && d.dtype != DD_F64 && d.dtype != DD_C128) return DD_ERR_INVALID;
  if (!d.x || !d.X) return DD_ERR_INVALID;
  if ((uintptr_t)d.x % in_elem(d.dtype) || (uintptr_t)d.X % out_elem(d.dtype)) return DD_ERR_INVALID;
  if (d.alpha < 1) return DD_ERR_UNSUPPORTED;
  if ((int64_t)d.alpha * d.N > ((int64_t)1 << 31)) return DD_ERR_UNSUPPORTED;
  if (!is_smooth(d.N)) return DD_ERR_UNSUPPORTED;
  const uintptr_t x0 = (uintptr_t)d.x, x1 = x0 + (size_t)d.N * in_elem(d.dtype);
  const uintptr_t y0 = (uintptr_t)d.X, y1 = y0 + (size_t)d.alpha * d.N * out_elem(d.dtype);
  if (x0 < y1 && y0 < x1) return DD_ERR_INVALID;
  return DD_OK;
}

void fill_pointers(BatchItem& it, const dd_desc& d) {
  it.x = d.x;
  it.X = static_cast<cx<float>*>(d.X);
}

}  // namespace

extern "C" {

dd_status dense_dft_batch_plan(dd_batch_t* out, const dd_desc* descs, int32_t count, uint32_t flags) {
  if (!out) return DD_ERR_INVALID;
  *out = nullptr;
  if (!descs || count < 1) return DD_ERR_INVALID;
  if (flags & ~(uint32_t)DD_TWIDDLE_FP32) return DD_ERR_INVALID;
  for (int32_t i = 0; i < count; ++i) {
    const dd_status st = check_desc(descs[i]);
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
    const bool fp32 = d.dtype == DD_F32 || d.dtype == DD_C64;
    Sched sc;
    if (fp32 && batch_schedule(d.N, d.alpha, &sc)) {
      sched[i] = sc;
      b->kitems.push_back(i);
      auto key = std::make_pair(d.N, (int)d.alpha);
      if (!b->classes.count(key)) {
        ClassTables ct;
        ct.sc = sc;
        const int64_t M = (int64_t)d.alpha * d.N;
        st = make_stage_table(&ct.twL1, sc.N1, false, fp32tw, s);
        if (st == DD_OK) st = make_table(&ct.twPre, d.alpha, sc.N1, (int64_t)d.alpha * sc.N1, false, fp32tw, s);
        if (st == DD_OK && !sc.single) {
          st = make_table(&ct.twQ, d.alpha, sc.N2, M, false, fp32tw, s);
          if (st == DD_OK) st = make_table(&ct.twPost, sc.N1, sc.N2, d.N, false, fp32tw, s);
          if (st == DD_OK) st = make_stage_table(&ct.twL2, sc.N2, false, fp32tw, s);
        }
        b->classes[key] = ct;
      }
    } else {
      b->fb.push_back(i);
    }
  }

  // descriptor table, scratch layout, task list
  const int nk = (int)b->kitems.size();
  std::vector<BatchItem> items(nk);
  std::vector<int64_t> ysoff(nk, -1);
  size_t lds = 0;
  int64_t scratch_elems = 0;
  for (int k = 0; k < nk && st == DD_OK; ++k) {
    const dd_desc& d = descs[b->kitems[k]];
    const Sched& sc = sched[b->kitems[k]];
    const ClassTables& ct = b->classes[std::make_pair(d.N, (int)d.alpha)];
    BatchItem& it = items[k];
    std::memset(&it, 0, sizeof(it));
    fill_pointers(it, d);
    it.twL1 = static_cast<const cx<float>*>(ct.twL1);
    it.twPre = static_cast<const cx<float>*>(ct.twPre);
    it.twQ = static_cast<const cx<float>*>(ct.twQ);
    it.twPost = static_cast<const cx<float>*>(ct.twPost);
    it.twL2 = static_cast<const cx<float>*>(ct.twL2);
    it.N = d.N;
    it.N1 = sc.N1;
    it.N2 = sc.N2;
    it.alpha = d.alpha;
    it.real = d.dtype == DD_F32 ? 1 : 0;
    it.scale = (float)(d.T / (double)d.N);
    if (sc.single) {
      it.lines1 = 1;
      it.code1 = batch_code(BK_SINGLE, sc.N1);
      it.code2 = -1;
      lds = std::max(lds, lds_single_b(sc.N1, d.alpha));
    } else {
      const int C = batch_lines(sc.N1), RB = batch_lines(sc.N2);
      it.lines1 = C;
      it.ntile1 = (sc.N2 + C - 1) / C;
      it.jgroup = d.alpha;
      it.njg = 1;
      it.pre_lds = (size_t)d.alpha * sc.N1 * 8 <= 16 * 1024 ? 1 : 0;
      it.ntile2 = (d.alpha * sc.N1 + RB - 1) / RB;
      it.p1_tasks = it.ntile1 * it.njg;
      it.code1 = batch_code(BK_PASS1, sc.N1);
      it.code2 = batch_code(BK_PASS2, sc.N2);
      lds = std::max(lds, (size_t)pass1_lds_elems(sc.N1, C, it.pre_lds ? d.alpha * sc.N1 : 0) * 8);
      lds = std::max(lds, lds_pass2(sc.N2, RB, 4));
      ysoff[k] = scratch_elems;
      scratch_elems += (int64_t)d.alpha * d.N;
    }
  }
  b->lds = lds;
  b->scratch_bytes = (size_t)scratch_elems * 8;

  // queue: single-pass and pass-1 tasks (largest signals first; first
  // launch), then the pass-2 tasks in the same order (second launch)
  std::vector<int> order(nk);
  for (int k = 0; k < nk; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return (int64_t)items[a].alpha * items[a].N > (int64_t)items[c].alpha * items[c].N;
  });
  std::vector<BatchTask> tasks;
  for (int k : order) {
    const BatchItem& it = items[k];
    if (it.code2 < 0) {
      tasks.push_back(make_int4(k, BK_SINGLE, 0, it.code1));
    } else {
      for (int z = 0; z < it.p1_tasks; ++z) tasks.push_back(make_int4(k, BK_PASS1, z, it.code1));
    }
  }
  for (int k : order) {
    const BatchItem& it = items[k];
    if (it.code2 >= 0)
      for (int z = 0; z < it.ntile2; ++z) tasks.push_back(make_int4(k, BK_PASS2, z, it.code2));
  }
  b->ntasks = (int)tasks.size();
  b->n_first = 0;
  for (const BatchTask& t : tasks)
    if (t.y != BK_PASS2) ++b->n_first;

  if (st == DD_OK && nk > 0) {
    st = hip_status(hipMalloc(&b->scratch, b->scratch_bytes > 0 ? b->scratch_bytes : 8));
    for (int k = 0; k < nk; ++k)
      items[k].Y = ysoff[k] >= 0 ? static_cast<cx<float>*>(b->scratch) + ysoff[k] : nullptr;
    if (st == DD_OK) st = hip_status(hipHostMalloc((void**)&b->h_items, sizeof(BatchItem) * nk, hipHostMallocDefault));
    if (st == DD_OK) std::memcpy(b->h_items, items.data(), sizeof(BatchItem) * nk);
    if (st == DD_OK) st = hip_status(hipMalloc((void**)&b->d_items, sizeof(BatchItem) * nk));
    if (st == DD_OK) st = hip_status(hipMalloc((void**)&b->d_tasks, sizeof(BatchTask) * tasks.size()));
    if (st == DD_OK) st = hip_status(hipMalloc((void**)&b->d_ctl, sizeof(unsigned) * 2));
    if (st == DD_OK)
      st = hip_status(hipMemcpy(b->d_tasks, tasks.data(), sizeof(BatchTask) * tasks.size(), hipMemcpyHostToDevice));
    if (st == DD_OK) {
      hipDeviceProp_t prop;
      st = hip_status(hipGetDeviceProperties(&prop, b->device));
      const int per_cu = batch_max_blocks_per_cu(lds);
      b->grid = prop.multiProcessorCount * per_cu;
      b->grid1 = std::max(1, std::min(b->grid, b->n_first));
      b->grid2 = std::max(1, std::min(b->grid, b->ntasks - b->n_first));
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

dd_status dense_dft_batch_exec(dd_batch_t b, void* stream) {
  if (!b) return DD_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nk = (int)b->kitems.size();
  if (nk > 0) {
    hipError_t e = hipMemcpyAsync(b->d_items, b->h_items, sizeof(BatchItem) * nk, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_status(e);
    e = launch_batch(b->d_items, b->d_tasks, b->n_first, b->ntasks - b->n_first, b->d_ctl, b->grid1, b->grid2,
                     b->lds, s);
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
    if (check_desc(d) != DD_OK) return DD_ERR_INVALID;
  }
  for (int32_t i = 0; i < count; ++i) b->descs[i] = descs[i];
  for (size_t k = 0; k < b->kitems.size(); ++k) fill_pointers(b->h_items[k], descs[b->kitems[k]]);
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
  if (tasks) *tasks = b->ntasks;
  if (grid) *grid = b->grid;
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
