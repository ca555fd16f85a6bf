// dd_tune.cpp -- the tuner: measures every schedule the kernels can run a
// problem class with (one pass with each block width, or each two-pass split
// N = N1 * N2 with each j-group) on the current device and keeps the fastest
// in a process-wide table that plans, batches and servers consult; the table
// can be saved to and loaded from a text file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/dense_dft.h"
#include "dd_batch_host.hpp"
#include "dd_host.hpp"
#include "dd_launch.hpp"
#include "dd_tune.hpp"

namespace dd {

namespace {

struct Entry {
  dd_sched s;
  float ms;
};

std::mutex g_mu;
std::map<std::tuple<int64_t, int, int, int>, Entry> g_plan;  // N, alpha, input dtype, batch class
std::map<std::pair<int64_t, int>, Entry> g_batch;            // N, alpha
bool g_env_checked = false;

bool sched_sane(const dd_sched& s) {
  if (s.passes == 1) return s.lines >= 0 && s.lines <= 1024;
  return s.passes == 2 && s.N1 >= 1 && s.N2 >= 1 && s.jgroup >= 0 && s.chunk >= 0;
}

// Parse a saved table into the maps (g_mu held); false if it cannot be read.
bool load_locked(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    long long N, N1, N2, chunk;
    int alpha, dbl, bclass, passes, lines, jgroup;
    float ms;
    dd_sched s{};
    int dtype = -1;
    // plan2 (keyed by input dtype); plan (earlier files, keyed by precision:
    // the entry serves both input dtypes of that precision)
    const bool v2 = std::sscanf(line, "plan2 %lld %d %d %d %d %d %lld %lld %d %lld %f", &N, &alpha, &dtype, &bclass,
                                &passes, &lines, &N1, &N2, &jgroup, &chunk, &ms) == 11;
    const bool v1 = !v2 && std::sscanf(line, "plan %lld %d %d %d %d %d %lld %lld %d %lld %f", &N, &alpha, &dbl,
                                       &bclass, &passes, &lines, &N1, &N2, &jgroup, &chunk, &ms) == 11;
    if (v1 || v2) {
      s.passes = passes;
      s.lines = lines;
      s.N1 = N1;
      s.N2 = N2;
      s.jgroup = jgroup;
      s.chunk = chunk;
      const bool ok = N >= 1 && alpha >= 1 && bclass >= 0 && bclass <= 12 && sched_sane(s);
      if (ok && v2 && dtype >= DD_F32 && dtype <= DD_C128)
        g_plan[std::make_tuple((int64_t)N, alpha, dtype, bclass)] = Entry{s, ms};
      if (ok && v1 && (dbl == 0 || dbl == 1))
        for (int d : {dbl ? (int)DD_F64 : (int)DD_F32, dbl ? (int)DD_C128 : (int)DD_C64})
          g_plan[std::make_tuple((int64_t)N, alpha, d, bclass)] = Entry{s, ms};
    } else if (std::sscanf(line, "batch %lld %d %d %lld %lld %f", &N, &alpha, &passes, &N1, &N2, &ms) == 6) {
      s.passes = passes;
      s.N1 = N1;
      s.N2 = N2;
      if (N >= 1 && alpha >= 1 && (passes == 1 || passes == 2) && sched_sane(s))
        g_batch[std::make_pair((int64_t)N, alpha)] = Entry{s, ms};
    }
  }
  std::fclose(f);
  return true;
}

// The file named by DD_TUNE_DB, once per process (g_mu held).
void env_once_locked() {
  if (g_env_checked) return;
  g_env_checked = true;
  if (const char* p = std::getenv("DD_TUNE_DB")) (void)load_locked(p);
}

// Mean time of one call of `run` on stream s, in ms: one warm-up call, then
// enough calls for about 4 ms.
template <typename F>
dd_status time_calls(hipStream_t s, F&& run, float* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  dd_status st = hip_status(hipEventCreate(&e0));
  if (st == DD_OK) st = hip_status(hipEventCreate(&e1));
  float t = 0.f;
  int reps = 1;
  for (int round = 0; round < 2 && st == DD_OK; ++round) {
    if (round == 0) st = run();  // warm-up
    if (st == DD_OK) st = hip_status(hipEventRecord(e0, s));
    for (int i = 0; i < reps && st == DD_OK; ++i) st = run();
    if (st == DD_OK) st = hip_status(hipEventRecord(e1, s));
    if (st == DD_OK) st = hip_status(hipEventSynchronize(e1));
    if (st == DD_OK) st = hip_status(hipEventElapsedTime(&t, e0, e1));
    if (round == 0) reps = std::max(2, std::min(64, (int)std::ceil(4.0 / std::max(t, 1e-3f))));
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  *ms = t / reps;
  return st;
}

bool same_sched(const dd_sched& a, const dd_sched& b) {
  return a.passes == b.passes && a.lines == b.lines && a.N1 == b.N1 && a.N2 == b.N2 && a.jgroup == b.jgroup &&
         a.chunk == b.chunk;
}

}  // namespace

int tune_batch_class(int64_t batch) {
  int b = 0;
  while (b < 12 && ((int64_t)2 << b) <= batch) ++b;
  return b;
}

bool tune_lookup_plan(int64_t N, int alpha, int dtype, int64_t batch, dd_sched* out) {
  std::lock_guard<std::mutex> g(g_mu);
  env_once_locked();
  auto it = g_plan.find(std::make_tuple(N, alpha, dtype, tune_batch_class(batch)));
  if (it == g_plan.end()) return false;
  *out = it->second.s;
  return true;
}

void tune_store_plan(int64_t N, int alpha, int dtype, int64_t batch, const dd_sched& s, float ms) {
  std::lock_guard<std::mutex> g(g_mu);
  env_once_locked();
  g_plan[std::make_tuple(N, alpha, dtype, tune_batch_class(batch))] = Entry{s, ms};
}

bool tune_lookup_batch(int64_t N, int alpha, dd_sched* out) {
  std::lock_guard<std::mutex> g(g_mu);
  env_once_locked();
  auto it = g_batch.find(std::make_pair(N, alpha));
  if (it == g_batch.end()) return false;
  *out = it->second.s;
  return true;
}

void tune_store_batch(int64_t N, int alpha, const dd_sched& s, float ms) {
  std::lock_guard<std::mutex> g(g_mu);
  env_once_locked();
  g_batch[std::make_pair(N, alpha)] = Entry{s, ms};
}

}  // namespace dd

using namespace dd;

extern "C" {

dd_status dense_dft_tune(int64_t N, int32_t alpha, int64_t batch, dd_dtype dtype, dd_tune_info* info) {
  if (!info) return DD_ERR_INVALID;
  *info = dd_tune_info{};
  // the default plan validates the problem and fixes the reference time
  dd_plan_t p0 = nullptr;
  dd_status st = dense_dft_plan(&p0, N, alpha, 1.0, batch, dtype, DD_NO_WORKSPACE);
  if (st != DD_OK) return st;
  dd_sched def{};
  (void)dense_dft_plan_get_sched(p0, &def);
  (void)dense_dft_destroy(p0);

  const bool dbl = dtype == DD_F64 || dtype == DD_C128;
  const size_t in_bytes = dtype == DD_F32 ? 4 : dtype == DD_C128 ? 16 : 8;
  const size_t out_bytes = dbl ? 16 : 8;
  int32_t nc = 0;
  (void)dense_dft_sched_candidates(N, alpha, batch, dtype, nullptr, 0, &nc);
  std::vector<dd_sched> cands(std::max(nc, 1));
  st = dense_dft_sched_candidates(N, alpha, batch, dtype, cands.data(), nc, &nc);
  if (st != DD_OK) return st;
  cands.resize(nc);
  // the schedule in effect before this call is measured first
  cands.insert(cands.begin(), def);

  void *x = nullptr, *X = nullptr, *ws = nullptr;
  size_t ws_cap = 0;
  hipStream_t s = nullptr;
  const size_t nx = (size_t)batch * N * in_bytes, nX = (size_t)batch * alpha * N * out_bytes;
  st = hip_status(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  if (st == DD_OK) st = hip_status(hipMalloc(&x, nx));
  if (st == DD_OK) st = hip_status(hipMalloc(&X, nX));
  if (st == DD_OK) st = hip_status(hipMemset(x, 0, nx));
  float best = 0.f, t_def = 0.f;
  dd_sched best_s = def;
  int measured = 0;
  for (size_t i = 0; i < cands.size() && st == DD_OK; ++i) {
    if (i > 0 && same_sched(cands[i], def)) continue;
    dd_plan_t p = nullptr;
    if (dense_dft_plan_sched(&p, N, alpha, 1.0, batch, dtype, DD_NO_WORKSPACE, &cands[i]) != DD_OK) continue;
    size_t need = 0;
    (void)dense_dft_workspace_size(p, &need);
    if (need > ws_cap) {
      if (ws) (void)hipFree(ws);
      ws = nullptr;
      ws_cap = 0;
      st = hip_status(hipMalloc(&ws, need));
      if (st == DD_OK) ws_cap = need;
    }
    float t = 0.f;
    if (st == DD_OK) st = time_calls(s, [&] { return dense_dft_exec(p, x, X, ws, s); }, &t);
    dd_sched got{};
    (void)dense_dft_plan_get_sched(p, &got);
    (void)dense_dft_destroy(p);
    if (st != DD_OK) break;
    ++measured;
    if (i == 0) t_def = t;
    if (measured == 1 || t < best) {
      best = t;
      best_s = got;
    }
  }
  if (s) (void)hipStreamDestroy(s);
  void* bufs[] = {x, X, ws};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (st != DD_OK) return st;
  tune_store_plan(N, alpha, (int)dtype, batch, best_s, best);
  info->best = best_s;
  info->ms_best = best;
  info->ms_default = t_def;
  info->candidates = measured;
  return DD_OK;
}

dd_status dense_dft_tune_batch(int64_t N, int32_t alpha, dd_tune_info* info) {
  if (!info) return DD_ERR_INVALID;
  *info = dd_tune_info{};
  dd_status st = batch_check_shape(N, alpha, 1.0, DD_C64);
  if (st != DD_OK) return st;
  Sched cands[16];
  const int nc = batch_candidates(N, alpha, cands, 16);
  Sched def;
  if (nc == 0 || !batch_default_schedule(N, alpha, &def)) return DD_ERR_UNSUPPORTED;
  // enough signals of the class to fill the device: about 2^24 bins
  const int64_t M = (int64_t)alpha * N;
  const int count = (int)std::max<int64_t>(1, std::min<int64_t>(256, ((int64_t)1 << 24) / M));
  void *x = nullptr, *X = nullptr;
  hipStream_t s = nullptr;
  st = hip_status(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  if (st == DD_OK) st = hip_status(hipMalloc(&x, (size_t)count * N * 8));
  if (st == DD_OK) st = hip_status(hipMalloc(&X, (size_t)count * M * 8));
  if (st == DD_OK) st = hip_status(hipMemset(x, 0, (size_t)count * N * 8));
  std::vector<dd_desc> descs(count);
  for (int i = 0; i < count; ++i)
    descs[i] = dd_desc{N, alpha, 1.0, DD_C64, static_cast<char*>(x) + (size_t)i * N * 8,
                       static_cast<char*>(X) + (size_t)i * M * 8};
  float best = 0.f, t_def = 0.f;
  Sched best_s = def;
  int measured = 0;
  for (int i = -1; i < nc && st == DD_OK; ++i) {
    const Sched& c = i < 0 ? def : cands[i];
    if (i >= 0 && c.single == def.single && c.N1 == def.N1 && c.N2 == def.N2) continue;
    dd_batch_t b = nullptr;
    st = batch_plan_forced(&b, descs.data(), count, 0, &c);
    if (st != DD_OK) break;
    float t = 0.f;
    st = time_calls(s, [&] { return dense_dft_batch_exec(b, s); }, &t);
    (void)dense_dft_batch_destroy(b);
    if (st != DD_OK) break;
    ++measured;
    if (i < 0) t_def = t;
    if (measured == 1 || t < best) {
      best = t;
      best_s = c;
    }
  }
  if (s) (void)hipStreamDestroy(s);
  if (x) (void)hipFree(x);
  if (X) (void)hipFree(X);
  if (st != DD_OK) return st;
  dd_sched r{};
  r.passes = best_s.single ? 1 : 2;
  r.N1 = best_s.N1;
  r.N2 = best_s.N2;
  tune_store_batch(N, alpha, r, best / count);
  info->best = r;
  info->ms_best = best;
  info->ms_default = t_def;
  info->candidates = measured;
  return DD_OK;
}

dd_status dense_dft_tune_save(const char* path) {
  if (!path) return DD_ERR_INVALID;
  std::lock_guard<std::mutex> g(g_mu);
  env_once_locked();
  FILE* f = std::fopen(path, "w");
  if (!f) return DD_ERR_INVALID;
  std::fprintf(f, "# dense_dft tuning table v2\n");
  std::fprintf(f, "# plan2 N alpha input_dtype batch_class passes lines N1 N2 jgroup chunk ms\n");
  for (const auto& kv : g_plan) {
    const dd_sched& s = kv.second.s;
    std::fprintf(f, "plan2 %lld %d %d %d %d %d %lld %lld %d %lld %.6g\n", (long long)std::get<0>(kv.first),
                 std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first), s.passes, s.lines,
                 (long long)s.N1, (long long)s.N2, s.jgroup, (long long)s.chunk, kv.second.ms);
  }
  std::fprintf(f, "# batch N alpha passes N1 N2 ms_per_signal\n");
  for (const auto& kv : g_batch) {
    const dd_sched& s = kv.second.s;
    std::fprintf(f, "batch %lld %d %d %lld %lld %.6g\n", (long long)kv.first.first, kv.first.second, s.passes,
                 (long long)s.N1, (long long)s.N2, kv.second.ms);
  }
  const bool ok = std::fclose(f) == 0;
  return ok ? DD_OK : DD_ERR_INVALID;
}

dd_status dense_dft_tune_load(const char* path) {
  if (!path) return DD_ERR_INVALID;
  std::lock_guard<std::mutex> g(g_mu);
  env_once_locked();
  return load_locked(path) ? DD_OK : DD_ERR_INVALID;
}

dd_status dense_dft_tune_clear(void) {
  std::lock_guard<std::mutex> g(g_mu);
  g_env_checked = true;
  g_plan.clear();
  g_batch.clear();
  return DD_OK;
}

dd_status dense_dft_tune_entries(int32_t* plans, int32_t* batch_classes) {
  std::lock_guard<std::mutex> g(g_mu);
  env_once_locked();
  if (plans) *plans = (int32_t)g_plan.size();
  if (batch_classes) *batch_classes = (int32_t)g_batch.size();
  return DD_OK;
}

}  // extern "C"
