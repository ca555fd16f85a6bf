// dd_batch_host.hpp -- host-side construction of batch descriptors, shared by
// the batch API (dd_batch_api.cpp) and the request server (dd_serve.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#include "../../include/dense_dft.h"
#include "dd_batch.hpp"
#include "dd_host.hpp"
#include "dd_launch.hpp"
#include "dd_tune.hpp"

namespace dd {

struct Sched {
  bool single = false;
  int N1 = 0, N2 = 1;
};

// Device twiddle tables of one (N, alpha) schedule class, FP32 rounded from FP64.
struct ClassTables {
  Sched sc;
  void* twL1 = nullptr;
  void* twPre = nullptr;
  void* twQ = nullptr;
  void* twPost = nullptr;
  void* twL2 = nullptr;
};

inline size_t batch_in_elem(dd_dtype t) { return t == DD_F32 ? 4 : t == DD_C128 ? 16 : 8; }
inline size_t batch_out_elem(dd_dtype t) { return (t == DD_F64 || t == DD_C128) ? 16 : 8; }

// Validation of a signal's shape (the plan's rules).
inline dd_status batch_check_shape(int64_t N, int alpha, double T, dd_dtype dtype) {
  if (N < 1 || !(T > 0.0) || !std::isfinite(T)) return DD_ERR_INVALID;
  if (dtype != DD_F32 && dtype != DD_C64 && dtype != DD_F64 && dtype != DD_C128) return DD_ERR_INVALID;
  if (alpha < 1) return DD_ERR_UNSUPPORTED;
  if ((int64_t)alpha * N > ((int64_t)1 << 31)) return DD_ERR_UNSUPPORTED;
  if (!is_smooth(N)) return DD_ERR_UNSUPPORTED;
  if (!scale_ok(T / (double)N, dtype == DD_F64 || dtype == DD_C128)) return DD_ERR_UNSUPPORTED;
  return DD_OK;
}

// Validation of one signal descriptor: shape, then pointers (non-null,
// aligned to the element size, x and X disjoint).
inline dd_status batch_check_desc(const dd_desc& d) {
  if (!d.x || !d.X) return DD_ERR_INVALID;
  const dd_status st = batch_check_shape(d.N, d.alpha, d.T, d.dtype);
  if (st != DD_OK) return st;
  if ((uintptr_t)d.x % batch_in_elem(d.dtype) || (uintptr_t)d.X % batch_out_elem(d.dtype)) return DD_ERR_INVALID;
  const uintptr_t x0 = (uintptr_t)d.x, x1 = x0 + (size_t)d.N * batch_in_elem(d.dtype);
  const uintptr_t y0 = (uintptr_t)d.X, y1 = y0 + (size_t)d.alpha * d.N * batch_out_elem(d.dtype);
  if (x0 < y1 && y0 < x1) return DD_ERR_INVALID;
  return DD_OK;
}

// Whether a schedule is runnable in the batch kernel for (N, alpha): one
// pass of a compiled length whose spectrum fits the block's LDS, or two
// passes N = N1 * N2 of compiled pass lengths.
inline bool batch_sched_valid(int64_t N, int alpha, const Sched& sc) {
  if (sc.single)
    return N <= 4096 && sc.N1 == N && batch_code(BK_SINGLE, (int)N) >= 0 && batch_single_groups((int)N, alpha) > 0;
  return sc.N1 >= 1 && sc.N2 >= 1 && (int64_t)sc.N1 * sc.N2 == N && batch_code(BK_PASS1, sc.N1) >= 0 &&
         batch_code(BK_PASS2, sc.N2) >= 0;
}

// Every schedule the batch kernel can run (N, alpha) with: the tuner's
// candidates.  Returns their number (at most `cap` written).
inline int batch_candidates(int64_t N, int alpha, Sched* out, int cap) {
  int n = 0;
  Sched one;
  one.single = true;
  one.N1 = (int)(N <= 4096 ? N : 0);
  one.N2 = 1;
  if (batch_sched_valid(N, alpha, one) && n < cap) out[n++] = one;
  for (int n2 = 2; n2 <= 4096; n2 *= 2) {
    if (N % n2 || N / n2 > 4096) continue;
    Sched two;
    two.single = false;
    two.N1 = (int)(N / n2);
    two.N2 = n2;
    if (batch_sched_valid(N, alpha, two) && n < cap) out[n++] = two;
  }
  return n;
}

// Built-in schedule of one FP32 signal in the batch kernel: one pass when
// its spectrum fits one block's LDS, else the most balanced N1 x N2 of the
// compiled pass lengths (N1 <= N2 on ties).  False: not runnable there.
inline bool batch_default_schedule(int64_t N, int alpha, Sched* out) {
  Sched c[16];
  const int n = batch_candidates(N, alpha, c, 16);
  int best = 1 << 30;
  for (int i = 0; i < n; ++i) {
    const int score = c[i].single ? -1 : std::abs(ilog2(c[i].N1) - ilog2(c[i].N2)) * 2 + (c[i].N1 > c[i].N2 ? 1 : 0);
    if (score < best) {
      best = score;
      *out = c[i];
    }
  }
  return n > 0;
}

// Schedule of (N, alpha) in the batch kernel: the tuned one if the tuning
// table has a runnable one, else the built-in rule.
inline bool batch_schedule(int64_t N, int alpha, Sched* out) {
  dd_sched t;
  if (tune_lookup_batch(N, alpha, &t)) {
    Sched sc;
    sc.single = t.passes == 1;
    sc.N1 = (int)t.N1;
    sc.N2 = (int)t.N2;
    if (batch_sched_valid(N, alpha, sc)) {
      *out = sc;
      return true;
    }
  }
  return batch_default_schedule(N, alpha, out);
}

// Whether a descriptor runs in the batch kernel (FP32 input, compiled lengths).
inline bool batch_kernel_ok(const dd_desc& d, Sched* sc) {
  return (d.dtype == DD_F32 || d.dtype == DD_C64) && batch_schedule(d.N, d.alpha, sc);
}

inline size_t batch_scratch_bytes(const dd_desc& d, const Sched& sc) {
  return sc.single ? 0 : (size_t)d.alpha * d.N * 8;
}

inline void free_class_tables(ClassTables& ct) {
  void* ts[] = {ct.twL1, ct.twPre, ct.twQ, ct.twPost, ct.twL2};
  for (void* t : ts)
    if (t) (void)hipFree(t);
  ct = ClassTables{};
}

// Tables of the class of (N, alpha) with schedule sc, generated on stream s.
inline dd_status make_class_tables(int64_t N, int alpha, const Sched& sc, bool fp32tw, hipStream_t s,
                                   ClassTables* ct) {
  ct->sc = sc;
  const int64_t M = (int64_t)alpha * N;
  dd_status st = make_stage_table(&ct->twL1, sc.N1, false, fp32tw, s, sc.single && single_narrow(sc.N1));
  if (st == DD_OK) st = make_table(&ct->twPre, alpha, sc.N1, (int64_t)alpha * sc.N1, false, fp32tw, s);
  if (st == DD_OK && !sc.single) {
    st = make_table(&ct->twQ, alpha, sc.N2, M, false, fp32tw, s);
    if (st == DD_OK) st = make_table(&ct->twPost, sc.N1, sc.N2, N, false, fp32tw, s);
    if (st == DD_OK) st = make_stage_table(&ct->twL2, sc.N2, false, fp32tw, s);
  }
  if (st != DD_OK) free_class_tables(*ct);
  return st;
}

// Fill every field of a descriptor except t1 / t2; Y is its scratch.
inline void fill_item(BatchItem& it, const dd_desc& d, const ClassTables& ct, cx<float>* Y) {
  const Sched& sc = ct.sc;
  std::memset(&it, 0, sizeof(it));
  it.x = d.x;
  it.X = static_cast<cx<float>*>(d.X);
  it.Y = Y;
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
    it.lines1 = batch_single_groups(sc.N1, d.alpha);
    it.p1_tasks = 1;
    it.code1 = batch_code(BK_SINGLE, sc.N1);
    it.code2 = -1;
  } else {
    const int C = batch_lines(sc.N1), RB = batch_lines2(sc.N2);
    it.lines1 = C;
    it.ntile1 = (sc.N2 + C - 1) / C;
    it.jgroup = d.alpha;
    it.njg = 1;
    // pre-twiddles in LDS: whole rows within 16 KiB, else their two factors
    // (the j loop then reads no global memory, so it does not wait for the
    // stores of the previous j)
    it.pre_lds = (size_t)d.alpha * sc.N1 * 8 <= 16 * 1024 ? 1 : 0;
    if (!it.pre_lds &&
        (size_t)pass1_lds_elems(sc.N1, C, pass1_pre_elems(2, d.alpha, sc.N1)) * 8 <= (size_t)BATCH_LDS_MAX)
      it.pre_lds = 2;
    it.q_lds = 0;
    const size_t with_q =
        (size_t)pass1_lds_elems(sc.N1, C, pass1_pre_elems(it.pre_lds, d.alpha, sc.N1) + d.alpha * C) * 8;
    if ((size_t)d.alpha * C * 8 <= 4096 && with_q <= (size_t)BATCH_LDS_MAX) it.q_lds = 1;
    // W_N^{k1 n2} from two rows of its table: the items of a batch belong to
    // many classes whose tables do not stay in the L2, and a task then reads
    // TL + EPT rows of its class's table instead of all N1 (that table is as
    // large as the signal)
    const int pre_q = pass1_pre_elems(it.pre_lds, d.alpha, sc.N1) + (it.q_lds ? d.alpha * C : 0);
    it.post_split =
        (size_t)pass1_lds_elems(sc.N1, C, pre_q + pass1_post_elems(sc.N1, C)) * 8 <= (size_t)BATCH_LDS_MAX ? 1 : 0;
    it.ntile2 = (d.alpha * sc.N1 + RB - 1) / RB;
    it.p1_tasks = it.ntile1 * it.njg;
    it.code1 = batch_code(BK_PASS1, sc.N1);
    it.code2 = batch_code(BK_PASS2, sc.N2);
  }
}

// LDS bytes the item's tasks need in the first (single-pass / pass-1) and
// the second (pass-2) queue kernel.
inline size_t item_lds1(const BatchItem& it) {
  if (it.code2 < 0) return batch_single_lds(it.N1, it.alpha, it.lines1);
  const int C = batch_lines(it.N1);
  return (size_t)pass1_lds_elems(it.N1, C,
                                 pass1_pre_elems(it.pre_lds, it.alpha, it.N1) + (it.q_lds ? it.alpha * C : 0) +
                                     (it.post_split ? pass1_post_elems(it.N1, C) : 0)) *
         8;
}
// (pass-2 tasks stage their stage twiddles after the row buffers)
inline size_t batch_lds2(int L) {
  return lds_pass2(L, batch_lines2(L), 4) + (size_t)pass2_tw_elems(L, batch_lines2(L), 0, 8) * 8;
}
inline size_t item_lds2(const BatchItem& it) { return it.code2 < 0 ? 0 : batch_lds2(it.N2); }

// Largest pass-2 LDS of any compiled pass-2 length (a server's fixed launch).
inline size_t batch_lds2_max() {
  size_t m = 0;
#define DD_L2(LL) m = std::max(m, batch_lds2(LL));
  DD_BATCH_P2(DD_L2)
#undef DD_L2
  return m;
}

// Task offsets of items already in queue order; fills the counts of meta.
inline void assign_task_offsets(BatchItem* items, int n, BatchMeta* meta) {
  int t1 = 0, t2 = 0;
  for (int k = 0; k < n; ++k) {
    items[k].t1 = t1;
    items[k].t2 = t2;
    t1 += items[k].p1_tasks;
    t2 += items[k].code2 < 0 ? 0 : items[k].ntile2;
  }
  meta->nitems = n;
  meta->n_first = t1;
  meta->n_second = t2;
  meta->pad_ = 0;
}

// Descriptor table of a batch launch: the host view in pinned, coherent
// (uncached on the device) memory that the staging kernel reads at launch,
// its device copy, and the two queue heads.
struct BatchTable {
  int cap = 0;
  BatchMeta* host = nullptr;      // host view: meta, then cap items
  const void* host_dev = nullptr; // the same memory as the device addresses it
  void* dev = nullptr;
  unsigned* ctl = nullptr;
  BatchItem* items() { return batch_table_items(host); }
};

inline void free_table(BatchTable& t) {
  if (t.host) (void)hipHostFree(t.host);
  if (t.dev) (void)hipFree(t.dev);
  if (t.ctl) (void)hipFree(t.ctl);
  t = BatchTable{};
}

inline dd_status alloc_table(BatchTable& t, int cap) {
  t.cap = cap;
  const size_t bytes = batch_table_bytes(cap);
  dd_status st = hip_status(hipHostMalloc((void**)&t.host, bytes, hipHostMallocMapped | hipHostMallocCoherent));
  void* hd = nullptr;
  if (st == DD_OK) st = hip_status(hipHostGetDevicePointer(&hd, t.host, 0));
  t.host_dev = hd;
  if (st == DD_OK) st = hip_status(hipMalloc(&t.dev, bytes));
  if (st == DD_OK) st = hip_status(hipMalloc((void**)&t.ctl, sizeof(unsigned) * 2));
  if (st == DD_OK) std::memset(t.host, 0, bytes);
  if (st != DD_OK) free_table(t);
  return st;
}

}  // namespace dd
