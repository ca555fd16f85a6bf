// dd_batch.hpp -- persistent batched execution of many alpha-dense DFTs of
// uneven N and alpha in one launch (definitions shared by host and device).
//
// Every signal of a batch is an "item" with its own schedule (one pass, or
// two passes N = N1 N2) and twiddle tables.  Its work is cut into block-sized
// tasks: single-pass signals, pass-1 column tiles and pass-2 row blocks.  A
// launch runs a fixed grid of blocks (256 threads in the first queue kernel,
// 512 in the second) that take tasks
// from a device queue until it is empty.  The single-pass and pass-1 tasks of
// all items form the first launch, the pass-2 tasks the second, so the kernel
// boundary publishes every scratch row before it is read and no block ever
// waits for another.
#pragma once

#include "dd_kernels.hpp"

namespace dd {

constexpr int BATCH_THREADS = 256;
// The first queue kernel holds two blocks per CU (its register use), so a
// block may take up to half of the CU's 160 KiB of LDS.
constexpr int BATCH_LDS_MAX = 80 * 1024;

// Lengths compiled into the batch kernel, per kind.
#define DD_BATCH_SINGLE(X) \
  X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(384) X(768) X(1536) X(3072) X(320) X(640) X(1280) X(2560)
#define DD_BATCH_P1(X) X(16) X(32) X(64) X(128) X(256) X(512) X(24) X(48) X(96) X(192) X(384) X(20) X(40) X(80) X(160) X(320)
#define DD_BATCH_P2(X) X(32) X(64) X(128) X(256) X(512)

enum BatchKind { BK_SINGLE = 0, BK_PASS1 = 1, BK_PASS2 = 2 };

// code = kind * 64 + L's position in the kind's list; -1 if not compiled.
__host__ __device__ constexpr int batch_code(int kind, int L) {
  int i = 0;
#define DD_POS(LL) \
  if (LL == L) return kind * 64 + i; \
  ++i;
  if (kind == BK_SINGLE) {
    DD_BATCH_SINGLE(DD_POS)
  } else if (kind == BK_PASS1) {
    DD_BATCH_P1(DD_POS)
  } else if (kind == BK_PASS2) {
    DD_BATCH_P2(DD_POS)
  }
#undef DD_POS
  return -1;
}

// Lines per 256-thread block for a pass kernel of length L.
__host__ __device__ constexpr int batch_lines(int L) { return BATCH_THREADS / line_threads(L); }
// The pass-2 queue kernel runs blocks of 512 threads (its rows hold no
// tables, so a wave needs few registers): rows per task for length L.  At
// L = 512 that is 16 rows, so its scattered output stores are whole 128-byte
// lines (with 8 rows, 64-byte pieces: measured 1.5x the time per byte).
constexpr int BATCH_THREADS2 = 512;
__host__ __device__ constexpr int batch_lines2(int L) { return BATCH_THREADS2 / line_threads(L); }
// Thread groups sharing one single-pass signal of length L (each takes its
// own values of j): as many as the block holds, but no more than alpha needs
// (rounded up to a power of two) and no more than the LDS holds; 0 if not
// even one fits.  A switch over the compiled lengths: the layout's row
// stride is a compile-time constant.
__host__ __device__ inline int batch_single_groups(int L, int alpha) {
  switch (L) {
#define DD_SG(LL)                                                                                        \
  case LL: {                                                                                             \
    int g = BATCH_THREADS / single_line_threads(LL);                                                     \
    while (g > 1 && (g / 2 >= alpha || (size_t)single_groups_lds_elems<LL>(g, alpha) * 8 > (size_t)BATCH_LDS_MAX)) \
      g /= 2;                                                                                            \
    return (size_t)single_groups_lds_elems<LL>(g, alpha) * 8 <= (size_t)BATCH_LDS_MAX ? g : 0;          \
  }
    DD_BATCH_SINGLE(DD_SG)
#undef DD_SG
    default:
      return 0;
  }
}

// LDS bytes of a single-pass task of length L with `groups` thread groups.
__host__ __device__ inline size_t batch_single_lds(int L, int alpha, int groups) {
  switch (L) {
#define DD_SL(LL) \
  case LL:        \
    return (size_t)single_groups_lds_elems<LL>(groups, alpha) * 8;
    DD_BATCH_SINGLE(DD_SL)
#undef DD_SL
    default:
      return (size_t)-1;
  }
}

// Device descriptor of one signal of a batch (FP32 arithmetic; real float or
// complex float input).
struct BatchItem {
  const void* x;          // [N] input
  cx<float>* X;           // [alpha N] output
  cx<float>* Y;           // [alpha N] scratch (two-pass items)
  const cx<float>* twL1;  // stage twiddles of the N1 line (N for one pass)
  const cx<float>* twPre; // [j][n1] W_{alpha N1}^{j n1}
  const cx<float>* twQ;   // [j][n2] W_{alpha N}^{j n2}
  const cx<float>* twPost;// [k1][n2] W_N^{k1 n2}
  const cx<float>* twL2;  // stage twiddles of the N2 line
  int64_t N;
  int N1, N2, alpha, real;
  int lines1, ntile1, jgroup, njg, pre_lds;  // one pass: lines1 = thread groups sharing the signal
  int q_lds;              // pass 1: W_{alpha N}^{j n2} of a task's columns staged in LDS
  int post_split;         // pass 1: W_N^{k1 n2} as the product of two table rows (DenseArgs)
  int ntile2;
  int p1_tasks;           // pass-1 tasks of the item
  int code1, code2;       // code paths: single or pass 1; pass 2 (-1: one pass)
  int t1, t2;             // index of the item's first task in launch 1 / launch 2
  float scale;            // T / N
};

// Per-execution counts, read by the kernels from device memory (so that one
// captured graph serves batches of any composition).
struct BatchMeta {
  int nitems;             // items in the table, ordered by t1 (and t2)
  int n_first;            // tasks of launch 1: single-pass signals and pass-1 tiles
  int n_second;           // tasks of launch 2: pass-2 row blocks
  int pad_;
};

// Item k owns tasks [t1[k], t1[k+1]) of launch 1 and [t2[k], t2[k+1]) of
// launch 2; a block maps a task index to its item by binary search.
// Control words: [0] queue head of the first launch, [1] of the second.

// Descriptor table of one launch: a BatchMeta, then `cap` items; its size is
// rounded to whole 16-byte words.
static_assert(sizeof(BatchMeta) == 16, "the table header is one 16-byte word");
__host__ __device__ constexpr size_t batch_table_bytes(int cap) {
  return (sizeof(BatchMeta) + sizeof(BatchItem) * (size_t)cap + 15) / 16 * 16;
}
__host__ __device__ inline const BatchItem* batch_table_items(const BatchMeta* m) {
  return reinterpret_cast<const BatchItem*>(m + 1);
}
__host__ __device__ inline BatchItem* batch_table_items(BatchMeta* m) { return reinterpret_cast<BatchItem*>(m + 1); }

}  // namespace dd
