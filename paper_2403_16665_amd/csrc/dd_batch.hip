// dd_batch.hip -- the persistent batch kernel and its launchers.
#include <mutex>

#include "dd_batch.hpp"
#include "dd_launch.hpp"

namespace dd {

// Refresh the device copy of a batch's descriptor table from the pinned host
// table (read over the bus at launch time, so that a captured graph picks up
// whatever the host wrote before the replay), with the item count clamped to
// the table's capacity, and clear the two queue heads.
__global__ __launch_bounds__(256) void k_batch_stage(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                     int cap, unsigned* __restrict__ ctl) {
  __shared__ int s_n;
  if (threadIdx.x == 0) {
    const int n = reinterpret_cast<const BatchMeta*>(src)->nitems;
    s_n = n < 0 ? 0 : (n > cap ? cap : n);
  }
  __syncthreads();
  const int words = (int)((sizeof(BatchMeta) + sizeof(BatchItem) * (size_t)s_n + 15) / 16);
  constexpr int META_WORDS = (int)(sizeof(BatchMeta) / 16);
  for (int i = META_WORDS + blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x)
    dst[i] = src[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    BatchMeta m = *reinterpret_cast<const BatchMeta*>(src);
    m.nitems = s_n;
    *reinterpret_cast<BatchMeta*>(dst) = m;
  }
  if (blockIdx.x == 0 && threadIdx.x < 2) ctl[threadIdx.x] = 0u;
}

// One task of each code path.
__device__ __forceinline__ DenseArgs<float> item_args(const BatchItem& it) {
  DenseArgs<float> a{};
  a.batch = 1;
  a.x_stride = it.N;
  a.y_stride = (int64_t)it.alpha * it.N;
  a.ysig = (int64_t)it.alpha * it.N;
  a.yrow = it.N2;
  a.N1 = it.N1;
  a.N2 = it.N2;
  a.alpha = it.alpha;
  a.jgroup = it.jgroup;
  a.njg = it.njg;
  a.pre_lds = it.pre_lds;
  a.q_lds = it.q_lds;
  a.post_split = it.post_split;
  a.scale = it.scale;
  a.twPre = as_global(it.twPre);
  a.twQ = as_global(it.twQ);
  a.twPost = as_global(it.twPost);
  return a;
}

template <int L>
__device__ __forceinline__ void run_single(const BatchItem* __restrict__ items, int item, int sub, unsigned char* smem,
                                           int tid) {
  const BatchItem& it = items[item];
  DenseArgs<float> a = item_args(it);
  a.lines = 1;
  a.twL = as_global(it.twL1);
  body_single_groups<float, AnyIn<float>, L>(AnyIn<float>{as_global(it.x), it.real}, as_global(it.X), a, sub,
                                             it.lines1, BATCH_THREADS, smem, tid);
}

template <int L>
__device__ __forceinline__ void run_pass1(const BatchItem* __restrict__ items, int item, int sub, unsigned char* smem,
                                          int tid) {
  const BatchItem& it = items[item];
  DenseArgs<float> a = item_args(it);
  a.lines = batch_lines(L);
  a.ntile = it.ntile1;
  a.twL = as_global(it.twL1);
  body_pass1<float, AnyIn<float>, L, batch_lines(L)>(AnyIn<float>{as_global(it.x), it.real}, as_global(it.Y), a,
                                                     sub, smem, tid);
}

template <int L>
__device__ __forceinline__ void run_pass2(const BatchItem* __restrict__ items, int item, int sub, unsigned char* smem,
                                          int tid) {
  const BatchItem& it = items[item];
  DenseArgs<float> a = item_args(it);
  a.lines = batch_lines2(L);
  a.ntile = it.ntile2;
  a.twL = as_global(it.twL2);
  body_pass2<float, L, batch_lines2(L), batch_lines2(L), true>(as_global(it.Y), as_global(it.X), a, sub, smem,
                                                                tid);
}

// Persistent queue over the tasks of one launch (WHICH = 0: single-pass and
// pass-1 tasks; 1: pass-2 tasks): every block takes the next task until the
// queue is empty.  No task of a launch depends on another task of the same
// launch, so no block ever waits for another.  The pass-2 kernel holds only
// the light pass-2 paths, so it runs at the occupancy those allow; the first
// kernel holds the heavy paths and is held to two waves per SIMD (256 VGPRs).
template <int WHICH>
__device__ __forceinline__ void batch_loop(const BatchItem* __restrict__ items, const BatchMeta* __restrict__ meta,
                                           unsigned* __restrict__ head, unsigned char* smem) {
  __shared__ int s_task;
  const int nitems = meta->nitems;
  const int count = WHICH ? meta->n_second : meta->n_first;
  if (nitems <= 0) return;
  for (;;) {
    if (threadIdx.x == 0) s_task = (int)atomicAdd(head, 1u);
    __syncthreads();
    // uniform task index: the switch below is a scalar branch, not a
    // divergent one (which would merge the live ranges of every code path)
    const int ti = __builtin_amdgcn_readfirstlane(s_task);
    __syncthreads();  // every thread has read s_task before thread 0 overwrites it
    if (ti >= count) break;
    // item: the last k with t[k] <= ti (empty ranges are skipped by "last")
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      const int tm = WHICH ? items[mid].t2 : items[mid].t1;
      if (tm <= ti) lo = mid;
      else hi = mid - 1;
    }
    const int k = lo;
    const int sub = ti - (WHICH ? items[k].t2 : items[k].t1);
    const int code = WHICH ? items[k].code2 : items[k].code1;
    // The thread index passes through an opaque move every iteration, so that
    // no code path's thread-dependent address arithmetic is hoisted out of
    // the task loop (hoisted, the invariants of all paths stay live at once).
    int tid;
    asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
    if (WHICH == 0) {
      switch (code) {
#define DD_S(LL)                                  \
  case batch_code(BK_SINGLE, LL):                 \
    run_single<LL>(items, k, sub, smem, tid);     \
    break;
        DD_BATCH_SINGLE(DD_S)
#undef DD_S
#define DD_P1(LL)                                 \
  case batch_code(BK_PASS1, LL):                  \
    run_pass1<LL>(items, k, sub, smem, tid);      \
    break;
        DD_BATCH_P1(DD_P1)
#undef DD_P1
        default:
          break;
      }
    } else {
      switch (code) {
#define DD_P2(LL)                                 \
  case batch_code(BK_PASS2, LL):                  \
    run_pass2<LL>(items, k, sub, smem, tid);      \
    break;
        DD_BATCH_P2(DD_P2)
#undef DD_P2
        default:
          break;
      }
    }
  }
}

__global__ __launch_bounds__(BATCH_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void k_batch_first(
    const BatchItem* __restrict__ items, const BatchMeta* __restrict__ meta, unsigned* __restrict__ head) {
  extern __shared__ __align__(16) unsigned char smem[];
  batch_loop<0>(items, meta, head, smem);
}

__global__ __launch_bounds__(BATCH_THREADS2) void k_batch_second(const BatchItem* __restrict__ items,
                                                                const BatchMeta* __restrict__ meta,
                                                                unsigned* __restrict__ head) {
  extern __shared__ __align__(16) unsigned char smem[];
  batch_loop<1>(items, meta, head, smem);
}

hipError_t batch_set_lds(size_t lds1, size_t lds2) {
  // dynamic LDS plus the kernels' static word beyond the default 64 KiB
  // needs the attribute; it is set outside any stream capture.  The limits
  // only ever rise: a server's captured graphs launch with the largest
  // sizes, and a batch plan or tuner run made beside it must not lower them.
  // Tracked per device (the attribute is set on the current one).
  constexpr int MAXDEV = 64;
  static std::mutex mu;
  static size_t cur1[MAXDEV] = {}, cur2[MAXDEV] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (lds1 + 64 > 64 * 1024 && lds1 > cur1[dev]) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_batch_first), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds1);
    if (e == hipSuccess) cur1[dev] = lds1;
  }
  if (e == hipSuccess && lds2 + 64 > 64 * 1024 && lds2 > cur2[dev]) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_batch_second),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
    if (e == hipSuccess) cur2[dev] = lds2;
  }
  return e;
}

hipError_t launch_batch(const void* tab_host, void* tab_dev, int cap, unsigned* ctl, int grid1, int grid2,
                        size_t lds1, size_t lds2, hipStream_t s) {
  const int words = (int)(batch_table_bytes(cap) / 16);
  const int gstage = (words + 1023) / 1024;
  hipLaunchKernelGGL(k_batch_stage, dim3(gstage), dim3(256), 0, s, static_cast<const uint4*>(tab_host),
                     static_cast<uint4*>(tab_dev), cap, ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const BatchMeta* meta = static_cast<const BatchMeta*>(tab_dev);
  const BatchItem* items = batch_table_items(meta);
  hipLaunchKernelGGL(k_batch_first, dim3(grid1), dim3(BATCH_THREADS), lds1, s, items, meta, ctl);
  e = hipGetLastError();
  if (e != hipSuccess || grid2 <= 0) return e;
  hipLaunchKernelGGL(k_batch_second, dim3(grid2), dim3(BATCH_THREADS2), lds2, s, items, meta, ctl + 1);
  return hipGetLastError();
}

int batch_max_blocks_per_cu(int which, size_t lds) {
  int n = 0;
  const hipError_t e =
      which ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_second, BATCH_THREADS2, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_first, BATCH_THREADS, lds);
  if (e != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

}  // namespace dd
