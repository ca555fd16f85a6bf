// dd_launch.hpp -- host-side launch entry points for the templated kernels.
//
// Each kernel is instantiated for a fixed set of line lengths; the host picks
// the instantiation with a switch on the runtime length.  Launchers return
// hipErrorInvalidValue for a length that is not instantiated.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#include "dd_kernels.hpp"

namespace dd {

// Every line length a kernel is built for: 2^a (1..4096), 3*2^a (3..3072),
// 5*2^a (5..2560).
#define DD_ALL_LENGTHS(X)                                                                   \
  X(1) X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(3) \
  X(6) X(12) X(24) X(48) X(96) X(192) X(384) X(768) X(1536) X(3072) X(5) X(10) X(20)     \
  X(40) X(80) X(160) X(320) X(640) X(1280) X(2560)

// Lengths of the second pass (powers of two).
#define DD_POW2_LENGTHS(X) \
  X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

struct LaunchCfg {
  int64_t grid;
  int block;
  size_t lds;
  hipStream_t stream;
};

struct KGeom {
  int TL;       // threads per line
  int lines;    // default lines per block
  int block;    // compile-time block size bound of the kernel
};

bool len_supported(int L);
bool pass2_len_supported(int L);
KGeom geom_single(int L, int rbytes);
KGeom geom_pass(int L, int rbytes);
KGeom geom_pass2(int L, int rbytes);  // forward pass 2 of complex input (lines_pass2)

// Overloads per arithmetic type R (float, double) and input type (real R or
// complex cx<R>); defined in dd_single_*.hip / dd_pass_*.hip.
#define DD_DECL_LAUNCHERS(R)                                                                     \
  hipError_t launch_single(int L, const LaunchCfg& c, const R* x, cx<R>* X, const DenseArgs<R>& a);     \
  hipError_t launch_single(int L, const LaunchCfg& c, const cx<R>* x, cx<R>* X, const DenseArgs<R>& a); \
  hipError_t launch_pass1(int L, const LaunchCfg& c, const R* x, cx<R>* Y, const DenseArgs<R>& a);      \
  hipError_t launch_pass1(int L, const LaunchCfg& c, const cx<R>* x, cx<R>* Y, const DenseArgs<R>& a);  \
  hipError_t launch_pass2(int L, const LaunchCfg& c, const cx<R>* Y, cx<R>* X, const DenseArgs<R>& a);  \
  hipError_t launch_pass2_half(int L, const LaunchCfg& c, const cx<R>* Y, cx<R>* X, const DenseArgs<R>& a); \
  hipError_t launch_twiddle(cx<R>* out, int64_t rows, int64_t cols, int64_t r0, int64_t den, int fp32, \
                            hipStream_t s);
DD_DECL_LAUNCHERS(float)
DD_DECL_LAUNCHERS(double)
#undef DD_DECL_LAUNCHERS
// Blocks of the one-pass kernel (real or complex input, arithmetic of the
// tag's type) resident per CU at this block and LDS size; 0 if unknown.
int single_occupancy(int L, bool real, float tag, int block, size_t lds);
int single_occupancy(int L, bool real, double tag, int block, size_t lds);

struct BatchItem;
struct BatchMeta;
// Persistent batch (dd_batch.hip).  batch_set_lds raises the two queue
// kernels' dynamic-LDS limits to lds1 / lds2 bytes when needed (call it
// before launching or capturing launch_batch with those sizes).
// launch_batch: the staging kernel (copies the descriptor table of `cap`
// items from its pinned host view `tab_host` to `tab_dev`, clears the two
// queue heads in ctl), then the first queue kernel over the single-pass and
// pass-1 tasks, then (grid2 > 0) the second over the pass-2 tasks.
// batch_max_blocks_per_cu: occupancy of queue kernel `which` (0, 1).
hipError_t batch_set_lds(size_t lds1, size_t lds2);
hipError_t launch_batch(const void* tab_host, void* tab_dev, int cap, unsigned* ctl, int grid1, int grid2,
                        size_t lds1, size_t lds2, hipStream_t s);
int batch_max_blocks_per_cu(int which, size_t lds);

// LDS bytes of each kernel for a given length and lines per block.
// One pass: `lines` signals per block, `groups` exchange rows per signal.
inline size_t lds_single(int L, int lines, int alpha, int rbytes, int groups = 1) {
  return (size_t)lines * ((size_t)groups * (L + L / 16 + 1) + (size_t)alpha * L) * 2 * rbytes;
}
inline size_t lds_pass1(int L, int lines, int rbytes, int pre_elems) {
  return (size_t)pass1_lds_elems(L, lines, pre_elems) * 2 * rbytes;
}
inline size_t lds_pass2(int L, int lines, int rbytes, int rows = 0) {
  return (size_t)pass2_lds_elems(L, lines, rows) * 2 * rbytes;
}

// Pad of the two-pass scratch rows (elements).  The lanes of a pass-1
// wavefront store rows alpha * (N2 + pad) elements apart; with whole rows of
// N2 that stride is a power of two, and for long row groups every store of
// the wavefront falls on one memory channel (measured for the scratch writes
// of 2^22 x alpha 16 alone: 16-byte pieces 630 -> 234 us, 32-byte pieces
// 531 -> 171 us, 64-byte pieces 241 -> 137 us with 512 bytes per row; row
// groups below 64 KiB showed no effect).  Only rows of at least 4 KiB get
// the pad, so it adds at most 1/8 to the scratch.
inline int64_t scratch_row_pad(int64_t N2, int alpha, int cx_bytes) {
  const int64_t rb = N2 * cx_bytes;
  return rb >= 4096 && alpha * rb >= 64 * 1024 ? 512 / cx_bytes : 0;
}
// Scratch bytes that one signal's two-pass execution needs at most, whatever
// its split, given its unpadded spectrum of `bytes`.
inline size_t scratch_bytes_bound(size_t bytes) { return bytes >= 64 * 1024 ? bytes + bytes / 8 : bytes; }

// A dispatch's grid size is a 32-bit count of work-items; launches are kept
// below 2^31 of them, and larger batches are split over several launches.
constexpr int64_t MAX_LAUNCH_ITEMS = 0x7fffffff;
inline int64_t max_launch_blocks(int block) { return block > 0 ? MAX_LAUNCH_ITEMS / block : 0; }

// With DD_DEBUG set in the environment, a failed launch is reported on
// stderr with its geometry.
inline hipError_t report_launch(hipError_t e, const char* what, const LaunchCfg& c) {
  if (e != hipSuccess && std::getenv("DD_DEBUG"))
    std::fprintf(stderr, "dense_dft: %s failed: %s (grid %lld, block %d, LDS %zu bytes)\n", what,
                 hipGetErrorString(e), (long long)c.grid, c.block, c.lds);
  return e;
}

// Kernel launch with the dynamic-LDS attribute raised when needed.
template <typename K, typename... Args>
inline hipError_t launch_kernel(K kern, const LaunchCfg& c, Args... args) {
  if (c.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds);
    if (e != hipSuccess) {
      (void)hipGetLastError();  // do not leave the error for the next launch to report
      return report_launch(e, "raising the LDS limit", c);
    }
  }
  if (c.grid <= 0) return hipSuccess;
  if (c.grid > max_launch_blocks(c.block)) return report_launch(hipErrorInvalidConfiguration, "grid size", c);
  hipLaunchKernelGGL(kern, dim3((unsigned)c.grid), dim3(c.block), c.lds, c.stream, args...);
  return report_launch(hipGetLastError(), "kernel launch", c);
}

}  // namespace dd
