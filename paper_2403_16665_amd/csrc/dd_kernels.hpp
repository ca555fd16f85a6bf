// dd_kernels.hpp -- the alpha-dense DFT kernels for gfx950.
//
// Method (paper Section 3, eq. (9)-(13), unrolled): with m = alpha k + j,
//   X_{alpha k + j} = (T/N) sum_n [x_n W_{alpha N}^{j n}] W_N^{k n},
// i.e. alpha pre-twiddled length-N FFTs whose outputs interleave.  The
// pre-twiddle is the first, pruned level of the paper's recursion: the level
// whose inputs are one sample and (alpha-1) implied zeros (Section 4) is
// just this multiply.
//
// Single pass (whole signal in one block): for each j, pre-twiddle, length-N
// Stockham FFT in registers + LDS, write into an LDS image of the alpha*N
// spectrum at alpha k + j; then one coalesced store of the whole spectrum.
//
// Two passes, N = N1 N2, n = N2 n1 + n2, m = m1 + alpha N1 k2 with
// m1 = alpha k1 + j (the same identity applied to the four-step split):
//   pass 1: for each column n2, the alpha-dense DFT of length N1 of
//           x[N2 n1 + n2] (alpha pre-twiddled N1-point FFTs), times the
//           inter-pass twiddle W_{alpha N}^{m1 n2} = W_N^{k1 n2} W_{alpha N}^{j n2}
//           -> scratch Y[m1][n2]
//   pass 2: for each row m1, the plain N2-point FFT over n2
//           -> X[m1 + alpha N1 k2], stored as contiguous runs of rows.
// Every twiddle exponent is an exact integer below its modulus.
#pragma once

#include <type_traits>

#include "dd_fft.hpp"

namespace dd {

template <typename R>
struct DenseArgs {
  int64_t batch;      // signals handled by this launch
  int64_t x_stride;   // input elements between signals
  int64_t y_stride;   // complex elements between signals of the output
  int64_t ysig;       // two passes: complex elements between signals of the scratch
  int yrow;           // two passes: complex elements between scratch rows m1 (N2, or N2 and a pad
                      // that keeps the rows of a wavefront's stores off one memory channel)
  int N1, N2, alpha;
  int lines;          // lines per block: signals (single), columns (pass 1), rows (pass 2)
  int ntile;          // column tiles (pass 1) or row blocks (pass 2) per signal
  int jgroup, njg;    // pass 1: j values per block and number of j groups; one pass: thread groups
                      // sharing a signal (jgroup; group g takes j = g, g + jgroup, ...)
  int pre_lds;        // pass 1: pre-twiddles of the block's j range staged in LDS: 1 whole rows,
                      // 2 the entries n1 < TL and n1 = TL e of each row (their product is the factor)
  int q_lds;          // pass 1: W_{alpha N}^{j n2} of the block's j range and columns staged in LDS
                      // (a global load inside the j loop would wait for the previous j's stores:
                      // loads and stores share one in-order counter)
  int post_split;     // pass 1: W_N^{k1 n2} of element k1 = t + TL e formed as the product of the
                      // table's rows t and TL e (the block's columns of rows TL e staged in LDS),
                      // so that a block reads TL + EPT rows of the table instead of N1
  int hrows;          // 0: every row m1 of the scratch; real input: floor(alpha N1 / 2) + 1, the rows
                      // m1 <= alpha N1 / 2 that pass 1 stores and pass 2 transforms (the others are
                      // conjugate mirrors, X_{alpha N - m} = conj(X_m))
  R scale;            // T / N
  const cx<R>* twL;   // stage twiddles of the line FFT of this kernel ([s][k] per stage)
  const cx<R>* twPre; // W_{alpha N1}^{j n1}, laid out [j][n1]
  const cx<R>* twQ;   // W_{alpha N}^{j n2}, laid out [j][n2]
  const cx<R>* twPost;// W_N^{k1 n2}, laid out [k1][n2]
};

// A pointer into global memory, so marked for the compiler.  A pointer a kernel
// reads from a descriptor in memory (not a kernel argument) is generic to it,
// and generic accesses compile to flat loads and stores, which count on the LDS
// counter as well as the memory counter: the LDS wait before every exchange
// barrier then also waits for all stores still in flight.  The pointer passes
// through the global address space behind an empty asm (a plain cast pair, or
// an assumption on the address, is folded away before the compiler infers
// address spaces), so every access derived from it is a global one.  The
// pointers it is used on are uniform: the asm keeps them in scalar registers.
template <typename T>
__device__ __forceinline__ T* as_global(T* p) {
  __attribute__((address_space(1))) T* g;
  asm("" : "=s"(g) : "0"((__attribute__((address_space(1))) T*)p));
  return (T*)g;
}

// Store of a final output bin, marked non-temporal: the spectrum is not read
// again by the transform, and keeping it out of the caches leaves the
// Infinity Cache to the scratch that pass 2 reads back (measured: pass 2 of a
// 64-signal chunk 125 -> 87 us).
template <typename R>
__device__ __forceinline__ void store_out(cx<R>* p, cx<R> v) {
  R* q = reinterpret_cast<R*>(p);
  __builtin_nontemporal_store(v.re, q);
  __builtin_nontemporal_store(v.im, q + 1);
}

// Load of a value read once (the spectra the inverse transform consumes),
// marked non-temporal for the same reason (the inverse of the default shape:
// 0.811 -> 0.768 ms, pass B finding more of its scratch in the cache).
template <typename R>
__device__ __forceinline__ cx<R> load_once(const cx<R>* p) {
  const R* q = reinterpret_cast<const R*>(p);
  return {__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1)};
}

template <typename R> __device__ __forceinline__ cx<R> load_in(const float* p, int64_t i) { return {(R)p[i], (R)0}; }
template <typename R> __device__ __forceinline__ cx<R> load_in(const double* p, int64_t i) { return {(R)p[i], (R)0}; }
template <typename R> __device__ __forceinline__ cx<R> load_in(const cx<float>* p, int64_t i) { cx<float> v = p[i]; return {(R)v.re, (R)v.im}; }
template <typename R> __device__ __forceinline__ cx<R> load_in(const cx<double>* p, int64_t i) { cx<double> v = p[i]; return {(R)v.re, (R)v.im}; }

// Input accessors: element (base + off) of a signal's samples as cx<R>.  The
// base is uniform across the block, the offset per lane (keeps the address
// arithmetic in scalar registers).
template <typename R, typename In>
struct PtrIn {
  const In* p;
  __device__ __forceinline__ cx<R> operator()(int64_t base, unsigned off) const { return load_in<R>(p + base, off); }
  __device__ __forceinline__ bool is_real() const { return std::is_floating_point<In>::value; }
};
// Runtime choice between real float and complex float samples (mixed batches).
template <typename R>
struct AnyIn {
  const void* p;
  int real;
  __device__ __forceinline__ cx<R> operator()(int64_t base, unsigned off) const {
    return real ? load_in<R>(static_cast<const float*>(p) + base, off)
                : load_in<R>(static_cast<const cx<float>*>(p) + base, off);
  }
  __device__ __forceinline__ bool is_real() const { return real != 0; }
};

// LDS elements of pass 1 for a tile of C columns (host and device): the
// exchange buffer, the stage twiddles and `pre` staged pre-twiddles.
__host__ __device__ constexpr int pass1_lds_elems(int L, int C, int pre) {
  return L * C + (L / 16 + 1) * 8 + line_tw_size(make_line_plan(L)) + pre;
}

// LDS elements of pass 2 for blocks of RB rows that transform `rows` rows
// (RB, or RB + 1 for real input): the row exchange buffers, reused as the
// staging buffer of the transposed store.
__host__ __device__ constexpr int pass2_lds_elems(int L, int RB, int rows = 0) {
  return (rows ? rows : RB) * (L + L / 16 + 1) > L * (RB + 1) ? (rows ? rows : RB) * (L + L / 16 + 1)
                                                             : L * (RB + 1);
}
// Stage twiddles of a pass-2 task staged in LDS after its row buffers (the
// batch kernel's pass-2 tasks), when both fit a CU's LDS: entries, 0 if not.
__host__ __device__ constexpr int pass2_tw_elems(int L, int RB, int rows, int cx_bytes) {
  return (pass2_lds_elems(L, RB, rows) + line_tw_size(make_line_plan(L))) * cx_bytes <= 160 * 1024
             ? line_tw_size(make_line_plan(L)) : 0;
}

// LDS of one block of a pass kernel may take all of a CU's 160 KiB: the wider
// the tile, the longer the contiguous runs of its scattered stores.
constexpr int LDS_PASS_MAX = 160 * 1024;

constexpr int line_threads(int L) { return L / make_line_plan(L).EPT; }
// LDS elements of pass 1's staged pre-twiddles for jg values of j: mode 1
// whole rows W_{alpha N1}^{j n1}, mode 2 the entries n1 < TL and n1 = TL e
// of each row (TL threads per line, EPT elements each), 0 none.
constexpr int pass1_pre_elems(int mode, int jg, int L) {
  return mode == 1 ? jg * L : mode == 2 ? jg * (line_threads(L) + L / line_threads(L)) : 0;
}
// LDS elements of pass 1's staged rows TL e of the [k1][n2] table for C
// columns (post_split), EPT elements per thread.
constexpr int pass1_post_elems(int L, int C) { return (L / line_threads(L)) * C; }
// Threads per line of the one-pass kernels (their plan: single_narrow).
constexpr int single_line_threads(int L) { return L / make_line_plan(L, single_narrow(L)).EPT; }

// Launch geometry shared by host and device.
template <int L, int RBYTES>
struct Geom {
  static constexpr int TL = line_threads(L);
  static constexpr int CX = 2 * RBYTES;
  static constexpr int pass_lds(int lines) {
    return CX * (pass1_lds_elems(L, lines, 0) > pass2_lds_elems(L, lines) ? pass1_lds_elems(L, lines, 0)
                                                                           : pass2_lds_elems(L, lines));
  }
  // pass 1 / pass 2: aim for 16 lines, at most 512 threads (so that a wave
  // may hold 256 VGPRs), LDS within a CU
  static constexpr int lines_pass() {
    int l = 16;
    if (TL * l < 256) l = 256 / TL;
    while (l > 1 && TL * l > 512) l /= 2;
    while (l > 1 && pass_lds(l) > LDS_PASS_MAX) l /= 2;
    return l;
  }
  static constexpr int BLOCK_PASS = TL * lines_pass();
  // forward pass 2 alone: up to 1024 threads (its rows hold no tables, so a
  // wave needs few registers), LDS within a CU -- the more rows per block,
  // the longer the contiguous runs of its scattered output stores
  static constexpr int lines_pass2() {
    int l = 16;
    if (TL * l < 256) l = 256 / TL;
    while (l > 1 && TL * l > 1024) l /= 2;
    while (l > 1 && CX * pass2_lds_elems(L, l) > LDS_PASS_MAX) l /= 2;
    return l;
  }
  // single pass: up to 256 threads (one line if TL >= 256)
  static constexpr int TLS = single_line_threads(L);
  static constexpr int lines_single() { return TLS >= 256 ? 1 : 256 / TLS; }
  static constexpr int BLOCK_SINGLE = TLS * lines_single();
};

// ---------------------------------------------------------------------------
// Block bodies.  `bid` is the block's index in its launch (or the task index
// of a persistent batch), `nt` the number of threads taking part, `smem` the
// dynamic LDS base, `tid` the thread's index in the block.
// ---------------------------------------------------------------------------

// Single pass: block = a.lines signals, each shared by a.jgroup groups of TL
// threads; group g of a signal takes the values j = g, g + jgroup, ... and
// thread t of a group owns samples t + TL e.  LDS: one exchange row per group
// (RowLayout), then the lines' spectrum images.  The block first loads its
// signals' samples into the head of their images (one coalesced read of each
// sample, however many groups share the signal).  Threads beyond
// a.lines * a.jgroup * TL only take part in synchronisation.
template <typename R, class InAcc, int L>
__device__ __forceinline__ void body_single(const InAcc& x, cx<R>* __restrict__ X, const DenseArgs<R>& a,
                                            int64_t bid, int nt, unsigned char* smem, int tid) {
  constexpr LinePlan P = make_line_plan(L, single_narrow(L));
  constexpr int EPT = P.EPT;
  constexpr int TL = L / EPT;
  const int G = a.jgroup;
  cx<R>* ex = reinterpret_cast<cx<R>*>(smem);
  cx<R>* img = ex + RowLayout<L>::elems(a.lines * G);
  const int t = tid % TL, gi = tid / TL, line = gi / G, g = gi % G;
  const bool member = line < a.lines;
  const int64_t sig0 = bid * a.lines;
  const int64_t sig = sig0 + line;
  const bool active = member && sig < a.batch;
  const int M1 = a.alpha * L;
  const int64_t nl = min((int64_t)a.lines, a.batch - sig0);
  for (int i = tid; i < nl * L; i += nt) {
    const int sl = i / L, n = i - sl * L;
    img[sl * M1 + n] = cscale(x((sig0 + sl) * a.x_stride, (unsigned)n), a.scale);
  }
  __syncthreads();
  cx<R>* im = img + (int64_t)(member ? line : 0) * M1;
  cx<R> xv[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) xv[e] = active ? lds_read(im + t + TL * e) : cx<R>{(R)0, (R)0};
  __syncthreads();  // every group holds its samples before any writes its spectrum over them
  const RowLayout<L> lay(member ? gi : 0);
  // real samples: X_{alpha L - m} = conj(X_m), so with m = alpha k + j the
  // bins of alpha - j are conj(X_{alpha (L - 1 - k) + j}); only j <= alpha/2
  // are transformed, and each j in [1, alpha/2) also fills its mirror
  const bool herm = x.is_real();
  const int jmax = herm ? a.alpha / 2 : a.alpha - 1;
  for (int j0 = 0; j0 <= jmax; j0 += G) {  // uniform over the block
    const int j = j0 + g;
    const bool act = member && j <= jmax;
    cx<R> v[EPT];
    if (j == 0 || !act) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) v[e] = xv[e];
    } else {
      const cx<R>* __restrict__ pre = a.twPre + j * L + t;
#pragma unroll
      for (int e = 0; e < EPT; ++e) v[e] = cmul(xv[e], pre[TL * e]);
    }
    line_fft<R, L, (TL <= 64), single_narrow(L)>(v, t, ex, lay, a.twL, act);
    if (act) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) im[a.alpha * (t + TL * e) + j] = v[e];
      if (herm && j >= 1 && 2 * j < a.alpha) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) im[a.alpha * (L - 1 - t - TL * e) + a.alpha - j] = cconj(v[e]);
      }
    }
  }
  __syncthreads();
  const int64_t total = nl * M1;
  cx<R>* dst = X + sig0 * a.y_stride;  // y_stride == alpha * L
  for (int64_t i = tid; i < total; i += nt) store_out(dst + i, img[i]);
  __syncthreads();  // the image is reused by the next task of a persistent block
}

// One pass, one signal per block, `groups` groups of TL threads: group g
// takes the values j = g, g + groups, ... (the batch kernel's blocks have a
// fixed width, so the alpha pre-twiddled FFTs of one signal share it rather
// than leaving all but TL threads idle).  Threads beyond the groups take part
// in the barriers only.  LDS: one exchange row per group, then the alpha*L
// spectrum image, stored contiguously at the end.
template <int L>
__host__ __device__ constexpr int single_groups_lds_elems(int groups, int alpha) {
  return RowLayout<L>::elems(groups) + alpha * L;
}

template <typename R, class InAcc, int L>
__device__ __forceinline__ void body_single_groups(const InAcc& x, cx<R>* __restrict__ X, const DenseArgs<R>& a,
                                                   int64_t sig, int groups, int nt, unsigned char* smem, int tid) {
  constexpr LinePlan P = make_line_plan(L, single_narrow(L));
  constexpr int EPT = P.EPT;
  constexpr int TL = L / EPT;
  cx<R>* ex = reinterpret_cast<cx<R>*>(smem);
  cx<R>* img = ex + RowLayout<L>::elems(groups);
  const int t = tid % TL, g = tid / TL;
  const bool member = g < groups;
  const int M1 = a.alpha * L;
  // the samples pass through the head of the image: one coalesced read of
  // each, however many groups share the signal (as in body_single)
  for (int i = tid; i < L; i += nt) img[i] = cscale(x(sig * a.x_stride, (unsigned)i), a.scale);
  __syncthreads();
  cx<R> xv[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) xv[e] = member ? lds_read(img + t + TL * e) : cx<R>{(R)0, (R)0};
  __syncthreads();  // every group holds its samples before any writes its spectrum over them
  const RowLayout<L> lay(member ? g : 0);
  // real samples: only j <= alpha/2 are transformed (as in body_single)
  const bool herm = x.is_real();
  const int jmax = herm ? a.alpha / 2 : a.alpha - 1;
  for (int j0 = 0; j0 <= jmax; j0 += groups) {  // uniform over the block
    const int j = j0 + g;
    const bool act = member && j <= jmax;
    cx<R> v[EPT];
    if (j == 0 || !act) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) v[e] = xv[e];
    } else {
      const cx<R>* __restrict__ pre = a.twPre + j * L + t;
#pragma unroll
      for (int e = 0; e < EPT; ++e) v[e] = cmul(xv[e], pre[TL * e]);
    }
    line_fft<R, L, (TL <= 64), single_narrow(L)>(v, t, ex, lay, a.twL, act);
    if (act) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) img[a.alpha * (t + TL * e) + j] = v[e];
      if (herm && j >= 1 && 2 * j < a.alpha) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) img[a.alpha * (L - 1 - t - TL * e) + a.alpha - j] = cconj(v[e]);
      }
    }
  }
  __syncthreads();
  cx<R>* dst = X + sig * a.y_stride;  // y_stride == alpha * L
  for (int i = tid; i < M1; i += nt) store_out(dst + i, img[i]);
  __syncthreads();  // the image is reused by the next task of a persistent block
}

// Pass 1: block = (signal, tile of C columns n2, group of j values).  Thread
// (c, t) with c fastest owns column n2 = tile*C + c, samples n1 = t + TL e.
// Output Y[alpha k1 + j][n2] times the inter-pass twiddle
// W_{alpha N}^{m1 n2} = W_N^{k1 n2} W_{alpha N}^{j n2}.  (Applying it in pass 2
// instead was measured slower: pass 2 is the more loaded of the two.)
// Columns are fastest across the block so that every store instruction
// writes whole 128-byte lines of C columns.  (A wavefront-private column
// group would avoid the block barriers of the exchange but stores 32-byte
// pieces that reach memory as partial lines: measured 1.8x the write
// traffic.)
// HALF: the kernel may be given a.hrows > 0 (real input) and then stores
// only the rows m1 < a.hrows; without it every row is stored.  A real
// column's alpha-dense DFT is Hermitian, C[alpha N1 - m1] = conj(C[m1]), with
// alpha N1 - m1 = alpha (N1 - 1 - k1) + (alpha - j): when a block holds every
// j it transforms only j <= alpha / 2 and also stores the rows of alpha - j.
// The inter-pass twiddle of row alpha N1 - m1 is W_{N2}^{n2} times the
// conjugate of that of m1, so Y[alpha N1 - m1][n2] = conj(Y[m1][n2]) W_{N2}^{n2}
// and each thread stores those rows from its own values.  In double
// precision and for lines of 5 * 2^a (20 elements per thread) that costs
// occupancy or spills, so there the transform of j is reversed through LDS
// and twiddled for the rows of alpha - j.
// Copies n table entries into LDS with nt threads, U entries per thread per
// round: a round issues all its loads before the first LDS write waits for
// them (loads complete in order, so one wait covers the round).
template <typename R, int U, class Get>
__device__ __forceinline__ void stage_to_lds(cx<R>* dst, int n, int tid, int nt, Get get) {
  for (int i0 = tid; i0 < n; i0 += U * nt) {
    cx<R> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * nt;
      v[u] = i < n ? get(i) : cx<R>{(R)0, (R)0};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * nt;
      if (i < n) dst[i] = v[u];
    }
  }
}

template <typename R, class InAcc, int L, int C, bool HALF = false>
__device__ __forceinline__ void body_pass1(const InAcc& x, cx<R>* __restrict__ Y, const DenseArgs<R>& a,
                                           int64_t bid, unsigned char* smem, int tid) {
  constexpr LinePlan P = make_line_plan(L);
  constexpr int EPT = P.EPT;
  constexpr int TL = L / EPT;
  constexpr int NT = C * TL;
  constexpr int TWN = line_tw_size(P);
  cx<R>* ex = reinterpret_cast<cx<R>*>(smem);
  cx<R>* tws = ex + ColLayout<C>::elems(L);   // stage twiddles
  cx<R>* pre = tws + TWN;                     // [j - j0][n1] pre-twiddles (when a.pre_lds)
  const int jg = (int)(bid % a.njg);
  bid /= a.njg;
  const int tile = (int)(bid % a.ntile);
  const int64_t sig = bid / a.ntile;
  const int c = tid % C, t = tid / C;
  const int N2 = a.N2;
  const int n2 = tile * C + c;
  const ColLayout<C> lay(c);
  const int j0 = jg * a.jgroup;
  const int j1 = min(a.alpha, j0 + a.jgroup);

  // the block's column.  Long columns (many loads per thread, from HBM) are
  // issued before the tables below, so that their latency overlaps the
  // tables' (2^22 x alpha 16, pass 1 at N1 = 2048 197 -> 189 us); short ones
  // after (at N1 = 128 first cost 39.5 against 38.8 us per chunk).
  constexpr bool COL_FIRST = L >= 1024;
  const bool colok = n2 < N2;  // a tile wider than N2 has idle columns
  cx<R> xv[EPT], pw[EPT];
  const unsigned in_off = (unsigned)(N2 * t + n2);          // lane part of N2 n1 + n2
  const unsigned in_step = (unsigned)(N2 * TL);             // n1 -> n1 + TL
  auto load_column = [&]() {
    if (colok) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) xv[e] = x(sig * a.x_stride + (int64_t)in_step * e, in_off);
      if (a.post_split) {
        pw[0] = a.twPost[in_off];  // W_N^{t n2}; the other elements after the staging
      } else {
#pragma unroll
        for (int e = 0; e < EPT; ++e) pw[e] = (a.twPost + in_step * e)[in_off];  // W_N^{k1 n2}, k1 = t + TL e
      }
    } else {
#pragma unroll
      for (int e = 0; e < EPT; ++e) xv[e] = pw[e] = {(R)0, (R)0};
    }
  };
  if constexpr (COL_FIRST) load_column();

  // twiddle tables of this block into LDS (read every j; from L2 their latency
  // sits on the critical path of each iteration, and a global load inside
  // the j loop waits for the previous j's stores: loads and stores share one
  // in-order completion counter).  Each copy gathers several entries per
  // thread before it writes any, so that one wait covers their loads.
  stage_to_lds<R, 4>(tws, TWN, tid, NT, [&](int i) { return a.twL[i]; });
  int pre_n = 0;
  if (a.pre_lds == 1) {
    // the block's rows of W_{alpha N1}^{j n1}, whole
    pre_n = (j1 - j0) * L;
    stage_to_lds<R, 4>(pre, pre_n, tid, NT, [&](int i) { return a.twPre[j0 * L + i]; });
  } else if (a.pre_lds == 2) {
    // columns too long to stage whole: the entries n1 = t ([j - j0][t]) and
    // n1 = TL e ([j - j0][e]) of the same rows, whose product is the factor
    const int na = (j1 - j0) * TL, nb = (j1 - j0) * EPT;
    pre_n = na + nb;
    stage_to_lds<R, 4>(pre, pre_n, tid, NT, [&](int i) {
      return i < na ? a.twPre[(j0 + i / TL) * L + i % TL] : a.twPre[(j0 + (i - na) / EPT) * L + TL * ((i - na) % EPT)];
    });
  }
  cx<R>* qs = pre + pre_n;  // [j - j0][c] W_{alpha N}^{j n2} (when a.q_lds)
  const int nq = a.q_lds ? (j1 - j0) * C : 0;
  cx<R>* ps = qs + nq;      // [e][c] W_N^{TL e n2} (when a.post_split)
  const int np = a.post_split ? EPT * C : 0;
  // both in one copy: entries i < nq of qs, then the np of ps
  stage_to_lds<R, 4>(qs, nq + np, tid, NT, [&](int i) {
    if (i < nq) {
      const int col = tile * C + i % C;
      return col < a.N2 ? a.twQ[(j0 + i / C) * a.N2 + col] : cx<R>{(R)0, (R)0};
    }
    const int k = i - nq, col = tile * C + k % C;
    return col < a.N2 ? a.twPost[(int64_t)TL * (k / C) * a.N2 + col] : cx<R>{(R)0, (R)0};
  });

  if constexpr (!COL_FIRST) load_column();
#pragma unroll
  for (int e = 0; e < EPT; ++e) xv[e] = cscale(xv[e], a.scale);
  __syncthreads();
  if (a.post_split && colok) {
    // W_N^{(t + TL e) n2} = W_N^{t n2} W_N^{TL e n2}
#pragma unroll
    for (int e = EPT - 1; e >= 1; --e) pw[e] = cmul(pw[0], ps[e * C + c]);
  }
  const int S = a.yrow;  // scratch row stride
  const unsigned out_off = (unsigned)(a.alpha * S * t + n2);  // lane part of (alpha k1 + j) S + n2
  const unsigned out_step = (unsigned)(a.alpha * S * TL);
  cx<R>* ys = Y + sig * a.ysig;
  constexpr bool REG_MIRROR = HALF && sizeof(R) == 4 && L % 5 != 0;
  // SPLIT: with N1 and EPT even and hrows = alpha N1 / 2 + 1, every mirrored
  // j keeps the rows k1 < N1 / 2 (elements e < EPT / 2) and its partner
  // alpha - j the rows N1 - 1 - k1 < N1 / 2 (elements e >= EPT / 2): fixed
  // element ranges, no per-lane predicates
  constexpr bool SPLIT = REG_MIRROR && L % 2 == 0 && EPT % 2 == 0;
  const bool sym = HALF && a.hrows > 0 && a.njg == 1 && (!SPLIT || a.hrows == a.alpha * L / 2 + 1);
  // W_{N2}^{n2} = W_N^{N1 n2} (the mirror rows' factor), from rows 1 and
  // N1 - 1 of the post-twiddle table; N1 = 1 takes it from W_{alpha N}^{j n2}
  // W_{alpha N}^{(alpha - j) n2} in the loop
  cx<R> wn2 = {(R)1, (R)0};
  if constexpr (REG_MIRROR && L >= 2)
    if (sym && colok) wn2 = cmul(a.twPost[N2 + n2], a.twPost[(L - 1) * N2 + n2]);
  // The j loop, in two instances.  Loads and stores share one in-order
  // completion counter, so any global load the loop may issue (pre-twiddles
  // or W_{alpha N}^{j n2} not staged in LDS) makes the compiler wait there
  // for all earlier memory operations -- every store of the previous j --
  // and, where the two kinds of operand merge, it waits in every case.  The
  // LOCAL instance, taken when both are staged in LDS, reads only LDS inside
  // the loop; the column's tables loaded before it are made complete first,
  // so its stores stream out while the next transforms run.
  auto jloop = [&](auto local_tag) {
    constexpr bool LOCAL = decltype(local_tag)::value;
    if constexpr (LOCAL) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) asm volatile("" : : "v"(pw[e].re), "v"(pw[e].im));
      asm volatile("" : : "v"(wn2.re), "v"(wn2.im));
    }
    auto qval = [&](int jj) -> cx<R> {  // W_{alpha N}^{jj n2}
      if constexpr (LOCAL) return lds_read(qs + (jj - j0) * C + c);
      else return a.q_lds ? lds_read(qs + (jj - j0) * C + c) : a.twQ[jj * N2 + n2];
    };
    for (int j = j0; j < j1; ++j) {
      if (sym && 2 * j > a.alpha) break;  // stored with their partners alpha - j
      cx<R> v[EPT];
      if (j == 0) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) v[e] = xv[e];
      } else if (a.pre_lds == 1) {
        const cx<R>* pj = pre + (j - j0) * L + t;               // W_{alpha N1}^{j n1}
#pragma unroll
        for (int e = 0; e < EPT; ++e) v[e] = cmul(xv[e], pj[TL * e]);
      } else if (LOCAL || a.pre_lds == 2) {
        // W_{alpha N1}^{j (t + TL e)} = W_{alpha N1}^{j t} W_{alpha N1}^{j TL e}
        const cx<R> pt = pre[(j - j0) * TL + t];
        const cx<R>* pe = pre + (j1 - j0) * TL + (j - j0) * EPT;
#pragma unroll
        for (int e = 0; e < EPT; ++e) v[e] = cmul(xv[e], e == 0 ? pt : cmul(pt, pe[e]));
      } else {
        const cx<R>* __restrict__ pj = a.twPre + j * L + t;
#pragma unroll
        for (int e = 0; e < EPT; ++e) v[e] = cmul(xv[e], pj[TL * e]);
      }
      line_fft<R, L, false>(v, t, ex, lay, tws);
      if (colok) {
        const cx<R> q = qval(j);
        cx<R>* yj = ys + (int64_t)j * S;
        unsigned out_off_j = out_off;
        if constexpr (REG_MIRROR) asm volatile("" : "+v"(out_off_j));
        // rows kept: k1 < (hrows - j) / alpha, i.e. m1 = alpha k1 + j < hrows
        const int klim = HALF && a.hrows > 0 ? (a.hrows - j + a.alpha - 1) / a.alpha : L;
        // real input, every j in the block: the rows of jd = alpha - j too, at
        // k1' = N1 - 1 - k1 = (TL - 1 - t) + TL (EPT - 1 - e) (the primary
        // store's form with lane offset alpha S (TL - 1 - t) + n2), kept
        // while below hrows
        const bool mir = REG_MIRROR && sym && j >= 1 && 2 * j < a.alpha;
        const int jd = a.alpha - j;
        cx<R>* yd = ys + (int64_t)jd * S;
        unsigned off_d = (unsigned)(a.alpha * S * (TL - 1 - t) + n2);
        if constexpr (REG_MIRROR) asm volatile("" : "+v"(off_d));
        const int klim_d = mir ? (a.hrows - jd + a.alpha - 1) / a.alpha : 0;
        cx<R> w = wn2;
        if constexpr (REG_MIRROR && L == 1)
          if (mir) w = cmul(q, qval(jd));
        if (SPLIT && mir) {
#pragma unroll
          for (int e = 0; e < EPT / 2; ++e) (yj + out_step * e)[out_off_j] = cmul(v[e], cmul(pw[e], q));
          // conj(v pw q) w = conj(v) conj(pw) (conj(q) w)
          const cx<R> qw = cmul(cconj(q), w);
#pragma unroll
          for (int e = EPT / 2; e < EPT; ++e)
            (yd + out_step * (EPT - 1 - e))[off_d] = cmul(cconj(v[e]), cmul(cconj(pw[e]), qw));
        } else {
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            const cx<R> u = cmul(v[e], cmul(pw[e], q));
            if (!HALF || t + TL * e < klim) (yj + out_step * e)[out_off_j] = u;
            if constexpr (REG_MIRROR && !SPLIT)
              if (L - 1 - t - TL * e < klim_d) (yd + out_step * (EPT - 1 - e))[off_d] = cmul(cconj(u), w);
          }
        }
      }
      if constexpr (HALF && !REG_MIRROR) {
        if (sym && j >= 1 && 2 * j < a.alpha) {
          const int jd = a.alpha - j;
          __syncthreads();  // the transform's last exchange has been read
#pragma unroll
          for (int e = 0; e < EPT; ++e) ex[lay(t + TL * e)] = v[e];
          __syncthreads();
          if (colok) {
            const cx<R> q = qval(jd);
            cx<R>* yj = ys + (int64_t)jd * S;
            const int klim = (a.hrows - jd + a.alpha - 1) / a.alpha;
#pragma unroll
            for (int e = 0; e < EPT; ++e)
              if (t + TL * e < klim)
                (yj + out_step * e)[out_off] = cmul(cconj(ex[lay(L - 1 - t - TL * e)]), cmul(pw[e], q));
          }
          __syncthreads();  // before the next transform's exchange
        }
      }
    }
  };
  if (a.pre_lds != 0 && a.q_lds) jloop(std::true_type{});
  else jloop(std::false_type{});
  __syncthreads();  // LDS tables are rewritten by the next task of a persistent block
}

// Pass 2: block = (signal, block of RB consecutive rows m1).  Thread (t, r)
// with t fastest owns row m1 = block*RB + r, elements n2 = t + TL e.  Output
// X[m1 + alpha N1 k2] is staged in LDS and written as runs of RB bins.
// Real input (a.hrows > 0): only rows m1 <= H = floor(alpha N1 / 2) are
// transformed.  With m = m1 + alpha N1 k2 and 1 <= m1 <= H, the bin
// alpha N - m = (alpha N1 - m1) + alpha N1 (N2 - 1 - k2) is conj(X_m); rows
// m1 < alpha N1 - H are stored as they are and rows 1..H also as their
// conjugate mirrors, which fill rows alpha N1 - H .. alpha N1 - 1 exactly once.
// With ROWS = RB + 1 a block also transforms the first row of the next block,
// so that its mirrored rows, (block*RB, block*RB + RB], land on whole runs.
// TW_LDS: the stage twiddles are staged in LDS beside the row loads (the
// batch kernel's tasks, which are bound by their latency: the uneven batch
// 1.316 -> 1.282 ms); the plain kernel, bound by memory, reads them from the
// L2 (staged, its pass 2 of 256 x 65536 took 62.5 instead of 59.7 us).
template <typename R, int L, int RB, int ROWS = RB, bool TW_LDS = false>
__device__ __forceinline__ void body_pass2(const cx<R>* __restrict__ Y, cx<R>* __restrict__ X,
                                           const DenseArgs<R>& a, int64_t bid, unsigned char* smem, int tid) {
  static_assert(ROWS == RB || ROWS == RB + 1, "a block transforms RB or RB + 1 rows");
  constexpr LinePlan P = make_line_plan(L);
  constexpr int EPT = P.EPT;
  constexpr int TL = L / EPT;
  cx<R>* ex = reinterpret_cast<cx<R>*>(smem);
  const int rb = (int)(bid % a.ntile);
  const int64_t sig = bid / a.ntile;
  const int t = tid % TL, r = tid / TL;
  const int rows = a.alpha * a.N1;
  const int lim = a.hrows > 0 ? a.hrows : rows;   // rows transformed
  const int prim = a.hrows > 0 ? rows - (a.hrows - 1) : rows;  // rows stored as they are
  const int m1 = rb * RB + r;
  const bool ok = m1 < lim;
  const cx<R>* ys = Y + sig * a.ysig + (int64_t)rb * RB * a.yrow;
  const unsigned row_off = (unsigned)(r * a.yrow + t);
  cx<R> v[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) v[e] = ok ? (ys + TL * e)[row_off] : cx<R>{(R)0, (R)0};
  const RowLayout<L> lay(r);
  constexpr int TWS = TW_LDS ? pass2_tw_elems(L, RB, ROWS, (int)sizeof(cx<R>)) : 0;
  if constexpr (TWS > 0) {
    cx<R>* tws = ex + pass2_lds_elems(L, RB, ROWS);
    stage_to_lds<R, 4>(tws, TWS, tid, ROWS * TL, [&](int i) { return a.twL[i]; });
    __syncthreads();
    line_fft<R, L, (TL <= 64)>(v, t, ex, lay, tws);
  } else {
    line_fft<R, L, (TL <= 64)>(v, t, ex, lay, a.twL);
  }
  __syncthreads();
  constexpr int SR = RB + 1;  // staging row stride (odd, spreads banks)
#pragma unroll
  for (int e = 0; e < EPT; ++e) ex[(t + TL * e) * SR + r] = v[e];
  __syncthreads();
  cx<R>* xs = X + sig * a.y_stride;
  constexpr int total = RB * L;
  constexpr int NT = ROWS * TL;
  // Runs of RB bins shorter than a 128-byte line are completed by the
  // neighbouring block (the same XCD): those stores stay cached so that the
  // L2 merges the two halves (non-temporal, each half went to memory as a
  // partial line: 2^22 x alpha 16, pass 2 at N2 = 2048 450 -> 348 us, at
  // N2 = 4096 1209 -> 540 us).
  constexpr bool WHOLE = RB * (int)sizeof(cx<R>) >= 128;
  auto put = [&](cx<R>* p, cx<R> v) {
    if constexpr (WHOLE) store_out(p, v);
    else *p = v;
  };
#pragma unroll 4
  for (int i = tid; i < total; i += NT) {
    const int rr = i % RB, k2 = i / RB;
    const int m = rb * RB + rr;
    if (m < prim) put(xs + (int64_t)m + (int64_t)rows * k2, ex[k2 * SR + rr]);
  }
  if (a.hrows > 0) {
    // conjugate mirrors: consecutive i -> consecutive target rows rows - m
#pragma unroll 4
    for (int i = tid; i < total; i += NT) {
      const int rr = RB - 1 - i % RB + (ROWS - RB), kk = i / RB;
      const int m = rb * RB + rr;
      if (m >= 1 && m < lim) put(xs + (int64_t)(rows - m) + (int64_t)rows * kk, cconj(ex[(L - 1 - kk) * SR + rr]));
    }
  }
  __syncthreads();  // the staging buffer is reused by the next task of a persistent block
}

// ---------------------------------------------------------------------------
// Standalone kernels (one launch per pass).
// ---------------------------------------------------------------------------

// The blocks of a launch are dealt to the 8 XCDs in turn, each XCD with its
// own L2.  Renumbered so that every XCD takes a contiguous range of tiles,
// neighbouring tiles, which share cache lines of input and output, meet in
// one L2 (the blocks beyond the last full round of 8 keep their index).
__device__ __forceinline__ int64_t xcd_contiguous(int64_t bid, int64_t nblocks) {
  constexpr int XCDS = 8;
  const int64_t per = nblocks / XCDS;
  if (bid >= per * XCDS) return bid;
  return (bid % XCDS) * per + bid / XCDS;
}

template <typename R, typename In, int L, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_single(const In* __restrict__ x, cx<R>* __restrict__ X,
                                                  DenseArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  body_single<R, PtrIn<R, In>, L>(PtrIn<R, In>{x}, X, a, blockIdx.x, blockDim.x, smem_raw, threadIdx.x);
}

template <typename R, typename In, int L, int C>
__global__ __launch_bounds__(C * (L / make_line_plan(L).EPT)) void k_pass1(const In* __restrict__ x,
                                                                          cx<R>* __restrict__ Y,
                                                                          DenseArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  body_pass1<R, PtrIn<R, In>, L, C, std::is_floating_point<In>::value>(PtrIn<R, In>{x}, Y, a,
                                                                      xcd_contiguous(blockIdx.x, gridDim.x), smem_raw,
                                    threadIdx.x);
}

template <typename R, int L, int RB, int ROWS>
__global__ __launch_bounds__(ROWS * (L / make_line_plan(L).EPT)) void k_pass2(const cx<R>* __restrict__ Y,
                                                                             cx<R>* __restrict__ X,
                                                                             DenseArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  body_pass2<R, L, RB, ROWS>(Y, X, a, xcd_contiguous(blockIdx.x, gridDim.x), smem_raw, threadIdx.x);
}

// ---------------------------------------------------------------------------
// Twiddle tables: out[r][c] = W_den^{((r + r0) c) mod den}, exponent reduced
// exactly in 64-bit integers, then sin/cos in FP64 (each entry rounded once to R) or,
// for the FP32 variant, angle and sin/cos in FP32 from the same exact q.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_twiddle(cx<R>* __restrict__ out, int64_t rows, int64_t cols, int64_t r0,
                          int64_t den, int fp32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const uint64_t r = (uint64_t)(i / cols + r0), c = (uint64_t)(i % cols);
  const uint64_t q = (r * c) % (uint64_t)den;
  if (fp32) {
    float s, co;
    const float ang = (float)q * (float)(6.283185307179586476925286766559 / (double)den);
    sincosf(ang, &s, &co);
    out[i] = {(R)co, (R)(-s)};
  } else {
    double s, co;
    sincospi(2.0 * (double)q / (double)den, &s, &co);
    out[i] = {(R)co, (R)(-s)};
  }
}

}  // namespace dd
