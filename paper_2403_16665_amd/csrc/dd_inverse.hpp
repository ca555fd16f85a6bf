// dd_inverse.hpp -- block bodies and kernels of the inverse alpha-transform.
//
// The inverse (the reading of eq. (7), second line, with the factor 1/(alpha T)
// that undoes the forward transform of eq. (2)):
//
//     x_n = (1/(alpha T)) sum_{m < alpha N} X_m W_{alpha N}^{-mn},   n < N.
//
// It is the adjoint of the forward transform.  With
// F(n) = sum_m conj(X_m) W_{alpha N}^{mn}, x_n = conj(F(n)) / (alpha T), and
// m = alpha k + j splits F like the forward identity, read backwards:
//
//     F(n) = sum_j W_{alpha N}^{jn} sum_k conj(X_{alpha k + j}) W_N^{kn},
//
// alpha length-N FFTs of the strided subsequences, each times the forward
// pre-twiddle table, summed over j.  The two-pass form mirrors the forward
// passes (n = N2 n1 + n2, m = m1 + alpha N1 k2, m1 = alpha k1 + j):
//   pass A: G[m1][n2] = W_{alpha N}^{m1 n2} sum_{k2} conj(X_{m1 + alpha N1 k2}) W_{N2}^{k2 n2},
//   pass B: F(N2 n1 + n2) = sum_j W_{alpha N1}^{j n1} sum_{k1} G[alpha k1 + j][n2] W_{N1}^{k1 n1},
// so one plan's twiddle tables serve both directions.  (Applying the
// inter-pass factor in pass B instead, with W_N^{k1 n2} kept in registers
// across j, was measured slower: pass B then holds 32 more registers.)
#pragma once

#include "dd_launch.hpp"

namespace dd {

// One pass: block = a.lines signals, each shared by a.jgroup groups of TL
// threads (group g takes j = g, g + jgroup, ...).  Their alpha*L spectra are
// staged in LDS with one contiguous load; for each j, thread t of a group
// gathers the elements k = t + TL e of the subsequence X_{alpha k + j}.  Each
// group sums its values of j in registers; with several groups the partial
// sums meet in the groups' exchange rows and the signal's first group adds
// them in order of g.
template <typename R, int L>
__device__ __forceinline__ void body_single_inv(const cx<R>* __restrict__ X, cx<R>* __restrict__ x,
                                                const DenseArgs<R>& a, int64_t bid, int nt, unsigned char* smem,
                                                int tid) {
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
  const cx<R>* src = X + sig0 * a.y_stride;  // y_stride == alpha * L
  for (int64_t i = tid; i < nl * M1; i += nt) img[i] = load_once(src + i);
  __syncthreads();
  const RowLayout<L> lay(member ? gi : 0);
  const cx<R>* im = img + (int64_t)(active ? line : 0) * M1;
  cx<R> acc[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) acc[e] = {(R)0, (R)0};
  for (int j0 = 0; j0 < a.alpha; j0 += G) {  // uniform over the block
    const int j = j0 + g;
    const bool act = member && j < a.alpha;
    cx<R> v[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e)
      v[e] = active && act ? cconj(im[a.alpha * (t + TL * e) + j]) : cx<R>{(R)0, (R)0};
    line_fft<R, L, (TL <= 64), single_narrow(L)>(v, t, ex, lay, a.twL, act);
    if (act) {
      if (j == 0) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) acc[e] = cadd(acc[e], v[e]);
      } else {
        const cx<R>* __restrict__ pj = a.twPre + j * L + t;  // W_{alpha N}^{j n}
#pragma unroll
        for (int e = 0; e < EPT; ++e) acc[e] = cadd(acc[e], cmul(v[e], pj[TL * e]));
      }
    }
  }
  if (G > 1) {  // uniform
    __syncthreads();  // every group's last transform has read its exchange row
    if (member) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) ex[lay(t + TL * e)] = acc[e];
    }
    __syncthreads();
    if (active && g == 0) {
      for (int h = 1; h < G; ++h) {
        const RowLayout<L> lh(line * G + h);
#pragma unroll
        for (int e = 0; e < EPT; ++e) acc[e] = cadd(acc[e], lds_read(ex + lh(t + TL * e)));
      }
    }
  }
  if (active && g == 0) {
    cx<R>* xs = x + sig * a.x_stride;
#pragma unroll
    for (int e = 0; e < EPT; ++e) store_out(xs + t + TL * e, cscale(cconj(acc[e]), a.scale));
  }
}

// Which pass applies the inter-pass twiddle W_{alpha N}^{m1 n2}.  In single
// precision pass B, as it reads G back (pass A would load 2 x EPT table
// entries per thread, twice its data loads; pass B holds W_N^{k1 n2} for its
// column across every j, as the forward pass 1 does).  In double precision
// pass A: held in pass B the factors spill registers.
template <typename R>
__host__ __device__ constexpr bool inv_twiddle_in_b() { return sizeof(R) == 4; }

// Pass A: block = (signal, RB consecutive rows m1).  The RB x N2 values
// X_{m1 + alpha N1 k2} of its rows are read as runs of RB bins (the forward
// pass 2's store pattern) through an LDS transpose; thread (t, r) then owns
// row m1 = block*RB + r, elements k2 = t + TL e.  Rows of G are stored
// contiguously.
template <typename R, int L, int RB>
__device__ __forceinline__ void body_passA(const cx<R>* __restrict__ X, cx<R>* __restrict__ G,
                                           const DenseArgs<R>& a, int64_t bid, unsigned char* smem, int tid) {
  constexpr LinePlan P = make_line_plan(L);
  constexpr int EPT = P.EPT;
  constexpr int TL = L / EPT;
  constexpr int SR = RB + 1;  // staging row stride (odd, spreads banks)
  constexpr int total = RB * L;
  constexpr int NT = RB * TL;
  cx<R>* ex = reinterpret_cast<cx<R>*>(smem);
  const int rb = (int)(bid % a.ntile);
  const int64_t sig = bid / a.ntile;
  const int t = tid % TL, r = tid / TL;
  const int rows = a.alpha * a.N1;
  const int m1 = rb * RB + r;
  const bool ok = m1 < rows;
  const cx<R>* xs = X + sig * a.y_stride;
  // element i = tid + u NT of the block's RB x L values: row rr = tid % RB
  // (NT is a multiple of RB), k2 = tid / RB + u TL; all EPT loads are issued
  // before the first LDS write, so their latencies overlap
  static_assert(total == EPT * NT, "one value per thread per element slot");
  const int rr = tid % RB, kb = tid / RB;
  const int mrow = rb * RB + rr;
  cx<R> g[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u)
    g[u] = mrow < rows ? load_once(xs + (int64_t)mrow + (int64_t)rows * (kb + u * TL)) : cx<R>{(R)0, (R)0};
#pragma unroll
  for (int u = 0; u < EPT; ++u) ex[(kb + u * TL) * SR + rr] = g[u];
  __syncthreads();
  cx<R> v[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) v[e] = cconj(ex[(t + TL * e) * SR + r]);
  __syncthreads();  // the staging area becomes the FFT's exchange buffer
  const RowLayout<L> lay(r);
  line_fft<R, L, (TL <= 64)>(v, t, ex, lay, a.twL);
  if (ok) {
    cx<R>* gr = G + sig * a.y_stride + (int64_t)m1 * L + t;
    if constexpr (inv_twiddle_in_b<R>()) {
      // the row's transform as it is: pass B applies the inter-pass twiddle
      // as it reads the row back
#pragma unroll
      for (int e = 0; e < EPT; ++e) gr[TL * e] = v[e];
    } else {
      // W_{alpha N}^{m1 n2} = W_N^{k1 n2} W_{alpha N}^{j n2}, m1 = alpha k1 + j;
      // every twiddle load before the first store (loads and stores share
      // one in-order completion counter, so a load issued after a store
      // would wait for that store too)
      const int k1 = m1 / a.alpha, j = m1 - k1 * a.alpha;
      const cx<R>* __restrict__ pw = a.twPost + (int64_t)k1 * L + t;
      const cx<R>* __restrict__ q = a.twQ + (int64_t)j * L + t;
      cx<R> w[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) w[e] = pw[TL * e];
#pragma unroll
      for (int e = 0; e < EPT; ++e) w[e] = cmul(w[e], q[TL * e]);
#pragma unroll
      for (int e = 0; e < EPT; ++e) gr[TL * e] = cmul(v[e], w[e]);
    }
  }
}

// Pass B: block = (signal, tile of C columns n2), every j.  Thread (c, t)
// with c fastest owns column n2 = tile*C + c; for each j it reads the
// elements k1 = t + TL e of G[alpha k1 + j][n2] (rows of C columns), times
// the inter-pass twiddle W_{alpha N}^{m1 n2} = W_N^{k1 n2} W_{alpha N}^{j n2}
// when this pass applies it (m1 = alpha k1 + j; the first factor is held for
// every j, as in the forward pass 1, which forms the same product), runs the
// length-N1 FFT and accumulates it times W_{alpha N1}^{j n1}; x[N2 n1 + n2]
// is stored once, as rows of C columns.
template <typename R, int L, int C>
__device__ __forceinline__ void body_passB(const cx<R>* __restrict__ G, cx<R>* __restrict__ x,
                                           const DenseArgs<R>& a, int64_t bid, unsigned char* smem, int tid) {
  constexpr LinePlan P = make_line_plan(L);
  constexpr int EPT = P.EPT;
  constexpr int TL = L / EPT;
  constexpr int NT = C * TL;
  constexpr int TWN = line_tw_size(P);
  cx<R>* ex = reinterpret_cast<cx<R>*>(smem);
  cx<R>* tws = ex + ColLayout<C>::elems(L);  // stage twiddles
  cx<R>* pre = tws + TWN;                    // [j][n1] W_{alpha N1}^{j n1} (when a.pre_lds)
  const int tile = (int)(bid % a.ntile);
  const int64_t sig = bid / a.ntile;
  const int c = tid % C, t = tid / C;
  const int N2 = a.N2;
  const int n2 = tile * C + c;
  const bool colok = n2 < N2;
  const ColLayout<C> lay(c);
  for (int i = tid; i < TWN; i += NT) tws[i] = a.twL[i];
  if (a.pre_lds)
    for (int i = tid; i < a.alpha * L; i += NT) pre[i] = a.twPre[i];
  __syncthreads();
  const cx<R>* gs = G + sig * a.y_stride;
  const unsigned in_off = (unsigned)(a.alpha * N2 * t + n2);  // lane part of (alpha k1 + j) N2 + n2
  const unsigned in_step = (unsigned)(a.alpha * N2 * TL);     // k1 -> k1 + TL
  const unsigned tw_off = (unsigned)(N2 * t + n2);  // lane part of N2 k1 + n2
  const unsigned tw_step = (unsigned)(N2 * TL);
  constexpr bool TWB = inv_twiddle_in_b<R>();
  cx<R> acc[EPT], pw[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    acc[e] = {(R)0, (R)0};
    if constexpr (TWB) pw[e] = colok ? (a.twPost + tw_step * e)[tw_off] : cx<R>{(R)0, (R)0};  // W_N^{k1 n2}
  }
  for (int j = 0; j < a.alpha; ++j) {
    cx<R> v[EPT];
    const cx<R>* gj = gs + (int64_t)j * N2;
#pragma unroll
    for (int e = 0; e < EPT; ++e) v[e] = colok ? (gj + in_step * e)[in_off] : cx<R>{(R)0, (R)0};
    if constexpr (TWB) {
      const cx<R> q = colok ? a.twQ[j * N2 + n2] : cx<R>{(R)0, (R)0};  // W_{alpha N}^{j n2}
#pragma unroll
      for (int e = 0; e < EPT; ++e) v[e] = cmul(v[e], cmul(pw[e], q));
    }
    line_fft<R, L, false>(v, t, ex, lay, tws);
    if (j == 0) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) acc[e] = cadd(acc[e], v[e]);
    } else if (a.pre_lds) {
      const cx<R>* pj = pre + j * L + t;
#pragma unroll
      for (int e = 0; e < EPT; ++e) acc[e] = cadd(acc[e], cmul(v[e], pj[TL * e]));
    } else {
      const cx<R>* __restrict__ pj = a.twPre + j * L + t;
#pragma unroll
      for (int e = 0; e < EPT; ++e) acc[e] = cadd(acc[e], cmul(v[e], pj[TL * e]));
    }
  }
  if (colok) {
    cx<R>* xs = x + sig * a.x_stride + n2;
    const unsigned out_step = (unsigned)(N2 * TL);
    const unsigned out_off = (unsigned)(N2 * t);
#pragma unroll
    for (int e = 0; e < EPT; ++e) store_out(xs + out_step * e + out_off, cscale(cconj(acc[e]), a.scale));
  }
}

template <typename R, int L, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_single_inv(const cx<R>* __restrict__ X, cx<R>* __restrict__ x,
                                                      DenseArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  body_single_inv<R, L>(X, x, a, blockIdx.x, blockDim.x, smem_raw, threadIdx.x);
}

template <typename R, int L, int RB>
__global__ __launch_bounds__(RB * (L / make_line_plan(L).EPT)) void k_passA(const cx<R>* __restrict__ X,
                                                                            cx<R>* __restrict__ G,
                                                                            DenseArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  body_passA<R, L, RB>(X, G, a, xcd_contiguous(blockIdx.x, gridDim.x), smem_raw, threadIdx.x);
}

template <typename R, int L, int C>
__global__ __launch_bounds__(C * (L / make_line_plan(L).EPT)) void k_passB(const cx<R>* __restrict__ G,
                                                                           cx<R>* __restrict__ x,
                                                                           DenseArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  body_passB<R, L, C>(G, x, a, xcd_contiguous(blockIdx.x, gridDim.x), smem_raw, threadIdx.x);
}

// Launchers, defined for both precisions in dd_inv_f32.hip / dd_inv_f64.hip.
#define DD_DECL_INV(R)                                                                                      \
  hipError_t launch_single_inv(int L, const LaunchCfg& c, const cx<R>* X, cx<R>* x, const DenseArgs<R>& a); \
  hipError_t launch_passA(int L, const LaunchCfg& c, const cx<R>* X, cx<R>* G, const DenseArgs<R>& a);      \
  hipError_t launch_passB(int L, const LaunchCfg& c, const cx<R>* G, cx<R>* x, const DenseArgs<R>& a);
DD_DECL_INV(float)
DD_DECL_INV(double)
#undef DD_DECL_INV

// The line length selects the instantiation, as for the forward kernels.
template <typename R>
hipError_t launch_single_inv_impl(int L, const LaunchCfg& c, const cx<R>* X, cx<R>* x, const DenseArgs<R>& a) {
  switch (L) {
#define DD_CASE(LL)                                                   \
  case LL: {                                                          \
    constexpr int B = Geom<LL, (int)sizeof(R)>::BLOCK_SINGLE;         \
    return launch_kernel(k_single_inv<R, LL, B>, c, X, x, a);         \
  }
    DD_ALL_LENGTHS(DD_CASE)
#undef DD_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename R>
hipError_t launch_passA_impl(int L, const LaunchCfg& c, const cx<R>* X, cx<R>* G, const DenseArgs<R>& a) {
  switch (L) {
#define DD_CASE(LL)                                                   \
  case LL: {                                                          \
    constexpr int RB = Geom<LL, (int)sizeof(R)>::lines_pass();        \
    return launch_kernel(k_passA<R, LL, RB>, c, X, G, a);             \
  }
    DD_POW2_LENGTHS(DD_CASE)
#undef DD_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename R>
hipError_t launch_passB_impl(int L, const LaunchCfg& c, const cx<R>* G, cx<R>* x, const DenseArgs<R>& a) {
  switch (L) {
#define DD_CASE(LL)                                                   \
  case LL: {                                                          \
    constexpr int C = Geom<LL, (int)sizeof(R)>::lines_pass();         \
    return launch_kernel(k_passB<R, LL, C>, c, G, x, a);              \
  }
    DD_ALL_LENGTHS(DD_CASE)
#undef DD_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace dd
