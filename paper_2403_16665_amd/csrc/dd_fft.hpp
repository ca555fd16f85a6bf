// dd_fft.hpp -- device building blocks of the alpha-dense DFT on gfx950.
//
// Complex arithmetic, fixed-radix forward DFTs (radix 2, 3, 4, 5, 8, 16) and
// a Stockham autosort engine that transforms one line of length L held by
// TL = L / EPT threads, EPT elements per thread in registers, exchanging
// through LDS between radix stages.
//
// Sign convention: forward transform with W_L = exp(-2 pi i / L), the
// convention the paper fixes for W (Section 3).  Each radix-r stage is the
// divide-and-conquer step of Section 3 (eq. (9)-(13)) generalised from the
// even/odd split (r = 2) to r-way splits: twiddle by W_{Ns r}^{k s}, then an
// r-point DFT.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dd {

template <typename R>
struct cx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> cscale(cx<R> a, R s) { return {a.re * s, a.im * s}; }
template <typename R>
__device__ __forceinline__ cx<R> cconj(cx<R> a) { return {a.re, -a.im}; }
// A read through an LDS-qualified pointer.  Where either an LDS value or some
// other value is chosen (a global table entry, or the thread's own register
// array), the compiler would otherwise load through a pointer selected at run
// time: a flat load, and a register array forced into private memory.
template <typename R>
__device__ __forceinline__ cx<R> lds_read(const cx<R>* p) {
  const __attribute__((address_space(3))) R* q = (const __attribute__((address_space(3))) R*)p;
  return {q[0], q[1]};
}

// -i * a
template <typename R>
__device__ __forceinline__ cx<R> cmul_negi(cx<R> a) { return {a.im, -a.re}; }

// ---------------------------------------------------------------------------
// Fixed-radix forward DFTs.  v[s*ST] for s < r are the inputs, overwritten by
// outputs Y_k at v[k*ST] (natural order).
// ---------------------------------------------------------------------------
template <typename R, int ST>
__device__ __forceinline__ void dft2(cx<R>* v) {
  cx<R> a = v[0], b = v[ST];
  v[0] = cadd(a, b);
  v[ST] = csub(a, b);
}

template <typename R>
__device__ __forceinline__ void dft4v(cx<R>& v0, cx<R>& v1, cx<R>& v2, cx<R>& v3) {
  cx<R> a = cadd(v0, v2), b = csub(v0, v2), c = cadd(v1, v3), d = csub(v1, v3);
  v0 = cadd(a, c);
  v2 = csub(a, c);
  v1 = {b.re + d.im, b.im - d.re};  // b - i d
  v3 = {b.re - d.im, b.im + d.re};  // b + i d
}

template <typename R, int ST>
__device__ __forceinline__ void dft4(cx<R>* v) {
  dft4v(v[0], v[ST], v[2 * ST], v[3 * ST]);
}

template <typename R, int ST>
__device__ __forceinline__ void dft8(cx<R>* v) {
  const R h = (R)0.70710678118654752440084436210485;
  cx<R> e0 = v[0], e1 = v[2 * ST], e2 = v[4 * ST], e3 = v[6 * ST];
  cx<R> o0 = v[ST], o1 = v[3 * ST], o2 = v[5 * ST], o3 = v[7 * ST];
  dft4v(e0, e1, e2, e3);
  dft4v(o0, o1, o2, o3);
  // W8^1 o1, W8^2 o2 = -i o2, W8^3 o3
  cx<R> t1 = {(o1.re + o1.im) * h, (o1.im - o1.re) * h};
  cx<R> t2 = cmul_negi(o2);
  cx<R> t3 = {(o3.im - o3.re) * h, -(o3.re + o3.im) * h};
  v[0] = cadd(e0, o0);
  v[4 * ST] = csub(e0, o0);
  v[ST] = cadd(e1, t1);
  v[5 * ST] = csub(e1, t1);
  v[2 * ST] = cadd(e2, t2);
  v[6 * ST] = csub(e2, t2);
  v[3 * ST] = cadd(e3, t3);
  v[7 * ST] = csub(e3, t3);
}

template <typename R, int ST>
__device__ __forceinline__ void dft16(cx<R>* v) {
  // s = s2 + 4 s1, k = k1 + 4 k2:
  // Y_{k1+4k2} = sum_{s2} W4^{k2 s2} W16^{k1 s2} [sum_{s1} v_{s2+4s1} W4^{k1 s1}]
  const R c1 = (R)0.92387953251128675612818318939679;  // cos(pi/8)
  const R s1 = (R)0.38268343236508977172845998403040;  // sin(pi/8)
  const R h = (R)0.70710678118654752440084436210485;
  cx<R> a[4][4];
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2) {
    a[s2][0] = v[(s2)*ST];
    a[s2][1] = v[(s2 + 4) * ST];
    a[s2][2] = v[(s2 + 8) * ST];
    a[s2][3] = v[(s2 + 12) * ST];
    dft4v(a[s2][0], a[s2][1], a[s2][2], a[s2][3]);
  }
  // twiddles W16^{k1 s2}
  // s2=1: k1=1 W^1, k1=2 W^2, k1=3 W^3
  a[1][1] = cmul(a[1][1], cx<R>{c1, -s1});
  a[1][2] = {(a[1][2].re + a[1][2].im) * h, (a[1][2].im - a[1][2].re) * h};
  a[1][3] = cmul(a[1][3], cx<R>{s1, -c1});
  // s2=2: W^2, W^4=-i, W^6
  a[2][1] = {(a[2][1].re + a[2][1].im) * h, (a[2][1].im - a[2][1].re) * h};
  a[2][2] = cmul_negi(a[2][2]);
  a[2][3] = {(a[2][3].im - a[2][3].re) * h, -(a[2][3].re + a[2][3].im) * h};
  // s2=3: W^3, W^6, W^9
  a[3][1] = cmul(a[3][1], cx<R>{s1, -c1});
  a[3][2] = {(a[3][2].im - a[3][2].re) * h, -(a[3][2].re + a[3][2].im) * h};
  a[3][3] = cmul(a[3][3], cx<R>{-c1, s1});
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<R> y0 = a[0][k1], y1 = a[1][k1], y2 = a[2][k1], y3 = a[3][k1];
    dft4v(y0, y1, y2, y3);
    v[(k1)*ST] = y0;
    v[(k1 + 4) * ST] = y1;
    v[(k1 + 8) * ST] = y2;
    v[(k1 + 12) * ST] = y3;
  }
}

template <typename R, int ST>
__device__ __forceinline__ void dft3(cx<R>* v) {
  const R sq = (R)0.86602540378443864676372317075294;  // sin(2 pi / 3)
  cx<R> v0 = v[0], v1 = v[ST], v2 = v[2 * ST];
  cx<R> t = cadd(v1, v2), d = csub(v1, v2);
  cx<R> m = {v0.re - (R)0.5 * t.re, v0.im - (R)0.5 * t.im};
  // Y1 = m - i sq d, Y2 = m + i sq d
  v[0] = cadd(v0, t);
  v[ST] = {m.re + sq * d.im, m.im - sq * d.re};
  v[2 * ST] = {m.re - sq * d.im, m.im + sq * d.re};
}

template <typename R, int ST>
__device__ __forceinline__ void dft5(cx<R>* v) {
  const R c1 = (R)0.30901699437494742410229341718282;   // cos(2 pi/5)
  const R c2 = (R)-0.80901699437494742410229341718282;  // cos(4 pi/5)
  const R s1 = (R)0.95105651629515357211643933337938;   // sin(2 pi/5)
  const R s2 = (R)0.58778525229247312916870595463907;   // sin(4 pi/5)
  cx<R> v0 = v[0];
  cx<R> t1 = cadd(v[ST], v[4 * ST]), d1 = csub(v[ST], v[4 * ST]);
  cx<R> t2 = cadd(v[2 * ST], v[3 * ST]), d2 = csub(v[2 * ST], v[3 * ST]);
  cx<R> a1 = {v0.re + c1 * t1.re + c2 * t2.re, v0.im + c1 * t1.im + c2 * t2.im};
  cx<R> a2 = {v0.re + c2 * t1.re + c1 * t2.re, v0.im + c2 * t1.im + c1 * t2.im};
  cx<R> b1 = {s1 * d1.re + s2 * d2.re, s1 * d1.im + s2 * d2.im};
  cx<R> b2 = {s2 * d1.re - s1 * d2.re, s2 * d1.im - s1 * d2.im};
  v[0] = {v0.re + t1.re + t2.re, v0.im + t1.im + t2.im};
  // Y1 = a1 - i b1, Y4 = a1 + i b1, Y2 = a2 - i b2, Y3 = a2 + i b2
  v[ST] = {a1.re + b1.im, a1.im - b1.re};
  v[4 * ST] = {a1.re - b1.im, a1.im + b1.re};
  v[2 * ST] = {a2.re + b2.im, a2.im - b2.re};
  v[3 * ST] = {a2.re - b2.im, a2.im + b2.re};
}

template <typename R, int RAD, int ST>
__device__ __forceinline__ void dft(cx<R>* v) {
  if constexpr (RAD == 2) dft2<R, ST>(v);
  else if constexpr (RAD == 3) dft3<R, ST>(v);
  else if constexpr (RAD == 4) dft4<R, ST>(v);
  else if constexpr (RAD == 5) dft5<R, ST>(v);
  else if constexpr (RAD == 8) dft8<R, ST>(v);
  else if constexpr (RAD == 16) dft16<R, ST>(v);
  else static_assert(RAD == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// Line plans: for a supported length L, the elements per thread EPT and the
// radix sequence.  L = 2^a (radices 16, 8, 4, 2; EPT 16), L = 3*2^a
// (radix 3 then 4s and a 2; EPT 12) and L = 5*2^a (radix 5 then 4s and a 2;
// EPT 20).  Lines shorter than EPT are done by one thread.
// ---------------------------------------------------------------------------
struct LinePlan {
  int L, EPT, nst;
  int rad[12];
};

// narrow: a radix-5 line takes 10 elements per thread instead of 20.  The
// one-pass kernels use it for 5 * 2^a <= 640 (single_narrow): a line there
// is a whole signal, its transforms run one after another, and 20 elements
// per thread spill registers (measured: 320 x alpha 16, 0.187 -> 0.086 ms);
// the passes' column transforms keep 20 (fewer exchange stages).
constexpr LinePlan make_line_plan(int L, bool narrow = false) {
  LinePlan p{L, 1, 0, {0}};
  int odd = 1, r = L;
  while (r % 2 == 0) r /= 2;
  odd = r;                 // 1, 3 or 5
  int pw = L / odd;        // power of two part
  if (odd == 1) {
    p.EPT = L < 16 ? L : 16;
    int rem = L;
    while (rem > 1) {
      int rr = rem >= 16 ? 16 : rem;  // 16s, then the leftover 8/4/2
      p.rad[p.nst++] = rr;
      rem /= rr;
    }
  } else {
    int cap = odd == 3 ? 12 : (narrow ? 10 : 20);
    p.EPT = L < cap ? L : cap;
    p.rad[p.nst++] = odd;
    int rem = pw;
    while (rem > 1) {
      int rr = rem >= 4 ? 4 : 2;
      if (p.EPT % rr != 0) rr = 2;
      p.rad[p.nst++] = rr;
      rem /= rr;
    }
  }
  return p;
}

constexpr int line_ns(const LinePlan& p, int st) {
  int ns = 1;
  for (int i = 0; i < st; ++i) ns *= p.rad[i];
  return ns;
}

// Stage twiddle table: for stage st (radix RAD, span NS) the entries
// W_{NS RAD}^{k s} for s < RAD, k < NS, laid out [s][k] at offset
// line_tw_offset(p, st); total line_tw_size(p) entries.
constexpr int line_tw_offset(const LinePlan& p, int st) {
  int off = 0;
  for (int i = 1; i < st; ++i) off += p.rad[i] * line_ns(p, i);
  return off;
}
constexpr int line_tw_size(const LinePlan& p) { return p.nst > 1 ? line_tw_offset(p, p.nst) : 0; }

constexpr bool single_narrow(int L) { return L % 5 == 0 && L <= 640; }

constexpr bool line_plan_ok(int L, bool narrow = false) {
  LinePlan p = make_line_plan(L, narrow);
  int prod = 1;
  for (int i = 0; i < p.nst; ++i) {
    if (p.EPT % p.rad[i] != 0) return false;
    prod *= p.rad[i];
  }
  return prod == L && L % p.EPT == 0;
}

// LDS layouts.  Position i of line `line` lives at index addr(line, i).
// RowLayout: each line contiguous, one pad element per 16 (breaks the
//   power-of-two strides of the Stockham writes across LDS banks).
// ColLayout: lines interleaved (line fastest), pad of 8 elements every 16
//   positions.
template <int L>
struct RowLayout {
  static constexpr int STRIDE = L + L / 16 + 1;
  int base;
  __device__ __forceinline__ RowLayout(int line) : base(line * STRIDE) {}
  __device__ __forceinline__ int operator()(int i) const { return base + i + (i >> 4); }
  static constexpr int elems(int lines) { return lines * STRIDE; }
};

template <int LINES>
struct ColLayout {
  int line;
  __device__ __forceinline__ ColLayout(int l) : line(l) {}
  __device__ __forceinline__ int operator()(int i) const { return i * LINES + line + (i >> 4) * 8; }
  static __host__ __device__ constexpr int elems(int L) { return L * LINES + (L / 16 + 1) * 8; }
};

// Exchange synchronisation between radix stages: the whole block, or only the
// wavefront when every line lies inside one wavefront (LDS operations of a
// wavefront complete in order; the fence keeps the compiler from moving LDS
// accesses across it).
template <bool WAVE>
__device__ __forceinline__ void exchange_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// One Stockham stage.  On entry (first stage) v[e] holds line element t + TL e.
// Butterfly b = t + TL i (i < NB = EPT/RAD) reads elements b + s L/RAD,
// twiddles them by W_{NS RAD}^{(b mod NS) s}, applies the RAD-point DFT and
// writes output s to position (b / NS) NS RAD + b mod NS + s NS.  After the
// last stage v[e] holds output element k = t + TL e (natural order).
template <typename R, int L, int ST, bool WAVE, bool NARROW, class Lay>
__device__ __forceinline__ void line_stage(cx<R>* v, int t, cx<R>* lds, const Lay& lay,
                                           const cx<R>* __restrict__ twL, bool act) {
  constexpr LinePlan P = make_line_plan(L, NARROW);
  constexpr int EPT = P.EPT;
  constexpr int TL = L / EPT;
  constexpr int RAD = P.rad[ST];
  constexpr int NB = EPT / RAD;
  constexpr int NS = line_ns(P, ST);
  constexpr bool FIRST = ST == 0;
  constexpr bool LAST = ST == P.nst - 1;
  if constexpr (!FIRST) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int b = t + TL * i;
#pragma unroll
      for (int s = 0; s < RAD; ++s)
        if (act) v[i + s * NB] = lds_read(lds + lay(b + s * (L / RAD)));
    }
    const cx<R>* __restrict__ tws = twL + line_tw_offset(P, ST);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int b = t + TL * i;
      const int k = b % NS;
#pragma unroll
      for (int s = 1; s < RAD; ++s) v[i + s * NB] = cmul(v[i + s * NB], tws[s * NS + k]);
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) dft<R, RAD, NB>(v + i);
  if constexpr (!LAST) {
    exchange_sync<WAVE>();  // every thread has read its inputs of this stage
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int b = t + TL * i;
      const int base = (b / NS) * NS * RAD + (b % NS);
#pragma unroll
      for (int s = 0; s < RAD; ++s)
        if (act) lds[lay(base + s * NS)] = v[i + s * NB];
    }
    exchange_sync<WAVE>();
    line_stage<R, L, ST + 1, WAVE, NARROW, Lay>(v, t, lds, lay, twL, act);
  }
}

// Forward length-L transform of one line.  All threads of the block (WAVE
// false) or of the wavefront (WAVE true, every line inside one wavefront)
// must call it; its first synchronisation also orders it after any earlier
// use of `lds`.  twL is the stage twiddle table (line_tw_size entries).
// Threads with act == false take part in the synchronisation only (no LDS
// access); their registers come out unchanged.
template <typename R, int L, bool WAVE, bool NARROW = false, class Lay>
__device__ __forceinline__ void line_fft(cx<R>* v, int t, cx<R>* lds, const Lay& lay,
                                         const cx<R>* __restrict__ twL, bool act = true) {
  constexpr LinePlan P = make_line_plan(L, NARROW);
  if constexpr (P.nst > 0) line_stage<R, L, 0, WAVE, NARROW, Lay>(v, t, lds, lay, twL, act);
}

}  // namespace dd
