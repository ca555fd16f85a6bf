// dd_api.cpp -- planner and C ABI of the alpha-dense DFT library (host code).
//
// A plan fixes N, alpha, T, batch and dtype (the problem as the paper states
// it, Section 2: N samples over [0, T], alpha*N bins spaced 1/(alpha T)),
// chooses the schedule, and owns the device twiddle tables.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/dense_dft.h"
#include "dd_host.hpp"
#include "dd_inverse.hpp"
#include "dd_launch.hpp"
#include "dd_tune.hpp"

using namespace dd;

namespace dd {
hipError_t launch_fold(dd_dtype dtype, const void* x, void* y, int64_t batch, int64_t N, int64_t Np, int p,
                       hipStream_t s);  // dd_fold.hip
}

struct dd_plan {
  int device = 0;
  int64_t N = 0, N1 = 0, N2 = 1, batch = 0;
  int alpha = 1;
  double T = 1.0;
  dd_dtype dtype = DD_C64;
  uint32_t flags = 0;
  bool dbl = false;
  int in_bytes = 8, rbytes = 4;
  int passes = 1;
  // single pass (forward and inverse): s_lines signals per block, s_groups
  // thread groups per signal (each takes its own values of j)
  int s_lines = 1, s_groups = 1, s_TL = 1;
  size_t s_lds = 0;
  // two passes
  int p1_lines = 1, p1_TL = 1, p1_ntile = 1, p1_jgroup = 1, p1_njg = 1, p1_pre_lds = 0, p1_q_lds = 0;
  size_t p1_lds = 0;
  int p2_lines = 1, p2_TL = 1, p2_ntile = 1;
  size_t p2_lds = 0;
  // the forward pass 2 of complex input: wider blocks (up to 1024 threads)
  int p2f_lines = 1, p2f_ntile = 1;
  size_t p2f_lds = 0;
  // real input: pass 1 stores the scratch rows m1 <= alpha N1 / 2 and pass 2
  // transforms them in blocks of p2_lines + 1 rows (when those fit the LDS)
  bool p2_half = false;
  size_t p2h_lds = 0;
  // the scratch: rows m1 of y_row elements (N2 and a pad), y_sig per signal
  int64_t y_row = 1, y_sig = 1;
  // inverse pass B (every j per block): pre-twiddles staged in LDS, its LDS
  int inv_pre_lds = 0;
  size_t inv_p1_lds = 0;
  // alpha = 1/dec_p (dec_p > 1): the fold into the workspace, then the plain
  // plan `inner` of length N/dec_p
  int dec_p = 1;
  dd_plan* inner = nullptr;
  size_t fold_bytes = 0;
  int64_t chunk = 1;
  // device tables (element type cx<float> or cx<double>)
  void* twL1 = nullptr;   // stage twiddles of the N1 (or N) line FFT
  void* twL2 = nullptr;   // stage twiddles of the N2 line FFT
  void* twPre = nullptr;  // [j][n1] W_{alpha N1}^{j n1}
  void* twQ = nullptr;    // [j][n2] W_{alpha N}^{j n2}
  void* twPost = nullptr; // [k1][n2] W_N^{k1 n2}
  void* ws = nullptr;     // default workspace
  size_t ws_bytes = 0;
  // per-launch event timing (dense_dft_profile_begin / _end)
  bool prof_on = false;
  int prof_n = 0;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_kind;
};

namespace {

size_t cx_bytes(const dd_plan* p) { return (size_t)2 * p->rbytes; }

void free_events(dd_plan* p) {
  for (hipEvent_t e : p->prof_ev) (void)hipEventDestroy(e);
  p->prof_ev.clear();
  p->prof_kind.clear();
  p->prof_on = false;
  p->prof_n = 0;
}

// Launch wrapper: brackets the launch with events while profiling is on.
template <typename F>
hipError_t timed_launch(dd_plan* p, int kind, hipStream_t s, F&& launch) {
  const bool rec = p->prof_on && p->prof_n < (int)p->prof_kind.size();
  if (rec) {
    hipError_t e = hipEventRecord(p->prof_ev[2 * p->prof_n], s);
    if (e != hipSuccess) return e;
  }
  hipError_t e = launch();
  if (e != hipSuccess) return e;
  if (rec) {
    e = hipEventRecord(p->prof_ev[2 * p->prof_n + 1], s);
    p->prof_kind[p->prof_n] = kind;
    ++p->prof_n;
  }
  return e;
}

void free_tables(dd_plan* p) {
  void** bufs[] = {&p->twL1, &p->twL2, &p->twPre, &p->twQ, &p->twPost, &p->ws};
  for (void** b : bufs) {
    if (*b) (void)hipFree(*b);
    *b = nullptr;
  }
}

// narrow: the table of a one-pass plan's line (the one-pass kernels' plan)
dd_status gen_stage_table(dd_plan* p, void** out, int L, bool fp32, hipStream_t s, bool narrow = false) {
  return make_stage_table(out, L, p->dbl, fp32, s, narrow);
}

dd_status gen_table(dd_plan* p, void** out, int64_t rows, int64_t cols, int64_t den, bool fp32,
                    hipStream_t s) {
  return make_table(out, rows, cols, den, p->dbl, fp32, s);
}

// Choose N = N1 * N2 for the two-pass schedule: N1 any instantiated length,
// N2 a power of two >= 2, as balanced as possible (N1 <= N2 on ties); for
// N <= 4096 (signals whose spectra are too large for a one-pass block), N2
// as close to 256 as the factors allow: short columns and long rows
// (measured at 2^24 bins: 1024 = 4 x 256 64 us against 98 us for 32 x 32,
// 640 = 5 x 128 69 us against 159 us for 20 x 32).
bool factor_two_pass(int64_t N, int rbytes, int64_t* N1, int64_t* N2) {
  int best = 1 << 30;
  bool found = false;
  for (int64_t n2 = 2; n2 <= 4096; n2 *= 2) {
    if (N % n2) continue;
    const int64_t n1 = N / n2;
    if (n1 > 4096 || !len_supported((int)n1) || !pass2_len_supported((int)n2)) continue;
    if (lds_pass1((int)n1, geom_pass((int)n1, rbytes).lines, rbytes, 0) > (size_t)LDS_PASS_MAX) continue;
    int score = N <= 4096 ? std::abs(ilog2(n2) - 8) * 2 + (n2 > 256 ? 1 : 0)
                          : std::abs(ilog2(n1) - ilog2(n2)) * 2 + (n1 > n2 ? 1 : 0);
    if (n2 < 16) score += 8;  // narrow column tiles store short runs
    if (n2 % geom_pass((int)n1, rbytes).lines != 0) score += 4;  // idle columns in pass 1
    if (score < best) {
      best = score;
      *N1 = n1;
      *N2 = n2;
      found = true;
    }
  }
  return found;
}

// One-pass blocks hold the spectrum of `lines` signals in LDS within this.
constexpr size_t SINGLE_BUDGET = 150 * 1024;

// One-pass block shapes.  A signal's jn transformed values of j are shared by
// G thread groups in ceil(jn / G) rounds; the group counts worth running are
// the fewest that finish in 1, 2, ... rounds, within the block (gl groups).
// Signals per block: the most that fit beside them, then powers of two below.
std::vector<int> single_group_options(int jn, int gl) {
  std::vector<int> o;
  for (int r = 1; r <= jn; ++r) {
    const int G = (jn + r - 1) / r;
    if (G <= gl && (o.empty() || o.back() != G)) o.push_back(G);
  }
  return o;
}
std::vector<int> single_line_options(int gl, int G) {
  std::vector<int> o;
  const int top = gl / G;
  if (top >= 1) o.push_back(top);
  int l = 1;
  while (2 * l <= top) l *= 2;
  for (; l >= 1; l /= 2)
    if (l != top) o.push_back(l);
  return o;
}
int single_jn(int alpha, bool real) { return real ? alpha / 2 + 1 : alpha; }

// The built-in one-pass shape (a zero argument is chosen, a nonzero one
// kept).  Score: the lanes a CU holds doing work -- resident blocks (from the
// runtime's occupancy of the kernel, which counts registers, LDS and
// wavefront slots; without a device, from LDS and 32 wavefront slots, at most
// 16 blocks) times the block's threads, each wavefront counted at the share
// of its lanes in use, times the share of group slots with a j to transform.
// Among the shapes within 10% of the best score the smallest block wins
// (measured: at equal resident lanes, more and smaller blocks wait less at
// their barriers), then fewer rounds over j, then more signals per block.
void single_shape(int L, int alpha, bool real, int rbytes, int64_t batch, int* lines_io, int* groups_io) {
  const KGeom g = geom_single(L, rbytes);
  const int jn = single_jn(alpha, real);
  struct Shape {
    int lines, groups, block, rounds;
    double score;
  };
  std::vector<Shape> shapes;
  double best = 0;
  for (const int G : single_group_options(jn, g.lines)) {
    if (*groups_io > 0 && G != *groups_io) continue;
    for (const int l : single_line_options(g.lines, G)) {
      if (*lines_io > 0 && l != *lines_io) continue;
      if (l > 1 && l > batch) continue;
      const size_t lds = lds_single(L, l, alpha, rbytes, G);
      if (lds > SINGLE_BUDGET) continue;
      const int block = l * G * g.TL;
      const int waves = (block + 63) / 64;
      int64_t blocks = rbytes == 4 ? single_occupancy(L, real, 0.0f, block, lds)
                                   : single_occupancy(L, real, 0.0, block, lds);
      if (blocks <= 0) {
        blocks = (int64_t)(160 * 1024 / lds);
        if (blocks > 32 / waves) blocks = 32 / waves;
        if (blocks > 16) blocks = 16;
      }
      const int rounds = (jn + G - 1) / G;
      double lanes = (double)blocks * block * block / (64.0 * waves);
      if (lanes > 1024) lanes = 1024;
      const double score = lanes * jn / ((double)rounds * G);
      shapes.push_back({l, G, block, rounds, score});
      if (score > best) best = score;
    }
  }
  const Shape* pick = nullptr;
  for (const Shape& c : shapes) {
    if (c.score < 0.9 * best) continue;
    const bool better = !pick || c.block < pick->block ||
                        (c.block == pick->block &&
                         (c.rounds < pick->rounds || (c.rounds == pick->rounds && c.lines > pick->lines)));
    if (better) pick = &c;
  }
  if (*lines_io <= 0) *lines_io = pick ? pick->lines : 1;
  if (*groups_io <= 0) *groups_io = pick ? pick->groups : 1;
}

// Built-in schedule rules: one pass when the alpha*N spectrum of a signal
// takes at most 32 KiB (or N < 256, or no two-pass split exists) and fits
// the LDS of one block, else the two-pass split of factor_two_pass; tile
// choices left to configure().  Larger spectra leave a one-pass block LDS-bound (one
// or two blocks per CU): measured at 2^24 bins per launch, two passes took
// 64-75 us where one pass took 75-181 us (1024 x 8, 512 x 16, 640 x 8,
// 1280 x 4, 2048 x 8, 3072 x 4), while at 4096 bins one pass stayed ahead
// (1024 x 4 55 against 67 us, 512 x 8 59 against 66).
bool default_sched(int64_t N, int alpha, int rbytes, dd_sched* sc) {
  *sc = dd_sched{};
  int64_t N1 = 0, N2 = 0;
  const bool split = factor_two_pass(N, rbytes, &N1, &N2);
  const bool small = (int64_t)alpha * N * 2 * rbytes <= 32 * 1024 || N < 256 || !split;
  if (small && N <= 4096 && len_supported((int)N) && lds_single((int)N, 1, alpha, rbytes) <= SINGLE_BUDGET) {
    sc->passes = 1;
    sc->N1 = N;
    sc->N2 = 1;
    return true;
  }
  if (!split) return false;
  sc->passes = 2;
  sc->N1 = N1;
  sc->N2 = N2;
  return true;
}

// Fill the plan's launch geometry from a schedule (zero fields take the
// built-in rule); DD_ERR_UNSUPPORTED if the schedule does not fit N, alpha
// and the compiled kernels.
dd_status configure(dd_plan* p, const dd_sched& sc) {
  const int64_t N = p->N, batch = p->batch;
  const int alpha = p->alpha;
  const int64_t M = (int64_t)alpha * N;
  if (sc.passes == 1) {
    if (N > 4096 || !len_supported((int)N)) return DD_ERR_UNSUPPORTED;
    const KGeom g = geom_single((int)N, p->rbytes);
    if (lds_single((int)N, 1, alpha, p->rbytes) > SINGLE_BUDGET) return DD_ERR_UNSUPPORTED;
    if (sc.lines < 0 || sc.jgroup < 0 || sc.jgroup > alpha) return DD_ERR_UNSUPPORTED;
    const bool real = p->dtype == DD_F32 || p->dtype == DD_F64;
    int lines = sc.lines, groups = sc.jgroup;
    if (lines == 0 || groups == 0) single_shape((int)N, alpha, real, p->rbytes, batch, &lines, &groups);
    if ((int64_t)lines * groups > g.lines || lds_single((int)N, lines, alpha, p->rbytes, groups) > SINGLE_BUDGET)
      return DD_ERR_UNSUPPORTED;
    if (lines > batch) lines = (int)batch;
    p->passes = 1;
    p->N1 = N;
    p->N2 = 1;
    p->s_lines = lines;
    p->s_groups = groups;
    p->s_TL = g.TL;
    p->s_lds = lds_single((int)N, lines, alpha, p->rbytes, groups);
    p->ws_bytes = 0;
    return DD_OK;
  }
  if (sc.passes != 2) return DD_ERR_UNSUPPORTED;
  const int64_t N1 = sc.N1, N2 = sc.N2;
  if (N1 < 1 || N2 < 1 || N1 * N2 != N || N1 > 4096 || N2 > 4096) return DD_ERR_UNSUPPORTED;
  if (!len_supported((int)N1) || !pass2_len_supported((int)N2)) return DD_ERR_UNSUPPORTED;
  if (sc.jgroup > alpha || sc.jgroup < 0 || sc.chunk < 0) return DD_ERR_UNSUPPORTED;
  p->passes = 2;
  p->N1 = N1;
  p->N2 = N2;
  const KGeom g1 = geom_pass((int)N1, p->rbytes);
  const KGeom g2 = geom_pass((int)N2, p->rbytes);
  p->p1_lines = g1.lines;  // compile-time column count of the kernel
  p->p1_TL = g1.TL;
  p->p1_ntile = (int)((N2 + g1.lines - 1) / g1.lines);
  p->p2_lines = g2.lines;
  p->p2_TL = g2.TL;
  p->p2_ntile = (int)((alpha * N1 + g2.lines - 1) / g2.lines);
  p->p2_lds = lds_pass2((int)N2, g2.lines, p->rbytes);
  const KGeom g2f = geom_pass2((int)N2, p->rbytes);
  p->p2f_lines = g2f.lines;
  p->p2f_ntile = (int)((alpha * N1 + g2f.lines - 1) / g2f.lines);
  p->p2f_lds = lds_pass2((int)N2, g2f.lines, p->rbytes);
  p->p2h_lds = lds_pass2((int)N2, g2.lines, p->rbytes, g2.lines + 1);
  p->p2_half = (p->dtype == DD_F32 || p->dtype == DD_F64) && p->p2h_lds <= (size_t)LDS_PASS_MAX;
  // scratch rows padded off a power-of-two stride (scratch_row_pad)
  p->y_row = N2 + scratch_row_pad(N2, alpha, (int)cx_bytes(p));
  p->y_sig = (int64_t)alpha * N1 * p->y_row;
  (void)M;
  // signals per pass pair: by default the scratch of one chunk within 128 MiB
  const size_t per_sig = (size_t)p->y_sig * cx_bytes(p);
  int64_t chunk = sc.chunk;
  if (chunk <= 0) chunk = (int64_t)((128u << 20) / per_sig);
  if (chunk < 1) chunk = 1;
  if (chunk > batch) chunk = batch;
  p->chunk = chunk;
  // j values per pass-1 block: by default all alpha (x and the
  // post-twiddles are read once per block) unless that leaves fewer than
  // two blocks per CU
  int jg = sc.jgroup;
  if (jg <= 0) {
    jg = alpha;
    while (jg > 1 && chunk * p->p1_ntile * ((alpha + jg - 1) / jg) < 512) jg = (jg + 1) / 2;
  }
  p->p1_jgroup = jg;
  p->p1_njg = (alpha + jg - 1) / jg;
  // stage the block's pre-twiddles in LDS: whole rows when they take at most
  // 16 KiB, else their two factors (mode 2) when that costs no block of
  // residency per CU.  The j loop then reads no global memory, so each j's
  // stores stream out while the next j is transformed (2^22 x alpha 16,
  // padded scratch rows: pass 1 at N1 = 4096 319 -> 284 us, at 2048
  // 233 -> 189 us; with unpadded rows the overlapping stores of successive
  // j fell on one memory channel and it was slower, 337 -> 512 us).
  const size_t pre_bytes = (size_t)jg * N1 * cx_bytes(p);
  const size_t cu_lds = 160 * 1024;
  p->p1_pre_lds = pre_bytes <= 16 * 1024 &&
                  lds_pass1((int)N1, g1.lines, p->rbytes, pass1_pre_elems(1, jg, (int)N1)) <= (size_t)LDS_PASS_MAX
                      ? 1 : 0;
  if (!p->p1_pre_lds) {
    const size_t l0 = lds_pass1((int)N1, g1.lines, p->rbytes, 0);
    const size_t l2 = lds_pass1((int)N1, g1.lines, p->rbytes, pass1_pre_elems(2, jg, (int)N1));
    if (l2 <= (size_t)LDS_PASS_MAX && cu_lds / l2 == cu_lds / l0) p->p1_pre_lds = 2;
  }
  p->p1_lds = lds_pass1((int)N1, g1.lines, p->rbytes, pass1_pre_elems(p->p1_pre_lds, jg, (int)N1));
  // and the block's W_{alpha N}^{j n2} when they take at most 4 KiB and do
  // not cost a block of residency per CU
  {
    const int pre_el = pass1_pre_elems(p->p1_pre_lds, jg, (int)N1);
    const int q_el = jg * g1.lines;
    const size_t with_q = lds_pass1((int)N1, g1.lines, p->rbytes, pre_el + q_el);
    p->p1_q_lds = (size_t)q_el * cx_bytes(p) <= 4096 && with_q <= (size_t)LDS_PASS_MAX &&
                  cu_lds / with_q == cu_lds / p->p1_lds ? 1 : 0;
    if (p->p1_q_lds) p->p1_lds = with_q;
  }
  // a chunk's launches must stay within one dispatch's grid: the default
  // chunk shrinks to fit, a requested one that does not fit is refused
  {
    const int64_t b1 = max_launch_blocks(p->p1_lines * p->p1_TL) / ((int64_t)p->p1_ntile * p->p1_njg);
    int64_t b2 = max_launch_blocks((p->p2_lines + 1) * p->p2_TL) / p->p2_ntile;
    const int64_t b2f = max_launch_blocks(p->p2f_lines * p->p2_TL) / p->p2f_ntile;
    if (b2f < b2) b2 = b2f;
    const int64_t cap = b1 < b2 ? b1 : b2;
    if (cap < 1 || (sc.chunk > 0 && chunk > cap)) return DD_ERR_UNSUPPORTED;
    if (chunk > cap) chunk = cap;
    p->chunk = chunk;
  }
  const size_t inv_pre = (size_t)alpha * N1 * cx_bytes(p);
  p->inv_pre_lds =
      inv_pre <= 16 * 1024 && lds_pass1((int)N1, g1.lines, p->rbytes, alpha * (int)N1) <= (size_t)LDS_PASS_MAX ? 1 : 0;
  p->inv_p1_lds = lds_pass1((int)N1, g1.lines, p->rbytes, p->inv_pre_lds ? alpha * (int)N1 : 0);
  // a column of 4096 doubles with its exchange padding and twiddles exceeds
  // the LDS of a workgroup
  if (p->p1_lds > (size_t)LDS_PASS_MAX || p->p2_lds > (size_t)LDS_PASS_MAX || p->p2f_lds > (size_t)LDS_PASS_MAX ||
      p->inv_p1_lds > (size_t)LDS_PASS_MAX)
    return DD_ERR_UNSUPPORTED;
  p->ws_bytes = (size_t)chunk * per_sig;
  return DD_OK;
}

// The tuned schedule of the plan's class if the tuning table has one the
// kernels can run, else the built-in rules.
dd_status configure_auto(dd_plan* p) {
  dd_sched sc;
  if (tune_lookup_plan(p->N, p->alpha, (int)p->dtype, p->batch, &sc) && configure(p, sc) == DD_OK) return DD_OK;
  return default_sched(p->N, p->alpha, p->rbytes, &sc) ? configure(p, sc) : DD_ERR_UNSUPPORTED;
}

// The resolved schedule of a configured plan.
dd_sched resolved(const dd_plan* p) {
  dd_sched o{};
  o.passes = p->passes;
  o.lines = p->passes == 1 ? p->s_lines : 0;
  o.N1 = p->N1;
  o.N2 = p->N2;
  o.jgroup = p->passes == 2 ? p->p1_jgroup : p->s_groups;
  o.chunk = p->passes == 2 ? p->chunk : 0;
  return o;
}

// Plan with the schedule `force`, or (NULL) the tuned schedule of this
// problem class if the tuning table has one, else the built-in rules.
dd_status plan_build(dd_plan_t* out, int64_t N, int32_t alpha, double T, int64_t batch, dd_dtype dtype,
                     uint32_t flags, const dd_sched* force) {
  if (!out) return DD_ERR_INVALID;
  *out = nullptr;
  if (N < 1 || batch < 1 || !(T > 0.0) || !std::isfinite(T)) return DD_ERR_INVALID;
  if (dtype != DD_F32 && dtype != DD_C64 && dtype != DD_F64 && dtype != DD_C128) return DD_ERR_INVALID;
  if (flags & ~(uint32_t)(DD_TWIDDLE_FP32 | DD_NO_WORKSPACE)) return DD_ERR_INVALID;
  if (alpha < 1) return DD_ERR_UNSUPPORTED;
  const int64_t M = (int64_t)alpha * N;
  if (M > ((int64_t)1 << 31) || batch > INT64_MAX / M) return DD_ERR_UNSUPPORTED;
  if (!is_smooth(N)) return DD_ERR_UNSUPPORTED;
  if (!scale_ok(T / (double)N, dtype == DD_F64 || dtype == DD_C128)) return DD_ERR_UNSUPPORTED;

  dd_plan* p = new (std::nothrow) dd_plan;
  if (!p) return DD_ERR_NOMEM;
  p->N = N;
  p->alpha = alpha;
  p->T = T;
  p->batch = batch;
  p->dtype = dtype;
  p->flags = flags;
  p->dbl = dtype == DD_F64 || dtype == DD_C128;
  p->rbytes = p->dbl ? 8 : 4;
  p->in_bytes = dtype == DD_F32 ? 4 : dtype == DD_C128 ? 16 : 8;
  const bool fp32tw = !p->dbl && (flags & DD_TWIDDLE_FP32);
  dd_status st = force ? configure(p, *force) : configure_auto(p);
  if (st != DD_OK) {
    delete p;
    return st;
  }
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return DD_ERR_DEVICE;
  }

  // Device tables, generated on the GPU (FP64 unless the FP32 variant).
  hipStream_t s = nullptr;
  st = gen_stage_table(p, &p->twL1, (int)p->N1, fp32tw, s, p->passes == 1 && single_narrow((int)p->N1));
  if (st == DD_OK) st = gen_table(p, &p->twPre, alpha, p->N1, (int64_t)alpha * p->N1, fp32tw, s);
  if (st == DD_OK && p->passes == 2) {
    st = gen_stage_table(p, &p->twL2, (int)p->N2, fp32tw, s);
    if (st == DD_OK) st = gen_table(p, &p->twQ, alpha, p->N2, M, fp32tw, s);
    if (st == DD_OK) st = gen_table(p, &p->twPost, p->N1, p->N2, N, fp32tw, s);
    if (st == DD_OK && !(flags & DD_NO_WORKSPACE)) st = hip_status(hipMalloc(&p->ws, p->ws_bytes));
  }
  if (st == DD_OK) st = hip_status(hipStreamSynchronize(s));
  if (st != DD_OK) {
    free_tables(p);
    delete p;
    return st;
  }
  *out = p;
  return DD_OK;
}

}  // namespace

extern "C" {

const char* dense_dft_status_string(dd_status s) {
  switch (s) {
    case DD_OK: return "ok";
    case DD_ERR_INVALID: return "invalid argument";
    case DD_ERR_UNSUPPORTED: return "unsupported size or parameter";
    case DD_ERR_NOMEM: return "out of memory";
    case DD_ERR_DEVICE: return "device error";
    case DD_ERR_BUSY: return "busy";
    case DD_ERR_TOO_LARGE: return "request exceeds the memory budget";
    case DD_ERR_TIMEOUT: return "timed out";
    case DD_ERR_CLOSED: return "closed";
  }
  return "unknown status";
}

int32_t dense_dft_version(void) { return 100; }

dd_status dense_dft_plan(dd_plan_t* out, int64_t N, int32_t alpha, double T, int64_t batch, dd_dtype dtype,
                         uint32_t flags) {
  return plan_build(out, N, alpha, T, batch, dtype, flags, nullptr);
}

dd_status dense_dft_plan_sched(dd_plan_t* out, int64_t N, int32_t alpha, double T, int64_t batch, dd_dtype dtype,
                               uint32_t flags, const dd_sched* sched) {
  if (!sched) {
    if (out) *out = nullptr;
    return DD_ERR_INVALID;
  }
  return plan_build(out, N, alpha, T, batch, dtype, flags, sched);
}

dd_status dense_dft_plan_get_sched(dd_plan_t p, dd_sched* out) {
  if (!p || !out) return DD_ERR_INVALID;
  *out = resolved(p->inner ? p->inner : p);
  return DD_OK;
}

dd_status dense_dft_plan_decimated(dd_plan_t* out, int64_t N, int32_t p, double T, int64_t batch, dd_dtype dtype,
                                   uint32_t flags) {
  if (!out) return DD_ERR_INVALID;
  *out = nullptr;
  if (N < 1 || batch < 1 || !(T > 0.0) || !std::isfinite(T)) return DD_ERR_INVALID;
  if (dtype != DD_F32 && dtype != DD_C64 && dtype != DD_F64 && dtype != DD_C128) return DD_ERR_INVALID;
  if (flags & ~(uint32_t)(DD_TWIDDLE_FP32 | DD_NO_WORKSPACE)) return DD_ERR_INVALID;
  if (p < 1 || N % p != 0) return DD_ERR_UNSUPPORTED;
  if (p == 1) return plan_build(out, N, 1, T, batch, dtype, flags, nullptr);
  const int64_t Np = N / p;
  if (batch > INT64_MAX / N) return DD_ERR_UNSUPPORTED;
  // the inner plan's factor T'/N' with T' = T/p is the transform's T/N
  dd_plan_t in = nullptr;
  dd_status st = plan_build(&in, Np, 1, T / p, batch, dtype, flags | DD_NO_WORKSPACE, nullptr);
  if (st != DD_OK) return st;
  dd_plan* w = new (std::nothrow) dd_plan;
  if (!w) {
    dense_dft_destroy(in);
    return DD_ERR_NOMEM;
  }
  w->device = in->device;
  w->N = N;
  w->alpha = 1;
  w->T = T;
  w->batch = batch;
  w->dtype = dtype;
  w->flags = flags;
  w->dbl = in->dbl;
  w->rbytes = in->rbytes;
  w->in_bytes = in->in_bytes;
  w->passes = in->passes;
  w->N1 = in->N1;
  w->N2 = in->N2;
  w->dec_p = p;
  w->inner = in;
  w->fold_bytes = ((size_t)batch * Np * in->in_bytes + 255) / 256 * 256;
  w->ws_bytes = w->fold_bytes + in->ws_bytes;
  if (!(flags & DD_NO_WORKSPACE)) {
    st = hip_status(hipMalloc(&w->ws, w->ws_bytes));
    if (st != DD_OK) {
      dense_dft_destroy(in);
      delete w;
      return st == DD_ERR_DEVICE ? DD_ERR_NOMEM : st;
    }
  }
  *out = w;
  return DD_OK;
}

dd_status dense_dft_sched_candidates(int64_t N, int32_t alpha, int64_t batch, dd_dtype dtype, dd_sched* out,
                                     int32_t cap, int32_t* count) {
  if (!count || cap < 0 || (cap > 0 && !out)) return DD_ERR_INVALID;
  *count = 0;
  if (N < 1 || batch < 1) return DD_ERR_INVALID;
  if (dtype != DD_F32 && dtype != DD_C64 && dtype != DD_F64 && dtype != DD_C128) return DD_ERR_INVALID;
  if (alpha < 1) return DD_ERR_UNSUPPORTED;
  if ((int64_t)alpha * N > ((int64_t)1 << 31) || !is_smooth(N)) return DD_ERR_UNSUPPORTED;
  // a host-only plan record: configure() validates each schedule
  dd_plan p;
  p.N = N;
  p.alpha = alpha;
  p.batch = batch;
  p.dtype = dtype;
  p.dbl = dtype == DD_F64 || dtype == DD_C128;
  p.rbytes = p.dbl ? 8 : 4;
  std::vector<dd_sched> c;
  auto add = [&](const dd_sched& sc) {
    if (configure(&p, sc) != DD_OK) return;
    const dd_sched r = resolved(&p);
    for (const dd_sched& o : c)
      if (o.passes == r.passes && o.lines == r.lines && o.N1 == r.N1 && o.N2 == r.N2 && o.jgroup == r.jgroup &&
          o.chunk == r.chunk)
        return;
    c.push_back(r);
  };
  if (configure_auto(&p) == DD_OK) add(resolved(&p));
  if (N <= 4096 && len_supported((int)N)) {
    const KGeom g = geom_single((int)N, p.rbytes);
    for (const int groups : single_group_options(single_jn(alpha, dtype == DD_F32 || dtype == DD_F64), g.lines))
      for (const int lines : single_line_options(g.lines, groups)) {
        if (lines > batch) continue;
        dd_sched sc{};
        sc.passes = 1;
        sc.lines = lines;
        sc.jgroup = groups;
        sc.N1 = N;
        sc.N2 = 1;
        add(sc);
      }
  }
  for (int64_t n2 = 2; n2 <= 4096; n2 *= 2) {
    if (N % n2) continue;
    for (int jg = alpha;; jg = (jg + 1) / 2) {
      dd_sched sc{};
      sc.passes = 2;
      sc.N1 = N / n2;
      sc.N2 = n2;
      sc.jgroup = jg;
      add(sc);
      if (jg == alpha && configure(&p, sc) == DD_OK) {
        // larger chunks: more pass-1 blocks resident per CU (each block
        // runs every j of its columns in turn)
        const int64_t c0 = p.chunk;
        for (const int64_t ch : {c0 + c0 / 2, 2 * c0}) {
          if (ch > batch) continue;
          dd_sched sc2 = sc;
          sc2.chunk = ch;
          add(sc2);
        }
      }
      if (jg == 1) break;
    }
  }
  for (size_t i = 0; i < c.size() && (int32_t)i < cap; ++i) out[i] = c[i];
  *count = (int32_t)c.size();
  return c.empty() ? DD_ERR_UNSUPPORTED : DD_OK;
}

dd_status dense_dft_workspace_size(dd_plan_t p, size_t* bytes) {
  if (!p || !bytes) return DD_ERR_INVALID;
  *bytes = p->ws_bytes;
  return DD_OK;
}

dd_status dense_dft_plan_info(dd_plan_t p, int32_t* passes, int64_t* N1, int64_t* N2) {
  if (!p) return DD_ERR_INVALID;
  if (passes) *passes = p->passes;
  if (N1) *N1 = p->N1;
  if (N2) *N2 = p->N2;
  return DD_OK;
}

}  // extern "C"

namespace {

// chunk: signals per pass pair of a two-pass plan (the plan's own, or fewer
// when the scratch is smaller than the plan's workspace); each signal's
// arithmetic does not depend on it.
template <typename R, typename In>
dd_status exec_typed(dd_plan* p, const In* x, cx<R>* X, cx<R>* ws, hipStream_t s, int64_t chunk) {
  const R scale = (R)(p->T / (double)p->N);
  const int64_t M = (int64_t)p->alpha * p->N;
  if (p->passes == 1) {
    DenseArgs<R> a{};
    a.batch = p->batch;
    a.x_stride = p->N;
    a.y_stride = M;
    a.N1 = (int)p->N;
    a.N2 = 1;
    a.alpha = p->alpha;
    a.lines = p->s_lines;
    a.jgroup = p->s_groups;
    a.scale = scale;
    a.twL = static_cast<const cx<R>*>(p->twL1);
    a.twPre = static_cast<const cx<R>*>(p->twPre);
    const int block = p->s_lines * p->s_groups * p->s_TL;
    const int64_t per = max_launch_blocks(block) * p->s_lines;  // signals per launch
    for (int64_t b0 = 0; b0 < p->batch; b0 += per) {
      a.batch = p->batch - b0 < per ? p->batch - b0 : per;
      LaunchCfg c{(a.batch + p->s_lines - 1) / p->s_lines, block, p->s_lds, s};
      const hipError_t e =
          timed_launch(p, 1, s, [&] { return launch_single((int)p->N, c, x + b0 * p->N, X + b0 * M, a); });
      if (e != hipSuccess) return hip_status(e);
    }
    return DD_OK;
  }
  for (int64_t c0 = 0; c0 < p->batch; c0 += chunk) {
    const int64_t nb = p->batch - c0 < chunk ? p->batch - c0 : chunk;
    DenseArgs<R> a1{};
    a1.batch = nb;
    a1.x_stride = p->N;
    a1.y_stride = M;
    a1.ysig = p->y_sig;
    a1.yrow = (int)p->y_row;
    a1.N1 = (int)p->N1;
    a1.N2 = (int)p->N2;
    a1.alpha = p->alpha;
    a1.lines = p->p1_lines;
    a1.ntile = p->p1_ntile;
    a1.jgroup = p->p1_jgroup;
    a1.njg = p->p1_njg;
    a1.pre_lds = p->p1_pre_lds;
    a1.q_lds = p->p1_q_lds;
    // real samples: the spectrum is Hermitian, so only the scratch rows
    // m1 <= H = alpha N1 / 2 are stored and transformed (the rest are mirrors)
    const bool half = std::is_floating_point<In>::value && p->p2_half;
    const int A = p->alpha * (int)p->N1, H = A / 2;
    a1.hrows = half ? H + 1 : 0;
    a1.scale = scale;
    a1.twL = static_cast<const cx<R>*>(p->twL1);
    a1.twPre = static_cast<const cx<R>*>(p->twPre);
    a1.twQ = static_cast<const cx<R>*>(p->twQ);
    a1.twPost = static_cast<const cx<R>*>(p->twPost);
    LaunchCfg c1{nb * p->p1_ntile * p->p1_njg, p->p1_lines * p->p1_TL, p->p1_lds, s};
    hipError_t e = timed_launch(p, 2, s, [&] { return launch_pass1((int)p->N1, c1, x + c0 * p->N, ws, a1); });
    if (e != hipSuccess) return hip_status(e);
    DenseArgs<R> a2 = a1;
    a2.lines = half ? p->p2_lines : p->p2f_lines;
    a2.ntile = half ? (A - H + p->p2_lines - 1) / p->p2_lines : p->p2f_ntile;  // blocks of stored rows
    a2.twL = static_cast<const cx<R>*>(p->twL2);
    LaunchCfg c2{nb * a2.ntile, half ? (p->p2_lines + 1) * p->p2_TL : p->p2f_lines * p->p2_TL,
                 half ? p->p2h_lds : p->p2f_lds, s};
    e = timed_launch(p, 3, s, [&] {
      return half ? launch_pass2_half((int)p->N2, c2, ws, X + c0 * M, a2)
                  : launch_pass2((int)p->N2, c2, ws, X + c0 * M, a2);
    });
    if (e != hipSuccess) return hip_status(e);
  }
  return DD_OK;
}

// The inverse transform: the adjoint of the forward schedule, with the same
// tables and geometry (kinds 4, 5, 6 in the profile: one pass, pass A, pass B).
template <typename R>
dd_status exec_inverse_typed(dd_plan* p, const cx<R>* X, cx<R>* x, cx<R>* ws, hipStream_t s) {
  const R scale = (R)(1.0 / ((double)p->alpha * p->T));
  const int64_t M = (int64_t)p->alpha * p->N;
  if (p->passes == 1) {
    DenseArgs<R> a{};
    a.batch = p->batch;
    a.x_stride = p->N;
    a.y_stride = M;
    a.N1 = (int)p->N;
    a.N2 = 1;
    a.alpha = p->alpha;
    a.lines = p->s_lines;
    a.jgroup = p->s_groups;
    a.scale = scale;
    a.twL = static_cast<const cx<R>*>(p->twL1);
    a.twPre = static_cast<const cx<R>*>(p->twPre);
    const int block = p->s_lines * p->s_groups * p->s_TL;
    const int64_t per = max_launch_blocks(block) * p->s_lines;  // signals per launch
    for (int64_t b0 = 0; b0 < p->batch; b0 += per) {
      a.batch = p->batch - b0 < per ? p->batch - b0 : per;
      LaunchCfg c{(a.batch + p->s_lines - 1) / p->s_lines, block, p->s_lds, s};
      const hipError_t e =
          timed_launch(p, 4, s, [&] { return launch_single_inv((int)p->N, c, X + b0 * M, x + b0 * p->N, a); });
      if (e != hipSuccess) return hip_status(e);
    }
    return DD_OK;
  }
  for (int64_t c0 = 0; c0 < p->batch; c0 += p->chunk) {
    const int64_t nb = p->batch - c0 < p->chunk ? p->batch - c0 : p->chunk;
    DenseArgs<R> a{};
    a.batch = nb;
    a.x_stride = p->N;
    a.y_stride = M;
    a.N1 = (int)p->N1;
    a.N2 = (int)p->N2;
    a.alpha = p->alpha;
    a.scale = scale;
    a.twPre = static_cast<const cx<R>*>(p->twPre);
    a.twQ = static_cast<const cx<R>*>(p->twQ);
    a.twPost = static_cast<const cx<R>*>(p->twPost);
    DenseArgs<R> aA = a;
    aA.lines = p->p2_lines;
    aA.ntile = p->p2_ntile;
    aA.twL = static_cast<const cx<R>*>(p->twL2);
    LaunchCfg cA{nb * p->p2_ntile, p->p2_lines * p->p2_TL, p->p2_lds, s};
    hipError_t e = timed_launch(p, 5, s, [&] { return launch_passA((int)p->N2, cA, X + c0 * M, ws, aA); });
    if (e != hipSuccess) return hip_status(e);
    DenseArgs<R> aB = a;
    aB.lines = p->p1_lines;
    aB.ntile = p->p1_ntile;
    aB.pre_lds = p->inv_pre_lds;
    aB.twL = static_cast<const cx<R>*>(p->twL1);
    LaunchCfg cB{nb * p->p1_ntile, p->p1_lines * p->p1_TL, p->inv_p1_lds, s};
    e = timed_launch(p, 6, s, [&] { return launch_passB((int)p->N1, cB, ws, x + c0 * p->N, aB); });
    if (e != hipSuccess) return hip_status(e);
  }
  return DD_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

// The forward transform of a validated plain plan, by input dtype.
dd_status exec_dispatch(dd_plan* p, const void* x, void* X, void* ws, hipStream_t s, int64_t chunk) {
  switch (p->dtype) {
    case DD_F32:
      return exec_typed<float>(p, static_cast<const float*>(x), static_cast<cx<float>*>(X),
                               static_cast<cx<float>*>(ws), s, chunk);
    case DD_C64:
      return exec_typed<float>(p, static_cast<const cx<float>*>(x), static_cast<cx<float>*>(X),
                               static_cast<cx<float>*>(ws), s, chunk);
    case DD_F64:
      return exec_typed<double>(p, static_cast<const double*>(x), static_cast<cx<double>*>(X),
                                static_cast<cx<double>*>(ws), s, chunk);
    case DD_C128:
      return exec_typed<double>(p, static_cast<const cx<double>*>(x), static_cast<cx<double>*>(X),
                                static_cast<cx<double>*>(ws), s, chunk);
  }
  return DD_ERR_INVALID;
}

// Scratch of dense_dft_exec_static: a fixed device array that each device
// the library runs on holds until the process ends.  Host code never uses
// the array's name as an address (on the host it is a stand-in, not device
// memory): its device address is looked up once per device and kept.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)DD_STATIC_SCRATCH_BYTES;

}  // namespace

static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {

constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu;
void* g_static_ptr[STATIC_MAX_DEVICES] = {};

// Device address of `scratch` on `dev` (made current for the lookup).
dd_status static_scratch(int dev, void** out) {
  if (dev < 0 || dev >= STATIC_MAX_DEVICES) return DD_ERR_DEVICE;
  std::lock_guard<std::mutex> g(g_static_mu);
  if (!g_static_ptr[dev]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return DD_ERR_DEVICE;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return DD_ERR_DEVICE;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return DD_ERR_DEVICE;
    }
    g_static_ptr[dev] = ptr;
  }
  *out = g_static_ptr[dev];
  return DD_OK;
}

}  // namespace

extern "C" {

dd_status dense_dft_exec_static(dd_plan_t p, const void* x, void* X, void* stream) {
  if (!p || !x || !X) return DD_ERR_INVALID;
  if (p->inner) return DD_ERR_UNSUPPORTED;
  const size_t out_cx = cx_bytes(p);
  if ((uintptr_t)x % p->in_bytes != 0 || (uintptr_t)X % out_cx != 0) return DD_ERR_INVALID;
  const size_t in_total = (size_t)p->batch * p->N * p->in_bytes;
  const size_t out_total = (size_t)p->batch * p->alpha * p->N * out_cx;
  if (overlaps(x, in_total, X, out_total)) return DD_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->passes == 1) return exec_dispatch(p, x, X, nullptr, s, p->chunk);
  // two passes: as many signals per pass pair as the array holds, at most
  // the plan's own chunk (within one dispatch's grid)
  const size_t per_sig = (size_t)p->y_sig * out_cx;
  if (per_sig > STATIC_SCRATCH_BYTES) return DD_ERR_TOO_LARGE;
  int64_t chunk = (int64_t)(STATIC_SCRATCH_BYTES / per_sig);
  if (chunk > p->chunk) chunk = p->chunk;
  void* ws = nullptr;
  const dd_status st = static_scratch(p->device, &ws);
  if (st != DD_OK) return st;
  return exec_dispatch(p, x, X, ws, s, chunk);
}

dd_status dense_dft_exec(dd_plan_t p, const void* x, void* X, void* workspace, void* stream) {
  if (!p || !x || !X) return DD_ERR_INVALID;
  if (p->inner) {
    // alpha = 1/p: fold into the workspace, then the plain length-N/p plan
    const size_t in_total = (size_t)p->batch * p->N * p->in_bytes;
    const size_t out_total = (size_t)p->batch * p->inner->N * cx_bytes(p);
    if ((uintptr_t)x % p->in_bytes != 0 || (uintptr_t)X % cx_bytes(p) != 0) return DD_ERR_INVALID;
    if (overlaps(x, in_total, X, out_total)) return DD_ERR_INVALID;
    void* ws = workspace ? workspace : p->ws;
    if (!ws || (uintptr_t)ws % 16 != 0) return DD_ERR_INVALID;
    if (overlaps(ws, p->ws_bytes, x, in_total) || overlaps(ws, p->ws_bytes, X, out_total)) return DD_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e = launch_fold(p->dtype, x, ws, p->batch, p->N, p->inner->N, p->dec_p, s);
    if (e != hipSuccess) return hip_status(e);
    void* iws = p->inner->ws_bytes ? static_cast<char*>(ws) + p->fold_bytes : nullptr;
    return dense_dft_exec(p->inner, ws, X, iws, stream);
  }
  const size_t out_cx = cx_bytes(p);
  const size_t in_align = p->in_bytes;
  if ((uintptr_t)x % in_align != 0 || (uintptr_t)X % out_cx != 0) return DD_ERR_INVALID;
  const size_t in_total = (size_t)p->batch * p->N * p->in_bytes;
  const size_t out_total = (size_t)p->batch * p->alpha * p->N * out_cx;
  if (overlaps(x, in_total, X, out_total)) return DD_ERR_INVALID;
  void* ws = workspace ? workspace : p->ws;
  if (p->passes == 2) {
    if (!ws || (uintptr_t)ws % out_cx != 0) return DD_ERR_INVALID;
    if (overlaps(ws, p->ws_bytes, X, out_total) || overlaps(ws, p->ws_bytes, x, in_total))
      return DD_ERR_INVALID;
  }
  return exec_dispatch(p, x, X, ws, static_cast<hipStream_t>(stream), p->chunk);
}

dd_status dense_dft_exec_inverse(dd_plan_t p, const void* X, void* x, void* workspace, void* stream) {
  if (!p || !X || !x) return DD_ERR_INVALID;
  if (p->inner) return DD_ERR_UNSUPPORTED;  // alpha < 1 is a one-way transform (the fold loses information)
  if (!scale_ok(1.0 / ((double)p->alpha * p->T), p->dbl)) return DD_ERR_UNSUPPORTED;
  const size_t cxb = cx_bytes(p);
  if ((uintptr_t)X % cxb != 0 || (uintptr_t)x % cxb != 0) return DD_ERR_INVALID;
  const size_t in_total = (size_t)p->batch * p->alpha * p->N * cxb;
  const size_t out_total = (size_t)p->batch * p->N * cxb;
  if (overlaps(X, in_total, x, out_total)) return DD_ERR_INVALID;
  void* ws = workspace ? workspace : p->ws;
  if (p->passes == 2) {
    if (!ws || (uintptr_t)ws % cxb != 0) return DD_ERR_INVALID;
    if (overlaps(ws, p->ws_bytes, X, in_total) || overlaps(ws, p->ws_bytes, x, out_total)) return DD_ERR_INVALID;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->dbl)
    return exec_inverse_typed<double>(p, static_cast<const cx<double>*>(X), static_cast<cx<double>*>(x),
                                      static_cast<cx<double>*>(ws), s);
  return exec_inverse_typed<float>(p, static_cast<const cx<float>*>(X), static_cast<cx<float>*>(x),
                                   static_cast<cx<float>*>(ws), s);
}

dd_status dense_dft_destroy(dd_plan_t p) {
  if (!p) return DD_ERR_INVALID;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  free_events(p);
  free_tables(p);
  (void)hipSetDevice(cur);
  if (p->inner) dense_dft_destroy(p->inner);
  delete p;
  return DD_OK;
}

dd_status dense_dft_profile_begin(dd_plan_t p, int32_t max_launches) {
  if (!p || max_launches < 1) return DD_ERR_INVALID;
  if (p->inner) return dense_dft_profile_begin(p->inner, max_launches);
  free_events(p);
  try {
    p->prof_ev.resize(2 * (size_t)max_launches, nullptr);
    p->prof_kind.assign((size_t)max_launches, 0);
  } catch (...) {
    free_events(p);
    return DD_ERR_NOMEM;
  }
  for (auto& e : p->prof_ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      free_events(p);
      return DD_ERR_DEVICE;
    }
  }
  p->prof_n = 0;
  p->prof_on = true;
  return DD_OK;
}

dd_status dense_dft_profile_end(dd_plan_t p, int32_t* kinds, float* ms, int32_t cap, int32_t* count) {
  if (!p || !count || (cap > 0 && (!kinds || !ms))) return DD_ERR_INVALID;
  if (p->inner) return dense_dft_profile_end(p->inner, kinds, ms, cap, count);
  dd_status st = DD_OK;
  const int n = p->prof_n;
  if (n > 0 && hipEventSynchronize(p->prof_ev[2 * n - 1]) != hipSuccess) st = DD_ERR_DEVICE;
  int w = 0;
  for (int i = 0; st == DD_OK && i < n && w < cap; ++i, ++w) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, p->prof_ev[2 * i], p->prof_ev[2 * i + 1]) != hipSuccess) st = DD_ERR_DEVICE;
    kinds[w] = p->prof_kind[i];
    ms[w] = t;
  }
  *count = w;
  free_events(p);
  return st;
}

}  // extern "C"
