// HIP kernels of the levelized STA sweep for CDNA4 (gfx950, wave64), and the C ABI calls
// that launch them (sta_forward, sta_backward).
//
// Data layout (canonical order from sta_levelize): nets sorted by level, pins net-major
// with the driver first.  The forward sweep keeps one 48-byte record per net - the
// driver's arrival time and slew for the four conditions and its smoothed late arrival -
// and derives a sink's state on demand from its driver record plus the sink's
// {wire delay, impulse}.  A level therefore gathers one record per cell input and writes
// one record per net; per-pin outputs are written by the backward sweep, which visits
// every pin anyway.
//
// Lane mapping (the pin-based scheme of Sec. 3.1, re-derived for 64-lane wavefronts):
// net-level work (RC delay, backward net step, adjoint) gives each net a group of 4, 8,
// 16, 32 or 64 lanes chosen from its sink count, packing 16 small nets into one wave and
// giving a heavy-tailed net the whole wave; reductions over a net's sinks are xor
// butterflies inside the group (fixed order, no atomics, Sec. 3.1.1).  Cell-level work
// gives each cell 4 lanes, one per timing condition (the condition axis of Alg. 1).
#include <cmath>

#include "sta_internal.h"

namespace sta {
namespace {

constexpr float kInf = __builtin_huge_valf();

// ---------------------------------------------------------------------------- helpers
// Table cell of v along an axis: upper_bound(axis, v) - 1 clamped to [0, 5], computed as
// the number of interior breakpoints not above v.
__device__ __forceinline__ int find_cell(float v, const float (&k)[STA_LUT_N - 2]) {
  return (int)(v >= k[0]) + (int)(v >= k[1]) + (int)(v >= k[2]) + (int)(v >= k[3]) + (int)(v >= k[4]);
}

struct LutVal {
  float d, s;          // delay and output slew
  float ddx, ddy;      // d delay / d input slew, d delay / d load
  float dsx, dsy;      // d slew / d input slew, d slew / d load
};

// Bilinear table lookup with linear extrapolation (Sec. 3.1.2).  The delay and slew tables
// of one arc and output transition share the cell, so both come from two 16-byte loads of
// precomputed coefficients v = a + b*tx + c*ty + d*tx*ty.
template <bool kPartials>
__device__ __forceinline__ LutVal lut_eval(const float4* __restrict__ grid, const float4* __restrict__ coef,
                                           const LutKeys& keys, int arc, int tr, float xv, float yv) {
  const int cell = find_cell(xv, keys.x) * (STA_LUT_N - 1) + find_cell(yv, keys.y);
  const float4 g = grid[cell];
  const float tx = (xv - g.x) * g.y;
  const float ty = (yv - g.z) * g.w;
  const float4* c = coef + ((size_t)(arc * 2 + tr) * kLutCells + cell) * 2;
  const float4 cd = c[0];
  const float4 cs = c[1];
  const float bd = fmaf(cd.w, ty, cd.y);
  const float bs = fmaf(cs.w, ty, cs.y);
  LutVal r;
  r.d = fmaf(tx, bd, fmaf(cd.z, ty, cd.x));
  r.s = fmaf(tx, bs, fmaf(cs.z, ty, cs.x));
  if (kPartials) {
    r.ddx = bd * g.y;
    r.dsx = bs * g.y;
    r.ddy = fmaf(cd.w, tx, cd.z) * g.w;
    r.dsy = fmaf(cs.w, tx, cs.z) * g.w;
  } else {
    r.ddx = r.ddy = r.dsx = r.dsy = 0.f;
  }
  return r;
}

// Slew at a sink: the driver slew combined with the wire's impulse.
__device__ __forceinline__ float sink_slew(float drv_slew, float imp) {
  return sqrtf(fmaf(drv_slew, drv_slew, imp * imp));
}

// Running log-sum-exp (Eq. 4) with the maximum as the shift.
__device__ __forceinline__ void lse_push(float& m, float& s, float v, float inv_gamma) {
  if (v > m) {
    s = fmaf(s, expf((m - v) * inv_gamma), 1.0f);
    m = v;
  } else {
    s += expf((v - m) * inv_gamma);
  }
}

__device__ __forceinline__ float grp_sum(float v, int G) {
  for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ float grp_min(float v, int G) {
  for (int o = 1; o < G; o <<= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float grp_max(float v, int G) {
  for (int o = 1; o < G; o <<= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ float sgnf(float v) { return (v > 0.f) ? 1.f : ((v < 0.f) ? -1.f : 0.f); }

// Lane-group assignment of one wave inside a GroupRange (all lanes of a wave agree on the
// class; lanes of one group agree on the net).
struct GroupSlot {
  int G;        // lanes per net
  int gl;       // lane index inside the group
  int entry;    // schedule entry, valid if active
  bool active;
};

__device__ __forceinline__ bool group_slot(const GroupRange& r, int wave, int lane, GroupSlot& s) {
  if (wave >= r.wave_off[kNumClasses]) return false;
  int c = 0;
  while (c < kNumClasses - 1 && wave >= r.wave_off[c + 1]) ++c;
  s.G = 4 << c;
  s.gl = lane & (s.G - 1);
  s.entry = r.cls_off[c] + (wave - r.wave_off[c]) * (64 >> (2 + c)) + (lane >> (2 + c));
  s.active = s.entry < r.cls_off[c + 1];
  return true;
}

// ---------------------------------------------------------------------------- RC (Alg. 1)
struct RcArgs {
  const int* net_off;
  const float* pin_cap;
  const float* x;
  const float* y;
  const int* io_perm;        // canonical -> caller index, or NULL
  const int* sched;
  GroupRange range;
  float2* wire;
  float* load;
  float4* rec;
  int N0;
  float r, c, pi_at, pi_slew;
};

// RC net delay of every net (Sec. 3.1.1, Eq. 1-3, star nets): per sink the wire delay and
// impulse, per net the root load by a group reduction.  Level-0 (primary input) records
// are initialised here too.
__global__ __launch_bounds__(kBlock) void k_rc(RcArgs a) {
  const int wave = (int)((blockIdx.x * kBlock + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  GroupSlot gs;
  if (!group_slot(a.range, wave, lane, gs)) return;
  const int n = gs.active ? a.sched[gs.entry] : 0;
  int p0 = 0, p1 = 0;
  float xd = 0.f, yd = 0.f;
  if (gs.active) {
    p0 = a.net_off[n];
    p1 = a.net_off[n + 1];
    const int q = a.io_perm ? a.io_perm[p0] : p0;
    xd = a.x[q];
    yd = a.y[q];
  }
  float sum = 0.f;
  for (int p = p0 + 1 + gs.gl; p < p1; p += gs.G) {
    const int q = a.io_perm ? a.io_perm[p] : p;
    const float cp = a.pin_cap[p];
    const float len = fabsf(a.x[q] - xd) + fabsf(a.y[q] - yd);
    const float res = a.r * len;                 // Res(fa(u) -> u)
    const float cw = a.c * len;                  // wire capacitance, half at each end
    const float cap = fmaf(0.5f, cw, cp);        // Cap(u) of the sink node
    const float load = cap;                      // Eq. 1 at a leaf
    const float dly = 1e-3f * res * load;        // Eq. 2 (ohm * fF = 1e-3 ps)
    const float arg = 2.0f * (1e-3f * res * cap) * dly - dly * dly;   // Eq. 3
    const float imp = arg > 0.f ? sqrtf(arg) : 0.f;
    a.wire[p] = make_float2(dly, imp);
    sum += cp + cw;                              // the sink's Load plus the root half of the wire
  }
  sum = grp_sum(sum, gs.G);
  if (gs.active && gs.gl == 0) {
    a.load[n] = a.pin_cap[p0] + sum;             // Eq. 1 at the root
    a.wire[p0] = make_float2(0.f, 0.f);
    if (n < a.N0) {
      float4* r = a.rec + 3 * (size_t)n;
      r[0] = make_float4(a.pi_at, a.pi_at, a.pi_at, a.pi_at);
      r[1] = make_float4(a.pi_slew, a.pi_slew, a.pi_slew, a.pi_slew);
      r[2] = make_float4(a.pi_at, a.pi_at, 0.f, 0.f);
    }
  }
}

// ---------------------------------------------------------------------------- forward level
struct FwdArgs {
  const int* cell_type;
  const int* type_arc0;
  const int8_t* unate;
  const int* cin_off;
  const int* cin_src;
  const int* cin_pin;
  const float2* wire;
  const float* load;
  float4* rec;
  const float4* grid;
  const float4* coef;
  LutKeys keys;
  int N0;
  float gamma, inv_gamma;
  int smooth;
};

// One level of forward propagation (Sec. 3.1.2): 4 lanes per cell, lane k handles
// condition k = 2*mode + transition over all of the cell's arcs.
__global__ __launch_bounds__(kBlock) void k_fwd_level(FwdArgs a, int c0, int c1) {
  const int gid = (int)(blockIdx.x * kBlock + threadIdx.x);
  const int cell = c0 + (gid >> 2);
  if (cell >= c1) return;
  const int k = gid & 3, m = k >> 1, t = k & 1;
  const int n = a.N0 + cell;
  const float load = a.load[n];
  const int arc0 = a.type_arc0[a.cell_type[cell]];
  const int j0 = a.cin_off[cell], j1 = a.cin_off[cell + 1];
  float best_at = m ? -kInf : kInf;
  float best_sl = best_at;
  float lm = -kInf, ls = 0.f;
  for (int j = j0; j < j1; ++j) {
    const int arc = arc0 + (j - j0);
    const int tp = a.unate[arc] > 0 ? t : 1 - t;     // input transition
    const int kp = 2 * m + tp;
    const float* src = reinterpret_cast<const float*>(a.rec + 3 * (size_t)a.cin_src[j]);
    const float2 w = a.wire[a.cin_pin[j]];
    const float at_in = src[kp] + w.x;
    const float sl_in = sink_slew(src[4 + kp], w.y);
    const LutVal v = lut_eval<false>(a.grid, a.coef, a.keys, arc, t, sl_in, load);
    const float cand = at_in + v.d;
    if (m) {
      best_at = fmaxf(best_at, cand);
      best_sl = fmaxf(best_sl, v.s);
      if (a.smooth) lse_push(lm, ls, (src[8 + tp] + w.x) + v.d, a.inv_gamma);
    } else {
      best_at = fminf(best_at, cand);
      best_sl = fminf(best_sl, v.s);
    }
  }
  float* o = reinterpret_cast<float*>(a.rec + 3 * (size_t)n);
  o[k] = best_at;
  o[4 + k] = best_sl;
  if (m) o[8 + t] = a.smooth ? fmaf(a.gamma, logf(ls), lm) : __builtin_nanf("");
}

// ---------------------------------------------------------------------------- endpoints
struct EpArgs {
  const int* ep_pin;
  const int* ep_net;
  const float4* rec;
  const float2* wire;
  double* part;        // [blocks][5]
  double* fin;         // [8]
  double* scalars;     // [4] or NULL
  float4* ratp;
  float4* adjp;
  const double* scale_dev;
  int E, n_blocks;
  float rat_late, hold, gamma, inv_gamma, scale;
  int smooth, wns_mode;
};

struct EpVals {
  float worst;    // hard late slack, worst transition
  float sg;       // smoothed slack s_e
  float w0, w1;   // d s_e / d slack_g(e, t)
};

__device__ __forceinline__ EpVals endpoint_values(const EpArgs& a, int i) {
  const int e = a.ep_pin[i];
  const float* r = reinterpret_cast<const float*>(a.rec + 3 * (size_t)a.ep_net[i]);
  const float dl = a.wire[e].x;
  EpVals v;
  v.worst = fminf(a.rat_late - (r[2] + dl), a.rat_late - (r[3] + dl));
  // s_e = -LSE(-slack_g(rise), -slack_g(fall))
  const float u0 = -(a.rat_late - (r[8] + dl));
  const float u1 = -(a.rat_late - (r[9] + dl));
  const float mx = fmaxf(u0, u1);
  const float e0 = expf((u0 - mx) * a.inv_gamma), e1 = expf((u1 - mx) * a.inv_gamma);
  const float z = e0 + e1;
  v.sg = -(mx + a.gamma * logf(z));
  v.w0 = e0 / z;
  v.w1 = e1 / z;
  return v;
}

template <int NT>
__device__ __forceinline__ double block_reduce(double v, double* sh, bool is_max) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const double b = sh[threadIdx.x + o];
      sh[threadIdx.x] = is_max ? fmax(sh[threadIdx.x], b) : sh[threadIdx.x] + b;
    }
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Per-block partial sums over endpoints, in float64 and a fixed order: hard TNS, hard
// worst slack, smoothed TNS terms, and a shifted sum of exponentials for smoothed WNS.
__global__ __launch_bounds__(kBlock) void k_ep_partials(EpArgs a) {
  __shared__ double sh[kBlock];
  const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
  const bool act = i < a.E;
  double tns = 0.0, wmin = __builtin_huge_val(), tnsg = 0.0, v = -__builtin_huge_val();
  if (act) {
    const EpVals ev = endpoint_values(a, i);
    tns = fmin(0.0, (double)ev.worst);
    wmin = ev.worst;
    const double s = ev.sg, g = a.gamma;
    // -LSE_g(0, -s) = -(max(0,-s) + g*log1p(exp(-|s|/g)))
    tnsg = -(fmax(0.0, -s) + g * log1p(exp(-fabs(s) / g)));
    v = -s;
  }
  tns = block_reduce<kBlock>(tns, sh, false);
  wmin = -block_reduce<kBlock>(-wmin, sh, true);
  tnsg = block_reduce<kBlock>(tnsg, sh, false);
  const double mb = block_reduce<kBlock>(v, sh, true);
  const double ex = act ? exp((v - mb) / (double)a.gamma) : 0.0;
  const double sb = block_reduce<kBlock>(ex, sh, false);
  if (threadIdx.x == 0) {
    double* p = a.part + 5 * (size_t)blockIdx.x;
    p[0] = tns;
    p[1] = wmin;
    p[2] = tnsg;
    p[3] = mb;
    p[4] = sb;
  }
}

__global__ __launch_bounds__(kBlock) void k_ep_finalize(EpArgs a) {
  __shared__ double sh[kBlock];
  double tns = 0.0, wmin = __builtin_huge_val(), tnsg = 0.0, mx = -__builtin_huge_val();
  for (int b = threadIdx.x; b < a.n_blocks; b += kBlock) {
    const double* p = a.part + 5 * (size_t)b;
    tns += p[0];
    wmin = fmin(wmin, p[1]);
    tnsg += p[2];
    mx = fmax(mx, p[3]);
  }
  tns = block_reduce<kBlock>(tns, sh, false);
  wmin = -block_reduce<kBlock>(-wmin, sh, true);
  tnsg = block_reduce<kBlock>(tnsg, sh, false);
  const double M = fmax(0.0, block_reduce<kBlock>(mx, sh, true));   // {0} joins the WNS_g set
  double tot = 0.0;
  for (int b = threadIdx.x; b < a.n_blocks; b += kBlock) {
    const double* p = a.part + 5 * (size_t)b;
    if (p[4] > 0.0) tot += p[4] * exp((p[3] - M) / (double)a.gamma);
  }
  tot = block_reduce<kBlock>(tot, sh, false);
  if (threadIdx.x == 0) {
    tot += exp(-M / (double)a.gamma);
    const double lse_all = M + (double)a.gamma * log(tot);
    const double nan = __builtin_nan("");
    a.fin[0] = fmin(0.0, wmin);
    a.fin[1] = tns;
    a.fin[2] = a.smooth ? -lse_all : nan;
    a.fin[3] = a.smooth ? tnsg : nan;
    a.fin[4] = lse_all;
    if (a.scalars) {
      for (int q = 0; q < 4; ++q) a.scalars[q] = a.fin[q];
    }
  }
}

// Seeds of the backward sweep at the endpoints: constrained required times, and the
// adjoint of the smoothed objective with respect to each endpoint's smoothed arrival.
__global__ __launch_bounds__(kBlock) void k_ep_seed(EpArgs a) {
  const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (i >= a.E) return;
  const int e = a.ep_pin[i];
  a.ratp[e] = make_float4(a.hold, a.hold, a.rat_late, a.rat_late);
  float g0 = 0.f, g1 = 0.f;
  if (a.adjp) {
    const EpVals ev = endpoint_values(a, i);
    float coef;
    if (a.wns_mode) {
      coef = (float)exp((-(double)ev.sg - a.fin[4]) / (double)a.gamma);   // d WNS_g / d s_e
    } else {
      coef = 1.0f / (1.0f + expf(ev.sg * a.inv_gamma));                    // d TNS_g / d s_e
    }
    // d s_e / d atg(e, t) = -w_t; the objective's adjoint scales by `scale`.
    const float sc = a.scale_dev ? a.scale * (float)a.scale_dev[0] : a.scale;
    g0 = -sc * coef * ev.w0;
    g1 = -sc * coef * ev.w1;
    a.adjp[e] = make_float4(g0, g1, 0.f, 0.f);
  }
}

// ---------------------------------------------------------------------------- outputs
struct ExpandArgs {
  const int* net_off;
  const int* io_perm;
  const int* sched;
  GroupRange range;
  const float4* rec;
  const float2* wire;
  float4* at;
  float4* slew;
  float2* atg;
};

// Per-pin arrival, slew and smoothed arrival from the net records (forward outputs).
__global__ __launch_bounds__(kBlock) void k_expand(ExpandArgs a) {
  const int wave = (int)((blockIdx.x * kBlock + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  GroupSlot gs;
  if (!group_slot(a.range, wave, lane, gs) || !gs.active) return;
  const int n = a.sched[gs.entry];
  const int p0 = a.net_off[n], p1 = a.net_off[n + 1];
  const float4 at = a.rec[3 * (size_t)n], sl = a.rec[3 * (size_t)n + 1], ag = a.rec[3 * (size_t)n + 2];
  for (int p = p0 + gs.gl; p < p1; p += gs.G) {
    const float2 w = a.wire[p];
    const int q = a.io_perm ? a.io_perm[p] : p;
    if (a.at) a.at[q] = make_float4(at.x + w.x, at.y + w.x, at.z + w.x, at.w + w.x);
    if (a.slew)
      a.slew[q] = make_float4(sink_slew(sl.x, w.y), sink_slew(sl.y, w.y), sink_slew(sl.z, w.y), sink_slew(sl.w, w.y));
    if (a.atg) a.atg[q] = make_float2(ag.x + w.x, ag.y + w.x);
  }
}

// ---------------------------------------------------------------------------- backward level
struct BwdArgs {
  const int* net_off;
  const float* pin_cap;
  const int* cell_type;
  const int* type_arc0;
  const int8_t* unate;
  const int* cin_off;
  const int* cin_src;
  const int* cin_pin;
  const int* sched;
  const GroupRange* lvl;
  const int* io_perm;
  const float* x;
  const float* y;
  const float4* grid;
  const float4* coef;
  LutKeys keys;
  const float4* rec;
  const float2* wire;
  const float* load;
  float4* ratp;
  float4* adjp;
  float4* at_out;
  float4* slew_out;
  float4* rat_out;
  float4* slack_out;
  float* dx;
  float* dy;
  int N0;
  float r, c, inv_gamma;
  int grad;
};

// One level of backward propagation (Sec. 2.1 stage 4, Sec. 3.1.2) fused with the adjoint
// of the smoothed objective (Sec. 3.2).  Per net, one lane group:
//  1. net step over the sinks: per-pin outputs, RAT(driver) = min/max over sinks of
//     RAT(sink) - wire delay, sums of the sinks' adjoints into the driver;
//  2. cell step on lanes 0..3 (one condition each): every input's required time, the
//     softmax split of the driver's adjoint over the arcs (the LSE gradient), the slew
//     adjoint through the table partials and the arg-max slew arc, and the load adjoint;
//  3. Elmore adjoint: each sink's wire-length adjoint and d/dx, d/dy of every pin.
__global__ __launch_bounds__(kBlock) void k_bwd_level(BwdArgs a, int level) {
  const int wave = (int)((blockIdx.x * kBlock + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const GroupRange rg = a.lvl[level];
  GroupSlot gs;
  if (!group_slot(rg, wave, lane, gs)) return;
  const int G = gs.G, gl = gs.gl;
  const int n = gs.active ? a.sched[gs.entry] : 0;
  int p0 = 0, p1 = 0;
  float xd = 0.f, yd = 0.f;
  float4 at_d = make_float4(0.f, 0.f, 0.f, 0.f), sl_d = at_d;
  if (gs.active) {
    p0 = a.net_off[n];
    p1 = a.net_off[n + 1];
    at_d = a.rec[3 * (size_t)n];
    sl_d = a.rec[3 * (size_t)n + 1];
    if (a.grad) {
      const int q = a.io_perm ? a.io_perm[p0] : p0;
      xd = a.x[q];
      yd = a.y[q];
    }
  }
  const float k1e3r = 1e-3f * a.r;

  // 1. Net step.
  float rq0 = -kInf, rq1 = -kInf, rq2 = kInf, rq3 = kInf;
  float ab0 = 0.f, ab1 = 0.f, sb0 = 0.f, sb1 = 0.f;
  float sxr = 0.f, sxn = 0.f, syr = 0.f, syn = 0.f;
  for (int p = p0 + 1 + gl; p < p1; p += G) {
    const float4 rt = a.ratp[p];
    const float2 w = a.wire[p];
    const float4 ats = make_float4(at_d.x + w.x, at_d.y + w.x, at_d.z + w.x, at_d.w + w.x);
    const float4 sls = make_float4(sink_slew(sl_d.x, w.y), sink_slew(sl_d.y, w.y), sink_slew(sl_d.z, w.y),
                                   sink_slew(sl_d.w, w.y));
    const int q = a.io_perm ? a.io_perm[p] : p;
    if (a.at_out) a.at_out[q] = ats;
    if (a.slew_out) a.slew_out[q] = sls;
    if (a.rat_out) a.rat_out[q] = rt;
    if (a.slack_out) a.slack_out[q] = make_float4(ats.x - rt.x, ats.y - rt.y, rt.z - ats.z, rt.w - ats.w);
    rq0 = fmaxf(rq0, rt.x - w.x);
    rq1 = fmaxf(rq1, rt.y - w.x);
    rq2 = fminf(rq2, rt.z - w.x);
    rq3 = fminf(rq3, rt.w - w.x);
    if (a.grad) {
      const float4 aj = a.adjp[p];
      const float q0 = sls.z > 0.f ? aj.z / sls.z : 0.f;   // s_bar(s,t) / slew(s,late,t)
      const float q1 = sls.w > 0.f ? aj.w / sls.w : 0.f;
      ab0 += aj.x;
      ab1 += aj.y;
      sb0 += q0 * sl_d.z;
      sb1 += q1 * sl_d.w;
      const float dbar = aj.x + aj.y;                      // adjoint of the wire delay
      const float ibar = (q0 + q1) * w.y;                  // adjoint of the impulse
      const float xs = a.x[q], ys = a.y[q];
      const float len = fabsf(xs - xd) + fabsf(ys - yd);
      // d Delay / d len = d Impulse / d len = 1e-3 r (Cpin + c len) for a star sink.
      const float rest = (dbar + ibar) * (k1e3r * fmaf(a.c, len, a.pin_cap[p]));
      const float gx = sgnf(xs - xd), gy = sgnf(ys - yd);
      sxr += gx * rest;
      sxn += gx;
      syr += gy * rest;
      syn += gy;
    }
  }
  rq0 = grp_max(rq0, G);
  rq1 = grp_max(rq1, G);
  rq2 = grp_min(rq2, G);
  rq3 = grp_min(rq3, G);
  if (a.grad) {
    ab0 = grp_sum(ab0, G);
    ab1 = grp_sum(ab1, G);
    sb0 = grp_sum(sb0, G);
    sb1 = grp_sum(sb1, G);
    sxr = grp_sum(sxr, G);
    sxn = grp_sum(sxn, G);
    syr = grp_sum(syr, G);
    syn = grp_sum(syn, G);
  }

  // 2. Cell step.
  float lbar = 0.f;
  if (gs.active && n >= a.N0 && gl < 4) {
    const int k = gl, m = k >> 1, t = k & 1;
    const float rat_o = k == 0 ? rq0 : (k == 1 ? rq1 : (k == 2 ? rq2 : rq3));
    const int cell = n - a.N0;
    const float load = a.load[n];
    const int arc0 = a.type_arc0[a.cell_type[cell]];
    const int j0 = a.cin_off[cell], nin = a.cin_off[cell + 1] - j0;
    float xg[STA_MAX_FANIN], ddx[STA_MAX_FANIN], ddy[STA_MAX_FANIN], dsx[STA_MAX_FANIN], dsy[STA_MAX_FANIN];
    int pin[STA_MAX_FANIN], tpv[STA_MAX_FANIN];
    float xmax = -kInf, smax = -kInf;
    int jstar = 0;
#pragma unroll
    for (int jj = 0; jj < STA_MAX_FANIN; ++jj) {
      if (jj < nin) {
        const int j = j0 + jj;
        const int arc = arc0 + jj;
        const int tp = a.unate[arc] > 0 ? t : 1 - t;
        const int kp = 2 * m + tp;
        const float* src = reinterpret_cast<const float*>(a.rec + 3 * (size_t)a.cin_src[j]);
        const int pj = a.cin_pin[j];
        const float2 w = a.wire[pj];
        const float sl_in = sink_slew(src[4 + kp], w.y);
        const LutVal v = lut_eval<true>(a.grid, a.coef, a.keys, arc, t, sl_in, load);
        // RAT(input, k') = RAT(output, k) - arc delay.
        reinterpret_cast<float*>(a.ratp + pj)[kp] = rat_o - v.d;
        pin[jj] = pj;
        tpv[jj] = tp;
        xg[jj] = (src[8 + tp] + w.x) + v.d;
        ddx[jj] = v.ddx;
        ddy[jj] = v.ddy;
        dsx[jj] = v.dsx;
        dsy[jj] = v.dsy;
        xmax = fmaxf(xmax, xg[jj]);
        if (v.s > smax) {      // first maximum: ties go to the lowest arc
          smax = v.s;
          jstar = jj;
        }
      }
    }
    if (a.grad && m == 1) {
      const float abar = t ? ab1 : ab0;
      const float sbar = t ? sb1 : sb0;
      float ez[STA_MAX_FANIN];
      float z = 0.f;
#pragma unroll
      for (int jj = 0; jj < STA_MAX_FANIN; ++jj) {
        if (jj < nin) {
          ez[jj] = expf((xg[jj] - xmax) * a.inv_gamma);
          z += ez[jj];
        }
      }
      const float inv_z = 1.0f / z;
#pragma unroll
      for (int jj = 0; jj < STA_MAX_FANIN; ++jj) {
        if (jj < nin) {
          const float dbar = ez[jj] * inv_z * abar;       // softmax weight times the adjoint
          const float s_j = jj == jstar ? sbar : 0.f;
          float* adj = reinterpret_cast<float*>(a.adjp + pin[jj]);
          adj[tpv[jj]] = dbar;
          adj[2 + tpv[jj]] = fmaf(dbar, ddx[jj], s_j * dsx[jj]);
          lbar = fmaf(dbar, ddy[jj], fmaf(s_j, dsy[jj], lbar));
        }
      }
    }
  }

  // 3. Elmore adjoint and outputs.
  if (a.grad) {
    const int base = lane & ~(G - 1);
    lbar = __shfl(lbar, base + 2) + __shfl(lbar, base + 3);
  }
  if (!gs.active) return;
  if (a.grad && (a.dx || a.dy)) {
    const float cl = a.c * lbar;
    for (int p = p0 + 1 + gl; p < p1; p += G) {
      const float4 aj = a.adjp[p];
      const float2 w = a.wire[p];
      const float slz = sink_slew(sl_d.z, w.y), slw = sink_slew(sl_d.w, w.y);
      const float q0 = slz > 0.f ? aj.z / slz : 0.f;
      const float q1 = slw > 0.f ? aj.w / slw : 0.f;
      const int q = a.io_perm ? a.io_perm[p] : p;
      const float xs = a.x[q], ys = a.y[q];
      const float len = fabsf(xs - xd) + fabsf(ys - yd);
      const float rest = ((aj.x + aj.y) + (q0 + q1) * w.y) * (k1e3r * fmaf(a.c, len, a.pin_cap[p]));
      const float lb = cl + rest;                          // adjoint of the wire length
      if (a.dx) a.dx[q] = sgnf(xs - xd) * lb;
      if (a.dy) a.dy[q] = sgnf(ys - yd) * lb;
    }
  }
  if (gl == 0) {
    const int q = a.io_perm ? a.io_perm[p0] : p0;
    if (a.at_out) a.at_out[q] = at_d;
    if (a.slew_out) a.slew_out[q] = sl_d;
    if (a.rat_out) a.rat_out[q] = make_float4(rq0, rq1, rq2, rq3);
    if (a.slack_out) a.slack_out[q] = make_float4(at_d.x - rq0, at_d.y - rq1, rq2 - at_d.z, rq3 - at_d.w);
    if (a.grad) {
      const float cl = a.c * lbar;
      if (a.dx) a.dx[q] = -(sxr + cl * sxn);
      if (a.dy) a.dy[q] = -(syr + cl * syn);
    }
  }
}

inline unsigned blocks_for_waves(int waves) { return (unsigned)((waves * 64 + kBlock - 1) / kBlock); }

// Event pair around one launch while profiling is on (sta_profile_enable).
struct LaunchTimer {
  sta_graph* g;
  hipStream_t s;
  int kind;
  hipEvent_t start = nullptr, stop = nullptr;
  LaunchTimer(sta_graph* g_, hipStream_t s_, int kind_) : g(g_), s(s_), kind(kind_) {
    if (!g->profiling) return;
    start = take();
    stop = take();
    if (start && stop) (void)hipEventRecord(start, s);
  }
  ~LaunchTimer() {
    if (!start || !stop) return;
    (void)hipEventRecord(stop, s);
    g->timed.push_back({kind, start, stop});
  }
  hipEvent_t take() {
    if (!g->event_pool.empty()) {
      hipEvent_t e = g->event_pool.back();
      g->event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
  }
};

sta_status check_ready(sta_graph* g) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  if (!g->levelized) return fail(STA_E_STATE, "graph is not levelized");
  if (!g->uploaded) {
    sta_status s = sta_graph_upload(g);
    if (s != STA_OK) return s;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != g->dev.device) return fail(STA_E_STATE, "graph lives on another device than the current one");
  return STA_OK;
}

}  // namespace
}  // namespace sta

using namespace sta;

extern "C" sta_status sta_forward(sta_graph* g, const float* x, const float* y, sta_fwd_out* out, uint32_t flags,
                                  float gamma_ps, sta_stream stream) {
  sta_status st = check_ready(g);
  if (st != STA_OK) return st;
  if (!out || !out->state) return fail(STA_E_INVALID, "forward state buffer is required");
  if (!x || !y) return fail(STA_E_INVALID, "x and y are required");
  const bool smooth = (flags & STA_SMOOTH) != 0;
  if (smooth && !(gamma_ps > 0.f && std::isfinite(gamma_ps))) return fail(STA_E_INVALID, "gamma must be positive");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const DeviceGraph& d = g->dev;
  char* sb = static_cast<char*>(out->state);
  float4* rec = reinterpret_cast<float4*>(sb + g->state.rec);
  float2* wire = reinterpret_cast<float2*>(sb + g->state.wire);
  float* load = reinterpret_cast<float*>(sb + g->state.load);
  const int* io = (flags & STA_CANONICAL_IO) ? nullptr : d.pin_perm;

  RcArgs ra{d.net_off, d.pin_cap, x, y, io, d.sched_all, g->all_range, wire, load, rec, g->N0,
            g->cons.r_per_um, g->cons.c_per_um, g->cons.pi_at, g->cons.pi_slew};
  {
    LaunchTimer t(g, s, STA_K_RC);
    k_rc<<<blocks_for_waves(g->all_range.wave_off[kNumClasses]), kBlock, 0, s>>>(ra);
  }

  FwdArgs fa{d.cell_type, d.type_arc0, d.unate, d.cin_off, d.cin_src, d.cin_pin, wire, load, rec,
             d.lut_grid, d.lut_coef, lut_keys(g), g->N0, gamma_ps, smooth ? 1.0f / gamma_ps : 0.f, smooth ? 1 : 0};
  for (int l = 1; l < g->L; ++l) {
    const int c0 = g->level_off[l] - g->N0, c1 = g->level_off[l + 1] - g->N0;
    const unsigned blocks = (unsigned)((4 * (c1 - c0) + kBlock - 1) / kBlock);
    LaunchTimer t(g, s, STA_K_FWD_LEVEL);
    k_fwd_level<<<blocks, kBlock, 0, s>>>(fa, c0, c1);
  }

  EpArgs ea{d.ep_pin, d.ep_net, rec, wire, reinterpret_cast<double*>(sb + g->state.part),
            reinterpret_cast<double*>(sb + g->state.fin), out->scalars, nullptr, nullptr, nullptr, g->E, g->n_ep_blocks,
            g->cons.t_clk - g->cons.setup, g->cons.hold, smooth ? gamma_ps : 1.0f, smooth ? 1.0f / gamma_ps : 1.0f,
            1.0f, smooth ? 1 : 0, 0};
  if (g->n_ep_blocks > 0) {
    LaunchTimer t(g, s, STA_K_EP_PARTIAL);
    k_ep_partials<<<g->n_ep_blocks, kBlock, 0, s>>>(ea);
  }
  {
    LaunchTimer t(g, s, STA_K_EP_FINAL);
    k_ep_finalize<<<1, kBlock, 0, s>>>(ea);
  }

  if (out->at || out->slew || out->atg) {
    ExpandArgs xa{d.net_off, io, d.sched_all, g->all_range, rec, wire, reinterpret_cast<float4*>(out->at),
                  reinterpret_cast<float4*>(out->slew), reinterpret_cast<float2*>(out->atg)};
    LaunchTimer t(g, s, STA_K_EXPAND);
    k_expand<<<blocks_for_waves(g->all_range.wave_off[kNumClasses]), kBlock, 0, s>>>(xa);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "forward launch");
  return STA_OK;
}

extern "C" sta_status sta_backward(sta_graph* g, const float* x, const float* y, const sta_fwd_out* fwd,
                                   sta_bwd_out* out, uint32_t flags, float gamma_ps, sta_stream stream) {
  sta_status st = check_ready(g);
  if (st != STA_OK) return st;
  if (!fwd || !fwd->state || !out || !out->workspace) return fail(STA_E_INVALID, "state and workspace are required");
  const bool grad = (flags & STA_GRAD) != 0;
  if (grad && (!x || !y)) return fail(STA_E_INVALID, "x and y are required for the gradient");
  if (grad && !(gamma_ps > 0.f && std::isfinite(gamma_ps))) return fail(STA_E_INVALID, "gamma must be positive");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const DeviceGraph& d = g->dev;
  char* sb = static_cast<char*>(fwd->state);
  char* wb = static_cast<char*>(out->workspace);
  float4* rec = reinterpret_cast<float4*>(sb + g->state.rec);
  float2* wire = reinterpret_cast<float2*>(sb + g->state.wire);
  float* load = reinterpret_cast<float*>(sb + g->state.load);
  float4* ratp = reinterpret_cast<float4*>(wb + g->work.ratp);
  float4* adjp = reinterpret_cast<float4*>(wb + g->work.adjp);
  const int* io = (flags & STA_CANONICAL_IO) ? nullptr : d.pin_perm;

  EpArgs ea{d.ep_pin, d.ep_net, rec, wire, reinterpret_cast<double*>(sb + g->state.part),
            reinterpret_cast<double*>(sb + g->state.fin), nullptr, ratp, grad ? adjp : nullptr, out->grad_scale_dev, g->E,
            g->n_ep_blocks, g->cons.t_clk - g->cons.setup, g->cons.hold, grad ? gamma_ps : 1.0f,
            grad ? 1.0f / gamma_ps : 1.0f, out->grad_scale, 1, (flags & STA_GRAD_WNS) ? 1 : 0};
  if (g->E > 0) {
    LaunchTimer t(g, s, STA_K_EP_SEED);
    k_ep_seed<<<g->n_ep_blocks, kBlock, 0, s>>>(ea);
  }

  BwdArgs ba{d.net_off, d.pin_cap, d.cell_type, d.type_arc0, d.unate, d.cin_off, d.cin_src, d.cin_pin, d.sched,
             d.lvl, io, x, y, d.lut_grid, d.lut_coef, lut_keys(g), rec, wire, load, ratp, adjp,
             reinterpret_cast<float4*>(out->at), reinterpret_cast<float4*>(out->slew),
             reinterpret_cast<float4*>(out->rat), reinterpret_cast<float4*>(out->slack), out->dx, out->dy, g->N0,
             g->cons.r_per_um, g->cons.c_per_um, grad ? 1.0f / gamma_ps : 0.f, grad ? 1 : 0};
  for (int l = g->L - 1; l >= 0; --l) {
    const int waves = g->lvl_ranges[l].wave_off[kNumClasses];
    if (waves > 0) {
      LaunchTimer t(g, s, STA_K_BWD_LEVEL);
      k_bwd_level<<<blocks_for_waves(waves), kBlock, 0, s>>>(ba, l);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "backward launch");
  return STA_OK;
}

extern "C" sta_status sta_profile_enable(sta_graph* g, int32_t on) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  for (auto& t : g->timed) {
    g->event_pool.push_back(t.start);
    g->event_pool.push_back(t.stop);
  }
  g->timed.clear();
  g->profiling = on != 0;
  return STA_OK;
}

extern "C" sta_status sta_profile_read(sta_graph* g, int64_t* launches, double* total_ms) {
  if (!g || !launches || !total_ms) return fail(STA_E_INVALID, "NULL argument");
  for (int k = 0; k < STA_K_COUNT; ++k) {
    launches[k] = 0;
    total_ms[k] = 0.0;
  }
  for (auto& t : g->timed) {
    hipError_t e = hipEventSynchronize(t.stop);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, t.start, t.stop);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    launches[t.kind] += 1;
    total_ms[t.kind] += ms;
  }
  return STA_OK;
}
