// HIP kernels of the levelized STA sweep for CDNA4 (gfx950, wave64), and the C ABI calls
// that launch them (sta_forward, sta_backward).
//
// Data layout (canonical order from sta_levelize): nets sorted by (level, pins), pins
// net-major with the driver first.  The forward sweep keeps one 64-byte record per net -
// per timing condition a 16-byte chunk {arrival time, slew, smoothed arrival (late
// conditions), 0} of the driver - and derives a sink's state on demand from its driver
// record plus the sink's {wire delay, impulse}.  A lane serving one condition of a cell
// input therefore gathers one aligned chunk, and the four condition lanes of an input
// share one 64-byte line.  A level writes one record per net; per-pin outputs are written
// by the backward sweep, which visits every pin anyway.
//
// Lane mapping (the pin-based scheme of Sec. 3.1, re-derived for 64-lane wavefronts).  A
// level holds a few thousand nets, so a level kernel occupies about one wave per SIMD and
// its time is the instruction chain of one lane: work is spread over lanes to keep that
// chain short.
//  * Cell step: 16 lanes per cell, one per (timing condition, arc) - the condition axis of
//    Alg. 1 times the arcs - so every lane does one table lookup; max/min, log-sum-exp,
//    softmax and arg max over a condition's arcs reduce over 4 lanes with DPP quad
//    permutes.
//  * Net step: a group of 16, 32 or 64 lanes per net (one sink per lane), or a whole
//    256-thread workgroup for nets over 64 sinks; reductions over a net's sinks are DPP
//    and xor butterflies inside the group, across waves through LDS in a fixed order
//    (no atomics, Sec. 3.1.1).
//  * The one-pass RC kernel and the forward output expansion use groups from 4 lanes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>

#include "sta_internal.h"

namespace sta {
namespace {

constexpr float kInf = __builtin_huge_valf();
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kCellLanes = 16;   // backward cell step: lanes per cell, 4 conditions x 4 arcs
constexpr int kArcLanes = 4;     // arcs handled at once per condition; wider cells loop
constexpr int kRecChunks = 4;    // float4 chunks per arrival record, one per condition

// Element i of an array through a 32-bit byte offset from its base.  The base is uniform,
// so loads and stores take the scalar-base form with one 32-bit offset register instead of
// a 64-bit address per lane.  The library rejects graphs with an array of 4 GiB or more.
template <class T>
__device__ __forceinline__ T* at32(T* base, uint32_t i) {
  using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return reinterpret_cast<T*>(reinterpret_cast<C*>(base) + (uint64_t)(i * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ T ld(const T* __restrict__ base, uint32_t i) {
  return *at32(base, i);
}

// Placement snapshots of one graph share its topology; snapshot blockIdx.y of a launch
// works on its own copy of the per-call buffers, `state` / `work` bytes (state and
// workspace) or `pins` / `scal` elements (per-pin arrays, scalars) after snapshot 0's.
struct Snap {
  size_t state, work, pins, scal;
};

// kSnap = false compiles the one-snapshot kernels, in which these offsets vanish.
template <bool kSnap = true, class T>
__device__ __forceinline__ T* snap_bytes(T* p, size_t stride) {
  using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  if (!kSnap) return p;
  return p ? reinterpret_cast<T*>(reinterpret_cast<C*>(p) + stride * blockIdx.y) : p;
}
template <bool kSnap = true, class T>
__device__ __forceinline__ T* snap_elems(T* p, size_t stride) {
  if (!kSnap) return p;
  return p ? p + stride * blockIdx.y : p;
}
// The same for an explicit snapshot index.
template <bool kSnap = true, class T>
__device__ __forceinline__ T* snap_bytes(T* p, size_t stride, int sn) {
  using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  if (!kSnap) return p;
  return p ? reinterpret_cast<T*>(reinterpret_cast<C*>(p) + stride * (size_t)sn) : p;
}
template <bool kSnap = true, class T>
__device__ __forceinline__ T* snap_elems(T* p, size_t stride, int sn) {
  if (!kSnap) return p;
  return p ? p + stride * (size_t)sn : p;
}

// Block and snapshot a workgroup of a level launch works on.  Workgroups go to the 8 XCDs
// round-robin in launch order.  When the snapshot count is a multiple of 8, workgroup b
// takes snapshot (b mod 8) + 8 * floor((b / 8) / X) and block (b / 8) mod X of the X blocks
// of one snapshot, a bijection under which every snapshot runs on one XCD: the records,
// wires and sink state that a level gathers at random of that snapshot then meet in one
// L2, and the scattered stores to a line are merged there.  Otherwise snapshot blockIdx.y
// takes block blockIdx.x (the x extent is padded to a multiple of 8, so that the copies of
// a block share an XCD and its topology lines).
struct SnapBlock {
  int x, s;
};
template <bool kSnap>
__device__ __forceinline__ SnapBlock snap_block() {
  if (!kSnap) return SnapBlock{(int)blockIdx.x, 0};
  const uint32_t X = gridDim.x, S = gridDim.y;
  if (S % 8u != 0u) return SnapBlock{(int)blockIdx.x, (int)blockIdx.y};
  const uint32_t b = blockIdx.y * X + blockIdx.x;
  const uint32_t r = b >> 3;
  return SnapBlock{(int)(r % X), (int)((b & 7u) + 8u * (r / X))};
}

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
__device__ __forceinline__ int lut_cell(const LutKeys& keys, float xv, float yv) {
  return find_cell(xv, keys.x) * (STA_LUT_N - 1) + find_cell(yv, keys.y);
}
__device__ __forceinline__ uint32_t lut_coef_at(int arc, int tr, int cell) {
  return ((uint32_t)(arc * 2 + tr) * kLutCells + (uint32_t)cell) * 2;
}
template <bool kPartials>
__device__ __forceinline__ LutVal lut_apply(const float4& g, const float4& cd, const float4& cs, float xv, float yv) {
  const float tx = (xv - g.x) * g.y;
  const float ty = (yv - g.z) * g.w;
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
template <bool kPartials>
__device__ __forceinline__ LutVal lut_eval(const float4* __restrict__ grid, const float4* __restrict__ coef,
                                           const LutKeys& keys, int arc, int tr, float xv, float yv) {
  const int cell = lut_cell(keys, xv, yv);
  const uint32_t ci = lut_coef_at(arc, tr, cell);
  return lut_apply<kPartials>(ld(grid, (uint32_t)cell), ld(coef, ci), ld(coef, ci + 1), xv, yv);
}

// Table memory read as constant (it is never written while a kernel runs), so that a load
// whose address is uniform over the wave can take the scalar path.
struct alignas(16) Raw4 { float x, y, z, w; };
typedef const __attribute__((address_space(4))) Raw4 ConstRaw4;
__device__ __forceinline__ float4 ld_const(const float4* base, uint32_t i) {
  ConstRaw4* p = (ConstRaw4*)(const __attribute__((address_space(4))) void*)base;
  return make_float4(p[i].x, p[i].y, p[i].z, p[i].w);
}

// The same lookup in the snapshot-lane kernels, whose wave usually serves one arc for 64
// snapshots that fall in one table cell: the first active lane's coefficients come through
// scalar loads for the whole wave, and only lanes that want another cell load their own
// through the vector cache (none, when every lane shares the cell).  The values, and so the
// results, are the same either way.
template <bool kPartials>
__device__ __forceinline__ LutVal lut_eval_si(const float4* __restrict__ grid, const float4* __restrict__ coef,
                                              const LutKeys& keys, int arc, int tr, float xv, float yv) {
  const int cell = lut_cell(keys, xv, yv);
  const uint32_t ci = lut_coef_at(arc, tr, cell);
  const uint32_t c0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)ci);
  const uint32_t k0 = (uint32_t)__builtin_amdgcn_readfirstlane(cell);
  float4 g = ld_const(grid, k0), cd = ld_const(coef, c0), cs = ld_const(coef, c0 + 1);
  if (ci != c0) {
    g = ld(grid, (uint32_t)cell);
    cd = ld(coef, ci);
    cs = ld(coef, ci + 1);
  }
  return lut_apply<kPartials>(g, cd, cs, xv, yv);
}

// Hardware approximations (about 1 ulp) of exp, log, square root and reciprocal: one
// instruction each instead of the correctly rounded library sequences, in the level kernels'
// per-lane arithmetic, whose times are compared with the oracle within 1e-4 relative.
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
__device__ __forceinline__ float flog(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Positions (in float4) of a sink's required times and adjoint in the backward workspace:
// the two are interleaved per sink.
__device__ __forceinline__ uint32_t rat_at(uint32_t p) { return 2u * p; }
__device__ __forceinline__ uint32_t adj_at(uint32_t p) { return 2u * p + 1u; }
__device__ __forceinline__ int rat_at(int p) { return 2 * p; }
__device__ __forceinline__ int adj_at(int p) { return 2 * p + 1; }

// Slew at a sink: the driver slew combined with the wire's impulse.
__device__ __forceinline__ float sink_slew(float drv_slew, float imp) {
  return fsqrt(fmaf(drv_slew, drv_slew, imp * imp));
}

// Merges log-sum-exp partials (m, s) <- (m, s) + (m2, s2), each meaning m + gamma*log(s)
// (Eq. 4 with the maximum as the shift).
__device__ __forceinline__ void lse_merge(float& m, float& s, float m2, float s2, float inv_gamma) {
  if (m2 > m) {
    s = fmaf(s, fexp((m - m2) * inv_gamma), s2);
    m = m2;
  } else if (s2 > 0.f) {
    s = fmaf(s2, fexp((m2 - m) * inv_gamma), s);
  }
}

__device__ __forceinline__ float sgnf(float v) { return (v > 0.f) ? 1.f : ((v < 0.f) ? -1.f : 0.f); }

// DPP lane permutes inside a row of 16 lanes: quad xor 1, quad xor 2, reverse within 8,
// reverse within 16.  Successive steps pair every value with every other exactly once, so
// sums, minima and maxima come out identical on all lanes of the row.
enum : int { kDppQuadX1 = 0xB1, kDppQuadX2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140 };

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

enum RedOp { kSum = 0, kMin = 1, kMax = 2 };

template <int OP>
__device__ __forceinline__ float red2(float a, float b) {
  return OP == kSum ? a + b : (OP == kMin ? fminf(a, b) : fmaxf(a, b));
}

// Reduction over the 4 lanes of a quad (the arcs of one condition).
template <int OP>
__device__ __forceinline__ float quad_reduce(float v) {
  v = red2<OP>(v, dpp<kDppQuadX1>(v));
  return red2<OP>(v, dpp<kDppQuadX2>(v));
}

// Largest value over a quad with its lane's arc index; ties go to the lowest index.
__device__ __forceinline__ void quad_argmax(float& v, int& j) {
  float v2 = dpp<kDppQuadX1>(v);
  int j2 = dpp_i<kDppQuadX1>(j);
  if (v2 > v || (v2 == v && j2 < j)) { v = v2; j = j2; }
  v2 = dpp<kDppQuadX2>(v);
  j2 = dpp_i<kDppQuadX2>(j);
  if (v2 > v || (v2 == v && j2 < j)) { v = v2; j = j2; }
}

// The arc lanes of one condition in a backward cell step: 4 (a quad), 2 (a pair) or 1.
template <int OP, int AL>
__device__ __forceinline__ float arc_reduce(float v) {
  if (AL >= 2) v = red2<OP>(v, dpp<kDppQuadX1>(v));
  return AL == 4 ? red2<OP>(v, dpp<kDppQuadX2>(v)) : v;
}
template <int AL>
__device__ __forceinline__ void arc_argmax(float& v, int& j) {
  if (AL == 4) {
    quad_argmax(v, j);
    return;
  }
  if (AL == 1) return;
  const float v2 = dpp<kDppQuadX1>(v);
  const int j2 = dpp_i<kDppQuadX1>(j);
  if (v2 > v || (v2 == v && j2 < j)) { v = v2; j = j2; }
}

// Reduction over an aligned group of G lanes (G = 4, 8, 16, 32 or 64) of a wave.
template <int OP, int G>
__device__ __forceinline__ float wave_group_reduce(float v) {
  v = red2<OP>(v, dpp<kDppQuadX1>(v));
  v = red2<OP>(v, dpp<kDppQuadX2>(v));
  if (G >= 8) v = red2<OP>(v, dpp<kDppHalfMirror>(v));
  if (G >= 16) v = red2<OP>(v, dpp<kDppMirror>(v));
  if (G >= 32) v = red2<OP>(v, __shfl_xor(v, 16));
  if (G >= 64) v = red2<OP>(v, __shfl_xor(v, 32));
  return v;
}

// Reduction over the lanes of a group of runtime size G = 4..64 (flat kernels).
__device__ __forceinline__ float wave_group_sum(float v, int G) {
  for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

// ---------------------------------------------------------------------------- lane groups
// Which net (schedule entry) a thread serves inside a GroupRange launch.  Blocks
// [0, n_heavy) take one heavy net each (all 256 threads); the remaining blocks hold waves
// of the wave classes.  All lanes of a wave agree on the class, all lanes of a group on
// the net, and all threads of a block on `block`.
struct GroupSlot {
  int G;        // lanes per net
  int gl;       // lane index inside the group
  int entry;    // schedule entry, valid if active
  bool active;
  bool block;   // a whole workgroup serves one net
};

__device__ __forceinline__ bool group_slot(const GroupRange& r, GroupSlot& s) {
  const int nh = r.cls_off[kNumClasses + 1] - r.cls_off[kNumClasses];
  if ((int)blockIdx.x < nh) {
    s.block = true;
    s.G = kBlock;
    s.gl = threadIdx.x;
    s.entry = r.cls_off[kNumClasses] + (int)blockIdx.x;
    s.active = true;
    return true;
  }
  s.block = false;
  const int wave = ((int)blockIdx.x - nh) * kWavesPerBlock + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (wave >= r.wave_off[kNumClasses]) return false;
  int c = 0;
  while (c < kNumClasses - 1 && wave >= r.wave_off[c + 1]) ++c;
  const int lg = r.g0 + c;           // log2 of the group size
  s.G = 1 << lg;
  s.gl = lane & (s.G - 1);
  s.entry = r.cls_off[c] + (wave - r.wave_off[c]) * (64 >> lg) + (lane >> lg);
  s.active = s.entry < r.cls_off[c + 1];
  return true;
}

// The same mapping for a level kernel, whose smallest group is 2^G0 >= 4 lanes, so that at
// most five wave classes (4/8/16/32/64 lanes) exist.  The level's ranges arrive as scalars -
// heavy nets [h0, h0 + nh), class c entries [e_c, e_{c+1}) on waves [w_c, w_{c+1}) with
// w_0 = 0 - and the class is found without indexing an array.
template <int G0>
__device__ __forceinline__ bool level_slot(int bx, int nh, int h0, int e0, int e1, int e2, int e3, int e4, int e5,
                                           int w1, int w2, int w3, int w4, int w5, GroupSlot& s) {
  if (bx < nh) {
    s.block = true;
    s.G = kBlock;
    s.gl = threadIdx.x;
    s.entry = h0 + bx;
    s.active = true;
    return true;
  }
  s.block = false;
  const int wave = (bx - nh) * kWavesPerBlock + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // Groups of 16 lanes and more have three classes at most (e4 = e3, w4 = w3), and then e4,
  // e5, w4 and w5, which are not preloaded, are not read; 8-lane groups have four.
  if (wave >= (G0 >= 4 ? w3 : (G0 == 3 ? w4 : w5))) return false;
  const int c = (wave >= w1) + (wave >= w2) + (G0 <= 3 ? (wave >= w3) : 0) + (G0 <= 2 ? (wave >= w4) : 0);
  const int eb = c == 0 ? e0 : (c == 1 ? e1 : (c == 2 ? e2 : (c == 3 ? e3 : e4)));
  const int ee = c == 0 ? e1 : (c == 1 ? e2 : (c == 2 ? e3 : (c == 3 ? e4 : e5)));
  const int wb = c == 0 ? 0 : (c == 1 ? w1 : (c == 2 ? w2 : (c == 3 ? w3 : w4)));
  const int lg = G0 + c;
  s.G = 1 << lg;
  s.gl = lane & (s.G - 1);
  s.entry = eb + (wave - wb) * (64 >> lg) + (lane >> lg);
  s.active = s.entry < ee;
  return true;
}

inline unsigned range_grid(const GroupRange& r) {
  const int nh = r.cls_off[kNumClasses + 1] - r.cls_off[kNumClasses];
  return (unsigned)(nh + (r.wave_off[kNumClasses] + kWavesPerBlock - 1) / kWavesPerBlock);
}

// Sum over the 256 threads of a workgroup (fixed order: wave butterflies, then waves in
// order through LDS).  `sh` holds kWavesPerBlock floats.
__device__ __forceinline__ float block_sum(float v, float* sh) {
  v = wave_group_reduce<kSum, 64>(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = sh[0];
  for (int q = 1; q < kWavesPerBlock; ++q) r += sh[q];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------- RC (Alg. 1)
struct RcArgs {
  const int* __restrict__ net_off;
  const float* __restrict__ pin_cap;
  const float* __restrict__ x;
  const float* __restrict__ y;
  const int* __restrict__ io_perm;        // canonical -> caller index, or NULL
  const int* __restrict__ sched;
  GroupRange range;
  float2* __restrict__ wire;
  float* __restrict__ load;
  float4* __restrict__ rec;
  int N0, N;
  float r, c, pi_at, pi_slew;
  Snap snap;
  const int* __restrict__ parent;       // RC trees: canonical parent pin, -1 at drivers
  const int* __restrict__ tree_order;   // RC trees: each net's pins in breadth-first order
  float4* __restrict__ tree;            // RC trees: pass values, two float4 per pin
  const int4* __restrict__ tree_node;   // RC trees: {depth, first child position, children, 0}
  const int* __restrict__ chunk_net;    // RC trees: net ranges of the LDS chunks
  const int* __restrict__ chunk_depth;  // RC trees: deepest depth per chunk (-1: skipped)
  const int* __restrict__ net_list;     // RC trees: the nets of the fallback kernel
  int n_list;
  int n_chunks;
  const int* __restrict__ sink_base;    // checkpointing (stars): first wire slot of each net's
                                        // sinks; NULL: a sink's slot is its pin
};

// One sink p of a star net whose driver sits at (xd, yd): wire delay and impulse (Eq. 2-3)
// to wire[slot] (slot = p without checkpointing); returns what the sink adds to the root load
// (Eq. 1): its pin cap plus the whole wire, half of which sits at each end.
__device__ __forceinline__ float rc_sink(const RcArgs& a, const float* __restrict__ xs, const float* __restrict__ ys,
                                         float2* __restrict__ wire, int p, int slot, float xd, float yd) {
  const int q = a.io_perm ? a.io_perm[p] : p;
  const float cp = a.pin_cap[p];
  const float len = fabsf(xs[q] - xd) + fabsf(ys[q] - yd);
  const float res = a.r * len;                 // Res(fa(u) -> u)
  const float cw = a.c * len;                  // wire capacitance, half at each end
  const float cap = fmaf(0.5f, cw, cp);        // Cap(u) of the sink node
  const float load = cap;                      // Eq. 1 at a leaf
  const float dly = 1e-3f * res * load;        // Eq. 2 (ohm * fF = 1e-3 ps)
  const float arg = 2.0f * (1e-3f * res * cap) * dly - dly * dly;   // Eq. 3
  const float imp = arg > 0.f ? sqrtf(arg) : 0.f;
  wire[slot] = make_float2(dly, imp);
  return cp + cw;
}

// Root of net n (driver pin p0) once its sinks' contributions are summed: the root load,
// a zero wire at the driver (wires by pin only), and the arrival record of a primary-input
// net.
__device__ __forceinline__ void rc_root(const RcArgs& a, float2* __restrict__ wire, float* __restrict__ loads,
                                        float4* __restrict__ rec, int n, int p0, float sum, bool is_total = false) {
  loads[n] = is_total ? sum : a.pin_cap[p0] + sum;   // Eq. 1 at the root
  if (!a.sink_base) wire[p0] = make_float2(0.f, 0.f);
  if (n < a.N0) {
    float4* r = rec + kRecChunks * (size_t)n;
    r[0] = make_float4(a.pi_at, a.pi_slew, 0.f, 0.f);
    r[1] = make_float4(a.pi_at, a.pi_slew, 0.f, 0.f);
    r[2] = make_float4(a.pi_at, a.pi_slew, a.pi_at, 0.f);
    r[3] = make_float4(a.pi_at, a.pi_slew, a.pi_at, 0.f);
  }
}

// RC net delay of every net (Sec. 3.1.1, Eq. 1-3, star nets): per sink the wire delay and
// impulse, per net the root load by a group reduction.  Level-0 (primary input) records
// are initialised here too.
__global__ __launch_bounds__(kBlock) void k_rc(RcArgs a) {
  __shared__ float sh[kWavesPerBlock];
  const float* __restrict__ xs = snap_elems(a.x, a.snap.pins);
  const float* __restrict__ ys = snap_elems(a.y, a.snap.pins);
  float2* __restrict__ wire = snap_bytes(a.wire, a.snap.state);
  float* __restrict__ loads = snap_bytes(a.load, a.snap.state);
  float4* __restrict__ rec = snap_bytes(a.rec, a.snap.state);
  GroupSlot gs;
  if (!group_slot(a.range, gs)) return;
  const int n = gs.active ? a.sched[gs.entry] : 0;
  int p0 = 0, p1 = 0;
  float xd = 0.f, yd = 0.f;
  if (gs.active) {
    p0 = a.net_off[n];
    p1 = a.net_off[n + 1];
    const int q = a.io_perm ? a.io_perm[p0] : p0;
    xd = xs[q];
    yd = ys[q];
  }
  // Wire slots: a net's sinks take consecutive slots from sink_base[n] under checkpointing.
  const int sk0 = (gs.active && a.sink_base) ? a.sink_base[n] - (p0 + 1) : 0;
  float sum = 0.f;
  for (int p = p0 + 1 + gs.gl; p < p1; p += gs.G) sum += rc_sink(a, xs, ys, wire, p, sk0 + p, xd, yd);
  sum = gs.block ? block_sum(sum, sh) : wave_group_sum(sum, gs.G);
  if (gs.active && gs.gl == 0) rc_root(a, wire, loads, rec, n, p0, sum);
}

// The same in the CTE scheme (Alg. 2): a workgroup takes 256 consecutive nets, one per
// thread, and pools their sinks into one task list.  A work-efficient exclusive scan
// (up-sweep, then down-sweep) over the per-net sink counts numbers the tasks; threads take
// tasks with a stride of 256 and find a task's net by binary search for the last net whose
// first task is not above it.  The model here is the same for the four timing conditions,
// so a task is one sink rather than one (sink, condition) pair.  Root loads are summed in
// task order from LDS, in chunks of kCteChunk tasks, by each net's own thread.
constexpr int kCteChunk = 1024;

// Work-efficient exclusive scan (Blelloch: up-sweep, then down-sweep) of the values of the
// first kN threads of a workgroup (a power of two up to its size) into pre[0, kN); returns
// the total.  Every thread of the workgroup calls it; it first waits until every thread is
// done with the previous scan's pre[] and total.
template <int kN = kBlock>
__device__ __forceinline__ int cte_scan(int work, int* pre, int* total_sh) {
  const int t = threadIdx.x;
  __syncthreads();
  if (t < kN) pre[t] = work;
  for (int d = 1; d < kN; d <<= 1) {           // pre[t] becomes the sum of its subtree
    __syncthreads();
    if (t < kN && ((t + 1) & (2 * d - 1)) == 0) pre[t] += pre[t - d];
  }
  __syncthreads();
  if (t == kN - 1) {
    *total_sh = pre[t];
    pre[t] = 0;
  }
  for (int d = kN / 2; d >= 1; d >>= 1) {      // exclusive prefix sums
    __syncthreads();
    if (t < kN && ((t + 1) & (2 * d - 1)) == 0) {
      const int l = pre[t - d];
      pre[t - d] = pre[t];
      pre[t] += l;
    }
  }
  __syncthreads();
  return *total_sh;
}

// Owner of a task among kN items: the last one whose first task is not above it
// (upper_bound - 1 on the exclusive scan).
template <int kN = kBlock>
__device__ __forceinline__ int cte_owner(const int* pre, int task) {
  int lo = 0, hi = kN;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= task) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kBlock) void k_rc_cte(RcArgs a) {
  __shared__ int pre[kBlock];
  __shared__ int first[kBlock];
  __shared__ float dx_[kBlock], dy_[kBlock];
  __shared__ float part[kCteChunk];
  __shared__ int total_sh;
  const float* __restrict__ xs = snap_elems(a.x, a.snap.pins);
  const float* __restrict__ ys = snap_elems(a.y, a.snap.pins);
  float2* __restrict__ wire = snap_bytes(a.wire, a.snap.state);
  float* __restrict__ loads = snap_bytes(a.load, a.snap.state);
  float4* __restrict__ rec = snap_bytes(a.rec, a.snap.state);
  const int t = threadIdx.x;
  const int n = (int)blockIdx.x * kBlock + t;
  const bool own = n < a.N;
  int p0 = 0, work = 0;
  float xd = 0.f, yd = 0.f;
  if (own) {
    p0 = a.net_off[n];
    work = a.net_off[n + 1] - p0 - 1;
    const int q = a.io_perm ? a.io_perm[p0] : p0;
    xd = xs[q];
    yd = ys[q];
  }
  first[t] = p0 + 1;
  dx_[t] = xd;
  dy_[t] = yd;
  const int total = cte_scan(work, pre, &total_sh);
  const int my0 = pre[t], my1 = t + 1 < kBlock ? pre[t + 1] : total;
  float sum = 0.f;
  for (int c0 = 0; c0 < total; c0 += kCteChunk) {
    const int c1 = min(total, c0 + kCteChunk);
    for (int task = c0 + t; task < c1; task += kBlock) {
      const int lo = cte_owner(pre, task);
      const int p = first[lo] + (task - pre[lo]);
      part[task - c0] = rc_sink(a, xs, ys, wire, p, p, dx_[lo], dy_[lo]);   // wires by pin
    }
    __syncthreads();
    for (int i = max(my0, c0); i < min(my1, c1); ++i) sum += part[i - c0];
    __syncthreads();
  }
  if (own) rc_root(a, wire, loads, rec, n, p0, sum);
}

// The same with one thread per net walking its sinks in order (the net-per-thread mapping
// of earlier GPU timers, kept as the baseline of the lane-group and CTE schemes).
__global__ __launch_bounds__(kBlock) void k_rc_thread(RcArgs a) {
  const float* __restrict__ xs = snap_elems(a.x, a.snap.pins);
  const float* __restrict__ ys = snap_elems(a.y, a.snap.pins);
  float2* __restrict__ wire = snap_bytes(a.wire, a.snap.state);
  float* __restrict__ loads = snap_bytes(a.load, a.snap.state);
  float4* __restrict__ rec = snap_bytes(a.rec, a.snap.state);
  const int n = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (n >= a.N) return;
  const int p0 = a.net_off[n], p1 = a.net_off[n + 1];
  const int q = a.io_perm ? a.io_perm[p0] : p0;
  const float xd = xs[q], yd = ys[q];
  float sum = 0.f;
  for (int p = p0 + 1; p < p1; ++p) sum += rc_sink(a, xs, ys, wire, p, p, xd, yd);   // wires by pin
  rc_root(a, wire, loads, rec, n, p0, sum);
}

// RC net delay on RC trees, one thread per net walking its pins in breadth-first order
// (parents before children), for nets too big for the LDS chunks of k_rc_tree_chunk.  Segment u runs from parent pin fa(u) to pin u; Cap(u) holds the
// pin and half of every segment touching it.  Load sums the children's Loads bottom-up
// (Eq. 1), Delay adds the parent's delay top-down (Eq. 2 on a tree), and the impulse takes
// the second moment: LDelay(u) = Cap(u) Delay(u) + the children's LDelay bottom-up,
// Beta(u) = Beta(fa(u)) + Res(fa(u) -> u) LDelay(u) top-down, Impulse = sqrt(2 Beta - Delay^2)
// (Eq. 3 on a star).  The pass values stay in `tree` for the adjoint (k_rc_tree_adjoint).
__global__ __launch_bounds__(kBlock) void k_rc_tree(RcArgs a) {
  const float* __restrict__ xs = snap_elems(a.x, a.snap.pins);
  const float* __restrict__ ys = snap_elems(a.y, a.snap.pins);
  float2* __restrict__ wire = snap_bytes(a.wire, a.snap.state);
  float* __restrict__ loads = snap_bytes(a.load, a.snap.state);
  float4* __restrict__ rec = snap_bytes(a.rec, a.snap.state);
  float4* __restrict__ T = snap_bytes(a.tree, a.snap.state);
  const int k = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (k >= a.n_list) return;
  const int n = a.net_list[k];
  const int b = a.net_off[n], e = a.net_off[n + 1];
  const float kr = 1e-3f * a.r, hc = 0.5f * a.c;   // ohm * fF = 1e-3 ps
  // Lengths and own caps ({length, Cap, Load, Delay}, {LDelay, Beta, Impulse, 0} per pin).
  for (int q = b; q < e; ++q) {
    float len = 0.f;
    if (q > b) {
      const int f = a.parent[q];
      const int qo = a.io_perm ? a.io_perm[q] : q, fo = a.io_perm ? a.io_perm[f] : f;
      len = fabsf(xs[qo] - xs[fo]) + fabsf(ys[qo] - ys[fo]);
    }
    T[2 * (size_t)q] = make_float4(len, fmaf(hc, len, a.pin_cap[q]), 0.f, 0.f);
  }
  for (int q = b + 1; q < e; ++q) T[2 * (size_t)a.parent[q]].y += hc * T[2 * (size_t)q].x;   // segments out of a pin
  for (int q = b; q < e; ++q) T[2 * (size_t)q].z = T[2 * (size_t)q].y;
  for (int j = e - 1; j > b; --j) {                 // Load, children first
    const int u = a.tree_order[j];
    T[2 * (size_t)a.parent[u]].z += T[2 * (size_t)u].z;
  }
  for (int j = b + 1; j < e; ++j) {                 // Delay, parents first
    const int u = a.tree_order[j];
    const float4 t = T[2 * (size_t)u];
    T[2 * (size_t)u].w = T[2 * (size_t)a.parent[u]].w + kr * t.x * t.z;
  }
  for (int q = b; q < e; ++q) T[2 * (size_t)q + 1] = make_float4(T[2 * (size_t)q].y * T[2 * (size_t)q].w, 0.f, 0.f, 0.f);
  for (int j = e - 1; j > b; --j) {                 // LDelay, children first
    const int u = a.tree_order[j];
    T[2 * (size_t)a.parent[u] + 1].x += T[2 * (size_t)u + 1].x;
  }
  for (int j = b + 1; j < e; ++j) {                 // Beta and the impulse, parents first
    const int u = a.tree_order[j];
    const float4 t = T[2 * (size_t)u];
    const float beta = T[2 * (size_t)a.parent[u] + 1].y + kr * t.x * T[2 * (size_t)u + 1].x;
    const float arg = 2.0f * beta - t.w * t.w;
    const float imp = arg > 0.f ? sqrtf(arg) : 0.f;
    T[2 * (size_t)u + 1].y = beta;
    T[2 * (size_t)u + 1].z = imp;
    wire[u] = make_float2(t.w, imp);
  }
  rc_root(a, wire, loads, rec, n, b, T[2 * (size_t)b].z, true);
}

// Adjoint of the tree passes for one net per thread (nets too big for k_rc_tree_adjoint_chunk): from the backward sweep's adjoints of each
// sink's Delay and Impulse and of the root Load (tree_adj), back through the four passes in
// reverse (Beta and Delay children-first, LDelay and Load parents-first), to the segment
// lengths, Cap and Res, and through |dx| + |dy| to the pins' coordinates.
struct TreeAdjArgs {
  const int* __restrict__ net_off;
  const int* __restrict__ parent;
  const int* __restrict__ tree_order;
  const int* __restrict__ io_perm;
  const float* __restrict__ x;
  const float* __restrict__ y;
  const float4* __restrict__ tree;      // forward pass values (state)
  const float2* __restrict__ tree_adj;  // per sink {d/dDelay, d/dImpulse}, at the driver {d/dLoad, 0}
  float4* __restrict__ bar;             // scratch, two float4 per pin
  float* __restrict__ dx;
  float* __restrict__ dy;
  int N;
  float r, c;
  Snap snap;
  const int4* __restrict__ tree_node;
  const int* __restrict__ chunk_net;
  const int* __restrict__ chunk_depth;
  const int* __restrict__ net_list;
  int n_list;
  int n_chunks;
};

__global__ __launch_bounds__(kBlock) void k_rc_tree_adjoint(TreeAdjArgs a) {
  const float* __restrict__ xs = snap_elems(a.x, a.snap.pins);
  const float* __restrict__ ys = snap_elems(a.y, a.snap.pins);
  const float4* __restrict__ T = snap_bytes(a.tree, a.snap.state);
  const float2* __restrict__ A = snap_bytes(a.tree_adj, a.snap.work);
  float4* __restrict__ B = snap_bytes(a.bar, a.snap.work);   // {dDelay, dBeta, dLDelay, dLoad}, {dCap, dlen, gx, gy}
  float* __restrict__ dx = snap_elems(a.dx, a.snap.pins);
  float* __restrict__ dy = snap_elems(a.dy, a.snap.pins);
  const int k = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (k >= a.n_list) return;
  const int n = a.net_list[k];
  const int b = a.net_off[n], e = a.net_off[n + 1];
  const float kr = 1e-3f * a.r, hc = 0.5f * a.c;
  for (int q = b; q < e; ++q) {                     // seeds: the impulse into Beta and Delay
    float dd = 0.f, db = 0.f, dl = 0.f;
    if (q == b) {
      dl = A[q].x;
    } else {
      const float2 g = A[q];
      const float dly = T[2 * (size_t)q].w, imp = T[2 * (size_t)q + 1].z;
      dd = g.x;
      if (imp > 0.f) {
        db = g.y / imp;
        dd -= g.y * dly / imp;
      }
    }
    B[2 * (size_t)q] = make_float4(dd, db, 0.f, dl);
    B[2 * (size_t)q + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  for (int j = e - 1; j > b; --j) {                 // Beta, children first
    const int u = a.tree_order[j];
    const float bb = B[2 * (size_t)u].y;
    B[2 * (size_t)a.parent[u]].y += bb;
    B[2 * (size_t)u + 1].y += kr * T[2 * (size_t)u + 1].x * bb;
    B[2 * (size_t)u].z += kr * T[2 * (size_t)u].x * bb;
  }
  for (int j = b; j < e; ++j) {                     // LDelay, parents first
    const int u = a.tree_order[j];
    if (j > b) B[2 * (size_t)u].z += B[2 * (size_t)a.parent[u]].z;
    const float ld = B[2 * (size_t)u].z;
    B[2 * (size_t)u + 1].x += ld * T[2 * (size_t)u].w;
    B[2 * (size_t)u].x += ld * T[2 * (size_t)u].y;
  }
  for (int j = e - 1; j > b; --j) {                 // Delay, children first
    const int u = a.tree_order[j];
    const float dd = B[2 * (size_t)u].x;
    const float4 t = T[2 * (size_t)u];
    B[2 * (size_t)a.parent[u]].x += dd;
    B[2 * (size_t)u + 1].y += kr * t.z * dd;
    B[2 * (size_t)u].w += kr * t.x * dd;
  }
  for (int j = b; j < e; ++j) {                     // Load, parents first
    const int u = a.tree_order[j];
    if (j > b) B[2 * (size_t)u].w += B[2 * (size_t)a.parent[u]].w;
    B[2 * (size_t)u + 1].x += B[2 * (size_t)u].w;
  }
  for (int q = b + 1; q < e; ++q) {                 // Cap and Res to lengths, lengths to x, y
    const int f = a.parent[q];
    const float lb = B[2 * (size_t)q + 1].y + hc * (B[2 * (size_t)q + 1].x + B[2 * (size_t)f + 1].x);
    const int qo = a.io_perm ? a.io_perm[q] : q, fo = a.io_perm ? a.io_perm[f] : f;
    const float gx = lb * sgnf(xs[qo] - xs[fo]), gy = lb * sgnf(ys[qo] - ys[fo]);
    B[2 * (size_t)q + 1].z += gx;
    B[2 * (size_t)q + 1].w += gy;
    B[2 * (size_t)f + 1].z -= gx;
    B[2 * (size_t)f + 1].w -= gy;
  }
  for (int q = b; q < e; ++q) {
    const int qo = a.io_perm ? a.io_perm[q] : q;
    if (dx) dx[qo] = B[2 * (size_t)q + 1].z;
    if (dy) dy[qo] = B[2 * (size_t)q + 1].w;
  }
}

// The RC tree passes for a chunk of whole nets (at most kTreeChunk pins) per workgroup, in LDS:
// each thread holds kTreePer pins, and the passes run depth by depth with a barrier between
// depths - Load and LDelay from the deepest depth up, each node summing its children (a run
// of breadth-first positions) in order; Delay and Beta from the root down, each node reading
// its parent.  Same values as k_rc_tree, kept in `tree` for the adjoint.
constexpr int kTreePer = kTreeChunk / kBlock;
static_assert(kTreePer * kBlock == kTreeChunk, "chunk must be a multiple of the workgroup");

__global__ __launch_bounds__(kBlock) void k_rc_tree_chunk(RcArgs a) {
  __shared__ float Llen[kTreeChunk], Lcap[kTreeChunk], Lload[kTreeChunk], Ldly[kTreeChunk], Lld[kTreeChunk],
      Lbeta[kTreeChunk];
  if ((int)blockIdx.x >= a.n_chunks) return;              // padding blocks of a snapshot grid
  const int maxd = a.chunk_depth[blockIdx.x];
  if (maxd < 0) return;                                   // a net left to the fallback kernel
  const float* __restrict__ xs = snap_elems(a.x, a.snap.pins);
  const float* __restrict__ ys = snap_elems(a.y, a.snap.pins);
  float2* __restrict__ wire = snap_bytes(a.wire, a.snap.state);
  float* __restrict__ loads = snap_bytes(a.load, a.snap.state);
  float4* __restrict__ rec = snap_bytes(a.rec, a.snap.state);
  float4* __restrict__ T = snap_bytes(a.tree, a.snap.state);
  const int n_lo = a.chunk_net[blockIdx.x], n_hi = a.chunk_net[blockIdx.x + 1];
  const int p_lo = a.net_off[n_lo], np = a.net_off[n_hi] - p_lo;
  const float kr = 1e-3f * a.r, hc = 0.5f * a.c;
  int dep[kTreePer], par[kTreePer], fc[kTreePer], nch[kTreePer];
  float len[kTreePer];
#pragma unroll
  for (int k = 0; k < kTreePer; ++k) {
    const int i = (int)threadIdx.x + k * kBlock;
    dep[k] = -1;
    par[k] = -1;
    fc[k] = nch[k] = 0;
    len[k] = 0.f;
    if (i < np) {
      const int q = p_lo + i;
      const int4 t = a.tree_node[q];
      dep[k] = t.x;
      fc[k] = t.y;
      nch[k] = t.z;
      const int f = a.parent[q];
      if (f >= 0) {
        par[k] = f - p_lo;
        const int qo = a.io_perm ? a.io_perm[q] : q, fo = a.io_perm ? a.io_perm[f] : f;
        len[k] = fabsf(xs[qo] - xs[fo]) + fabsf(ys[qo] - ys[fo]);
      }
      Llen[i] = len[k];
      Lcap[i] = fmaf(hc, len[k], a.pin_cap[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTreePer; ++k) {                    // half of every segment out of a pin
    const int i = (int)threadIdx.x + k * kBlock;
    if (nch[k] > 0) {
      float c = Lcap[i];
      for (int j = 0; j < nch[k]; ++j) c = fmaf(hc, Llen[a.tree_order[fc[k] + j] - p_lo], c);
      Lcap[i] = c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTreePer; ++k) {
    const int i = (int)threadIdx.x + k * kBlock;
    if (dep[k] >= 0) Lload[i] = Lcap[i];
  }
  for (int d = maxd - 1; d >= 0; --d) {                   // Load (Eq. 1), deepest first
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTreePer; ++k) {
      const int i = (int)threadIdx.x + k * kBlock;
      if (dep[k] == d && nch[k] > 0) {
        float v = Lload[i];
        for (int j = 0; j < nch[k]; ++j) v += Lload[a.tree_order[fc[k] + j] - p_lo];
        Lload[i] = v;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kTreePer; ++k)
    if (dep[k] == 0) Ldly[(int)threadIdx.x + k * kBlock] = 0.f;
  for (int d = 1; d <= maxd; ++d) {                       // Delay, from the root down
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTreePer; ++k) {
      const int i = (int)threadIdx.x + k * kBlock;
      if (dep[k] == d) Ldly[i] = Ldly[par[k]] + kr * len[k] * Lload[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTreePer; ++k) {
    const int i = (int)threadIdx.x + k * kBlock;
    if (dep[k] >= 0) Lld[i] = Lcap[i] * Ldly[i];
  }
  for (int d = maxd - 1; d >= 0; --d) {                   // LDelay, deepest first
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTreePer; ++k) {
      const int i = (int)threadIdx.x + k * kBlock;
      if (dep[k] == d && nch[k] > 0) {
        float v = Lld[i];
        for (int j = 0; j < nch[k]; ++j) v += Lld[a.tree_order[fc[k] + j] - p_lo];
        Lld[i] = v;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kTreePer; ++k)
    if (dep[k] == 0) Lbeta[(int)threadIdx.x + k * kBlock] = 0.f;
  for (int d = 1; d <= maxd; ++d) {                       // Beta, from the root down
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTreePer; ++k) {
      const int i = (int)threadIdx.x + k * kBlock;
      if (dep[k] == d) Lbeta[i] = Lbeta[par[k]] + kr * len[k] * Lld[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTreePer; ++k) {
    const int i = (int)threadIdx.x + k * kBlock;
    if (dep[k] < 0) continue;
    const int q = p_lo + i;
    const float dly = Ldly[i], beta = Lbeta[i];
    const float arg = 2.0f * beta - dly * dly;
    const float imp = arg > 0.f ? sqrtf(arg) : 0.f;
    if (dep[k] > 0) wire[q] = make_float2(dly, imp);
    T[2 * (size_t)q] = make_float4(len[k], Lcap[i], Lload[i], dly);
    T[2 * (size_t)q + 1] = make_float4(Lld[i], beta, imp, 0.f);
  }
  for (int n = n_lo + (int)threadIdx.x; n < n_hi; n += kBlock) {
    const int p0 = a.net_off[n];
    rc_root(a, wire, loads, rec, n, p0, Lload[p0 - p_lo], true);
  }
}

// Adjoint of the tree passes for a chunk of nets per workgroup in LDS (see k_rc_tree_chunk):
// seeds from the sweep (the impulse into Beta and Delay), then Beta and Delay totals summed
// over children from the deepest depth up, LDelay and Load totals passed down from parents,
// Cap and Res to segment lengths, and lengths to the coordinates of both segment ends.
__global__ __launch_bounds__(kBlock) void k_rc_tree_adjoint_chunk(TreeAdjArgs a) {
  __shared__ float Db[kTreeChunk], Bb[kTreeChunk], LDb[kTreeChunk], Lb[kTreeChunk], Cb[kTreeChunk],
      Gx[kTreeChunk], Gy[kTreeChunk];
  if ((int)blockIdx.x >= a.n_chunks) return;
  const int maxd = a.chunk_depth[blockIdx.x];
  if (maxd < 0) return;
  const float* __restrict__ xs = snap_elems(a.x, a.snap.pins);
  const float* __restrict__ ys = snap_elems(a.y, a.snap.pins);
  const float4* __restrict__ T = snap_bytes(a.tree, a.snap.state);
  const float2* __restrict__ A = snap_bytes(a.tree_adj, a.snap.work);
  float* __restrict__ dx = snap_elems(a.dx, a.snap.pins);
  float* __restrict__ dy = snap_elems(a.dy, a.snap.pins);
  const int n_lo = a.chunk_net[blockIdx.x], n_hi = a.chunk_net[blockIdx.x + 1];
  const int p_lo = a.net_off[n_lo], np = a.net_off[n_hi] - p_lo;
  const float kr = 1e-3f * a.r, hc = 0.5f * a.c;
  int dep[kTreePer], par[kTreePer], fc[kTreePer], nch[kTreePer];
  float len[kTreePer], cap[kTreePer], load[kTreePer], dly[kTreePer], ld[kTreePer], lenb[kTreePer];
  float sx[kTreePer], sy[kTreePer];
#pragma unroll
  for (int k = 0; k < kTreePer; ++k) {
    const int i = (int)threadIdx.x + k * kBlock;
    dep[k] = -1;
    par[k] = -1;
    fc[k] = nch[k] = 0;
    len[k] = cap[k] = load[k] = dly[k] = ld[k] = lenb[k] = sx[k] = sy[k] = 0.f;
    if (i < np) {
      const int q = p_lo + i;
      const int4 t = a.tree_node[q];
      dep[k] = t.x;
      fc[k] = t.y;
      nch[k] = t.z;
      const int f = a.parent[q];
      const float4 t0 = T[2 * (size_t)q], t1 = T[2 * (size_t)q + 1];
      len[k] = t0.x;
      cap[k] = t0.y;
      load[k] = t0.z;
      dly[k] = t0.w;
      ld[k] = t1.x;
      float dd = 0.f, db = 0.f, dl = 0.f;
      const float2 g = A[q];
      if (f < 0) {
        dl = g.x;                                          // the root load's adjoint
      } else {
        par[k] = f - p_lo;
        const int qo = a.io_perm ? a.io_perm[q] : q, fo = a.io_perm ? a.io_perm[f] : f;
        sx[k] = sgnf(xs[qo] - xs[fo]);
        sy[k] = sgnf(ys[qo] - ys[fo]);
        dd = g.x;
        if (t1.z > 0.f) {                                  // Impulse = sqrt(2 Beta - Delay^2)
          db = g.y / t1.z;
          dd -= g.y * t0.w / t1.z;
        }
      }
      Db[i] = dd;
      Bb[i] = db;
      Lb[i] = dl;
      Cb[i] = 0.f;
    }
  }
  for (int d = maxd - 1; d >= 0; --d) {                   // Beta totals, deepest first
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTreePer; ++k) {
      const int i = (int)threadIdx.x + k * kBlock;
      if (dep[k] == d && nch[k] > 0) {
        float v = Bb[i];
        for (int j = 0; j < nch[k]; ++j) v += Bb[a.tree_order[fc[k] + j] - p_lo];
        Bb[i] = v;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTreePer; ++k) {
    const int i = (int)threadIdx.x + k * kBlock;
    if (dep[k] < 0) continue;
    lenb[k] = kr * ld[k] * Bb[i];
    LDb[i] = kr * len[k] * Bb[i];
  }
  for (int d = 1; d <= maxd; ++d) {                       // LDelay totals, from the root down
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTreePer; ++k) {
      const int i = (int)threadIdx.x + k * kBlock;
      if (dep[k] == d) LDb[i] += LDb[par[k]];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTreePer; ++k) {
    const int i = (int)threadIdx.x + k * kBlock;
    if (dep[k] < 0) continue;
    Cb[i] += LDb[i] * dly[k];
    Db[i] += LDb[i] * cap[k];
  }
  for (int d = maxd - 1; d >= 0; --d) {                   // Delay totals, deepest first
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTreePer; ++k) {
      const int i = (int)threadIdx.x + k * kBlock;
      if (dep[k] == d && nch[k] > 0) {
        float v = Db[i];
        for (int j = 0; j < nch[k]; ++j) v += Db[a.tree_order[fc[k] + j] - p_lo];
        Db[i] = v;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTreePer; ++k) {
    const int i = (int)threadIdx.x + k * kBlock;
    if (dep[k] <= 0) continue;
    lenb[k] += kr * load[k] * Db[i];
    Lb[i] += kr * len[k] * Db[i];
  }
  for (int d = 1; d <= maxd; ++d) {                       // Load totals, from the root down
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTreePer; ++k) {
      const int i = (int)threadIdx.x + k * kBlock;
      if (dep[k] == d) Lb[i] += Lb[par[k]];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTreePer; ++k) {
    const int i = (int)threadIdx.x + k * kBlock;
    if (dep[k] >= 0) Cb[i] += Lb[i];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTreePer; ++k) {                    // Cap: half of the segment at each end
    const int i = (int)threadIdx.x + k * kBlock;
    if (dep[k] < 0) continue;
    if (dep[k] > 0) lenb[k] += hc * (Cb[i] + Cb[par[k]]);
    Gx[i] = lenb[k] * sx[k];
    Gy[i] = lenb[k] * sy[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTreePer; ++k) {                    // both ends of every segment
    const int i = (int)threadIdx.x + k * kBlock;
    if (dep[k] < 0) continue;
    float gx = Gx[i], gy = Gy[i];
    for (int j = 0; j < nch[k]; ++j) {
      const int c = a.tree_order[fc[k] + j] - p_lo;
      gx -= Gx[c];
      gy -= Gy[c];
    }
    const int q = p_lo + i;
    const int qo = a.io_perm ? a.io_perm[q] : q;
    if (dx) dx[qo] = gx;
    if (dy) dy[qo] = gy;
  }
}

// ---------------------------------------------------------------------------- cell inputs
// Padded slots of one level's cell inputs: input j of the k-th cell is ell[base + j*nc + k];
// an empty slot holds source net -1.
struct Slots {
  int base, F, c0, nc;
};

struct ArcIn {          // one cell input seen from one condition
  float at, slew, atg;  // arrival, slew and smoothed arrival at the input pin
  int arc, tp, pin;
  int slot;             // the input pin's sink workspace slot
  bool valid;
};

// Input slot entries are {source record slot, input pin, arc with the sign bit set for
// negative unateness, the input pin's sink slot (its wire and its workspace records)}.
__device__ __forceinline__ int ell_arc(const int4& e) { return e.z & 0x7fffffff; }
__device__ __forceinline__ bool ell_positive(const int4& e) { return e.z >= 0; }

// Input j of cell kc for output condition (m, t): the source net's driver record plus the
// wire to the input pin, in the input transition the arc's unateness selects.  Missing
// inputs (j past the cell's fanin) read net 0 and come back invalid.
__device__ __forceinline__ ArcIn arc_input(const int4* __restrict__ ell, const Slots& sl, int kc, int j,
                                           const float4* __restrict__ rec, const float2* __restrict__ wire,
                                           int m, int t);

// The same from an input slot entry already loaded (entries of empty slots are valid
// addresses: source -1 reads record 0, pin 0, arc 0).
__device__ __forceinline__ ArcIn arc_input_entry(const int4 e, bool valid, const float4* __restrict__ rec,
                                                 const float2* __restrict__ wire, int m, int t) {
  ArcIn r;
  r.valid = valid && e.x >= 0;
  r.arc = ell_arc(e);
  r.tp = ell_positive(e) ? t : 1 - t;
  r.pin = e.y;
  r.slot = e.w;
  const int kp = 2 * m + r.tp;
  const float4 c = ld(rec, (uint32_t)(kRecChunks * max(e.x, 0) + kp));
  const float2 w = ld(wire, (uint32_t)e.w);
  r.at = c.x + w.x;
  r.slew = sink_slew(c.y, w.y);
  r.atg = c.z + w.x;
  return r;
}

__device__ __forceinline__ ArcIn arc_input(const int4* __restrict__ ell, const Slots& sl, int kc, int j,
                                           const float4* __restrict__ rec, const float2* __restrict__ wire,
                                           int m, int t) {
  const int4 e = ell[sl.base + (size_t)min(j, sl.F - 1) * sl.nc + kc];
  ArcIn r;
  r.valid = j < sl.F && e.x >= 0;
  r.arc = ell_arc(e);
  r.tp = ell_positive(e) ? t : 1 - t;
  r.pin = e.y;
  r.slot = e.w;
  const int kp = 2 * m + r.tp;
  const float4 c = rec[kRecChunks * (size_t)max(e.x, 0) + kp];   // {AT, slew, smoothed AT} of kp
  const float2 w = wire[e.w];
  r.at = c.x + w.x;
  r.slew = sink_slew(c.y, w.y);
  r.atg = c.z + w.x;
  return r;
}

// ---------------------------------------------------------------------------- forward level
// Arguments of a forward level that the first loads do not need.
struct FwdArgs {
  const float2* __restrict__ wire;
  const float4* __restrict__ grid;
  const float4* __restrict__ coef;
  LutKeys keys;
  float gamma, inv_gamma;
  int smooth;
};

// One level of forward propagation (Sec. 3.1.2).  16 lanes per cell: lane (k, j) looks up
// arc j for condition k = 2*mode + transition; the 4 arc lanes of a condition then merge
// by max (late) / min (early), worst slew, and log-sum-exp of the late candidates (Eq. 4).
// The values the first loads depend on come first, as scalar parameters, so that they are
// preloaded into scalar registers at wave launch instead of read from the argument buffer:
// the level's cell count, its first net, its input slots (base, width), the smallest
// record slot recomputed (cells whose net's record lies below it are kept records and
// skipped), the state bytes of one snapshot, the record slot map (NULL: slot = net) and
// snapshot 0's load and record arrays.
template <bool kSnap>
__global__ __launch_bounds__(kBlock) void k_fwd_level(int nc, int n0, int base, int F, int min_slot, int snap_state,
                                                      const int4* __restrict__ ell, const float* __restrict__ loads0,
                                                      const int* __restrict__ loc, float4* __restrict__ rec0,
                                                      FwdArgs a) {
  const Slots sl{base, F, 0, nc};
  const SnapBlock sb = snap_block<kSnap>();
  const float* loads = snap_bytes<kSnap>(loads0, (size_t)snap_state, sb.s);
  float4* rec = snap_bytes<kSnap>(rec0, (size_t)snap_state, sb.s);
  a.wire = snap_bytes<kSnap>(a.wire, (size_t)snap_state, sb.s);
  const int gid = sb.x * kBlock + (int)threadIdx.x;
  const int kc = gid / kCellLanes;
  if (kc >= sl.nc) return;                     // uniform over the cell's 16 lanes
  const int lane = gid & (kCellLanes - 1);
  const int k = lane >> 2, jl = lane & 3, m = k >> 1, t = k & 1;
  const int n = n0 + kc;
  // Loads in three waves, each issued as soon as its addresses are known: the first input
  // slot entry and the root load; the source record and wire; the table coefficients.
  const int4 e0 = ld(ell, (uint32_t)(sl.base + min(jl, sl.F - 1) * sl.nc + kc));
  const float load = ld(loads, (uint32_t)n);
  const int slot = loc ? ld(loc, (uint32_t)n) : n;
  if (slot < min_slot) return;                 // kept record, not recomputed
  float best_at = m ? -kInf : kInf;
  float best_sl = best_at;
  float lm = -kInf, ls = 0.f;
  for (int j0 = 0; j0 < sl.F; j0 += kArcLanes) {
    const ArcIn in = j0 == 0 ? arc_input_entry(e0, jl < sl.F, rec, a.wire, m, t)
                             : arc_input(ell, sl, kc, j0 + jl, rec, a.wire, m, t);
    const LutVal v = lut_eval<false>(a.grid, a.coef, a.keys, in.arc, t, in.slew, load);
    float cand = m ? -kInf : kInf, s = cand, g = -kInf;
    if (in.valid) {
      cand = in.at + v.d;
      s = v.s;
      g = in.atg + v.d;
    }
    if (m) {
      best_at = fmaxf(best_at, quad_reduce<kMax>(cand));
      best_sl = fmaxf(best_sl, quad_reduce<kMax>(s));
      if (a.smooth) {
        const float gm = quad_reduce<kMax>(g);
        const float gs = quad_reduce<kSum>(in.valid ? fexp((g - gm) * a.inv_gamma) : 0.f);
        lse_merge(lm, ls, gm, gs, a.inv_gamma);
      }
    } else {
      best_at = fminf(best_at, quad_reduce<kMin>(cand));
      best_sl = fminf(best_sl, quad_reduce<kMin>(s));
    }
  }
  if (jl == 0) {
    const float ag = m ? (a.smooth ? fmaf(a.gamma, flog(ls), lm) : __builtin_nanf("")) : 0.f;
    *at32(rec, (uint32_t)(kRecChunks * slot + k)) = make_float4(best_at, best_sl, ag, 0.f);
  }
}

// The same level with 4 * L lanes per cell, L = 1 or 2 lanes per condition k: lane (k, jl)
// looks up arcs jl, jl + L, ... of each chunk of 4 (their loads issued together), merges
// them in registers and then, for L = 2, with the other lane of its pair.  Same arguments
// and results up to the order of the log-sum-exp terms; a quarter (L = 1) or half (L = 2)
// of the waves of k_fwd_level, at the price of serial lookups in each lane.
template <int L>
__device__ __forceinline__ float pair_reduce_max(float v) {
  return L == 2 ? fmaxf(v, dpp<kDppQuadX1>(v)) : v;
}
template <int L>
__device__ __forceinline__ float pair_reduce_min(float v) {
  return L == 2 ? fminf(v, dpp<kDppQuadX1>(v)) : v;
}
template <int L>
__device__ __forceinline__ float pair_reduce_sum(float v) {
  return L == 2 ? v + dpp<kDppQuadX1>(v) : v;
}

template <bool kSnap, int L>
__global__ __launch_bounds__(kBlock) void k_fwd_level_narrow(int nc, int n0, int base, int F, int min_slot,
                                                             int snap_state, const int4* __restrict__ ell,
                                                             const float* __restrict__ loads0,
                                                             const int* __restrict__ loc, float4* __restrict__ rec0,
                                                             FwdArgs a) {
  constexpr int kLanes = 4 * L;                // lanes per cell
  constexpr int kArcs = kArcLanes / L;         // arcs per lane in a chunk of 4
  const Slots sl{base, F, 0, nc};
  const SnapBlock sb = snap_block<kSnap>();
  const float* loads = snap_bytes<kSnap>(loads0, (size_t)snap_state, sb.s);
  float4* rec = snap_bytes<kSnap>(rec0, (size_t)snap_state, sb.s);
  a.wire = snap_bytes<kSnap>(a.wire, (size_t)snap_state, sb.s);
  const int gid = sb.x * kBlock + (int)threadIdx.x;
  const int kc = gid / kLanes;
  if (kc >= sl.nc) return;                     // uniform over the cell's lanes
  const int lane = gid & (kLanes - 1);
  const int k = lane / L, jl = lane % L, m = k >> 1, t = k & 1;
  const int n = n0 + kc;
  // Loads in three waves, each issued as soon as its addresses are known: the input slot
  // entries and the root load; the source records and wires; the table coefficients.
  int4 e[kArcs];
#pragma unroll
  for (int i = 0; i < kArcs; ++i)
    e[i] = ld(ell, (uint32_t)(sl.base + min(jl + L * i, sl.F - 1) * sl.nc + kc));
  const float load = ld(loads, (uint32_t)n);
  const int slot = loc ? ld(loc, (uint32_t)n) : n;
  if (slot < min_slot) return;                 // kept record, not recomputed
  float best_at = m ? -kInf : kInf;
  float best_sl = best_at;
  float lm = -kInf, ls = 0.f;
  for (int j0 = 0; j0 < sl.F; j0 += kArcLanes) {
    ArcIn in[kArcs];
#pragma unroll
    for (int i = 0; i < kArcs; ++i) {
      const int j = j0 + jl + L * i;
      in[i] = j0 == 0 ? arc_input_entry(e[i], j < sl.F, rec, a.wire, m, t)
                      : arc_input(ell, sl, kc, j, rec, a.wire, m, t);
    }
    LutVal v[kArcs];
#pragma unroll
    for (int i = 0; i < kArcs; ++i) v[i] = lut_eval<false>(a.grid, a.coef, a.keys, in[i].arc, t, in[i].slew, load);
    const float neutral = m ? -kInf : kInf;
    float g[kArcs];
    float cm = neutral, sm = neutral, gm = -kInf;
#pragma unroll
    for (int i = 0; i < kArcs; ++i) {
      const float cand = in[i].valid ? in[i].at + v[i].d : neutral;
      const float s = in[i].valid ? v[i].s : neutral;
      g[i] = in[i].valid ? in[i].atg + v[i].d : -kInf;
      if (m) {
        cm = fmaxf(cm, cand);
        sm = fmaxf(sm, s);
        gm = fmaxf(gm, g[i]);
      } else {
        cm = fminf(cm, cand);
        sm = fminf(sm, s);
      }
    }
    if (m) {
      best_at = fmaxf(best_at, pair_reduce_max<L>(cm));
      best_sl = fmaxf(best_sl, pair_reduce_max<L>(sm));
      if (a.smooth) {
        gm = pair_reduce_max<L>(gm);
        float gs = 0.f;
#pragma unroll
        for (int i = 0; i < kArcs; ++i) gs += in[i].valid ? fexp((g[i] - gm) * a.inv_gamma) : 0.f;
        lse_merge(lm, ls, gm, pair_reduce_sum<L>(gs), a.inv_gamma);
      }
    } else {
      best_at = fminf(best_at, pair_reduce_min<L>(cm));
      best_sl = fminf(best_sl, pair_reduce_min<L>(sm));
    }
  }
  if (jl == 0) {
    const float ag = m ? (a.smooth ? fmaf(a.gamma, flog(ls), lm) : __builtin_nanf("")) : 0.f;
    *at32(rec, (uint32_t)(kRecChunks * slot + k)) = make_float4(best_at, best_sl, ag, 0.f);
  }
}

// ---------------------------------------------------------------------------- endpoints
struct EpArgs {
  const int* __restrict__ ep_pin;
  const int* __restrict__ ep_net;
  const int* __restrict__ ep_design;      // design of each endpoint
  const int* __restrict__ ep_design_off;  // [n_designs+1]
  const int* __restrict__ ep_blk_off;     // [n_designs+1] partial blocks by design
  const float4* __restrict__ rec;
  const float2* __restrict__ wire;
  double* part;        // [blocks][5]
  double* fin;         // [designs][8]
  double* scalars;     // [designs][4] or NULL
  float4* sink;        // per sink {RAT}, {adjoint} (see rat_at / adj_at)
  int seed_adj;        // also seed the adjoint
  const double* scale_dev;
  int E, n_designs;
  float rat_late, hold, gamma, inv_gamma, scale;
  int smooth, wns_mode;
  Snap snap;
  float4* epv;        // per endpoint {s_e, w_rise, w_fall, worst slack}: written by the partials
                      // (by k_ep_values under checkpointing), read by the seeds
  const int* ep_sslot;  // checkpointing: each endpoint's workspace slot (NULL: its pin)
  int from_epv = 0;     // the partials read epv instead of records (checkpointing)
};

// The endpoint arguments of snapshot blockIdx.y.
__device__ __forceinline__ EpArgs ep_snap(const EpArgs& a0) {
  EpArgs a = a0;
  a.rec = snap_bytes(a.rec, a.snap.state);
  a.wire = snap_bytes(a.wire, a.snap.state);
  a.part = snap_bytes(a.part, a.snap.state);
  a.fin = snap_bytes(a.fin, a.snap.state);
  a.scalars = snap_elems(a.scalars, a.snap.scal);
  a.sink = snap_bytes(a.sink, a.snap.work);
  a.epv = snap_bytes(a.epv, a.snap.state);
  return a;
}

struct EpVals {
  float worst;    // hard late slack, worst transition
  float sg;       // smoothed slack s_e
  float w0, w1;   // d s_e / d slack_g(e, t)
};

__device__ __forceinline__ EpVals endpoint_values(const EpArgs& a, int i) {
  const int e = a.ep_pin[i];
  const float4 c2 = a.rec[kRecChunks * (size_t)a.ep_net[i] + 2];   // late rise
  const float4 c3 = a.rec[kRecChunks * (size_t)a.ep_net[i] + 3];   // late fall
  const float dl = a.wire[a.ep_sslot ? a.ep_sslot[i] : e].x;
  EpVals v;
  v.worst = fminf(a.rat_late - (c2.x + dl), a.rat_late - (c3.x + dl));
  // s_e = -LSE(-slack_g(rise), -slack_g(fall))
  const float u0 = -(a.rat_late - (c2.z + dl));
  const float u1 = -(a.rat_late - (c3.z + dl));
  const float mx = fmaxf(u0, u1);
  const float e0 = expf((u0 - mx) * a.inv_gamma), e1 = expf((u1 - mx) * a.inv_gamma);
  const float z = e0 + e1;
  v.sg = -(mx + a.gamma * logf(z));
  v.w0 = e0 / z;
  v.w1 = e1 / z;
  return v;
}

// Sums and maxima of K doubles at once over the 256 threads of a workgroup: xor butterflies
// inside each wave (symmetric, so every lane ends with the same bits), then the four wave
// results in wave order through LDS.  `sh` holds 4 * K doubles.
template <int K>
__device__ __forceinline__ void block_reduce(double (&v)[K], const bool (&is_max)[K], double* sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double w = __shfl_xor(v[k], o);
      v[k] = is_max[k] ? fmax(v[k], w) : v[k] + w;
    }
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[(threadIdx.x >> 6) * K + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double r = sh[k];
    for (int q = 1; q < kWavesPerBlock; ++q) r = is_max[k] ? fmax(r, sh[q * K + k]) : r + sh[q * K + k];
    v[k] = r;
  }
  __syncthreads();
}

// Per-block partial sums over endpoints, in float64 and a fixed order: hard TNS, hard
// worst slack, smoothed TNS terms, and a shifted sum of exponentials for smoothed WNS.
// Each design's endpoints fill their own run of blocks.
__global__ __launch_bounds__(kBlock) void k_ep_partials(EpArgs a0) {
  __shared__ double sh[kBlock];
  const EpArgs a = ep_snap(a0);
  int dsg = 0;
  while (dsg + 1 < a.n_designs && (int)blockIdx.x >= a.ep_blk_off[dsg + 1]) ++dsg;
  const int i = a.ep_design_off[dsg] + ((int)blockIdx.x - a.ep_blk_off[dsg]) * kBlock + (int)threadIdx.x;
  const bool act = i < a.ep_design_off[dsg + 1];
  double tns = 0.0, wmin = __builtin_huge_val(), tnsg = 0.0, v = -__builtin_huge_val();
  if (act) {
    EpVals ev;
    if (a.from_epv) {                                  // taken per segment (k_ep_values)
      const float4 q = a.epv[i];
      ev = EpVals{q.w, q.x, q.y, q.z};
    } else {
      ev = endpoint_values(a, i);
      a.epv[i] = make_float4(ev.sg, ev.w0, ev.w1, ev.worst);   // kept for the backward's seeds
    }
    tns = fmin(0.0, (double)ev.worst);
    wmin = ev.worst;
    // -LSE_g(0, -s) = -(max(0,-s) + g*log1p(exp(-|s|/g))), each term in float (about 1e-7
    // relative); the sums run in float64 in a fixed order.
    tnsg = -(double)(fmaxf(0.f, -ev.sg) + a.gamma * log1pf(expf(-fabsf(ev.sg) * a.inv_gamma)));
    v = -(double)ev.sg;
  }
  double r4[4] = {tns, -wmin, tnsg, v};
  block_reduce<4>(r4, {false, true, false, true}, sh);
  tns = r4[0];
  wmin = -r4[1];
  tnsg = r4[2];
  const double mb = r4[3];
  double r1[1] = {act ? (double)expf((float)(v - mb) * a.inv_gamma) : 0.0};
  block_reduce<1>(r1, {false}, sh);
  const double sb = r1[0];
  if (threadIdx.x == 0) {
    double* p = a.part + 5 * (size_t)blockIdx.x;
    p[0] = tns;
    p[1] = wmin;
    p[2] = tnsg;
    p[3] = mb;
    p[4] = sb;
  }
}

// Scalars of design blockIdx.x from its partial blocks (fixed order).
__global__ __launch_bounds__(kBlock) void k_ep_finalize(EpArgs a0) {
  __shared__ double sh[kBlock];
  const EpArgs a = ep_snap(a0);
  const int dsg = blockIdx.x;
  const int b0 = a.ep_blk_off[dsg], b1 = a.ep_blk_off[dsg + 1];
  double tns = 0.0, wmin = __builtin_huge_val(), tnsg = 0.0, mx = -__builtin_huge_val();
  for (int b = b0 + (int)threadIdx.x; b < b1; b += kBlock) {
    const double* p = a.part + 5 * (size_t)b;
    tns += p[0];
    wmin = fmin(wmin, p[1]);
    tnsg += p[2];
    mx = fmax(mx, p[3]);
  }
  double r4[4] = {tns, -wmin, tnsg, mx};
  block_reduce<4>(r4, {false, true, false, true}, sh);
  tns = r4[0];
  wmin = -r4[1];
  tnsg = r4[2];
  const double M = fmax(0.0, r4[3]);   // {0} joins the WNS_g set
  double tot = 0.0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += kBlock) {
    const double* p = a.part + 5 * (size_t)b;
    if (p[4] > 0.0) tot += p[4] * exp((p[3] - M) / (double)a.gamma);
  }
  double r1[1] = {tot};
  block_reduce<1>(r1, {false}, sh);
  tot = r1[0];
  if (threadIdx.x == 0) {
    tot += exp(-M / (double)a.gamma);
    const double lse_all = M + (double)a.gamma * log(tot);
    const double nan = __builtin_nan("");
    double* fin = a.fin + 8 * (size_t)dsg;
    fin[0] = fmin(0.0, wmin);
    fin[1] = tns;
    fin[2] = a.smooth ? -lse_all : nan;
    fin[3] = a.smooth ? tnsg : nan;
    fin[4] = lse_all;
    if (a.scalars) {
      for (int q = 0; q < 4; ++q) a.scalars[4 * (size_t)dsg + q] = fin[q];
    }
  }
}

// Seeds of the backward sweep at the endpoints: constrained required times, and the
// adjoint of the smoothed objective with respect to each endpoint's smoothed arrival.
// Seeds of the endpoints list[0..n) (every endpoint when list is NULL and n = E).
__global__ __launch_bounds__(kBlock) void k_ep_seed(EpArgs a0, const int* __restrict__ list, int n) {
  const int t = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (t >= n) return;
  const int i = list ? list[t] : t;
  const EpArgs a = ep_snap(a0);
  const int e = a.ep_sslot ? a.ep_sslot[i] : a.ep_pin[i];   // the endpoint's workspace slot
  a.sink[rat_at(e)] = make_float4(a.hold, a.hold, a.rat_late, a.rat_late);
  if (a.seed_adj) {
    // s_e and its weights as the forward computed them (same coordinates and gamma).
    const float4 q = a.epv[i];
    EpVals ev;
    ev.sg = q.x;
    ev.w0 = q.y;
    ev.w1 = q.z;
    float coef;
    if (a.wns_mode) {
      const double lse_all = a.fin[8 * (size_t)a.ep_design[i] + 4];
      coef = (float)exp((-(double)ev.sg - lse_all) / (double)a.gamma);     // d WNS_g / d s_e
    } else {
      coef = 1.0f / (1.0f + expf(ev.sg * a.inv_gamma));                    // d TNS_g / d s_e
    }
    // d s_e / d atg(e, t) = -w_t; the objective's adjoint scales by `scale`.
    const float sc = a.scale_dev ? a.scale * (float)a.scale_dev[0] : a.scale;
    a.sink[adj_at(e)] = make_float4(-sc * coef * ev.w0, -sc * coef * ev.w1, 0.f, 0.f);
  }
}

// Under checkpointing: the values of the endpoints list[0..n), taken while their nets'
// records and wire values are in the segment's slots; the partials and seeds read them.
__global__ __launch_bounds__(kBlock) void k_ep_values(EpArgs a0, const int* __restrict__ list, int n) {
  const int t = (int)(blockIdx.x * kBlock + threadIdx.x);
  if (t >= n) return;
  const EpArgs a = ep_snap(a0);
  const int i = list[t];
  const EpVals ev = endpoint_values(a, i);
  a.epv[i] = make_float4(ev.sg, ev.w0, ev.w1, ev.worst);
}

// ---------------------------------------------------------------------------- outputs
// Streaming store of a per-pin output: written once, read by no later kernel of the sweep,
// so it bypasses the cache instead of waiting in L2 for the end-of-kernel writeback.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_stream(float4* p, const float4 v) {
  const f4v x = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(x, reinterpret_cast<f4v*>(p));
}
__device__ __forceinline__ void store_stream(float2* p, const float2 v) {
  const f2v x = {v.x, v.y};
  __builtin_nontemporal_store(x, reinterpret_cast<f2v*>(p));
}


struct ExpandArgs {
  const int* __restrict__ net_off;
  const int* __restrict__ io_perm;
  const int* __restrict__ sched;
  GroupRange range;
  const float4* __restrict__ rec;
  const float2* __restrict__ wire;
  float4* at;
  float4* slew;
  float2* atg;
  Snap snap;
};

// Per-pin arrival, slew and smoothed arrival from the net records (forward outputs).
__global__ __launch_bounds__(kBlock) void k_expand(ExpandArgs a) {
  const float4* __restrict__ rec = snap_bytes(a.rec, a.snap.state);
  const float2* __restrict__ wire = snap_bytes(a.wire, a.snap.state);
  float4* at_out = snap_elems(a.at, a.snap.pins);
  float4* slew_out = snap_elems(a.slew, a.snap.pins);
  float2* atg_out = snap_elems(a.atg, a.snap.pins);
  GroupSlot gs;
  if (!group_slot(a.range, gs) || !gs.active) return;
  const int n = a.sched[gs.entry];
  const int p0 = a.net_off[n], p1 = a.net_off[n + 1];
  const float4 c0 = rec[kRecChunks * (size_t)n], c1 = rec[kRecChunks * (size_t)n + 1],
               c2 = rec[kRecChunks * (size_t)n + 2], c3 = rec[kRecChunks * (size_t)n + 3];
  const float4 at = make_float4(c0.x, c1.x, c2.x, c3.x), sl = make_float4(c0.y, c1.y, c2.y, c3.y);
  const float2 ag = make_float2(c2.z, c3.z);
  for (int p = p0 + gs.gl; p < p1; p += gs.G) {
    const float2 w = wire[p];
    const int q = a.io_perm ? a.io_perm[p] : p;
    if (at_out) store_stream(at_out + q, make_float4(at.x + w.x, at.y + w.x, at.z + w.x, at.w + w.x));
    if (slew_out)
      store_stream(slew_out + q,
                   make_float4(sink_slew(sl.x, w.y), sink_slew(sl.y, w.y), sink_slew(sl.z, w.y), sink_slew(sl.w, w.y)));
    if (atg_out) store_stream(atg_out + q, make_float2(ag.x + w.x, ag.y + w.x));
  }
}

// ---------------------------------------------------------------------------- backward level
struct BwdArgs {
  const int* __restrict__ net_off;
  const float* __restrict__ pin_cap;
  const int4* __restrict__ ell;
  const int* __restrict__ io_perm;
  const float* __restrict__ x;
  const float* __restrict__ y;
  const float4* __restrict__ grid;
  const float4* __restrict__ coef;
  LutKeys keys;
  const float4* __restrict__ rec;
  const float2* __restrict__ wire;
  const float* __restrict__ load;
  const int* __restrict__ loc;       // record slot of each net, NULL: slot = net
  float4* sink;                      // per sink {RAT}, {adjoint} (see rat_at / adj_at)
  float4* __restrict__ at_out;
  float4* __restrict__ slew_out;
  float4* __restrict__ rat_out;
  float4* __restrict__ slack_out;
  float* __restrict__ dx;
  float* __restrict__ dy;
  int N0;
  float r, c, inv_gamma;
  int grad;
  Snap snap;
  float2* tree_adj;   // RC trees: the Elmore adjoint is left to k_rc_tree_adjoint (else NULL)
  const int* __restrict__ sink_base;  // checkpointing: first workspace slot of each net's sinks
                                      // (NULL: a sink's slot is its pin)
};

// Accumulators of the net step (reduced over the group).
enum { R_E0, R_E1, R_L0, R_L1, A_R, A_F, S_R, S_F, X_RS, X_N, Y_RS, Y_N, N_ACC };

struct SinkKeep {     // what phase 3 needs of a sink, kept in registers
  float gx, gy, rest;
  int q;
};

// What the net step reads of one sink.  Loaded apart from its use, so that the loads of
// a group's sinks are in flight while the cell step walks its own chain of loads.
struct SinkIn {
  float4 rt, aj;
  float2 w;
  float xs, ys, cp;
  int q;
};

// Sink p, whose workspace slot is `slot` (its pin without checkpointing).
template <bool kCanon, bool kGrad>
__device__ __forceinline__ SinkIn sink_load(const BwdArgs& a, int p, int slot) {
  SinkIn in;
  const uint32_t u = (uint32_t)p;
  in.rt = ld(a.sink, rat_at((uint32_t)slot));
  in.w = ld(a.wire, (uint32_t)slot);
  in.q = kCanon ? p : ld(a.io_perm, u);
  in.aj = make_float4(0.f, 0.f, 0.f, 0.f);
  in.xs = in.ys = in.cp = 0.f;
  if (kGrad) {
    in.aj = ld(a.sink, adj_at((uint32_t)slot));
    in.xs = ld(a.x, (uint32_t)in.q);
    in.ys = ld(a.y, (uint32_t)in.q);
    in.cp = ld(a.pin_cap, u);
  }
  return in;
}

// Net step of one sink: per-pin outputs and its contribution to the driver's reductions.
template <bool kGrad>
__device__ __forceinline__ SinkKeep sink_step(const BwdArgs& a, const SinkIn& in, const float4& at_d,
                                              const float4& sl_d, float xd, float yd, float (&acc)[N_ACC],
                                              bool write, int pc) {
  const float4 rt = in.rt, aj = in.aj;
  const float2 w = in.w;
  const int q = in.q;
  const float xs = in.xs, ys = in.ys, cp = in.cp;
  const float4 ats = make_float4(at_d.x + w.x, at_d.y + w.x, at_d.z + w.x, at_d.w + w.x);
  const float4 sls = make_float4(sink_slew(sl_d.x, w.y), sink_slew(sl_d.y, w.y), sink_slew(sl_d.z, w.y),
                                 sink_slew(sl_d.w, w.y));
  if (write) {
    const uint32_t uq = (uint32_t)q;
    if (a.at_out) store_stream(at32(a.at_out, uq), ats);
    if (a.slew_out) store_stream(at32(a.slew_out, uq), sls);
    if (a.rat_out) store_stream(at32(a.rat_out, uq), rt);
    if (a.slack_out)
      store_stream(at32(a.slack_out, uq), make_float4(ats.x - rt.x, ats.y - rt.y, rt.z - ats.z, rt.w - ats.w));
  }
  acc[R_E0] = fmaxf(acc[R_E0], rt.x - w.x);
  acc[R_E1] = fmaxf(acc[R_E1], rt.y - w.x);
  acc[R_L0] = fminf(acc[R_L0], rt.z - w.x);
  acc[R_L1] = fminf(acc[R_L1], rt.w - w.x);
  SinkKeep k{0.f, 0.f, 0.f, q};
  if (kGrad) {
    const float q0 = sls.z > 0.f ? aj.z * frcp(sls.z) : 0.f;   // s_bar(s,t) / slew(s,late,t)
    const float q1 = sls.w > 0.f ? aj.w * frcp(sls.w) : 0.f;
    acc[A_R] += aj.x;
    acc[A_F] += aj.y;
    acc[S_R] += q0 * sl_d.z;
    acc[S_F] += q1 * sl_d.w;
    const float dbar = aj.x + aj.y;                      // adjoint of the wire delay
    const float ibar = (q0 + q1) * w.y;                  // adjoint of the impulse
    if (a.tree_adj && write) *at32(a.tree_adj, (uint32_t)pc) = make_float2(dbar, ibar);
    const float len = fabsf(xs - xd) + fabsf(ys - yd);
    // d Delay / d len = d Impulse / d len = 1e-3 r (Cpin + c len) for a star sink.
    k.rest = (dbar + ibar) * (1e-3f * a.r * fmaf(a.c, len, cp));
    k.gx = sgnf(xs - xd);
    k.gy = sgnf(ys - yd);
    acc[X_RS] += k.gx * k.rest;
    acc[X_N] += k.gx;
    acc[Y_RS] += k.gy * k.rest;
    acc[Y_N] += k.gy;
  }
  return k;
}

struct ArcBwd {         // one arc of the cell step, seen from one condition's lane
  float d, xg, s, ddx, ddy, dsx, dsy;
  int pin, tp, slot;
  bool valid;
};

__device__ __forceinline__ ArcBwd arc_backward(const BwdArgs& a, const Slots& sl, int kc, int j, int m, int t,
                                               float load) {
  const ArcIn in = arc_input(a.ell, sl, kc, j, a.rec, a.wire, m, t);
  ArcBwd r;
  r.valid = in.valid;
  r.pin = in.pin;
  r.tp = in.tp;
  r.slot = in.slot;
  r.d = r.s = r.ddx = r.ddy = r.dsx = r.dsy = 0.f;
  r.xg = -kInf;
  if (in.valid) {
    const LutVal v = lut_eval<true>(a.grid, a.coef, a.keys, in.arc, t, in.slew, load);
    r.d = v.d;
    r.s = v.s;
    r.xg = in.atg + v.d;
    r.ddx = v.ddx;
    r.ddy = v.ddy;
    r.dsx = v.dsx;
    r.dsy = v.dsy;
  }
  return r;
}

// The cell-step lookup of an input already gathered: its table values at the input slew
// and the root load.  The lookup runs for every lane (indices are valid for any entry), and
// lanes without an arc come back invalid.
__device__ __forceinline__ ArcBwd arc_from_input(const BwdArgs& a, const ArcIn& in, int t, float load) {
  const LutVal v = lut_eval<true>(a.grid, a.coef, a.keys, in.arc, t, in.slew, load);
  ArcBwd r;
  r.valid = in.valid;
  r.pin = in.pin;
  r.tp = in.tp;
  r.slot = in.slot;
  r.d = in.valid ? v.d : 0.f;
  r.s = in.valid ? v.s : 0.f;
  r.xg = in.valid ? in.atg + v.d : -kInf;
  r.ddx = in.valid ? v.ddx : 0.f;
  r.ddy = in.valid ? v.ddy : 0.f;
  r.dsx = in.valid ? v.dsx : 0.f;
  r.dsy = in.valid ? v.dsy : 0.f;
  return r;
}

// Group-wide reduction of the net-step accumulators (G = 16/32/64 wave groups, or a whole
// workgroup when `block`).
template <int G>
__device__ __forceinline__ void reduce_acc(float (&v)[N_ACC], bool block, float* sh) {
  v[R_E0] = wave_group_reduce<kMax, G>(v[R_E0]);
  v[R_E1] = wave_group_reduce<kMax, G>(v[R_E1]);
  v[R_L0] = wave_group_reduce<kMin, G>(v[R_L0]);
  v[R_L1] = wave_group_reduce<kMin, G>(v[R_L1]);
#pragma unroll
  for (int i = A_R; i < N_ACC; ++i) v[i] = wave_group_reduce<kSum, G>(v[i]);
  if (block) {
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int i = 0; i < N_ACC; ++i) sh[w * N_ACC + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N_ACC; ++i) {
      float r = sh[i];
      for (int q = 1; q < kWavesPerBlock; ++q) {
        const float b = sh[q * N_ACC + i];
        r = i <= R_E1 ? fmaxf(r, b) : (i <= R_L1 ? fminf(r, b) : r + b);
      }
      v[i] = r;
    }
    __syncthreads();
  }
}

// Backward work of one net, Sec. 2.1 stage 4 and Sec. 3.1.2, fused with the adjoint of the
// smoothed objective (Sec. 3.2).  G lanes serve the net (a wave group, or the 256 threads of
// a workgroup when `block`; the workgroup then reduces through LDS):
//  1. net step over the sinks: per-pin outputs, RAT(driver) = min/max over sinks of
//     RAT(sink) - wire delay, sums of the sinks' adjoints into the driver;
//  2. cell step on the group's first 16 lanes, lane (k, j) for condition k and arc j:
//     every input's required time, the softmax split of the driver's adjoint over the arcs
//     (the LSE gradient), the slew adjoint through the table partials and the arg-max slew
//     arc, and the load adjoint;
//  3. Elmore adjoint: each sink's wire-length adjoint and d/dx, d/dy of every pin.
// The cell step's loads and table lookups depend only on forward state, so they are issued
// before the sink reduction they later combine with.
template <int G, bool kCanon, bool kGrad>
__device__ __forceinline__ void bwd_net(const BwdArgs& a, const Slots& sl, const GroupSlot& gs, float* sh) {
  const int gl = gs.gl;
  const bool block = gs.block;
  const int n = gs.active ? gs.entry : 0;      // level ranges index canonical nets
  // The loads are issued in three waves, each as soon as its addresses are known, with
  // indices clamped to valid entries instead of branches so that the compiler keeps every
  // wave's loads in flight together:
  //  1. pin range, record slot, the cell input's slot entry, the root load;
  //  2. the sinks' required times, adjoints, wires, coordinates and caps, the driver's
  //     record and coordinates, and the input's source record and wire;
  //  3. the table coefficients at the input slew.
  // The cell step spreads the 4 conditions over the group's first 16 lanes (4 arc lanes per
  // condition, one arc each per chunk of 4), over 8 lanes in 8-lane groups (2 arc lanes, two
  // arcs each) or over 4 lanes in 4-lane groups (one lane, all four arcs).
  constexpr int AL = G == 4 ? 1 : (G == 8 ? 2 : kArcLanes);   // arc lanes per condition
  constexpr int NA = kArcLanes / AL;           // arcs per lane in a chunk of 4
  constexpr int CL = 4 * AL;                   // cell lanes
  const int lanec = gl & (CL - 1);
  const int k = lanec / AL, jl = lanec % AL, m = k >> 1, t = k & 1;
  const bool cell_lane = gs.active && n >= a.N0 && gl < CL;
  const int kc = cell_lane ? n - a.N0 - sl.c0 : 0;   // position of the cell in its level
  const int p0 = ld(a.net_off, (uint32_t)n);
  const int p1v = ld(a.net_off, (uint32_t)n + 1u);
  int4 e[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i)
    e[i] = ld(a.ell, cell_lane ? (uint32_t)(sl.base + min(jl + AL * i, sl.F - 1) * sl.nc + kc) : 0u);
  const float load = ld(a.load, (uint32_t)n);
  const int slot = a.loc ? ld(a.loc, (uint32_t)n) : n;
  const int p1 = gs.active ? p1v : p0;
  // workspace slot of sink p: sk0 + p (its pin without checkpointing)
  const int sk0 = a.sink_base ? ld(a.sink_base, (uint32_t)n) - (p0 + 1) : 0;

  // Wave 2: the cell input's source record and wire first (the table lookup waits for
  // them), then the driver's record and coordinates and the sinks, whose loads stay in
  // flight through the lookup.
  ArcIn ain[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    ain[i].valid = cell_lane && jl + AL * i < sl.F && e[i].x >= 0;
    ain[i].arc = ell_arc(e[i]);
    ain[i].tp = ell_positive(e[i]) ? t : 1 - t;
    ain[i].pin = e[i].y;
    ain[i].slot = e[i].w;
    const int kp = 2 * m + ain[i].tp;
    const float4 c = ld(a.rec, (uint32_t)(kRecChunks * max(e[i].x, 0) + kp));
    const float2 w = ld(a.wire, (uint32_t)e[i].w);
    ain[i].at = c.x + w.x;
    ain[i].slew = sink_slew(c.y, w.y);
    ain[i].atg = c.z + w.x;
  }
  const uint32_t rs = (uint32_t)(kRecChunks * slot);
  const float4 c0 = ld(a.rec, rs), c1 = ld(a.rec, rs + 1), c2 = ld(a.rec, rs + 2), c3 = ld(a.rec, rs + 3);
  const float4 at_d = make_float4(c0.x, c1.x, c2.x, c3.x);
  const float4 sl_d = make_float4(c0.y, c1.y, c2.y, c3.y);
  float xd = 0.f, yd = 0.f;
  if (kGrad) {
    const int q = kCanon ? p0 : ld(a.io_perm, (uint32_t)p0);
    xd = ld(a.x, (uint32_t)q);
    yd = ld(a.y, (uint32_t)q);
  }
  const int s0 = p0 + 1 + gl;
  const int gstride = block ? kBlock : G;
  const bool has0 = s0 < p1;
  const bool has1 = block && s0 + gstride < p1;
  const SinkIn in0 = sink_load<kCanon, kGrad>(a, has0 ? s0 : p0, has0 ? sk0 + s0 : 0);
  SinkIn in1{};
  if (block) in1 = sink_load<kCanon, kGrad>(a, has1 ? s0 + gstride : p0, has1 ? sk0 + s0 + gstride : 0);
  __builtin_amdgcn_sched_barrier(0);          // keep wave 2 ahead of the lookup below

  // 2a. Cell-step lookups (wave 3): lane (k, jl) of the cell lanes takes arcs jl + AL * i.
  ArcBwd arc0[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) arc0[i] = arc_from_input(a, ain[i], t, load);
  // Softmax normaliser and arg-max slew over the condition's arcs (all chunks of 4): the
  // lane's own arcs first, then across the condition's arc lanes.
  float xmax, z, smax;
  int jstar;
  if constexpr (NA == 1) {
    xmax = arc_reduce<kMax, AL>(arc0[0].valid ? arc0[0].xg : -kInf);
    z = arc_reduce<kSum, AL>(arc0[0].valid ? fexp((arc0[0].xg - xmax) * a.inv_gamma) : 0.f);
    smax = arc0[0].valid ? arc0[0].s : -kInf;
    jstar = arc0[0].valid ? jl : STA_MAX_FANIN;
  } else {
    xmax = -kInf;
    z = 0.f;
    smax = -kInf;
    jstar = STA_MAX_FANIN;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      xmax = fmaxf(xmax, arc0[i].valid ? arc0[i].xg : -kInf);
      const bool take = arc0[i].valid && (jstar == STA_MAX_FANIN || arc0[i].s > smax);
      smax = take ? arc0[i].s : smax;
      jstar = take ? jl + AL * i : jstar;
    }
    xmax = arc_reduce<kMax, AL>(xmax);
#pragma unroll
    for (int i = 0; i < NA; ++i) z += arc0[i].valid ? fexp((arc0[i].xg - xmax) * a.inv_gamma) : 0.f;
    z = arc_reduce<kSum, AL>(z);
  }
  arc_argmax<AL>(smax, jstar);
  for (int j0 = kArcLanes; j0 < sl.F; j0 += kArcLanes) {    // cells wider than 4 inputs
    ArcBwd v[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      v[i].valid = false;
      if (cell_lane) v[i] = arc_backward(a, sl, kc, j0 + jl + AL * i, m, t, load);
    }
    float cm = -kInf, cz = 0.f, s2 = -kInf;
    int j2 = STA_MAX_FANIN;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      cm = fmaxf(cm, v[i].valid ? v[i].xg : -kInf);
      const bool take = v[i].valid && (j2 == STA_MAX_FANIN || v[i].s > s2);
      s2 = take ? v[i].s : s2;
      j2 = take ? j0 + jl + AL * i : j2;
    }
    cm = arc_reduce<kMax, AL>(cm);
#pragma unroll
    for (int i = 0; i < NA; ++i) cz += v[i].valid ? fexp((v[i].xg - cm) * a.inv_gamma) : 0.f;
    cz = arc_reduce<kSum, AL>(cz);
    lse_merge(xmax, z, cm, cz, a.inv_gamma);
    arc_argmax<AL>(s2, j2);
    if (s2 > smax) {
      smax = s2;
      jstar = j2;
    }
  }

  // 1. Net step.  Sinks beyond the two a lane holds (nets over 512 sinks) are recomputed in
  //    phase 3.
  float acc[N_ACC] = {-kInf, -kInf, kInf, kInf, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  SinkKeep keep0{0.f, 0.f, 0.f, 0}, keep1{0.f, 0.f, 0.f, 0};
  if (has0) keep0 = sink_step<kGrad>(a, in0, at_d, sl_d, xd, yd, acc, true, s0);
  if (has1) keep1 = sink_step<kGrad>(a, in1, at_d, sl_d, xd, yd, acc, true, s0 + gstride);
  if (block) {
    for (int p = s0 + 2 * gstride; p < p1; p += gstride)
      sink_step<kGrad>(a, sink_load<kCanon, kGrad>(a, p, sk0 + p), at_d, sl_d, xd, yd, acc, true, p);
  }
  reduce_acc<G>(acc, block, sh);

  // 2b. Cell step: required times of the inputs and the adjoint split.
  const float rat_o = k == 0 ? acc[R_E0] : (k == 1 ? acc[R_E1] : (k == 2 ? acc[R_L0] : acc[R_L1]));
  const float abar = t ? acc[A_F] : acc[A_R];
  const float sbar = t ? acc[S_F] : acc[S_R];
  const float inv_z = frcp(z);
  float lb = 0.f;
  for (int j0 = 0; j0 < sl.F; j0 += kArcLanes) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      ArcBwd v = arc0[i];
      if (j0 > 0) {
        v.valid = false;
        if (cell_lane) v = arc_backward(a, sl, kc, j0 + jl + AL * i, m, t, load);
      }
      if (cell_lane && v.valid) {
        // RAT(input, k') = RAT(output, k) - arc delay.
        float* sw = reinterpret_cast<float*>(a.sink);
        *at32(sw, 4 * rat_at((uint32_t)v.slot) + (uint32_t)(2 * m + v.tp)) = rat_o - v.d;
        if (kGrad && m == 1) {
          const float dbar = fexp((v.xg - xmax) * a.inv_gamma) * inv_z * abar;   // softmax weight x adjoint
          const float s_j = (j0 + jl + AL * i) == jstar ? sbar : 0.f;
          const uint32_t aj = 4 * adj_at((uint32_t)v.slot);
          *at32(sw, aj + (uint32_t)v.tp) = dbar;
          *at32(sw, aj + 2u + (uint32_t)v.tp) = fmaf(dbar, v.ddx, s_j * v.dsx);
          lb = fmaf(dbar, v.ddy, fmaf(s_j, v.dsy, lb));
        }
      }
    }
  }

  // 3. Load adjoint of the root: arcs summed over the arc lanes of late rise + late fall
  //    (cell lanes 2 * AL and 3 * AL).
  float lbar = 0.f;
  if (kGrad) {
    lb = arc_reduce<kSum, AL>(lb);
    if (!block) {
      const int base = (threadIdx.x & 63) & ~(G - 1);
      lbar = __shfl(lb, base + 2 * AL) + __shfl(lb, base + 3 * AL);
    } else {
      if (threadIdx.x == 2 * AL) sh[0] = lb;
      if (threadIdx.x == 3 * AL) sh[1] = lb;
      __syncthreads();
      lbar = sh[0] + sh[1];
      __syncthreads();
    }
  }
  if (!gs.active) return;
  if (kGrad && (a.dx || a.dy) && !a.tree_adj) {
    const float cl = a.c * lbar;
    if (has0) {
      if (a.dx) *at32(a.dx, (uint32_t)keep0.q) = keep0.gx * (cl + keep0.rest);
      if (a.dy) *at32(a.dy, (uint32_t)keep0.q) = keep0.gy * (cl + keep0.rest);
    }
    if (has1) {
      if (a.dx) *at32(a.dx, (uint32_t)keep1.q) = keep1.gx * (cl + keep1.rest);
      if (a.dy) *at32(a.dy, (uint32_t)keep1.q) = keep1.gy * (cl + keep1.rest);
    }
    if (block) {
      for (int p = s0 + 2 * gstride; p < p1; p += gstride) {
        float scratch[N_ACC] = {};
        const SinkKeep kk =
            sink_step<kGrad>(a, sink_load<kCanon, kGrad>(a, p, sk0 + p), at_d, sl_d, xd, yd, scratch, false, p);
        if (a.dx) a.dx[kk.q] = kk.gx * (cl + kk.rest);
        if (a.dy) a.dy[kk.q] = kk.gy * (cl + kk.rest);
      }
    }
  }
  if (gl == 0) {
    const uint32_t q = (uint32_t)(kCanon ? p0 : ld(a.io_perm, (uint32_t)p0));
    if (a.at_out) store_stream(at32(a.at_out, q), at_d);
    if (a.slew_out) store_stream(at32(a.slew_out, q), sl_d);
    if (a.rat_out) store_stream(at32(a.rat_out, q), make_float4(acc[R_E0], acc[R_E1], acc[R_L0], acc[R_L1]));
    if (a.slack_out)
      store_stream(at32(a.slack_out, q),
                   make_float4(at_d.x - acc[R_E0], at_d.y - acc[R_E1], acc[R_L0] - at_d.z, acc[R_L1] - at_d.w));
    if (kGrad && a.tree_adj) {
      *at32(a.tree_adj, (uint32_t)p0) = make_float2(lbar, 0.f);
    } else if (kGrad) {
      const float cl = a.c * lbar;
      if (a.dx) *at32(a.dx, q) = -(acc[X_RS] + cl * acc[X_N]);
      if (a.dy) *at32(a.dy, q) = -(acc[Y_RS] + cl * acc[Y_N]);
    }
  }
}

// One level of backward propagation: heavy nets first (one workgroup each), then waves of
// 4-, 8-, 16-, 32- and 64-lane groups.  The level's ranges (see level_slot) and the pointers of
// the first loads come first, as scalar parameters preloaded into scalar registers (14
// dwords are); the ranges of the fourth and fifth classes (groups of 8 and 4 lanes only)
// come last.
template <int G0, bool kSnap, bool kCanon, bool kGrad>
__global__ __launch_bounds__(kBlock) void k_bwd_level(int nh, int h0, int e0, int e1, int e2, int e3, int w1, int w2,
                                                      int w3, int snap_state, const int* __restrict__ net_off,
                                                      const float4* __restrict__ rec, BwdArgs a0, Slots sl, int e4,
                                                      int w4, int e5, int w5) {
  __shared__ float sh[kWavesPerBlock * N_ACC];
  BwdArgs a = a0;
  a.net_off = net_off;
  const SnapBlock sb = snap_block<kSnap>();
  a.rec = snap_bytes<kSnap>(rec, (size_t)snap_state, sb.s);
  a.wire = snap_bytes<kSnap>(a.wire, (size_t)snap_state, sb.s);
  a.load = snap_bytes<kSnap>(a.load, (size_t)snap_state, sb.s);
  a.sink = snap_bytes<kSnap>(a.sink, a.snap.work, sb.s);
  a.x = snap_elems<kSnap>(a.x, a.snap.pins, sb.s);
  a.y = snap_elems<kSnap>(a.y, a.snap.pins, sb.s);
  a.at_out = snap_elems<kSnap>(a.at_out, a.snap.pins, sb.s);
  a.slew_out = snap_elems<kSnap>(a.slew_out, a.snap.pins, sb.s);
  a.rat_out = snap_elems<kSnap>(a.rat_out, a.snap.pins, sb.s);
  a.slack_out = snap_elems<kSnap>(a.slack_out, a.snap.pins, sb.s);
  a.dx = snap_elems<kSnap>(a.dx, a.snap.pins, sb.s);
  a.dy = snap_elems<kSnap>(a.dy, a.snap.pins, sb.s);
  a.tree_adj = snap_bytes<kSnap>(a.tree_adj, a.snap.work, sb.s);
  GroupSlot gs;
  if (!level_slot<G0>(sb.x, nh, h0, e0, e1, e2, e3, e4, e5, w1, w2, w3, w4, w5, gs)) return;
  if (gs.block || gs.G == 64) {
    bwd_net<64, kCanon, kGrad>(a, sl, gs, sh);
  } else if (gs.G == 32) {
    bwd_net<32, kCanon, kGrad>(a, sl, gs, sh);
  } else if (G0 >= 4 || gs.G == 16) {
    bwd_net<16, kCanon, kGrad>(a, sl, gs, sh);
  } else if (G0 == 3 || gs.G == 8) {
    if constexpr (G0 <= 3) bwd_net<8, kCanon, kGrad>(a, sl, gs, sh);
  } else {
    if constexpr (G0 == 2) bwd_net<4, kCanon, kGrad>(a, sl, gs, sh);
  }
}

// One backward level's launch, with the kernel compiled for its smallest group, snapshot
// count, pin order and gradient flag.
struct BwdLaunch {
  int nh, h0, e0, e1, e2, e3, e4, e5, w1, w2, w3, w4, w5, ss;
  const int* net_off;
  const float4* rec;
  BwdArgs ba;
  Slots sl;
};

template <int G0, bool kSnap, bool kCanon, bool kGrad>
void bwd_launch(dim3 grid, hipStream_t s, const BwdLaunch& L) {
  k_bwd_level<G0, kSnap, kCanon, kGrad><<<grid, kBlock, 0, s>>>(L.nh, L.h0, L.e0, L.e1, L.e2, L.e3, L.w1, L.w2, L.w3,
                                                                  L.ss, L.net_off, L.rec, L.ba, L.sl, L.e4, L.w4, L.e5,
                                                                  L.w5);
}

template <int G0, bool kSnap>
void bwd_launch(dim3 grid, hipStream_t s, const BwdLaunch& L, bool canon, bool grad) {
  if (canon)
    grad ? bwd_launch<G0, kSnap, true, true>(grid, s, L) : bwd_launch<G0, kSnap, true, false>(grid, s, L);
  else
    grad ? bwd_launch<G0, kSnap, false, true>(grid, s, L) : bwd_launch<G0, kSnap, false, false>(grid, s, L);
}

Slots level_slots(const sta_graph* g, int l) {
  Slots sl{0, 1, 0, 0};
  if (l >= 1) {
    sl.base = g->ell_base[l];
    sl.F = g->ell_slots[l];
    sl.c0 = g->level_off[l] - g->N0;
    sl.nc = g->level_off[l + 1] - g->level_off[l];
  }
  return sl;
}

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
  // Snapshot offsets of the state reach the level kernels as 32-bit scalars.
  if (!g->snap_inner && g->n_snap > 1 && g->state.total > (size_t)INT32_MAX)
    return fail(STA_E_INVALID, "forward state of one snapshot exceeds 2 GiB; sweep fewer pins per snapshot");
  // Snapshot-inner arrays are addressed through 32-bit byte offsets over all snapshots.
  if (g->snap_inner) {
    const uint64_t S = (uint64_t)g->n_snap, lim = 1ull << 32;
    if (32ull * (uint64_t)g->P * S >= lim || 16ull * 4ull * (uint64_t)std::max(1, g->n_rec) * S >= lim ||
        40ull * (uint64_t)std::max(1, g->n_ep_blocks) * S >= lim)
      return fail(STA_E_INVALID, "with STA_SNAP_INNER an array of all snapshots reaches 4 GiB; sweep fewer");
  }
  return STA_OK;
}

// Launch timing while profiling is on (sta_profile_enable).  Consecutive launches of one
// kind form a run bracketed by one event pair, so that no event sits between two dependent
// launches of a level loop: the per-launch average is then the kernels' own back-to-back
// duration.  A run ends when a launch of another kind starts or the call ends (end_run).
hipEvent_t take_event(sta_graph* g) {
  if (!g->event_pool.empty()) {
    hipEvent_t e = g->event_pool.back();
    g->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

void end_run(sta_graph* g, hipStream_t s) {
  if (g->run_kind < 0) return;
  hipEvent_t stop = take_event(g);
  if (stop && g->run_start) {
    (void)hipEventRecord(stop, s);
    g->timed.push_back({g->run_kind, g->run_count, g->run_start, stop});
  }
  g->run_kind = -1;
  g->run_count = 0;
  g->run_start = nullptr;
}

struct LaunchTimer {
  LaunchTimer(sta_graph* g, hipStream_t s, int kind) {
    if (!g->profiling) return;
    if (g->run_kind != kind) {
      end_run(g, s);
      g->run_kind = kind;
      g->run_start = take_event(g);
      if (g->run_start) (void)hipEventRecord(g->run_start, s);
    }
    ++g->run_count;
  }
};

// Component i of v set to x (i known only at run time).
__device__ __forceinline__ void set_comp(float4& v, int i, float x) {
  v.x = i == 0 ? x : v.x;
  v.y = i == 1 ? x : v.y;
  v.z = i == 2 ? x : v.z;
  v.w = i == 3 ? x : v.w;
}

// ============================================================================ CTE levels
// The level kernels in the CTE scheme (Alg. 2; Sec. 3.1.2 applies the RC stage's mappings to
// arrival propagation and slack computation): a workgroup takes kCteItems consecutive items
// of a level, one per thread of its first kCteItems (cells in the forward, nets in the
// backward), a work-efficient scan of their work numbers a pool of tasks (a cell's inputs, a
// net's sinks), all 256 threads take tasks with a stride of 256, find the owning item with
// cte_owner and leave their results in LDS, and each item's own thread merges its tasks in
// task order (loops unrolled so that an item of many tasks reads its LDS entries in batches).  One snapshot, star nets, no
// checkpointing (a net's record slot is the net, a sink's workspace slot its pin).  A
// workgroup takes kCteItems items rather than one per thread: a level holds a few thousand
// cells, and 256 per workgroup would leave most of the chip idle.
constexpr int kCteLevelTasks = 512;   // tasks staged in LDS at a time
constexpr int kCteItems = 16;         // items per workgroup

// Valid inputs of cell kc: its input slots hold them first, then empty slots (source -1).
// The slot entries are loaded together (a cell has at most STA_MAX_FANIN inputs).
__device__ __forceinline__ int cell_fanin(const int4* __restrict__ ell, const Slots& sl, int kc) {
  int f = 0;
#pragma unroll
  for (int j = 0; j < STA_MAX_FANIN; ++j)
    f += j < sl.F && ell[sl.base + (size_t)min(j, sl.F - 1) * sl.nc + kc].x >= 0 ? 1 : 0;
  return f;
}

// Forward level: a task is one input j of a cell, looked up for the four conditions; the
// cell's thread merges its inputs in order (max / min arrival, worst slew, and the log-sum-exp
// of the late smoothed candidates, Eq. 4) and writes the cell's output record.
__global__ __launch_bounds__(kBlock) void k_fwd_level_cte(int nc, int n0, int base, int F,
                                                          const int4* __restrict__ ell,
                                                          const float* __restrict__ loads,
                                                          float4* __restrict__ rec, FwdArgs a) {
  __shared__ int pre[kBlock];
  __shared__ int total_sh;
  __shared__ float load_sh[kBlock];
  __shared__ float part[10][kCteLevelTasks];   // per task: arrival and slew of conditions 0..3,
                                               // then the late smoothed candidates
  const Slots sl{base, F, 0, nc};
  const int t = threadIdx.x;
  const int kc = (int)blockIdx.x * kCteItems + t;
  const bool own = t < kCteItems && kc < nc;
  const int n = n0 + kc;
  int work = 0;
  if (own) {
    work = cell_fanin(ell, sl, kc);
    load_sh[t] = loads[n];
  }
  const int total = cte_scan<kCteItems>(work, pre, &total_sh);
  const int my0 = own ? pre[t] : 0, my1 = own ? (t + 1 < kCteItems ? pre[t + 1] : total) : 0;
  float bat[4], bsl[4], lm[2] = {-kInf, -kInf}, ls[2] = {0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 4; ++k) bat[k] = bsl[k] = k >= 2 ? -kInf : kInf;
  for (int c0 = 0; c0 < total; c0 += kCteLevelTasks) {
    const int c1 = min(total, c0 + kCteLevelTasks);
    for (int task = c0 + t; task < c1; task += kBlock) {
      const int o = cte_owner<kCteItems>(pre, task);
      const int ko = (int)blockIdx.x * kCteItems + o, j = task - pre[o];
      const int4 e = ell[sl.base + (size_t)j * sl.nc + ko];
      const float load = load_sh[o];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int m = k >> 1, tr = k & 1;
        const ArcIn in = arc_input_entry(e, true, rec, a.wire, m, tr);
        const LutVal v = lut_eval<false>(a.grid, a.coef, a.keys, in.arc, tr, in.slew, load);
        part[k][task - c0] = in.at + v.d;
        part[4 + k][task - c0] = v.s;
        if (m) part[8 + tr][task - c0] = in.atg + v.d;
      }
    }
    __syncthreads();
#pragma unroll 8
    for (int i = max(my0, c0); i < min(my1, c1); ++i) {
      const int q = i - c0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k >= 2) {
          bat[k] = fmaxf(bat[k], part[k][q]);
          bsl[k] = fmaxf(bsl[k], part[4 + k][q]);
        } else {
          bat[k] = fminf(bat[k], part[k][q]);
          bsl[k] = fminf(bsl[k], part[4 + k][q]);
        }
      }
      if (a.smooth) {
        lse_merge(lm[0], ls[0], part[8][q], 1.f, a.inv_gamma);
        lse_merge(lm[1], ls[1], part[9][q], 1.f, a.inv_gamma);
      }
    }
    __syncthreads();
  }
  if (!own) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int m = k >> 1, tr = k & 1;
    const float ag = m ? (a.smooth ? fmaf(a.gamma, flog(ls[tr]), lm[tr]) : __builtin_nanf("")) : 0.f;
    rec[kRecChunks * (size_t)n + k] = make_float4(bat[k], bsl[k], ag, 0.f);
  }
}

// Backward level over nets [lo, hi): three task pools in turn.  The net step pools the
// sinks (per-pin outputs, and each sink's share of the driver's reductions, merged by the
// net's thread in sink order); the cell step pools the inputs of the driving cell (the late
// lookups, whose softmax normaliser and arg-max slew the net's thread takes in input order,
// then the four conditions' required times and adjoints written to the input pins and the
// load adjoint summed in input order); the Elmore adjoint pools the sinks again.
template <bool kCanon, bool kGrad>
__global__ __launch_bounds__(kBlock) void k_bwd_level_cte(int lo, int hi, Slots sl, BwdArgs a) {
  __shared__ int pre[kBlock];
  __shared__ int first[kBlock];
  __shared__ int total_sh;
  __shared__ float4 at_sh[kBlock], sl_sh[kBlock];
  __shared__ float xd_sh[kBlock], yd_sh[kBlock], load_sh[kBlock];
  __shared__ float ro_sh[4][kBlock];            // the net's required times by condition
  __shared__ float gs_sh[8][kBlock];            // abar[2], sbar[2], xmax[2], 1/z[2]
  __shared__ int js_sh[2][kBlock];              // arg-max slew input per transition
  __shared__ float cl_sh[kBlock];               // c * load adjoint
  __shared__ float part[N_ACC][kCteLevelTasks];
  const int t = threadIdx.x;
  const int n = lo + (int)blockIdx.x * kCteItems + t;
  const bool own = t < kCteItems && n < hi;
  const bool cell = own && n >= a.N0 && sl.F > 0;
  const int kc = n - a.N0 - sl.c0;
  int p0 = 0, sinks = 0;
  float4 at_d = make_float4(0.f, 0.f, 0.f, 0.f), sl_d = at_d;
  float xd = 0.f, yd = 0.f;
  if (own) {
    p0 = a.net_off[n];
    sinks = a.net_off[n + 1] - p0 - 1;
    float4 c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = a.rec[kRecChunks * (size_t)n + k];
    at_d = make_float4(c[0].x, c[1].x, c[2].x, c[3].x);
    sl_d = make_float4(c[0].y, c[1].y, c[2].y, c[3].y);
    if (kGrad) {
      const int q = kCanon ? p0 : a.io_perm[p0];
      xd = a.x[q];
      yd = a.y[q];
    }
    if (cell) load_sh[t] = a.load[n];
  }
  first[t] = p0 + 1;
  at_sh[t] = at_d;
  sl_sh[t] = sl_d;
  xd_sh[t] = xd;
  yd_sh[t] = yd;

  // Net step over the sinks.
  float acc[N_ACC] = {-kInf, -kInf, kInf, kInf, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int total = cte_scan<kCteItems>(sinks, pre, &total_sh);
  int my0 = own ? pre[t] : 0, my1 = own ? (t + 1 < kCteItems ? pre[t + 1] : total) : 0;
  for (int c0 = 0; c0 < total; c0 += kCteLevelTasks) {
    const int c1 = min(total, c0 + kCteLevelTasks);
    for (int task = c0 + t; task < c1; task += kBlock) {
      const int o = cte_owner<kCteItems>(pre, task);
      const int p = first[o] + (task - pre[o]);
      float v[N_ACC] = {-kInf, -kInf, kInf, kInf, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      (void)sink_step<kGrad>(a, sink_load<kCanon, kGrad>(a, p, p), at_sh[o], sl_sh[o], xd_sh[o], yd_sh[o], v, true, p);
#pragma unroll
      for (int i = 0; i < N_ACC; ++i) part[i][task - c0] = v[i];
    }
    __syncthreads();
#pragma unroll 8
    for (int i = max(my0, c0); i < min(my1, c1); ++i) {
      const int q = i - c0;
      acc[R_E0] = fmaxf(acc[R_E0], part[R_E0][q]);
      acc[R_E1] = fmaxf(acc[R_E1], part[R_E1][q]);
      acc[R_L0] = fminf(acc[R_L0], part[R_L0][q]);
      acc[R_L1] = fminf(acc[R_L1], part[R_L1][q]);
#pragma unroll
      for (int k = A_R; k < N_ACC; ++k) acc[k] += part[k][q];
    }
    __syncthreads();
  }
  ro_sh[0][t] = acc[R_E0];
  ro_sh[1][t] = acc[R_E1];
  ro_sh[2][t] = acc[R_L0];
  ro_sh[3][t] = acc[R_L1];

  // Cell step over the driving cell's inputs.
  total = cte_scan<kCteItems>(cell ? cell_fanin(a.ell, sl, kc) : 0, pre, &total_sh);
  my0 = own ? pre[t] : 0;
  my1 = own ? (t + 1 < kCteItems ? pre[t + 1] : total) : 0;
  float lbar = 0.f;
  if (kGrad) {
    // Late lookups: softmax normaliser and arg-max slew per output transition.
    float xmax[2] = {-kInf, -kInf}, z[2] = {0.f, 0.f}, smax[2] = {-kInf, -kInf};
    int jstar[2] = {STA_MAX_FANIN, STA_MAX_FANIN};
    for (int c0 = 0; c0 < total; c0 += kCteLevelTasks) {
      const int c1 = min(total, c0 + kCteLevelTasks);
      for (int task = c0 + t; task < c1; task += kBlock) {
        const int o = cte_owner<kCteItems>(pre, task);
        const int ko = lo + (int)blockIdx.x * kCteItems + o - a.N0 - sl.c0, j = task - pre[o];
        const int4 e = a.ell[sl.base + (size_t)j * sl.nc + ko];
#pragma unroll
        for (int tr = 0; tr < 2; ++tr) {
          const ArcIn in = arc_input_entry(e, true, a.rec, a.wire, 1, tr);
          const LutVal v = lut_eval<false>(a.grid, a.coef, a.keys, in.arc, tr, in.slew, load_sh[o]);
          part[2 * tr][task - c0] = in.atg + v.d;
          part[2 * tr + 1][task - c0] = v.s;
        }
      }
      __syncthreads();
  #pragma unroll 8
    for (int i = max(my0, c0); i < min(my1, c1); ++i) {
        const int q = i - c0, j = i - my0;
#pragma unroll
        for (int tr = 0; tr < 2; ++tr) {
          lse_merge(xmax[tr], z[tr], part[2 * tr][q], 1.f, a.inv_gamma);
          if (jstar[tr] == STA_MAX_FANIN || part[2 * tr + 1][q] > smax[tr]) {
            smax[tr] = part[2 * tr + 1][q];
            jstar[tr] = j;
          }
        }
      }
      __syncthreads();
    }
    gs_sh[0][t] = acc[A_R];
    gs_sh[1][t] = acc[A_F];
    gs_sh[2][t] = acc[S_R];
    gs_sh[3][t] = acc[S_F];
    gs_sh[4][t] = xmax[0];
    gs_sh[5][t] = xmax[1];
    gs_sh[6][t] = frcp(z[0]);
    gs_sh[7][t] = frcp(z[1]);
    js_sh[0][t] = jstar[0];
    js_sh[1][t] = jstar[1];
  }
  __syncthreads();
  for (int c0 = 0; c0 < total; c0 += kCteLevelTasks) {
    const int c1 = min(total, c0 + kCteLevelTasks);
    for (int task = c0 + t; task < c1; task += kBlock) {
      const int o = cte_owner<kCteItems>(pre, task);
      const int ko = lo + (int)blockIdx.x * kCteItems + o - a.N0 - sl.c0, j = task - pre[o];
      const int4 e = a.ell[sl.base + (size_t)j * sl.nc + ko];
      float4 rat_in = make_float4(0.f, 0.f, 0.f, 0.f), adj_in = rat_in;
      float lb = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int m = k >> 1, tr = k & 1;
        const ArcIn in = arc_input_entry(e, true, a.rec, a.wire, m, tr);
        const LutVal v = lut_eval<kGrad>(a.grid, a.coef, a.keys, in.arc, tr, in.slew, load_sh[o]);
        set_comp(rat_in, 2 * m + in.tp, ro_sh[k][o] - v.d);
        if (kGrad && m == 1) {
          const float dbar = fexp((in.atg + v.d - gs_sh[4 + tr][o]) * a.inv_gamma) * gs_sh[6 + tr][o] * gs_sh[tr][o];
          const float s_j = j == js_sh[tr][o] ? gs_sh[2 + tr][o] : 0.f;
          set_comp(adj_in, in.tp, dbar);
          set_comp(adj_in, 2 + in.tp, fmaf(dbar, v.ddx, s_j * v.dsx));
          lb = fmaf(dbar, v.ddy, fmaf(s_j, v.dsy, lb));
        }
      }
      a.sink[rat_at(e.w)] = rat_in;
      if (kGrad) a.sink[adj_at(e.w)] = adj_in;
      part[0][task - c0] = lb;
    }
    __syncthreads();
    if (kGrad) {
#pragma unroll 8
      for (int i = max(my0, c0); i < min(my1, c1); ++i) lbar += part[0][i - c0];
    }
    __syncthreads();
  }

  // The driver's outputs.
  const float cl = a.c * lbar;
  if (own) {
    const uint32_t o0 = (uint32_t)(kCanon ? p0 : a.io_perm[p0]);
    if (a.at_out) store_stream(at32(a.at_out, o0), at_d);
    if (a.slew_out) store_stream(at32(a.slew_out, o0), sl_d);
    if (a.rat_out) store_stream(at32(a.rat_out, o0), make_float4(acc[R_E0], acc[R_E1], acc[R_L0], acc[R_L1]));
    if (a.slack_out)
      store_stream(at32(a.slack_out, o0),
                   make_float4(at_d.x - acc[R_E0], at_d.y - acc[R_E1], acc[R_L0] - at_d.z, acc[R_L1] - at_d.w));
    if (kGrad) {
      if (a.dx) a.dx[o0] = -(acc[X_RS] + cl * acc[X_N]);
      if (a.dy) a.dy[o0] = -(acc[Y_RS] + cl * acc[Y_N]);
    }
  }
  if (!kGrad || !(a.dx || a.dy)) return;

  // Elmore adjoint over the sinks.
  cl_sh[t] = cl;
  total = cte_scan<kCteItems>(sinks, pre, &total_sh);
  for (int task = t; task < total; task += kBlock) {
    const int o = cte_owner<kCteItems>(pre, task);
    const int p = first[o] + (task - pre[o]);
    float scratch[N_ACC] = {};
    const SinkKeep k =
        sink_step<kGrad>(a, sink_load<kCanon, kGrad>(a, p, p), at_sh[o], sl_sh[o], xd_sh[o], yd_sh[o], scratch, false, p);
    if (a.dx) a.dx[k.q] = k.gx * (cl_sh[o] + k.rest);
    if (a.dy) a.dy[k.q] = k.gy * (cl_sh[o] + k.rest);
  }
}

// ============================================================================ snapshot lanes
// The snapshot-inner layout (sta_set_snapshot_layout(g, STA_SNAP_INNER)): every per-call and
// state array holds the S snapshots of an item side by side, element (i, s) at i*S + s (an
// arrival record's chunk k of net slot r at (4r + k)*S + s; a sink's required times at
// 2p*S + s and its adjoint at (2p + 1)*S + s).  The lanes of a wave then take snapshots: a
// wave serves one net or cell for 64 snapshots (or 64 >> sl2 items of 1 << sl2 lanes each
// when S <= 32), so the topology and tables it reads are the same for every lane of an item,
// and every state load or store moves one contiguous run per item.  Sums over a net's sinks
// and merges over a cell's arcs run inside each lane, in index order; nets of more than
// kSiHeavy sinks take a whole workgroup (kSiRcBlock threads in the RC stage; in the
// backward the schedule's lane_block, 256, 512 or 1024) whose threads split the sinks and
// meet in LDS in thread order.  The light nets' waves come in workgroups of the same size:
// smaller workgroups let a CU start new waves sooner after its slowest one, larger ones give
// a heavy net more threads per snapshot.
constexpr int kSiRcBlock = 256;

struct SiLane {
  int item;   // item of the lane counted from the launch's first (or, in a heavy workgroup,
              // the thread's position among the threads of its snapshot)
  int s;      // snapshot
  bool on;    // s < S
};

__device__ __forceinline__ SiLane si_lane(int sl2, int S, int wave) {
  const int lane = threadIdx.x & 63;
  SiLane r;
  r.item = (wave << (6 - sl2)) + (lane >> sl2);
  r.s = (lane & ((1 << sl2) - 1)) + 64 * (int)blockIdx.y;
  r.on = r.s < S;
  return r;
}

__device__ __forceinline__ uint32_t si_at(int i, uint32_t S, int s) { return (uint32_t)i * S + (uint32_t)s; }

// Record r in the snapshot-lane kernels: three planes in its four 16-byte rows of S elements,
// row 0 the arrival times of the four conditions (early rise, early fall, late rise, late
// fall), row 1 their slews, the first half of row 2 (float2 element 2 (4 r + 2) S + s) the
// late rise and fall smoothed arrivals; row 3 is unused.  A record of a snapshot moves 40
// bytes, and a reader takes only the planes it needs.
__device__ __forceinline__ float4 rec_at_si(const float4* __restrict__ rec, int r, uint32_t S, int s) {
  return ld(rec, si_at(kRecChunks * r, S, s));
}
__device__ __forceinline__ float4 rec_sl_si(const float4* __restrict__ rec, int r, uint32_t S, int s) {
  return ld(rec, si_at(kRecChunks * r + 1, S, s));
}
__device__ __forceinline__ uint32_t rec_ag_at(int r, uint32_t S, int s) {
  return 2u * (uint32_t)(kRecChunks * r + 2) * S + (uint32_t)s;
}
__device__ __forceinline__ float2 rec_ag_si(const float4* __restrict__ rec, int r, uint32_t S, int s) {
  return ld(reinterpret_cast<const float2*>(rec), rec_ag_at(r, S, s));
}
__device__ __forceinline__ void rec_store_si(float4* __restrict__ rec, int r, uint32_t S, int s, const float4& at,
                                             const float4& sl, const float2& ag) {
  *at32(rec, si_at(kRecChunks * r, S, s)) = at;
  *at32(rec, si_at(kRecChunks * r + 1, S, s)) = sl;
  *at32(reinterpret_cast<float2*>(rec), rec_ag_at(r, S, s)) = ag;
}
// Value of mode m (0 early, 1 late) for the input transition that drives output transition t
// through an arc of unateness `same`, from a plane of the four conditions.
__device__ __forceinline__ float plane_pick(const float4& v, int m, bool same, int t) {
  const bool rise = same == (t == 0);
  return m ? (rise ? v.z : v.w) : (rise ? v.x : v.y);
}

// Workgroups of heavy nets: each takes 1 << hl2 snapshots, so that (workgroup size) >> hl2
// threads split the sinks of each snapshot; hl2 = sl2 for nets of up to kSiHuge sinks (a
// workgroup per net and block of up to 64 snapshots) and min(sl2, 3) beyond (a workgroup per
// 8 snapshots).
// Workgroup hb of a class serves net hb / nch of the class and snapshot chunk hb % nch.
__device__ __forceinline__ int chunks_of(int S, int hl2) { return (S + (1 << hl2) - 1) >> hl2; }

// Snapshots a backward heavy workgroup of kb threads takes (log2): each snapshot keeps at least
// 8 threads for nets of up to kSiHuge sinks (64 snapshots at kb = 512) and at least 64 beyond
// (8 snapshots).  Wider splits were measured slower: their extra workgroups take wave slots
// the level's other nets need in the same round.
__host__ __device__ constexpr int si_log2(int v) { return v <= 1 ? 0 : 1 + si_log2(v >> 1); }
constexpr int kSiHeavyTpsL2 = 3;     // log2 of the threads per snapshot: nets of up to kSiHuge sinks
constexpr int kSiHugeTpsL2 = 6;      // and beyond
__host__ __device__ inline int si_bwd_hl2(int sl2, int kb, bool huge) {
  const int l2 = si_log2(kb) - (huge ? kSiHugeTpsL2 : kSiHeavyTpsL2);
  return sl2 < l2 ? sl2 : l2;
}
constexpr int kSiCacheHeavy = 16;    // sinks a heavy workgroup's thread keeps on chip (all of a
                                     // net of up to 128 sinks at 8 threads per snapshot)
constexpr int kSiRows = 29;          // LDS rows of kB floats in the backward: N_ACC reductions
                                     // and lbar, then the sink cache (kSiHeavy rows outside
                                     // heavy workgroups)
__device__ __forceinline__ SiLane si_heavy_lane(int hl2, int S, int chunk) {
  const int lane = threadIdx.x & 63, w = (int)(threadIdx.x >> 6);
  SiLane r;
  r.item = (w << (6 - hl2)) + (lane >> hl2);
  r.s = chunk * (1 << hl2) + (lane & ((1 << hl2) - 1));
  r.on = r.s < S;
  return r;
}

// ---------------------------------------------------------------- RC net delay, snapshot lanes
struct RcSiArgs {
  const int* __restrict__ net_off;
  const float* __restrict__ pin_cap;
  const float* __restrict__ x;          // [pins][S], canonical order or through io_perm
  const float* __restrict__ y;
  const int* __restrict__ io_perm;
  const int* __restrict__ heavy;        // nets of kSiHeavy+1..kSiHuge sinks
  const int* __restrict__ huge;         // nets of more than kSiHuge sinks
  float2* __restrict__ wire;            // [P][S]
  float* __restrict__ load;             // [N][S]
  float4* __restrict__ rec;             // [4 N][S]
  int N, N0, S, sl2, n_heavy, n_huge;
  int max_sinks;                        // nets with more sinks are a heavy workgroup's
  float r, c, pi_at, pi_slew;
};

// Sink p of a star net in snapshot s: wire delay and impulse (Eq. 2-3) and its share of the
// root load (Eq. 1), as rc_sink computes them.
__device__ __forceinline__ float rc_sink_si(const RcSiArgs& a, int p, int s, float xd, float yd) {
  const uint32_t S = (uint32_t)a.S;
  const int q = a.io_perm ? ld(a.io_perm, (uint32_t)p) : p;
  const float cp = ld(a.pin_cap, (uint32_t)p);
  const float len = fabsf(ld(a.x, si_at(q, S, s)) - xd) + fabsf(ld(a.y, si_at(q, S, s)) - yd);
  const float res = a.r * len;
  const float cw = a.c * len;
  const float cap = fmaf(0.5f, cw, cp);
  const float dly = 1e-3f * res * cap;
  const float arg = 2.0f * (1e-3f * res * cap) * dly - dly * dly;
  const float imp = arg > 0.f ? sqrtf(arg) : 0.f;
  *at32(a.wire, si_at(p, S, s)) = make_float2(dly, imp);
  return cp + cw;
}

__device__ __forceinline__ void rc_root_si(const RcSiArgs& a, int n, int p0, int s, float sum) {
  const uint32_t S = (uint32_t)a.S;
  *at32(a.load, si_at(n, S, s)) = ld(a.pin_cap, (uint32_t)p0) + sum;
  *at32(a.wire, si_at(p0, S, s)) = make_float2(0.f, 0.f);
  if (n < a.N0)
    rec_store_si(a.rec, n, S, s, make_float4(a.pi_at, a.pi_at, a.pi_at, a.pi_at),
                 make_float4(a.pi_slew, a.pi_slew, a.pi_slew, a.pi_slew), make_float2(a.pi_at, a.pi_at));
}

__device__ __forceinline__ void driver_xy_si(const float* __restrict__ x, const float* __restrict__ y,
                                             const int* __restrict__ io, int p0, uint32_t S, int s, float& xd,
                                             float& yd) {
  const int q = io ? ld(io, (uint32_t)p0) : p0;
  xd = ld(x, si_at(q, S, s));
  yd = ld(y, si_at(q, S, s));
}

// The RC of heavy net n for the snapshots of one workgroup (threads split the sinks).
__device__ __forceinline__ void rc_heavy_si(const RcSiArgs& a, int n, const SiLane& ln, int hl2, float* sh) {
  const uint32_t S = (uint32_t)a.S;
  const int lanes = 1 << hl2;
  const int p0 = ld(a.net_off, (uint32_t)n), p1 = ld(a.net_off, (uint32_t)n + 1u);
  float sum = 0.f;
  if (ln.on) {
    float xd, yd;
    driver_xy_si(a.x, a.y, a.io_perm, p0, S, ln.s, xd, yd);
    for (int p = p0 + 1 + ln.item; p < p1; p += kSiRcBlock / lanes) sum += rc_sink_si(a, p, ln.s, xd, yd);
  }
  sh[threadIdx.x] = sum;
  __syncthreads();
  if ((int)threadIdx.x < lanes && ln.on) {
    float tot = 0.f;
    for (int t = (int)threadIdx.x; t < kSiRcBlock; t += lanes) tot += sh[t];
    rc_root_si(a, n, p0, ln.s, tot);
  }
}

// RC of every net: huge and heavy nets first (workgroups per net and snapshot chunk), then
// (64 >> sl2) nets per wave.
__global__ __launch_bounds__(kSiRcBlock) void k_rc_si(RcSiArgs a) {
  __shared__ float sh[kSiRcBlock];
  const int w = (int)(threadIdx.x >> 6);
  const int b = (int)blockIdx.x;
  const int hl2u = min(a.sl2, 3), nchu = chunks_of(a.S, hl2u), nchh = chunks_of(a.S, a.sl2);
  const int nbu = a.n_huge * nchu, nbh = a.n_heavy * nchh;
  if (b < nbu + nbh) {
    if (blockIdx.y != 0) return;               // these workgroups cover their snapshots along x
    if (b < nbu)
      rc_heavy_si(a, ld(a.huge, (uint32_t)(b / nchu)), si_heavy_lane(hl2u, a.S, b % nchu), hl2u, sh);
    else
      rc_heavy_si(a, ld(a.heavy, (uint32_t)((b - nbu) / nchh)), si_heavy_lane(a.sl2, a.S, (b - nbu) % nchh), a.sl2,
                  sh);
    return;
  }
  const SiLane ln = si_lane(a.sl2, a.S, (b - nbu - nbh) * (kSiRcBlock / 64) + w);
  const int n = ln.item;
  if (n >= a.N || !ln.on) return;
  const int p0 = ld(a.net_off, (uint32_t)n), p1 = ld(a.net_off, (uint32_t)n + 1u);
  if (p1 - p0 - 1 > a.max_sinks) return;       // a heavy workgroup's net
  const uint32_t S = (uint32_t)a.S;
  float xd, yd;
  driver_xy_si(a.x, a.y, a.io_perm, p0, S, ln.s, xd, yd);
  float sum = 0.f;
  for (int p = p0 + 1; p < p1; ++p) sum += rc_sink_si(a, p, ln.s, xd, yd);
  rc_root_si(a, n, p0, ln.s, sum);
}

// ---------------------------------------------------------------- forward level, snapshot lanes
struct FwdSiArgs {
  const int4* __restrict__ ell;
  const float* __restrict__ load;
  const float2* __restrict__ wire;
  float4* __restrict__ rec;
  const float4* __restrict__ grid;
  const float4* __restrict__ coef;
  LutKeys keys;
  float gamma, inv_gamma;
  int smooth, S, sl2;
};

// Chunk of a source record in the input transition of output transition t (unateness
// `same`: positive unate keeps the transition) for mode m, from the two chunks of that mode.
__device__ __forceinline__ float4 pick_tr(bool same, int t, const float4& c_r, const float4& c_f) {
  return (same == (t == 0)) ? c_r : c_f;
}

// One forward level (Sec. 3.1.2): each lane takes one cell of one snapshot and merges its
// arcs in registers, condition by condition, as k_fwd_level_narrow with one lane per
// condition does: max / min arrival, worst slew, log-sum-exp of the late candidates (Eq. 4).
__global__ __launch_bounds__(kBlock) void k_fwd_level_si(int nc, int n0, int base, int F, FwdSiArgs a) {
  const SiLane ln = si_lane(a.sl2, a.S, (int)blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6));
  const int kc = ln.item;
  if (kc >= nc || !ln.on) return;
  const uint32_t S = (uint32_t)a.S;
  const int s = ln.s, n = n0 + kc;
  const float load = ld(a.load, si_at(n, S, s));
  float bat[4], bsl[4], lm[2] = {-kInf, -kInf}, ls[2] = {0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 4; ++k) bat[k] = bsl[k] = k >= 2 ? -kInf : kInf;
  for (int j0 = 0; j0 < F; j0 += kArcLanes) {
    int4 e[kArcLanes];
    bool valid[kArcLanes];
    float2 w[kArcLanes];
#pragma unroll
    for (int i = 0; i < kArcLanes; ++i) {
      const int j = j0 + i;
      e[i] = ld(a.ell, (uint32_t)(base + min(j, F - 1) * nc + kc));
      valid[i] = j < F && e[i].x >= 0;
    }
#pragma unroll
    for (int i = 0; i < kArcLanes; ++i) w[i] = ld(a.wire, si_at(e[i].y, S, s));
    float4 rat_[kArcLanes], rsl[kArcLanes];
    float2 rag[kArcLanes];
#pragma unroll
    for (int i = 0; i < kArcLanes; ++i) {
      const int src = max(e[i].x, 0);
      rat_[i] = rec_at_si(a.rec, src, S, s);
      rsl[i] = rec_sl_si(a.rec, src, S, s);
      rag[i] = rec_ag_si(a.rec, src, S, s);
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int k = 2 * m + t;
        const float neutral = m ? -kInf : kInf;
        float cm = neutral, sm = neutral, gm = -kInf, g[kArcLanes];
#pragma unroll
        for (int i = 0; i < kArcLanes; ++i) {
          const bool same = ell_positive(e[i]);
          const float sl_in = sink_slew(plane_pick(rsl[i], m, same, t), w[i].y);
          const LutVal v = lut_eval_si<false>(a.grid, a.coef, a.keys, ell_arc(e[i]), t, sl_in, load);
          const float cand = valid[i] ? (plane_pick(rat_[i], m, same, t) + w[i].x) + v.d : neutral;
          const float sv = valid[i] ? v.s : neutral;
          const float ag_in = (same == (t == 0)) ? rag[i].x : rag[i].y;
          g[i] = valid[i] ? (ag_in + w[i].x) + v.d : -kInf;
          if (m) {
            cm = fmaxf(cm, cand);
            sm = fmaxf(sm, sv);
            gm = fmaxf(gm, g[i]);
          } else {
            cm = fminf(cm, cand);
            sm = fminf(sm, sv);
          }
        }
        if (m) {
          bat[k] = fmaxf(bat[k], cm);
          bsl[k] = fmaxf(bsl[k], sm);
          if (a.smooth) {
            float gs = 0.f;
#pragma unroll
            for (int i = 0; i < kArcLanes; ++i) gs += valid[i] ? fexp((g[i] - gm) * a.inv_gamma) : 0.f;
            lse_merge(lm[t], ls[t], gm, gs, a.inv_gamma);
          }
        } else {
          bat[k] = fminf(bat[k], cm);
          bsl[k] = fminf(bsl[k], sm);
        }
      }
    }
  }
  const float2 ag = a.smooth ? make_float2(fmaf(a.gamma, flog(ls[0]), lm[0]), fmaf(a.gamma, flog(ls[1]), lm[1]))
                             : make_float2(__builtin_nanf(""), __builtin_nanf(""));
  rec_store_si(a.rec, n, S, s, make_float4(bat[0], bat[1], bat[2], bat[3]), make_float4(bsl[0], bsl[1], bsl[2], bsl[3]),
               ag);
}

// ---------------------------------------------------------------- endpoints, snapshot lanes
struct EpSiArgs {
  const int* __restrict__ ep_pin;
  const int* __restrict__ ep_net;
  const int* __restrict__ ep_design;
  const int* __restrict__ ep_design_off;
  const int* __restrict__ ep_blk_off;
  const float4* __restrict__ rec;
  const float2* __restrict__ wire;
  double* part;        // [blocks * 5][S]
  double* fin;         // [designs * 8][S]
  double* scalars;     // [S][designs][4] or NULL
  float4* sink;        // [2 P][S]
  float4* epv;         // [E][S]
  const double* scale_dev;
  int E, n_designs, S, sl2, seed_adj, smooth, wns_mode;
  float rat_late, hold, gamma, inv_gamma, scale;
};

__device__ __forceinline__ EpVals endpoint_values_si(const EpSiArgs& a, int i, int s) {
  const uint32_t S = (uint32_t)a.S;
  const int e = ld(a.ep_pin, (uint32_t)i), r = ld(a.ep_net, (uint32_t)i);
  const float4 at = rec_at_si(a.rec, r, S, s);    // late rise and fall in .z, .w
  const float2 ag = rec_ag_si(a.rec, r, S, s);
  const float dl = ld(a.wire, si_at(e, S, s)).x;
  EpVals v;
  v.worst = fminf(a.rat_late - (at.z + dl), a.rat_late - (at.w + dl));
  const float u0 = -(a.rat_late - (ag.x + dl));
  const float u1 = -(a.rat_late - (ag.y + dl));
  const float mx = fmaxf(u0, u1);
  const float e0 = expf((u0 - mx) * a.inv_gamma), e1 = expf((u1 - mx) * a.inv_gamma);
  const float z = e0 + e1;
  v.sg = -(mx + a.gamma * logf(z));
  v.w0 = e0 / z;
  v.w1 = e1 / z;
  return v;
}

// Merges (m2, s2) into the shifted sum of exponentials (m, s): sum exp((v - m) / gamma).
__device__ __forceinline__ void lse_merge_d(double& m, double& s, double m2, double s2, double g) {
  if (s2 <= 0.0) return;
  if (s <= 0.0) {
    m = m2;
    s = s2;
  } else if (m2 > m) {
    s = s * exp((m - m2) / g) + s2;
    m = m2;
  } else {
    s += s2 * exp((m2 - m) / g);
  }
}

// Per-block partials of each snapshot over the block's endpoints (the blocks of k_ep_partials),
// in float64: each thread sums its endpoints in order, then the threads of a snapshot meet in
// LDS in thread order.  kEpSiThreads threads serve a block's kBlock endpoints, so that each
// wave walks few of them (the float64 log and exp per endpoint and snapshot are long).
constexpr int kEpSiThreads = 1024;
__global__ __launch_bounds__(kEpSiThreads) void k_ep_partials_si(EpSiArgs a) {
  __shared__ double sh[5 * kEpSiThreads];
  const uint32_t S = (uint32_t)a.S;
  int dsg = 0;
  while (dsg + 1 < a.n_designs && (int)blockIdx.x >= a.ep_blk_off[dsg + 1]) ++dsg;
  const int i0 = a.ep_design_off[dsg] + ((int)blockIdx.x - a.ep_blk_off[dsg]) * kBlock;
  const int i1 = min(i0 + kBlock, a.ep_design_off[dsg + 1]);
  const SiLane ln = si_lane(a.sl2, a.S, (int)(threadIdx.x >> 6));
  double tns = 0.0, wmin = __builtin_huge_val(), tnsg = 0.0, m = 0.0, sm = 0.0;
  if (ln.on) {
    for (int i = i0 + ln.item; i < i1; i += kEpSiThreads >> a.sl2) {
      const EpVals ev = endpoint_values_si(a, i, ln.s);
      *at32(a.epv, si_at(i, S, ln.s)) = make_float4(ev.sg, ev.w0, ev.w1, 0.f);
      tns += fmin(0.0, (double)ev.worst);
      wmin = fmin(wmin, (double)ev.worst);
      // Each term in float (about 1e-7 relative), summed in float64 in the fixed order.
      tnsg += -(double)(fmaxf(0.f, -ev.sg) + a.gamma * log1pf(expf(-fabsf(ev.sg) * a.inv_gamma)));
      const double v = -(double)ev.sg;
      if (sm <= 0.0) {
        m = v;
        sm = 1.0;
      } else if (v > m) {
        sm = fma(sm, (double)expf((float)(m - v) * a.inv_gamma), 1.0);
        m = v;
      } else {
        sm += (double)expf((float)(v - m) * a.inv_gamma);
      }
    }
  }
  const int t = (int)threadIdx.x;
  sh[t] = tns;
  sh[kEpSiThreads + t] = wmin;
  sh[2 * kEpSiThreads + t] = tnsg;
  sh[3 * kEpSiThreads + t] = m;
  sh[4 * kEpSiThreads + t] = sm;
  __syncthreads();
  if (t < (1 << a.sl2) && ln.on) {
    double r0 = 0.0, r1 = __builtin_huge_val(), r2 = 0.0, r3 = 0.0, r4 = 0.0;
    for (int u = t; u < kEpSiThreads; u += 1 << a.sl2) {
      r0 += sh[u];
      r1 = fmin(r1, sh[kEpSiThreads + u]);
      r2 += sh[2 * kEpSiThreads + u];
      lse_merge_d(r3, r4, sh[3 * kEpSiThreads + u], sh[4 * kEpSiThreads + u], (double)a.gamma);
    }
    double* p = a.part;
    const int b = (int)blockIdx.x;
    p[si_at(5 * b + 0, S, ln.s)] = r0;
    p[si_at(5 * b + 1, S, ln.s)] = r1;
    p[si_at(5 * b + 2, S, ln.s)] = r2;
    p[si_at(5 * b + 3, S, ln.s)] = r4 > 0.0 ? r3 : -__builtin_huge_val();
    p[si_at(5 * b + 4, S, ln.s)] = r4;
  }
}

// Scalars of design blockIdx.x in snapshot blockIdx.y, from its partial blocks (fixed order:
// threads over blocks, then block_reduce), as k_ep_finalize.
__global__ __launch_bounds__(kBlock) void k_ep_finalize_si(EpSiArgs a) {
  __shared__ double sh[kBlock];
  const uint32_t S = (uint32_t)a.S;
  const int dsg = blockIdx.x, s = blockIdx.y;
  const int b0 = a.ep_blk_off[dsg], b1 = a.ep_blk_off[dsg + 1];
  const double g = a.gamma;
  double tns = 0.0, wmin = __builtin_huge_val(), tnsg = 0.0, mx = -__builtin_huge_val();
  for (int b = b0 + (int)threadIdx.x; b < b1; b += kBlock) {
    tns += a.part[si_at(5 * b + 0, S, s)];
    wmin = fmin(wmin, a.part[si_at(5 * b + 1, S, s)]);
    tnsg += a.part[si_at(5 * b + 2, S, s)];
    mx = fmax(mx, a.part[si_at(5 * b + 3, S, s)]);
  }
  double r4[4] = {tns, -wmin, tnsg, mx};
  block_reduce<4>(r4, {false, true, false, true}, sh);
  const double M = fmax(0.0, r4[3]);   // {0} joins the WNS_g set
  double tot = 0.0;
  for (int b = b0 + (int)threadIdx.x; b < b1; b += kBlock) {
    const double p4 = a.part[si_at(5 * b + 4, S, s)];
    if (p4 > 0.0) tot += p4 * exp((a.part[si_at(5 * b + 3, S, s)] - M) / g);
  }
  double r1[1] = {tot};
  block_reduce<1>(r1, {false}, sh);
  if (threadIdx.x == 0) {
    const double lse_all = M + g * log(r1[0] + exp(-M / g));
    const double nan = __builtin_nan("");
    const double v[5] = {fmin(0.0, -r4[1]), r4[0], a.smooth ? -lse_all : nan, a.smooth ? r4[2] : nan, lse_all};
    for (int q = 0; q < 5; ++q) a.fin[si_at(8 * dsg + q, S, s)] = v[q];
    if (a.scalars) {
      for (int q = 0; q < 4; ++q) a.scalars[((size_t)s * a.n_designs + dsg) * 4 + q] = v[q];
    }
  }
}

// Backward seeds of every (endpoint, snapshot), as k_ep_seed.
__global__ __launch_bounds__(kBlock) void k_ep_seed_si(EpSiArgs a) {
  const SiLane ln = si_lane(a.sl2, a.S, (int)blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6));
  const int i = ln.item;
  if (i >= a.E || !ln.on) return;
  const uint32_t S = (uint32_t)a.S;
  const int s = ln.s;
  const int e = ld(a.ep_pin, (uint32_t)i);
  *at32(a.sink, si_at(2 * e, S, s)) = make_float4(a.hold, a.hold, a.rat_late, a.rat_late);
  if (a.seed_adj) {
    const float4 q = ld(a.epv, si_at(i, S, s));
    float coef;
    if (a.wns_mode) {
      const double lse_all = a.fin[si_at(8 * ld(a.ep_design, (uint32_t)i) + 4, S, s)];
      coef = (float)exp((-(double)q.x - lse_all) / (double)a.gamma);
    } else {
      coef = 1.0f / (1.0f + expf(q.x * a.inv_gamma));
    }
    const float sc = a.scale_dev ? a.scale * (float)a.scale_dev[0] : a.scale;
    *at32(a.sink, si_at(2 * e + 1, S, s)) = make_float4(-sc * coef * q.y, -sc * coef * q.z, 0.f, 0.f);
  }
}

// ---------------------------------------------------------------- per-pin forward outputs
struct ExpandSiArgs {
  const int* __restrict__ net_off;
  const int* __restrict__ io_perm;
  const float4* __restrict__ rec;
  const float2* __restrict__ wire;
  float4* at;
  float4* slew;
  float2* atg;
  int N, S, sl2;
};

__global__ __launch_bounds__(kBlock) void k_expand_si(ExpandSiArgs a) {
  const SiLane ln = si_lane(a.sl2, a.S, (int)blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6));
  const int n = ln.item;
  if (n >= a.N || !ln.on) return;
  const uint32_t S = (uint32_t)a.S;
  const int s = ln.s;
  const int p0 = ld(a.net_off, (uint32_t)n), p1 = ld(a.net_off, (uint32_t)n + 1u);
  const float4 at = rec_at_si(a.rec, n, S, s), sl = rec_sl_si(a.rec, n, S, s);
  const float2 ag = a.atg ? rec_ag_si(a.rec, n, S, s) : make_float2(0.f, 0.f);
  for (int p = p0; p < p1; ++p) {
    const float2 w = ld(a.wire, si_at(p, S, s));
    const uint32_t o = si_at(a.io_perm ? ld(a.io_perm, (uint32_t)p) : p, S, s);
    if (a.at) store_stream(at32(a.at, o), make_float4(at.x + w.x, at.y + w.x, at.z + w.x, at.w + w.x));
    if (a.slew)
      store_stream(at32(a.slew, o), make_float4(sink_slew(sl.x, w.y), sink_slew(sl.y, w.y), sink_slew(sl.z, w.y),
                                                sink_slew(sl.w, w.y)));
    if (a.atg) store_stream(at32(a.atg, o), make_float2(ag.x + w.x, ag.y + w.x));
  }
}

// ---------------------------------------------------------------- backward level, snapshot lanes
struct BwdSiArgs {
  const int* __restrict__ net_off;
  const float* __restrict__ pin_cap;
  const int4* __restrict__ ell;
  const int* __restrict__ io_perm;
  const float* __restrict__ x;
  const float* __restrict__ y;
  const float4* __restrict__ grid;
  const float4* __restrict__ coef;
  LutKeys keys;
  const float4* __restrict__ rec;
  const float2* __restrict__ wire;
  const float* __restrict__ load;
  float4* __restrict__ sink;   // a net's sinks are read, other nets' input pins written
  float4* __restrict__ at_out;
  float4* __restrict__ slew_out;
  float4* __restrict__ rat_out;
  float4* __restrict__ slack_out;
  float* __restrict__ dx;
  float* __restrict__ dy;
  int N0, S, sl2;
  float r, c, inv_gamma;
};

struct SinkSi {
  float gx, gy, rest;
  uint32_t o;   // the pin's element in the caller's per-pin arrays
};

// Sink p of snapshot s in the net step (as sink_step): per-pin outputs when `write`, and its
// contribution to the driver's reductions.
template <bool kGrad>
__device__ __forceinline__ SinkSi sink_si(const BwdSiArgs& a, int p, int s, const float4& at_d, const float4& sl_d,
                                          float xd, float yd, float (&acc)[N_ACC], bool write) {
  const uint32_t S = (uint32_t)a.S;
  const float4 rt = ld(a.sink, si_at(2 * p, S, s));
  const float2 w = ld(a.wire, si_at(p, S, s));
  const uint32_t o = si_at(a.io_perm ? ld(a.io_perm, (uint32_t)p) : p, S, s);
  const float4 ats = make_float4(at_d.x + w.x, at_d.y + w.x, at_d.z + w.x, at_d.w + w.x);
  const float4 sls = make_float4(sink_slew(sl_d.x, w.y), sink_slew(sl_d.y, w.y), sink_slew(sl_d.z, w.y),
                                 sink_slew(sl_d.w, w.y));
  if (write) {
    if (a.at_out) store_stream(at32(a.at_out, o), ats);
    if (a.slew_out) store_stream(at32(a.slew_out, o), sls);
    if (a.rat_out) store_stream(at32(a.rat_out, o), rt);
    if (a.slack_out)
      store_stream(at32(a.slack_out, o), make_float4(ats.x - rt.x, ats.y - rt.y, rt.z - ats.z, rt.w - ats.w));
  }
  acc[R_E0] = fmaxf(acc[R_E0], rt.x - w.x);
  acc[R_E1] = fmaxf(acc[R_E1], rt.y - w.x);
  acc[R_L0] = fminf(acc[R_L0], rt.z - w.x);
  acc[R_L1] = fminf(acc[R_L1], rt.w - w.x);
  SinkSi k{0.f, 0.f, 0.f, o};
  if (kGrad) {
    const float4 aj = ld(a.sink, si_at(2 * p + 1, S, s));
    const float xs = ld(a.x, o), ys = ld(a.y, o), cp = ld(a.pin_cap, (uint32_t)p);
    const float q0 = sls.z > 0.f ? aj.z * frcp(sls.z) : 0.f;
    const float q1 = sls.w > 0.f ? aj.w * frcp(sls.w) : 0.f;
    acc[A_R] += aj.x;
    acc[A_F] += aj.y;
    acc[S_R] += q0 * sl_d.z;
    acc[S_F] += q1 * sl_d.w;
    const float dbar = aj.x + aj.y;
    const float ibar = (q0 + q1) * w.y;
    const float len = fabsf(xs - xd) + fabsf(ys - yd);
    k.rest = (dbar + ibar) * (1e-3f * a.r * fmaf(a.c, len, cp));
    k.gx = sgnf(xs - xd);
    k.gy = sgnf(ys - yd);
    acc[X_RS] += k.gx * k.rest;
    acc[X_N] += k.gx;
    acc[Y_RS] += k.gy * k.rest;
    acc[Y_N] += k.gy;
  }
  return k;
}

// Cell step of cell kc in snapshot s, one pass over its arcs: the inputs' required times, and
// with the gradient the split of the driver's adjoint over the arcs and the slew and load
// adjoints, which it returns.  The softmax weight of an arc is exp((x_j - ATg) / gamma), with
// ATg the driver's smoothed arrival that the forward kept (its maximum plus gamma times the log
// of its sum, Eq. 4); the slew adjoint goes to the first arc whose output slew equals the
// driver's kept worst slew (the forward took that maximum over the same lookups, bit for bit).
template <bool kGrad>
__device__ __forceinline__ float cell_step_si(const BwdSiArgs& a, const Slots& sl, int kc, int s, float load,
                                              const float (&acc)[N_ACC], float2 atg, float2 worst) {
  const uint32_t S = (uint32_t)a.S;
  const float rat_o[4] = {acc[R_E0], acc[R_E1], acc[R_L0], acc[R_L1]};
  const float abar[2] = {acc[A_R], acc[A_F]}, sbar[2] = {acc[S_R], acc[S_F]};
  const float ag[2] = {atg.x, atg.y}, smax[2] = {worst.x, worst.y};
  bool open[2] = {true, true};    // the worst-slew arc of the transition not met yet
  float lb[2] = {0.f, 0.f};
#pragma unroll 2
  for (int j = 0; j < sl.F; ++j) {
    const int4 e = ld(a.ell, (uint32_t)(sl.base + j * sl.nc + kc));
    if (e.x < 0) continue;
    const bool same = ell_positive(e);
    const float2 w = ld(a.wire, si_at(e.y, S, s));
    const float4 isl = rec_sl_si(a.rec, e.x, S, s);             // the input's slews
    const float2 iag = kGrad ? rec_ag_si(a.rec, e.x, S, s) : make_float2(0.f, 0.f);
    float4 rat_in = make_float4(0.f, 0.f, 0.f, 0.f), adj_in = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int m = k >> 1, t = k & 1;
      const int tp = same ? t : 1 - t;
      const LutVal v =
          lut_eval_si<kGrad>(a.grid, a.coef, a.keys, ell_arc(e), t, sink_slew(plane_pick(isl, m, same, t), w.y), load);
      set_comp(rat_in, 2 * m + tp, rat_o[k] - v.d);
      if (kGrad && m == 1) {
        const float xg = (((same == (t == 0)) ? iag.x : iag.y) + w.x) + v.d;
        const float dbar = fexp((xg - ag[t]) * a.inv_gamma) * abar[t];
        const bool star = open[t] && v.s == smax[t];
        open[t] = open[t] && !star;
        const float s_j = star ? sbar[t] : 0.f;
        set_comp(adj_in, tp, dbar);
        set_comp(adj_in, 2 + tp, fmaf(dbar, v.ddx, s_j * v.dsx));
        lb[t] = fmaf(dbar, v.ddy, fmaf(s_j, v.dsy, lb[t]));
      }
    }
    *at32(a.sink, si_at(2 * e.y, S, s)) = rat_in;
    if (kGrad) *at32(a.sink, si_at(2 * e.y + 1, S, s)) = adj_in;
  }
  return lb[0] + lb[1];
}

// Backward work of net n for the lane's snapshot (the three phases of bwd_net).  In a heavy
// workgroup (kHeavy) of kB threads the kB >> hl2 threads of a snapshot split the sinks and their
// reductions meet in LDS in thread order; the first thread of each snapshot then runs the
// cell step.
template <bool kGrad, bool kHeavy, int kB>
__device__ __forceinline__ void bwd_net_si(const BwdSiArgs& a, const Slots& sl, int n, const SiLane& ln, int hl2,
                                           float* sh) {
  const uint32_t S = (uint32_t)a.S;
  const int s = ln.on ? ln.s : 0;
  const int p0 = ld(a.net_off, (uint32_t)n), p1 = ld(a.net_off, (uint32_t)n + 1u);
  const float4 at_d = rec_at_si(a.rec, n, S, s);
  const float4 sl_d = rec_sl_si(a.rec, n, S, s);
  const float2 ag_d = kGrad ? rec_ag_si(a.rec, n, S, s) : make_float2(0.f, 0.f);
  float xd = 0.f, yd = 0.f;
  if (kGrad && ln.on) driver_xy_si(a.x, a.y, a.io_perm, p0, S, s, xd, yd);
  float acc[N_ACC] = {-kInf, -kInf, kInf, kInf, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const int lanes = 1 << hl2;                   // heavy workgroups: snapshots per workgroup
  const int first = kHeavy ? ln.item : 0;
  const int stride = kHeavy ? kB / lanes : 1;
  // What the Elmore adjoint needs of a thread's first sinks stays on chip: the sink's share in
  // this thread's column of the LDS array (rows from `crow`), the signs of its x and y offsets
  // as 2-bit codes (sign + 1) in two registers.  The adjoint pass then reads none of those
  // sinks again.  A lane outside heavy workgroups keeps kSiHeavy sinks (all of a net of that
  // class), a heavy workgroup's thread kSiCacheHeavy.
  constexpr int kCache = kHeavy ? kSiCacheHeavy : kSiHeavy;
  constexpr int crow = kHeavy ? N_ACC + 1 : 0;
  static_assert(crow + kCache <= kSiRows && 2 * kCache <= 32, "sink cache must fit the LDS array and codes");
  uint32_t gxs = 0, gys = 0;
  if (ln.on) {
    int i = 0;
#pragma unroll 4
    for (int p = p0 + 1 + first; p < p1; p += stride, ++i) {
      const SinkSi k = sink_si<kGrad>(a, p, s, at_d, sl_d, xd, yd, acc, true);
      if (kGrad && i < kCache) {
        sh[(crow + i) * kB + threadIdx.x] = k.rest;
        gxs |= (uint32_t)(int)(k.gx + 1.f) << (2 * i);
        gys |= (uint32_t)(int)(k.gy + 1.f) << (2 * i);
      }
    }
  }
  const bool leader = !kHeavy || (int)threadIdx.x < lanes;
  if (kHeavy) {
    // Tree over the threads of each snapshot (thread t and t + h meet while h >= lanes), in a
    // fixed order: the leaders end with the totals.
    const int t = (int)threadIdx.x;
#pragma unroll
    for (int i = 0; i < N_ACC; ++i) sh[i * kB + t] = acc[i];
    for (int h = kB >> 1; h >= lanes; h >>= 1) {
      __syncthreads();
      if (t < h) {
        acc[R_E0] = fmaxf(acc[R_E0], sh[R_E0 * kB + t + h]);
        acc[R_E1] = fmaxf(acc[R_E1], sh[R_E1 * kB + t + h]);
        acc[R_L0] = fminf(acc[R_L0], sh[R_L0 * kB + t + h]);
        acc[R_L1] = fminf(acc[R_L1], sh[R_L1 * kB + t + h]);
#pragma unroll
        for (int i = A_R; i < N_ACC; ++i) acc[i] += sh[i * kB + t + h];
        if (h > lanes) {
#pragma unroll
          for (int i = 0; i < N_ACC; ++i) sh[i * kB + t] = acc[i];
        }
      }
    }
  }
  float lbar = 0.f;
  if (leader && ln.on) {
    if (n >= a.N0)
      lbar = cell_step_si<kGrad>(a, sl, n - a.N0 - sl.c0, s, ld(a.load, si_at(n, S, s)), acc, ag_d,
                                 make_float2(sl_d.z, sl_d.w));
    const uint32_t o0 = si_at(a.io_perm ? ld(a.io_perm, (uint32_t)p0) : p0, S, s);
    if (a.at_out) store_stream(at32(a.at_out, o0), at_d);
    if (a.slew_out) store_stream(at32(a.slew_out, o0), sl_d);
    if (a.rat_out) store_stream(at32(a.rat_out, o0), make_float4(acc[R_E0], acc[R_E1], acc[R_L0], acc[R_L1]));
    if (a.slack_out)
      store_stream(at32(a.slack_out, o0),
                   make_float4(at_d.x - acc[R_E0], at_d.y - acc[R_E1], acc[R_L0] - at_d.z, acc[R_L1] - at_d.w));
    if (kGrad) {
      const float cl = a.c * lbar;
      if (a.dx) *at32(a.dx, o0) = -(acc[X_RS] + cl * acc[X_N]);
      if (a.dy) *at32(a.dy, o0) = -(acc[Y_RS] + cl * acc[Y_N]);
    }
  }
  if (kHeavy) {
    if (leader) sh[N_ACC * kB + threadIdx.x] = lbar;
    __syncthreads();
    lbar = sh[N_ACC * kB + (threadIdx.x & (unsigned)(lanes - 1))];
  }
  // Elmore adjoint of every sink: the cached ones from LDS and their codes, the rest (beyond
  // the cache) read again.
  if (kGrad && ln.on && (a.dx || a.dy)) {
    const float cl = a.c * lbar;
    int p = p0 + 1 + first;
    for (int i = 0; i < kCache && p < p1; ++i, p += stride) {
      const uint32_t o = si_at(a.io_perm ? ld(a.io_perm, (uint32_t)p) : p, S, s);
      const float rest = sh[(crow + i) * kB + threadIdx.x];
      const float gx = (float)((int)((gxs >> (2 * i)) & 3u) - 1);
      const float gy = (float)((int)((gys >> (2 * i)) & 3u) - 1);
      if (a.dx) *at32(a.dx, o) = gx * (cl + rest);
      if (a.dy) *at32(a.dy, o) = gy * (cl + rest);
    }
#pragma unroll 4
    for (; p < p1; p += stride) {
      float scratch[N_ACC] = {};
      const SinkSi k = sink_si<kGrad>(a, p, s, at_d, sl_d, xd, yd, scratch, false);
      if (a.dx) *at32(a.dx, k.o) = k.gx * (cl + k.rest);
      if (a.dy) *at32(a.dy, k.o) = k.gy * (cl + k.rest);
    }
  }
}

// One backward level: the level's huge nets [nu0, ne) and heavy nets [nh0, nu0) first, a
// workgroup per net and snapshot chunk, then the nets [nb, nh0), (64 >> sl2) per wave.
template <bool kGrad, int kB>
__global__ __launch_bounds__(kB) void k_bwd_level_si(int nb, int nh0, int nu0, int ne, Slots sl, BwdSiArgs a) {
  __shared__ float sh[(kGrad ? kSiRows : N_ACC + 1) * kB];   // the sink cache only with the gradient
  const int w = (int)(threadIdx.x >> 6);
  const int b = (int)blockIdx.x;
  const int hl2u = si_bwd_hl2(a.sl2, kB, true), hl2h = si_bwd_hl2(a.sl2, kB, false);
  const int nchu = chunks_of(a.S, hl2u), nchh = chunks_of(a.S, hl2h);
  const int nbu = (ne - nu0) * nchu, nbh = (nu0 - nh0) * nchh;
  if (b < nbu + nbh) {
    if (blockIdx.y != 0) return;               // these workgroups cover their snapshots along x
    if (b < nbu)
      bwd_net_si<kGrad, true, kB>(a, sl, nu0 + b / nchu, si_heavy_lane(hl2u, a.S, b % nchu), hl2u, sh);
    else
      bwd_net_si<kGrad, true, kB>(a, sl, nh0 + (b - nbu) / nchh, si_heavy_lane(hl2h, a.S, (b - nbu) % nchh), hl2h, sh);
    return;
  }
  const SiLane ln = si_lane(a.sl2, a.S, (b - nbu - nbh) * (kB / 64) + w);
  const int n = nb + ln.item;
  if (n >= nh0 || !ln.on) return;
  bwd_net_si<kGrad, false, kB>(a, sl, n, ln, a.sl2, sh);
}

}  // namespace
}  // namespace sta

using namespace sta;

namespace sta {
namespace {

Snap snap_of(const sta_graph* g) {
  return Snap{g->state.total, g->work.total, (size_t)g->P, 4 * (size_t)g->n_designs};
}

// Grid of a launch over all snapshots.  With several snapshots, the x extent is rounded up to
// a multiple of the 8 XCDs (spare blocks exit at once): consecutive workgroups go to
// consecutive XCDs, so every snapshot's copy of a block then runs on the same XCD and the
// topology it reads is fetched into one L2.
dim3 snap_grid(const sta_graph* g, unsigned blocks) {
  if (g->n_snap > 1) blocks = (blocks + 7u) / 8u * 8u;
  return dim3(blocks, (unsigned)g->n_snap, 1);
}

// Grid of a level launch over all snapshots: with a multiple of 8 snapshots the level
// kernels place each snapshot on one XCD (snap_block) and need no padding.
dim3 level_grid(const sta_graph* g, unsigned blocks) {
  if (g->n_snap % 8 == 0) return dim3(blocks, (unsigned)g->n_snap, 1);
  return snap_grid(g, blocks);
}

// One forward level with the schedule's lanes per cell (16: k_fwd_level, 8 or 4:
// k_fwd_level_narrow).
template <int L>
void fwd_narrow_launch(dim3 grid, bool snap, hipStream_t s, const Slots& sl, int n0, int min_slot, int ss,
                       const int4* ell, const float* load, const int* loc, float4* rec, const FwdArgs& fa) {
  if (snap)
    k_fwd_level_narrow<true, L><<<grid, kBlock, 0, s>>>(sl.nc, n0, sl.base, sl.F, min_slot, ss, ell, load, loc, rec, fa);
  else
    k_fwd_level_narrow<false, L><<<grid, kBlock, 0, s>>>(sl.nc, n0, sl.base, sl.F, min_slot, ss, ell, load, loc, rec,
                                                         fa);
}

void fwd_level_launch(const sta_graph* g, hipStream_t s, const Slots& sl, int min_slot, int ss, const int4* ell,
                      const float* load, const int* loc, float4* rec, const FwdArgs& fa) {
  const int lanes = g->sched_cfg.fwd_cell_lanes;
  const unsigned blocks = (unsigned)(((size_t)lanes * sl.nc + kBlock - 1) / kBlock);
  if (blocks == 0) return;
  const int n0 = g->N0 + sl.c0;
  const bool snap = g->n_snap > 1;
  const dim3 grid = snap ? level_grid(g, blocks) : dim3(blocks);
  if (lanes == 4) {
    fwd_narrow_launch<1>(grid, snap, s, sl, n0, min_slot, ss, ell, load, loc, rec, fa);
  } else if (lanes == 8) {
    fwd_narrow_launch<2>(grid, snap, s, sl, n0, min_slot, ss, ell, load, loc, rec, fa);
  } else if (snap) {
    k_fwd_level<true><<<grid, kBlock, 0, s>>>(sl.nc, n0, sl.base, sl.F, min_slot, ss, ell, load, loc, rec, fa);
  } else {
    k_fwd_level<false><<<grid, kBlock, 0, s>>>(sl.nc, n0, sl.base, sl.F, min_slot, ss, ell, load, loc, rec, fa);
  }
}

// RC pass p of a checkpointed star graph (rc_ranges: 0 the kept nets, 1 + j segment j's other
// nets), in lane groups over rc_sched (uploaded in sched_all's place).
void rc_pass(const sta_graph* g, hipStream_t s, RcArgs ra, int p) {
  ra.sched = g->dev.sched_all;
  ra.range = g->rc_ranges[p];
  const unsigned blocks = range_grid(ra.range);
  if (blocks > 0) k_rc<<<snap_grid(g, blocks), kBlock, 0, s>>>(ra);
}

// ---------------------------------------------------------------- snapshot-inner launches
struct SiDims {
  int S, sl2;
  unsigned gy;   // blocks of 64 snapshots (sl2 = 6) along y
  int hch, uch;  // workgroups per heavy and per huge net (chunks_of)
  bool split;    // heavy nets take workgroups (else every net one lane: one thread per net)
};

SiDims si_dims(const sta_graph* g) {
  const int S = g->n_snap;
  int sl2 = 0;
  while ((1 << sl2) < S && sl2 < 6) ++sl2;
  const int hw = 1 << sl2, uw = 1 << std::min(sl2, 3);
  return SiDims{S, sl2, (unsigned)(sl2 == 6 ? (S + 63) / 64 : 1), (S + hw - 1) / hw, (S + uw - 1) / uw,
                g->snap_inner};
}

// Workgroups of `waves` waves covering `items` items at 64 >> sl2 items per wave.
unsigned si_blocks(int items, int sl2, int waves) {
  const int per = waves << (6 - sl2);
  return (unsigned)((items + per - 1) / per);
}

EpSiArgs ep_si_args(const sta_graph* g, char* sb, double* scalars, float4* sink, const double* scale_dev, int seed_adj,
                    int smooth, int wns_mode, float gamma, float scale) {
  const DeviceGraph& d = g->dev;
  const SiDims D = si_dims(g);
  const size_t S = (size_t)D.S;
  return EpSiArgs{d.ep_pin, d.ep_net, d.ep_design, d.ep_design_off, d.ep_blk_off,
                  reinterpret_cast<float4*>(sb + S * g->state.rec), reinterpret_cast<float2*>(sb + S * g->state.wire),
                  reinterpret_cast<double*>(sb + S * g->state.part), reinterpret_cast<double*>(sb + S * g->state.fin),
                  scalars, sink, reinterpret_cast<float4*>(sb + S * g->state.epv), scale_dev, g->E, g->n_designs, D.S,
                  D.sl2, seed_adj, smooth, wns_mode, g->cons.t_clk - g->cons.setup, g->cons.hold, gamma,
                  1.0f / gamma, scale};
}

sta_status launch_forward_si(sta_graph* g, const float* x, const float* y, const sta_fwd_out* out, uint32_t flags,
                             float gamma_ps, hipStream_t s) {
  const bool smooth = (flags & STA_SMOOTH) != 0;
  const DeviceGraph& d = g->dev;
  const SiDims D = si_dims(g);
  const size_t S = (size_t)D.S;
  char* sb = static_cast<char*>(out->state);
  float4* rec = reinterpret_cast<float4*>(sb + S * g->state.rec);
  float2* wire = reinterpret_cast<float2*>(sb + S * g->state.wire);
  float* load = reinterpret_cast<float*>(sb + S * g->state.load);
  const int* io = (flags & STA_CANONICAL_IO) ? nullptr : d.pin_perm;
  {
    LaunchTimer t(g, s, STA_K_RC);
    const int nh = D.split ? (int)g->si_heavy.size() : 0, nu = D.split ? (int)g->si_huge.size() : 0;
    const RcSiArgs ra{d.net_off, d.pin_cap, x, y, io, d.si_heavy, d.si_huge, wire, load, rec, g->N, g->N0, D.S, D.sl2,
                      nh, nu, D.split ? kSiHeavy : INT32_MAX, g->cons.r_per_um, g->cons.c_per_um, g->cons.pi_at,
                      g->cons.pi_slew};
    k_rc_si<<<dim3((unsigned)(nh * D.hch + nu * D.uch) + si_blocks(g->N, D.sl2, kSiRcBlock / 64), D.gy), kSiRcBlock, 0,
              s>>>(ra);
  }
  const FwdSiArgs fa{d.ell, load, wire, rec, d.lut_grid, d.lut_coef, lut_keys(g), gamma_ps,
                     smooth ? 1.0f / gamma_ps : 0.f, smooth ? 1 : 0, D.S, D.sl2};
  for (int l = 1; l < g->L; ++l) {
    const Slots sl = level_slots(g, l);
    if (sl.nc == 0) continue;
    LaunchTimer t(g, s, STA_K_FWD_LEVEL);
    k_fwd_level_si<<<dim3(si_blocks(sl.nc, D.sl2, kWavesPerBlock), D.gy), kBlock, 0, s>>>(sl.nc, g->N0 + sl.c0,
                                                                                            sl.base, sl.F, fa);
  }
  const EpSiArgs ea = ep_si_args(g, sb, out->scalars, nullptr, nullptr, 0, smooth ? 1 : 0, 0, smooth ? gamma_ps : 1.0f,
                                 1.0f);
  if (g->n_ep_blocks > 0) {
    LaunchTimer t(g, s, STA_K_EP_PARTIAL);
    k_ep_partials_si<<<dim3(g->n_ep_blocks, D.gy), kEpSiThreads, 0, s>>>(ea);
  }
  {
    LaunchTimer t(g, s, STA_K_EP_FINAL);
    k_ep_finalize_si<<<dim3(g->n_designs, D.S), kBlock, 0, s>>>(ea);
  }
  if (out->at || out->slew || out->atg) {
    const ExpandSiArgs xa{d.net_off, io, rec, wire, reinterpret_cast<float4*>(out->at),
                          reinterpret_cast<float4*>(out->slew), reinterpret_cast<float2*>(out->atg), g->N, D.S, D.sl2};
    LaunchTimer t(g, s, STA_K_EXPAND);
    k_expand_si<<<dim3(si_blocks(g->N, D.sl2, kWavesPerBlock), D.gy), kBlock, 0, s>>>(xa);
  }
  if (g->profiling) end_run(g, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "forward launch");
  return STA_OK;
}

sta_status launch_backward_si(sta_graph* g, const float* x, const float* y, const sta_fwd_out* fwd,
                              const sta_bwd_out* out, uint32_t flags, float gamma_ps, hipStream_t s) {
  const bool grad = (flags & STA_GRAD) != 0;
  const DeviceGraph& d = g->dev;
  const SiDims D = si_dims(g);
  const size_t S = (size_t)D.S;
  char* sb = static_cast<char*>(fwd->state);
  char* wb = static_cast<char*>(out->workspace);
  float4* sink = reinterpret_cast<float4*>(wb + S * g->work.sink);
  const int* io = (flags & STA_CANONICAL_IO) ? nullptr : d.pin_perm;
  const EpSiArgs ea = ep_si_args(g, sb, nullptr, sink, out->grad_scale_dev, grad ? 1 : 0, 1,
                                 (flags & STA_GRAD_WNS) ? 1 : 0, grad ? gamma_ps : 1.0f, out->grad_scale);
  if (g->E > 0) {
    LaunchTimer t(g, s, STA_K_EP_SEED);
    k_ep_seed_si<<<dim3(si_blocks(g->E, D.sl2, kWavesPerBlock), D.gy), kBlock, 0, s>>>(ea);
  }
  const BwdSiArgs ba{d.net_off, d.pin_cap, d.ell, io, x, y, d.lut_grid, d.lut_coef, lut_keys(g),
                     reinterpret_cast<const float4*>(sb + S * g->state.rec),
                     reinterpret_cast<const float2*>(sb + S * g->state.wire),
                     reinterpret_cast<const float*>(sb + S * g->state.load), sink,
                     reinterpret_cast<float4*>(out->at), reinterpret_cast<float4*>(out->slew),
                     reinterpret_cast<float4*>(out->rat), reinterpret_cast<float4*>(out->slack), out->dx, out->dy,
                     g->N0, D.S, D.sl2, g->cons.r_per_um, g->cons.c_per_um, grad ? 1.0f / gamma_ps : 0.f};
  const int kb = g->sched_cfg.lane_block;    // 256, 512 or 1024 (sta_set_schedule checks)
  for (int l = g->L - 1; l >= 0; --l) {
    const int lo = g->level_off[l], hi = g->level_off[l + 1];
    const int hs = D.split ? g->si_hs[l] : hi, us = D.split ? g->si_us[l] : hi;
    if (hi == lo) continue;
    const int uch = (D.S + (1 << si_bwd_hl2(D.sl2, kb, true)) - 1) >> si_bwd_hl2(D.sl2, kb, true);
    const int hch = (D.S + (1 << si_bwd_hl2(D.sl2, kb, false)) - 1) >> si_bwd_hl2(D.sl2, kb, false);
    const unsigned blocks = (unsigned)((hi - us) * uch + (us - hs) * hch) + si_blocks(hs - lo, D.sl2, kb / 64);
    LaunchTimer t(g, s, STA_K_BWD_LEVEL);
    const Slots sl = level_slots(g, l);
    const dim3 grid(blocks, D.gy);
    if (kb == 256) {
      if (grad) k_bwd_level_si<true, 256><<<grid, 256, 0, s>>>(lo, hs, us, hi, sl, ba);
      else k_bwd_level_si<false, 256><<<grid, 256, 0, s>>>(lo, hs, us, hi, sl, ba);
    } else if (kb == 1024) {
      if (grad) k_bwd_level_si<true, 1024><<<grid, 1024, 0, s>>>(lo, hs, us, hi, sl, ba);
      else k_bwd_level_si<false, 1024><<<grid, 1024, 0, s>>>(lo, hs, us, hi, sl, ba);
    } else {
      if (grad) k_bwd_level_si<true, 512><<<grid, 512, 0, s>>>(lo, hs, us, hi, sl, ba);
      else k_bwd_level_si<false, 512><<<grid, 512, 0, s>>>(lo, hs, us, hi, sl, ba);
    }
  }
  if (g->profiling) end_run(g, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "backward launch");
  return STA_OK;
}

sta_status launch_forward(sta_graph* g, const float* x, const float* y, const sta_fwd_out* out, uint32_t flags,
                          float gamma_ps, hipStream_t s) {
  if (g->lanes_kernels()) return launch_forward_si(g, x, y, out, flags, gamma_ps, s);
  const bool smooth = (flags & STA_SMOOTH) != 0;
  const DeviceGraph& d = g->dev;
  char* sb = static_cast<char*>(out->state);
  float4* rec = reinterpret_cast<float4*>(sb + g->state.rec);
  float2* wire = reinterpret_cast<float2*>(sb + g->state.wire);
  float* load = reinterpret_cast<float*>(sb + g->state.load);
  const int* io = (flags & STA_CANONICAL_IO) ? nullptr : d.pin_perm;

  const Snap sn = snap_of(g);
  const bool tree = !g->c_parent.empty();
  const int n_chunks = (int)g->tree_blk_depth.size(), n_big = (int)g->tree_big.size();
  RcArgs ra{d.net_off, d.pin_cap, x, y, io, d.sched_all, g->all_range, wire, load, rec, g->N0, g->N,
            g->cons.r_per_um, g->cons.c_per_um, g->cons.pi_at, g->cons.pi_slew, sn, d.parent, d.tree_order,
            tree ? reinterpret_cast<float4*>(sb + g->state.tree) : nullptr, d.tree_node, d.tree_blk_net,
            d.tree_blk_depth, d.tree_big, n_big, n_chunks, d.sink_base};
  // With checkpointing the wire values share slots like the sink workspace: the RC stage runs
  // in passes (lane groups), the kept nets' here and each segment's before its levels.
  const bool rc_passes = !g->rc_ranges.empty();
  {
    LaunchTimer t(g, s, STA_K_RC);
    const unsigned per_net = (unsigned)((g->N + kBlock - 1) / kBlock);
    if (rc_passes) {
      rc_pass(g, s, ra, 0);
    } else if (tree) {
      if (n_chunks > 0) k_rc_tree_chunk<<<snap_grid(g, (unsigned)n_chunks), kBlock, 0, s>>>(ra);
      if (n_big > 0) k_rc_tree<<<snap_grid(g, (unsigned)((n_big + kBlock - 1) / kBlock)), kBlock, 0, s>>>(ra);
    } else if (g->sched_cfg.rc_scheme == STA_RC_CTE)
      k_rc_cte<<<snap_grid(g, per_net), kBlock, 0, s>>>(ra);
    else if (g->sched_cfg.rc_scheme == STA_RC_THREAD)
      k_rc_thread<<<snap_grid(g, per_net), kBlock, 0, s>>>(ra);
    else
      k_rc<<<snap_grid(g, range_grid(g->all_range)), kBlock, 0, s>>>(ra);
  }

  EpArgs ea{d.ep_pin, d.ep_net, d.ep_design, d.ep_design_off, d.ep_blk_off, rec, wire,
            reinterpret_cast<double*>(sb + g->state.part), reinterpret_cast<double*>(sb + g->state.fin), out->scalars,
            nullptr, 0, nullptr, g->E, g->n_designs, g->cons.t_clk - g->cons.setup, g->cons.hold,
            smooth ? gamma_ps : 1.0f, smooth ? 1.0f / gamma_ps : 1.0f, 1.0f, smooth ? 1 : 0, 0, sn,
            reinterpret_cast<float4*>(sb + g->state.epv), d.ep_sslot};
  // Under checkpointing each group of endpoints takes its values while its segment's records
  // and wire values are in their slots: group 0 (level-0 nets) after the RC stage, segment j's
  // before segment j + 1's RC pass, the last after the sweep.
  const bool ckpt = g->ckpt_stride > 0;
  auto ep_values = [&](int grp) {
    const int lo = g->ep_grp_off[(size_t)grp], n = g->ep_grp_off[(size_t)grp + 1] - lo;
    if (n <= 0) return;
    LaunchTimer t(g, s, STA_K_EP_PARTIAL);
    k_ep_values<<<dim3((unsigned)((n + kBlock - 1) / kBlock), g->n_snap), kBlock, 0, s>>>(ea, d.ep_grp + lo, n);
  };
  if (ckpt) ep_values(0);
  const FwdArgs fa{wire, d.lut_grid, d.lut_coef, lut_keys(g), gamma_ps, smooth ? 1.0f / gamma_ps : 0.f,
                   smooth ? 1 : 0};
  const bool cte = g->sched_cfg.level_scheme == STA_LEVEL_CTE;
  for (int l = 1; l < g->L; ++l) {
    if (ckpt) {                                // a segment starts: its nets' RC pass
      const auto it = std::find(g->seg_lo.begin(), g->seg_lo.end() - 1, l);
      if (it != g->seg_lo.end() - 1) {
        const int j = (int)(it - g->seg_lo.begin());
        if (j > 0) ep_values(j);               // the previous segment's endpoints
        if (rc_passes) {
          LaunchTimer t(g, s, STA_K_RC);
          rc_pass(g, s, ra, 1 + j);
        }
      }
    }
    const Slots sl = level_slots(g, l);
    if (sl.nc == 0) continue;
    LaunchTimer t(g, s, STA_K_FWD_LEVEL);
    if (cte)
      k_fwd_level_cte<<<(unsigned)((sl.nc + kCteItems - 1) / kCteItems), kBlock, 0, s>>>(
          sl.nc, g->N0 + sl.c0, sl.base, sl.F, d.ell, load, rec, fa);
    else
      fwd_level_launch(g, s, sl, 0, (int)sn.state, d.ell, load, d.rec_loc, rec, fa);
  }

  if (ckpt && g->seg_lo.size() > 1) ep_values((int)g->seg_lo.size() - 1);   // the last segment's
  ea.from_epv = ckpt ? 1 : 0;
  if (g->n_ep_blocks > 0) {
    LaunchTimer t(g, s, STA_K_EP_PARTIAL);
    k_ep_partials<<<dim3(g->n_ep_blocks, g->n_snap), kBlock, 0, s>>>(ea);
  }
  {
    LaunchTimer t(g, s, STA_K_EP_FINAL);
    k_ep_finalize<<<dim3(g->n_designs, g->n_snap), kBlock, 0, s>>>(ea);
  }

  if (out->at || out->slew || out->atg) {
    ExpandArgs xa{d.net_off, io, d.sched_all, g->all_range, rec, wire, reinterpret_cast<float4*>(out->at),
                  reinterpret_cast<float4*>(out->slew), reinterpret_cast<float2*>(out->atg), sn};
    LaunchTimer t(g, s, STA_K_EXPAND);
    k_expand<<<snap_grid(g, range_grid(g->all_range)), kBlock, 0, s>>>(xa);
  }
  if (g->profiling) end_run(g, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "forward launch");
  return STA_OK;
}

sta_status launch_backward(sta_graph* g, const float* x, const float* y, const sta_fwd_out* fwd,
                           const sta_bwd_out* out, uint32_t flags, float gamma_ps, hipStream_t s) {
  if (g->lanes_kernels()) return launch_backward_si(g, x, y, fwd, out, flags, gamma_ps, s);
  const bool grad = (flags & STA_GRAD) != 0;
  const DeviceGraph& d = g->dev;
  char* sb = static_cast<char*>(fwd->state);
  char* wb = static_cast<char*>(out->workspace);
  float4* rec = reinterpret_cast<float4*>(sb + g->state.rec);
  float2* wire = reinterpret_cast<float2*>(sb + g->state.wire);
  float* load = reinterpret_cast<float*>(sb + g->state.load);
  float4* sink = reinterpret_cast<float4*>(wb + g->work.sink);
  const int* io = (flags & STA_CANONICAL_IO) ? nullptr : d.pin_perm;

  EpArgs ea{d.ep_pin, d.ep_net, d.ep_design, d.ep_design_off, d.ep_blk_off, rec, wire,
            reinterpret_cast<double*>(sb + g->state.part), reinterpret_cast<double*>(sb + g->state.fin), nullptr, sink,
            grad ? 1 : 0, out->grad_scale_dev, g->E, g->n_designs, g->cons.t_clk - g->cons.setup,
            g->cons.hold, grad ? gamma_ps : 1.0f, grad ? 1.0f / gamma_ps : 1.0f, out->grad_scale, 1,
            (flags & STA_GRAD_WNS) ? 1 : 0, snap_of(g), reinterpret_cast<float4*>(sb + g->state.epv), d.ep_sslot};
  // Seeds: every endpoint at once, or under checkpointing each group right before its
  // segment's levels (its slots may be a segment buffer's), level-0 nets' first.
  auto ep_seed = [&](const int* list, int n) {
    if (n <= 0) return;
    LaunchTimer t(g, s, STA_K_EP_SEED);
    k_ep_seed<<<dim3((unsigned)((n + kBlock - 1) / kBlock), g->n_snap), kBlock, 0, s>>>(ea, list, n);
  };
  if (g->ckpt_stride <= 0)
    ep_seed(nullptr, g->E);
  else
    ep_seed(d.ep_grp, g->ep_grp_off[1]);

  const bool tree = !g->c_parent.empty();
  BwdArgs ba{d.net_off, d.pin_cap, d.ell, io, x, y, d.lut_grid, d.lut_coef, lut_keys(g),
             rec, wire, load, d.rec_loc, sink, reinterpret_cast<float4*>(out->at),
             reinterpret_cast<float4*>(out->slew), reinterpret_cast<float4*>(out->rat),
             reinterpret_cast<float4*>(out->slack), out->dx, out->dy, g->N0,
             g->cons.r_per_um, g->cons.c_per_um, grad ? 1.0f / gamma_ps : 0.f, grad ? 1 : 0, snap_of(g),
             (grad && tree) ? reinterpret_cast<float2*>(wb + g->work.tree_adj) : nullptr, d.sink_base};
  const int ss = (int)g->state.total;
  const bool cte = g->sched_cfg.level_scheme == STA_LEVEL_CTE;
  auto bwd_level = [&](int l) {
    if (cte) {
      const int lo = g->level_off[l], hi = g->level_off[l + 1];
      if (hi == lo) return;
      LaunchTimer t(g, s, STA_K_BWD_LEVEL);
      const dim3 grid((unsigned)((hi - lo + kCteItems - 1) / kCteItems));
      const Slots sl = level_slots(g, l);
      if (io == nullptr) {
        if (grad) k_bwd_level_cte<true, true><<<grid, kBlock, 0, s>>>(lo, hi, sl, ba);
        else k_bwd_level_cte<true, false><<<grid, kBlock, 0, s>>>(lo, hi, sl, ba);
      } else {
        if (grad) k_bwd_level_cte<false, true><<<grid, kBlock, 0, s>>>(lo, hi, sl, ba);
        else k_bwd_level_cte<false, false><<<grid, kBlock, 0, s>>>(lo, hi, sl, ba);
      }
      return;
    }
    const GroupRange& r = g->lvl_ranges[l];
    const unsigned blocks = range_grid(r);
    if (blocks == 0) return;
    LaunchTimer t(g, s, STA_K_BWD_LEVEL);
    const int nh = r.cls_off[kNumClasses + 1] - r.cls_off[kNumClasses], h0 = r.cls_off[kNumClasses];
    const int* c = r.cls_off;
    const int* w = r.wave_off;
    const Slots sl = level_slots(g, l);
    const BwdLaunch L{nh, h0, c[0], c[1], c[2], c[3], c[4], c[5], w[1], w[2], w[3], w[4], w[5], ss, d.net_off, rec, ba, sl};
    const bool snap = g->n_snap > 1, canon = io == nullptr;
    const dim3 grid = snap ? level_grid(g, blocks) : dim3(blocks);
    switch (r.g0 * 2 + (snap ? 1 : 0)) {
      case 4: bwd_launch<2, false>(grid, s, L, canon, grad); break;
      case 5: bwd_launch<2, true>(grid, s, L, canon, grad); break;
      case 6: bwd_launch<3, false>(grid, s, L, canon, grad); break;
      case 7: bwd_launch<3, true>(grid, s, L, canon, grad); break;
      case 8: bwd_launch<4, false>(grid, s, L, canon, grad); break;
      case 9: bwd_launch<4, true>(grid, s, L, canon, grad); break;
      case 10: bwd_launch<5, false>(grid, s, L, canon, grad); break;
      case 11: bwd_launch<5, true>(grid, s, L, canon, grad); break;
      case 12: bwd_launch<6, false>(grid, s, L, canon, grad); break;
      default: bwd_launch<6, true>(grid, s, L, canon, grad); break;
    }
  };
  if (g->ckpt_stride <= 0) {
    for (int l = g->L - 1; l >= 0; --l) bwd_level(l);
  } else {
    // Segments last to first: rebuild the records the forward dropped (the kept ones are
    // left alone), then that segment's backward levels.  The recomputation needs the
    // smoothed arrival only where the gradient reads it.
    const FwdArgs fa{wire, d.lut_grid, d.lut_coef, lut_keys(g), gamma_ps, grad ? 1.0f / gamma_ps : 0.f,
                     grad ? 1 : 0};
    const RcArgs ra{d.net_off, d.pin_cap, x, y, io, d.sched_all, g->all_range, wire, load, rec, g->N0, g->N,
                    g->cons.r_per_um, g->cons.c_per_um, g->cons.pi_at, g->cons.pi_slew, snap_of(g), nullptr,
                    nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, d.sink_base};
    for (int j = (int)g->seg_lo.size() - 2; j >= 0; --j) {
      const int lo = g->seg_lo[j], hi = g->seg_lo[j + 1];
      if (!g->rc_ranges.empty()) {             // the segment's wire values, rewritten
        LaunchTimer t(g, s, STA_K_RC);
        rc_pass(g, s, ra, 1 + j);
      }
      for (int l = lo; l < hi; ++l) {
        const Slots sl = level_slots(g, l);
        if (sl.nc == 0) continue;
        LaunchTimer t(g, s, STA_K_RECOMPUTE);
        fwd_level_launch(g, s, sl, g->n_kept, ss, d.ell, load, d.rec_loc, rec, fa);
      }
      ep_seed(d.ep_grp + g->ep_grp_off[(size_t)j + 1], g->ep_grp_off[(size_t)j + 2] - g->ep_grp_off[(size_t)j + 1]);
      for (int l = hi - 1; l >= lo; --l) bwd_level(l);
    }
    bwd_level(0);
  }
  if (grad && tree && (out->dx || out->dy)) {
    // The Elmore adjoint through each net's tree, from the sweep's per-sink adjoints.
    const TreeAdjArgs ta{d.net_off, d.parent, d.tree_order, io, x, y,
                         reinterpret_cast<const float4*>(sb + g->state.tree),
                         reinterpret_cast<const float2*>(wb + g->work.tree_adj),
                         reinterpret_cast<float4*>(wb + g->work.tree_bar), out->dx, out->dy, g->N,
                         g->cons.r_per_um, g->cons.c_per_um, snap_of(g), d.tree_node, d.tree_blk_net,
                         d.tree_blk_depth, d.tree_big, (int)g->tree_big.size(), (int)g->tree_blk_depth.size()};
    LaunchTimer t(g, s, STA_K_RC_ADJOINT);
    if (ta.n_chunks > 0) k_rc_tree_adjoint_chunk<<<snap_grid(g, (unsigned)ta.n_chunks), kBlock, 0, s>>>(ta);
    if (ta.n_list > 0)
      k_rc_tree_adjoint<<<snap_grid(g, (unsigned)((ta.n_list + kBlock - 1) / kBlock)), kBlock, 0, s>>>(ta);
  }
  if (g->profiling) end_run(g, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "backward launch");
  return STA_OK;
}

uint64_t bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, sizeof(u));
  return u;
}

// Runs `launch` on stream s, through a captured hipGraph when `use_graph` is set: the
// launches are recorded on a private stream the first time (or when the key changed) and
// the graph is replayed on s.
template <class F>
sta_status run_maybe_captured(sta_graph* g, sta_graph::Captured& cap, bool use_graph,
                              const std::vector<uint64_t>& key, hipStream_t s, F launch) {
  if (!use_graph || g->profiling) return launch(s);
  if (!(cap.valid && cap.key == key)) {
    if (cap.exec) (void)hipGraphExecDestroy(cap.exec);
    if (cap.graph) (void)hipGraphDestroy(cap.graph);
    cap = sta_graph::Captured{};
    hipError_t e;
    if (!g->cap_stream) {
      e = hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    }
    e = hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    sta_status st = launch(g->cap_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(g->cap_stream, &graph);
    if (st != STA_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(e, "hipGraphInstantiate");
    }
    cap.graph = graph;
    cap.exec = exec;
    cap.key = key;
    cap.valid = true;
  }
  hipError_t e = hipGraphLaunch(cap.exec, s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return STA_OK;
}

uint64_t ptr(const void* p) { return (uint64_t)(uintptr_t)p; }

// Remembers how the forward into `state` was run (see sta_graph::fwd_seen).
void note_forward(sta_graph* g, const void* state, bool smooth, float gamma) {
  auto& v = g->fwd_seen;
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i].state == state) {
      v.erase(v.begin() + (long)i);
      break;
    }
  if (v.size() >= sta_graph::kFwdSeen) v.erase(v.begin());
  v.push_back(sta_graph::FwdSeen{state, smooth, gamma, g->lanes_kernels()});
}

// The two families of level kernels keep records in different layouts (the snapshot-lane
// and thread-per-net kernels in planes): a backward reads a state that a forward of its own
// family wrote.  A state this graph's forward calls never wrote passes here.
sta_status check_state_family(const sta_graph* g, const void* state) {
  for (auto it = g->fwd_seen.rbegin(); it != g->fwd_seen.rend(); ++it) {
    if (it->state != state) continue;
    if (it->lanes != g->lanes_kernels())
      return fail(STA_E_STATE, "the forward state was computed under a schedule of the other kernel family "
                               "(snapshot lanes or thread per net against lane groups); run sta_forward again");
    return STA_OK;
  }
  return STA_OK;
}

// A gradient needs the smoothed arrivals of a forward with the same gamma on this graph.
sta_status check_grad_state(const sta_graph* g, const void* state, float gamma) {
  for (auto it = g->fwd_seen.rbegin(); it != g->fwd_seen.rend(); ++it) {
    if (it->state != state) continue;
    if (!it->smooth)
      return fail(STA_E_STATE, "the gradient needs a forward state computed with STA_SMOOTH");
    if (bits(it->gamma) != bits(gamma))
      return fail(STA_E_STATE, "the gradient's gamma differs from the gamma of the forward state");
    if (it->lanes != g->lanes_kernels())
      return fail(STA_E_STATE, "the forward state was computed under a schedule of the other kernel family "
                               "(snapshot lanes or thread per net against lane groups); run sta_forward again");
    return STA_OK;
  }
  return fail(STA_E_STATE, "the forward state was not produced by sta_forward on this graph");
}

}  // namespace
}  // namespace sta

extern "C" sta_status sta_forward(sta_graph* g, const float* x, const float* y, sta_fwd_out* out, uint32_t flags,
                                  float gamma_ps, sta_stream stream) {
  sta_status st = check_ready(g);
  if (st != STA_OK) return st;
  if (!out || !out->state) return fail(STA_E_INVALID, "forward state buffer is required");
  if (!x || !y) return fail(STA_E_INVALID, "x and y are required");
  if ((flags & STA_SMOOTH) && !(gamma_ps > 0.f && std::isfinite(gamma_ps)))
    return fail(STA_E_INVALID, "gamma must be positive");
  if (g->ckpt_stride > 0 && (out->at || out->slew || out->atg))
    return fail(STA_E_INVALID, "per-pin forward outputs need the full arrival state; with checkpointing take "
                               "them from sta_backward");
  const std::vector<uint64_t> key{ptr(x), ptr(y), ptr(out->state), ptr(out->at), ptr(out->slew), ptr(out->atg),
                                  ptr(out->scalars), flags, bits(gamma_ps)};
  const sta_fwd_out o = *out;
  st = run_maybe_captured(g, g->cap_fwd, (flags & STA_GRAPH) != 0, key, reinterpret_cast<hipStream_t>(stream),
                          [&](hipStream_t s) { return launch_forward(g, x, y, &o, flags, gamma_ps, s); });
  if (st == STA_OK) note_forward(g, out->state, (flags & STA_SMOOTH) != 0, gamma_ps);
  return st;
}

extern "C" sta_status sta_backward(sta_graph* g, const float* x, const float* y, const sta_fwd_out* fwd,
                                   sta_bwd_out* out, uint32_t flags, float gamma_ps, sta_stream stream) {
  sta_status st = check_ready(g);
  if (st != STA_OK) return st;
  if (!fwd || !fwd->state || !out || !out->workspace) return fail(STA_E_INVALID, "state and workspace are required");
  const bool grad = (flags & STA_GRAD) != 0;
  if (grad && (!x || !y)) return fail(STA_E_INVALID, "x and y are required for the gradient");
  if (grad && !(gamma_ps > 0.f && std::isfinite(gamma_ps))) return fail(STA_E_INVALID, "gamma must be positive");
  st = check_state_family(g, fwd->state);
  if (st != STA_OK) return st;
  if (grad) {
    st = check_grad_state(g, fwd->state, gamma_ps);
    if (st != STA_OK) return st;
  }
  const std::vector<uint64_t> key{ptr(x), ptr(y), ptr(fwd->state), ptr(out->workspace), ptr(out->at), ptr(out->slew),
                                  ptr(out->rat), ptr(out->slack), ptr(out->dx), ptr(out->dy), bits(out->grad_scale),
                                  ptr(out->grad_scale_dev), flags, bits(gamma_ps)};
  const sta_fwd_out f = *fwd;
  const sta_bwd_out o = *out;
  return run_maybe_captured(g, g->cap_bwd, (flags & STA_GRAPH) != 0, key, reinterpret_cast<hipStream_t>(stream),
                            [&](hipStream_t s) { return launch_backward(g, x, y, &f, &o, flags, gamma_ps, s); });
}

namespace sta {
namespace {

// Backward workspace of sta_backward_noalloc: a fixed array in device memory, one copy per
// device, held from the code object's load until the process ends.  Host code never passes
// its name to a kernel (on the host it names a stand-in, not device memory): it takes the
// device address once per device from hipGetSymbolAddress and uses that.
constexpr size_t kNoallocBytes = (size_t)STA_NOALLOC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

sta_status scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(STA_E_DEVICE, "device id beyond the library's table");
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(STA_E_DEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return STA_OK;
}

}  // namespace
}  // namespace sta

extern "C" sta_status sta_backward_noalloc(sta_graph* g, const float* x, const float* y, const sta_fwd_out* fwd,
                                           sta_bwd_out* out, uint32_t flags, float gamma_ps, sta_stream stream) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  if (!g->levelized) return fail(STA_E_STATE, "graph is not levelized");
  // Uploading allocates: the graph must already be on the device.
  if (!g->uploaded) return fail(STA_E_STATE, "graph is not uploaded; call sta_graph_upload first");
  if (flags & STA_GRAPH) return fail(STA_E_INVALID, "STA_GRAPH captures a hipGraph, which allocates");
  if (g->profiling) return fail(STA_E_STATE, "profiling creates events; disable it for this call");
  sta_status st = check_ready(g);
  if (st != STA_OK) return st;
  if (!fwd || !fwd->state || !out) return fail(STA_E_INVALID, "state and outputs are required");
  if (out->workspace) return fail(STA_E_INVALID, "workspace must be NULL: the library's own array is used");
  const size_t need = (size_t)g->n_snap * g->work.total;
  if (need > kNoallocBytes)
    return fail(STA_E_NOMEM, "backward workspace of " + std::to_string(need) + " bytes exceeds the " +
                                 std::to_string(kNoallocBytes) + "-byte fixed array of sta_backward_noalloc");
  const bool grad = (flags & STA_GRAD) != 0;
  if (grad && (!x || !y)) return fail(STA_E_INVALID, "x and y are required for the gradient");
  if (grad && !(gamma_ps > 0.f && std::isfinite(gamma_ps))) return fail(STA_E_INVALID, "gamma must be positive");
  st = check_state_family(g, fwd->state);
  if (st != STA_OK) return st;
  if (grad) {
    st = check_grad_state(g, fwd->state, gamma_ps);
    if (st != STA_OK) return st;
  }
  void* ws = nullptr;
  st = scratch_on(g->dev.device, &ws);
  if (st != STA_OK) return st;
  sta_bwd_out o = *out;
  o.workspace = ws;
  return launch_backward(g, x, y, fwd, &o, flags, gamma_ps, reinterpret_cast<hipStream_t>(stream));
}

namespace sta {
namespace {
// Shape bucket of a graph for the tuning cache (sta_tune_cached).
std::vector<int64_t> tune_bucket(const sta_graph* g) {
  int lg = 0;
  while ((1ll << lg) < (int64_t)g->P) ++lg;
  return {lg, g->n_snap, g->snap_inner ? 1 : 0, g->ckpt_stride > 0 ? 1 : 0, g->c_parent.empty() ? 0 : 1,
          g->n_designs > 1 ? 1 : 0};
}
std::mutex tune_mu;
std::map<std::vector<int64_t>, sta_schedule> tune_cache;
}  // namespace
}  // namespace sta

extern "C" sta_status sta_tune_cached(sta_graph* g, sta_schedule* sch) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  if (!g->levelized) return fail(STA_E_STATE, "graph is not levelized");
  sta_schedule c{};
  {
    std::lock_guard<std::mutex> lk(tune_mu);
    auto it = tune_cache.find(tune_bucket(g));
    if (it == tune_cache.end()) return fail(STA_E_STATE, "no tuned schedule for this graph's shape bucket yet");
    c = it->second;
  }
  const sta_status st = sta_set_schedule(g, &c);
  if (st == STA_OK && sch) *sch = c;
  return st;
}

extern "C" sta_status sta_tune(sta_graph* g, const float* x, const float* y, float gamma_ps, int32_t reps,
                               sta_schedule* best, sta_stream stream) {
  sta_status st = check_ready(g);
  if (st != STA_OK) return st;
  if (!x || !y) return fail(STA_E_INVALID, "x and y are required");
  if (!(gamma_ps > 0.f && std::isfinite(gamma_ps))) return fail(STA_E_INVALID, "gamma must be positive");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t P = (size_t)g->P;
  const size_t S = (size_t)g->n_snap;
  const size_t sizes[] = {S * g->state.total, S * g->work.total, S * 16 * P, S * 16 * P, S * 16 * P, S * 16 * P,
                          S * 4 * P, S * 4 * P, S * 32 * (size_t)g->n_designs};
  void* buf[9] = {};
  for (int i = 0; i < 9; ++i) {
    hipError_t e = hipMalloc(&buf[i], sizes[i]);
    if (e != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipFree(buf[j]);
      return hip_fail(e, "hipMalloc");
    }
  }
  sta_fwd_out fo{buf[0], nullptr, nullptr, nullptr, static_cast<double*>(buf[8])};
  sta_bwd_out bo{buf[1], static_cast<float*>(buf[2]), static_cast<float*>(buf[3]), static_cast<float*>(buf[4]),
                 static_cast<float*>(buf[5]), static_cast<float*>(buf[6]), static_cast<float*>(buf[7]), 1.0f, nullptr};
  const uint32_t ff = STA_SMOOTH | STA_CANONICAL_IO, bf = STA_RAT | STA_GRAD | STA_CANONICAL_IO;
  const sta_schedule start = g->sched_cfg;
  sta_schedule best_s = start;
  float best_ms = 1e30f;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  // Times one candidate and keeps it if it is the fastest so far.
  auto try_schedule = [&](const sta_schedule& cand) {
    st = sta_set_schedule(g, &cand);
    for (int r = -1; r < reps && st == STA_OK; ++r) {
      if (r == 0) (void)hipEventRecord(e0, s);
      st = launch_forward(g, x, y, &fo, ff, gamma_ps, s);
      if (st == STA_OK) st = launch_backward(g, x, y, &fo, &bo, bf, gamma_ps, s);
    }
    if (st != STA_OK) return;
    (void)hipEventRecord(e1, s);
    hipError_t e = hipEventSynchronize(e1);
    if (e != hipSuccess) {
      st = hip_fail(e, "hipEventSynchronize");
      return;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) {
      best_ms = ms;
      best_s = cand;
    }
  };
  // The snapshot-lane kernels take the workgroup size of their backward level.  Otherwise lane
  // groups of the level and one-pass kernels, then the other RC mappings (Alg. 2's task pool,
  // one thread per net) on the best of those, then 8 and 4 lanes per forward cell, then the
  // task pool in the level kernels and one thread per net in every stage.
  for (int kb : {256, 512, 1024}) {
    if (!g->snap_inner || st != STA_OK) break;
    sta_schedule c = start;
    c.lane_block = kb;
    try_schedule(c);
  }
  for (int sweep = 2; sweep <= 6 && st == STA_OK && !g->snap_inner; ++sweep)
    for (int flat = 2; flat <= 4 && st == STA_OK; ++flat)
      for (int heavy : {32, 64})
        if (st == STA_OK)
          try_schedule(sta_schedule{sweep, flat, heavy, STA_RC_GROUPS, 16, STA_LEVEL_GROUPS, start.lane_block});
  const sta_schedule lanes = best_s;
  for (int rc : {STA_RC_CTE, STA_RC_THREAD})
    if (st == STA_OK && !g->snap_inner)
      try_schedule(
          sta_schedule{lanes.sweep_group_log2, lanes.flat_group_log2, lanes.heavy_sinks, rc, 16, STA_LEVEL_GROUPS,
                       lanes.lane_block});
  const sta_schedule wide = best_s;
  for (int fl : {8, 4}) {
    sta_schedule narrow = wide;
    narrow.fwd_cell_lanes = fl;
    if (st == STA_OK && !g->snap_inner) try_schedule(narrow);
  }
  if (st == STA_OK && !g->snap_inner && g->n_snap == 1 && g->ckpt_stride == 0 && g->c_parent.empty()) {
    const sta_schedule pin_based = best_s;
    sta_schedule cte = pin_based;           // the CTE task pool in the level kernels too
    cte.rc_scheme = STA_RC_CTE;
    cte.level_scheme = STA_LEVEL_CTE;
    try_schedule(cte);
    sta_schedule thread = pin_based;        // one thread per net in every stage
    thread.level_scheme = STA_LEVEL_THREAD;
    if (st == STA_OK) try_schedule(thread);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (void* p : buf) (void)hipFree(p);
  if (st != STA_OK) {
    (void)sta_set_schedule(g, &start);
    return st;
  }
  st = sta_set_schedule(g, &best_s);
  if (st == STA_OK) {
    std::lock_guard<std::mutex> lk(tune_mu);
    tune_cache[tune_bucket(g)] = best_s;
  }
  if (best) *best = best_s;
  return st;
}

extern "C" sta_status sta_profile_enable(sta_graph* g, int32_t on) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  for (auto& t : g->timed) {
    g->event_pool.push_back(t.start);
    g->event_pool.push_back(t.stop);
  }
  g->timed.clear();
  if (g->run_start) g->event_pool.push_back(g->run_start);
  g->run_kind = -1;
  g->run_count = 0;
  g->run_start = nullptr;
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
    launches[t.kind] += t.count;
    total_ms[t.kind] += ms;
  }
  return STA_OK;
}
