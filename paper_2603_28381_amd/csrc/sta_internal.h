// Internal declarations shared by the host code and the HIP kernels of libsta.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "sta.h"

namespace sta {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64s)
constexpr int kNumClasses = 5;       // wave lane groups of 4, 8, 16, 32, 64 lanes per net
constexpr int kHeavy = kNumClasses;  // class of nets served by a whole workgroup
constexpr int kLutCells = (STA_LUT_N - 1) * (STA_LUT_N - 1);
constexpr int kFlatG0Default = 2;    // flat kernels (RC, outputs): smallest group 4 lanes
constexpr int kSweepG0Default = 2;   // level kernels: smallest backward group 4 lanes (one per condition)
constexpr int kTreeChunk = 1024;     // RC trees: pins of whole nets swept by one workgroup in LDS
constexpr int kSiHeavy = 12;         // snapshot-inner layout: nets with more sinks take a whole
                                     // workgroup for up to 64 snapshots,
constexpr int kSiHuge = 128;         // nets with more than this a workgroup per 8 snapshots (RC,
                                     // and the backward in 512-thread workgroups)

// Lane-group class of a net with `sinks` sink pins when the smallest group has 1 << g0
// lanes: the smallest wave group (doubling from 1 << g0) in which every lane holds at most
// one sink; nets with more than 64 sinks get a whole workgroup.
inline int net_class(int sinks, int g0, int heavy_sinks) {
  if (sinks > heavy_sinks) return kHeavy;
  int c = 0;
  for (int G = 1 << g0; G <= 64; G <<= 1, ++c)
    if (sinks <= G) return c;
  return kHeavy;
}

// A batch of nets processed by one launch: schedule entries [cls_off[c], cls_off[c+1])
// belong to class c, served by groups of (1 << g0) << c lanes.  Heavy nets take blocks
// [0, n_heavy) of the launch, one each; wave classes are served by waves
// [wave_off[c], wave_off[c+1]) of the blocks after them.
struct GroupRange {
  int cls_off[kNumClasses + 2];
  int wave_off[kNumClasses + 1];
  int g0;
};

// Breakpoints compared against when locating a table cell (held in scalar registers).
struct LutKeys {
  float x[STA_LUT_N - 2];   // slew_axis[1..5]
  float y[STA_LUT_N - 2];   // load_axis[1..5]
};

// Byte offsets of the pieces of the forward state buffer.
struct StateLayout {
  size_t rec;      // float4[4 * record slots]: per net and condition k {AT, slew, smoothed AT
                   // (late k; 0 for early k), 0}
  size_t wire;     // float2 per sink slot {wire delay, impulse} (slot = pin, zero at drivers,
                   // without checkpointing)
  size_t load;     // float[N]: root load of each net (Eq. 1)
  size_t tree;     // RC trees only, float4[2 * P]: per pin {length, Cap, Load, Delay} and
                   // {LDelay, Beta, Impulse, 0} of the tree passes
  size_t part;     // double[n_ep_blocks * 5]: endpoint partial sums
  size_t fin;      // double[n_designs * 8]: finished scalars and the WNS_g normaliser per design
  size_t epv;      // float4[E]: per endpoint {smoothed slack s_e, d s_e / d slack_g (rise, fall), 0}
  size_t total;
};

struct WorkLayout {
  size_t sink;     // float4[2 * P]: per sink its required time by condition, then its adjoint
                   // {a_rise, a_fall, s_rise, s_fall}; interleaved, so that the scattered
                   // writes of one sink fill one aligned 32-byte segment
  size_t tree_adj; // RC trees only, float2[P]: adjoints of each sink's {Delay, Impulse} and
                   // of each net's root load (at its driver), from the backward sweep
  size_t tree_bar; // RC trees only, float4[2 * P]: adjoint scratch of the tree passes
  size_t total;
};

struct DeviceGraph {
  int device = -1;
  std::vector<void*> allocs;
  int* net_off = nullptr;      // [N+1] canonical
  float* pin_cap = nullptr;    // [P]
  int4* ell = nullptr;         // cell inputs {source net, pin, arc, unateness}, padded slots per level
  int* ep_pin = nullptr;       // [E] endpoints, grouped by design
  int* ep_net = nullptr;       // [E] record slot of the endpoint's net
  int* ep_design = nullptr;    // [E] design of each endpoint
  int* ep_design_off = nullptr;  // [n_designs+1] endpoint ranges by design
  int* ep_blk_off = nullptr;   // [n_designs+1] partial-sum blocks by design
  int* pin_perm = nullptr;     // [P] original id of each canonical pin
  int* sched_all = nullptr;    // [N] all nets ordered by class (checkpointing on stars: rc_sched)
  int* rec_loc = nullptr;      // [N] record slot of each net (checkpointing only)
  int* parent = nullptr;       // [P] RC trees only: canonical parent pin, -1 at drivers
  int* tree_order = nullptr;   // [P] RC trees only: each net's pins in breadth-first order
  int4* tree_node = nullptr;   // [P] RC trees only: {depth, first child position, children, 0}
  int* tree_blk_net = nullptr;    // RC trees only: chunk net ranges
  int* tree_blk_depth = nullptr;  // RC trees only: deepest depth of each chunk
  int* tree_big = nullptr;        // RC trees only: nets over the chunk size
  float4* lut_grid = nullptr;  // [36] {x_i, 1/(x_i+1 - x_i), y_j, 1/(y_j+1 - y_j)}
  float4* lut_coef = nullptr;  // [n_arcs * 2 * 36 * 2] bilinear coefficients {a, b, c, d}
  int* sink_base = nullptr;    // [N] checkpointing (stars): first slot of each net's sinks
  int* ep_sslot = nullptr;     // [E] checkpointing (stars): workspace slot of each endpoint
  int* ep_grp = nullptr;       // [E] checkpointing: endpoint indices grouped by segment
  int* si_heavy = nullptr;     // snapshot-inner RC: canonical nets of kSiHeavy+1..kSiHuge sinks,
  int* si_huge = nullptr;      // and of more than kSiHuge
  size_t bytes = 0;
};

}  // namespace sta

struct sta_graph {
  // Input copy (original ids).
  int P = 0, N = 0, C = 0, A = 0, T = 0, n_arcs = 0;
  std::vector<int> net_off, net_pins, cell_type, cell_in_off, cell_in_pins, cell_out_pin;
  std::vector<float> pin_cap;
  std::vector<int8_t> pin_kind;
  std::vector<int> pin_parent;                 // RC tree parent pin (original ids), empty: stars
  std::vector<int> arc_off;
  std::vector<int8_t> unate;
  std::vector<float> slew_axis, load_axis, tables;
  sta_constraints cons{};

  // Levelization (canonical order).
  bool levelized = false;
  int L = 0, N0 = 0, E = 0, max_level_nets = 0;
  std::vector<int> level, level_off, net_perm, pin_perm;
  std::vector<int> c_net_off, c_cell_type, c_cin_off, c_cin_src, c_cin_pin, ep_pin, ep_net;
  std::vector<int4> c_cin;                     // packed cell inputs (device layout)
  std::vector<float> c_pin_cap;
  std::vector<int> sched_all;
  // Designs of a batch (one for a plain graph): pins [design_pin_off[d], design_pin_off[d+1])
  // by original id; endpoints grouped by design, each design's partial blocks contiguous.
  int n_designs = 1;
  std::vector<int> design_pin_off{0, 0};
  std::vector<int> ep_design, ep_design_off, ep_blk_off;
  std::vector<int4> ell;                       // padded per-level cell-input slots
  std::vector<int> ell_base, ell_slots;        // per level: first entry, slots per cell
  std::vector<int> c_parent, c_tree_order;     // RC trees: canonical parent pin (-1 at the
                                               // driver); each net's pins in breadth-first order
  std::vector<int4> c_tree_node;               // RC trees, per canonical pin: {depth, breadth-first
                                               // position of the first child, children, 0}
  std::vector<int> tree_blk_net, tree_blk_depth;  // RC trees: chunks of whole nets of at most
                                               // kTreeChunk pins (net ranges, deepest depth)
  std::vector<int> tree_big;                   // RC trees: nets over kTreeChunk pins
  std::vector<sta::GroupRange> lvl_ranges;   // per level
  sta::GroupRange all_range{};                 // all nets
  sta_schedule sched_cfg{sta::kSweepG0Default, sta::kFlatG0Default, 64, STA_RC_GROUPS, 16, STA_LEVEL_GROUPS, 512};
  // Checkpointing (stride 0 = off): record slot of each canonical net (kept nets first,
  // level-0 nets at their own index, then the shared segment buffer), segment boundaries
  // seg_lo (levels [seg_lo[j], seg_lo[j+1])), and the endpoints' record slots.
  int ckpt_stride = 0, n_rec = 0, n_kept = 0;
  int n_snap = 1;                              // placement snapshots per call (shared topology)
  bool snap_inner = false;                     // STA_SNAP_INNER: snapshot-innermost arrays, lanes
                                               // over snapshots
  // The snapshot-lane kernels run the sweep: with the snapshot-inner layout, and for one
  // snapshot under the thread-per-net schedule (one lane per item, no heavy-net workgroups).
  bool lanes_kernels() const { return snap_inner || sched_cfg.level_scheme == STA_LEVEL_THREAD; }
  std::vector<int> si_heavy, si_huge;          // canonical nets of kSiHeavy+1..kSiHuge sinks,
                                               // and of more than kSiHuge
  std::vector<int> si_hs, si_us;               // per level: its first net of more than kSiHeavy
                                               // and of more than kSiHuge sinks (a level's nets
                                               // ascend in pin count)
  std::vector<int> rec_loc, seg_lo, ep_rec;
  // Checkpointing: endpoint indices by the segment of their net, group g at
  // ep_grp[ep_grp_off[g] .. ep_grp_off[g + 1]) (group 0: level-0 nets, 1 + j: segment j).
  std::vector<int> ep_grp, ep_grp_off;
  // Sink workspace slots under checkpointing (star nets): a sink's required times and
  // adjoint live from the cell step (or, at an endpoint, the seed) that writes them to its
  // net's step; sinks whose net and reading cell share a segment, and endpoints, share a
  // segment buffer, the others keep a slot.  A net's sinks take consecutive slots from sink_base[net] (kept nets first,
  // then each segment's other nets from the buffer's start).  Empty without segmentation:
  // the slot of a sink is its pin.
  std::vector<int> sink_base, sslot, ep_sslot;
  int n_sslots = 0, n_sslots_kept = 0;
  // The per-sink wire values follow the same slots, so the RC stage runs in passes: the
  // nets with kept slots once before the sweep (rc_ranges[0]), the other nets of segment j
  // before each forward or recomputed pass over it (rc_ranges[1 + j]); rc_sched lists the
  // nets of each pass by lane-group class and takes sched_all's place on the device (the
  // kernels that read sched_all otherwise do not run under checkpointing).  rc_seg: each
  // net's pass (-1 kept, else j).
  std::vector<int> rc_seg, rc_sched;
  std::vector<sta::GroupRange> rc_ranges;
  sta::StateLayout state{};
  sta::WorkLayout work{};
  int n_ep_blocks = 0;

  // Device copy.
  bool uploaded = false;
  sta::DeviceGraph dev;

  // Launch sequences captured into hipGraphs (STA_GRAPH), keyed by the call's arguments.
  struct Captured {
    bool valid = false;
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  Captured cap_fwd, cap_bwd;
  hipStream_t cap_stream = nullptr;

  // The smoothing flag and gamma of the latest sta_forward into each state buffer (most
  // recent last, at most kFwdSeen entries), so that sta_backward can refuse a gradient
  // against a state computed without the smoothed arrival or with another gamma, or by the
  // other family of level kernels (lanes: the snapshot-lane / thread-per-net kernels, whose
  // backward takes the softmax normaliser and worst-slew arc from their forward's records).
  struct FwdSeen { const void* state; bool smooth; float gamma; bool lanes; };
  static constexpr size_t kFwdSeen = 256;
  std::vector<FwdSeen> fwd_seen;

  // Event timing of launches (sta_profile_enable).
  bool profiling = false;
  // A run of consecutive launches of one kind, bracketed by one event pair.
  struct TimedLaunch { int kind; int count; hipEvent_t start, stop; };
  std::vector<TimedLaunch> timed;
  int run_kind = -1;                 // kind of the open run, -1 if none
  int run_count = 0;
  hipEvent_t run_start = nullptr;
  std::vector<hipEvent_t> event_pool;
};

namespace sta {
void set_error(const std::string& msg);
sta_status fail(sta_status code, const std::string& msg);
sta_status hip_fail(hipError_t e, const char* what);
void compute_layouts(sta_graph* g);
void build_lut_coefficients(const sta_graph* g, std::vector<float4>& grid, std::vector<float4>& coef);
LutKeys lut_keys(const sta_graph* g);
void drop_captured(sta_graph* g);
void build_schedule(sta_graph* g);
}  // namespace sta
