/*
 * sta.h - C ABI of a levelized static timing analysis (STA) engine for AMD MI355X (gfx950).
 *
 * The engine runs the four stages of parallel STA described in Warp-STAR
 * (arXiv 2603.28381, Sec. 2.1): RC net delay, levelization, forward propagation of
 * arrival times (AT) and backward propagation of required times (RAT) and slack, plus
 * the LSE-smoothed total/worst negative slack of Sec. 3.2 (Eq. 4) and its gradient
 * with respect to pin coordinates.  Every step of the sweep runs in hand-written HIP
 * kernels; the host side only validates, levelizes and launches.
 *
 * Conventions
 *  - Units: um (coordinates), ohm, fF, ps.
 *  - Timing condition index k = 2*mode + transition; mode 0 = early, 1 = late;
 *    transition 0 = rise, 1 = fall.  Per-pin 4-condition arrays are [pin][k], float32.
 *  - Status codes are returned by every call; no C++ exception crosses the ABI.
 *    sta_last_error() returns a thread-local message for the last failing call.
 *  - Host arrays passed in are copied; the caller may free them when the call returns.
 *  - Pointers documented as "device" are caller-owned device memory (for example torch
 *    tensors).  Work is enqueued on the given HIP stream and is asynchronous: keep the
 *    buffers alive until the stream has synchronized.
 *  - Calls that touch one sta_graph from several threads or streams at once race;
 *    serialize them.
 */
#ifndef STA_H
#define STA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STA_ABI_VERSION 1
#define STA_LUT_N 7          /* NLDM tables are 7 x 7 */
#define STA_MAX_FANIN 8      /* inputs per cell */

typedef int32_t sta_status;
#define STA_OK 0
#define STA_PENDING 1
#define STA_E_INVALID (-1)   /* malformed input (bad CSR, index out of range, ...) */
#define STA_E_CYCLE (-2)     /* combinational loop found while levelizing */
#define STA_E_NOMEM (-3)     /* device or host allocation failed, or a budget is exceeded */
#define STA_E_DEVICE (-4)    /* a HIP runtime call failed */
#define STA_E_BUSY (-5)      /* a queue is full; try again later */
#define STA_E_STATE (-6)     /* call made in the wrong state (e.g. not levelized) */
#define STA_E_UNKNOWN_TICKET (-7)

/* Pin kinds. PI and CELL_OUT pins drive nets; CELL_IN, FF_D and PO pins are sinks.
 * FF_D (flop data) and PO (primary output) pins are the timing endpoints. */
#define STA_PIN_PI 0
#define STA_PIN_CELL_IN 1
#define STA_PIN_CELL_OUT 2
#define STA_PIN_FF_D 3
#define STA_PIN_PO 4

typedef struct sta_graph sta_graph;
typedef void* sta_stream;     /* a hipStream_t; NULL means the null stream */

/* Netlist as a DAG of pins, cells and nets (Sec. 2.1): every net has one driver, listed
 * first in its pin list, and one or more sinks.  Every cell has 1..STA_MAX_FANIN input
 * pins and one output pin. */
typedef struct sta_netlist {
  int32_t n_pins, n_nets, n_cells;
  const int32_t* net_offsets;      /* [n_nets+1], CSR offsets into net_pins */
  const int32_t* net_pins;         /* [n_pins], each pin exactly once, driver first */
  const int32_t* cell_type;        /* [n_cells], index into the library */
  const int32_t* cell_in_offsets;  /* [n_cells+1], CSR offsets into cell_in_pins */
  const int32_t* cell_in_pins;     /* [n_cell_inputs], input j of a cell uses arc j of its type */
  const int32_t* cell_out_pin;     /* [n_cells] */
  const float* pin_cap;            /* [n_pins], pin capacitance, fF */
  const int8_t* pin_kind;          /* [n_pins], STA_PIN_* */
  const int32_t* pin_parent;       /* [n_pins] or NULL.  NULL: every net is a star (each sink
                                      wired straight to its driver).  Otherwise the RC tree of
                                      each net: the pin of the same net whose wire segment feeds
                                      this pin, -1 at drivers; following parents must reach the
                                      driver.  Trees use the recursive Eq. 1, the parent's delay
                                      in Eq. 2 and the second moment of the impulse (TAU 2015
                                      model cited for Eq. 1-3); a star gives the same values.
                                      Trees add 32 bytes per pin to the forward state and 40 to
                                      the backward workspace. */
} sta_netlist;

/* NLDM cell library (Sec. 3.1.2: cell arc delay by table interpolation).  One arc per
 * cell input.  tables[arc][q][i][j], q = 0 delay-rise, 1 delay-fall, 2 slew-rise,
 * 3 slew-fall (the output transition); row i follows slew_axis (input slew), column j
 * follows load_axis (load of the driven net).  Lookups interpolate bilinearly and
 * extrapolate linearly from the edge cell.  Axes must be strictly increasing. */
typedef struct sta_library {
  int32_t n_cell_types;
  const int32_t* arc_offsets;      /* [n_cell_types+1] */
  const int8_t* arc_unate;         /* [n_arcs], +1 positive unate, -1 negative unate */
  const float* slew_axis;          /* [STA_LUT_N], ps */
  const float* load_axis;          /* [STA_LUT_N], fF */
  const float* tables;             /* [n_arcs][4][STA_LUT_N][STA_LUT_N], ps */
} sta_library;

/* Constraints and wire model.  Endpoints: late RAT = t_clk - setup, early RAT = hold.
 * Primary inputs: AT = pi_at, slew = pi_slew.  Wires: r_per_um ohm/um, c_per_um fF/um. */
typedef struct sta_constraints {
  float t_clk, setup, hold, pi_at, pi_slew, r_per_um, c_per_um;
} sta_constraints;

typedef struct sta_graph_info {
  int32_t n_pins, n_nets, n_cells, n_cell_inputs, n_endpoints;
  int32_t n_levels;                /* net levels, 0 .. n_levels-1; 0 until levelized */
  int32_t n_pi_nets;               /* nets at level 0 */
  int32_t max_level_nets;          /* widest level */
  int64_t fwd_state_bytes;         /* size of sta_fwd_out.state (all snapshots) */
  int64_t bwd_workspace_bytes;     /* size of sta_bwd_out.workspace (all snapshots) */
  int64_t device_bytes;            /* graph data held on the device after upload */
  int32_t n_designs;               /* designs in the graph: 1, or the size of a batch */
  int32_t n_snapshots;             /* placement snapshots swept per call (sta_set_snapshots) */
} sta_graph_info;

/* sta_forward / sta_backward flags */
#define STA_SMOOTH (1u << 0)        /* compute the LSE-smoothed late arrival (Eq. 4) */
#define STA_CANONICAL_IO (1u << 1)  /* x, y and per-pin outputs use the canonical pin order */
#define STA_RAT (1u << 2)           /* backward: required times and slack per pin */
#define STA_GRAD (1u << 3)          /* backward: gradient of the smoothed objective */
#define STA_GRAD_WNS (1u << 4)      /* with STA_GRAD: differentiate WNS_g instead of TNS_g */
#define STA_GRAPH (1u << 5)         /* capture the call's launches into a hipGraph on first use and
                                       replay it while every argument stays the same */

/* Forward outputs.  state is required; every other pointer may be NULL. */
typedef struct sta_fwd_out {
  void* state;      /* device, >= fwd_state_bytes: per-net arrival state, wire delays and
                       loads kept for sta_backward; opaque */
  float* at;        /* device [n_pins][4] arrival times */
  float* slew;      /* device [n_pins][4] slews */
  float* atg;       /* device [n_pins][2] smoothed late arrival (rise, fall) */
  double* scalars;  /* device [n_designs][4]: WNS, TNS, WNS_g, TNS_g (g: smoothed with gamma) */
} sta_fwd_out;

/* Backward outputs.  workspace is required; every other pointer may be NULL. */
typedef struct sta_bwd_out {
  void* workspace;  /* device, >= bwd_workspace_bytes; opaque, contents undefined after */
  float* at;        /* device [n_pins][4] arrival times (written here instead of forward) */
  float* slew;      /* device [n_pins][4] */
  float* rat;       /* device [n_pins][4] required arrival times; +inf/-inf if unconstrained */
  float* slack;     /* device [n_pins][4]; late RAT - AT, early AT - RAT */
  float* dx;        /* device [n_pins] d objective / d x, times grad_scale */
  float* dy;        /* device [n_pins] */
  float grad_scale; /* multiplies the gradient (the incoming gradient of an autograd graph) */
  const double* grad_scale_dev; /* device scalar, or NULL; if set, also multiplies the gradient */
} sta_bwd_out;

/* ---------------------------------------------------------------------------------------
 * Graph construction.  Checks the netlist (Sec. 2.1: one driver per net, every pin in
 * exactly one net, cell pins consistent with their kinds and the library) and copies it.
 * Errors: STA_E_INVALID with a message; *out is left NULL.
 * ------------------------------------------------------------------------------------- */
sta_status sta_build_graph(const sta_netlist* nl, const sta_library* lib,
                           const sta_constraints* cons, sta_graph** out);

/* Levelization (Sec. 2.1 stage 2; Sec. 3.1.2): a net's level is 0 if a primary input
 * drives it, else 1 + the deepest level among the nets feeding its driving cell.  Builds
 * the canonical order: nets sorted by (level, pin count, original id) - the pin count key
 * makes the nets of one lane-group size class contiguous inside each level, so a level
 * launch maps each wave to one class; pins renumbered net by net, driver first, then
 * sinks in input order; cells ordered like the nets they drive.
 * Host only, idempotent.  Errors: STA_E_CYCLE for a combinational loop. */
sta_status sta_levelize(sta_graph* g, int32_t* n_levels_out);

/* Copies the levelization out (caller-allocated host arrays, sizes from sta_graph_info):
 * level[n_nets] by original net id, level_offsets[n_levels+1] over canonical nets,
 * net_perm[n_nets] and pin_perm[n_pins] giving the original id at each canonical
 * position.  Any pointer may be NULL.  STA_E_STATE if not levelized. */
sta_status sta_get_levelization(const sta_graph* g, int32_t* level, int32_t* level_offsets,
                                int32_t* net_perm, int32_t* pin_perm);

/* Uploads the levelized graph, schedule and library tables to the current HIP device.
 * Idempotent; sta_forward calls it when needed.  Errors: STA_E_STATE, STA_E_DEVICE,
 * STA_E_NOMEM. */
sta_status sta_graph_upload(sta_graph* g);

sta_status sta_graph_info_get(const sta_graph* g, sta_graph_info* info);

/* Batch of designs swept together: a new graph whose netlist is the disjoint union of the
 * given graphs (design d's pins, nets and cells follow design d-1's; identical libraries
 * are stored once).  Levelizing it aligns every design's level l in one level l, so each
 * level launch of sta_forward / sta_backward covers the nets of all designs; results equal
 * per-design calls.  Placement snapshots of one netlist are passed as the same graph
 * repeated.  Graphs must share constraints and table axes (else STA_E_INVALID); the inputs
 * stay owned by the caller and may be destroyed afterwards.  Scalars of the batch are
 * per design.  Use sta_batch_pin_map to route per-design coordinates and results. */
sta_status sta_batch_create(sta_graph* const* graphs, int32_t n_graphs, sta_graph** out);

/* For each canonical pin of a levelized batch: its design and its pin id in that design's
 * own numbering (caller-allocated arrays of n_pins; either may be NULL).
 * Errors: STA_E_STATE if not levelized. */
sta_status sta_batch_pin_map(const sta_graph* g, int32_t* design, int32_t* pin);
void sta_graph_destroy(sta_graph* g);

/* ---------------------------------------------------------------------------------------
 * Forward sweep.  RC net delay of every net (Sec. 3.1.1, Eq. 1-3, star nets, wire length
 * |dx|+|dy|, half of each wire's capacitance at each end), then levels 1..L-1 in order:
 * cell-arc delay and slew by table lookup, late AT = max over inputs of (input AT + arc
 * delay), early = min; worst slew; with STA_SMOOTH the late merge is also taken with
 * LSE (Eq. 4).  Sink AT = driver AT + wire delay; sink slew = sqrt(driver slew^2 +
 * Impulse^2).  Endpoint scalars (WNS, TNS over late worst transition; smoothed WNS_g,
 * TNS_g) go to out->scalars.
 * x, y: device [n_pins] float32 pin coordinates.  gamma_ps > 0 with STA_SMOOTH.
 * Errors: STA_E_STATE if not levelized, STA_E_INVALID for NULL state or bad gamma.
 * ------------------------------------------------------------------------------------- */
sta_status sta_forward(sta_graph* g, const float* x, const float* y, sta_fwd_out* out,
                       uint32_t flags, float gamma_ps, sta_stream stream);

/* Backward sweep over levels L-1..0 (Sec. 2.1 stage 4; Sec. 3.1.2): RAT from the
 * endpoints, RAT(driver) = min over sinks (max early) of RAT(sink) - wire delay,
 * RAT(cell input) = RAT(output) - arc delay, slack.  With STA_GRAD the adjoint of the
 * smoothed objective (Sec. 3.2) runs in the same sweep (operation fusion): gradient of
 * TNS_g (or WNS_g with STA_GRAD_WNS) with respect to x, y.  x, y must hold the same
 * coordinates given to sta_forward, and fwd->state its result (computed with STA_SMOOTH
 * for STA_GRAD) on the same graph; flags must carry the same STA_CANONICAL_IO and gamma_ps
 * the same value as that call.  Without checkpointing the backward only reads fwd->state,
 * so several backward calls on one state (e.g. a required-time sweep and a gradient sweep
 * on two streams, each with its own workspace) may run concurrently; with checkpointing
 * it rebuilds records inside the state and calls on one state must not overlap.
 * The forward and the backward of a state run under schedules of one kernel family: the
 * snapshot-lane layout and STA_LEVEL_THREAD keep the state's records in another layout than
 * the lane-group schemes, and their backward takes each cell's softmax normaliser and
 * worst-slew arc from the forward's records.
 * Errors: STA_E_STATE (not levelized / not uploaded; a state that the latest of this graph's
 * sta_forward calls into it computed under a schedule of the other kernel family; with
 * STA_GRAD also a state that call did not compute with STA_SMOOTH and the same gamma_ps, or
 * that no sta_forward on this graph produced), STA_E_INVALID.
 * ------------------------------------------------------------------------------------- */
sta_status sta_backward(sta_graph* g, const float* x, const float* y, const sta_fwd_out* fwd,
                        sta_bwd_out* out, uint32_t flags, float gamma_ps, sta_stream stream);

/* ---------------------------------------------------------------------------------------
 * Backward sweep that allocates nothing, for callers that cannot allocate device memory:
 * code under hipGraph stream capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same sweep, arguments, results and errors as sta_backward (the same kernels), except:
 *  - out->workspace must be NULL.  The workspace is a fixed array of
 *    STA_NOALLOC_WORKSPACE_BYTES inside the library, one per device, held from the library's
 *    first use of that device until the process ends.  Its address is looked up once per
 *    device, on the first call there; nothing is allocated or freed by any call.
 *  - the graph must already be uploaded to the current device (sta_graph_upload, or a
 *    sta_forward on it): uploading allocates.  STA_E_STATE otherwise, and while profiling
 *    (sta_profile_enable) is on, since that creates events.
 *  - STA_GRAPH is refused (STA_E_INVALID): capturing and instantiating a graph allocates.
 *    The call may itself be recorded by a caller's stream capture.
 *  - every call on one device shares that device's array, which keeps the last call's
 *    contents (the sweep writes every entry it reads, so nothing needs clearing).  Calls
 *    that overlap on one device race: serialize them, for example on one stream.
 * Errors: STA_E_NOMEM when the graph's bwd_workspace_bytes (all snapshots) exceed
 * STA_NOALLOC_WORKSPACE_BYTES, with the sizes in the message; STA_E_DEVICE when the array's
 * device address cannot be obtained; otherwise as sta_backward.
 * ------------------------------------------------------------------------------------- */
#define STA_NOALLOC_WORKSPACE_BYTES (96ll << 20)   /* 96 MiB: star designs of 3.1M pins */
sta_status sta_backward_noalloc(sta_graph* g, const float* x, const float* y, const sta_fwd_out* fwd,
                                sta_bwd_out* out, uint32_t flags, float gamma_ps, sta_stream stream);

/* ---------------------------------------------------------------------------------------
 * Placement snapshots.  With n_snapshots = S > 1 every sta_forward / sta_backward call sweeps
 * S placements of the same graph at once: the topology, library tables and launch plan are
 * shared, and launches get a second grid dimension over snapshots.  Every per-call buffer
 * then holds S copies back to back: x, y [S][n_pins]; at, slew, rat, slack [S][n_pins][4];
 * atg [S][n_pins][2]; dx, dy [S][n_pins]; scalars [S][n_designs][4]; state and workspace
 * S times their one-snapshot size (fwd_state_bytes and bwd_workspace_bytes report the
 * total).  Snapshot s computes exactly what a call with S = 1 on its coordinates computes.
 * Errors: STA_E_INVALID for S outside 1..65535; sta_forward / sta_backward return
 * STA_E_INVALID when one snapshot's state would exceed 2 GiB.
 * ------------------------------------------------------------------------------------- */
sta_status sta_set_snapshots(sta_graph* g, int32_t n_snapshots);

/* ---------------------------------------------------------------------------------------
 * Snapshot layout.  STA_SNAP_OUTER (default): per-call arrays hold the S snapshots back to
 * back, as above, and each snapshot is swept by its own workgroups with the lane-group
 * schedule.  STA_SNAP_INNER: every per-call array has the snapshot innermost - x, y
 * [n_pins][S]; at, slew, rat, slack [n_pins][S][4]; atg [n_pins][S][2]; dx, dy [n_pins][S];
 * scalars stay [S][n_designs][4] - and so does the opaque state and workspace; the lanes of
 * a wave then take snapshots (one net or cell for 64 snapshots, or for S <= 32 several
 * items of a power of two of lanes each), so topology and table reads serve every snapshot
 * and each state access is one contiguous run.  Same results up to float summation order
 * (a net's sinks and the endpoints are summed in index order per snapshot); of the schedule
 * only lane_block applies, and sta_tune picks it.  Meant for S of 32 or more.
 * Errors: STA_E_STATE if not levelized; STA_E_INVALID for an unknown layout, and for
 * STA_SNAP_INNER with checkpointing on or RC trees (pin_parent); sta_forward / sta_backward
 * return STA_E_INVALID when an array of all snapshots would reach 4 GiB.
 * ------------------------------------------------------------------------------------- */
#define STA_SNAP_OUTER 0
#define STA_SNAP_INNER 1
sta_status sta_set_snapshot_layout(sta_graph* g, int32_t layout);

/* ---------------------------------------------------------------------------------------
 * Lane-group schedule.  Nets are served by lane groups sized from their sink count: the
 * level kernels use groups of (1 << sweep_group_log2) lanes and doublings up to a wave
 * (4 lanes at least: a backward cell step spreads 4 conditions x 4 arcs over 16 lanes, over
 * 8 lanes with two arcs each in 8-lane groups, or over 4 lanes with all arcs in each), the
 * one-pass kernels (RC, output expansion) groups from (1 << flat_group_log2) lanes, and
 * nets with more than heavy_sinks sinks take a whole 256-thread workgroup.  rc_scheme
 * picks the mapping of the RC net delay stage (Sec. 3.1.1): these lane groups (the
 * pin-based scheme of Alg. 1), the CTE task pool of Alg. 2 (a workgroup pools the sinks of
 * 256 nets and rebalances them over its threads), or one thread per net.  fwd_cell_lanes
 * is the number of lanes per cell in the forward level kernel: 16 (one per condition and
 * arc, merged across lanes), 8 (two per condition, two arcs each) or 4 (one per condition,
 * each lane looking up all of the cell's arcs): fewer lanes launch fewer waves, which pays
 * when many snapshots fill the chip, while one design's short levels favour 16.
 * level_scheme STA_LEVEL_THREAD runs the whole sweep with one thread per net and per cell
 * (the snapshot-lane kernels with one lane per item; other fields then do not apply), and
 * STA_LEVEL_CTE runs the level kernels in the CTE scheme (Alg. 2 applied to arrival
 * propagation and slack computation, Sec. 3.1.2: a workgroup pools the inputs of 16 cells,
 * or the sinks and then the driving cells' inputs of 16 nets, and rebalances them over its
 * 256 threads; rc_scheme still picks the RC stage).  Both need one snapshot, no checkpointing,
 * the snapshot-outer layout and star nets (else STA_E_INVALID; sta_set_checkpointing,
 * sta_set_snapshots and sta_set_snapshot_layout refuse what they exclude while set).
 * lane_block tiles the snapshot-lane backward level (STA_SNAP_INNER): the threads of one
 * workgroup, which serves one net of more than 12 sinks or a wave's worth of light nets
 * per 64 threads; smaller workgroups let a CU start new waves sooner after its slowest one,
 * larger ones give a heavy net more threads per snapshot.  Defaults
 * {2, 2, 64, STA_RC_GROUPS, 16, STA_LEVEL_GROUPS, 512}.
 * Setting a schedule rebuilds the launch plan (no result changes beyond float summation
 * order).  Errors: STA_E_INVALID for out-of-range fields,
 * STA_E_STATE if not levelized.
 * ------------------------------------------------------------------------------------- */
#define STA_RC_GROUPS 0   /* lane groups per net (Alg. 1) */
#define STA_RC_CTE 1      /* workgroup task pool (Alg. 2) */
#define STA_RC_THREAD 2   /* one thread per net */

#define STA_LEVEL_GROUPS 0   /* level kernels: lane groups per net, 4-16 lanes per cell */
#define STA_LEVEL_THREAD 1   /* one thread per net and per cell in every stage (RC, levels,
                                endpoints), the mapping of earlier GPU timers; one snapshot,
                                no checkpointing, star nets */
#define STA_LEVEL_CTE 2      /* level kernels over a workgroup task pool (Alg. 2); one
                                snapshot, no checkpointing, star nets */

typedef struct sta_schedule {
  int32_t sweep_group_log2;   /* 2..6 */
  int32_t flat_group_log2;    /* 2..6 */
  int32_t heavy_sinks;        /* 1..64 */
  int32_t rc_scheme;          /* STA_RC_GROUPS, STA_RC_CTE or STA_RC_THREAD */
  int32_t fwd_cell_lanes;     /* 16, 8 or 4 */
  int32_t level_scheme;       /* STA_LEVEL_GROUPS, STA_LEVEL_THREAD or STA_LEVEL_CTE */
  int32_t lane_block;         /* STA_SNAP_INNER: threads per workgroup of the backward level,
                                 256, 512 or 1024 */
} sta_schedule;

sta_status sta_get_schedule(const sta_graph* g, sta_schedule* sch);
sta_status sta_set_schedule(sta_graph* g, const sta_schedule* sch);

/* Autotuner: times one forward+backward (smoothed, gradient, canonical IO, every per-pin
 * output) of g on the given coordinates for each candidate schedule, `reps` times after a
 * warm-up, keeps the fastest (copied to *best if not NULL) and leaves it set.  Candidates:
 * with STA_SNAP_INNER lane_block 256, 512 and 1024 and nothing else; otherwise
 * sweep_group_log2 2..6 x flat_group_log2 2..4 x heavy_sinks {32, 64} with lane-group RC
 * and 16 forward lanes, then on the best of those the CTE and thread RC mappings, then 8
 * and 4 forward lanes, then (one snapshot, no checkpointing, star nets) the CTE scheme in
 * the RC stage and the level kernels, and one thread per net in every stage.  Allocates
 * and frees its own device buffers; synchronizes the stream.  Errors: as sta_forward. */
sta_status sta_tune(sta_graph* g, const float* x, const float* y, float gamma_ps, int32_t reps,
                    sta_schedule* best, sta_stream stream);

/* Tuned schedules are cached per shape bucket, process-wide: the pin count's power of two,
 * the snapshot count, the snapshot layout, whether checkpointing is on, whether the graph
 * has RC trees and whether it batches several designs.  sta_tune stores its result under
 * g's bucket (replacing an earlier one); sta_tune_cached sets the cached schedule of g's
 * bucket on g (copied to *sch if not NULL) without timing anything.  Errors: STA_E_STATE
 * if g is not levelized or its bucket has no tuned schedule yet (g keeps its schedule). */
sta_status sta_tune_cached(sta_graph* g, sta_schedule* sch);

/* ---------------------------------------------------------------------------------------
 * Per-level checkpointing of the arrival state (the memory/time trade-off of reverse-mode
 * differentiation applied to the level sweep).  With a stride of k levels, levels 1..L-1
 * are cut into segments of k levels.  The forward keeps the arrival record (AT, slew,
 * smoothed AT of the driver) only of the nets still needed after their segment ends: nets
 * read by a cell in a later segment (the live frontier of a segment boundary; the graph is
 * a DAG, so a net can be read many levels later) and level-0 nets.  All other nets of a
 * segment share one buffer that the next segment overwrites; the forward takes the values
 * of a segment's endpoints (late arrival, smoothed slack and its weights) before that.
 * sta_backward walks the segments last to first, recomputes the dropped records of a
 * segment from the frontier, seeds its endpoints, then runs its backward levels.  Results are
 * bit-identical to the run without checkpointing; fwd_state_bytes shrinks (see
 * sta_get_checkpointing), and on star-net graphs bwd_workspace_bytes too (a sink's required
 * times and adjoint live from the cell step or endpoint seed writing them to its net's step:
 * nets whose sinks are all written and read inside one segment share a buffer that the next
 * segment reuses; each sink's wire delay and impulse in the state follow the same slots, so the RC
 * stage then runs in lane groups, in passes before each segment); the backward pays one
 * extra forward pass, and RC pass, over the dropped nets.
 *
 * stride_levels: 0 switches checkpointing off, a negative value picks ceil(sqrt(L-1)).
 * Changing it rebuilds the launch plan, changes fwd_state_bytes and releases the device
 * copy (uploaded again on the next call): state buffers must be allocated anew.  With
 * checkpointing on, sta_forward does not produce per-pin outputs (at/slew/atg must be
 * NULL; take them from sta_backward), and sta_backward must get the forward's gamma.
 * Errors: STA_E_STATE if not levelized.
 * ------------------------------------------------------------------------------------- */
sta_status sta_set_checkpointing(sta_graph* g, int32_t stride_levels);
/* Current stride (0 = off), number of arrival records the state holds (kept nets plus the
 * shared segment buffer; n_nets without checkpointing) and of those, the kept nets. */
sta_status sta_get_checkpointing(const sta_graph* g, int32_t* stride_levels, int32_t* record_slots,
                                 int32_t* kept_nets);

/* ---------------------------------------------------------------------------------------
 * Serving: timing queries of resident designs with continuous batching.
 *
 * A server owns a scheduler thread and `max_slots` slots, each a HIP stream with a device
 * buffer it keeps between requests (from a stream-ordered pool).  Designs are added once
 * and stay resident in HBM (topology, library tables and their placement coordinates).
 * Clients submit requests from any thread; each request is one forward sweep (slack query:
 * WNS, TNS and their smoothed forms) or one forward + backward sweep (also d TNS_g / dx,
 * dy), optionally on new coordinates.  The scheduler admits queued requests in arrival
 * order as soon as a slot is free whose buffer holds the request, or can grow to hold it
 * with the resident designs and every slot buffer within the budget; requests that arrive
 * while others run start at once and their levels overlap on the device.  Requests of one
 * design, kind and gamma that wait together are batched by level depth: up to max_merge of
 * them (a power of two) run as placement snapshots of one sweep, each level launch
 * advancing all of them (sta_set_snapshots), on one slot.  A slot captures the launch
 * sequence of each (design, kind, coordinates, gamma, snapshots) once into a hipGraph and
 * replays it, so a sweep costs a few host calls.  Every snapshot is computed by the same
 * arithmetic in the same order as a call of its own, so a result is bitwise the same alone,
 * beside other requests and merged with them.
 * ------------------------------------------------------------------------------------- */
typedef struct sta_server sta_server;

typedef struct sta_server_config {
  int64_t hbm_budget_bytes;    /* device memory for resident designs plus requests in flight */
  int32_t max_slots;           /* requests on the device at once (1..64) */
  int32_t queue_capacity;      /* requests waiting for admission before STA_E_BUSY (>= 1) */
  int32_t max_merge;           /* requests swept together as snapshots, at most (0 or 1: each
                                  alone; else a power of two up to 64).  Merging needs the
                                  snapshot-outer layout and lane-group schedules (a design
                                  under STA_SNAP_INNER, STA_LEVEL_THREAD or STA_LEVEL_CTE
                                  runs alone). */
} sta_server_config;

#define STA_REQ_FWD 0          /* forward sweep: scalars only */
#define STA_REQ_FWD_BWD 1      /* forward + backward: scalars and the gradient of TNS_g */

typedef struct sta_request {
  int32_t design;              /* id from sta_server_add_design */
  int32_t kind;                /* STA_REQ_FWD or STA_REQ_FWD_BWD */
  const float* x;              /* host [n_pins] by original pin id, copied at submit; NULL: */
  const float* y;              /*   the design's resident coordinates (both or neither) */
  float gamma_ps;              /* LSE smoothing (> 0) */
} sta_request;

typedef struct sta_result {
  int32_t kind;
  int32_t n_pins;
  double scalars[4];           /* WNS, TNS, WNS_g, TNS_g (ps) */
  const float* dx;             /* host [n_pins] by original pin id (STA_REQ_FWD_BWD), owned */
  const float* dy;             /*   by the server until sta_release; NULL otherwise */
  double queue_ms;             /* submit -> admitted to a slot */
  double latency_ms;           /* submit -> results on the host */
} sta_result;

/* Creates a server on the current device.  Errors: STA_E_INVALID for out-of-range fields,
 * STA_E_DEVICE if the device lacks stream-ordered memory pools. */
sta_status sta_server_create(const sta_server_config* cfg, sta_server** out);
/* Makes a levelized graph with one snapshot resident (uploading it to the server's device
 * if needed) with host coordinates x, y [n_pins] by original pin id.  The caller keeps g alive until
 * sta_server_destroy and makes no other calls on it meanwhile.  Errors: STA_E_STATE (not
 * levelized, or uploaded to another device), STA_E_NOMEM when the design does not fit the
 * budget. */
sta_status sta_server_add_design(sta_server* s, sta_graph* g, const float* x, const float* y, int32_t* id);
/* Queues a request (non-blocking; copies x, y to pinned staging).  Errors: STA_E_INVALID,
 * STA_E_NOMEM if the request can never fit the budget, STA_E_BUSY if the queue is full. */
sta_status sta_submit(sta_server* s, const sta_request* r, uint64_t* ticket);
/* STA_PENDING while queued or running; STA_OK with *r filled once done; the status of the
 * failure if the request failed; STA_E_UNKNOWN_TICKET for a ticket never issued or released. */
sta_status sta_poll(sta_server* s, uint64_t ticket, sta_result* r);
/* Blocks until the ticket is done (or failed), then as sta_poll. */
sta_status sta_wait(sta_server* s, uint64_t ticket, sta_result* r);
/* Releases a finished ticket's result buffers, or cancels a queued one.  STA_E_BUSY for a
 * request on the device, STA_E_UNKNOWN_TICKET otherwise. */
sta_status sta_release(sta_server* s, uint64_t ticket);
/* Waits for the requests on the device, drops queued ones and frees everything. */
void sta_server_destroy(sta_server* s);

/* Counters of a server since it was created.  A slot captures the launch sequence of each
 * (design, kind, new-or-resident coordinates, gamma) it runs the first time, keeping at most
 * 64 per slot (the oldest is dropped first); captures run outside the server's lock, so
 * clients can submit and poll meanwhile. */
typedef struct sta_server_stats {
  int64_t completed;           /* requests finished successfully */
  int64_t captures;            /* launch sequences captured into hipGraphs */
  double capture_ms;           /* host time of the requests that captured, admission to enqueued */
  int64_t sweeps;              /* launch sequences issued (one per admitted batch) */
  int64_t merged;              /* requests that ran in a sweep with at least one other */
  int64_t slot_grows;          /* slot buffers (re)allocated from the pool */
  double grow_ms;              /* host time of those allocations */
  int64_t pinned_allocs;       /* pinned host staging buffers allocated (sta_submit reuses */
  double pinned_ms;            /*   released ones of the same size), and their host time */
} sta_server_stats;
sta_status sta_server_stats_get(sta_server* s, sta_server_stats* out);
/* Changes max_merge (as in sta_server_config) for sweeps admitted from now on, for example to
 * warm every slot on single requests before merging.  Errors: STA_E_INVALID. */
sta_status sta_server_set_max_merge(sta_server* s, int32_t max_merge);

/* ---------------------------------------------------------------------------------------
 * Kernel timing with HIP events (a profiling aid).  While enabled, each run of consecutive
 * launches of one kernel family that sta_forward / sta_backward make for g (for example
 * all backward levels) is bracketed by two events on its stream, and hipGraph replay is
 * off.  sta_profile_read waits for those events and returns, per kernel family (STA_K_*),
 * the number of launches and their summed duration in milliseconds since the last enable;
 * the arrays hold STA_K_COUNT entries.  Errors: STA_E_DEVICE.
 * ------------------------------------------------------------------------------------- */
#define STA_K_RC 0           /* RC net delay, all nets */
#define STA_K_FWD_LEVEL 1    /* one forward level */
#define STA_K_EP_PARTIAL 2   /* endpoint partial sums */
#define STA_K_EP_FINAL 3     /* endpoint scalars */
#define STA_K_EXPAND 4       /* per-pin forward outputs */
#define STA_K_EP_SEED 5      /* backward seeds */
#define STA_K_BWD_LEVEL 6    /* one backward level (RAT, slack, adjoint) */
#define STA_K_RECOMPUTE 7    /* one forward level recomputed from a checkpoint */
#define STA_K_RC_ADJOINT 8   /* Elmore adjoint through RC trees (graphs with pin_parent) */
#define STA_K_COUNT 9
sta_status sta_profile_enable(sta_graph* g, int32_t on);
sta_status sta_profile_read(sta_graph* g, int64_t* launches, double* total_ms);

const char* sta_last_error(void);
int32_t sta_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STA_H */
