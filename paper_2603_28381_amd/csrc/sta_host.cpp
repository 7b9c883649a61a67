// Host side of libsta: input validation, levelization, canonical ordering, lane-group
// schedules, device upload and the C ABI bookkeeping calls.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>

#include "sta_internal.h"

namespace sta {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

sta_status fail(sta_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

sta_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? STA_E_NOMEM : STA_E_DEVICE;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

void compute_layouts(sta_graph* g) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  g->ep_blk_off.assign(g->n_designs + 1, 0);
  for (int d = 0; d < g->n_designs; ++d) {
    const int e = g->ep_design_off[d + 1] - g->ep_design_off[d];
    g->ep_blk_off[d + 1] = g->ep_blk_off[d] + (e + kBlock - 1) / kBlock;
  }
  g->n_ep_blocks = g->ep_blk_off[g->n_designs];
  g->state.rec = take(sizeof(float4) * 4 * (size_t)std::max(1, g->n_rec));
  g->state.wire = take(sizeof(float2) * (size_t)(g->n_sslots > 0 ? g->n_sslots : g->P));
  g->state.load = take(sizeof(float) * (size_t)g->N);
  const bool tree = !g->c_parent.empty();
  g->state.tree = take(tree ? 2 * sizeof(float4) * (size_t)g->P : 0);
  g->state.part = take(sizeof(double) * 5 * (size_t)std::max(1, g->n_ep_blocks));
  g->state.fin = take(sizeof(double) * 8 * (size_t)g->n_designs);
  g->state.epv = take(sizeof(float4) * (size_t)std::max(1, g->E));
  g->state.total = off;
  off = 0;
  g->work.sink = take(2 * sizeof(float4) * (size_t)(g->n_sslots > 0 ? g->n_sslots : g->P));
  g->work.tree_adj = take(tree ? sizeof(float2) * (size_t)g->P : 0);
  g->work.tree_bar = take(tree ? 2 * sizeof(float4) * (size_t)g->P : 0);
  g->work.total = off;
}

// Bilinear interpolation over cell (i, j) written as a + b*tx + c*ty + d*tx*ty, with
// tx, ty the unclamped local coordinates; linear extrapolation reuses the edge cell.
void build_lut_coefficients(const sta_graph* g, std::vector<float4>& grid, std::vector<float4>& coef) {
  const int n = STA_LUT_N, m = n - 1;
  grid.resize(kLutCells);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double x0 = g->slew_axis[i], x1 = g->slew_axis[i + 1];
      double y0 = g->load_axis[j], y1 = g->load_axis[j + 1];
      grid[i * m + j] = make_float4((float)x0, (float)(1.0 / (x1 - x0)), (float)y0, (float)(1.0 / (y1 - y0)));
    }
  coef.resize((size_t)g->n_arcs * 2 * kLutCells * 2);
  for (int a = 0; a < g->n_arcs; ++a)
    for (int tr = 0; tr < 2; ++tr)
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
          for (int q = 0; q < 2; ++q) {   // q = 0 delay table, 1 slew table
            const float* T = &g->tables[(((size_t)a * 4 + (size_t)(2 * q + tr)) * n) * n];
            double t00 = T[i * n + j], t10 = T[(i + 1) * n + j], t01 = T[i * n + j + 1],
                   t11 = T[(i + 1) * n + j + 1];
            size_t idx = ((((size_t)a * 2 + tr) * kLutCells) + (size_t)(i * m + j)) * 2 + q;
            coef[idx] = make_float4((float)t00, (float)(t10 - t00), (float)(t01 - t00),
                                    (float)(t11 - t10 - t01 + t00));
          }
}

LutKeys lut_keys(const sta_graph* g) {
  LutKeys k;
  for (int i = 0; i < STA_LUT_N - 2; ++i) {
    k.x[i] = g->slew_axis[i + 1];
    k.y[i] = g->load_axis[i + 1];
  }
  return k;
}

// Lane-group schedule of a set of nets: stable order by class, and per-class wave counts.
static GroupRange group_range(const int* cls_count, int base, int g0) {
  GroupRange r{};
  r.g0 = g0;
  int off = base, waves = 0;
  for (int c = 0; c < kNumClasses; ++c) {
    r.cls_off[c] = off;
    r.wave_off[c] = waves;
    const int G = (1 << g0) << c;
    off += cls_count[c];
    if (cls_count[c] > 0) waves += (cls_count[c] + 64 / G - 1) / (64 / G);   // 64/G nets per wave
  }
  r.wave_off[kNumClasses] = waves;
  r.cls_off[kHeavy] = off;
  r.cls_off[kHeavy + 1] = off + cls_count[kHeavy];
  return r;
}

// Record slots under checkpointing (stride k > 0): a net of level l >= 1 belongs to
// segment (l-1)/k, which ends at level 1 + k*((l-1)/k + 1).  It is kept if a cell of a
// level at or past that end reads it, or if l = 0; kept nets get slots in canonical order
// (level-0 nets first, so their slot is their index), the other nets of a segment share the
// slots after them.  Without checkpointing slot = net.  Endpoints need no kept record: the
// forward takes their values while their segment is in the buffer, and the backward seeds
// them right before their segment (ep_grp).
// Sink workspace slots under checkpointing (see sta_graph::sink_base).  lvl: level of each
// canonical net.
static void build_sink_slots(sta_graph* g, const std::vector<int>& lvl) {
  const int N = g->N, P = g->P, k = g->ckpt_stride;
  auto seg = [&](int l) { return l == 0 ? -1 : (l - 1) / k; };
  std::vector<int> reader_level(P, -1);          // level of the cell reading each input pin
  for (int c = 0; c < g->C; ++c)
    for (int a = g->c_cin_off[c]; a < g->c_cin_off[c + 1]; ++a) reader_level[g->c_cin_pin[a]] = lvl[g->N0 + c];
  std::vector<char> is_ep(P, 0);
  for (int e : g->ep_pin) is_ep[e] = 1;
  std::vector<char> kept(N, 0);
  for (int n = 0; n < N; ++n) {
    const int l = lvl[n];
    for (int p = g->c_net_off[n] + 1; p < g->c_net_off[n + 1] && !kept[n]; ++p)
      if (l == 0 || (reader_level[p] < 0 ? !is_ep[p] : seg(reader_level[p]) != seg(l))) kept[n] = 1;
  }
  g->sink_base.assign(N, 0);
  int next = 0;
  for (int n = 0; n < N; ++n)
    if (kept[n]) {
      g->sink_base[n] = next;
      next += g->c_net_off[n + 1] - g->c_net_off[n] - 1;
    }
  const int kept_slots = next;
  int widest = 0;
  for (size_t j = 0; j + 1 < g->seg_lo.size(); ++j) {
    int t = 0;
    for (int n = g->level_off[g->seg_lo[j]]; n < g->level_off[g->seg_lo[j + 1]]; ++n)
      if (!kept[n]) {
        g->sink_base[n] = kept_slots + t;
        t += g->c_net_off[n + 1] - g->c_net_off[n] - 1;
      }
    widest = std::max(widest, t);
  }
  g->n_sslots_kept = kept_slots;
  g->n_sslots = std::max(1, kept_slots + widest);
  g->rc_seg.assign(N, -1);
  for (int n = 0; n < N; ++n)
    if (!kept[n]) g->rc_seg[n] = seg(lvl[n]);
  g->sslot.assign(P, 0);
  for (int n = 0; n < N; ++n)
    for (int p = g->c_net_off[n] + 1; p < g->c_net_off[n + 1]; ++p)
      g->sslot[p] = g->sink_base[n] + (p - g->c_net_off[n] - 1);
  g->ep_sslot.resize(g->ep_pin.size());
  for (size_t i = 0; i < g->ep_pin.size(); ++i) g->ep_sslot[i] = g->sslot[g->ep_pin[i]];
}

static void build_checkpoints(sta_graph* g) {
  const int N = g->N, L = g->L, k = g->ckpt_stride;
  g->seg_lo.clear();
  g->sink_base.clear();
  g->sslot.clear();
  g->ep_sslot.clear();
  g->ep_grp.clear();
  g->ep_grp_off.clear();
  g->rc_seg.clear();
  g->n_sslots = g->n_sslots_kept = 0;
  if (k <= 0) {
    g->rec_loc.clear();
    g->n_rec = g->n_kept = N;
    g->ep_rec = g->ep_net;
    return;
  }
  for (int l = 1; l < L; l += k) g->seg_lo.push_back(l);
  g->seg_lo.push_back(std::max(L, 1));
  std::vector<int> lvl(N), maxc(N, -1);
  for (int l = 0; l < L; ++l)
    for (int n = g->level_off[l]; n < g->level_off[l + 1]; ++n) lvl[n] = l;
  for (int c = 0; c < g->C; ++c) {
    const int lc = lvl[g->N0 + c];
    for (int a = g->c_cin_off[c]; a < g->c_cin_off[c + 1]; ++a)
      maxc[g->c_cin_src[a]] = std::max(maxc[g->c_cin_src[a]], lc);
  }
  std::vector<char> kept(N, 0);
  for (int n = 0; n < N; ++n) {
    const int l = lvl[n];
    if (l == 0 || maxc[n] >= 1 + k * ((l - 1) / k + 1)) kept[n] = 1;
  }
  g->rec_loc.assign(N, 0);
  int nk = 0;
  for (int n = 0; n < N; ++n)
    if (kept[n]) g->rec_loc[n] = nk++;
  int widest = 0;
  for (size_t j = 0; j + 1 < g->seg_lo.size(); ++j) {
    int t = 0;
    for (int n = g->level_off[g->seg_lo[j]]; n < g->level_off[g->seg_lo[j + 1]]; ++n)
      if (!kept[n]) g->rec_loc[n] = nk + t++;
    widest = std::max(widest, t);
  }
  g->n_kept = nk;
  g->n_rec = nk + widest;
  g->ep_rec.resize(g->ep_net.size());
  for (size_t i = 0; i < g->ep_net.size(); ++i) g->ep_rec[i] = g->rec_loc[g->ep_net[i]];
  // Endpoints grouped by their net: group 0 the level-0 nets' (kept records and slots),
  // group 1 + j segment j's; ascending endpoint index within a group.
  const int n_seg = (int)g->seg_lo.size() - 1;
  g->ep_grp_off.assign((size_t)n_seg + 2, 0);
  auto grp = [&](int i) { const int l = lvl[g->ep_net[i]]; return l == 0 ? 0 : 1 + (l - 1) / k; };
  for (size_t i = 0; i < g->ep_net.size(); ++i) ++g->ep_grp_off[(size_t)grp((int)i) + 1];
  for (int j = 0; j <= n_seg; ++j) g->ep_grp_off[(size_t)j + 1] += g->ep_grp_off[(size_t)j];
  g->ep_grp.assign(g->ep_net.size(), 0);
  std::vector<int> fill(g->ep_grp_off.begin(), g->ep_grp_off.end() - 1);
  for (size_t i = 0; i < g->ep_net.size(); ++i) g->ep_grp[(size_t)fill[(size_t)grp((int)i)]++] = (int)i;
  if (g->c_parent.empty()) build_sink_slots(g, lvl);
}

// Lane-group work lists: per-level ranges for the level kernels and all nets ordered by
// class for the one-pass kernels.  Depends on the schedule only.
void build_groups(sta_graph* g) {
  const int N = g->N;
  std::vector<int> cls(N);
  for (int n = 0; n < N; ++n)
    cls[n] = net_class(g->c_net_off[n + 1] - g->c_net_off[n] - 1, g->sched_cfg.sweep_group_log2,
                       g->sched_cfg.heavy_sinks);
  // Within a level, canonical nets are sorted by size, so classes are contiguous ranges and
  // a level's GroupRange indexes canonical net ids directly.
  g->lvl_ranges.assign(g->L, GroupRange{});
  for (int l = 0; l < g->L; ++l) {
    int b = g->level_off[l], e = g->level_off[l + 1];
    int cnt[kNumClasses + 1] = {0, 0, 0, 0, 0, 0};
    for (int n = b; n < e; ++n) cnt[cls[n]]++;
    g->lvl_ranges[l] = group_range(cnt, b, g->sched_cfg.sweep_group_log2);
  }
  for (int n = 0; n < N; ++n)
    cls[n] = net_class(g->c_net_off[n + 1] - g->c_net_off[n] - 1, g->sched_cfg.flat_group_log2,
                       g->sched_cfg.heavy_sinks);
  int cnt[kNumClasses + 1] = {0, 0, 0, 0, 0, 0};
  for (int n = 0; n < N; ++n) cnt[cls[n]]++;
  int pos[kNumClasses + 1];
  int o = 0;
  for (int c = 0; c <= kNumClasses; ++c) { pos[c] = o; o += cnt[c]; }
  g->sched_all.assign(N, 0);
  for (int n = 0; n < N; ++n) g->sched_all[pos[cls[n]]++] = n;
  g->all_range = group_range(cnt, 0, g->sched_cfg.flat_group_log2);
  // RC passes under checkpointing: kept nets, then each segment's other nets, by class.
  g->rc_sched.clear();
  g->rc_ranges.clear();
  if (!g->rc_seg.empty()) {
    const int n_pass = (int)g->seg_lo.size();      // kept nets, then one pass per segment
    std::vector<std::vector<int>> by(n_pass * (kNumClasses + 1));
    for (int n = 0; n < N; ++n) by[(g->rc_seg[n] + 1) * (kNumClasses + 1) + cls[n]].push_back(n);
    for (int j = 0; j < n_pass; ++j) {
      int pc[kNumClasses + 1];
      const int base = (int)g->rc_sched.size();
      for (int c = 0; c <= kNumClasses; ++c) {
        const std::vector<int>& v = by[j * (kNumClasses + 1) + c];
        pc[c] = (int)v.size();
        g->rc_sched.insert(g->rc_sched.end(), v.begin(), v.end());
      }
      g->rc_ranges.push_back(group_range(pc, base, g->sched_cfg.flat_group_log2));
    }
  }
  // Snapshot-inner layout: each level's nets of more than kSiHeavy sinks (a suffix of the
  // level, whose nets ascend in pin count) and the list of all of them.
  g->si_heavy.clear();
  g->si_huge.clear();
  g->si_hs.assign(g->L, 0);
  g->si_us.assign(g->L, 0);
  auto sinks = [&](int n) { return g->c_net_off[n + 1] - g->c_net_off[n] - 1; };
  for (int l = 0; l < g->L; ++l) {
    int u = g->level_off[l + 1];
    while (u > g->level_off[l] && sinks(u - 1) > kSiHuge) --u;
    int h = u;
    while (h > g->level_off[l] && sinks(h - 1) > kSiHeavy) --h;
    g->si_hs[l] = h;
    g->si_us[l] = u;
    for (int n = h; n < u; ++n) g->si_heavy.push_back(n);
    for (int n = u; n < g->level_off[l + 1]; ++n) g->si_huge.push_back(n);
  }
}

// Record slots and the cell inputs in a padded slot layout per level: input j of the k-th
// cell of level l is entry ell_base[l] + j * (cells of l) + k; missing inputs hold source -1.
void build_ell(sta_graph* g) {
  build_checkpoints(g);
  g->ell.clear();
  g->ell_base.assign(g->L, 0);
  g->ell_slots.assign(g->L, 0);
  for (int l = 1; l < g->L; ++l) {
    const int c0 = g->level_off[l] - g->N0, c1 = g->level_off[l + 1] - g->N0, nc = c1 - c0;
    int F = 1;
    for (int c = c0; c < c1; ++c) F = std::max(F, g->c_cin_off[c + 1] - g->c_cin_off[c]);
    g->ell_base[l] = (int)g->ell.size();
    g->ell_slots[l] = F;
    g->ell.resize(g->ell.size() + (size_t)F * nc, make_int4(-1, 0, 0, 0));
    for (int c = c0; c < c1; ++c)
      for (int j = 0; j < g->c_cin_off[c + 1] - g->c_cin_off[c]; ++j) {
        // {source net, input pin, arc with the sign bit set for negative unateness, the
        // input pin's sink workspace slot}
        const int4 e = g->c_cin[g->c_cin_off[c] + j];
        g->ell[g->ell_base[l] + (size_t)j * nc + (c - c0)] =
            make_int4(e.x, e.y, (int)((uint32_t)e.z | (e.w < 0 ? 0x80000000u : 0u)), g->sslot.empty() ? e.y : g->sslot[e.y]);
      }
  }
  if (g->ckpt_stride > 0)
    for (int4& e : g->ell)
      if (e.x >= 0) e.x = g->rec_loc[e.x];      // sources addressed by record slot
  if (g->ell.empty()) g->ell.push_back(make_int4(-1, 0, 0, 0));
}

void build_schedule(sta_graph* g) {
  build_ell(g);
  build_groups(g);
}

void drop_captured(sta_graph* g) {
  for (sta_graph::Captured* c : {&g->cap_fwd, &g->cap_bwd}) {
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    *c = sta_graph::Captured{};
  }
}

void free_device(sta_graph* g) {
  drop_captured(g);
  if (g->cap_stream) {
    (void)hipStreamDestroy(g->cap_stream);
    g->cap_stream = nullptr;
  }
  if (g->dev.device >= 0) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(g->dev.device);
    for (void* p : g->dev.allocs) (void)hipFree(p);
    if (cur >= 0) (void)hipSetDevice(cur);
  }
  g->dev = DeviceGraph{};
  g->uploaded = false;
}

}  // namespace sta

using namespace sta;
namespace sta { void free_device(sta_graph* g); }

extern "C" {

const char* sta_last_error(void) { return g_last_error.c_str(); }

int32_t sta_version(void) { return STA_ABI_VERSION; }

sta_status sta_build_graph(const sta_netlist* nl, const sta_library* lib, const sta_constraints* cons,
                           sta_graph** out) {
  if (!out) return fail(STA_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!nl || !lib || !cons) return fail(STA_E_INVALID, "NULL netlist, library or constraints");
  const int P = nl->n_pins, N = nl->n_nets, C = nl->n_cells, T = lib->n_cell_types;
  if (P <= 0 || N <= 0 || C < 0 || T <= 0) return fail(STA_E_INVALID, "sizes must be positive");
  if (!nl->net_offsets || !nl->net_pins || !nl->pin_cap || !nl->pin_kind ||
      (C > 0 && (!nl->cell_type || !nl->cell_in_offsets || !nl->cell_in_pins || !nl->cell_out_pin)))
    return fail(STA_E_INVALID, "NULL netlist array");
  if (!lib->arc_offsets || !lib->arc_unate || !lib->slew_axis || !lib->load_axis || !lib->tables)
    return fail(STA_E_INVALID, "NULL library array");
  // Library.
  if (lib->arc_offsets[0] != 0) return fail(STA_E_INVALID, "arc_offsets[0] must be 0");
  for (int t = 0; t < T; ++t) {
    int k = lib->arc_offsets[t + 1] - lib->arc_offsets[t];
    if (k < 1 || k > STA_MAX_FANIN) return fail(STA_E_INVALID, "cell type arc count out of 1..STA_MAX_FANIN");
  }
  const int n_arcs = lib->arc_offsets[T];
  for (int a = 0; a < n_arcs; ++a)
    if (lib->arc_unate[a] != 1 && lib->arc_unate[a] != -1) return fail(STA_E_INVALID, "arc_unate must be +1 or -1");
  for (int i = 0; i + 1 < STA_LUT_N; ++i)
    if (!(lib->slew_axis[i] < lib->slew_axis[i + 1]) || !(lib->load_axis[i] < lib->load_axis[i + 1]))
      return fail(STA_E_INVALID, "table axes must be strictly increasing");
  for (size_t i = 0; i < (size_t)n_arcs * 4 * STA_LUT_N * STA_LUT_N; ++i)
    if (!std::isfinite(lib->tables[i])) return fail(STA_E_INVALID, "non-finite table entry");
  // Nets: CSR, one driver first, every pin exactly once.
  if (nl->net_offsets[0] != 0 || nl->net_offsets[N] != P) return fail(STA_E_INVALID, "net_offsets must span 0..n_pins");
  for (int n = 0; n < N; ++n)
    if (nl->net_offsets[n + 1] <= nl->net_offsets[n]) return fail(STA_E_INVALID, "empty net or non-monotone net_offsets");
  if (C > 0) {
    if (nl->cell_in_offsets[0] != 0) return fail(STA_E_INVALID, "cell_in_offsets[0] must be 0");
    for (int c = 0; c < C; ++c)
      if (nl->cell_in_offsets[c + 1] <= nl->cell_in_offsets[c]) return fail(STA_E_INVALID, "cell without inputs or non-monotone cell_in_offsets");
  }
  std::vector<int> net_of_pin(P, -1);
  for (int n = 0; n < N; ++n) {
    int b = nl->net_offsets[n], e = nl->net_offsets[n + 1];
    if (e - b < 1) return fail(STA_E_INVALID, "empty net or non-monotone net_offsets");
    for (int i = b; i < e; ++i) {
      int p = nl->net_pins[i];
      if (p < 0 || p >= P) return fail(STA_E_INVALID, "net pin index out of range");
      if (net_of_pin[p] != -1) return fail(STA_E_INVALID, "pin listed in more than one net");
      net_of_pin[p] = n;
      int k = nl->pin_kind[p];
      bool drv = (k == STA_PIN_PI || k == STA_PIN_CELL_OUT);
      if (k < 0 || k > STA_PIN_PO) return fail(STA_E_INVALID, "bad pin kind");
      if ((i == b) != drv) return fail(STA_E_INVALID, "net must have exactly one driver (PI or cell output), listed first");
    }
  }
  for (int p = 0; p < P; ++p) {
    if (net_of_pin[p] < 0) return fail(STA_E_INVALID, "pin in no net");
    if (!std::isfinite(nl->pin_cap[p]) || nl->pin_cap[p] < 0) return fail(STA_E_INVALID, "pin capacitance must be finite and >= 0");
  }
  // Cells: kinds and counts consistent with the library.
  if (C > 0) {
    if (nl->cell_in_offsets[0] != 0) return fail(STA_E_INVALID, "cell_in_offsets[0] must be 0");
    std::vector<int8_t> used(P, 0);
    for (int c = 0; c < C; ++c) {
      int t = nl->cell_type[c];
      if (t < 0 || t >= T) return fail(STA_E_INVALID, "cell type out of range");
      int b = nl->cell_in_offsets[c], e = nl->cell_in_offsets[c + 1];
      if (e - b != lib->arc_offsets[t + 1] - lib->arc_offsets[t])
        return fail(STA_E_INVALID, "cell input count differs from its type's arc count");
      for (int i = b; i < e; ++i) {
        int p = nl->cell_in_pins[i];
        if (p < 0 || p >= P) return fail(STA_E_INVALID, "cell input pin out of range");
        if (nl->pin_kind[p] != STA_PIN_CELL_IN || used[p]) return fail(STA_E_INVALID, "cell input must be an unused CELL_IN pin");
        used[p] = 1;
      }
      int o = nl->cell_out_pin[c];
      if (o < 0 || o >= P) return fail(STA_E_INVALID, "cell output pin out of range");
      if (nl->pin_kind[o] != STA_PIN_CELL_OUT || used[o]) return fail(STA_E_INVALID, "cell output must be an unused CELL_OUT pin");
      used[o] = 1;
    }
    for (int p = 0; p < P; ++p) {
      int k = nl->pin_kind[p];
      if ((k == STA_PIN_CELL_IN || k == STA_PIN_CELL_OUT) && !used[p])
        return fail(STA_E_INVALID, "cell pin not attached to any cell");
    }
  } else {
    for (int p = 0; p < P; ++p)
      if (nl->pin_kind[p] == STA_PIN_CELL_IN || nl->pin_kind[p] == STA_PIN_CELL_OUT)
        return fail(STA_E_INVALID, "cell pin without cells");
  }
  // RC trees: a parent inside the pin's own net, none at the driver, no cycle.
  if (nl->pin_parent) {
    std::vector<int> depth(P, -1);
    std::vector<int> stack;
    for (int n = 0; n < N; ++n) {
      const int b = nl->net_offsets[n], e = nl->net_offsets[n + 1];
      if (nl->pin_parent[nl->net_pins[b]] != -1) return fail(STA_E_INVALID, "pin_parent of a driver must be -1");
      depth[nl->net_pins[b]] = 0;
      for (int i = b + 1; i < e; ++i) {
        const int p = nl->net_pins[i], q = nl->pin_parent[p];
        if (q < 0 || q >= P || net_of_pin[q] != n || q == p)
          return fail(STA_E_INVALID, "pin_parent must be another pin of the same net");
      }
      for (int i = b + 1; i < e; ++i) {        // walk up to a pin of known depth
        int p = nl->net_pins[i];
        stack.clear();
        while (depth[p] < 0) {
          stack.push_back(p);
          if ((int)stack.size() > e - b) return fail(STA_E_INVALID, "pin_parent has a cycle");
          p = nl->pin_parent[p];
        }
        for (int j = (int)stack.size() - 1; j >= 0; --j) depth[stack[j]] = depth[nl->pin_parent[stack[j]]] + 1;
      }
    }
  }
  if (!(std::isfinite(cons->t_clk) && std::isfinite(cons->pi_slew) && cons->pi_slew >= 0 &&
        cons->r_per_um >= 0 && cons->c_per_um >= 0))
    return fail(STA_E_INVALID, "bad constraints");

  sta_graph* g = new (std::nothrow) sta_graph();
  if (!g) return fail(STA_E_NOMEM, "host allocation failed");
  try {
    const int A = C > 0 ? nl->cell_in_offsets[C] : 0;
    g->P = P; g->N = N; g->C = C; g->A = A; g->T = T; g->n_arcs = n_arcs;
    g->net_off.assign(nl->net_offsets, nl->net_offsets + N + 1);
    g->net_pins.assign(nl->net_pins, nl->net_pins + P);
    g->pin_cap.assign(nl->pin_cap, nl->pin_cap + P);
    g->pin_kind.assign(nl->pin_kind, nl->pin_kind + P);
    if (nl->pin_parent) g->pin_parent.assign(nl->pin_parent, nl->pin_parent + P);
    if (C > 0) {
      g->cell_type.assign(nl->cell_type, nl->cell_type + C);
      g->cell_in_off.assign(nl->cell_in_offsets, nl->cell_in_offsets + C + 1);
      g->cell_in_pins.assign(nl->cell_in_pins, nl->cell_in_pins + A);
      g->cell_out_pin.assign(nl->cell_out_pin, nl->cell_out_pin + C);
    } else {
      g->cell_in_off.assign(1, 0);
    }
    g->arc_off.assign(lib->arc_offsets, lib->arc_offsets + T + 1);
    g->unate.assign(lib->arc_unate, lib->arc_unate + n_arcs);
    g->slew_axis.assign(lib->slew_axis, lib->slew_axis + STA_LUT_N);
    g->load_axis.assign(lib->load_axis, lib->load_axis + STA_LUT_N);
    g->tables.assign(lib->tables, lib->tables + (size_t)n_arcs * 4 * STA_LUT_N * STA_LUT_N);
    g->cons = *cons;
    g->design_pin_off = {0, P};
  } catch (const std::bad_alloc&) {
    delete g;
    return fail(STA_E_NOMEM, "host allocation failed");
  }
  *out = g;
  return STA_OK;
}

sta_status sta_batch_create(sta_graph* const* graphs, int32_t n, sta_graph** out) {
  if (!out) return fail(STA_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!graphs || n < 1) return fail(STA_E_INVALID, "need at least one graph");
  for (int d = 0; d < n; ++d)
    if (!graphs[d]) return fail(STA_E_INVALID, "NULL graph in batch");
  const sta_graph* g0 = graphs[0];
  for (int d = 1; d < n; ++d) {
    const sta_graph* h = graphs[d];
    if (std::memcmp(&h->cons, &g0->cons, sizeof(sta_constraints)) != 0)
      return fail(STA_E_INVALID, "batched graphs must share constraints and wire model");
    if (h->slew_axis != g0->slew_axis || h->load_axis != g0->load_axis)
      return fail(STA_E_INVALID, "batched graphs must share table axes");
  }
  sta_graph* u = new (std::nothrow) sta_graph();
  if (!u) return fail(STA_E_NOMEM, "host allocation failed");
  try {
    u->cons = g0->cons;
    u->slew_axis = g0->slew_axis;
    u->load_axis = g0->load_axis;
    u->n_designs = n;
    u->design_pin_off.assign(n + 1, 0);
    u->arc_off.assign(1, 0);
    // Libraries: identical libraries are stored once.
    std::vector<int> type_base(n, 0);
    std::vector<int> lib_owner;   // design whose library each stored library is
    for (int d = 0; d < n; ++d) {
      const sta_graph* h = graphs[d];
      int found = -1;
      for (int o : lib_owner) {
        const sta_graph* q = graphs[o];
        if (q->arc_off == h->arc_off && q->unate == h->unate && q->tables == h->tables) {
          found = o;
          break;
        }
      }
      if (found >= 0) {
        type_base[d] = type_base[found];
        continue;
      }
      lib_owner.push_back(d);
      type_base[d] = u->T;
      const int arc_base = u->n_arcs;
      for (int t = 0; t < h->T; ++t) u->arc_off.push_back(arc_base + h->arc_off[t + 1]);
      u->unate.insert(u->unate.end(), h->unate.begin(), h->unate.end());
      u->tables.insert(u->tables.end(), h->tables.begin(), h->tables.end());
      u->T += h->T;
      u->n_arcs += h->n_arcs;
    }
    // Netlists, ids offset design by design.
    bool any_tree = false;
    for (int d = 0; d < n; ++d) any_tree = any_tree || !graphs[d]->pin_parent.empty();
    u->net_off.assign(1, 0);
    u->cell_in_off.assign(1, 0);
    for (int d = 0; d < n; ++d) {
      const sta_graph* h = graphs[d];
      const int pb = u->P, ab = u->A;
      u->design_pin_off[d] = pb;
      for (int i = 0; i < h->N; ++i) u->net_off.push_back(pb + h->net_off[i + 1]);
      for (int q = 0; q < h->P; ++q) u->net_pins.push_back(pb + h->net_pins[q]);
      u->pin_cap.insert(u->pin_cap.end(), h->pin_cap.begin(), h->pin_cap.end());
      u->pin_kind.insert(u->pin_kind.end(), h->pin_kind.begin(), h->pin_kind.end());
      for (int c = 0; c < h->C; ++c) {
        u->cell_type.push_back(type_base[d] + h->cell_type[c]);
        u->cell_in_off.push_back(ab + h->cell_in_off[c + 1]);
        u->cell_out_pin.push_back(pb + h->cell_out_pin[c]);
      }
      for (int i = 0; i < h->A; ++i) u->cell_in_pins.push_back(pb + h->cell_in_pins[i]);
      if (any_tree) {                           // star members join as depth-one trees
        for (int q = 0; q < h->P; ++q) u->pin_parent.push_back(-1);
        for (int i = 0; i < h->N; ++i)
          for (int q = h->net_off[i] + 1; q < h->net_off[i + 1]; ++q) {
            const int p = h->net_pins[q];
            u->pin_parent[pb + p] = pb + (h->pin_parent.empty() ? h->net_pins[h->net_off[i]] : h->pin_parent[p]);
          }
      }
      u->P += h->P;
      u->N += h->N;
      u->C += h->C;
      u->A += h->A;
    }
    u->design_pin_off[n] = u->P;
  } catch (const std::bad_alloc&) {
    delete u;
    return fail(STA_E_NOMEM, "host allocation failed");
  }
  *out = u;
  return STA_OK;
}

sta_status sta_batch_pin_map(const sta_graph* g, int32_t* design, int32_t* pin) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  if (!g->levelized) return fail(STA_E_STATE, "graph is not levelized");
  for (int q = 0; q < g->P; ++q) {
    const int orig = g->pin_perm[q];
    const int d = (int)(std::upper_bound(g->design_pin_off.begin(), g->design_pin_off.end(), orig) -
                        g->design_pin_off.begin()) - 1;
    if (design) design[q] = d;
    if (pin) pin[q] = orig - g->design_pin_off[d];
  }
  return STA_OK;
}

sta_status sta_levelize(sta_graph* g, int32_t* n_levels_out) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  if (g->levelized) {
    if (n_levels_out) *n_levels_out = g->L;
    return STA_OK;
  }
  try {
    const int P = g->P, N = g->N, C = g->C;
    std::vector<int> net_of_pin(P);
    for (int n = 0; n < N; ++n)
      for (int i = g->net_off[n]; i < g->net_off[n + 1]; ++i) net_of_pin[g->net_pins[i]] = n;
    std::vector<int> cell_of_out(P, -1);
    for (int c = 0; c < C; ++c) cell_of_out[g->cell_out_pin[c]] = c;
    std::vector<int> cell_of_net(N, -1);
    for (int n = 0; n < N; ++n) cell_of_net[n] = cell_of_out[g->net_pins[g->net_off[n]]];
    // Successor lists of the net DAG (m -> n when a sink of m is an input of n's cell).
    std::vector<int> indeg(N, 0), succ_off(N + 1, 0);
    for (int n = 0; n < N; ++n) {
      int c = cell_of_net[n];
      if (c < 0) continue;
      for (int i = g->cell_in_off[c]; i < g->cell_in_off[c + 1]; ++i) {
        succ_off[net_of_pin[g->cell_in_pins[i]] + 1]++;
        indeg[n]++;
      }
    }
    for (int n = 0; n < N; ++n) succ_off[n + 1] += succ_off[n];
    std::vector<int> succ(succ_off[N]), fill(succ_off.begin(), succ_off.end() - 1);
    for (int n = 0; n < N; ++n) {
      int c = cell_of_net[n];
      if (c < 0) continue;
      for (int i = g->cell_in_off[c]; i < g->cell_in_off[c + 1]; ++i)
        succ[fill[net_of_pin[g->cell_in_pins[i]]]++] = n;
    }
    // Kahn frontiers: a net is placed once all its predecessors are.
    std::vector<int> level(N, 0), frontier, next;
    for (int n = 0; n < N; ++n)
      if (indeg[n] == 0) frontier.push_back(n);
    int placed = 0;
    while (!frontier.empty()) {
      next.clear();
      for (int m : frontier) {
        ++placed;
        for (int i = succ_off[m]; i < succ_off[m + 1]; ++i) {
          int n = succ[i];
          level[n] = std::max(level[n], level[m] + 1);
          if (--indeg[n] == 0) next.push_back(n);
        }
      }
      frontier.swap(next);
    }
    if (placed != N) return fail(STA_E_CYCLE, "combinational cycle: " + std::to_string(N - placed) + " nets never become ready");
    int L = 0;
    for (int n = 0; n < N; ++n) L = std::max(L, level[n] + 1);
    // Canonical net order: (level, pins of the net, original id).  Sorting by size inside
    // a level makes each lane-group class a contiguous range of the level.
    std::vector<int> lcount(L + 1, 0);
    for (int n = 0; n < N; ++n) lcount[level[n] + 1]++;
    for (int l = 0; l < L; ++l) lcount[l + 1] += lcount[l];
    g->level_off = lcount;
    g->net_perm.resize(N);
    std::iota(g->net_perm.begin(), g->net_perm.end(), 0);
    std::stable_sort(g->net_perm.begin(), g->net_perm.end(), [&](int a, int b) {
      if (level[a] != level[b]) return level[a] < level[b];
      return g->net_off[a + 1] - g->net_off[a] < g->net_off[b + 1] - g->net_off[b];
    });
    std::vector<int> net_new(N);
    for (int i = 0; i < N; ++i) net_new[g->net_perm[i]] = i;
    // Canonical pins, net by net.
    g->pin_perm.assign(P, 0);
    g->c_net_off.assign(N + 1, 0);
    std::vector<int> pin_new(P);
    int k = 0;
    for (int i = 0; i < N; ++i) {
      int n = g->net_perm[i];
      g->c_net_off[i] = k;
      for (int q = g->net_off[n]; q < g->net_off[n + 1]; ++q) {
        g->pin_perm[k] = g->net_pins[q];
        pin_new[g->net_pins[q]] = k;
        ++k;
      }
    }
    g->c_net_off[N] = P;
    g->c_pin_cap.resize(P);
    for (int i = 0; i < P; ++i) g->c_pin_cap[i] = g->pin_cap[g->pin_perm[i]];
    // RC trees in canonical ids, and each net's pins in breadth-first order from its driver.
    g->c_parent.clear();
    g->c_tree_order.clear();
    if (!g->pin_parent.empty()) {
      g->c_parent.resize(P);
      for (int q = 0; q < P; ++q) {
        const int pp = g->pin_parent[g->pin_perm[q]];
        g->c_parent[q] = pp < 0 ? -1 : pin_new[pp];
      }
      g->c_tree_order.resize(P);
      std::vector<int> child_off, child;
      for (int i = 0; i < N; ++i) {
        const int b = g->c_net_off[i], e = g->c_net_off[i + 1];
        child_off.assign(e - b + 1, 0);
        for (int q = b + 1; q < e; ++q) ++child_off[g->c_parent[q] - b + 1];
        for (int j = 0; j < e - b; ++j) child_off[j + 1] += child_off[j];
        child.assign(e - b, 0);
        std::vector<int> fill(child_off.begin(), child_off.end() - 1);
        for (int q = b + 1; q < e; ++q) child[fill[g->c_parent[q] - b]++] = q;
        int head = b, tail = b;
        g->c_tree_order[tail++] = b;
        while (head < tail) {
          const int u = g->c_tree_order[head++];
          for (int j = child_off[u - b]; j < child_off[u - b + 1]; ++j) g->c_tree_order[tail++] = child[j];
        }
      }
      // Per pin: depth, and its children as a run of breadth-first positions.
      g->c_tree_node.assign(P, make_int4(0, 0, 0, 0));
      for (int i = 0; i < N; ++i) {
        const int b = g->c_net_off[i], e = g->c_net_off[i + 1];
        int next = b + 1;                        // children of the j-th pin in order follow
        for (int j = b; j < e; ++j) {
          const int u = g->c_tree_order[j];
          int4& t = g->c_tree_node[u];
          t.x = u == b ? 0 : g->c_tree_node[g->c_parent[u]].x + 1;
          t.y = next;
          while (next < e && g->c_parent[g->c_tree_order[next]] == u) ++next;
          t.z = next - t.y;
        }
      }
      // Chunks of whole nets for the LDS kernels (depth -1: a net too big for one, left to the
      // fallback kernel).
      g->tree_blk_net.assign(1, 0);
      g->tree_blk_depth.clear();
      g->tree_big.clear();
      int pins = 0, depth = 0;
      for (int i = 0; i < N; ++i) {
        const int np = g->c_net_off[i + 1] - g->c_net_off[i];
        int dn = 0;
        for (int q = g->c_net_off[i]; q < g->c_net_off[i + 1]; ++q) dn = std::max(dn, g->c_tree_node[q].x);
        if (np > kTreeChunk) {
          if (i > g->tree_blk_net.back()) {
            g->tree_blk_depth.push_back(depth);
            g->tree_blk_net.push_back(i);
          }
          g->tree_big.push_back(i);
          g->tree_blk_depth.push_back(-1);
          g->tree_blk_net.push_back(i + 1);
          pins = depth = 0;
          continue;
        }
        if (pins + np > kTreeChunk) {
          g->tree_blk_depth.push_back(depth);
          g->tree_blk_net.push_back(i);
          pins = depth = 0;
        }
        pins += np;
        depth = std::max(depth, dn);
      }
      if (N > g->tree_blk_net.back()) {
        g->tree_blk_depth.push_back(depth);
        g->tree_blk_net.push_back(N);
      }
    }
    // Level 0 holds exactly the PI-driven nets; every later net is driven by a cell.
    const int N0 = lcount[1];
    for (int i = 0; i < N; ++i) {
      bool pi = g->pin_kind[g->net_pins[g->net_off[g->net_perm[i]]]] == STA_PIN_PI;
      if (pi != (i < N0)) return fail(STA_E_INVALID, "a primary input drives a net that also has a cell driver");
    }
    g->N0 = N0;
    // Canonical cells: cell c drives canonical net N0 + c.
    const int Cc = N - N0;
    if (Cc != C) return fail(STA_E_INVALID, "every cell must drive exactly one net");
    g->c_cell_type.assign(C, 0);
    g->c_cin_off.assign(C + 1, 0);
    g->c_cin_src.assign(g->A, 0);
    g->c_cin_pin.assign(g->A, 0);
    g->c_cin.clear();
    g->c_cin.reserve(g->A);
    int a = 0;
    for (int cc = 0; cc < C; ++cc) {
      int c = cell_of_net[g->net_perm[N0 + cc]];
      g->c_cell_type[cc] = g->cell_type[c];
      g->c_cin_off[cc] = a;
      for (int i = g->cell_in_off[c]; i < g->cell_in_off[c + 1]; ++i) {
        int p = g->cell_in_pins[i];
        g->c_cin_pin[a] = pin_new[p];
        g->c_cin_src[a] = net_new[net_of_pin[p]];
        const int arc = g->arc_off[g->cell_type[c]] + (i - g->cell_in_off[c]);
        g->c_cin.push_back(make_int4(g->c_cin_src[a], g->c_cin_pin[a], arc, (int)g->unate[arc]));
        ++a;
      }
    }
    g->c_cin_off[C] = a;
    // Endpoints in canonical order, grouped by design.
    g->ep_pin.clear();
    g->ep_net.clear();
    g->ep_design.clear();
    std::vector<std::vector<int>> ep_by_design(g->n_designs);
    for (int i = 0; i < N; ++i)
      for (int q = g->c_net_off[i] + 1; q < g->c_net_off[i + 1]; ++q) {
        const int orig = g->pin_perm[q];
        const int kd = g->pin_kind[orig];
        if (kd == STA_PIN_FF_D || kd == STA_PIN_PO) {
          const int dsg = (int)(std::upper_bound(g->design_pin_off.begin(), g->design_pin_off.end(), orig) -
                                g->design_pin_off.begin()) - 1;
          ep_by_design[dsg].push_back(q);
        }
      }
    std::vector<int> net_of_canon_pin(P);
    for (int i = 0; i < N; ++i)
      for (int q = g->c_net_off[i]; q < g->c_net_off[i + 1]; ++q) net_of_canon_pin[q] = i;
    g->ep_design_off.assign(g->n_designs + 1, 0);
    for (int dsg = 0; dsg < g->n_designs; ++dsg) {
      for (int q : ep_by_design[dsg]) {
        g->ep_pin.push_back(q);
        g->ep_net.push_back(net_of_canon_pin[q]);
        g->ep_design.push_back(dsg);
      }
      g->ep_design_off[dsg + 1] = (int)g->ep_pin.size();
    }
    g->E = (int)g->ep_pin.size();
    g->level = level;
    g->L = L;
    g->max_level_nets = 0;
    for (int l = 0; l < L; ++l) g->max_level_nets = std::max(g->max_level_nets, lcount[l + 1] - lcount[l]);
    build_schedule(g);
    compute_layouts(g);
    // The kernels address arrays through 32-bit byte offsets from their bases.
    const uint64_t lim = 1ull << 32;
    if (16ull * (uint64_t)P >= lim || 64ull * (uint64_t)N >= lim || 16ull * (uint64_t)g->ell.size() >= lim)
      return fail(STA_E_INVALID, "graph too large: a per-pin, per-net or per-input array reaches 4 GiB");
    g->levelized = true;
  } catch (const std::bad_alloc&) {
    return fail(STA_E_NOMEM, "host allocation failed");
  }
  if (n_levels_out) *n_levels_out = g->L;
  return STA_OK;
}

sta_status sta_get_levelization(const sta_graph* g, int32_t* level, int32_t* level_offsets, int32_t* net_perm,
                                int32_t* pin_perm) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  if (!g->levelized) return fail(STA_E_STATE, "graph is not levelized");
  if (level) std::copy(g->level.begin(), g->level.end(), level);
  if (level_offsets) std::copy(g->level_off.begin(), g->level_off.end(), level_offsets);
  if (net_perm) std::copy(g->net_perm.begin(), g->net_perm.end(), net_perm);
  if (pin_perm) std::copy(g->pin_perm.begin(), g->pin_perm.end(), pin_perm);
  return STA_OK;
}

sta_status sta_get_schedule(const sta_graph* g, sta_schedule* sch) {
  if (!g || !sch) return fail(STA_E_INVALID, "NULL argument");
  *sch = g->sched_cfg;
  return STA_OK;
}

sta_status sta_set_schedule(sta_graph* g, const sta_schedule* sch) {
  if (!g || !sch) return fail(STA_E_INVALID, "NULL argument");
  if (sch->sweep_group_log2 < 2 || sch->sweep_group_log2 > 6 || sch->flat_group_log2 < 2 ||
      sch->flat_group_log2 > 6 || sch->heavy_sinks < 1 || sch->heavy_sinks > 64 || sch->rc_scheme < STA_RC_GROUPS ||
      sch->rc_scheme > STA_RC_THREAD ||
      (sch->fwd_cell_lanes != 16 && sch->fwd_cell_lanes != 8 && sch->fwd_cell_lanes != 4) ||
      (sch->level_scheme != STA_LEVEL_GROUPS && sch->level_scheme != STA_LEVEL_THREAD &&
       sch->level_scheme != STA_LEVEL_CTE) ||
      (sch->lane_block != 256 && sch->lane_block != 512 && sch->lane_block != 1024))
    return fail(STA_E_INVALID, "schedule out of range");
  if (!g->levelized) return fail(STA_E_STATE, "graph is not levelized");
  if (sch->level_scheme != STA_LEVEL_GROUPS && (g->n_snap != 1 || g->snap_inner || g->ckpt_stride > 0 ||
                                                !g->c_parent.empty()))
    return fail(STA_E_INVALID, "one thread per net and the CTE level kernels need one snapshot, no checkpointing "
                               "and star nets");
  g->sched_cfg = *sch;
  try {
    build_groups(g);
  } catch (const std::bad_alloc&) {
    return fail(STA_E_NOMEM, "host allocation failed");
  }
  drop_captured(g);
  if (g->uploaded) {
    const std::vector<int>& sched = g->rc_sched.empty() ? g->sched_all : g->rc_sched;
    hipError_t e = hipMemcpy(g->dev.sched_all, sched.data(), sched.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  }
  return STA_OK;
}

sta_status sta_set_checkpointing(sta_graph* g, int32_t stride_levels) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  if (!g->levelized) return fail(STA_E_STATE, "graph is not levelized");
  int k = stride_levels;
  if (k < 0) k = std::max(1, (int)std::ceil(std::sqrt((double)std::max(1, g->L - 1))));
  if (k > 0 && (g->lanes_kernels() || g->sched_cfg.level_scheme != STA_LEVEL_GROUPS))
    return fail(STA_E_INVALID,
                "checkpointing is not available with STA_SNAP_INNER, one thread per net or the CTE level kernels");
  g->ckpt_stride = k;
  try {
    build_ell(g);
    build_groups(g);
    compute_layouts(g);
  } catch (const std::bad_alloc&) {
    return fail(STA_E_NOMEM, "host allocation failed");
  }
  free_device(g);
  return STA_OK;
}

sta_status sta_set_snapshots(sta_graph* g, int32_t n_snapshots) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  if (n_snapshots < 1 || n_snapshots > 65535) return fail(STA_E_INVALID, "snapshot count out of range");
  if (n_snapshots > 1 && g->sched_cfg.level_scheme != STA_LEVEL_GROUPS)
    return fail(STA_E_INVALID, "one thread per net and the CTE level kernels sweep one snapshot");
  g->n_snap = n_snapshots;
  drop_captured(g);
  return STA_OK;
}

sta_status sta_set_snapshot_layout(sta_graph* g, int32_t layout) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  if (layout != STA_SNAP_OUTER && layout != STA_SNAP_INNER) return fail(STA_E_INVALID, "unknown snapshot layout");
  if (!g->levelized) return fail(STA_E_STATE, "graph is not levelized");
  if (layout == STA_SNAP_INNER && g->ckpt_stride > 0)
    return fail(STA_E_INVALID, "STA_SNAP_INNER is not available with checkpointing");
  if (layout == STA_SNAP_INNER && !g->c_parent.empty())
    return fail(STA_E_INVALID, "STA_SNAP_INNER is not available for RC trees");
  if (layout == STA_SNAP_INNER && g->sched_cfg.level_scheme != STA_LEVEL_GROUPS)
    return fail(STA_E_INVALID, "STA_SNAP_INNER replaces the level schedule; set lane groups first");
  g->snap_inner = layout == STA_SNAP_INNER;
  drop_captured(g);
  return STA_OK;
}

sta_status sta_get_checkpointing(const sta_graph* g, int32_t* stride_levels, int32_t* record_slots,
                                 int32_t* kept_nets) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  if (!g->levelized) return fail(STA_E_STATE, "graph is not levelized");
  if (stride_levels) *stride_levels = g->ckpt_stride;
  if (record_slots) *record_slots = g->n_rec;
  if (kept_nets) *kept_nets = g->n_kept;
  return STA_OK;
}

sta_status sta_graph_info_get(const sta_graph* g, sta_graph_info* info) {
  if (!g || !info) return fail(STA_E_INVALID, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->n_pins = g->P;
  info->n_nets = g->N;
  info->n_cells = g->C;
  info->n_cell_inputs = g->A;
  info->n_endpoints = g->levelized ? g->E : 0;
  info->n_levels = g->levelized ? g->L : 0;
  info->n_pi_nets = g->levelized ? g->N0 : 0;
  info->max_level_nets = g->levelized ? g->max_level_nets : 0;
  info->fwd_state_bytes = g->levelized ? (int64_t)g->state.total * g->n_snap : 0;
  info->bwd_workspace_bytes = g->levelized ? (int64_t)g->work.total * g->n_snap : 0;
  info->device_bytes = g->uploaded ? (int64_t)g->dev.bytes : 0;
  info->n_designs = g->n_designs;
  info->n_snapshots = g->n_snap;
  return STA_OK;
}

void sta_graph_destroy(sta_graph* g) {
  if (!g) return;
  for (auto& t : g->timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (hipEvent_t e : g->event_pool) (void)hipEventDestroy(e);
  if (g->run_start) (void)hipEventDestroy(g->run_start);
  free_device(g);
  delete g;
}

sta_status sta_graph_upload(sta_graph* g) {
  if (!g) return fail(STA_E_INVALID, "graph is NULL");
  if (!g->levelized) return fail(STA_E_STATE, "graph is not levelized");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (g->uploaded) {
    if (g->dev.device == dev) return STA_OK;
    return fail(STA_E_STATE, "graph was uploaded to another device");
  }
  DeviceGraph& d = g->dev;
  d.device = dev;
  std::vector<float4> grid, coef;
  build_lut_coefficients(g, grid, coef);

  auto up = [&](auto*& dst, const auto& src) -> sta_status {
    using T = std::remove_reference_t<decltype(*dst)>;
    size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
    void* p = nullptr;
    hipError_t err = hipMalloc(&p, bytes);
    if (err != hipSuccess) return hip_fail(err, "hipMalloc");
    d.allocs.push_back(p);
    d.bytes += bytes;
    if (!src.empty()) {
      err = hipMemcpy(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
      if (err != hipSuccess) return hip_fail(err, "hipMemcpy");
    }
    dst = static_cast<T*>(p);
    return STA_OK;
  };
  sta_status s = STA_OK;
  if ((s = up(d.net_off, g->c_net_off)) || (s = up(d.pin_cap, g->c_pin_cap)) || (s = up(d.ell, g->ell)) ||
      (s = up(d.ep_pin, g->ep_pin)) || (s = up(d.ep_net, g->ep_rec)) || (s = up(d.pin_perm, g->pin_perm)) ||
      (s = up(d.ep_design, g->ep_design)) || (s = up(d.ep_design_off, g->ep_design_off)) ||
      (s = up(d.ep_blk_off, g->ep_blk_off)) ||
      (s = up(d.sched_all, g->rc_sched.empty() ? g->sched_all : g->rc_sched)) || (s = up(d.si_heavy, g->si_heavy)) || (s = up(d.si_huge, g->si_huge)) ||
      (!g->sink_base.empty() && ((s = up(d.sink_base, g->sink_base)) || (s = up(d.ep_sslot, g->ep_sslot)))) ||
      (g->ckpt_stride > 0 && ((s = up(d.rec_loc, g->rec_loc)) || (s = up(d.ep_grp, g->ep_grp)))) ||
      (!g->c_parent.empty() && ((s = up(d.parent, g->c_parent)) || (s = up(d.tree_order, g->c_tree_order)) ||
                                (s = up(d.tree_node, g->c_tree_node)) || (s = up(d.tree_blk_net, g->tree_blk_net)) ||
                                (s = up(d.tree_blk_depth, g->tree_blk_depth)) || (s = up(d.tree_big, g->tree_big)))) ||
      (s = up(d.lut_grid, grid)) || (s = up(d.lut_coef, coef))) {
    free_device(g);
    return s;
  }
  g->uploaded = true;
  return STA_OK;
}

}  // extern "C"
