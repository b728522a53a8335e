// Host runtime of catpc: context and workspace, validation, the batched and
// plain stage chains, hipGraph replay of the batched chain, late fetch.
// Public C ABI: include/catpc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/catpc.h"
#include "internal.h"

using namespace catpc;

namespace {

thread_local std::string g_err;

catpc_status fail(catpc_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

catpc_status hip_fail(hipError_t e, const char* what) {
  return fail(CATPC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                  \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return hip_fail(_e, #expr);  \
  } while (0)

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
  size_t row_first, hdr, bins, sorted, raw_up, raw_dn, mask, blk_sec, blk_cnt, blk_off, grp_off, start_glob, batch_off,
      chain,
      owner, sel_cnt, sel_local, sel_loc, sel_grp, sel_mask, mrec, mkey_a, mkey_b, mpair, mover, mslot, mchunk, counters;
  size_t total;
};

// Workspace layout; `hot_only` leaves out the arrays of the selection and the
// merging (the stage chain of the batched form never touches them).
Layout plan(int32_t R, int64_t H, int32_t S, bool hot_only = false) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t p = o; o += align_up(bytes); return p; };
  const size_t nblk = (size_t)(H / kHitsPerBlock) + 8;
  L.row_first = take(sizeof(int32_t) * (size_t)S * (R + 1));
  L.hdr = take(sizeof(RowHdr) * (size_t)S * R);
  L.bins = take(sizeof(int32_t) * (2 * (size_t)H + 2 * (size_t)S * R + 8));
  L.sorted = take(sizeof(SortedHit) * (size_t)(H + 1));
  L.raw_up = take(sizeof(int32_t) * (size_t)(H + 1));
  L.raw_dn = take(sizeof(int32_t) * (size_t)(H + 1));
  L.mask = take(sizeof(uint64_t) * (nblk * (kHitsPerBlock / 64) + 8));
  L.blk_sec = take(sizeof(int32_t) * (nblk + 8));
  L.blk_cnt = take(sizeof(int32_t) * (nblk + 8));
  L.blk_off = take(sizeof(int64_t) * (nblk + 8));
  L.grp_off = take(sizeof(int64_t) * (nblk / 1024 + 8));
  L.start_glob = take(sizeof(int32_t) * (size_t)(H + 1));
  L.batch_off = take(sizeof(int32_t) * ((size_t)S + 2));
  L.chain = take(sizeof(ChainHit) * (size_t)(H + 1));
  const size_t slots = hot_only ? 0 : (size_t)(H / 3) + 2;  // tracklets <= H/3: seeds are disjoint chains of >= 3 hits
  L.owner = take(hot_only ? 0 : sizeof(unsigned) * (size_t)(H + 1));
  L.sel_cnt = take(sizeof(int32_t) * slots);
  L.sel_local = take(sizeof(int32_t) * slots);
  L.sel_loc = take(sizeof(int2) * slots);
  L.sel_grp = take(hot_only ? 0 : sizeof(longlong2) * (slots / 1024 + 8));
  L.sel_mask = take(sizeof(uint16_t) * slots * (size_t)sel_chunks(R));
  L.mrec = take(sizeof(float4) * slots);
  L.mkey_a = take(sizeof(unsigned long long) * slots);
  L.mkey_b = take(sizeof(unsigned long long) * slots);
  L.mpair = take(sizeof(int2) * (size_t)kMergePairsPerSlot * slots);
  L.mover = take(sizeof(int32_t) * slots);
  L.mslot = take(sizeof(int32_t) * slots);
  L.mchunk = take(hot_only ? 0 : sizeof(int32_t) * ((size_t)S + 1));
  L.counters = take(sizeof(unsigned long long) * kNumCounters);
  L.total = o;
  return L;
}

// The workspace arrays of layout L inside the device block b.
Workspace carve(char* b, const Layout& L) {
  Workspace w;
  w.row_first = (int32_t*)(b + L.row_first);
  w.hdr = (RowHdr*)(b + L.hdr);
  w.bins = (int32_t*)(b + L.bins);
  w.sorted = (SortedHit*)(b + L.sorted);
  w.raw_up = (int32_t*)(b + L.raw_up);
  w.raw_dn = (int32_t*)(b + L.raw_dn);
  w.start_mask = (uint64_t*)(b + L.mask);
  w.blk_sec = (int32_t*)(b + L.blk_sec);
  w.blk_cnt = (int32_t*)(b + L.blk_cnt);
  w.blk_off = (int64_t*)(b + L.blk_off);
  w.grp_off = (int64_t*)(b + L.grp_off);
  w.start_glob = (int32_t*)(b + L.start_glob);
  w.batch_off = (int32_t*)(b + L.batch_off);
  w.chain = (ChainHit*)(b + L.chain);
  w.owner = (unsigned*)(b + L.owner);
  w.sel_cnt = (int32_t*)(b + L.sel_cnt);
  w.sel_local = (int32_t*)(b + L.sel_local);
  w.sel_loc = (int2*)(b + L.sel_loc);
  w.sel_grp = (longlong2*)(b + L.sel_grp);
  w.sel_mask = (uint16_t*)(b + L.sel_mask);
  w.mrec = (float4*)(b + L.mrec);
  w.mkey_a = (unsigned long long*)(b + L.mkey_a);
  w.mkey_b = (unsigned long long*)(b + L.mkey_b);
  w.mpair = (int2*)(b + L.mpair);
  w.mover = (int32_t*)(b + L.mover);
  w.mslot = (int32_t*)(b + L.mslot);
  w.mchunk = (int32_t*)(b + L.mchunk);
  w.counters = (unsigned long long*)(b + L.counters);
  return w;
}

// Arguments of the last captured batched chain; replay only if identical.
struct GraphKey {
  catpc_input in;
  catpc_output out;
  catpc_params params;
  catpc_tuning tuning;
  bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(GraphKey)) == 0; }
};

// Arguments of the last captured selection chain.
struct SelKey {
  catpc_input in;
  catpc_output trk;
  catpc_tracks out;
  int32_t min_hits;
  int32_t use_graph;
  bool operator==(const SelKey& o) const { return std::memcmp(this, &o, sizeof(SelKey)) == 0; }
};

}  // namespace

struct catpc_ctx {
  int device = 0;
  int n_cu = 256;
  int32_t n_rows = 0;
  int64_t max_hits = 0;
  int32_t max_sectors = 0;
  float* row_x = nullptr;  // device [n_rows]
  float4* rowk = nullptr;  // device [n_rows]: x_{r+1}/x_r, x_{r-1}/x_r, chord weight, 0 (binary32 divisions)
  catpc_params params{};
  catpc_tuning tuning{};
  Consts consts{};
  void* ws_mem = nullptr;
  Workspace ws{};
  unsigned long long* host_counters = nullptr;  // pinned [kNumCounters]
  int64_t* host_total = nullptr;                 // pinned [1]
  // last track call
  bool have_last = false;
  catpc_input last_in{};
  catpc_output last_out{};
  // graph cache
  bool have_graph = false;
  GraphKey key{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture_stream = nullptr;  // the batched chain is captured here, replayed on the caller's stream
  // last selection call and its graph
  bool have_sel = false;
  catpc_tracks sel_out{};
  bool have_sel_graph = false;
  SelKey sel_key{};
  hipGraph_t sel_graph = nullptr;
  hipGraphExec_t sel_exec = nullptr;
};

namespace {

Consts make_consts(const catpc_params& p) {
  Consts c;
  c.kb = -0.00299792458f * p.bz;
  c.sy2 = p.sigma_y * p.sigma_y;
  c.sz2 = p.sigma_z * p.sigma_z;
  c.wy = p.nf_win_y;
  c.wz = p.nf_win_z;
  c.chi2 = p.nf_chi2_max;
  c.nsig = p.tc_gate_nsigma;
  c.max_miss = p.tc_max_miss;
  c.min_hits = p.min_hits;
  c.precision = p.precision;
  c.sy2d = (double)p.sigma_y * (double)p.sigma_y;
  c.kbd = -0.00299792458 * (double)p.bz;
  c.sz2d = (double)p.sigma_z * (double)p.sigma_z;
  return c;
}

catpc_status check_params(const catpc_params* p) {
  if (!p) return fail(CATPC_E_INVALID, "params is NULL");
  if (!(p->sigma_y > 0) || !(p->sigma_z > 0)) return fail(CATPC_E_INVALID, "cluster errors must be > 0");
  if (!(p->nf_win_y >= 0) || !(p->nf_win_z >= 0) || !(p->nf_chi2_max >= 0) || !(p->tc_gate_nsigma >= 0))
    return fail(CATPC_E_INVALID, "windows and cuts must be >= 0");
  if (p->tc_max_miss < 0 || p->min_hits < 0) return fail(CATPC_E_INVALID, "tc_max_miss and min_hits must be >= 0");
  if (p->precision < 0 || p->precision > 2) return fail(CATPC_E_INVALID, "precision must be 0, 1 or 2");
  return CATPC_OK;
}

catpc_status check_tuning(const catpc_tuning* t) {
  if (!(t->bin_hits >= 0.25f && t->bin_hits <= 64.0f)) return fail(CATPC_E_INVALID, "bin_hits out of [0.25, 64]");
  if (t->nf_block < 64 || t->nf_block > 256 || t->nf_block % 64)
    return fail(CATPC_E_INVALID, "nf_block must be a multiple of 64 in [64, 256]");
  if (t->tc_block < 64 || t->tc_block > 256 || t->tc_block % 64)
    return fail(CATPC_E_INVALID, "tc_block must be a multiple of 64 in [64, 256]");
  if (t->tc_waves_per_cu < 1 || t->tc_waves_per_cu > 32) return fail(CATPC_E_INVALID, "tc_waves_per_cu out of [1, 32]");
  if (t->use_graph < 0 || t->use_graph > 1) return fail(CATPC_E_INVALID, "use_graph must be 0 or 1");
  if (t->nf_rows < 1 || t->nf_rows > 32) return fail(CATPC_E_INVALID, "nf_rows out of [1, 32]");
  if (t->nf_lds_kb < 0 || t->nf_lds_kb > 64) return fail(CATPC_E_INVALID, "nf_lds_kb out of [0, 64]");
  if (t->tc_xcd < 0 || t->tc_xcd > 1) return fail(CATPC_E_INVALID, "tc_xcd must be 0 or 1");
  if (t->tc_occupancy != 0 && t->tc_occupancy != 5 && t->tc_occupancy != 6 && t->tc_occupancy != 8)
    return fail(CATPC_E_INVALID, "tc_occupancy must be 0, 5, 6 or 8");
  if (t->tc_sync < 0 || t->tc_sync > 1) return fail(CATPC_E_INVALID, "tc_sync must be 0 or 1");
  if (t->merge_pair_cap < 0) return fail(CATPC_E_INVALID, "merge_pair_cap must be >= 0");
  return CATPC_OK;
}

catpc_status check_io_within(int64_t max_hits, int32_t max_sectors, const catpc_input* in, const catpc_output* out,
                             bool need_host_off) {
  if (!in || !out) return fail(CATPC_E_INVALID, "input or output is NULL");
  if (in->n_sectors < 0 || in->n_sectors > max_sectors)
    return fail(CATPC_E_INVALID, "n_sectors out of [0, max_sectors]");
  if (in->n_hits < 0 || in->n_hits > max_hits) return fail(CATPC_E_INVALID, "n_hits out of [0, max_hits]");
  if (in->n_sectors == 0) return CATPC_OK;
  if (!in->hit_offset) return fail(CATPC_E_INVALID, "hit_offset is NULL");
  if (in->n_hits > 0 && (!in->y || !in->z || !in->row)) return fail(CATPC_E_INVALID, "hit arrays are NULL");
  if (!out->tracklet_offset) return fail(CATPC_E_INVALID, "tracklet_offset is required");
  if (in->n_hits > 0 && (!out->link_up || !out->link_dn || !out->start_hit))
    return fail(CATPC_E_INVALID, "link_up, link_dn and start_hit are required");
  if (out->tracklet_capacity < 0) return fail(CATPC_E_INVALID, "tracklet_capacity < 0");
  if (out->tracklet_capacity > 0 &&
      (!out->x_ref || !out->param || !out->cov || !out->row_hit || !out->start_row || !out->first_row ||
       !out->last_row || !out->n_hits || !out->flags))
    return fail(CATPC_E_INVALID, "tracklet arrays are NULL");
  if (out->tracklet_capacity > 0 && ((uintptr_t)out->row_hit & 15))
    return fail(CATPC_E_INVALID, "row_hit is not 16-byte aligned");
  if (need_host_off) {
    const int64_t* h = in->hit_offset_host;
    if (!h) return fail(CATPC_E_INVALID, "hit_offset_host is required");
    if (h[0] != 0 || h[in->n_sectors] != in->n_hits) return fail(CATPC_E_INVALID, "hit_offset_host inconsistent");
    for (int32_t s = 0; s < in->n_sectors; ++s)
      if (h[s + 1] < h[s]) return fail(CATPC_E_INVALID, "hit_offset_host not monotone");
  } else if (in->hit_offset_host) {
    const int64_t* h = in->hit_offset_host;
    if (h[0] != 0 || h[in->n_sectors] != in->n_hits) return fail(CATPC_E_INVALID, "hit_offset_host inconsistent");
  }
  return CATPC_OK;
}

catpc_status check_io(const catpc_ctx* ctx, const catpc_input* in, const catpc_output* out, bool need_host_off) {
  if (!ctx) return fail(CATPC_E_INVALID, "ctx is NULL");
  return check_io_within(ctx->max_hits, ctx->max_sectors, in, out, need_host_off);
}

Inputs inputs_of(const catpc_input* in) {
  Inputs I;
  I.x = in->x;
  I.y = in->y;
  I.z = in->z;
  I.row = in->row;
  I.hit_offset = in->hit_offset;
  return I;
}

TrackletOut tracklets_of(const catpc_output* out) {
  TrackletOut T;
  T.x_ref = out->x_ref;
  T.param = out->param;
  T.cov = out->cov;
  T.row_hit = out->row_hit;
  T.start_row = out->start_row;
  T.first_row = out->first_row;
  T.last_row = out->last_row;
  T.n_hits = out->n_hits;
  T.flags = out->flags;
  return T;
}

// What the stage chain needs: the pad-row geometry on the device, method
// constants, launch shape and workspace -- from a context, or from the fixed
// device array of the no-allocation entry point.
struct Chain {
  int32_t n_rows = 0;
  const float* row_x = nullptr;  // device [n_rows]
  const float4* rowk = nullptr;  // device [n_rows]
  Consts consts{};
  int32_t precision = 0;
  catpc_tuning tuning{};
  int n_cu = 256;
  Workspace ws{};
};

Chain chain_of(const catpc_ctx* ctx) {
  Chain c;
  c.n_rows = ctx->n_rows;
  c.row_x = ctx->row_x;
  c.rowk = ctx->rowk;
  c.consts = ctx->consts;
  c.precision = ctx->params.precision;
  c.tuning = ctx->tuning;
  c.n_cu = ctx->n_cu;
  c.ws = ctx->ws;
  return c;
}

// Persistent grid of the tracklet kernel; `max_tracklets` (if >= 0) bounds
// the useful number of waves (a seed has at least three hits).
int tc_grid(const Chain& c, int64_t max_tracklets = -1) {
  int64_t waves = (int64_t)c.n_cu * (c.tuning.tc_waves_per_cu > 0 ? c.tuning.tc_waves_per_cu : 8);
  if (max_tracklets >= 0) waves = std::min<int64_t>(waves, std::max<int64_t>(1, (max_tracklets + 63) / 64));
  const int64_t wpb = c.tuning.tc_block / 64;
  return (int)((waves + wpb - 1) / wpb);
}

// The stage chain for sectors [s0, s1) with hits [h0, h1).  With `ev`
// (CATPC_N_STAGES + 1 events) an event is recorded before each stage and after
// the last one.
catpc_status enqueue_span(const Chain& c, const catpc_input* in, const catpc_output* out, Span sp, hipStream_t st,
                          hipEvent_t* ev = nullptr) {
  const Inputs I = inputs_of(in);
  const Workspace& ws = c.ws;
  int32_t* up = out->nf_up ? out->nf_up : ws.raw_up;
  int32_t* dn = out->nf_dn ? out->nf_dn : ws.raw_dn;
  const int nb = c.tuning.nf_block;
  auto mark = [&](int k) -> hipError_t { return ev ? hipEventRecord(ev[k], st) : hipSuccess; };
  HIP_TRY(mark(0));
  HIP_TRY(launch_row_index(I, sp, c.n_rows, c.row_x, ws, nb, st));
  HIP_TRY(mark(1));
  HIP_TRY(launch_grid(I, sp, c.n_rows, c.tuning.bin_hits, ws, st));
  HIP_TRY(mark(2));
  HIP_TRY(launch_neighbours(I, sp, c.n_rows, c.rowk, c.consts, ws, up, dn, nb, c.tuning.nf_rows,
                            c.tuning.nf_lds_kb * 1024, st));
  HIP_TRY(mark(3));
  HIP_TRY(launch_clean_start(I, sp, up, dn, out->link_up, out->link_dn, ws, st));
  HIP_TRY(mark(4));
  HIP_TRY(launch_scan(sp, out->tracklet_offset, ws, st));
  HIP_TRY(mark(5));
  HIP_TRY(launch_compact(I, sp, out->tracklet_offset, out->start_hit, ws, st));
  HIP_TRY(mark(6));
  if (out->tracklet_capacity > 0) {
    HIP_TRY(launch_tracklets(I, sp, c.n_rows, c.row_x, c.consts, ws, out->tracklet_offset, 0,
                             out->tracklet_capacity, tracklets_of(out), tc_grid(c, (sp.h1 - sp.h0) / 3 + 1),
                             c.tuning.tc_block, c.tuning.tc_xcd ? kXcds : 1, c.tuning.tc_occupancy,
                             c.tuning.tc_sync, st));
  }
  HIP_TRY(mark(7));
  return CATPC_OK;
}

catpc_status enqueue_refit(const Chain& c, const catpc_input* in, const catpc_output* out, Span sp, int64_t first,
                           hipStream_t st) {
  if (c.precision == 0 || out->tracklet_capacity == 0) return CATPC_OK;
  HIP_TRY(launch_refit64(inputs_of(in), sp, c.n_rows, c.row_x, c.consts, c.ws, out->tracklet_offset, first,
                         out->tracklet_capacity, tracklets_of(out), c.n_cu * 4, st));
  return CATPC_OK;
}

catpc_status enqueue_batch(const Chain& c, const catpc_input* in, const catpc_output* out, hipStream_t st) {
  HIP_TRY(launch_reset(c.ws.counters, kNumCounters, st));
  if (in->n_sectors == 0) return CATPC_OK;
  Span sp{0, in->n_sectors, 0, in->n_hits};
  catpc_status rc = enqueue_span(c, in, out, sp, st);
  if (rc) return rc;
  return enqueue_refit(c, in, out, sp, 0, st);
}

void drop_graph(catpc_ctx* ctx) {
  if (ctx->exec) (void)hipGraphExecDestroy(ctx->exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  ctx->exec = nullptr;
  ctx->graph = nullptr;
  ctx->have_graph = false;
  if (ctx->sel_exec) (void)hipGraphExecDestroy(ctx->sel_exec);
  if (ctx->sel_graph) (void)hipGraphDestroy(ctx->sel_graph);
  ctx->sel_exec = nullptr;
  ctx->sel_graph = nullptr;
  ctx->have_sel_graph = false;
}

// Capture `enqueue` on the context's capture stream into (graph, exec) unless
// the cached graph was made with the same key, then replay it on `st`.
template <class Key, class F>
catpc_status replay(catpc_ctx* ctx, bool& have, Key& cached, hipGraph_t& graph, hipGraphExec_t& exec, const Key& k,
                    F&& enqueue, hipStream_t st) {
  if (!have || !(k == cached)) {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    have = false;
    hipStream_t cs = ctx->capture_stream;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const catpc_status rc = enqueue(cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    const hipError_t e2 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (e2 != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(e2, "hipGraphInstantiate");
    }
    graph = g;
    cached = k;
    have = true;
  }
  HIP_TRY(hipGraphLaunch(exec, st));
  return CATPC_OK;
}

catpc_status enqueue_select(catpc_ctx* ctx, const catpc_input* in, const catpc_output* trk, const catpc_tracks* out,
                            hipStream_t st) {
  TrackletOut T{};
  T.row_hit = trk->row_hit;
  T.n_hits = trk->n_hits;
  T.flags = trk->flags;
  TracksOut O;
  O.track_offset = out->track_offset;
  O.track_tracklet = out->track_tracklet;
  O.track_n_hits = out->track_n_hits;
  O.track_hit_offset = out->track_hit_offset;
  O.track_capacity = out->track_capacity;
  O.track_hits = out->track_hits;
  O.hit_capacity = out->hit_capacity;
  HIP_TRY(launch_select(inputs_of(in), in->n_sectors, trk->tracklet_offset, trk->tracklet_capacity,
                        ctx->max_hits / 3 + 1, ctx->n_rows, T, ctx->consts, ctx->ws, O, in->n_hits,
                        ctx->n_cu * 8, st));
  return CATPC_OK;
}

}  // namespace

extern "C" {

void catpc_default_params(catpc_params* p) {
  if (!p) return;
  p->bz = 0.5f;
  p->sigma_y = 0.1f;
  p->sigma_z = 0.1f;
  p->nf_win_y = 3.0f;
  p->nf_win_z = 3.0f;
  p->nf_chi2_max = 0.2f;
  p->tc_gate_nsigma = 3.0f;
  p->tc_max_miss = 4;
  p->min_hits = 10;
  p->precision = 0;
}

void catpc_default_tuning(catpc_tuning* t) {
  if (!t) return;
  t->bin_hits = 2.0f;
  t->nf_block = 256;
  t->tc_block = 256;
  t->tc_waves_per_cu = 20;
  t->use_graph = 1;
  t->nf_rows = 4;
  t->nf_lds_kb = 32;
  t->tc_xcd = 1;
  t->tc_occupancy = 0;
  t->tc_sync = 0;
  t->merge_pair_cap = 0;
}

int32_t catpc_row_stride(int32_t n_rows) { return n_rows > 0 ? row_stride(n_rows) : 0; }

size_t catpc_workspace_bytes(int32_t n_rows, int64_t max_hits, int32_t max_sectors) {
  if (n_rows < 3 || n_rows > kMaxRows || max_hits < 0 || max_sectors < 0) return 0;
  return plan(n_rows, max_hits, max_sectors).total + (sizeof(float) + sizeof(float4)) * (size_t)n_rows;
}

const char* catpc_last_error(void) { return g_err.c_str(); }

namespace {

catpc_status check_geometry(const catpc_geometry* g) {
  if (!g) return fail(CATPC_E_INVALID, "geometry is NULL");
  if (g->n_rows < 3 || g->n_rows > kMaxRows || !g->row_x)
    return fail(CATPC_E_INVALID, "need 3 <= n_rows <= 4096 and row_x");
  for (int32_t r = 0; r < g->n_rows; ++r)
    if (!(g->row_x[r] > 0.0f) || (r > 0 && !(g->row_x[r] > g->row_x[r - 1])))
      return fail(CATPC_E_INVALID, "row_x must be positive and strictly ascending");
  if (g->sectors_per_side < 0) return fail(CATPC_E_INVALID, "sectors_per_side must be >= 0");
  return CATPC_OK;
}

int sectors_per_side(const catpc_geometry* g) { return g->sectors_per_side > 0 ? g->sectors_per_side : 18; }

}  // namespace

catpc_status catpc_sector_frame(const catpc_geometry* geom, int32_t sector_id, double* alpha, int32_t* side) {
  if (!geom || !alpha || !side) return fail(CATPC_E_INVALID, "NULL argument");
  if (geom->sectors_per_side < 0) return fail(CATPC_E_INVALID, "sectors_per_side must be >= 0");
  const int n = sectors_per_side(geom);
  if (sector_id < 0 || sector_id >= 2 * n) return fail(CATPC_E_INVALID, "sector id out of range");
  const double pi = 3.14159265358979323846;
  *alpha = ((double)(sector_id % n) + 0.5) * (2.0 * pi / (double)n);
  *side = sector_id < n ? 1 : -1;
  return CATPC_OK;
}

catpc_status catpc_to_global(const catpc_geometry* geom, int32_t sector_id, int64_t n, const float* x,
                             const float* param, double* out) {
  double alpha = 0.0;
  int32_t side = 0;
  catpc_status rc = catpc_sector_frame(geom, sector_id, &alpha, &side);
  if (rc) return rc;
  if (n < 0 || (n > 0 && (!x || !param || !out))) return fail(CATPC_E_INVALID, "NULL array or n < 0");
  const double pi = 3.14159265358979323846;
  const double ca = std::cos(alpha), sa = std::sin(alpha);
  bool bad = false;
  for (int64_t i = 0; i < n; ++i) {
    const float* p = param + 5 * i;
    double* o = out + 6 * i;
    const double lx = x[i], ly = p[0], sp = p[2];
    o[0] = lx * ca - ly * sa;
    o[1] = lx * sa + ly * ca;
    o[2] = p[1];
    if (!(std::fabs(sp) <= 1.0)) {
      o[3] = std::nan("");
      bad = true;
    } else {
      double phi = std::asin(sp) + alpha;
      while (phi > pi) phi -= 2.0 * pi;
      while (phi <= -pi) phi += 2.0 * pi;
      o[3] = phi;
    }
    o[4] = p[3];
    o[5] = p[4];
  }
  return bad ? fail(CATPC_E_INVALID, "|sin phi| > 1 in an entry (its phi is NaN)") : CATPC_OK;
}

catpc_status catpc_create(const catpc_geometry* geom, const catpc_params* params, int64_t max_hits,
                          int32_t max_sectors, catpc_ctx** out) {
  if (!out) return fail(CATPC_E_INVALID, "out is NULL");
  *out = nullptr;
  catpc_status grc = check_geometry(geom);
  if (grc) return grc;
  const int32_t n_rows = geom->n_rows;
  const float* row_x = geom->row_x;
  if (max_hits < 0 || max_hits >= (int64_t)1 << 31) return fail(CATPC_E_INVALID, "max_hits out of [0, 2^31)");
  if (max_sectors < 0 || max_hits + (int64_t)max_sectors * n_rows >= (int64_t)1 << 31)
    return fail(CATPC_E_INVALID, "max_hits + max_sectors * n_rows must stay below 2^31");
  catpc_status rc = check_params(params);
  if (rc) return rc;
  catpc_ctx* ctx = new (std::nothrow) catpc_ctx();
  if (!ctx) return fail(CATPC_E_HIP, "host allocation failed");
  ctx->n_rows = n_rows;
  ctx->max_hits = max_hits;
  ctx->max_sectors = max_sectors;
  ctx->params = *params;
  ctx->consts = make_consts(*params);
  catpc_default_tuning(&ctx->tuning);
  hipError_t e = hipGetDevice(&ctx->device);
  if (e == hipSuccess) {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) == hipSuccess && ncu > 0)
      ctx->n_cu = ncu;
    const Layout L = plan(n_rows, max_hits, max_sectors);
    e = hipMalloc(&ctx->ws_mem, L.total);
    if (e == hipSuccess) e = hipMalloc((void**)&ctx->row_x, sizeof(float) * (size_t)n_rows);
    if (e == hipSuccess) e = hipMemcpy(ctx->row_x, row_x, sizeof(float) * (size_t)n_rows, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      // per-row neighbour-finder ratios, each one binary32 division as in the
      // per-hit formula (hoisted: they depend on the row only)
      std::vector<float4> k((size_t)n_rows);
      for (int32_t r = 0; r < n_rows; ++r) {
        float4 v = make_float4(0.0f, 0.0f, 0.0f, row_x[r]);
        if (r >= 1 && r + 1 < n_rows) {
          const float xr = row_x[r], xu = row_x[r + 1], xd = row_x[r - 1];
          v.x = xu / xr;
          v.y = xd / xr;
          v.z = (xr - xd) / (xu - xd);
        }
        k[(size_t)r] = v;
      }
      e = hipMalloc((void**)&ctx->rowk, sizeof(float4) * (size_t)n_rows);
      if (e == hipSuccess) e = hipMemcpy(ctx->rowk, k.data(), sizeof(float4) * (size_t)n_rows, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->host_counters, sizeof(unsigned long long) * kNumCounters, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->host_total, sizeof(int64_t), 0);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess) {
      ctx->ws = carve((char*)ctx->ws_mem, L);
      Workspace& w = ctx->ws;
      e = hipMemset(w.counters, 0, sizeof(unsigned long long) * kNumCounters);
    }
  }
  if (e != hipSuccess) {
    catpc_destroy(ctx);
    return hip_fail(e, "catpc_create");
  }
  *out = ctx;
  return CATPC_OK;
}

void catpc_destroy(catpc_ctx* ctx) {
  if (!ctx) return;
  drop_graph(ctx);
  if (ctx->ws_mem) (void)hipFree(ctx->ws_mem);
  if (ctx->row_x) (void)hipFree(ctx->row_x);
  if (ctx->rowk) (void)hipFree(ctx->rowk);
  if (ctx->host_counters) (void)hipHostFree(ctx->host_counters);
  if (ctx->host_total) (void)hipHostFree(ctx->host_total);
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  delete ctx;
}

catpc_status catpc_set_params(catpc_ctx* ctx, const catpc_params* params) {
  if (!ctx) return fail(CATPC_E_INVALID, "ctx is NULL");
  catpc_status rc = check_params(params);
  if (rc) return rc;
  ctx->params = *params;
  ctx->consts = make_consts(*params);
  return CATPC_OK;
}

catpc_status catpc_set_tuning(catpc_ctx* ctx, const catpc_tuning* t) {
  if (!ctx || !t) return fail(CATPC_E_INVALID, "ctx or tuning is NULL");
  catpc_status rc = check_tuning(t);
  if (rc) return rc;
  ctx->tuning = *t;
  return CATPC_OK;
}

catpc_status catpc_get_tuning(const catpc_ctx* ctx, catpc_tuning* t) {
  if (!ctx || !t) return fail(CATPC_E_INVALID, "ctx or tuning is NULL");
  *t = ctx->tuning;
  return CATPC_OK;
}

catpc_status catpc_track_batch(catpc_ctx* ctx, const catpc_input* in, const catpc_output* out, void* stream) {
  catpc_status rc = check_io(ctx, in, out, false);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  ctx->have_last = false;
  ctx->have_sel = false;
  if (ctx->tuning.use_graph && in->n_sectors > 0) {
    GraphKey k;
    std::memset(&k, 0, sizeof k);
    k.in.x = in->x;
    k.in.y = in->y;
    k.in.z = in->z;
    k.in.row = in->row;
    k.in.hit_offset = in->hit_offset;
    k.in.n_sectors = in->n_sectors;
    k.in.n_hits = in->n_hits;
    k.out = *out;
    k.params = ctx->params;
    k.tuning = ctx->tuning;
    rc = replay(ctx, ctx->have_graph, ctx->key, ctx->graph, ctx->exec, k,
                [&](hipStream_t cs) { return enqueue_batch(chain_of(ctx), in, out, cs); }, st);
    if (rc) return rc;
  } else {
    rc = enqueue_batch(chain_of(ctx), in, out, st);
    if (rc) return rc;
  }
  ctx->last_in = *in;
  ctx->last_in.hit_offset_host = nullptr;
  ctx->last_out = *out;
  ctx->have_last = true;
  return CATPC_OK;
}

catpc_status catpc_track_plain(catpc_ctx* ctx, const catpc_input* in, const catpc_output* out, void* stream) {
  catpc_status rc = check_io(ctx, in, out, true);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  ctx->have_last = false;
  ctx->have_sel = false;
  HIP_TRY(launch_reset(ctx->ws.counters, kNumCounters, st));
  const int64_t* h = in->hit_offset_host;
  for (int32_t s = 0; s < in->n_sectors; ++s) {
    Span sp{s, s + 1, h[s], h[s + 1]};
    rc = enqueue_span(chain_of(ctx), in, out, sp, st);
    if (rc) return rc;
  }
  if (in->n_sectors > 0) {
    rc = enqueue_refit(chain_of(ctx), in, out, Span{0, in->n_sectors, 0, in->n_hits}, 0, st);
    if (rc) return rc;
  }
  ctx->last_in = *in;
  ctx->last_in.hit_offset_host = nullptr;
  ctx->last_out = *out;
  ctx->have_last = true;
  return CATPC_OK;
}

catpc_status catpc_result(catpc_ctx* ctx, void* stream, int64_t* n_tracklets) {
  if (!ctx) return fail(CATPC_E_INVALID, "ctx is NULL");
  if (!ctx->have_last) return fail(CATPC_E_STATE, "no completed track call");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipMemcpyAsync(ctx->host_counters, ctx->ws.counters, sizeof(unsigned long long) * kNumCounters,
                         hipMemcpyDeviceToHost, st));
  int64_t total = 0;
  if (ctx->last_in.n_sectors > 0) {
    HIP_TRY(hipMemcpyAsync(ctx->host_total, ctx->last_out.tracklet_offset + ctx->last_in.n_sectors, sizeof(int64_t),
                           hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (ctx->last_in.n_sectors > 0) total = *ctx->host_total;
  if (n_tracklets) *n_tracklets = total;
  if (ctx->host_counters[kCtrError] & 1ull) return fail(CATPC_E_INVALID, "hits not sorted by row, or a row out of range");
  if (ctx->host_counters[kCtrError] & 8ull) return fail(CATPC_E_INVALID, "x[i] differs from row_x[row[i]]");
  if (total > ctx->last_out.tracklet_capacity)
    return fail(CATPC_E_CAPACITY, "more tracklets (" + std::to_string(total) + ") than output slots (" +
                                      std::to_string(ctx->last_out.tracklet_capacity) + ")");
  return CATPC_OK;
}

catpc_status catpc_fetch_tracklets(catpc_ctx* ctx, const catpc_input* in, int64_t first, const catpc_output* out,
                                   void* stream) {
  if (!ctx || !in || !out) return fail(CATPC_E_INVALID, "NULL argument");
  if (!ctx->have_last) return fail(CATPC_E_STATE, "no track call to fetch from");
  if (in->n_sectors != ctx->last_in.n_sectors || in->n_hits != ctx->last_in.n_hits || in->y != ctx->last_in.y ||
      in->z != ctx->last_in.z || in->row != ctx->last_in.row || in->hit_offset != ctx->last_in.hit_offset)
    return fail(CATPC_E_STATE, "fetch needs the input of the last track call");
  if (first < 0) return fail(CATPC_E_INVALID, "first < 0");
  if (out->tracklet_capacity < 0) return fail(CATPC_E_INVALID, "tracklet_capacity < 0");
  if (out->tracklet_capacity == 0 || in->n_sectors == 0) return CATPC_OK;
  if (!out->x_ref || !out->param || !out->cov || !out->row_hit || !out->start_row || !out->first_row ||
      !out->last_row || !out->n_hits || !out->flags)
    return fail(CATPC_E_INVALID, "tracklet arrays are NULL");
  if ((uintptr_t)out->row_hit & 15) return fail(CATPC_E_INVALID, "row_hit is not 16-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  const Span sp{0, in->n_sectors, 0, in->n_hits};
  const Inputs I = inputs_of(in);
  catpc_output o = *out;
  o.tracklet_offset = ctx->last_out.tracklet_offset;
  HIP_TRY(launch_reset(ctx->ws.counters, kXcds, st));
  HIP_TRY(launch_tracklets(I, sp, ctx->n_rows, ctx->row_x, ctx->consts, ctx->ws, o.tracklet_offset, first,
                           o.tracklet_capacity, tracklets_of(&o), tc_grid(chain_of(ctx)), ctx->tuning.tc_block,
                           ctx->tuning.tc_xcd ? kXcds : 1, ctx->tuning.tc_occupancy,
                           ctx->tuning.tc_sync, st));
  return enqueue_refit(chain_of(ctx), in, &o, sp, first, st);
}

catpc_status catpc_stage_times(catpc_ctx* ctx, const catpc_input* in, const catpc_output* out, void* stream,
                               float* ms) {
  catpc_status rc = check_io(ctx, in, out, false);
  if (rc) return rc;
  if (!ms) return fail(CATPC_E_INVALID, "ms is NULL");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  ctx->have_last = false;
  ctx->have_sel = false;
  hipEvent_t ev[CATPC_N_STAGES + 1] = {};
  for (int k = 0; k <= CATPC_N_STAGES; ++k) HIP_TRY(hipEventCreate(&ev[k]));
  HIP_TRY(launch_reset(ctx->ws.counters, kNumCounters, st));
  const Span sp{0, in->n_sectors, 0, in->n_hits};
  if (in->n_sectors > 0) {
    rc = enqueue_span(chain_of(ctx), in, out, sp, st, ev);
    if (!rc) rc = enqueue_refit(chain_of(ctx), in, out, sp, 0, st);
  } else {
    for (int k = 0; k < CATPC_N_STAGES; ++k) HIP_TRY(hipEventRecord(ev[k], st));
  }
  if (!rc) {
    HIP_TRY(hipEventRecord(ev[CATPC_N_STAGES], st));
    HIP_TRY(hipEventSynchronize(ev[CATPC_N_STAGES]));
    for (int k = 0; k < CATPC_N_STAGES; ++k) HIP_TRY(hipEventElapsedTime(&ms[k], ev[k], ev[k + 1]));
    ctx->last_in = *in;
    ctx->last_in.hit_offset_host = nullptr;
    ctx->last_out = *out;
    ctx->have_last = true;
  }
  for (int k = 0; k <= CATPC_N_STAGES; ++k) (void)hipEventDestroy(ev[k]);
  return rc;
}

catpc_status catpc_work_counts(catpc_ctx* ctx, void* stream, int64_t* counts) {
  if (!ctx || !counts) return fail(CATPC_E_INVALID, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipMemcpyAsync(ctx->host_counters, ctx->ws.counters, sizeof(unsigned long long) * kNumCounters,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int k = 0; k < 4; ++k) counts[k] = (int64_t)ctx->host_counters[kCtrCounts + k];
  return CATPC_OK;
}

catpc_status catpc_merge_counts(catpc_ctx* ctx, void* stream, int64_t* n_pairs, int64_t* n_steps) {
  if (!ctx) return fail(CATPC_E_INVALID, "ctx is NULL");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipMemcpyAsync(ctx->host_counters, ctx->ws.counters, sizeof(unsigned long long) * kNumCounters,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (n_pairs) *n_pairs = (int64_t)ctx->host_counters[kCtrMergePairs];
  if (n_steps) *n_steps = (int64_t)ctx->host_counters[kCtrMergeSteps];
  return CATPC_OK;
}

catpc_status catpc_phase_clocks(uint64_t* out, int32_t clear) {
  if (!clear && !out) return fail(CATPC_E_INVALID, "NULL argument");
  const hipError_t e = phase_clocks(reinterpret_cast<unsigned long long*>(out), clear != 0);
  if (e == hipErrorNotSupported) return fail(CATPC_E_INVALID, "not a profiling build (-DCATPC_PHASE_CLOCKS=1)");
  HIP_TRY(e);
  return CATPC_OK;
}

catpc_status catpc_fp32_probe(int32_t op, const float* a, const float* b, float* out, int64_t n, void* stream) {
  if (op < 0 || op > 5 || n < 0 || (n > 0 && (!a || !b || !out))) return fail(CATPC_E_INVALID, "bad probe arguments");
  HIP_TRY(launch_fp32_probe(op, a, b, out, n, (hipStream_t)stream));
  return CATPC_OK;
}

catpc_status catpc_select_tracklets(catpc_ctx* ctx, const catpc_input* in, const catpc_output* trk,
                                    const catpc_tracks* out, void* stream) {
  if (!ctx || !in || !trk || !out) return fail(CATPC_E_INVALID, "NULL argument");
  if (in->n_sectors < 0 || in->n_sectors > ctx->max_sectors || in->n_hits < 0 || in->n_hits > ctx->max_hits)
    return fail(CATPC_E_INVALID, "sizes beyond the context's maxima");
  if (in->n_sectors > 0 && !in->hit_offset) return fail(CATPC_E_INVALID, "hit_offset is NULL");
  if (!trk->tracklet_offset) return fail(CATPC_E_INVALID, "tracklet_offset is NULL");
  if (trk->tracklet_capacity < 0) return fail(CATPC_E_INVALID, "tracklet_capacity < 0");
  if (trk->tracklet_capacity > 0 && (!trk->row_hit || !trk->n_hits || !trk->flags))
    return fail(CATPC_E_INVALID, "row_hit, n_hits and flags are required");
  if (trk->tracklet_capacity > 0 && ((uintptr_t)trk->row_hit & 15))
    return fail(CATPC_E_INVALID, "row_hit is not 16-byte aligned");
  if (!out->track_offset) return fail(CATPC_E_INVALID, "track_offset is NULL");
  if (out->track_capacity < 0 || out->hit_capacity < 0) return fail(CATPC_E_INVALID, "negative capacity");
  if (out->track_capacity > 0 && (!out->track_tracklet || !out->track_n_hits || !out->track_hit_offset))
    return fail(CATPC_E_INVALID, "track arrays are NULL");
  if (out->hit_capacity > 0 && !out->track_hits) return fail(CATPC_E_INVALID, "track_hits is NULL");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  ctx->have_sel = false;
  catpc_status rc;
  if (ctx->tuning.use_graph) {
    SelKey k;
    std::memset(&k, 0, sizeof k);
    k.in.y = in->y;
    k.in.z = in->z;
    k.in.row = in->row;
    k.in.hit_offset = in->hit_offset;
    k.in.n_sectors = in->n_sectors;
    k.in.n_hits = in->n_hits;
    k.trk = *trk;
    k.out = *out;
    k.min_hits = ctx->params.min_hits;
    k.use_graph = 1;
    rc = replay(ctx, ctx->have_sel_graph, ctx->sel_key, ctx->sel_graph, ctx->sel_exec, k,
                [&](hipStream_t cs) { return enqueue_select(ctx, in, trk, out, cs); }, st);
  } else {
    rc = enqueue_select(ctx, in, trk, out, st);
  }
  if (rc) return rc;
  ctx->sel_out = *out;
  ctx->have_sel = true;
  return CATPC_OK;
}

catpc_status catpc_refit_tracks(catpc_ctx* ctx, const catpc_input* in, const catpc_output* trk,
                                const catpc_tracks* tracks, const catpc_fits* out, void* stream) {
  if (!ctx || !in || !trk || !tracks || !out) return fail(CATPC_E_INVALID, "NULL argument");
  if (in->n_sectors < 0 || in->n_sectors > ctx->max_sectors || in->n_hits < 0 || in->n_hits > ctx->max_hits)
    return fail(CATPC_E_INVALID, "sizes beyond the context's maxima");
  if (in->n_sectors > 0 && (!in->hit_offset || (in->n_hits > 0 && (!in->y || !in->z || !in->row))))
    return fail(CATPC_E_INVALID, "hit arrays are NULL");
  if (!trk->tracklet_offset || trk->tracklet_capacity < 0 ||
      (trk->tracklet_capacity > 0 && (!trk->x_ref || !trk->param || !trk->first_row)))
    return fail(CATPC_E_INVALID, "tracklet arrays are NULL");
  if (!tracks->track_offset || tracks->track_capacity < 0 || tracks->hit_capacity < 0 ||
      (tracks->track_capacity > 0 && (!tracks->track_tracklet || !tracks->track_n_hits || !tracks->track_hit_offset)) ||
      (tracks->hit_capacity > 0 && !tracks->track_hits))
    return fail(CATPC_E_INVALID, "track arrays are NULL");
  if (out->capacity < tracks->track_capacity) return fail(CATPC_E_INVALID, "fit capacity below track capacity");
  if (out->capacity > 0 && (!out->x || !out->param || !out->cov || !out->chi2 || !out->ndf || !out->flags))
    return fail(CATPC_E_INVALID, "fit arrays are NULL");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  if (in->n_sectors == 0 || out->capacity == 0) return CATPC_OK;
  TrackletOut T{};
  T.x_ref = trk->x_ref;
  T.param = trk->param;
  T.first_row = trk->first_row;
  TracksOut R;
  R.track_offset = tracks->track_offset;
  R.track_tracklet = tracks->track_tracklet;
  R.track_n_hits = tracks->track_n_hits;
  R.track_hit_offset = tracks->track_hit_offset;
  R.track_capacity = tracks->track_capacity;
  R.track_hits = tracks->track_hits;
  R.hit_capacity = tracks->hit_capacity;
  FitsOut F;
  F.x = out->x;
  F.param = out->param;
  F.cov = out->cov;
  F.chi2 = out->chi2;
  F.ndf = out->ndf;
  F.flags = out->flags;
  F.capacity = out->capacity;
  const int64_t lanes = std::min<int64_t>(out->capacity, (int64_t)ctx->n_cu * 4 * 256);
  HIP_TRY(launch_fullfit(inputs_of(in), in->n_sectors, ctx->n_rows, ctx->row_x, ctx->consts, trk->tracklet_offset,
                         T, trk->tracklet_capacity, R, F, ctx->ws, (int)((lanes + 255) / 256), st));
  return CATPC_OK;
}

void catpc_default_merge_params(catpc_merge_params* m) {
  if (!m) return;
  m->max_gap = 30;
  m->window = 10.0f;
  m->chi2_max = 25.0f;
}

catpc_status catpc_merge_tracks(catpc_ctx* ctx, const catpc_input* in, const catpc_output* trk,
                                const catpc_tracks* tracks, const catpc_fits* fits, const catpc_merge_params* mp,
                                const catpc_merges* out, void* stream) {
  if (!ctx || !in || !trk || !tracks || !fits || !out) return fail(CATPC_E_INVALID, "NULL argument");
  catpc_merge_params m;
  catpc_default_merge_params(&m);
  if (mp) m = *mp;
  if (m.max_gap < 1 || m.max_gap > kMaxRows || !(m.window >= 0.0f) || !(m.chi2_max >= 0.0f))
    return fail(CATPC_E_INVALID, "merge cuts: max_gap in [1, 4096], window and chi2_max >= 0");
  if (in->n_sectors < 0 || in->n_sectors > ctx->max_sectors || in->n_hits < 0 || in->n_hits > ctx->max_hits)
    return fail(CATPC_E_INVALID, "sizes beyond the context's maxima");
  if (in->n_sectors > 0 && (!in->hit_offset || (in->n_hits > 0 && !in->row)))
    return fail(CATPC_E_INVALID, "hit arrays are NULL");
  if (!trk->tracklet_offset || trk->tracklet_capacity < 0 ||
      (trk->tracklet_capacity > 0 && (!trk->x_ref || !trk->param || !trk->cov || !trk->first_row)))
    return fail(CATPC_E_INVALID, "tracklet arrays are NULL");
  if (!tracks->track_offset || tracks->track_capacity < 0 || tracks->hit_capacity < 0 ||
      (tracks->track_capacity > 0 && (!tracks->track_tracklet || !tracks->track_n_hits || !tracks->track_hit_offset)) ||
      (tracks->hit_capacity > 0 && !tracks->track_hits))
    return fail(CATPC_E_INVALID, "track arrays are NULL");
  if (fits->capacity < tracks->track_capacity || out->capacity < tracks->track_capacity)
    return fail(CATPC_E_INVALID, "fit or merge capacity below track capacity");
  if (fits->capacity > 0 && (!fits->x || !fits->param || !fits->cov || !fits->flags))
    return fail(CATPC_E_INVALID, "fit arrays are NULL");
  if (out->capacity > 0 && (!out->next || !out->prev || !out->head || !out->chi2))
    return fail(CATPC_E_INVALID, "merge arrays are NULL");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  if (in->n_sectors == 0 || tracks->track_capacity == 0) return CATPC_OK;
  TrackletOut T{};
  T.x_ref = trk->x_ref;
  T.param = trk->param;
  T.cov = trk->cov;
  T.first_row = trk->first_row;
  TracksOut R;
  R.track_offset = tracks->track_offset;
  R.track_tracklet = tracks->track_tracklet;
  R.track_n_hits = tracks->track_n_hits;
  R.track_hit_offset = tracks->track_hit_offset;
  R.track_capacity = tracks->track_capacity;
  R.track_hits = tracks->track_hits;
  R.hit_capacity = tracks->hit_capacity;
  FitsOut F{};
  F.x = fits->x;
  F.param = fits->param;
  F.cov = fits->cov;
  F.flags = fits->flags;
  F.capacity = fits->capacity;
  MergeOut M;
  M.next = out->next;
  M.prev = out->prev;
  M.head = out->head;
  M.chi2 = out->chi2;
  M.capacity = out->capacity;
  MergeCuts cuts;
  cuts.max_gap = m.max_gap;
  cuts.window = (double)m.window;
  cuts.chi2_max = (double)m.chi2_max;
  const int64_t slots = ctx->max_hits / 3 + 2;
  const int64_t lanes = std::min<int64_t>(std::min(tracks->track_capacity, slots), (int64_t)ctx->n_cu * 4 * 256);
  HIP_TRY(launch_merge(inputs_of(in), in->n_sectors, ctx->n_rows, ctx->row_x, ctx->consts, cuts,
                       trk->tracklet_offset, T, trk->tracklet_capacity, R, F, M, ctx->ws, slots,
                       (int)((lanes + 255) / 256), ctx->n_cu * 8, ctx->tuning.merge_pair_cap > 0 ? (int64_t)ctx->tuning.merge_pair_cap : kMergePairsPerSlot * slots, st));
  return CATPC_OK;
}

catpc_status catpc_select_result(catpc_ctx* ctx, void* stream, int64_t* n_tracks, int64_t* n_track_hits) {
  if (!ctx) return fail(CATPC_E_INVALID, "ctx is NULL");
  if (!ctx->have_sel) return fail(CATPC_E_STATE, "no selection call since the last track call");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipMemcpyAsync(ctx->host_counters, ctx->ws.counters, sizeof(unsigned long long) * kNumCounters,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int64_t nt = (int64_t)ctx->host_counters[kCtrSelTracks], nh = (int64_t)ctx->host_counters[kCtrSelHits];
  if (n_tracks) *n_tracks = nt;
  if (n_track_hits) *n_track_hits = nh;
  const unsigned long long err = ctx->host_counters[kCtrError];
  if (err & 4ull) return fail(CATPC_E_INVALID, "a tracklet record names a hit that is not in the row of its entry");
  if (err & 16ull) return fail(CATPC_E_CAPACITY, "a sector has more tracklets than the selection weights order");
  if (err & 2ull) return fail(CATPC_E_CAPACITY, "the tracklet output holds only part of the tracklets");
  if (nt > ctx->sel_out.track_capacity || nh > ctx->sel_out.hit_capacity)
    return fail(CATPC_E_CAPACITY, "more tracks (" + std::to_string(nt) + ") or track hits (" + std::to_string(nh) +
                                      ") than the output holds");
  return CATPC_OK;
}

catpc_status catpc_probe_copy(const void* src, void* dst, int64_t n_bytes, void* stream) {
  if (n_bytes < 0 || n_bytes % 16 || (n_bytes > 0 && (!src || !dst)) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
    return fail(CATPC_E_INVALID, "probe_copy needs 16-byte aligned pointers and a size that is a multiple of 16");
  if (n_bytes / 16 > (int64_t)UINT32_MAX * 1024) return fail(CATPC_E_INVALID, "probe_copy size too large");
  HIP_TRY(launch_probe_copy(src, dst, n_bytes / 16, (hipStream_t)stream));
  return CATPC_OK;
}

catpc_status catpc_probe_fma(float* out, int64_t n_threads, int32_t n_iter, void* stream) {
  if (n_threads < 0 || n_iter < 0 || (n_threads > 0 && !out) || n_threads > (int64_t)UINT32_MAX * 256)
    return fail(CATPC_E_INVALID, "bad probe_fma arguments");
  HIP_TRY(launch_probe_fma(out, n_threads, n_iter, (hipStream_t)stream));
  return CATPC_OK;
}

}  // extern "C"

// ------------------------------------------------------------ no allocation
// The workspace of catpc_track_batch_noalloc: a fixed device array in the
// library, one copy on each device the library runs on, held until the
// process ends.  Host code never uses this name as an address (in host code it
// is a stand-in, not the device array): the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
namespace {

constexpr size_t kScratchBytes = (size_t)96 << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};
int g_scratch_cu[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device) and the device's compute-unit count.
catpc_status scratch_here(char** base, int* n_cu) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CATPC_E_INVALID, "device id beyond the library's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0) ncu = 256;
    g_scratch_cu[dev] = ncu;
    g_scratch[dev] = (char*)p;
  }
  *base = g_scratch[dev];
  *n_cu = g_scratch_cu[dev];
  return CATPC_OK;
}

}  // namespace

extern "C" catpc_status catpc_track_batch_noalloc(int32_t n_rows, const float* row_x, const catpc_params* params,
                                                  const catpc_tuning* tuning, const catpc_input* in,
                                                  const catpc_output* out, uint64_t* status, void* stream) {
  if (n_rows < 3 || n_rows > kMaxRows || !row_x) return fail(CATPC_E_INVALID, "need 3 <= n_rows <= 4096 and row_x");
  catpc_status rc = check_params(params);
  if (rc) return rc;
  catpc_tuning t;
  catpc_default_tuning(&t);
  if (tuning) {
    rc = check_tuning(tuning);
    if (rc) return rc;
    t = *tuning;
  }
  t.use_graph = 0;
  if (!status) return fail(CATPC_E_INVALID, "status is NULL");
  if (!in || !out) return fail(CATPC_E_INVALID, "input or output is NULL");
  if (in->n_hits < 0 || in->n_sectors < 0) return fail(CATPC_E_INVALID, "negative size");
  const Layout L = plan(n_rows, in->n_hits, in->n_sectors, true);
  const size_t need = align_up(L.total) + sizeof(float4) * (size_t)n_rows;
  if (need > kScratchBytes)
    return fail(CATPC_E_INVALID, "input needs " + std::to_string(need) + " bytes of workspace; the fixed workspace "
                                 "holds " + std::to_string(kScratchBytes) + " (about 1.9 M hits in 36 sectors of 159 "
                                 "pad rows)");
  rc = check_io_within(in->n_hits, in->n_sectors, in, out, false);
  if (rc) return rc;
  char* base = nullptr;
  int n_cu = 256;
  rc = scratch_here(&base, &n_cu);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  Chain c;
  c.n_rows = n_rows;
  c.row_x = row_x;
  c.rowk = reinterpret_cast<const float4*>(base + align_up(L.total));
  c.consts = make_consts(*params);
  c.precision = params->precision;
  c.tuning = t;
  c.n_cu = n_cu;
  c.ws = carve(base, L);
  HIP_TRY(launch_reset(c.ws.counters, kNumCounters, st));
  HIP_TRY(launch_rowk(row_x, n_rows, reinterpret_cast<float4*>(base + align_up(L.total)), c.ws.counters, st));
  if (in->n_sectors > 0) {
    const Span sp{0, in->n_sectors, 0, in->n_hits};
    rc = enqueue_span(c, in, out, sp, st);
    if (!rc) rc = enqueue_refit(c, in, out, sp, 0, st);
    if (rc) return rc;
  }
  HIP_TRY(launch_status(c.ws.counters, status, st));
  return CATPC_OK;
}
