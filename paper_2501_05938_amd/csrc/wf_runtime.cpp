// wf_runtime.cpp -- the C ABI of libwf (include/wf.h): argument checking,
// per-context workspace, launch configuration, batched work lists with hipGraph
// replay, the autotuner and its persistent cache, and error reporting.
#include "../../include/wf.h"
#include "wf_internal.h"
#include "wf_host.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

using namespace wfk;
using namespace wfh;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

wf_status wfh::fail(wf_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

extern "C" const char* wf_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* wf_status_str(wf_status s) {
  switch (s) {
    case WF_OK: return "WF_OK";
    case WF_PENDING: return "WF_PENDING";
    case WF_EINVAL: return "WF_EINVAL";
    case WF_ENOMEM: return "WF_ENOMEM";
    case WF_E2BIG: return "WF_E2BIG";
    case WF_EHIP: return "WF_EHIP";
    case WF_ETIMEDOUT: return "WF_ETIMEDOUT";
    case WF_ENOTFOUND: return "WF_ENOTFOUND";
    case WF_ESHUTDOWN: return "WF_ESHUTDOWN";
    case WF_EUNSUPPORTED: return "WF_EUNSUPPORTED";
    default: return "WF_UNKNOWN";
  }
}

extern "C" const char* wf_version(void) { return "libwf 0.2 (gfx950)"; }

wf_status wfh::set_device(wf_ctx* ctx) {
  int cur = -1;
  WF_HIP(hipGetDevice(&cur));
  if (cur != ctx->device) WF_HIP(hipSetDevice(ctx->device));
  return WF_OK;
}

// ------------------------------------------------------------------ slots
// Set once a launch with XCD queues timed out: no later launch uses them.
static std::atomic<bool> xcd_off{false};

// Reads the device status of a slot's last launch.  wait: block until it is done.
// After a watchdog abort the slot is marked for re-arming; the refill happens on the
// stream of the slot's next launch (ensure_hand), so it is ordered before that launch.
static wf_status harvest(Slot& s, bool wait) {
  if (!s.pending) return WF_OK;
  hipError_t q = wait ? hipEventSynchronize(s.done) : hipEventQuery(s.done);
  if (q == hipErrorNotReady) return WF_PENDING;
  s.pending = false;
  if (q != hipSuccess) {
    s.needs_rearm = true;
    return fail(WF_EHIP, std::string("launch failed: ") + hipGetErrorString(q));
  }
  if (*s.host_err != DEV_OK) {
    *s.host_err = DEV_OK;
    s.needs_rearm = true;
    // A queue without a workgroup would stall its bands until the watchdog fires: after
    // a timed-out launch that used XCD queues, no later launch uses them.
    if (s.xcd_queues) xcd_off.store(true);
    return fail(WF_ETIMEDOUT, "device watchdog fired: a wait for a neighbouring band exceeded the limit "
                              "(NaN or reserved-value inputs, or an oversubscribed device)");
  }
  return WF_OK;
}

static wf_status note(wf_ctx* ctx, wf_status st) {
  if (st == WF_ETIMEDOUT || st == WF_EHIP) {
    if (ctx->sticky == WF_OK) ctx->sticky = st;
    return WF_OK;
  }
  return st;
}

static wf_status new_slot(wf_ctx* ctx, Slot** out) {
  std::unique_ptr<Slot> s(new Slot);
  if (hipMalloc(&s->ctl, CTL_WORDS * sizeof(uint32_t)) != hipSuccess) return fail(WF_ENOMEM, "cannot allocate a launch slot");
  WF_HIP(hipHostMalloc(&s->host_err, sizeof(uint32_t), hipHostMallocDefault));
  *s->host_err = 0;
  WF_HIP(hipEventCreateWithFlags(&s->done, hipEventDisableTiming));
  ctx->slots.push_back(std::move(s));
  *out = ctx->slots.back().get();
  return WF_OK;
}

// A free slot: the first unreserved slot whose last launch has finished, else a new
// one while the pool is below MAX_SLOTS, else the oldest unreserved slot after
// waiting for it.  Launches therefore never wait on one another's completion until
// MAX_SLOTS of them are in flight.
static wf_status acquire_slot(wf_ctx* ctx, Slot** out) {
  const size_t n = ctx->slots.size();
  for (size_t k = 0; k < n; ++k) {
    const size_t i = (ctx->next_slot + k) % n;
    Slot& s = *ctx->slots[i];
    if (s.reserved) continue;
    wf_status st = harvest(s, false);
    if (st == WF_PENDING) continue;
    st = note(ctx, st);
    if (st != WF_OK) return st;
    ctx->next_slot = (i + 1) % n;
    *out = &s;
    return WF_OK;
  }
  if ((int)n < wf_ctx::MAX_SLOTS) return new_slot(ctx, out);
  for (size_t k = 0; k < n; ++k) {
    const size_t i = (ctx->next_slot + k) % n;
    Slot& s = *ctx->slots[i];
    if (s.reserved) continue;
    wf_status st = note(ctx, harvest(s, true));
    if (st != WF_OK) return st;
    ctx->next_slot = (i + 1) % n;
    *out = &s;
    return WF_OK;
  }
  return fail(WF_ENOMEM, "every launch slot is held by a cached batch plan");
}

// Handoff rows of at least `need` elements armed with `sent`, on `stream`.
static wf_status ensure_hand(Slot& s, size_t need, uint32_t sent, hipStream_t stream) {
  if (need == 0) need = 64;
  if (s.hand_cap < need) {
    if (s.external) return fail(WF_E2BIG, "the problem needs more handoff rows than the fixed workspace holds");
    const size_t cap = std::max(need, s.hand_cap * 2);
    if (s.hand) WF_HIP(hipFree(s.hand));
    s.hand = nullptr;
    s.hand_cap = 0;
    if (hipMalloc(&s.hand, cap * sizeof(uint32_t)) != hipSuccess) {
      s.hand = nullptr;
      return fail(WF_ENOMEM, "cannot allocate handoff rows");
    }
    s.hand_cap = cap;
    s.needs_rearm = true;
  }
  if (s.hand_sent != sent || s.needs_rearm) {
    WF_HIP(launch_fill_u32(s.hand, sent, (int64_t)s.hand_cap, stream));
    s.hand_sent = sent;
    s.needs_rearm = false;
  }
  return WF_OK;
}

template <class T>
static wf_status ensure_buf(T** p, size_t* cap, size_t need) {
  if (*cap >= need) return WF_OK;
  if (*p) WF_HIP(hipFree(*p));
  *p = nullptr;
  *cap = 0;
  const size_t c = std::max<size_t>(need, 64);
  if (hipMalloc(p, c * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return fail(WF_ENOMEM, "cannot allocate descriptor table");
  }
  *cap = c;
  return WF_OK;
}

static wf_status finish_launch(Slot& s, hipStream_t stream, bool xcd_queues = false) {
  s.xcd_queues = xcd_queues;
  WF_HIP(hipMemcpyAsync(s.host_err, s.ctl + CTL_ERROR, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
  WF_HIP(hipEventRecord(s.done, stream));
  s.pending = true;
  return WF_OK;
}

// --------------------------------------------------------------- checking
// Positions are 32-bit inside the kernel, and a 64-row strip must span less than 4 GiB
// (the loaders address it with 32-bit byte offsets): 64 rows of 2^23 fp32 are 2 GiB.
static const int64_t MAX_N = (int64_t)1 << 23;

wf_status wfh::check_problem(const wf_problem* p, int64_t idx) {
  char where[64] = "";
  if (idx >= 0) snprintf(where, sizeof where, "problem %lld: ", (long long)idx);
  if (!p) return fail(WF_EINVAL, std::string(where) + "NULL problem");
  if (p->m < 0 || p->n < 0) return fail(WF_EINVAL, std::string(where) + "m and n must be >= 0");
  if (p->n > MAX_N) return fail(WF_EUNSUPPORTED, std::string(where) + "n above 2^23 is not supported");
  if (p->dtype != WF_F32 && p->dtype != WF_I32 && p->dtype != WF_F64)
    return fail(WF_EINVAL, std::string(where) + "unknown dtype");
  if (p->dtype == WF_F64 && (p->n > MAX_N / 2 || p->ld_cost > MAX_N / 2 || p->ld_out > MAX_N / 2))
    return fail(WF_EUNSUPPORTED, std::string(where) + "fp64 grids need n and leading dimensions <= 2^22");
  if (p->rule != WF_RULE_MIN && p->rule != WF_RULE_MAX) return fail(WF_EINVAL, std::string(where) + "unknown rule");
  if (p->mode != WF_MODE_FULL && p->mode != WF_MODE_EDGES) return fail(WF_EINVAL, std::string(where) + "unknown mode");
  if (p->flags != 0 && p->flags != WF_COST_ABSDIFF)
    return fail(WF_EINVAL, std::string(where) + "flags must be 0 or WF_COST_ABSDIFF");
  if (p->flags == WF_COST_ABSDIFF && p->dtype != WF_F32)
    return fail(WF_EUNSUPPORTED, std::string(where) + "WF_COST_ABSDIFF needs WF_F32");
  if (p->m == 0 || p->n == 0) return WF_OK;
  if (p->flags == WF_COST_ABSDIFF) {
    if (!p->seq_x || !p->seq_y) return fail(WF_EINVAL, std::string(where) + "seq_x or seq_y is NULL");
  } else {
    if (!p->cost) return fail(WF_EINVAL, std::string(where) + "cost is NULL");
    if (p->ld_cost < p->n) return fail(WF_EINVAL, std::string(where) + "ld_cost < n");
    if (p->ld_cost > MAX_N) return fail(WF_EUNSUPPORTED, std::string(where) + "ld_cost above 2^23 is not supported");
  }
  if (p->mode == WF_MODE_FULL) {
    if (!p->out) return fail(WF_EINVAL, std::string(where) + "out is NULL in FULL mode");
    if (p->ld_out < p->n) return fail(WF_EINVAL, std::string(where) + "ld_out < n");
  } else if (!p->last_row && !p->last_col && !p->final_cell) {
    return fail(WF_EINVAL, std::string(where) + "EDGES mode needs last_row, last_col or final_cell");
  }
  return WF_OK;
}

static wf_status check_tuning(const wf_tuning& t) {
  for (int i = 0; i < 3; ++i)
    if (t.reserved[i] != 0) return fail(WF_EINVAL, "wf_tuning.reserved must be 0");
  if (t.waves_per_wg < 0 || t.waves_per_wg > 2) return fail(WF_EINVAL, "waves_per_wg must be 0, 1 or 2");
  if (t.rows_per_lane < 0 || t.rows_per_lane > 2) return fail(WF_EINVAL, "rows_per_lane must be 0, 1 or 2");
  if (t.waves_per_wg == 2 && t.rows_per_lane == 2)
    return fail(WF_EUNSUPPORTED, "two compute waves of two rows per lane do not fit the LDS");
  if (t.max_wgs < 0 || t.order < 0 || t.order > 2 || t.use_graph < -1 || t.use_graph > 1)
    return fail(WF_EINVAL, "bad tuning value");
  return WF_OK;
}

// ------------------------------------------------------------ configuration
int wfh::choose_shape(int64_t m) {
  // One compute wave of one row per lane per workgroup, spread over the compute units.
  // Two rows per lane halve the bands (and the handoffs between workgroups on the
  // critical path), but measured at 16384 x 16384 each step of the walk then costs about
  // 50 ns instead of 31 (the wave is bound by the instructions it issues, not by the
  // chain's latency), so the walk is slower overall: 1.92 ms against 1.55 ms.
  (void)m;
  return 1;
}

// The LDS rings of one compute wave of one row per lane take about 66 KB of a compute
// unit's 160 KB, so two such workgroups fit; the other shapes take twice that.
int wfh::wgs_per_cu(int bs, int dtype) { return bs == 1 && dtype != WF_F64 ? 2 : 1; }

hipError_t wfh::launch_shape(int dtype, int rule, int bs, int nwg, const KArgs& args, hipStream_t stream) {
  return launch_sweep(dtype, rule, shape_waves(bs), shape_rows_per_lane(bs), nwg, args, stream);
}

// Band shape of explicit tuning values (0 = automatic for that field).
static int shape_of_tuning(const wf_tuning& t, int64_t m) {
  if (t.waves_per_wg == 0 && t.rows_per_lane == 0) return choose_shape(m);
  if (t.waves_per_wg == 2) return 2;
  if (t.rows_per_lane == 2) return 3;
  return 1;
}

uint32_t wfh::sentinel_of(int dtype) { return dtype == WF_I32 ? SENT_I32 : SENT_F32; }

GridDesc wfh::make_desc(const wf_problem* p, int bs, uint32_t* hand) {
  GridDesc d;
  std::memset(&d, 0, sizeof d);
  const bool absdiff = p->flags == WF_COST_ABSDIFF;
  d.cost = absdiff ? nullptr : p->cost;
  d.sx = absdiff ? p->seq_x : nullptr;
  d.sy = absdiff ? p->seq_y : nullptr;
  d.kind = absdiff ? 1 : 0;
  d.out = p->mode == WF_MODE_FULL ? p->out : nullptr;
  d.top = p->top;
  d.left = p->left;
  d.last_row = p->last_row;
  d.last_col = p->last_col;
  d.final_cell = p->final_cell;
  d.hand = hand;
  d.m = p->m;
  d.n = p->n;
  d.ld_cost = absdiff ? p->n : p->ld_cost;
  d.ld_out = p->mode == WF_MODE_FULL ? p->ld_out : 0;
  d.hand_ld = hand_ld_for(p->n, shape_rows_per_lane(bs));
  d.mode = p->mode;
  d.nbands = (int32_t)((p->m + shape_rows(bs) - 1) / shape_rows(bs));
  return d;
}

size_t wfh::hand_elems(const wf_problem* p, int bs) {
  const int64_t nb = (p->m + shape_rows(bs) - 1) / shape_rows(bs);
  // fp64 positions travel encoded in four words
  const size_t words = p->dtype == WF_F64 ? 4 : 1;
  return nb > 1 ? (size_t)(nb - 1) * (size_t)hand_ld_for(p->n, shape_rows_per_lane(bs)) * words : 0;
}

void wfh::xcd_queues(const wf_ctx* ctx, KArgs& a, int nwg) {
  const int nx = ctx->nx;
  if (nx < 2 || nwg < nx || a.grids || xcd_off.load()) return;
  // Runs of seg bands per XCD: at most one band per workgroup of the XCD's queue at a
  // time, and the grid's bands spread over all XCDs.
  const int64_t per_xcd = (a.nitems + nx - 1) / nx;
  a.nx = nx;
  a.seg = (int32_t)std::max<int64_t>(1, std::min<int64_t>(per_xcd, nwg / nx));
}

// Which XCD each workgroup of a launch runs on, from a probe launch: XCD queues are used
// only when consecutive workgroups run on consecutive XCDs (modulo nx, from wherever the
// dispatcher's turn stands), as a whole-chip (SPX) device deals them, so that a launch of
// at least nx workgroups has one on every XCD.
static void probe_xcds(wf_ctx* ctx) {
  ctx->nx = 1;
  if (const char* e = std::getenv("WF_XCD_QUEUES"))
    if (std::atoi(e) == 0) return;
  const int nwg = ctx->num_cus * 2;
  uint32_t* d = nullptr;
  if (hipMalloc(&d, (size_t)nwg * sizeof(uint32_t)) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  std::vector<uint32_t> h((size_t)nwg, 0u);
  const bool ok = launch_xcc_probe(d, nwg, nullptr) == hipSuccess &&
                  hipMemcpy(h.data(), d, (size_t)nwg * sizeof(uint32_t), hipMemcpyDeviceToHost) == hipSuccess;
  (void)hipFree(d);
  if (!ok) {
    (void)hipGetLastError();
    return;
  }
  uint32_t top = 0;
  for (uint32_t v : h) top = std::max(top, v);
  const int nx = (int)top + 1;
  if (nx < 2 || nx > MAX_XCD) return;
  for (int i = 0; i < nwg; ++i)
    if (h[(size_t)i] != (h[0] + (uint32_t)i) % (uint32_t)nx) return;
  ctx->nx = nx;
}

KArgs wfh::base_args(wf_ctx* ctx, uint32_t* ctl, int64_t nitems) {
  KArgs a;
  std::memset(&a, 0, sizeof a);
  a.nitems = nitems;
  a.ctl = ctl;
  a.watchdog_ticks = ctx->watchdog_ticks;
  a.fault_band = ctx->fault;  // the fault hook fires on one launch only
  ctx->fault = 0;
  return a;
}

// ------------------------------------------------------------ tuning cache
// WF_TUNE_CACHE names a JSON file holding the autotuner's choices per shape class:
//   {"version": 2, "entries": [{"class": "...", "shape": 3, "order": 2, "wgs": 256, "ms": 3.8}, ...]}
// (shape: the band shape, see wf_host.h).
static void load_tune_cache(wf_ctx* ctx) {
  std::ifstream f(ctx->tune_file);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t at = 0;
  auto field = [&](size_t from, const char* key, size_t end, std::string* sval, double* nval) -> bool {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = t.find(k, from);
    if (p == std::string::npos || p >= end) return false;
    p = t.find(':', p + k.size());
    if (p == std::string::npos || p >= end) return false;
    ++p;
    while (p < end && (t[p] == ' ' || t[p] == '\t' || t[p] == '\n')) ++p;
    if (sval) {
      if (t[p] != '"') return false;
      const size_t q = t.find('"', p + 1);
      if (q == std::string::npos || q > end) return false;
      *sval = t.substr(p + 1, q - p - 1);
      return true;
    }
    char* e = nullptr;
    *nval = std::strtod(t.c_str() + p, &e);
    return e != t.c_str() + p;
  };
  while ((at = t.find('{', at + 1)) != std::string::npos) {
    const size_t end = t.find('}', at);
    if (end == std::string::npos) break;
    std::string cls;
    double bs = 0, order = 0, wgs = 0, ms = 0;
    if (field(at, "class", end, &cls, nullptr) && field(at, "shape", end, nullptr, &bs) &&
        field(at, "order", end, nullptr, &order) && field(at, "wgs", end, nullptr, &wgs)) {
      field(at, "ms", end, nullptr, &ms);
      if ((bs >= 1 && bs <= SHAPE_MAX) && (order == 1 || order == 2) && wgs >= 0) {
        TuneEntry e;
        e.bs = (int)bs;
        e.order = (int)order;
        e.wgs = (int)wgs;
        e.ms = ms;
        ctx->tuned[cls] = e;
      }
    }
    at = end;
  }
}

static void save_tune_cache(const wf_ctx* ctx) {
  if (ctx->tune_file.empty()) return;
  const std::string tmp = ctx->tune_file + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\"version\": 2, \"entries\": [";
    bool first = true;
    for (const auto& kv : ctx->tuned) {
      f << (first ? "\n" : ",\n") << "  {\"class\": \"" << kv.first << "\", \"shape\": " << kv.second.bs
        << ", \"order\": " << kv.second.order << ", \"wgs\": " << kv.second.wgs << ", \"ms\": " << kv.second.ms << "}";
      first = false;
    }
    f << "\n]}\n";
  }
  std::rename(tmp.c_str(), ctx->tune_file.c_str());
}

// ------------------------------------------------------------------ public
extern "C" wf_status wf_init(int device, wf_ctx** out) {
  if (!out) return fail(WF_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  WF_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(WF_EINVAL, "no such device");
  hipDeviceProp_t prop;
  WF_HIP(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(WF_EUNSUPPORTED, std::string("libwf is built for gfx950, device is ") + prop.gcnArchName);
  std::unique_ptr<wf_ctx> ctx(new wf_ctx);
  ctx->device = device;
  ctx->num_cus = prop.multiProcessorCount;
  if (const char* w = std::getenv("WF_WATCHDOG_MS")) {
    long ms = std::atol(w);
    if (ms > 0) ctx->watchdog_ticks = (uint64_t)ms * 100000ull;
  }
  if (const char* f = std::getenv("WF_FAULT")) {
    // Test hook, drop_hand:<band>: in the context's first launch the given band (of every
    // grid) never hands its bottom row on, so the band below waits until the watchdog
    // fires and the launch drains.
    if (std::strncmp(f, "drop_hand:", 10) == 0) ctx->fault = (uint32_t)std::atol(f + 10) + 1u;
  }
  if (const char* f = std::getenv("WF_TUNE_CACHE")) {
    ctx->tune_file = f;
    load_tune_cache(ctx.get());
  }
  wf_status st = set_device(ctx.get());
  if (st != WF_OK) return st;
  probe_xcds(ctx.get());
  // wf_solve_noalloc's slot: its control words and handoff rows are the device's fixed
  // array, looked up here with the device current; its pinned error word and event are
  // made now so that the entry point itself allocates nothing.
  {
    uint32_t* scr = nullptr;
    WF_HIP(noalloc_scratch(&scr));
    std::unique_ptr<Slot> s(new Slot);
    s->external = true;
    s->reserved = true;
    s->ctl = scr;
    s->hand = scr + NOALLOC_CTL_WORDS;
    s->hand_cap = (size_t)(NOALLOC_WORDS - NOALLOC_CTL_WORDS);
    s->needs_rearm = true;
    WF_HIP(hipHostMalloc(&s->host_err, sizeof(uint32_t), hipHostMallocDefault));
    *s->host_err = 0;
    if (hipEventCreateWithFlags(&s->done, hipEventDisableTiming) != hipSuccess) {
      hipHostFree(s->host_err);
      return fail(WF_EHIP, "hipEventCreateWithFlags failed");
    }
    ctx->noalloc = s.get();
    ctx->slots.push_back(std::move(s));
  }
  *out = ctx.release();
  return WF_OK;
}

static void drop_plan(BatchPlanEntry& e, wf_ctx* ctx) {
  for (auto& L : e.lanes) {
    if (L.slot >= 0) {
      Slot& s = *ctx->slots[(size_t)L.slot];
      note(ctx, harvest(s, true));
      s.reserved = false;
    }
    if (L.exec) hipGraphExecDestroy(L.exec);
    if (L.graph) hipGraphDestroy(L.graph);
    if (L.staging) hipHostFree(L.staging);
    L = BatchPlanEntry::Lane();
  }
}

extern "C" wf_status wf_destroy(wf_ctx* ctx) {
  if (!ctx) return WF_OK;
  set_device(ctx);
  hipDeviceSynchronize();
  for (auto& e : ctx->plans) drop_plan(*e, ctx);
  for (auto& sp : ctx->slots) {
    Slot& s = *sp;
    if (s.external) {  // ctl and hand are not the slot's
      if (s.host_err) hipHostFree(s.host_err);
      if (s.done) hipEventDestroy(s.done);
      continue;
    }
    if (s.ctl) hipFree(s.ctl);
    if (s.hand) hipFree(s.hand);
    if (s.grids) hipFree(s.grids);
    if (s.items) hipFree(s.items);
    if (s.host_err) hipHostFree(s.host_err);
    if (s.done) hipEventDestroy(s.done);
  }
  delete ctx;
  return WF_OK;
}

extern "C" wf_status wf_set_watchdog(wf_ctx* ctx, int64_t ms) {
  if (!ctx) return fail(WF_EINVAL, "ctx is NULL");
  if (ms < 0 || ms > 3600 * 1000) return fail(WF_EINVAL, "watchdog must be 0 .. 3600000 ms");
  ctx->watchdog_ticks = (uint64_t)ms * 100000ull;
  return WF_OK;
}

// Wait for every launch of the context and report a device error, if any.
extern "C" wf_status wf_check(wf_ctx* ctx) {
  if (!ctx) return fail(WF_EINVAL, "ctx is NULL");
  wf_status st = set_device(ctx);
  if (st != WF_OK) return st;
  wf_status res = ctx->sticky;
  ctx->sticky = WF_OK;
  for (auto& s : ctx->slots) {
    wf_status r = harvest(*s, true);
    if (r != WF_OK && res == WF_OK) res = r;
  }
  if (res == WF_ETIMEDOUT) return fail(WF_ETIMEDOUT, "device watchdog fired");
  return res;
}

static wf_status report_sticky(wf_ctx* ctx) {
  // Non-blocking look at finished launches; report a device error once.
  for (auto& s : ctx->slots) {
    wf_status r = harvest(*s, false);
    if (r != WF_PENDING) note(ctx, r);
  }
  if (ctx->sticky != WF_OK) {
    wf_status s = ctx->sticky;
    ctx->sticky = WF_OK;
    return fail(s, s == WF_ETIMEDOUT ? "a previous launch on this context timed out"
                                     : "a previous launch on this context failed");
  }
  return WF_OK;
}

// One grid, one launch, at W compute waves per workgroup.
static wf_status solve_one(wf_ctx* ctx, const wf_problem* p, int bs, int max_wgs, hipStream_t stream) {
  Slot* s = nullptr;
  wf_status st = acquire_slot(ctx, &s);
  if (st != WF_OK) return st;
  st = ensure_hand(*s, hand_elems(p, bs), sentinel_of(p->dtype), stream);
  if (st != WF_OK) return st;
  KArgs a = base_args(ctx, s->ctl, 0);
  a.g0 = make_desc(p, bs, s->hand);
  a.nitems = a.g0.nbands;
  const int resident = ctx->num_cus * wgs_per_cu(bs, p->dtype);
  int nwg = (int)std::min<int64_t>(a.nitems, resident);
  if (max_wgs > 0) nwg = std::min(nwg, max_wgs);
  xcd_queues(ctx, a, nwg);
  // Optional trace (profiling hook): WF_TRACE_FILE=<path> makes wf_solve synchronous
  // and writes TRACE_WORDS uint64 per (band, compute wave) to <path>.
  const char* trace_file = std::getenv("WF_TRACE_FILE");
  uint64_t* trace = nullptr;
  const size_t trace_words = (size_t)a.nitems * shape_waves(bs) * TRACE_WORDS;
  // With WF_TRACE_CHUNKS=1 it also writes CTRACE_WORDS uint64 per (band, compute wave, chunk).
  const int64_t nc = ((4 * groups_for(p->n, shape_rows_per_lane(bs)) + 15) / 16 + CTRACE_EVERY - 1) / CTRACE_EVERY;
  const bool chunks = trace_file && *trace_file && std::getenv("WF_TRACE_CHUNKS");
  const size_t ctrace_words = chunks ? (size_t)a.nitems * shape_waves(bs) * (size_t)nc * CTRACE_WORDS : 0;
  uint64_t* ctrace = nullptr;
  if (trace_file && *trace_file) {
    WF_HIP(hipMalloc(&trace, trace_words * sizeof(uint64_t)));
    WF_HIP(launch_fill_u32((uint32_t*)trace, 0u, (int64_t)trace_words * 2, stream));
    a.trace = trace;
    if (chunks) {
      WF_HIP(hipMalloc(&ctrace, ctrace_words * sizeof(uint64_t)));
      WF_HIP(launch_fill_u32((uint32_t*)ctrace, 0u, (int64_t)ctrace_words * 2, stream));
      a.ctrace = ctrace;
      a.ctrace_nc = nc;
    }
  }
  WF_HIP(launch_fill_u32(s->ctl, 0u, CTL_WORDS, stream));
  WF_HIP(launch_shape(p->dtype, p->rule, bs, nwg, a, stream));
  if (trace) {
    std::vector<uint64_t> host(trace_words), chost(ctrace_words);
    WF_HIP(hipMemcpyAsync(host.data(), trace, trace_words * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    if (ctrace)
      WF_HIP(hipMemcpyAsync(chost.data(), ctrace, ctrace_words * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    WF_HIP(hipStreamSynchronize(stream));
    WF_HIP(hipFree(trace));
    if (ctrace) WF_HIP(hipFree(ctrace));
    if (FILE* f = std::fopen(trace_file, "wb")) {
      const uint64_t hdr[6] = {(uint64_t)a.nitems, (uint64_t)shape_waves(bs), (uint64_t)TRACE_WORDS, (uint64_t)nwg,
                               (uint64_t)(ctrace ? nc : 0), (uint64_t)CTRACE_WORDS};
      std::fwrite(hdr, sizeof hdr, 1, f);
      std::fwrite(host.data(), sizeof(uint64_t), host.size(), f);
      if (ctrace) std::fwrite(chost.data(), sizeof(uint64_t), chost.size(), f);
      std::fclose(f);
    }
  }
  return finish_launch(*s, stream, a.nx > 1);
}

static wf_status solve_entry(wf_ctx* ctx, const wf_problem* p, const wf_tuning* t, void* stream_) {
  if (!ctx) return fail(WF_EINVAL, "ctx is NULL");
  wf_status st = check_problem(p, -1);
  if (st != WF_OK) return st;
  wf_tuning tun;
  std::memset(&tun, 0, sizeof tun);
  if (t) tun = *t;
  st = check_tuning(tun);
  if (st != WF_OK) return st;
  st = set_device(ctx);
  if (st != WF_OK) return st;
  st = report_sticky(ctx);
  if (st != WF_OK) return st;
  if (p->m == 0 || p->n == 0) return WF_OK;
  const int bs = shape_of_tuning(tun, p->m);
  if (p->dtype == WF_F64 && bs != 1) return fail(WF_EUNSUPPORTED, "fp64 grids use 64-row bands only");
  return solve_one(ctx, p, bs, tun.max_wgs, (hipStream_t)stream_);
}

extern "C" wf_status wf_solve(wf_ctx* ctx, const wf_problem* p, void* stream) {
  return solve_entry(ctx, p, nullptr, stream);
}

// wf_solve on the fixed device array: the same launch as solve_one at one compute wave
// per workgroup, with nothing allocated.  The handoff rows the problem uses are re-armed
// on `stream` before every launch (a kernel, not hipMemsetAsync, so the call may be
// captured in a graph): the array is shared by every call on the device, so what an
// earlier call (or an aborted launch) left there is never trusted.  The call never waits
// for an earlier one: the device error word accumulates across launches and is copied to
// the slot's pinned word after each, so the latest copy covers every launch before it;
// once the host has seen an error there, the next call clears the word.
extern "C" wf_status wf_solve_noalloc(wf_ctx* ctx, const wf_problem* p, void* stream_) {
  if (!ctx) return fail(WF_EINVAL, "ctx is NULL");
  wf_status st = check_problem(p, -1);
  if (st != WF_OK) return st;
  if (!ctx->noalloc) return fail(WF_EHIP, "the context has no fixed workspace");
  const int bs = choose_shape(p->m);
  const size_t need = hand_elems(p, bs);
  if (p->m > 0 && p->n > 0 && need > ctx->noalloc->hand_cap) {
    char msg[200];
    snprintf(msg, sizeof msg, "problem needs %lld bytes of handoff rows; the fixed workspace holds %lld "
             "(WF_NOALLOC_SCRATCH_BYTES, less 256 bytes of control words)",
             (long long)(need * 4), (long long)(ctx->noalloc->hand_cap * 4));
    return fail(WF_E2BIG, msg);
  }
  st = set_device(ctx);
  if (st != WF_OK) return st;
  st = report_sticky(ctx);
  if (st != WF_OK) return st;
  if (p->m == 0 || p->n == 0) return WF_OK;
  Slot& s = *ctx->noalloc;
  hipStream_t stream = (hipStream_t)stream_;
  KArgs a = base_args(ctx, s.ctl, 0);
  a.g0 = make_desc(p, bs, s.hand);
  a.nitems = a.g0.nbands;
  const int nwg = (int)std::min<int64_t>(a.nitems, (int64_t)ctx->num_cus * wgs_per_cu(bs, p->dtype));
  xcd_queues(ctx, a, nwg);
  WF_HIP(launch_noalloc_prep(s.ctl, s.needs_rearm, s.hand, sentinel_of(p->dtype), (int64_t)need, stream));
  s.needs_rearm = false;
  WF_HIP(launch_shape(p->dtype, p->rule, bs, nwg, a, stream));
  return finish_launch(s, stream, a.nx > 1);
}

extern "C" wf_status wf_traceback(wf_ctx* ctx, const wf_problem* p, int32_t* path, int64_t* length, void* stream) {
  if (!ctx) return fail(WF_EINVAL, "ctx is NULL");
  if (!p || !path || !length) return fail(WF_EINVAL, "NULL problem, path or length");
  if (p->m < 1 || p->n < 1) return fail(WF_EINVAL, "traceback needs m, n >= 1");
  if (p->dtype != WF_F32 && p->dtype != WF_I32 && p->dtype != WF_F64) return fail(WF_EINVAL, "unknown dtype");
  if (p->rule != WF_RULE_MIN && p->rule != WF_RULE_MAX) return fail(WF_EINVAL, "unknown rule");
  if (!p->out) return fail(WF_EINVAL, "out (the computed grid) is NULL");
  if (p->ld_out < p->n) return fail(WF_EINVAL, "ld_out < n");
  wf_status st = set_device(ctx);
  if (st != WF_OK) return st;
  st = report_sticky(ctx);
  if (st != WF_OK) return st;
  WF_HIP(launch_traceback(p->dtype, p->rule, p->out, p->ld_out, p->m, p->n, p->top, p->left, path,
                          length, (hipStream_t)stream));
  return WF_OK;
}

extern "C" wf_status wf_solve_tuned(wf_ctx* ctx, const wf_problem* p, const wf_tuning* t, void* stream) {
  return solve_entry(ctx, p, t, stream);
}

extern "C" wf_status wf_solve_each(wf_ctx* ctx, const wf_problem* ps, int64_t count, void* const* streams,
                                   int32_t nstreams) {
  if (!ctx) return fail(WF_EINVAL, "ctx is NULL");
  if (count < 0 || (count > 0 && !ps)) return fail(WF_EINVAL, "bad problem array");
  if (nstreams < 1 || !streams) return fail(WF_EINVAL, "need at least one stream");
  for (int64_t i = 0; i < count; ++i) {
    wf_status st = check_problem(&ps[i], i);
    if (st != WF_OK) return st;
  }
  wf_status st = set_device(ctx);
  if (st != WF_OK) return st;
  st = report_sticky(ctx);
  if (st != WF_OK) return st;
  for (int64_t i = 0; i < count; ++i) {
    if (ps[i].m == 0 || ps[i].n == 0) continue;
    st = solve_one(ctx, &ps[i], choose_shape(ps[i].m), 0, (hipStream_t)streams[i % nstreams]);
    if (st != WF_OK) return st;
  }
  return WF_OK;
}

// ----------------------------------------------------------------- batched
static uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Grids in work order (largest first, so long critical paths start early) and the
// (grid, band) work list: grid-major (order 1) or band-interleaved (order 2).
static void build_work(const wf_problem* ps, int64_t count, int bs, int order, std::vector<int64_t>& perm,
                       std::vector<Item>& items, std::vector<size_t>& hand_off, size_t& hand_total) {
  perm.clear();
  items.clear();
  for (int64_t i = 0; i < count; ++i)
    if (ps[i].m > 0 && ps[i].n > 0) perm.push_back(i);
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int64_t a, int64_t b) { return ps[a].m * ps[a].n > ps[b].m * ps[b].n; });
  hand_off.resize(perm.size());
  hand_total = 0;
  std::vector<int32_t> nb(perm.size());
  int64_t max_bands = 0;
  for (size_t gi = 0; gi < perm.size(); ++gi) {
    hand_off[gi] = hand_total;
    hand_total += hand_elems(&ps[perm[gi]], bs);
    nb[gi] = (int32_t)((ps[perm[gi]].m + shape_rows(bs) - 1) / shape_rows(bs));
    max_bands = std::max<int64_t>(max_bands, nb[gi]);
  }
  if (order == 2) {
    for (int64_t b = 0; b < max_bands; ++b)
      for (size_t gi = 0; gi < perm.size(); ++gi)
        if (b < nb[gi]) items.push_back(Item{(uint32_t)gi, (uint32_t)b});
  } else {
    for (size_t gi = 0; gi < perm.size(); ++gi)
      for (int32_t b = 0; b < nb[gi]; ++b) items.push_back(Item{(uint32_t)gi, (uint32_t)b});
  }
}

static int batch_wgs(const wf_ctx* ctx, int bs, int dtype, int64_t nitems, int max_wgs) {
  int nwg = (int)std::min<int64_t>(nitems, (int64_t)ctx->num_cus * wgs_per_cu(bs, dtype));
  if (max_wgs > 0) nwg = std::min(nwg, max_wgs);
  return std::max(nwg, 1);
}

// A batched launch that is not kept for replay (autotuning trials, plain launches).
static wf_status batched_once(wf_ctx* ctx, const wf_problem* ps, int64_t count, int bs, int order, int max_wgs,
                              hipStream_t stream) {
  std::vector<int64_t> perm;
  std::vector<Item> items;
  std::vector<size_t> hand_off;
  size_t hand_total = 0;
  build_work(ps, count, bs, order, perm, items, hand_off, hand_total);
  if (items.empty()) return WF_OK;
  Slot* s = nullptr;
  wf_status st = acquire_slot(ctx, &s);
  if (st != WF_OK) return st;
  st = ensure_hand(*s, hand_total, sentinel_of(ps[perm[0]].dtype), stream);
  if (st == WF_OK) st = ensure_buf(&s->grids, &s->grids_cap, perm.size());
  if (st == WF_OK) st = ensure_buf(&s->items, &s->items_cap, items.size());
  if (st != WF_OK) return st;
  std::vector<GridDesc> descs(perm.size());
  for (size_t gi = 0; gi < perm.size(); ++gi) descs[gi] = make_desc(&ps[perm[gi]], bs, s->hand + hand_off[gi]);
  WF_HIP(hipMemcpyAsync(s->grids, descs.data(), descs.size() * sizeof(GridDesc), hipMemcpyHostToDevice, stream));
  WF_HIP(hipMemcpyAsync(s->items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice, stream));
  WF_HIP(hipStreamSynchronize(stream));  // the host arrays must outlive the copies
  KArgs a = base_args(ctx, s->ctl, (int64_t)items.size());
  a.grids = s->grids;
  a.items = s->items;
  WF_HIP(launch_fill_u32(s->ctl, 0u, CTL_WORDS, stream));
  WF_HIP(launch_shape(ps[perm[0]].dtype, ps[perm[0]].rule, bs, batch_wgs(ctx, bs, ps[perm[0]].dtype, a.nitems, max_wgs), a, stream));
  return finish_launch(*s, stream);
}

static std::vector<int64_t> shape_of(const wf_problem* ps, int64_t count) {
  std::vector<int64_t> v((size_t)count * 3);
  for (int64_t i = 0; i < count; ++i) {
    v[3 * i] = ps[i].m;
    v[3 * i + 1] = ps[i].n;
    v[3 * i + 2] = ps[i].mode;
  }
  return v;
}

// A cached batch plan: found by the batch's shapes and configuration, replayed with
// two lanes in turn.  Its tables are rebuilt only when the problem array changes.
static wf_status batched_plan(wf_ctx* ctx, const wf_problem* ps, int64_t count, int bs, int order, int max_wgs,
                              bool use_graph, hipStream_t stream) {
  const uint64_t cfg[5] = {(uint64_t)count, (uint64_t)bs, (uint64_t)order, (uint64_t)max_wgs, (uint64_t)use_graph};
  uint64_t h = fnv1a(1469598103934665603ull, cfg, sizeof cfg);
  const int dtype = ps[0].dtype, rule = ps[0].rule;
  const uint64_t dr[2] = {(uint64_t)dtype, (uint64_t)rule};
  h = fnv1a(h, dr, sizeof dr);
  BatchPlanEntry* e = nullptr;
  // Fast path: the very problem array of the plan's last launch.
  for (auto& p : ctx->plans)
    if (p->probs.size() == (size_t)count && p->bs == bs && p->order == order && p->use_graph == use_graph &&
        p->dtype == dtype && p->rule == rule &&
        std::memcmp(p->probs.data(), ps, (size_t)count * sizeof(wf_problem)) == 0) {
      e = p.get();
      break;
    }
  if (!e) {
    std::vector<int64_t> shape = shape_of(ps, count);
    h = fnv1a(h, shape.data(), shape.size() * sizeof(int64_t));
    for (auto& p : ctx->plans)
      if (p->hash == h && p->shape == shape && p->bs == bs && p->order == order && p->use_graph == use_graph &&
          p->dtype == dtype && p->rule == rule && p->probs.size() == (size_t)count) {
        e = p.get();
        break;
      }
    if (!e) {
      // New plan; evict the least recently used one beyond MAX_PLANS.
      if ((int)ctx->plans.size() >= wf_ctx::MAX_PLANS) {
        size_t lru = 0;
        for (size_t i = 1; i < ctx->plans.size(); ++i)
          if (ctx->plans[i]->last_use < ctx->plans[lru]->last_use) lru = i;
        drop_plan(*ctx->plans[lru], ctx);
        ctx->plans.erase(ctx->plans.begin() + (long)lru);
      }
      std::unique_ptr<BatchPlanEntry> n(new BatchPlanEntry);
      n->hash = h;
      n->shape = std::move(shape);
      n->bs = bs;
      n->order = order;
      n->dtype = dtype;
      n->rule = rule;
      n->use_graph = use_graph;
      build_work(ps, count, bs, order, n->perm, n->items, n->hand_off, n->hand_total);
      n->nwg = batch_wgs(ctx, bs, dtype, (int64_t)n->items.size(), max_wgs);
      ctx->plans.push_back(std::move(n));
      e = ctx->plans.back().get();
    }
    e->probs.assign(ps, ps + count);
  }
  e->last_use = ++ctx->use_clock;
  if (e->items.empty()) return WF_OK;
  BatchPlanEntry::Lane& L = e->lanes[e->replays % 2];
  ++e->replays;
  if (L.slot < 0) {
    Slot* s = nullptr;
    wf_status st = acquire_slot(ctx, &s);
    if (st != WF_OK) return st;
    s->reserved = true;
    for (size_t i = 0; i < ctx->slots.size(); ++i)
      if (ctx->slots[i].get() == s) L.slot = (int)i;
  }
  Slot& s = *ctx->slots[(size_t)L.slot];
  // The lane's previous replay must have finished before its tables or error word are reused.
  wf_status st = note(ctx, harvest(s, true));
  if (st != WF_OK) return st;
  st = ensure_hand(s, e->hand_total, sentinel_of(dtype), stream);
  if (st == WF_OK) st = ensure_buf(&s.grids, &s.grids_cap, e->perm.size());
  if (st == WF_OK) st = ensure_buf(&s.items, &s.items_cap, e->items.size());
  if (st != WF_OK) return st;
  if (!L.items_loaded) {
    // Synchronous: the plan's work list never changes, so this happens once per lane.
    WF_HIP(hipMemcpy(s.items, e->items.data(), e->items.size() * sizeof(Item), hipMemcpyHostToDevice));
    L.items_loaded = true;
  }
  std::vector<GridDesc> descs(e->perm.size());
  for (size_t gi = 0; gi < e->perm.size(); ++gi) descs[gi] = make_desc(&ps[e->perm[gi]], bs, s.hand + e->hand_off[gi]);
  if (L.descs.size() != descs.size() ||
      std::memcmp(L.descs.data(), descs.data(), descs.size() * sizeof(GridDesc)) != 0) {
    if (!L.staging) WF_HIP(hipHostMalloc((void**)&L.staging, descs.size() * sizeof(GridDesc), hipHostMallocDefault));
    std::memcpy(L.staging, descs.data(), descs.size() * sizeof(GridDesc));
    WF_HIP(hipMemcpyAsync(s.grids, L.staging, descs.size() * sizeof(GridDesc), hipMemcpyHostToDevice, stream));
    L.descs = std::move(descs);
  }
  KArgs a = base_args(ctx, s.ctl, (int64_t)e->items.size());
  a.grids = s.grids;
  a.items = s.items;
  if (use_graph) {
    if (!L.exec) {
      hipStream_t cap = nullptr;
      WF_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      hipError_t err = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (err == hipSuccess) {
        launch_fill_u32(s.ctl, 0u, CTL_WORDS, cap);
        launch_shape(dtype, rule, bs, e->nwg, a, cap);
        err = hipStreamEndCapture(cap, &L.graph);
      }
      if (err == hipSuccess) err = hipGraphInstantiate(&L.exec, L.graph, nullptr, nullptr, 0);
      hipStreamDestroy(cap);
      if (err != hipSuccess) return fail(WF_EHIP, std::string("graph capture: ") + hipGetErrorString(err));
    }
    WF_HIP(hipGraphLaunch(L.exec, stream));
  } else {
    WF_HIP(launch_fill_u32(s.ctl, 0u, CTL_WORDS, stream));
    WF_HIP(launch_shape(dtype, rule, bs, e->nwg, a, stream));
  }
  return finish_launch(s, stream);
}

// ------------------------------------------------------------- autotuning
// Shape class of a batch: dtype, rule, modes, and the binary magnitudes of the grid
// count, the total cells, the tallest and the widest grid.  Batches of one class
// share a tuned configuration.
static std::string shape_class(const wf_problem* ps, int64_t count) {
  int64_t cells = 0, mm = 0, mn = 0, full = 0, edges = 0;
  for (int64_t i = 0; i < count; ++i) {
    cells += ps[i].m * ps[i].n;
    mm = std::max(mm, ps[i].m);
    mn = std::max(mn, ps[i].n);
    (ps[i].mode == WF_MODE_FULL ? full : edges)++;
  }
  auto lg = [](int64_t v) { return v > 0 ? (int)std::floor(std::log2((double)v)) : -1; };
  char buf[128];
  snprintf(buf, sizeof buf, "d%d.r%d.%s.g%d.c%d.m%d.n%d", ps[0].dtype, ps[0].rule,
           edges == 0 ? "full" : (full == 0 ? "edges" : "mixed"), lg(count), lg(cells), lg(mm), lg(mn));
  return buf;
}

// Candidates: band shape (64-row bands; 128-row bands of two chained compute waves;
// 128-row bands of one wave with two rows per lane) x work order x workgroup count
// (every resident workgroup, or half of them).  Each runs twice back to back on `stream`, the second
// run timed with events (its host set-up overlaps the first run on the device).
static wf_status autotune(wf_ctx* ctx, const wf_problem* ps, int64_t count, int max_wgs, hipStream_t stream,
                          TuneEntry* out) {
  const std::string cls = shape_class(ps, count);
  auto it = ctx->tuned.find(cls);
  if (it != ctx->tuned.end()) {
    *out = it->second;
    return WF_OK;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  WF_HIP(hipEventCreate(&e0));
  WF_HIP(hipEventCreate(&e1));
  TuneEntry best;
  best.ms = -1;
  wf_status st = WF_OK;
  // fp64 grids have one band shape only.
  const int max_shape = ps[0].dtype == WF_F64 ? 1 : SHAPE_MAX;
  for (int bs = 1; bs <= max_shape && st == WF_OK; ++bs) {
    const int resident = ctx->num_cus * wgs_per_cu(bs, ps[0].dtype);
    const int wg_opts[2] = {max_wgs > 0 ? std::min(max_wgs, resident) : resident,
                            std::max(1, (max_wgs > 0 ? std::min(max_wgs, resident) : resident) / 2)};
    for (int order = 1; order <= 2 && st == WF_OK; ++order) {
      for (int wi = 0; wi < 2 && st == WF_OK; ++wi) {
        const int wgs = wg_opts[wi];
        st = batched_once(ctx, ps, count, bs, order, wgs, stream);
        if (st != WF_OK) break;
        hipError_t e = hipEventRecord(e0, stream);
        if (e == hipSuccess) st = batched_once(ctx, ps, count, bs, order, wgs, stream);
        if (st == WF_OK && e == hipSuccess) e = hipEventRecord(e1, stream);
        if (st == WF_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (st == WF_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (st == WF_OK && e != hipSuccess) st = fail(WF_EHIP, std::string("autotune: ") + hipGetErrorString(e));
        if (st != WF_OK) break;
        st = report_sticky(ctx);
        if (st != WF_OK) break;
        if (best.ms < 0 || ms < best.ms) {
          best.ms = ms;
          best.bs = bs;
          best.order = order;
          best.wgs = wgs;
        }
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != WF_OK) return st;
  ctx->tuned[cls] = best;
  save_tune_cache(ctx);
  *out = best;
  return WF_OK;
}

extern "C" wf_status wf_solve_batched(wf_ctx* ctx, const wf_problem* ps, int64_t count, const wf_tuning* t,
                                      void* stream_) {
  if (!ctx) return fail(WF_EINVAL, "ctx is NULL");
  if (count < 0 || (count > 0 && !ps)) return fail(WF_EINVAL, "bad problem array");
  if (count == 0) return WF_OK;
  for (int64_t i = 0; i < count; ++i) {
    wf_status st = check_problem(&ps[i], i);
    if (st != WF_OK) return st;
    if (ps[i].dtype != ps[0].dtype || ps[i].rule != ps[0].rule)
      return fail(WF_EUNSUPPORTED, "all problems of a batch must share dtype and rule");
  }
  wf_tuning tun;
  std::memset(&tun, 0, sizeof tun);
  if (t) tun = *t;
  wf_status st = check_tuning(tun);
  if (st != WF_OK) return st;
  st = set_device(ctx);
  if (st != WF_OK) return st;
  st = report_sticky(ctx);
  if (st != WF_OK) return st;
  hipStream_t stream = (hipStream_t)stream_;
  bool any = false;
  for (int64_t i = 0; i < count && !any; ++i) any = ps[i].m > 0 && ps[i].n > 0;
  if (!any) return WF_OK;
  int bs = 0, order = tun.order, wgs = tun.max_wgs;
  if (tun.waves_per_wg != 0 || tun.rows_per_lane != 0) bs = shape_of_tuning(tun, 0);
  if (bs == 0 && order == 0 && tun.use_graph != -1) {
    TuneEntry te;
    st = autotune(ctx, ps, count, tun.max_wgs, stream, &te);
    if (st != WF_OK) return st;
    bs = te.bs;
    order = te.order;
    wgs = te.wgs;
  }
  if (bs == 0) bs = 1;
  if (ps[0].dtype == WF_F64 && bs != 1) return fail(WF_EUNSUPPORTED, "fp64 grids use 64-row bands only");
  if (order == 0) order = 1;
  if (tun.use_graph == 1) return batched_plan(ctx, ps, count, bs, order, wgs, true, stream);
  return batched_once(ctx, ps, count, bs, order, wgs, stream);
}

// ------------------------------------------------------------- measurement
namespace wfk {
hipError_t launch_chain_probe(float* out, uint64_t* ticks, int steps, hipStream_t stream);
}

extern "C" wf_status wf_measure_step_ns(wf_ctx* ctx, int64_t steps, double* ns_per_step) {
  if (!ctx || !ns_per_step) return fail(WF_EINVAL, "ctx and ns_per_step must not be NULL");
  if (steps < 16 || steps > ((int64_t)1 << 30)) return fail(WF_EINVAL, "steps must be 16 .. 2^30");
  wf_status st = set_device(ctx);
  if (st != WF_OK) return st;
  float* out = nullptr;
  uint64_t* ticks = nullptr;
  WF_HIP(hipMalloc(&out, 64 * sizeof(float)));
  WF_HIP(hipMalloc(&ticks, sizeof(uint64_t)));
  uint64_t h = 0;
  hipError_t e = launch_chain_probe(out, ticks, (int)(steps / 16 * 16), nullptr);
  if (e == hipSuccess) e = hipMemcpy(&h, ticks, sizeof h, hipMemcpyDeviceToHost);
  hipFree(out);
  hipFree(ticks);
  if (e != hipSuccess) return fail(WF_EHIP, std::string("step probe: ") + hipGetErrorString(e));
  *ns_per_step = (double)h * 10.0 / (double)(steps / 16 * 16);  // the wall clock runs at 100 MHz
  return WF_OK;
}
