// wf_runtime.cpp -- the C ABI of libwf (include/wf.h): argument checking,
// per-context workspace, launch configuration, batched work lists with hipGraph
// replay, and error reporting.
#include "../../include/wf.h"
#include "wf_internal.h"
#include "wf_host.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
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

extern "C" const char* wf_version(void) { return "libwf 0.1 (gfx950)"; }

wf_status wfh::set_device(wf_ctx* ctx) {
  int cur = -1;
  WF_HIP(hipGetDevice(&cur));
  if (cur != ctx->device) WF_HIP(hipSetDevice(ctx->device));
  return WF_OK;
}

// Reads the device status of a finished slot; re-arms its handoff rows after an abort.
static wf_status harvest(wf_ctx* ctx, Slot& s, hipStream_t stream, bool wait) {
  if (!s.pending) return WF_OK;
  hipError_t q = wait ? hipEventSynchronize(s.done) : hipEventQuery(s.done);
  if (q == hipErrorNotReady) return WF_PENDING;
  if (q != hipSuccess) return fail(WF_EHIP, std::string("launch failed: ") + hipGetErrorString(q));
  s.pending = false;
  if (*s.host_err != DEV_OK) {
    *s.host_err = DEV_OK;
    if (s.hand && s.hand_cap) {
      hipError_t e = launch_fill_u32(s.hand, s.hand_sent, (int64_t)s.hand_cap, stream);
      if (e != hipSuccess) return fail(WF_EHIP, std::string("re-arm: ") + hipGetErrorString(e));
    }
    return fail(WF_ETIMEDOUT, "device watchdog fired: a wait for a neighbouring band exceeded the limit "
                              "(NaN or reserved-value inputs, or an oversubscribed device)");
  }
  return WF_OK;
}

static wf_status acquire_slot(wf_ctx* ctx, hipStream_t stream, Slot** out, int* index) {
  const int i = ctx->next_slot;
  ctx->next_slot = (ctx->next_slot + 1) % wf_ctx::NSLOT;
  Slot& s = ctx->slots[i];
  wf_status st = harvest(ctx, s, stream, true);
  if (st == WF_ETIMEDOUT) ctx->sticky = WF_ETIMEDOUT;
  else if (st != WF_OK) return st;
  if (!s.ctl) {
    WF_HIP(hipMalloc(&s.ctl, CTL_WORDS * sizeof(uint32_t)));
    WF_HIP(hipHostMalloc(&s.host_err, sizeof(uint32_t), hipHostMallocDefault));
    *s.host_err = 0;
    WF_HIP(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
  }
  *out = &s;
  if (index) *index = i;
  return WF_OK;
}

static wf_status ensure_hand(Slot& s, size_t need, uint32_t sent, hipStream_t stream) {
  if (need == 0) need = 64;
  if (s.hand_cap < need) {
    if (s.hand) WF_HIP(hipFree(s.hand));
    s.hand = nullptr;
    s.hand_cap = 0;
    size_t cap = std::max(need, s.hand_cap * 2);
    if (hipMalloc(&s.hand, cap * sizeof(uint32_t)) != hipSuccess) {
      s.hand = nullptr;
      return fail(WF_ENOMEM, "cannot allocate handoff rows");
    }
    s.hand_cap = cap;
    s.hand_sent = sent;
    WF_HIP(launch_fill_u32(s.hand, sent, (int64_t)cap, stream));
  } else if (s.hand_sent != sent) {
    s.hand_sent = sent;
    WF_HIP(launch_fill_u32(s.hand, sent, (int64_t)s.hand_cap, stream));
  }
  return WF_OK;
}

template <class T>
static wf_status ensure_buf(T** p, size_t* cap, size_t need) {
  if (*cap >= need) return WF_OK;
  if (*p) WF_HIP(hipFree(*p));
  *p = nullptr;
  *cap = 0;
  size_t c = std::max<size_t>(need, 64);
  if (hipMalloc(p, c * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return fail(WF_ENOMEM, "cannot allocate descriptor table");
  }
  *cap = c;
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
  if (p->dtype != WF_F32 && p->dtype != WF_I32) return fail(WF_EINVAL, std::string(where) + "unknown dtype");
  if (p->rule != WF_RULE_MIN && p->rule != WF_RULE_MAX) return fail(WF_EINVAL, std::string(where) + "unknown rule");
  if (p->mode != WF_MODE_FULL && p->mode != WF_MODE_EDGES) return fail(WF_EINVAL, std::string(where) + "unknown mode");
  if (p->flags != 0) return fail(WF_EINVAL, std::string(where) + "flags must be 0");
  if (p->m == 0 || p->n == 0) return WF_OK;
  if (!p->cost) return fail(WF_EINVAL, std::string(where) + "cost is NULL");
  if (p->ld_cost < p->n) return fail(WF_EINVAL, std::string(where) + "ld_cost < n");
  if (p->ld_cost > MAX_N) return fail(WF_EUNSUPPORTED, std::string(where) + "ld_cost above 2^23 is not supported");
  if (p->mode == WF_MODE_FULL) {
    if (!p->out) return fail(WF_EINVAL, std::string(where) + "out is NULL in FULL mode");
    if (p->ld_out < p->n) return fail(WF_EINVAL, std::string(where) + "ld_out < n");
  } else if (!p->last_row && !p->last_col && !p->final_cell) {
    return fail(WF_EINVAL, std::string(where) + "EDGES mode needs last_row, last_col or final_cell");
  }
  return WF_OK;
}

// ------------------------------------------------------------ configuration
int wfh::choose_waves(int64_t m) {
  // Bands of 64*W rows.  A workgroup's W strips share one compute unit's memory
  // pipeline (each strip has its own loader and storer), and that sharing costs more
  // than the LDS handoff between them saves: one strip per workgroup, spread over the
  // compute units, is fastest for a single grid.
  (void)m;
  return 1;
}

// The LDS rings of one compute wave take about 65 KB of a compute unit's 160 KB.
int wfh::wgs_per_cu(int W) { return W >= 2 ? 1 : 2; }

uint32_t wfh::sentinel_of(int dtype) { return dtype == WF_F32 ? SENT_F32 : SENT_I32; }

GridDesc wfh::make_desc(const wf_problem* p, int W, uint32_t* hand) {
  GridDesc d;
  d.cost = p->cost;
  d.out = p->mode == WF_MODE_FULL ? p->out : nullptr;
  d.top = p->top;
  d.left = p->left;
  d.last_row = p->last_row;
  d.last_col = p->last_col;
  d.final_cell = p->final_cell;
  d.hand = hand;
  d.m = p->m;
  d.n = p->n;
  d.ld_cost = p->ld_cost;
  d.ld_out = p->mode == WF_MODE_FULL ? p->ld_out : 0;
  d.hand_ld = hand_ld_for(p->n);
  d.mode = p->mode;
  d.nbands = (int32_t)((p->m + 64 * W - 1) / (64 * W));
  return d;
}

size_t wfh::hand_elems(const wf_problem* p, int W) {
  const int64_t nb = (p->m + 64 * W - 1) / (64 * W);
  return nb > 1 ? (size_t)(nb - 1) * (size_t)hand_ld_for(p->n) : 0;
}

static wf_status finish_launch(Slot& s, hipStream_t stream) {
  WF_HIP(hipMemcpyAsync(s.host_err, s.ctl + CTL_ERROR, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
  WF_HIP(hipEventRecord(s.done, stream));
  s.pending = true;
  return WF_OK;
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
  wf_status st = set_device(ctx.get());
  if (st != WF_OK) return st;
  *out = ctx.release();
  return WF_OK;
}

extern "C" wf_status wf_destroy(wf_ctx* ctx) {
  if (!ctx) return WF_OK;
  set_device(ctx);
  hipDeviceSynchronize();
  for (auto& kv : ctx->graphs) {
    if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) hipGraphDestroy(kv.second.graph);
  }
  for (auto& s : ctx->slots) {
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

// Wait for every launch of the context and report a device error, if any.
extern "C" wf_status wf_check(wf_ctx* ctx) {
  if (!ctx) return fail(WF_EINVAL, "ctx is NULL");
  wf_status st = set_device(ctx);
  if (st != WF_OK) return st;
  wf_status res = ctx->sticky;
  ctx->sticky = WF_OK;
  for (auto& s : ctx->slots) {
    wf_status r = harvest(ctx, s, nullptr, true);
    if (r != WF_OK && res == WF_OK) res = r;
  }
  if (res == WF_ETIMEDOUT) return fail(WF_ETIMEDOUT, "device watchdog fired");
  return res;
}

static wf_status report_sticky(wf_ctx* ctx) {
  // Non-blocking look at finished launches; report a device error once.
  for (auto& s : ctx->slots) {
    wf_status r = harvest(ctx, s, nullptr, false);
    if (r == WF_ETIMEDOUT) ctx->sticky = WF_ETIMEDOUT;
  }
  if (ctx->sticky != WF_OK) {
    wf_status s = ctx->sticky;
    ctx->sticky = WF_OK;
    return fail(s, "a previous launch on this context timed out");
  }
  return WF_OK;
}

extern "C" wf_status wf_solve(wf_ctx* ctx, const wf_problem* p, void* stream_) {
  if (!ctx) return fail(WF_EINVAL, "ctx is NULL");
  wf_status st = check_problem(p, -1);
  if (st != WF_OK) return st;
  st = set_device(ctx);
  if (st != WF_OK) return st;
  st = report_sticky(ctx);
  if (st != WF_OK) return st;
  if (p->m == 0 || p->n == 0) return WF_OK;
  hipStream_t stream = (hipStream_t)stream_;
  const int W = choose_waves(p->m);
  Slot* s = nullptr;
  st = acquire_slot(ctx, stream, &s, nullptr);
  if (st != WF_OK) return st;
  const uint32_t sent = sentinel_of(p->dtype);
  st = ensure_hand(*s, hand_elems(p, W), sent, stream);
  if (st != WF_OK) return st;
  KArgs a;
  std::memset(&a, 0, sizeof a);
  a.g0 = make_desc(p, W, s->hand);
  a.grids = nullptr;
  a.items = nullptr;
  a.nitems = a.g0.nbands;
  a.ctl = s->ctl;
  a.watchdog_ticks = ctx->watchdog_ticks;
  const int resident = ctx->num_cus * wgs_per_cu(W);
  const int nwg = (int)std::min<int64_t>(a.nitems, resident);
  // Optional trace (profiling hook): WF_TRACE_FILE=<path> makes wf_solve synchronous
  // and writes TRACE_WORDS uint64 per (band, compute wave) to <path>.
  const char* trace_file = std::getenv("WF_TRACE_FILE");
  uint64_t* trace = nullptr;
  const size_t trace_words = (size_t)a.nitems * W * TRACE_WORDS;
  // With WF_TRACE_CHUNKS=1 it also writes CTRACE_WORDS uint64 per (band, compute wave, chunk).
  const int64_t nc = ((4 * groups_for(p->n) + 15) / 16 + CTRACE_EVERY - 1) / CTRACE_EVERY;
  const bool chunks = trace_file && *trace_file && std::getenv("WF_TRACE_CHUNKS");
  const size_t ctrace_words = chunks ? (size_t)a.nitems * W * (size_t)nc * CTRACE_WORDS : 0;
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
  WF_HIP(launch_sweep(p->dtype, p->rule, W, nwg, a, stream));
  if (trace) {
    std::vector<uint64_t> host(trace_words), chost(ctrace_words);
    WF_HIP(hipMemcpyAsync(host.data(), trace, trace_words * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    if (ctrace)
      WF_HIP(hipMemcpyAsync(chost.data(), ctrace, ctrace_words * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    WF_HIP(hipStreamSynchronize(stream));
    WF_HIP(hipFree(trace));
    if (ctrace) WF_HIP(hipFree(ctrace));
    if (FILE* f = std::fopen(trace_file, "wb")) {
      const uint64_t hdr[6] = {(uint64_t)a.nitems, (uint64_t)W, (uint64_t)TRACE_WORDS, (uint64_t)nwg,
                               (uint64_t)(ctrace ? nc : 0), (uint64_t)CTRACE_WORDS};
      std::fwrite(hdr, sizeof hdr, 1, f);
      std::fwrite(host.data(), sizeof(uint64_t), host.size(), f);
      if (ctrace) std::fwrite(chost.data(), sizeof(uint64_t), chost.size(), f);
      std::fclose(f);
    }
  }
  return finish_launch(*s, stream);
}

// Batched: one persistent launch over the bands of all grids.
static std::string batch_key(const wf_problem* ps, int64_t count, int W, int nwg, int order) {
  std::string k;
  k.reserve(32 + 24 * (size_t)count);
  char buf[96];
  snprintf(buf, sizeof buf, "%lld/%d/%d/%d/%d/%d|", (long long)count, ps[0].dtype, ps[0].rule, W, nwg, order);
  k += buf;
  for (int64_t i = 0; i < count; ++i) {
    snprintf(buf, sizeof buf, "%lld,%lld,%d;", (long long)ps[i].m, (long long)ps[i].n, ps[i].mode);
    k += buf;
  }
  return k;
}

// One batched launch at a fixed configuration (arguments already checked).
static wf_status batched_run(wf_ctx* ctx, const wf_problem* ps, int64_t count, int W, int order, int max_wgs,
                             bool use_graph, hipStream_t stream) {
  wf_status st = WF_OK;
  // Grids in work order: largest first so the long critical paths start early.
  std::vector<int64_t> perm;
  perm.reserve((size_t)count);
  for (int64_t i = 0; i < count; ++i)
    if (ps[i].m > 0 && ps[i].n > 0) perm.push_back(i);
  if (perm.empty()) return WF_OK;
  std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) {
    return ps[a].m * ps[a].n > ps[b].m * ps[b].n;
  });
  std::vector<GridDesc> descs(perm.size());
  std::vector<Item> items;
  size_t hand_total = 0;
  std::vector<size_t> hand_off(perm.size());
  for (size_t gi = 0; gi < perm.size(); ++gi) {
    hand_off[gi] = hand_total;
    hand_total += hand_elems(&ps[perm[gi]], W);
  }
  int64_t max_bands = 0;
  for (size_t gi = 0; gi < perm.size(); ++gi) {
    descs[gi] = make_desc(&ps[perm[gi]], W, nullptr);
    max_bands = std::max<int64_t>(max_bands, descs[gi].nbands);
  }
  if (order == 2) {
    // Interleaved: band b of every grid before band b+1 of any grid.
    for (int64_t b = 0; b < max_bands; ++b)
      for (size_t gi = 0; gi < perm.size(); ++gi)
        if (b < descs[gi].nbands) items.push_back(Item{(uint32_t)gi, (uint32_t)b});
  } else {
    for (size_t gi = 0; gi < perm.size(); ++gi)
      for (int b = 0; b < descs[gi].nbands; ++b) items.push_back(Item{(uint32_t)gi, (uint32_t)b});
  }
  const int resident = ctx->num_cus * wgs_per_cu(W);
  int nwg = (int)std::min<int64_t>((int64_t)items.size(), resident);
  if (max_wgs > 0) nwg = std::min(nwg, max_wgs);

  const std::string key = use_graph ? batch_key(ps, count, W, nwg, order) : std::string();
  Slot* s = nullptr;
  int slot_index = -1;
  GraphEntry* ge = nullptr;
  if (use_graph) {
    auto it = ctx->graphs.find(key);
    if (it != ctx->graphs.end()) {
      ge = &it->second;
      slot_index = ge->slot;
      s = &ctx->slots[slot_index];
      st = harvest(ctx, *s, stream, true);
      if (st == WF_ETIMEDOUT) ctx->sticky = WF_ETIMEDOUT;
      else if (st != WF_OK) return st;
    }
  }
  if (!s) {
    st = acquire_slot(ctx, stream, &s, &slot_index);
    if (st != WF_OK) return st;
    // A slot that backs a cached graph is handed to this batch; drop that graph.
    for (auto it = ctx->graphs.begin(); it != ctx->graphs.end();) {
      if (it->second.slot == slot_index) {
        hipGraphExecDestroy(it->second.exec);
        hipGraphDestroy(it->second.graph);
        it = ctx->graphs.erase(it);
      } else {
        ++it;
      }
    }
  }
  const uint32_t sent = sentinel_of(ps[0].dtype);
  // Also on replay: a single-grid solve may have used this slot since, growing its
  // handoff rows or arming them with another dtype's sentinel.
  st = ensure_hand(*s, hand_total, sent, stream);
  if (st != WF_OK) return st;
  if (!ge) {
    st = ensure_buf(&s->grids, &s->grids_cap, descs.size());
    if (st != WF_OK) return st;
    st = ensure_buf(&s->items, &s->items_cap, items.size());
    if (st != WF_OK) return st;
  }
  for (size_t gi = 0; gi < descs.size(); ++gi) descs[gi].hand = s->hand + hand_off[gi];
  // The tables are copied on the stream (pointers may differ between calls with the same
  // shape); a replayed graph whose table is unchanged skips the copy.
  const bool same_table = ge && ge->descs.size() == descs.size() &&
                          std::memcmp(ge->descs.data(), descs.data(), descs.size() * sizeof(GridDesc)) == 0;
  if (!same_table) {
    WF_HIP(hipMemcpyAsync(s->grids, descs.data(), descs.size() * sizeof(GridDesc), hipMemcpyHostToDevice, stream));
    if (!ge) WF_HIP(hipMemcpyAsync(s->items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice, stream));
    // The host arrays must outlive the asynchronous copies.
    WF_HIP(hipStreamSynchronize(stream));
  }

  KArgs a;
  std::memset(&a, 0, sizeof a);
  a.grids = s->grids;
  a.items = s->items;
  a.nitems = (int64_t)items.size();
  a.ctl = s->ctl;
  a.watchdog_ticks = ctx->watchdog_ticks;

  if (use_graph) {
    if (!ge) {
      hipStream_t cap = nullptr;
      WF_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      GraphEntry e;
      e.slot = slot_index;
      hipError_t err = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (err == hipSuccess) {
        launch_fill_u32(s->ctl, 0u, CTL_WORDS, cap);
        launch_sweep(ps[0].dtype, ps[0].rule, W, nwg, a, cap);
        err = hipStreamEndCapture(cap, &e.graph);
      }
      if (err == hipSuccess) err = hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0);
      hipStreamDestroy(cap);
      if (err != hipSuccess) return fail(WF_EHIP, std::string("graph capture: ") + hipGetErrorString(err));
      ge = &(ctx->graphs[key] = e);
    }
    if (!same_table) ge->descs = descs;
    WF_HIP(hipGraphLaunch(ge->exec, stream));
  } else {
    WF_HIP(launch_fill_u32(s->ctl, 0u, CTL_WORDS, stream));
    WF_HIP(launch_sweep(ps[0].dtype, ps[0].rule, W, nwg, a, stream));
  }
  return finish_launch(*s, stream);
}

// Autotuning: the first batch of a given shape signature (and no explicit
// waves_per_wg / order) is run twice at every candidate configuration, the
// second run timed with events on the caller's stream, and the fastest is kept
// for that signature.  Every trial computes the full, correct result.
static std::string shape_signature(const wf_problem* ps, int64_t count) {
  return batch_key(ps, count, 0, 0, 0);
}

static wf_status autotune(wf_ctx* ctx, const wf_problem* ps, int64_t count, int max_wgs, hipStream_t stream,
                          int* W_out, int* order_out) {
  const std::string sig = shape_signature(ps, count);
  auto it = ctx->tuned.find(sig);
  if (it != ctx->tuned.end()) {
    *W_out = it->second.first;
    *order_out = it->second.second;
    return WF_OK;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  WF_HIP(hipEventCreate(&e0));
  WF_HIP(hipEventCreate(&e1));
  float best = -1.f;
  int bw = 1, bo = 1;
  static const int Ws[] = {1, 2};
  wf_status st = WF_OK;
  for (int W : Ws) {
    for (int order = 1; order <= 2 && st == WF_OK; ++order) {
      // Two runs back to back, timing the second: its host-side set-up overlaps the
      // first run on the device, so the events bracket device time only.
      st = batched_run(ctx, ps, count, W, order, max_wgs, false, stream);
      if (st != WF_OK) break;
      hipError_t e = hipEventRecord(e0, stream);
      if (e == hipSuccess) st = batched_run(ctx, ps, count, W, order, max_wgs, false, stream);
      if (st == WF_OK && e == hipSuccess) e = hipEventRecord(e1, stream);
      if (st == WF_OK && e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (st == WF_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (st == WF_OK && e != hipSuccess) st = fail(WF_EHIP, std::string("autotune: ") + hipGetErrorString(e));
      if (st != WF_OK) break;
      st = report_sticky(ctx);
      if (st != WF_OK) break;
      if (best < 0.f || ms < best) {
        best = ms;
        bw = W;
        bo = order;
      }
    }
    if (st != WF_OK) break;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != WF_OK) return st;
  ctx->tuned[sig] = std::make_pair(bw, bo);
  *W_out = bw;
  *order_out = bo;
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
  for (int i = 0; i < 4; ++i)
    if (tun.reserved[i] != 0) return fail(WF_EINVAL, "wf_tuning.reserved must be 0");
  if (tun.waves_per_wg < 0 || tun.waves_per_wg > 2) return fail(WF_EINVAL, "waves_per_wg must be 0, 1 or 2");
  if (tun.max_wgs < 0 || tun.order < 0 || tun.order > 2 || tun.use_graph < -1 || tun.use_graph > 1)
    return fail(WF_EINVAL, "bad tuning value");
  wf_status st = set_device(ctx);
  if (st != WF_OK) return st;
  st = report_sticky(ctx);
  if (st != WF_OK) return st;
  hipStream_t stream = (hipStream_t)stream_;
  bool any = false;
  for (int64_t i = 0; i < count && !any; ++i) any = ps[i].m > 0 && ps[i].n > 0;
  if (!any) return WF_OK;
  int W = tun.waves_per_wg, order = tun.order;
  if (W == 0 && order == 0 && tun.use_graph != -1) {
    st = autotune(ctx, ps, count, tun.max_wgs, stream, &W, &order);
    if (st != WF_OK) return st;
  }
  if (W == 0) {
    int64_t max_m = 0;
    for (int64_t i = 0; i < count; ++i) max_m = std::max(max_m, ps[i].m);
    W = choose_waves(max_m / 2 > 0 ? max_m / 2 : 1);
  }
  if (order == 0) order = 1;
  return batched_run(ctx, ps, count, W, order, tun.max_wgs, tun.use_graph == 1, stream);
}
