// wf_server.cpp -- serving front end: requests are admitted against a device
// memory budget as they arrive, batched into persistent sweep launches on
// several streams while earlier launches are still running (continuous
// batching), and completed asynchronously.
//
// One server thread owns every HIP call of the server.  Per pass it
//   1. retires launches whose completion event has fired (results stay in
//      server memory until wf_release) and frees the staging of host copies
//      that have landed,
//   2. admits queued requests while their memory fits the budget: in arrival
//      order, but a request that does not fit yet lets smaller ones behind it
//      in until it has waited `max_wait_skip_us` (then admission waits for it);
//      a host input is copied to the device on a copy stream at admission,
//   3. packs admitted requests that share dtype and rule into one launch on a
//      free stream: the launch stream waits for its requests' copies (or for
//      the caller's ready events of device inputs), seeded inputs are
//      generated on the device, handoff rows are armed, the descriptor table
//      and work list are uploaded from pinned staging, and the persistent
//      kernel runs their bands in ticket order.
// Launches on different streams overlap on the device: a launch's workgroups
// retire as its ticket list runs out, and the next launch's workgroups take
// their place.  Each launch has its own ticket counter, and a band only waits
// on a band of the same launch with a smaller ticket, so concurrent launches
// cannot deadlock one another.
//
// Copies of host inputs on their own streams overlap the sweeps of earlier
// launches: the copy/compute overlap that arXiv 2501.05938 builds its streamed
// time model on (Section 1; Section 2.2, Eq. 2).  Requests are then a two-stage
// flow shop (copy, then sweep), whose makespan is the max-plus recurrence of the
// sweep's max rule over a (requests x 2 stages) grid.
#include "../../include/wf.h"
#include "wf_host.h"
#include "wf_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace wfk;
using namespace wfh;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr size_t ALIGN = 256;
size_t round_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// First-fit allocator over one block of memory, with coalescing on release.
class Arena {
 public:
  void reset(char* base, size_t bytes) {
    base_ = base;
    size_ = bytes / ALIGN * ALIGN;
    free_.clear();
    if (size_) free_[0] = size_;
    in_use_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      in_use_ += bytes;
      peak_ = std::max(peak_, in_use_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
    in_use_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  char* base() const { return base_; }
  size_t size() const { return size_; }
  size_t in_use() const { return in_use_; }
  size_t peak() const { return peak_; }

 private:
  char* base_ = nullptr;
  size_t size_ = 0, in_use_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
};

enum ReqState { QUEUED, ADMITTED, LAUNCHED, DONE, FAILED };

struct Req {
  wf_request r;
  ReqState state = QUEUED;
  wf_status err = WF_OK;
  std::string msg;
  double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
  // Server memory: one arena block holding, in order, the input copy (host and
  // seeded inputs), the full output (FULL mode), last row, last column, final
  // cell and the handoff rows.
  size_t off = 0, bytes = 0;
  bool has_block = false;
  const void* in = nullptr;
  int64_t ld_in = 0;
  void* out = nullptr;
  void* last_row = nullptr;
  void* last_col = nullptr;
  void* final_cell = nullptr;
  uint32_t* hand = nullptr;
  size_t hand_n = 0;
  hipEvent_t copied = nullptr;  // recorded on a copy stream after the input landed (host inputs)
};

bool host_input(const wf_request& r) { return r.input_kind == WF_INPUT_HOST || r.input_kind == WF_INPUT_HOST_PINNED; }
bool owns_input(const wf_request& r) { return host_input(r) || r.input_kind == WF_INPUT_SEED; }

// Byte layout of a request's block.
struct Layout {
  size_t in = 0, out = 0, last_row = 0, last_col = 0, final_cell = 0, hand = 0, total = 0;
  size_t hand_n = 0;
};

Layout layout_of(const wf_request& r) {
  Layout L;
  size_t at = 0;
  const size_t m = (size_t)r.m, n = (size_t)r.n;
  if (owns_input(r)) {
    L.in = at;
    at += round_up(m * n * 4);
  }
  if (r.mode == WF_MODE_FULL) {
    L.out = at;
    at += round_up(m * n * 4);
  }
  L.last_row = at;
  at += round_up(n * 4);
  L.last_col = at;
  at += round_up(m * 4);
  L.final_cell = at;
  at += ALIGN;
  // Handoff rows for the finest banding (64 rows per band), so any band shape fits: at
  // 128-row bands there are at most half as many boundaries, each 64 positions longer
  // (and a handoff row is at least 64 positions).
  const int64_t nb = (r.m + 63) / 64;
  L.hand_n = nb > 1 ? (size_t)(nb - 1) * (size_t)hand_ld_for(r.n, 1) : 0;
  L.hand = at;
  at += round_up(std::max<size_t>(L.hand_n, 1) * 4);
  L.total = at;
  return L;
}

// Everything one in-flight launch owns.
struct LaunchSlot {
  hipStream_t stream = nullptr;
  uint32_t* ctl = nullptr;
  GridDesc* d_grids = nullptr;
  Item* d_items = nullptr;
  size_t grids_cap = 0, items_cap = 0;
  GridDesc* h_grids = nullptr;  // pinned staging, valid until `done` fires
  Item* h_items = nullptr;
  size_t h_grids_cap = 0, h_items_cap = 0;
  unsigned char* h_stage = nullptr;  // pinned staging of host inputs without copy streams
  size_t h_stage_cap = 0;
  uint32_t* host_err = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<uint64_t> tickets;
};

// A host input in flight on a copy stream: its staging is freed once `ev` has fired.
struct Copy {
  hipEvent_t ev;
  size_t stage_off, stage_bytes;
  bool staged;
  uint64_t ticket;
  int stream;  // index into copy_streams
};

template <class T>
wf_status grow_dev(T** p, size_t* cap, size_t need) {
  if (*cap >= need) return WF_OK;
  const size_t c = std::max<size_t>(std::max<size_t>(need, 256), 2 * *cap);
  if (*p) hipFree(*p);
  *p = nullptr;
  *cap = 0;
  if (hipMalloc(p, c * sizeof(T)) != hipSuccess) return fail(WF_ENOMEM, "cannot allocate a launch table");
  *cap = c;
  return WF_OK;
}

template <class T>
wf_status grow_host(T** p, size_t* cap, size_t need) {
  if (*cap >= need) return WF_OK;
  const size_t c = std::max<size_t>(std::max<size_t>(need, 256), 2 * *cap);
  if (*p) hipHostFree(*p);
  *p = nullptr;
  *cap = 0;
  if (hipHostMalloc((void**)p, c * sizeof(T), hipHostMallocDefault) != hipSuccess)
    return fail(WF_ENOMEM, "cannot allocate pinned staging");
  *cap = c;
  return WF_OK;
}

}  // namespace

// Seeded input generation for WF_INPUT_SEED requests (wf_seed.hip).
namespace wfk {
hipError_t launch_seed_fill(void* dst, int dtype, int64_t m, int64_t n, uint64_t seed, hipStream_t stream);
}

struct wf_server {
  wf_ctx* ctx = nullptr;
  wf_server_opts opts{};
  void* dev_base = nullptr;
  Arena arena;                    // device budget
  void* pin_base = nullptr;
  Arena staging;                  // pinned staging of pageable host inputs (copy streams only)
  std::vector<LaunchSlot> slots;
  std::vector<hipStream_t> copy_streams;
  size_t next_copy = 0;
  std::vector<hipEvent_t> event_pool;
  std::vector<Copy> copying;
  std::mutex mu;
  std::condition_variable cv;
  std::thread thread;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, Req> reqs;
  std::deque<uint64_t> queue;     // submitted, not admitted (arrival order)
  std::deque<uint64_t> admitted;  // admitted, not launched
  std::deque<uint64_t> finished;  // done or failed, not yet reported by wf_server_done
  int inflight = 0;
  uint64_t epoch = 0;             // bumped by every submit, release and stop
  std::string thread_error;       // a HIP failure inside the server thread

  void run();
  void retire(LaunchSlot& L, double t, hipError_t q);
  void reap_copies();
  void admit(double t);
  bool try_admit(Req& q, uint64_t ticket, double t);
  bool launch_one(std::unique_lock<std::mutex>& lk);
  wf_status enqueue(LaunchSlot& L, std::vector<Req*>& batch, int bs, int dtype, int rule);
  wf_status start_copy(Req& q, Copy* c);
};

void wf_server::retire(LaunchSlot& L, double t, hipError_t q) {
  const bool timed_out = q == hipSuccess && *L.host_err != DEV_OK;
  *L.host_err = DEV_OK;
  for (uint64_t tk : L.tickets) {
    auto it = reqs.find(tk);
    if (it == reqs.end()) continue;
    Req& r = it->second;
    r.t_done = t;
    if (q != hipSuccess) {
      r.state = FAILED;
      r.err = WF_EHIP;
      r.msg = std::string("the request's launch failed: ") + hipGetErrorString(q);
    } else if (timed_out) {
      r.state = FAILED;
      r.err = WF_ETIMEDOUT;
      r.msg = "device watchdog fired in the request's launch";
    } else {
      r.state = DONE;
    }
    finished.push_back(tk);
  }
  L.tickets.clear();
  L.busy = false;
  --inflight;
}

void wf_server::reap_copies() {
  // `copying` is in issue order and the copies of one stream complete in order, so only
  // each stream's oldest pending copy is queried (hundreds may be pending at once).
  uint32_t busy = 0;  // bit s: copy stream s has a copy still in flight
  size_t w = 0;
  for (size_t i = 0; i < copying.size(); ++i) {
    const Copy c = copying[i];
    const uint32_t bit = 1u << c.stream;
    if ((busy & bit) || hipEventQuery(c.ev) == hipErrorNotReady) {
      busy |= bit;
      copying[w++] = c;
      continue;
    }
    if (c.staged) staging.release(c.stage_off, c.stage_bytes);
    // The copy has landed: a launch not enqueued yet need not wait for it (the event
    // goes back to the pool and may be recorded again for another copy).
    auto it = reqs.find(c.ticket);
    if (it != reqs.end() && it->second.copied == c.ev) it->second.copied = nullptr;
    event_pool.push_back(c.ev);
  }
  copying.resize(w);
}

// Copy a host input to its device block on the next copy stream (pageable inputs go
// through pinned staging first; pinned ones are copied directly).
wf_status wf_server::start_copy(Req& q, Copy* c) {
  const size_t row = (size_t)q.r.n * 4, bytes = row * (size_t)q.r.m;
  const size_t si = next_copy++ % copy_streams.size();
  hipStream_t cs = copy_streams[si];
  c->stream = (int)si;
  c->staged = false;
  const char* src = (const char*)q.r.input;
  const bool dense = q.r.ld_input == q.r.n;
  if (q.r.input_kind == WF_INPUT_HOST_PINNED) {
    if (dense) {
      WF_HIP(hipMemcpyAsync((void*)q.in, src, bytes, hipMemcpyHostToDevice, cs));
    } else {
      WF_HIP(hipMemcpy2DAsync((void*)q.in, row, src, (size_t)q.r.ld_input * 4, row, (size_t)q.r.m,
                              hipMemcpyHostToDevice, cs));
    }
  } else {
    char* st = staging.base() + c->stage_off;
    for (int64_t i = 0; i < q.r.m; ++i) std::memcpy(st + (size_t)i * row, src + (size_t)i * (size_t)q.r.ld_input * 4, row);
    WF_HIP(hipMemcpyAsync((void*)q.in, st, bytes, hipMemcpyHostToDevice, cs));
    c->staged = true;
  }
  WF_HIP(hipEventRecord(c->ev, cs));
  q.copied = c->ev;
  return WF_OK;
}

bool wf_server::try_admit(Req& q, uint64_t ticket, double t) {
  const bool copy_now = host_input(q.r) && !copy_streams.empty();
  const size_t stage_bytes = (size_t)q.r.m * (size_t)q.r.n * 4;
  Copy c{nullptr, 0, 0, false, ticket};
  if (copy_now && q.r.input_kind == WF_INPUT_HOST && !staging.alloc(stage_bytes, &c.stage_off)) return false;
  size_t off = 0;
  if (!arena.alloc(q.bytes, &off)) {
    if (copy_now && q.r.input_kind == WF_INPUT_HOST) staging.release(c.stage_off, stage_bytes);
    return false;
  }
  const Layout Lo = layout_of(q.r);
  char* b = arena.base() + off;
  q.off = off;
  q.has_block = true;
  if (owns_input(q.r)) {
    q.in = b + Lo.in;
    q.ld_in = q.r.n;
  } else {
    q.in = q.r.input;
    q.ld_in = q.r.ld_input;
  }
  q.out = q.r.mode == WF_MODE_FULL ? (void*)(b + Lo.out) : nullptr;
  q.last_row = b + Lo.last_row;
  q.last_col = b + Lo.last_col;
  q.final_cell = b + Lo.final_cell;
  q.hand = (uint32_t*)(b + Lo.hand);
  q.hand_n = Lo.hand_n;
  q.state = ADMITTED;
  q.t_admit = t;
  if (copy_now) {
    c.stage_bytes = stage_bytes;
    if (event_pool.empty()) {
      hipEvent_t e = nullptr;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess) event_pool.push_back(e);
    }
    wf_status st = WF_EHIP;
    if (!event_pool.empty()) {
      c.ev = event_pool.back();
      event_pool.pop_back();
      st = start_copy(q, &c);
    }
    if (st != WF_OK) {
      q.state = FAILED;
      q.err = st == WF_EHIP && event_pool.empty() && !c.ev ? WF_ENOMEM : st;
      q.msg = wf_last_error();
      q.t_done = t;
      finished.push_back(ticket);
      if (c.ev) event_pool.push_back(c.ev);
      if (q.r.input_kind == WF_INPUT_HOST) staging.release(c.stage_off, stage_bytes);
      return true;
    }
    copying.push_back(c);
  }
  admitted.push_back(ticket);
  return true;
}

void wf_server::admit(double t) {
  // Arrival order; a request that does not fit yet lets requests behind it in until it
  // has waited max_wait_skip_us, after which nothing overtakes it.
  int skipped = 0;
  for (auto it = queue.begin(); it != queue.end();) {
    Req& q = reqs[*it];
    if (try_admit(q, *it, t)) {
      it = queue.erase(it);
      continue;
    }
    if (t - q.t_submit > opts.max_wait_skip_us * 1e-6 || ++skipped > 64) break;
    ++it;
  }
}

wf_status wf_server::enqueue(LaunchSlot& L, std::vector<Req*>& batch, int bs, int dtype, int rule) {
  hipStream_t s = L.stream;
  // Pageable host inputs without copy streams go through the slot's pinned staging buffer on the
  // launch stream: a copy from pageable memory is staged synchronously by the runtime in
  // the calling thread, which would make the server thread block on the device.
  size_t stage = 0;
  for (Req* q : batch)
    if (q->r.input_kind == WF_INPUT_HOST && !q->copied) stage += (size_t)q->r.m * (size_t)q->r.n * 4;
  if (stage) {
    wf_status st = grow_host(&L.h_stage, &L.h_stage_cap, stage);
    if (st != WF_OK) return st;
  }
  const uint32_t sent = sentinel_of(dtype);
  size_t at = 0;
  for (Req* q : batch) {
    if (q->copied) {
      WF_HIP(hipStreamWaitEvent(s, q->copied, 0));
    } else if (q->r.input_kind == WF_INPUT_HOST_PINNED) {
      // Pinned memory is copied by DMA directly, on the launch stream.
      const size_t row = (size_t)q->r.n * 4;
      if (q->r.ld_input == q->r.n)
        WF_HIP(hipMemcpyAsync((void*)q->in, q->r.input, row * (size_t)q->r.m, hipMemcpyHostToDevice, s));
      else
        WF_HIP(hipMemcpy2DAsync((void*)q->in, row, q->r.input, (size_t)q->r.ld_input * 4, row, (size_t)q->r.m,
                                hipMemcpyHostToDevice, s));
    } else if (host_input(q->r)) {
      const size_t row = (size_t)q->r.n * 4, bytes = row * (size_t)q->r.m;
      for (int64_t i = 0; i < q->r.m; ++i)
        std::memcpy(L.h_stage + at + (size_t)i * row, (const char*)q->r.input + (size_t)i * (size_t)q->r.ld_input * 4, row);
      WF_HIP(hipMemcpyAsync((void*)q->in, L.h_stage + at, bytes, hipMemcpyHostToDevice, s));
      at += bytes;
    } else if (q->r.input_kind == WF_INPUT_SEED) {
      WF_HIP(launch_seed_fill((void*)q->in, q->r.dtype, q->r.m, q->r.n, q->r.seed, s));
    } else if (q->r.ready_event) {
      WF_HIP(hipStreamWaitEvent(s, (hipEvent_t)q->r.ready_event, 0));
    }
  }
  // Descriptors, largest grid first, and the grid-major work list.
  std::sort(batch.begin(), batch.end(), [](const Req* a, const Req* b) { return a->r.m * a->r.n > b->r.m * b->r.n; });
  size_t nitems = 0;
  for (Req* q : batch) nitems += (size_t)((q->r.m + shape_rows(bs) - 1) / shape_rows(bs));
  wf_status st = grow_host(&L.h_grids, &L.h_grids_cap, batch.size());
  if (st == WF_OK) st = grow_host(&L.h_items, &L.h_items_cap, nitems);
  if (st == WF_OK) st = grow_dev(&L.d_grids, &L.grids_cap, batch.size());
  if (st == WF_OK) st = grow_dev(&L.d_items, &L.items_cap, nitems);
  if (st != WF_OK) return st;
  size_t k = 0;
  for (size_t gi = 0; gi < batch.size(); ++gi) {
    const Req* q = batch[gi];
    wf_problem p;
    std::memset(&p, 0, sizeof p);
    p.m = q->r.m;
    p.n = q->r.n;
    p.dtype = q->r.dtype;
    p.rule = q->r.rule;
    p.mode = q->r.mode;
    p.cost = q->in;
    p.ld_cost = q->ld_in;
    p.out = q->out;
    p.ld_out = q->r.n;
    p.last_row = q->last_row;
    p.last_col = q->last_col;
    p.final_cell = q->final_cell;
    GridDesc d = make_desc(&p, bs, q->hand);
    L.h_grids[gi] = d;
    for (int b = 0; b < d.nbands; ++b) L.h_items[k++] = Item{(uint32_t)gi, (uint32_t)b};
  }
  WF_HIP(hipMemcpyAsync(L.d_grids, L.h_grids, batch.size() * sizeof(GridDesc), hipMemcpyHostToDevice, s));
  WF_HIP(hipMemcpyAsync(L.d_items, L.h_items, nitems * sizeof(Item), hipMemcpyHostToDevice, s));
  // Every request's handoff rows (arena memory, so of unknown contents) armed in one launch.
  WF_HIP(launch_arm_hand(L.d_grids, (int)batch.size(), sent, s));
  KArgs a = base_args(ctx, L.ctl, (int64_t)nitems);
  a.grids = L.d_grids;
  a.items = L.d_items;
  const int nwg = (int)std::min<int64_t>((int64_t)nitems, (int64_t)ctx->num_cus * wgs_per_cu(bs, dtype));
  WF_HIP(launch_fill_u32(L.ctl, 0u, CTL_WORDS, s));
  WF_HIP(launch_shape(dtype, rule, bs, nwg, a, s));
  WF_HIP(hipMemcpyAsync(L.host_err, L.ctl + CTL_ERROR, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  WF_HIP(hipEventRecord(L.done, s));
  return WF_OK;
}

// Launch the admitted requests that share the oldest one's dtype and rule, if a
// stream is free.  Called with the lock held; drops it around the HIP calls.
bool wf_server::launch_one(std::unique_lock<std::mutex>& lk) {
  if (admitted.empty()) return false;
  LaunchSlot* L = nullptr;
  for (auto& s : slots)
    if (!s.busy) {
      L = &s;
      break;
    }
  if (!L) return false;
  const Req& first = reqs[admitted.front()];
  const int dtype = first.r.dtype, rule = first.r.rule;
  std::vector<Req*> batch;
  std::vector<uint64_t> tickets;
  int64_t max_m = 1;
  for (auto it = admitted.begin(); it != admitted.end() && (int)batch.size() < opts.max_batch;) {
    Req& q = reqs[*it];
    if (q.r.dtype == dtype && q.r.rule == rule) {
      batch.push_back(&q);
      tickets.push_back(*it);
      max_m = std::max(max_m, q.r.m);
      q.state = LAUNCHED;
      it = admitted.erase(it);
    } else {
      ++it;
    }
  }
  L->busy = true;
  L->tickets = tickets;
  ++inflight;
  const int bs = choose_shape(max_m);
  const double t = now_s();
  for (Req* q : batch) q->t_launch = t;
  // Requests in `batch` are LAUNCHED: wf_release refuses them, so the pointers stay valid.
  lk.unlock();
  wf_status st = enqueue(*L, batch, bs, dtype, rule);
  const std::string msg = st == WF_OK ? std::string() : std::string(wf_last_error());
  lk.lock();
  if (st != WF_OK) {
    for (uint64_t tk : tickets) {
      Req& q = reqs[tk];
      q.state = FAILED;
      q.err = st;
      q.msg = msg;
      q.t_done = now_s();
      finished.push_back(tk);
    }
    // Nothing may still run on the stream before the slot is reused.
    hipStreamSynchronize(L->stream);
    L->tickets.clear();
    L->busy = false;
    --inflight;
    thread_error = msg;
  }
  return true;
}

void wf_server::run() {
  hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    const double t = now_s();
    for (auto& L : slots) {
      if (!L.busy) continue;
      // Any result but "not ready" ends the launch: success, or a failed launch whose
      // requests are then reported as failed.
      const hipError_t q = hipEventQuery(L.done);
      if (q != hipErrorNotReady) retire(L, t, q);
    }
    reap_copies();
    if (!stop) admit(t);
    bool launched = false;
    while (!stop && launch_one(lk)) launched = true;
    if (stop && inflight == 0) break;
    if (launched) continue;
    const uint64_t seen = epoch;
    if (inflight > 0 || !copying.empty()) {
      // Work in flight: look at its events again shortly, or at once on a submit.
      cv.wait_for(lk, std::chrono::microseconds(20), [&] { return stop || epoch != seen; });
    } else {
      // Idle (or waiting for memory held by finished requests): sleep until something changes.
      cv.wait(lk, [&] { return stop || epoch != seen; });
    }
  }
}

// ------------------------------------------------------------------ public
extern "C" wf_status wf_server_create(wf_ctx* ctx, const wf_server_opts* opts, wf_server** out) {
  if (!ctx || !out) return fail(WF_EINVAL, "ctx and out must not be NULL");
  *out = nullptr;
  wf_server_opts o;
  std::memset(&o, 0, sizeof o);
  if (opts) o = *opts;
  for (int i = 0; i < 2; ++i)
    if (o.reserved[i] != 0) return fail(WF_EINVAL, "wf_server_opts.reserved must be 0");
  if (o.hbm_budget_bytes < 0 || o.max_inflight < 0 || o.max_batch < 0 || o.copy_streams < 0 ||
      o.staging_bytes < 0 || o.max_wait_skip_us < 0)
    return fail(WF_EINVAL, "negative option");
  if (o.hbm_budget_bytes == 0) o.hbm_budget_bytes = (int64_t)64 << 30;
  if (o.max_inflight == 0) o.max_inflight = 2;
  if (o.max_batch == 0) o.max_batch = 256;
  if (o.staging_bytes == 0) o.staging_bytes = (int64_t)256 << 20;
  if (o.max_wait_skip_us == 0) o.max_wait_skip_us = 20000;
  if (o.max_inflight > 32 || o.copy_streams > 8) return fail(WF_EINVAL, "max_inflight above 32 or copy_streams above 8");
  wf_status st = set_device(ctx);
  if (st != WF_OK) return st;
  std::unique_ptr<wf_server> s(new wf_server);
  s->ctx = ctx;
  s->opts = o;
  if (hipMalloc(&s->dev_base, (size_t)o.hbm_budget_bytes) != hipSuccess) {
    s->dev_base = nullptr;
    return fail(WF_ENOMEM, "cannot allocate the server's device memory budget");
  }
  s->arena.reset((char*)s->dev_base, (size_t)o.hbm_budget_bytes);
  auto cleanup = [&]() {
    for (auto& L : s->slots) {
      if (L.stream) hipStreamDestroy(L.stream);
      if (L.ctl) hipFree(L.ctl);
      if (L.host_err) hipHostFree(L.host_err);
      if (L.done) hipEventDestroy(L.done);
    }
    for (hipStream_t c : s->copy_streams) hipStreamDestroy(c);
    if (s->pin_base) hipHostFree(s->pin_base);
    hipFree(s->dev_base);
  };
  if (o.copy_streams > 0) {
    if (hipHostMalloc(&s->pin_base, (size_t)o.staging_bytes, hipHostMallocDefault) != hipSuccess) {
      s->pin_base = nullptr;
      cleanup();
      return fail(WF_ENOMEM, "cannot allocate the server's pinned staging");
    }
    s->staging.reset((char*)s->pin_base, (size_t)o.staging_bytes);
    for (int i = 0; i < o.copy_streams; ++i) {
      hipStream_t c = nullptr;
      if (hipStreamCreateWithFlags(&c, hipStreamNonBlocking) != hipSuccess) {
        cleanup();
        return fail(WF_EHIP, "cannot create a copy stream");
      }
      s->copy_streams.push_back(c);
    }
  }
  s->slots.resize((size_t)o.max_inflight);
  for (auto& L : s->slots) {
    if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(&L.ctl, CTL_WORDS * sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc((void**)&L.host_err, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) {
      cleanup();
      return fail(WF_EHIP, "cannot create the server's launch streams");
    }
    *L.host_err = DEV_OK;
  }
  wf_server* raw = s.get();
  s->thread = std::thread([raw] { raw->run(); });
  *out = s.release();
  return WF_OK;
}

extern "C" wf_status wf_submit(wf_server* s, const wf_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return fail(WF_EINVAL, "server, request and ticket must not be NULL");
  if (r->m < 0 || r->n < 0) return fail(WF_EINVAL, "m and n must be >= 0");
  if (r->dtype == WF_F64) return fail(WF_EUNSUPPORTED, "the server serves fp32 and int32 grids");
  if (r->dtype != WF_F32 && r->dtype != WF_I32) return fail(WF_EINVAL, "unknown dtype");
  if (r->rule != WF_RULE_MIN && r->rule != WF_RULE_MAX) return fail(WF_EINVAL, "unknown rule");
  if (r->mode != WF_MODE_FULL && r->mode != WF_MODE_EDGES) return fail(WF_EINVAL, "unknown mode");
  if (r->input_kind != WF_INPUT_DEVICE && r->input_kind != WF_INPUT_HOST && r->input_kind != WF_INPUT_SEED &&
      r->input_kind != WF_INPUT_HOST_PINNED)
    return fail(WF_EINVAL, "unknown input kind");
  const bool empty = r->m == 0 || r->n == 0;
  if (!empty && r->input_kind != WF_INPUT_SEED && (!r->input || r->ld_input < r->n))
    return fail(WF_EINVAL, "input is NULL or ld_input < n");
  if (r->n > ((int64_t)1 << 23) || (r->input_kind == WF_INPUT_DEVICE && r->ld_input > ((int64_t)1 << 23)))
    return fail(WF_EUNSUPPORTED, "n or ld_input above 2^23 is not supported");
  Req q;
  q.r = *r;
  q.t_submit = now_s();
  if (!empty) {
    q.bytes = layout_of(*r).total;
    if (q.bytes > s->arena.size()) return fail(WF_E2BIG, "the request can never fit the server's memory budget");
    if (r->input_kind == WF_INPUT_HOST && !s->copy_streams.empty() &&
        (size_t)r->m * (size_t)r->n * 4 > s->staging.size())
      return fail(WF_E2BIG, "the host input can never fit the server's pinned staging");
  }
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stop) return fail(WF_ESHUTDOWN, "server is shutting down");
  const uint64_t t = s->next_ticket++;
  if (empty) {
    q.state = DONE;
    q.t_admit = q.t_launch = q.t_done = q.t_submit;
    s->reqs.emplace(t, std::move(q));
  } else {
    s->reqs.emplace(t, std::move(q));
    s->queue.push_back(t);
    ++s->epoch;
    s->cv.notify_one();
  }
  *ticket = t;
  return WF_OK;
}

extern "C" wf_status wf_poll(wf_server* s, uint64_t ticket, wf_result* out) {
  if (!s || !out) return fail(WF_EINVAL, "server and out must not be NULL");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(WF_ENOTFOUND, "unknown or released ticket");
  const Req& q = it->second;
  if (q.state == FAILED) return fail(q.err, q.msg);
  if (q.state != DONE) return WF_PENDING;
  std::memset(out, 0, sizeof *out);
  out->out = q.out;
  out->ld_out = q.out ? q.r.n : 0;
  out->last_row = q.last_row;
  out->last_col = q.last_col;
  out->final_cell = q.final_cell;
  out->t_submit = q.t_submit;
  out->t_admit = q.t_admit;
  out->t_launch = q.t_launch;
  out->t_done = q.t_done;
  return WF_OK;
}

extern "C" wf_status wf_release(wf_server* s, uint64_t ticket) {
  if (!s) return fail(WF_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(WF_ENOTFOUND, "unknown or released ticket");
  Req& q = it->second;
  if (q.state == ADMITTED || q.state == LAUNCHED) return fail(WF_PENDING, "the request is still running");
  if (q.state == QUEUED) s->queue.erase(std::find(s->queue.begin(), s->queue.end(), ticket));
  if (q.has_block) s->arena.release(q.off, q.bytes);
  s->reqs.erase(it);
  ++s->epoch;
  s->cv.notify_one();  // memory freed: admission may proceed
  return WF_OK;
}

extern "C" wf_status wf_server_done(wf_server* s, uint64_t* tickets, int64_t cap, int64_t* count) {
  if (!s || !count) return fail(WF_EINVAL, "server and count must not be NULL");
  if (cap < 0 || (cap > 0 && !tickets)) return fail(WF_EINVAL, "tickets is NULL or cap < 0");
  std::lock_guard<std::mutex> g(s->mu);
  int64_t k = 0;
  while (k < cap && !s->finished.empty()) {
    const uint64_t tk = s->finished.front();
    s->finished.pop_front();
    if (s->reqs.count(tk)) tickets[k++] = tk;  // (released already through wf_poll: skipped)
  }
  *count = k;
  return WF_OK;
}

extern "C" wf_status wf_server_memory(wf_server* s, int64_t* in_use, int64_t* peak) {
  if (!s) return fail(WF_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  if (in_use) *in_use = (int64_t)s->arena.in_use();
  if (peak) *peak = (int64_t)s->arena.peak();
  return WF_OK;
}

extern "C" wf_status wf_server_destroy(wf_server* s) {
  if (!s) return WF_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    ++s->epoch;
    // Requests not yet launched are dropped; launched ones drain.  (wf_submit returns
    // WF_ESHUTDOWN from here on; every ticket is invalid once this call returns.)
    for (uint64_t t : s->queue) s->reqs.erase(t);
    for (uint64_t t : s->admitted) s->reqs.erase(t);
    s->queue.clear();
    s->admitted.clear();
    s->cv.notify_all();
  }
  if (s->thread.joinable()) s->thread.join();
  set_device(s->ctx);
  for (hipStream_t c : s->copy_streams) {
    hipStreamSynchronize(c);
    hipStreamDestroy(c);
  }
  for (auto& c : s->copying) hipEventDestroy(c.ev);
  for (hipEvent_t e : s->event_pool) hipEventDestroy(e);
  for (auto& L : s->slots) {
    if (L.stream) {
      hipStreamSynchronize(L.stream);
      hipStreamDestroy(L.stream);
    }
    if (L.ctl) hipFree(L.ctl);
    if (L.d_grids) hipFree(L.d_grids);
    if (L.d_items) hipFree(L.d_items);
    if (L.h_grids) hipHostFree(L.h_grids);
    if (L.h_items) hipHostFree(L.h_items);
    if (L.h_stage) hipHostFree(L.h_stage);
    if (L.host_err) hipHostFree(L.host_err);
    if (L.done) hipEventDestroy(L.done);
  }
  if (s->pin_base) hipHostFree(s->pin_base);
  if (s->dev_base) hipFree(s->dev_base);
  delete s;
  return WF_OK;
}
