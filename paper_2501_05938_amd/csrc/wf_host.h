// wf_host.h -- host-side pieces shared by the runtime (wf_runtime.cpp) and the
// serving front end (wf_server.cpp): the per-device context, launch slots,
// batch plans, argument checking and launch configuration.
#pragma once

#include "../../include/wf.h"
#include "wf_internal.h"

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

// A launch slot owns everything one in-flight launch mutates: control words,
// handoff rows, descriptor table and work list.  A slot is reused only once its
// last launch has completed (its event has fired and its error word was read).
struct Slot {
  uint32_t* ctl = nullptr;        // CTL_WORDS device words
  uint32_t* hand = nullptr;       // handoff rows (kept at the sentinel between launches)
  size_t hand_cap = 0;            // in uint32 elements
  uint32_t hand_sent = 0;         // sentinel the handoff rows currently hold
  wfk::GridDesc* grids = nullptr; // batched descriptor table
  size_t grids_cap = 0;
  wfk::Item* items = nullptr;     // batched work list
  size_t items_cap = 0;
  uint32_t* host_err = nullptr;   // pinned copy of ctl[CTL_ERROR] after the launch
  hipEvent_t done = nullptr;      // recorded after the launch and the error copy
  bool pending = false;           // a launch was recorded and not yet checked
  bool needs_rearm = false;       // an aborted launch left handoff rows written: refill before reuse
  bool reserved = false;          // held by a cached batch plan
  bool external = false;          // ctl/hand live in memory the slot does not own
  bool xcd_queues = false;        // its last launch used XCD queues
};

// A batch whose work list, descriptor tables and (optionally) captured graphs are
// kept for replay.  Two lanes, each with its own slot, let two replays be in flight.
struct BatchPlanEntry {
  uint64_t hash = 0;
  std::vector<wf_problem> probs;          // the problem array last launched through this plan
  std::vector<int64_t> shape;             // (m, n, mode) per problem: what the plan depends on
  int bs = 1, order = 1, nwg = 0, dtype = 0, rule = 0;
  bool use_graph = false;
  std::vector<int64_t> perm;              // problem index of descriptor k
  std::vector<wfk::Item> items;
  std::vector<size_t> hand_off;
  size_t hand_total = 0;
  struct Lane {
    int slot = -1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<wfk::GridDesc> descs;     // the table now in the slot's device copy
    wfk::GridDesc* staging = nullptr;     // pinned staging for table re-uploads
    bool items_loaded = false;            // the work list is in the slot's device copy
  };
  Lane lanes[2];
  uint64_t replays = 0;
  uint64_t last_use = 0;
};

struct TuneEntry {
  int bs = 1, order = 1, wgs = 0;  // band shape (wfh::shape_*), work order, workgroups
  double ms = 0;
};

struct wf_ctx {
  int device = 0;
  int num_cus = 256;
  uint64_t watchdog_ticks = 200000000ull;  // 2 s of the 100 MHz device wall clock
  uint32_t fault = 0;                      // test hook (WF_FAULT): band whose handoff the next launch drops, + 1
  static constexpr int MAX_SLOTS = 64;     // launches in flight per context before a launch blocks
  std::vector<std::unique_ptr<Slot>> slots;
  size_t next_slot = 0;
  static constexpr int MAX_PLANS = 8;
  std::vector<std::unique_ptr<BatchPlanEntry>> plans;
  uint64_t use_clock = 0;
  std::map<std::string, TuneEntry> tuned;  // shape class -> configuration
  std::string tune_file;                   // WF_TUNE_CACHE: where `tuned` persists (empty: memory only)
  wf_status sticky = WF_OK;                // device error seen, reported once
  Slot* noalloc = nullptr;                 // wf_solve_noalloc's slot: ctl/hand in the fixed device array
  // XCD queues of single-grid launches: the number of XCDs when the placement probe at
  // wf_init found workgroup w of a launch on XCD w % nx, else 1 (off).  WF_XCD_QUEUES=0
  // turns them off.
  int nx = 1;
};

namespace wfh {

// Record `msg` as this thread's last error and return `s`.
wf_status fail(wf_status s, const std::string& msg);
// Make the context's device current.
wf_status set_device(wf_ctx* ctx);
// Validate one problem (idx >= 0 names it in the message).
wf_status check_problem(const wf_problem* p, int64_t idx);
// Band shapes: 1 = one compute wave with one row per lane (64-row bands); 2 = two
// compute waves chained through LDS (128-row bands); 3 = one compute wave with two rows
// per lane (128-row bands).
constexpr int SHAPE_MAX = 3;
inline int shape_waves(int bs) { return bs == 2 ? 2 : 1; }
inline int shape_rows_per_lane(int bs) { return bs == 3 ? 2 : 1; }
inline int shape_rows(int bs) { return 64 * shape_waves(bs) * shape_rows_per_lane(bs); }
// Band shape for a single grid with m rows.
int choose_shape(int64_t m);
// Resident workgroups per compute unit at band shape bs (fp64 workgroups take 98 KB of LDS).
int wgs_per_cu(int bs, int dtype);
// Launch of the sweep kernel at band shape bs.
hipError_t launch_shape(int dtype, int rule, int bs, int nwg, const wfk::KArgs& args, hipStream_t stream);
// Handoff sentinel of a dtype.
uint32_t sentinel_of(int dtype);
// Kernel descriptor of a problem, cut into bands of shape bs.
wfk::GridDesc make_desc(const wf_problem* p, int bs, uint32_t* hand);
// Handoff-row elements a problem needs at band shape bs.
size_t hand_elems(const wf_problem* p, int bs);
// Arguments of a launch over `nitems` work items with the context's watchdog and fault hook.
// (Consumes the context's one-shot fault hook.)
wfk::KArgs base_args(wf_ctx* ctx, uint32_t* ctl, int64_t nitems);
// XCD queues for a single-grid launch of nwg workgroups (see KArgs::nx), when the context
// has them and the launch has a workgroup for every XCD.
void xcd_queues(const wf_ctx* ctx, wfk::KArgs& a, int nwg);

}  // namespace wfh

#define WF_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return wfh::fail(WF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)
