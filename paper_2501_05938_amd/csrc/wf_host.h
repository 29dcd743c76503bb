// wf_host.h -- host-side pieces shared by the runtime (wf_runtime.cpp) and the
// serving front end (wf_server.cpp): the per-device context, launch slots,
// argument checking and launch configuration.
#pragma once

#include "../../include/wf.h"
#include "wf_internal.h"

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

// A launch slot owns everything one in-flight launch mutates: control words,
// handoff rows, descriptor table and work list.  Slots are reused round-robin
// once their last launch has completed.
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
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int slot = -1;
  std::vector<wfk::GridDesc> descs;  // the descriptor table now in the slot's device copy
};

struct wf_ctx {
  int device = 0;
  int num_cus = 256;
  uint64_t watchdog_ticks = 200000000ull;  // 2 s of the 100 MHz device wall clock
  static constexpr int NSLOT = 8;
  Slot slots[NSLOT];
  int next_slot = 0;
  std::map<std::string, GraphEntry> graphs;
  std::map<std::string, std::pair<int, int>> tuned;  // batch shape signature -> (W, order)
  wf_status sticky = WF_OK;                // device error seen, reported once
};

namespace wfh {

// Record `msg` as this thread's last error and return `s`.
wf_status fail(wf_status s, const std::string& msg);
// Make the context's device current.
wf_status set_device(wf_ctx* ctx);
// Validate one problem (idx >= 0 names it in the message).
wf_status check_problem(const wf_problem* p, int64_t idx);
// Compute waves per workgroup for a grid (or batch) whose tallest grid has m rows.
int choose_waves(int64_t m);
// Resident workgroups per compute unit at W compute waves per workgroup.
int wgs_per_cu(int W);
// Handoff sentinel of a dtype.
uint32_t sentinel_of(int dtype);
// Kernel descriptor of a problem, cut into bands of 64*W rows.
wfk::GridDesc make_desc(const wf_problem* p, int W, uint32_t* hand);
// Handoff-row elements a problem needs at W.
size_t hand_elems(const wf_problem* p, int W);

}  // namespace wfh

#define WF_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return wfh::fail(WF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)
