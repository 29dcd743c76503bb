// Internal declarations shared by the kernel and runtime translation units of
// libwf (not part of the public ABI; see include/wf.h for that).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wf.h"

namespace wfk {

// Device copy of one problem.  `hand` holds the bottom-row handoff of every
// band but the last: band b writes row b, band b+1 reads it.
struct GridDesc {
  const void* cost;
  void* out;
  const void* top;
  const void* left;
  void* last_row;
  void* last_col;
  void* final_cell;
  uint32_t* hand;
  const void* sx;         // kind 1: the sequences whose absolute differences are the cell inputs
  const void* sy;
  int64_t m, n, ld_cost, ld_out, hand_ld;
  int32_t mode, nbands;
  int32_t kind, pad;      // kind 0: inputs read from `cost`; 1: |sx[i] - sy[j]|
};

// One work item: band `band` of grid `grid`.
struct Item {
  uint32_t grid, band;
};

struct KArgs {
  GridDesc g0;            // the grid when `grids` is null (single-grid launch)
  const GridDesc* grids;  // batched: descriptor table
  const Item* items;      // batched: work list in ticket order
  int64_t nitems;
  uint32_t* ctl;          // [0] ticket counter, [1] error code, [2] abort flag
  uint64_t watchdog_ticks;
  uint64_t* trace;        // optional: TRACE_WORDS per (work item, compute wave), see below
  uint64_t* ctrace;       // optional: CTRACE_WORDS per (work item, compute wave, chunk), see below
  int64_t ctrace_nc;      // chunks per (work item, compute wave) in ctrace
  uint32_t fault_band;    // test hook: band (of every grid) + 1 whose bottom row is never handed off; 0 = none
  // XCD queues (single-grid launches; nx <= 1: one global ticket counter).  A workgroup
  // on XCD x (hardware XCC id, modulo nx) takes tickets from queue x, which hands out, in
  // order, the tickets t with (t / seg) % nx == x: runs of seg consecutive bands share one
  // XCD, and a band hands its bottom row to the next band of its run through that XCD's
  // L2 instead of through memory.  Every queue needs a workgroup: the host uses queues
  // only for launches of at least nx workgroups on a device whose dispatcher deals
  // consecutive workgroups to consecutive XCDs.
  int32_t nx, seg;
};

// Per (work item, compute wave) trace record, written when KArgs::trace is set:
//   [0] grid << 32 | band << 8 | wave      [1] clock at band start (s_memtime)
//   [2] clock when the first top-boundary quad was valid   [3] clock at band end
//   [4] cycles waiting at chunk starts (c ring, H ring, T ring capacity)
//   [5] cycles waiting for top-boundary quads   [6] loader cycles waiting for a free c slot
//   [7] wall clock (100 MHz) at band start
constexpr int TRACE_WORDS = 8;
// Per-chunk trace record (compute waves, when KArgs::ctrace is set; chunks
// 0, CTRACE_EVERY, 2*CTRACE_EVERY, ...):
//   [0] wall clock on reaching the chunk start   [1] wall clock when its start conditions
//       were seen to hold (checked at the end of the chunk before)
//   [2] cycles spent so far waiting for top-boundary quads (needs KArgs::trace)
//   [3] which conditions were not met on arrival: 1 c ring, 2 H ring, 8 consumer's T ring
//   [4] loader: wall clock when the chunk's loads were issued  [5] when they had landed
//   [6] storer: wall clock when it began storing the chunk (or the last of a run of chunks
//       stored together)  [7] when it released the chunk's H slot
//   [8] feeder (compute wave 0): wall clock when the T ring first held every position the
//       chunk reads   [9] compute: wall clock when the chunk's T quads were validated
//   [10] compute, record s: wall clock right after the handoff store of chunk
//       s * CTRACE_EVERY + 4 was issued (the store that chunk s * CTRACE_EVERY of the next
//       band waits for)   [11] unused
constexpr int CTRACE_WORDS = 12;
constexpr int CTRACE_EVERY = 8;   // one record per this many chunks

// Control-word indices.
// CTL_QUEUE + x: ticket counter of XCD queue x (x < MAX_XCD).
constexpr int MAX_XCD = 8;
enum { CTL_TICKET = 0, CTL_ERROR = 1, CTL_ABORT = 2, CTL_QUEUE = 8, CTL_WORDS = CTL_QUEUE + MAX_XCD };
// Device error codes written to ctl[CTL_ERROR].
enum { DEV_OK = 0, DEV_TIMEOUT = 1 };

// Handoff sentinels ("not written yet"): a NaN pattern for fp32, INT32_MIN for int32.
constexpr uint32_t SENT_F32 = 0xFFFFFFFFu;
constexpr uint32_t SENT_I32 = 0x80000000u;

// Number of groups of 4 steps the walk of a strip of 64 R rows (R rows per lane) of an
// n-column grid takes: its last row finishes column n-1 at step n + 64 R - 2.
__host__ __device__ inline int64_t groups_for(int64_t n, int R) { return (n + 64 * R - 1 + 3) / 4; }
// Handoff row length in positions (>= 4 * groups_for(n, R)).
__host__ __device__ inline int64_t hand_ld_for(int64_t n, int R) { return ((4 * groups_for(n, R)) + 63) / 64 * 64; }

// Launch helpers implemented in wf_kernel.hip.
// dtype 0 = f32, 1 = i32, 2 = f64; rule 0 = min, 1 = max; W compute waves per workgroup of
// R rows per lane: (W, R) = (1, 1), (2, 1) or (1, 2); f64 only (1, 1).
hipError_t launch_sweep(int dtype, int rule, int W, int R, int nwg, const KArgs& args, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t stream);
// Arm the handoff rows of grids[0..ngrids) (device descriptor table) with `sent`, in one launch.
hipError_t launch_arm_hand(const GridDesc* grids, int ngrids, uint32_t sent, hipStream_t stream);
// Traceback of a computed grid (see wf_traceback): dtype 0 = f32, 1 = i32, 2 = f64.
hipError_t launch_traceback(int dtype, int rule, const void* H, int64_t ld, int64_t m, int64_t n, const void* top,
                            const void* left, int32_t* path, int64_t* length, hipStream_t stream);
// Records the XCD (hardware XCC id) each of nwg one-wave workgroups runs on into out[0..nwg).
hipError_t launch_xcc_probe(uint32_t* out, int nwg, hipStream_t stream);
// LDS bytes per workgroup (for occupancy decisions).
size_t lds_bytes(int W, int R);

// The allocation-free entry point's fixed device workspace: NOALLOC_CTL_WORDS control
// words (padded to 256 bytes), then handoff rows.  noalloc_scratch() returns its
// address on the current device.
constexpr int64_t NOALLOC_WORDS = (int64_t)WF_NOALLOC_SCRATCH_BYTES / 4;
constexpr int64_t NOALLOC_CTL_WORDS = 64;
hipError_t noalloc_scratch(uint32_t** ptr);
// Zero the control words at `ctl` (the error word only if reset_error) and arm `count`
// handoff-row words at `hand` with `sent`, in one launch.
hipError_t launch_noalloc_prep(uint32_t* ctl, bool reset_error, uint32_t* hand, uint32_t sent, int64_t count,
                               hipStream_t stream);

}  // namespace wfk
