// wf_kernel.hip -- the persistent anti-diagonal wavefront sweep for gfx950.
//
// Cell rule (see include/wf.h): H[i][j] = c[i][j] + op(H[i-1][j], H[i][j-1], H[i-1][j-1]).
//
// Work decomposition
//   A grid is cut into bands of 64*W rows.  Workgroups are persistent: they
//   take band tickets from a global counter in order, so a band only ever
//   waits on a band with a smaller ticket, which is held by a running
//   workgroup.  A workgroup holds W compute waves (64 rows each, lane r owns
//   row r) and staging waves that never mix load and store traffic: one
//   loader and one storer per compute wave, and one feeder.
//
// Compute wave (the hot loop)
//   Lane r handles column t - r at step t, so each step advances a 64-cell
//   anti-diagonal.  N comes from lane r-1 by a DPP wave_shr:1 of the previous
//   step's H, NW is the previous step's N, W is the lane's own previous H.
//   Lane 0's N is the bottom row of the strip above: it is supplied as the
//   DPP "old" value, which a disabled source lane leaves in place.  Per step:
//   one DPP move, one min3/max3, one add (a single rounding).
//   Inputs c come from an LDS ring filled by the loader, stored skewed
//   (row r, position p holds column p - r) so that all lanes read the same
//   position with one aligned 16-byte load per 4 steps; H goes to a second
//   LDS ring in the same layout.  The walk goes in chunks of 16 steps: the
//   control words and the chunk's T quads are checked once at its start, and
//   the next chunk's inputs are read while it runs.  The compute wave issues
//   no vector-memory loads, so it never waits on memory counters.
//
// Handoff of the bottom row (the N of the next strip's lane 0)
//   Inside a workgroup, lane 63 of compute wave w writes its 4 values of each
//   step group into the T ring of wave w+1 (LDS).  Across workgroups, the last
//   compute wave gathers a chunk's 16 values into lanes 60..63 and writes them
//   to a global handoff row with one device-coherent (sc1) store, and the
//   feeder of the next band polls that row and copies it into the T ring of
//   its compute wave 0.  Past a band's last position the T ring is padded with
//   absent values, so every chunk after the first four runs the same code.
//   Validity is carried by the data itself: slots hold a sentinel until
//   written, and a reader accepts a quad only when none of its four words is
//   the sentinel (a 16-byte read racing a 16-byte write may see part of it).
//   Consumers re-arm slots to the sentinel after use and publish how far they
//   have re-armed; a producer writes a slot, and a consumer reads ahead into
//   it, only once the slot's previous lap has been re-armed, so a stale value
//   can never pass for a fresh one.
//
// Every wait has a wall-clock watchdog; on expiry the workgroup raises a
// device-wide abort flag and all waits end, so a kernel always drains.
#include "wf_internal.h"

#include <stddef.h>
#include <type_traits>

namespace wfk {
namespace {

constexpr int CHUNK = 16;               // positions per IO chunk
constexpr int SLAB = 64 * CHUNK * 4;    // bytes of one chunk of 64 lane rows (16 positions each)
constexpr int C_SLOTS = 8;              // chunk slots of the c ring
constexpr int H_SLOTS = 8;              // chunk slots of the H ring (slack for the storer's jitter)
constexpr int RING_T = 512;             // positions held by the T ring
// A chunk slot holds R slabs: slab s holds grid row R*r + s of every lane r (R rows
// per lane).  Inside a slab, the 16 bytes of lane row r, quad q (positions 4q..4q+3 of
// the chunk) sit at (r/16)*1024 + (r%16)*64 + 16*(q ^ swz(r)): a 1024-byte block holds
// 16 whole rows of the chunk, each row's four quads in its own 64 contiguous bytes in
// a per-row order.  A 64-lane LDS-DMA load (lane L -> byte 16L) then fills one block
// with lanes 4j..4j+3 reading one row's 64 contiguous bytes, so the global accesses of
// four consecutive lanes coalesce; the storer reads the H ring the same way.  The
// per-row quad order spreads the compute wave's accesses to one quad of its 64 rows
// (64 bytes apart) over all banks: any 8 consecutive lanes hit 8 distinct 16-byte
// bank groups (row parity picks the half of 128 bytes, swz(r) the quad within it).
constexpr int QUAD = 16;
__device__ __forceinline__ int lane_off(int r) { return (r >> 4) * 1024 + (r & 15) * 64; }
__device__ __forceinline__ int swz(int r) { return (r >> 1) & 3; }
// Byte offset of lane row r's logical quad q inside a slab.
__device__ __forceinline__ int quad_off(int r, int q) { return lane_off(r) + QUAD * (q ^ swz(r)); }

typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4a4 __attribute__((ext_vector_type(4), aligned(4)));

// Per compute wave: the T ring and the control words.  The c and H rings (which depend
// on R) are in WaveRings.
struct alignas(16) WaveLds {
  uint32_t tring[RING_T];
  uint32_t c_ready;   // chunks of c committed to cring (IO -> compute)
  uint32_t h_done;    // positions of H stored out of hring (IO -> compute)
  uint32_t t_fed;     // T positions below this are in the ring (feeder or the compute wave above -> this
                      // wave; wave 0's also -> storer)
  uint32_t abort;     // workgroup abort flag (only lds[0].abort is used)
  uint32_t progress;  // (signed) position of the chunk being computed: earlier chunks are done (compute -> IO)
  uint32_t t_reset;   // T positions below this have been read (this wave -> feeder or the compute wave
                      // above): slots of positions < t_reset + RING_T are writable
  uint32_t pad[2];
  // trace counters (written only when KArgs::trace is set)
  uint64_t tr_start, tr_first, tr_end, tr_wall;
  uint64_t tr_chunk_wait;   // compute cycles waiting at chunk starts
  uint64_t tr_t_wait;       // compute cycles waiting for T quads
  uint64_t tr_load_wait;    // loader cycles waiting for a free c slot
  uint64_t tr_pad;
  uint64_t sink[64];        // lanes 1..63's half of the per-chunk progress store (never read)
};

template <int R>
struct alignas(16) WaveRings {
  unsigned char cring[C_SLOTS * R * SLAB];
  unsigned char hring[H_SLOTS * R * SLAB];
};

#define CBAR() asm volatile("" ::: "memory")

template <typename T> __device__ __forceinline__ uint32_t bits(T v) { return __builtin_bit_cast(uint32_t, v); }
template <typename T> __device__ __forceinline__ T from_bits(uint32_t u) { return __builtin_bit_cast(T, u); }

template <typename T> struct Num;
template <> struct Num<float> {
  static constexpr uint32_t SENT = SENT_F32;
  // The fp32 sentinel is the largest 32-bit pattern, so a quad holds it iff its unsigned max does.
  __device__ static uint32_t probe(u4 q) {
    uint32_t t = q.x > q.y ? q.x : q.y;
    t = t > q.z ? t : q.z;
    return t > q.w ? t : q.w;
  }
  // Probe of several quads from their probes.
  __device__ static uint32_t combine(uint32_t a, uint32_t b) { return a > b ? a : b; }
  template <int RULE> __device__ static float absent() { return RULE == 0 ? __builtin_inff() : -__builtin_inff(); }
  template <int RULE> __device__ static float op3(float a, float b, float c) {
    if constexpr (RULE == 0) return __builtin_fminf(__builtin_fminf(a, b), c);
    else return __builtin_fmaxf(__builtin_fmaxf(a, b), c);
  }
  __device__ static float add(float a, float b) { return a + b; }
};
template <> struct Num<int32_t> {
  static constexpr uint32_t SENT = SENT_I32;
  // The int32 sentinel is INT32_MIN, so a quad holds it iff its signed min does.
  __device__ static uint32_t probe(u4 q) {
    int32_t t = (int32_t)q.x < (int32_t)q.y ? (int32_t)q.x : (int32_t)q.y;
    t = t < (int32_t)q.z ? t : (int32_t)q.z;
    return (uint32_t)(t < (int32_t)q.w ? t : (int32_t)q.w);
  }
  __device__ static uint32_t combine(uint32_t a, uint32_t b) { return (int32_t)a < (int32_t)b ? a : b; }
  template <int RULE> __device__ static int32_t absent() { return RULE == 0 ? INT32_MAX : INT32_MIN + 1; }
  template <int RULE> __device__ static int32_t op3(int32_t a, int32_t b, int32_t c) {
    if constexpr (RULE == 0) { int32_t t = a < b ? a : b; return t < c ? t : c; }
    else { int32_t t = a > b ? a : b; return t > c ? t : c; }
  }
  __device__ static int32_t add(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }
};

// fp64 (its own sweep kernel below; the traceback uses the absent value).
template <> struct Num<double> {
  template <int RULE> __device__ static double absent() { return RULE == 0 ? __builtin_inf() : -__builtin_inf(); }
};

// Four absent boundary values (the T ring's padding past a band's last T position).
template <typename T, int RULE> __device__ __forceinline__ u4 absent4() {
  const uint32_t v = bits(Num<T>::template absent<RULE>());
  return u4{v, v, v, v};
}

// End of the T positions a walk of G groups with R rows per lane reads: its last chunk
// (number NC - 1, NC = ceil(4G / 16)) checks positions up to 16 (NC - 1) + 64 R + 16.
__host__ __device__ constexpr int t_pad_end(int G, int R) { return CHUNK * ((4 * G + CHUNK - 1) / CHUNK) + 64 * R; }
// First T position a walk reads: the quad of columns -3 .. 0 of the row above the band
// (position p holds the row above at column p - (64 R - 1)).
__host__ __device__ constexpr int t_first(int R) { return 64 * R - 4; }

// N for every lane: lane r receives lane r-1's `src`; lane 0 keeps `old`.
template <typename T> __device__ __forceinline__ T dpp_shr1(T old, T src) {
  return from_bits<T>((uint32_t)__builtin_amdgcn_update_dpp((int)bits(old), (int)bits(src), 0x138, 0xf, 0xf, false));
}

__device__ __forceinline__ uint32_t ld_ctl(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void st_ctl(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
typedef __attribute__((address_space(3))) unsigned char lds_u8;
typedef __attribute__((address_space(3))) u4 lds_u4;
typedef uint32_t u2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) u2 lds_u2;
typedef uint32_t u3 __attribute__((ext_vector_type(3)));
typedef __attribute__((address_space(3))) u3 lds_u3;
template <class P> __device__ __forceinline__ lds_u8* L8(P* p) { return (lds_u8*)(void*)p; }
__device__ __forceinline__ u4 lds_ld4(const lds_u8* p) { return *(const lds_u4*)p; }
__device__ __forceinline__ u4 lds_ld4_fresh(const lds_u8* p) { return *(const volatile lds_u4*)p; }
__device__ __forceinline__ void lds_st4(lds_u8* p, u4 v) { *(lds_u4*)p = v; }

// Buffer descriptor for a wave-uniform base; forced into scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  const uint64_t b = (uint64_t)base;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  void* p = (void*)(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}
constexpr int CPOL_SC1 = 16;  // device-scope coherent access
// The XCD (hardware XCC id, bits 3:0 of HW_REG_XCC_ID) the calling wave runs on.
__device__ __forceinline__ uint32_t xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20); }

typedef __attribute__((address_space(1))) uint32_t glb_u32;
__device__ __forceinline__ glb_u32* G32(uint32_t* p) { return (glb_u32*)(void*)p; }
// Global-address-space views of plain pointers.  Generic (flat) accesses would also
// count on the LDS counter, so every wait for an LDS access would wait for them too.
typedef __attribute__((address_space(1))) u4a4 glb_u4a4;
__device__ __forceinline__ glb_u4a4* G128(uint32_t* p) { return (glb_u4a4*)(void*)p; }
template <typename T> __device__ __forceinline__ const __attribute__((address_space(1))) T* GC(const void* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
__device__ __forceinline__ uint32_t ld_dev(uint32_t* p) {
  return __hip_atomic_load(G32(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Abort the whole launch: raise the workgroup flag and the device-wide flag.
template <class WL>
__device__ __forceinline__ void raise_abort(WL* lds, const KArgs& a) {
  st_ctl(&lds[0].abort, 1u);
  __hip_atomic_store(G32(a.ctl + CTL_ERROR), (uint32_t)DEV_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(G32(a.ctl + CTL_ABORT), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Idle-time watchdog.  A clock read is a scalar-memory round trip (hundreds of
// cycles), far longer than one poll, so the clock is read only once every
// WATCH_SPINS idle polls: the first read starts the idle period, later ones
// compare against it.  Progress resets the watch.
constexpr uint32_t WATCH_SPINS = 1024;
struct Watch {
  uint64_t t0 = 0;
  uint32_t spins = 0;
  __device__ void reset() {
    t0 = 0;
    spins = 0;
  }
  // True once the current idle period has lasted longer than `ticks`.
  __device__ bool tick(uint64_t ticks) {
    if ((++spins & (WATCH_SPINS - 1)) != 0u) return false;
    const uint64_t now = wall_clock64() | 1u;  // never 0
    if (t0 == 0) {
      t0 = now;
      return false;
    }
    return now - t0 > ticks;
  }
};

// Spin until cond() holds.  Returns false (without waiting further) if the launch is
// aborting; callers then run on to the end of the band, whose output is discarded.
// Compute waves watch only the workgroup flag (no global loads on their path, so the
// hot loop never waits on vector-memory counters); IO waves also poll the device flag
// and relay it into the workgroup flag.
template <bool DEVICE_FLAG, class F, class WL>
__device__ __forceinline__ bool wait_until(F&& cond, WL* lds, const KArgs& a) {
  if (cond()) return true;
  Watch w;
  uint32_t polls = 0;
  for (;;) {
    __builtin_amdgcn_s_sleep(1);
    if (cond()) return true;
    if (ld_ctl(&lds[0].abort)) return false;
    if (DEVICE_FLAG && (++polls & 255u) == 0u && ld_dev(a.ctl + CTL_ABORT)) {
      st_ctl(&lds[0].abort, 1u);
      return false;
    }
    if (w.tick(a.watchdog_ticks)) {
      raise_abort(lds, a);
      return false;
    }
  }
}

// Sampled per-chunk trace record of compute wave w (see CTRACE_WORDS), or null.
typedef __attribute__((address_space(1))) uint64_t glb_u64;
__device__ __forceinline__ glb_u64* chunk_rec(const KArgs& a, uint32_t item, int W, int w, int k) {
  if (!a.ctrace || (k % CTRACE_EVERY) != 0) return nullptr;
  return (glb_u64*)(void*)(a.ctrace + (((int64_t)item * W + w) * a.ctrace_nc + k / CTRACE_EVERY) * CTRACE_WORDS);
}

// ------------------------------------------------------------ compute wave
// Rare path of an inline spin, called every few thousand polls.  Returns the start
// of the idle period (taking it now when t0 is 0), or 0 when the wait must end: the
// launch is aborting, or the wait has outlasted the watchdog (then it raises the abort).
template <class WL>
__device__ __noinline__ uint64_t spin_check(WL* lds, uint32_t* ctl, uint64_t watchdog_ticks, uint64_t t0) {
  if (ld_ctl(&lds[0].abort)) return 0;
  const uint64_t now = wall_clock64() | 1u;
  if (t0 == 0) return now;
  if (now - t0 > watchdog_ticks) {
    st_ctl(&lds[0].abort, 1u);
    __hip_atomic_store(G32(ctl + CTL_ERROR), (uint32_t)DEV_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(G32(ctl + CTL_ABORT), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  return t0;
}

// Reads of chunk kn's inputs for one lane: its 4 R c quads (cq[q]: this lane's logical
// quad q in slab 0 of slot 0), and the chunk's four T quads (the T ring is fed up to the
// padding past the band's last position, so every chunk has four).  A read past the
// last chunk only picks up unused stale data.
template <int R>
__device__ __forceinline__ void read_c(int kn, const lds_u8* const (&cq)[4], u4 (&c)[R][4]) {
  const int sb = (kn % C_SLOTS) * (R * SLAB);
#pragma unroll
  for (int s = 0; s < R; ++s)
#pragma unroll
    for (int q = 0; q < 4; ++q) c[s][q] = lds_ld4(cq[q] + sb + s * SLAB);
}
template <int R>
__device__ __forceinline__ void read_t(int kn, const lds_u8* tr_base, u4 (&t)[4]) {
  // The chunk's 16 positions are contiguous in the ring (it holds a whole number of
  // chunks).  Their address is the same in every lane; held in one vector register, the
  // four reads take their distance from it as an immediate offset (a scalar address
  // would be copied into a vector register for each read).
  uint32_t tb = (uint32_t)(uintptr_t)(tr_base + ((CHUNK * kn + 64 * R) & (RING_T - 1)) * 4);
  asm volatile("" : "+v"(tb));
#pragma unroll
  for (int q = 0; q < 4; ++q) t[q] = lds_ld4_fresh((const lds_u8*)(uintptr_t)tb + 16 * q);
}

// Control words a chunk start checks, read ahead of time.  The counters only grow, so
// a check that passes on values read earlier also passes on current ones; one that
// fails falls back to waiting on fresh reads.  This wave's three words are read with one
// 12-byte LDS read and kept in vector registers until the check: taking scalar copies
// right after the read would make the walk wait for it mid-chunk, and so would a wider
// read whose unused register the compiler hands to the walk while the read is in flight
// (a register may not be rewritten before the read that targets it has landed).
struct CtlSnap {
  u3 own;                 // c_ready, h_done, t_fed of this wave
  uint32_t cons_t_reset;  // the consumer wave's t_reset (CONS == 1)
};
static_assert(offsetof(WaveLds, c_ready) % 16 == 0 && offsetof(WaveLds, h_done) == offsetof(WaveLds, c_ready) + 4 &&
                  offsetof(WaveLds, t_fed) == offsetof(WaveLds, c_ready) + 8,
              "c_ready, h_done and t_fed open an aligned quad");
static_assert(offsetof(WaveLds, progress) % 8 == 0 && offsetof(WaveLds, t_reset) == offsetof(WaveLds, progress) + 4,
              "progress and t_reset form an aligned pair (published with one store)");

template <int CONS>
__device__ __forceinline__ void snap_ctl(WaveLds& L, WaveLds* C, CtlSnap& s) {
  s.own = *(const volatile lds_u3*)L8(&L.c_ready);
  s.cons_t_reset = CONS == 1 ? ld_ctl(&C->t_reset) : 0u;
}

// Sampled per-chunk trace record of a compute wave's chunk k (crec: the wave's records),
// or null.
__device__ __forceinline__ glb_u64* chunk_trace(uint64_t* crec, int k) {
  return crec && (k % CTRACE_EVERY) == 0 ? (glb_u64*)(void*)(crec + (int64_t)(k / CTRACE_EVERY) * CTRACE_WORDS)
                                         : nullptr;
}

// Whether chunk k may start: the c ring holds chunk k + 1 (read during chunk k), chunk
// k's H slot is free, the T ring holds chunk k's positions, and (CONS == 1) the consumer
// has read the positions that chunk k's groups overwrite in its ring.  The check runs on
// a snapshot of the control words read before chunk k's T quads `t`; the snapshot's
// words are the same in every lane, so it is a vector compare per word and one branch on
// the combined lane mask.  When it fails, the wave waits on fresh snapshots and reads
// `t` again (after the snapshot that shows the ring holds them, so they are the fed
// values).  Run at the end of chunk k - 1, so that no snapshot stays live across the
// walk's loop edge (the compiler would move it to scalar registers, which makes the
// walk wait for the read mid-chunk).
template <int R, int CONS>
__device__ __forceinline__ void chunk_gate(int k, int NCc, WaveLds* lds, WaveLds& L, WaveLds* C, CtlSnap& snap,
                                           u4 (&t)[4], const KArgs& a, int lane, glb_u64* rec) {
  const int pos = CHUNK * k;
  const int need_c = k + 2 < NCc ? k + 2 : NCc;
  const int need_h = pos + CHUNK - H_SLOTS * CHUNK;
  const int need_f = pos + 64 * R + CHUNK;
  const int need_t = pos + CHUNK - RING_T;
  auto ok = [&](const CtlSnap& v) {
    const bool p = ((int)v.own.x >= need_c) & ((int)v.own.y >= need_h) & ((int)v.own.z >= need_f) &
                   (CONS != 1 || (int)v.cons_t_reset >= need_t);
    return __builtin_amdgcn_ballot_w64(p) != 0ull;
  };
  if (!ok(snap)) {
    const uint64_t c0 = a.trace ? __builtin_readcyclecounter() : 0;
    if (rec && lane == 0) {
      rec[3] = ((int)snap.own.x < need_c ? 1u : 0u) | ((int)snap.own.y < need_h ? 2u : 0u) |
               ((int)snap.own.z < need_f ? 4u : 0u) | (CONS == 1 && (int)snap.cons_t_reset < need_t ? 8u : 0u);
    }
    wait_until<false>([&] { snap_ctl<CONS>(L, C, snap); return ok(snap); }, lds, a);
    read_t<R>(k, L8(L.tring), t);
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the re-read quads are in registers
    if (a.trace && lane == 0) L.tr_chunk_wait += __builtin_readcyclecounter() - c0;
  }
  if (rec && lane == 0) {
    rec[1] = wall_clock64();
    rec[2] = L.tr_t_wait;
  }
}

// One chunk (4 groups of 4 steps) of the walk, computed from the inputs read during the
// previous chunk (cc, tc) while the next chunk's inputs are read into (cn, tn).
// Lane r owns the R rows R r .. R r + R - 1 of the strip (sub-rows s = 0 .. R-1); row
// R r + s handles column t - (R r + s) at step t.  Sub-row 0's N comes from lane r-1's
// last sub-row by DPP (lane 0: the T value), its NW is the previous step's N; sub-row
// s > 0 takes N and NW from sub-row s-1 of the same lane (its values one and two steps
// back).  The R cells of a step depend only on earlier steps, so they run side by side.
// The chunk's T quads are read near the end of the previous chunk, right after the
// control snapshot, which the previous chunk then checks (chunk_gate) after its last
// group, including the snapshot's count of fed T positions (the group loop runs without
// branches): when the ring did not yet hold them, it waits for the count and reads the
// quads again.
// KIND 0: the first 4 R chunks, where rows left of column 0 keep their boundary value;
// KIND 1: every later chunk.  MASK: KIND 0 chunks select the kept value per cell; without
// it (floating point, default left boundary, no row padding) a cell left of column 0 is
// computed like any other: its own and its upper neighbours' values are then all
// "absent" (infinite), the finite input added to an infinity gives the same infinity,
// and every such cell holds the absent value, which is its boundary value.  The T ring
// is fed past the band's last T position with absent values, so every chunk reads four
// quads; groups past the last one (g >= G) compute cells right of the grid, which
// nothing stores or reads.
// CONS: 0 = no consumer, 1 = the next compute wave (LDS), 2 = the next band (global
// handoff row).
template <typename T, int RULE, int R, int KIND, int CONS, bool MASK, bool LOCAL>
__device__ __forceinline__ void compute_chunk(
    int k, int G, int gT, int NCc, WaveLds* lds, WaveLds& L, WaveLds* C,
    __amdgpu_buffer_rsrc_t hand_out, const lds_u8* const (&cq)[4], lds_u8* const (&hq)[4], lds_u8* ct_base,
    const lds_u8* hrd, lds_u8* prog_at, bool lane63, int lane, const u4 (&cc)[R][4], u4 (&tc)[4], u4 (&cn)[R][4],
    u4 (&tn)[4], uint32_t& tprev_w,
    T (&H)[R], T (&Hp)[R], T& Np, CtlSnap& snap, const KArgs& a, uint64_t* crec, bool more) {
  const int pos = CHUNK * k;
  // Keep the chunk-start check (and the scalar copies of the control snapshot it takes)
  // from being scheduled into the previous chunk's walk.
  __builtin_amdgcn_sched_barrier(0);
  // Per-chunk records are sampled (every CTRACE_EVERY-th chunk): each clock read is a
  // scalar-memory round trip that would otherwise slow the walk being measured.
  glb_u64* rec = chunk_trace(crec, k);
  if (rec && lane == 0) rec[0] = wall_clock64();
  const lds_u8* tr_base = L8(L.tring);
  CBAR();
  // Publish, with one store, that the chunks before this one are done (progress) and that
  // this chunk's T quads are in registers, so the feeder (or the compute wave above) may
  // reuse their slots (t_reset); as the compute wave above the consumer, also how far
  // the consumer's T ring is written: every position of the earlier chunks.
  // Every lane stores, so the store needs no exec change: lane 0 to the control words
  // (prog_at), the others to the wave's sink.
  *(volatile lds_u2*)prog_at = u2{(uint32_t)pos, (uint32_t)(pos + 64 * R + CHUNK)};
  if (CONS == 1 && lane == 0) st_ctl(&C->t_fed, (uint32_t)pos);
  if (rec && lane == 0) rec[9] = wall_clock64();
  read_c<R>(k + 1, cq, cn);
  const int hb = (k % H_SLOTS) * (R * SLAB);
  lds_u8* ct = ct_base + (pos & (RING_T - 1)) * 4;
  // Bottom-row quads of the chunk for the next band, stored once at the end of the chunk
  // from lanes 60..63 (lane 60 + q: group q's quad).  Lane 63 computes them; lanes 60..62
  // read groups 0..2's from the H ring (hrd: lane 63's quad lane - 60 of slot 0) while
  // group 3 runs, and lane 63 keeps group 3's own.
  u4 hv = {0u, 0u, 0u, 0u}, h4_last = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int g = 4 * k + q;
    // The next chunk start's checks, read while this last group runs, then the next
    // chunk's T quads: LDS accesses of one wave complete in order, so when the
    // snapshot shows the ring holds them, these reads returned them.
    if (q == 3) {
      snap_ctl<CONS>(L, C, snap);
      read_t<R>(k + 1, tr_base, tn);
      if (CONS == 2) {
        asm volatile("" ::: "memory");  // after groups 0..2's H ring writes
        hv = lds_ld4(hrd + hb);
      }
    }
    const u4 tv = tc[q];
    const uint32_t tk[4] = {tprev_w, tv.x, tv.y, tv.z};
    if (KIND == 1 || g < gT) tprev_w = tv.w;
    u4 h4[R];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const T N = dpp_shr1<T>(from_bits<T>(tk[e]), H[R - 1]);
      T Hn[R];
      // The lower sub-rows first: they read only registers of this lane, which leaves the
      // DPP source (the last sub-row) written a few instructions before the next step's move.
#pragma unroll
      for (int sr = R - 1; sr >= 1; --sr)
        Hn[sr] = Num<T>::add(from_bits<T>(cc[sr][q][e]), Num<T>::template op3<RULE>(H[sr - 1], Hp[sr - 1], H[sr]));
      Hn[0] = Num<T>::add(from_bits<T>(cc[0][q][e]), Num<T>::template op3<RULE>(N, Np, H[0]));
      if (KIND == 0 && MASK) {
        // rows left of column 0 keep the left boundary
#pragma unroll
        for (int sr = 0; sr < R; ++sr) Hn[sr] = (4 * g + e < R * lane + sr) ? H[sr] : Hn[sr];
      }
      Np = N;
#pragma unroll
      for (int sr = 0; sr < R; ++sr) {
        Hp[sr] = H[sr];
        H[sr] = Hn[sr];
        h4[sr][e] = bits(H[sr]);
      }
    }
    // H into the ring, bottom row to the consumer.  Positions below t_first(R) are never
    // read by a consumer.
#pragma unroll
    for (int sr = 0; sr < R; ++sr) lds_st4(hq[q] + hb + sr * SLAB, h4[sr]);
    if (q == 3) h4_last = h4[R - 1];
    if (CONS == 1 && (KIND != 0 || g >= 16 * R - 1)) {
      // Past the last group the consumer's ring gets absent values (its padding).
      if (lane63) lds_st4(ct + 16 * q, g < G ? h4[R - 1] : absent4<T, RULE>());
    }
  }
  if (CONS == 2) {
    // Lane 60+q holds group 4k+q's quad.  Only positions [t_first(R), 4G) are written:
    // the others are never read by a consumer and stay at the sentinel.
    const int g = 4 * k + lane - 60;
    const u4 hand4 = lane63 ? h4_last : hv;
    if (lane >= 60 && g < G && (KIND != 0 || g >= 16 * R - 1)) {
      // LOCAL: the consumer is on this XCD (plain store through the shared L2).
      __builtin_amdgcn_raw_buffer_store_b128(hand4, hand_out, 16 * g, 0, LOCAL ? 0 : CPOL_SC1);
    }
    if (crec && (k % CTRACE_EVERY) == 4 && lane == 0)
      ((__attribute__((address_space(1))) uint64_t*)(void*)crec)[(int64_t)(k / CTRACE_EVERY) * CTRACE_WORDS + 10] =
          wall_clock64();
  }
  // The next chunk's start conditions, on the snapshot read during the last group.
  // (more: chunk k + 1 exists; a constant where the caller's loop bound says so)
  if (more) chunk_gate<R, CONS>(k + 1, NCc, lds, L, C, snap, tn, a, lane, chunk_trace(crec, k + 1));
}

template <typename T, int RULE, int R, int CONS, bool MASK, bool LOCAL>
__device__ __forceinline__ void compute_walk(int G, int gT, WaveLds* lds, WaveLds& L, WaveLds* C,
                                             __amdgpu_buffer_rsrc_t hand_out, const lds_u8* const (&cq)[4],
                                             lds_u8* const (&hq)[4], const lds_u8* hrd, int lane, const T (&Hinit)[R],
                                             const KArgs& a, uint64_t* crec) {
  const int NCc = (4 * G + CHUNK - 1) / CHUNK;
  lds_u8* ct_base = CONS == 1 ? L8(C->tring) : nullptr;
  const bool lane63 = lane == 63;
  lds_u8* const prog_at = lane == 0 ? L8(&L.progress) : L8(&L.sink[lane]);
  constexpr int TF = t_first(R);
  // First T quad: columns -3..0 of the row above (.z is the corner, .w column 0), read
  // once the ring holds it.
  {
    const uint64_t c0 = a.trace ? __builtin_readcyclecounter() : 0;
    wait_until<false>([&] { return (int)ld_ctl(&L.t_fed) >= TF + 4; }, lds, a);
    if (a.trace && lane == 0) L.tr_t_wait += __builtin_readcyclecounter() - c0;
  }
  const u4 tprev = lds_ld4_fresh(L8(L.tring) + TF * 4);
  if (a.trace && lane == 0) L.tr_first = __builtin_readcyclecounter();
  // NW of step 0: the corner for lane 0; for the other lanes the row above's column -1,
  // which lies left of the grid (absent by default; selected away when masked).
  T Np = lane == 0 ? from_bits<T>(tprev.z) : Num<T>::template absent<RULE>();
  uint32_t tprev_w = tprev.w;
  T H[R], Hp[R];
#pragma unroll
  for (int sr = 0; sr < R; ++sr) H[sr] = Hp[sr] = Hinit[sr];
  // Inputs of the current chunk and of the next one, in two register sets used in turn.
  u4 cA[R][4], tA[4], cB[R][4], tB[4];
  wait_until<false>([&] { return ld_ctl(&L.c_ready) >= 1u; }, lds, a);
  CBAR();
  read_c<R>(0, cq, cA);
  CtlSnap snap;
  snap_ctl<CONS>(L, C, snap);
  read_t<R>(0, L8(L.tring), tA);  // after the snapshot, as in every chunk
  chunk_gate<R, CONS>(0, NCc, lds, L, C, snap, tA, a, lane, chunk_trace(crec, 0));
#define WF_CHUNK_M(KIND, KK, CUR_C, CUR_T, NXT_C, NXT_T, MORE)                                                 \
  compute_chunk<T, RULE, R, KIND, CONS, MASK, LOCAL>(KK, G, gT, NCc, lds, L, C, hand_out, cq, hq, ct_base, hrd,      \
                                                    prog_at, lane63, lane, CUR_C, CUR_T, NXT_C, NXT_T, tprev_w, H, Hp, \
                                                    Np, snap, a, crec, MORE)
#define WF_CHUNK(KIND, KK, CUR_C, CUR_T, NXT_C, NXT_T) \
  WF_CHUNK_M(KIND, KK, CUR_C, CUR_T, NXT_C, NXT_T, (KK) + 1 < NCc)
  int k = 0;
  // The first 4 R chunks (groups 0 .. 16 R - 1, where rows left of column 0 are masked;
  // a walk always has at least that many).
  for (; k < 4 * R; k += 2) {
    WF_CHUNK(0, k, cA, tA, cB, tB);
    WF_CHUNK(0, k + 1, cB, tB, cA, tA);
  }
  // Every later chunk, an even number per pass so the register sets alternate without
  // copies (k stays even, so a last odd chunk uses set A): two per pass until k is a
  // multiple of 8, then eight per pass with k written as 8 j, so that each chunk's c and
  // H ring slots ((k + i) mod 8) are compile-time constants and their LDS addresses
  // become instruction offsets; two per pass for the rest.
  static_assert(C_SLOTS == 8 && H_SLOTS == 8, "eight chunks per pass cover each ring once");
  for (; (k & 7) != 0 && k + 1 < NCc; k += 2) {
    WF_CHUNK(1, k, cA, tA, cB, tB);
    WF_CHUNK(1, k + 1, cB, tB, cA, tA);
  }
  if ((k & 7) == 0) {
    int j = k >> 3;
    for (; 8 * j + 7 < NCc; ++j) {
      const int kb = 8 * j;
      // Chunks kb .. kb + 6 always have a successor (kb + 7 < NCc).
      WF_CHUNK_M(1, kb, cA, tA, cB, tB, true);
      WF_CHUNK_M(1, kb + 1, cB, tB, cA, tA, true);
      WF_CHUNK_M(1, kb + 2, cA, tA, cB, tB, true);
      WF_CHUNK_M(1, kb + 3, cB, tB, cA, tA, true);
      WF_CHUNK_M(1, kb + 4, cA, tA, cB, tB, true);
      WF_CHUNK_M(1, kb + 5, cB, tB, cA, tA, true);
      WF_CHUNK_M(1, kb + 6, cA, tA, cB, tB, true);
      WF_CHUNK(1, kb + 7, cB, tB, cA, tA);
    }
    k = 8 * j;
  }
  for (; k + 1 < NCc; k += 2) {
    WF_CHUNK(1, k, cA, tA, cB, tB);
    WF_CHUNK(1, k + 1, cB, tB, cA, tA);
  }
  if (k < NCc) WF_CHUNK(1, k, cA, tA, cB, tB);
#undef WF_CHUNK
#undef WF_CHUNK_M
  const int t_pad = t_pad_end(G, R);
  if (CONS == 1) {
    // The consumer's last chunks read T positions [16 NCc, t_pad), past every group of
    // this walk: fill them with absent values once its ring has room.
    wait_until<false>([&] { return (int)ld_ctl(&C->t_reset) + RING_T >= t_pad; }, lds, a);
    CBAR();
    const int p = CHUNK * NCc + 4 * lane;
    if (p < t_pad) lds_st4(L8(C->tring) + (p & (RING_T - 1)) * 4, absent4<T, RULE>());
  }
  CBAR();
  if (lane == 0) {
    st_ctl(&L.progress, (uint32_t)(4 * G));
    // Every T position this walk reads has been consumed: release the producer's tail.
    st_ctl(&L.t_reset, (uint32_t)t_pad);
    // The consumer's ring holds every position it reads, padding included.
    if (CONS == 1) st_ctl(&C->t_fed, (uint32_t)t_pad);
  }
}

template <typename T, int RULE, int W, int R>
__device__ __forceinline__ void compute_band(const GridDesc& g, int band, WaveLds* lds, WaveRings<R>* rings, int w,
                                             int lane, const KArgs& a, uint64_t* crec, bool hand_local) {
  WaveLds& L = lds[w];
  const int64_t m = g.m, n = g.n;
  const int64_t row0 = (int64_t)band * (64 * R * W) + 64 * R * w;
  if (row0 >= m) return;
  // The walk is the critical path: let it win the compute unit's shared units (LDS,
  // scalar and instruction issue) over the staging waves.
  __builtin_amdgcn_s_setprio(3);
  const int G = (int)groups_for(n, R);
  const int gT = n >= 2 ? (int)((n - 2) / 4 + 1) : 0;
  const bool lds_consumer = (w + 1 < W && row0 + 64 * R < m);
  // (The fault hook drops one band's handoff: its consumer then waits until the watchdog fires.)
  const bool glob_consumer = (w == W - 1) && (band + 1 < g.nbands) && a.fault_band != (uint32_t)band + 1u;
  if (a.trace && lane == 0) {
    L.tr_start = __builtin_readcyclecounter();
    L.tr_wall = wall_clock64();
  }
  T H[R];
#pragma unroll
  for (int sr = 0; sr < R; ++sr) {
    const int64_t row = row0 + R * lane + sr;
    H[sr] = Num<T>::template absent<RULE>();
    if (g.left && row < m) H[sr] = GC<T>(g.left)[row];
  }
  const lds_u8* cq[4];
  lds_u8* hq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    cq[q] = L8(rings[w].cring) + quad_off(lane, q);
    hq[q] = L8(rings[w].hring) + quad_off(lane, q);
  }
  // Lanes 60..62: the bottom row's quad lane - 60 in H ring slot 0 (the handoff gather).
  const lds_u8* hrd = L8(rings[w].hring) + quad_off(63, lane >= 60 && lane < 63 ? lane - 60 : 0) + (R - 1) * SLAB;
  // Cells left of column 0 need no per-cell selection when they stay at the absent
  // value by themselves (see compute_chunk): floating point, default left boundary, and
  // no row padding (the inputs read for them are then the finite tail of the row above).
  const bool unmasked = !std::is_integral<T>::value && g.left == nullptr && g.ld_cost == n;
  if (lds_consumer) {
    compute_walk<T, RULE, R, 1, true, false>(G, gT, lds, L, &lds[w + 1], __amdgpu_buffer_rsrc_t(), cq, hq, hrd, lane, H, a,
                                             crec);
  } else if (glob_consumer) {
    __amdgpu_buffer_rsrc_t hand_out = make_rsrc(g.hand + (int64_t)band * g.hand_ld, (uint32_t)(g.hand_ld * 4));
    // A consumer on this XCD polls through the shared L2, which a plain store reaches;
    // one on another XCD needs the handoff stores to go through to memory.
    if (unmasked) {
      if (hand_local) compute_walk<T, RULE, R, 2, false, true>(G, gT, lds, L, nullptr, hand_out, cq, hq, hrd, lane, H, a, crec);
      else compute_walk<T, RULE, R, 2, false, false>(G, gT, lds, L, nullptr, hand_out, cq, hq, hrd, lane, H, a, crec);
    } else {
      if (hand_local) compute_walk<T, RULE, R, 2, true, true>(G, gT, lds, L, nullptr, hand_out, cq, hq, hrd, lane, H, a, crec);
      else compute_walk<T, RULE, R, 2, true, false>(G, gT, lds, L, nullptr, hand_out, cq, hq, hrd, lane, H, a, crec);
    }
  } else {
    if (unmasked)
      compute_walk<T, RULE, R, 0, false, false>(G, gT, lds, L, nullptr, __amdgpu_buffer_rsrc_t(), cq, hq, hrd, lane, H, a,
                                                crec);
    else
      compute_walk<T, RULE, R, 0, true, false>(G, gT, lds, L, nullptr, __amdgpu_buffer_rsrc_t(), cq, hq, hrd, lane, H, a,
                                               crec);
  }
  if (a.trace && lane == 0) L.tr_end = __builtin_readcyclecounter();
}

// ------------------------------------------------------------- IO waves
// The staging work of compute wave w is split over waves that never mix load
// and store traffic: on gfx9 the vector-memory counter does not return loads
// and stores in order with respect to each other, so a wave holding both must
// drain everything before it can use any loaded value.
//   loader w : LDS-DMA loads of c, up to C_SLOTS - 1 chunks ahead -> c ring
//   storer w : H stage-out and handoff-row re-arming (stores only)
//   feeder   : the T ring of compute wave 0, from the top boundary or from the
//              band above (loads only)

__device__ __forceinline__ uint32_t pick(const u4& v, int e) {
  return e <= 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}

struct BandGeom {
  int64_t m, n, row0;
  int G, NC, T_END;
};

template <int W, int R>
__device__ __forceinline__ BandGeom band_geom(const GridDesc& g, int band, int w) {
  BandGeom b;
  b.m = g.m;
  b.n = g.n;
  b.row0 = (int64_t)band * (64 * R * W) + 64 * R * w;
  b.G = (int)groups_for(g.n, R);
  b.NC = (4 * b.G + CHUNK - 1) / CHUNK;
  b.T_END = 4 * b.G;
  return b;
}

// ------------------------------------------------------------- loader
// Chunk k of c for the 64 R rows of a strip goes straight from memory into c-ring
// slot k % C_SLOTS with LDS-DMA loads (buffer_load_dwordx4 ... lds): load (s, i)
// covers lane rows 16i .. 16i+15 of slab s, lane L reading grid row
// rho = R (16i + L/4) + s at positions 16k + 4q .. +3, q = (L%4) ^ swz(16i + L/4),
// i.e. columns col .. col+3 with col = 16k + 4q - rho.  The hardware writes lane L's
// 16 bytes at M0 + 16L, which is the slab layout.
//
// Offsets are taken from a buffer descriptor based at the strip's first row
// and ending at the grid's last element: quads left of a row's column 0 pick
// up the end of the row above, quads right of column n-1 the start of the row
// below (neither is ever used), and quads past the end of the grid are
// range-checked by the hardware (no access).  A quad that straddles the end of
// the grid and still holds columns of the row is rewritten with element loads.
//
// The loads are issued from inline assembly and waited for with explicit
// vmcnt values: the loader issues nothing else on that counter while DMA loads
// are in flight, and the compiler, which cannot see these loads, inserts no
// waits of its own for them.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void dma_quad16(__amdgpu_buffer_rsrc_t rsrc, uint32_t voff, uint32_t lds_addr) {
  // M0 holds the LDS destination; nothing else in this kernel uses M0.
  asm volatile("s_mov_b32 m0, %2\n\tbuffer_load_dwordx4 %0, %1, 0 offen lds"
               :: "v"(voff), "s"(rsrc), "s"(lds_addr) : "memory", "m0");
}
#pragma clang diagnostic pop

// Wait until at most `younger` chunks of 4 R DMA loads each are outstanding.
template <int R>
__device__ __forceinline__ void wait_dma(int younger) {
  switch (4 * R * younger) {
    case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
    case 4: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
    case 8: asm volatile("s_waitcnt vmcnt(8)" ::: "memory"); break;
    case 12: asm volatile("s_waitcnt vmcnt(12)" ::: "memory"); break;
    case 16: asm volatile("s_waitcnt vmcnt(16)" ::: "memory"); break;
    case 20: asm volatile("s_waitcnt vmcnt(20)" ::: "memory"); break;
    case 24: asm volatile("s_waitcnt vmcnt(24)" ::: "memory"); break;
    case 28: asm volatile("s_waitcnt vmcnt(28)" ::: "memory"); break;
    case 32: asm volatile("s_waitcnt vmcnt(32)" ::: "memory"); break;
    case 36: asm volatile("s_waitcnt vmcnt(36)" ::: "memory"); break;
    case 40: asm volatile("s_waitcnt vmcnt(40)" ::: "memory"); break;
    case 44: asm volatile("s_waitcnt vmcnt(44)" ::: "memory"); break;
    case 48: asm volatile("s_waitcnt vmcnt(48)" ::: "memory"); break;
    case 52: asm volatile("s_waitcnt vmcnt(52)" ::: "memory"); break;
    case 56: asm volatile("s_waitcnt vmcnt(56)" ::: "memory"); break;
    default: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
  }
}
static_assert(C_SLOTS <= 8, "wait_dma covers at most 7 younger chunks of 8 loads");

template <int R>
struct LoaderLanes {
  int64_t rel[R][4];  // element offset of (row, column 16k' + 4q - row) for k' = 0, from the strip base
  int rho[R][4];      // row inside the strip (not clamped)
  bool real[R][4];    // the row exists
};

// Idle step of a polling IO wave: sleep, then check abort and the watchdog.
// Only waves that may load from memory (DEVICE_FLAG) poll the device-wide flag;
// the others watch the workgroup flag, which those relay.
template <bool DEVICE_FLAG, class WL>
__device__ __forceinline__ bool io_idle(WL* lds, const KArgs& a, Watch& w, uint32_t& polls) {
  __builtin_amdgcn_s_sleep(1);
  if (ld_ctl(&lds[0].abort)) return false;
  if (DEVICE_FLAG && (++polls & 255u) == 0u && ld_dev(a.ctl + CTL_ABORT)) {
    st_ctl(&lds[0].abort, 1u);
    return false;
  }
  if (w.tick(a.watchdog_ticks)) {
    raise_abort(lds, a);
    return false;
  }
  return true;
}

// Logical quad a loader or storer lane moves: lane L covers physical quad L%4 of lane
// row 16i + L/4, whose swizzle is ((L/4) >> 1) & 3 whatever i.
__device__ __forceinline__ int io_quad(int lane) { return (lane & 3) ^ ((lane >> 3) & 3); }

// Loader of a dynamic-time-warping band (GridDesc::kind 1, fp32): the inputs of chunk
// k are computed rather than loaded.  Lane L covers the same (row, quad) cells as the
// grid loader and writes |x[row] - y[col]| for its four columns into the same slot
// position; x[row] stays in registers for the whole band, and a column outside [0, n)
// reads y as 0 (those cells are never used).  Only the m + n sequence values are read
// from memory.
template <int W, int R>
__device__ __forceinline__ void absdiff_loader_band(const GridDesc& g, const BandGeom& B, WaveLds& L,
                                                    unsigned char* cring, WaveLds* lds, int lane, const KArgs& a) {
  const int lq = io_quad(lane);
  float xv[R][4];
  int rho[R][4];
#pragma unroll
  for (int s = 0; s < R; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      rho[s][i] = R * (16 * i + (lane >> 2)) + s;
      const int64_t row = B.row0 + rho[s][i];
      xv[s][i] = row < B.m ? GC<float>(g.sx)[row] : 0.0f;
    }
  const __attribute__((address_space(1))) float* ys = GC<float>(g.sy);
  Watch t_idle;
  uint32_t polls = 0;
  bool ok = true;
  // The slot last held chunk k - C_SLOTS: wait until the compute wave is past it.
  auto slot_free = [&](int k) {
    while (ok && (int)ld_ctl(&L.progress) < 16 * (k - C_SLOTS + 1))
      ok = io_idle<false>(lds, a, t_idle, polls);
    if (ok) t_idle.reset();
    return ok;
  };
  auto write_slot = [&](int k, const u4 (&yq)[R][4]) {
    lds_u8* slot = L8(cring) + (k % C_SLOTS) * (R * SLAB);
#pragma unroll
    for (int s = 0; s < R; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const u4 y = yq[s][i];
        const uint32_t yv[4] = {y.x, y.y, y.z, y.w};
        uint32_t dv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float d = xv[s][i] - __builtin_bit_cast(float, yv[e]);  // one fp32 rounding
          dv[e] = bits(__builtin_fabsf(d));                              // exact
        }
        lds_st4(slot + SLAB * s + 1024 * i + 16 * lane, u4{dv[0], dv[1], dv[2], dv[3]});
      }
    // LDS accesses of one wave complete in order: a wave that sees the new count reads
    // the chunk written before it.
    CBAR();
    if (lane == 0) st_ctl(&L.c_ready, (uint32_t)(k + 1));
  };
  // Chunks with a quad reaching left of column 0 or right of column n - 1: element loads,
  // columns outside [0, n) read as 0 (those cells are never used).
  auto edge_chunk = [&](int k) {
    if (!slot_free(k)) return;
    u4 yq[R][4];
#pragma unroll
    for (int s = 0; s < R; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int col = 16 * k + 4 * lq - rho[s][i];
        uint32_t y4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int cc = col + e;
          const bool in = cc >= 0 && cc < B.n;
          y4[e] = in ? bits(ys[in ? cc : 0]) : 0u;
        }
        yq[s][i] = u4{y4[0], y4[1], y4[2], y4[3]};
      }
    write_slot(k, yq);
  };
  // Chunks [k_lo, k_hi) have every lane's quads inside [0, n): 16-byte loads through
  // registers, LOAD_DEPTH chunks in flight, in a straight-line loop (so the compiler's
  // waits count exactly the younger loads; loads past k_hi use an out-of-range offset,
  // read zeros and are never used).
  const int k_lo = (64 * R - 1 + 15) / 16;
  const int k_hi = B.n >= 16 ? (int)((B.n - 16) / 16 + 1 < B.NC ? (B.n - 16) / 16 + 1 : B.NC) : 0;
  int k = 0;
  for (; k < B.NC && k < k_lo && ok; ++k) edge_chunk(k);
  if (k_hi > k_lo && ok) {
    const __amdgpu_buffer_rsrc_t ry = make_rsrc(g.sy, (uint32_t)(B.n * 4));
    constexpr int LOAD_DEPTH = 4;
    u4 buf[LOAD_DEPTH][R][4];
    auto issue = [&](int kk, u4 (&b)[R][4]) {
#pragma unroll
      for (int s = 0; s < R; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int col = 16 * kk + 4 * lq - rho[s][i];
          b[s][i] = __builtin_amdgcn_raw_buffer_load_b128(ry, kk < k_hi ? (uint32_t)(col * 4) : 0xFFFFFFFFu, 0, 0);
        }
    };
#pragma unroll
    for (int j = 0; j < LOAD_DEPTH; ++j) issue(k_lo + j, buf[j]);
    for (int k0 = k_lo; k0 < k_hi && ok; k0 += LOAD_DEPTH) {
#pragma unroll
      for (int j = 0; j < LOAD_DEPTH; ++j) {
        const int kk = k0 + j;
        if (kk < k_hi && slot_free(kk)) write_slot(kk, buf[j]);
        issue(kk + LOAD_DEPTH, buf[j]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): no load still landing in registers
    k = k_hi;
  }
  for (; k < B.NC && ok; ++k) edge_chunk(k);
}

template <int W, int R>
__device__ __forceinline__ void loader_band(const GridDesc& g, int band, WaveLds* lds, WaveRings<R>* rings, int w,
                                            int lane, const KArgs& a, uint32_t item) {
  const BandGeom B = band_geom<W, R>(g, band, w);
  if (B.row0 >= B.m) return;
  if (g.kind == 1) {
    absdiff_loader_band<W, R>(g, B, lds[w], rings[w].cring, lds, lane, a);
    return;
  }
  WaveLds& L = lds[w];
  unsigned char* cring = rings[w].cring;
  // Elements from the strip's first row to the end of the grid.
  const int64_t span = (B.m - 1 - B.row0) * g.ld_cost + B.n;
  const uint32_t span_bytes = (uint32_t)(span * 4 < 0xFFFFFFF0ll ? span * 4 : 0xFFFFFFF0ll);
  const __amdgpu_buffer_rsrc_t rsrc = make_rsrc((const uint32_t*)g.cost + B.row0 * g.ld_cost, span_bytes);
  const int64_t last_rho = B.m - 1 - B.row0;
  const int lq = io_quad(lane);
  LoaderLanes<R> ln;
#pragma unroll
  for (int s = 0; s < R; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rho = R * (16 * i + (lane >> 2)) + s;
      const int64_t rr = rho < last_rho ? rho : last_rho;
      ln.rho[s][i] = rho;
      ln.real[s][i] = rho <= last_rho;
      ln.rel[s][i] = rr * g.ld_cost + 4 * lq - rho;
    }
  const uint32_t slot0 = (uint32_t)(uintptr_t)L8(cring);
  const int NC = B.NC;
  // Chunks [0, k_clean) of a full strip have every lane's quads inside the grid: they
  // are issued from precomputed byte offsets (chunk k adds 64k) with no per-lane checks
  // and need no fix-up.  The largest offset of chunk k is that of row 64 R - 1, quad 3.
  int k_clean = 0;
  if (B.row0 + 64 * R - 1 <= B.m - 1) {
    const int64_t max_rel = (int64_t)(64 * R - 1) * g.ld_cost + 12 - (64 * R - 1);
    const int64_t room = span - 4 - max_rel;
    if (room >= 0) k_clean = (int)(room / 16 + 1 < NC ? room / 16 + 1 : NC);
  }
  // With row padding (ld_cost > n), quads right of column n-1 would pick up the padding,
  // which may hold any bit pattern (even the handoff sentinel, once it has gone through
  // the cell rule).  From the first chunk where row 0's last quad reaches column n on,
  // such quads are replaced by zeros (the fix-up path below).
  const bool padded = g.ld_cost > B.n;
  if (padded) {
    const int k_pad = B.n >= 16 ? (int)((B.n - 16) / 16 + 1) : 0;  // first k with 16k + 15 >= n
    if (k_clean > k_pad) k_clean = k_pad;
  }
  uint32_t voff0[R][4];
#pragma unroll
  for (int s = 0; s < R; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) voff0[s][i] = (uint32_t)(ln.rel[s][i] * 4);  // used only for clean chunks
  int issued = 0, committed = 0;
  Watch t_idle;
  uint32_t polls = 0;
  // Clean chunks go through registers: LOAD_DEPTH chunks' loads in flight, each chunk
  // written into its c slot with ordinary LDS stores once it has landed and the slot
  // is free.  (Loads that write LDS directly, buffer_load ... lds, take the LDS away
  // from the compute wave whenever their data arrives; ordinary stores are arbitrated
  // like any wave's, and the compute wave's raised priority wins.)  The loop is straight
  // line, so the compiler's waits for the loads count exactly the younger ones: loads
  // past the clean chunks are issued at an out-of-range offset (they read zeros and are
  // never used) rather than skipped.
  if (k_clean > 0) {
    constexpr int LOAD_DEPTH = 4;
    u4 buf[LOAD_DEPTH][R][4];
    auto issue = [&](int k, u4 (&b)[R][4]) {
      const bool in = k < k_clean;
#pragma unroll
      for (int s = 0; s < R; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          b[s][i] = __builtin_amdgcn_raw_buffer_load_b128(rsrc, in ? voff0[s][i] + 64u * (uint32_t)k : 0xFFFFFFFFu, 0, 0);
    };
#pragma unroll
    for (int j = 0; j < LOAD_DEPTH; ++j) issue(j, buf[j]);
    bool ok = true;
    for (int k0 = 0; k0 < k_clean && ok; k0 += LOAD_DEPTH) {
#pragma unroll
      for (int j = 0; j < LOAD_DEPTH; ++j) {
        const int k = k0 + j;
        // The slot last held chunk k - C_SLOTS: wait until the compute wave is past it.
        if (ok && k < k_clean && (int)ld_ctl(&L.progress) < 16 * (k - C_SLOTS + 1)) {
          const uint64_t c0 = a.trace ? __builtin_readcyclecounter() : 0;
          while ((int)ld_ctl(&L.progress) < 16 * (k - C_SLOTS + 1))
            if (!(ok = io_idle<false>(lds, a, t_idle, polls))) break;
          if (a.trace && lane == 0) L.tr_load_wait += __builtin_readcyclecounter() - c0;
        }
        if (ok && k < k_clean) {
          t_idle.reset();
          lds_u8* slot = L8(cring) + (k % C_SLOTS) * (R * SLAB);
#pragma unroll
          for (int s = 0; s < R; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i) lds_st4(slot + SLAB * s + 1024 * i + 16 * lane, buf[j][s][i]);
          // LDS accesses of one wave complete in order: a wave that sees the new count
          // reads the chunk written before it.
          CBAR();
          if (lane == 0) st_ctl(&L.c_ready, (uint32_t)(k + 1));
        }
        issue(k + LOAD_DEPTH, buf[j]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): the DMA path below counts only its own loads
    if (!ok) return;
    issued = committed = k_clean;
  }
  // The remaining chunks (those holding the grid's end) are loaded straight into the c
  // ring (buffer_load ... lds), with the fix-ups below.
  for (;;) {
    // Issue every chunk whose slot the compute wave has released: slot k % C_SLOTS
    // last held chunk k - C_SLOTS, read completely once progress >= 16 (k - C_SLOTS + 1).
    while (issued < NC && (int)ld_ctl(&L.progress) >= 16 * (issued - C_SLOTS + 1)) {
      const uint32_t base = __builtin_amdgcn_readfirstlane(slot0 + (uint32_t)((issued % C_SLOTS) * (R * SLAB)));
      if (glb_u64* r = chunk_rec(a, item, W, w, issued))
        if (lane == 0) r[4] = wall_clock64();
      if (issued < k_clean) {
#pragma unroll
        for (int s = 0; s < R; ++s)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            dma_quad16(rsrc, voff0[s][i] + 64u * (uint32_t)issued, base + (uint32_t)(SLAB * s + 1024 * i));
      } else {
#pragma unroll
        for (int s = 0; s < R; ++s)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int64_t e = ln.rel[s][i] + 16 * issued;  // element offset from the strip base
            // Quads not wholly inside [strip base, end of grid) are not loaded at all (an
            // out-of-range offset): rows past the end of a ragged strip and the grid's tail.
            const uint32_t voff = (e < 0 || e + 4 > span) ? 0xFFFFFFFFu : (uint32_t)(e * 4);
            dma_quad16(rsrc, voff, base + (uint32_t)(SLAB * s + 1024 * i));
          }
      }
      ++issued;
    }
    if (committed < issued) {
      const int k = committed;
      wait_dma<R>(issued - committed - 1);
      if (glb_u64* r = chunk_rec(a, item, W, w, k))
        if (lane == 0) r[5] = wall_clock64();
      if (k < k_clean) {
        CBAR();
        if (lane == 0) st_ctl(&L.c_ready, (uint32_t)(k + 1));
        ++committed;
        t_idle.reset();
        continue;
      }
      // Quads that straddle the end of the grid and hold columns of a real row.
      bool fix[R][4];
      bool any = false;
#pragma unroll
      for (int s = 0; s < R; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t col = 16 * k + 4 * lq - ln.rho[s][i];
          const int64_t e = ln.rel[s][i] + 16 * k;
          fix[s][i] = ln.real[s][i] && col + 3 >= 0 &&
                      ((e + 4 > span && col <= B.n - 1) || (padded && col + 3 > B.n - 1));
          any |= fix[s][i];
        }
      if (__builtin_amdgcn_ballot_w64(any)) {
        typedef __attribute__((address_space(1))) const uint32_t g32;
        const g32* cbase = (const g32*)(const void*)((const uint32_t*)g.cost + B.row0 * g.ld_cost);
#pragma unroll
        for (int s = 0; s < R; ++s)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (!fix[s][i]) continue;
            const int64_t col = 16 * k + 4 * lq - ln.rho[s][i];
            u4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e)
              v[e] = (col + e >= 0 && col + e <= B.n - 1) ? cbase[(int64_t)ln.rho[s][i] * g.ld_cost + col + e] : 0u;
            lds_st4(L8(cring) + (k % C_SLOTS) * (R * SLAB) + SLAB * s + 1024 * i + 16 * lane, v);
          }
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
      }
      CBAR();
      if (lane == 0) st_ctl(&L.c_ready, (uint32_t)(k + 1));
      ++committed;
      t_idle.reset();
      continue;
    }
    if (committed == NC) break;
    const uint64_t c0 = a.trace ? __builtin_readcyclecounter() : 0;
    bool ok = true;
    while ((int)ld_ctl(&L.progress) < 16 * (issued - C_SLOTS + 1)) {
      if (!(ok = io_idle<false>(lds, a, t_idle, polls))) break;
    }
    if (a.trace && lane == 0) L.tr_load_wait += __builtin_readcyclecounter() - c0;
    if (!ok) break;
  }
  wait_dma<R>(0);  // nothing may still be writing the ring when the band ends
}

// Store chunk k of H (64 R rows x 16 positions) from the H ring: in slab s, lane L
// covers lane row r = 16i + L/4 (grid row rho = R r + s), logical quad q = io_quad(L),
// positions 16k + 4q .. +3 (contiguous LDS reads, and four consecutive lanes store one
// row's 64 contiguous bytes).
// Interior chunks (every quad inside the columns, none holding column n-1) take the
// fast path: full strips store their quads unconditionally (`qbase[s][i]` points at
// the lane's quad of chunk 0, column 4q - rho); the strip holding the last row
// skips the rows past it and copies that row's quads to last_row as well.
template <int R>
__device__ __forceinline__ bool store_interior(const BandGeom& B, int k) {
  return k >= 4 * R && 16 * (int64_t)k + 16 < B.n;
}

template <int R, bool LAST_STRIP>
__device__ __forceinline__ void store_chunk_fast(const GridDesc& g, const BandGeom& B, const unsigned char* hring,
                                                 int k, int lane, glb_u32* const (&qbase)[R][4]) {
  u4 v[R][4];
#pragma unroll
  for (int s = 0; s < R; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      v[s][i] = lds_ld4(L8(hring) + (k % H_SLOTS) * (R * SLAB) + SLAB * s + 1024 * i + 16 * lane);
  const bool full = g.mode == 0;
  const int lq = io_quad(lane);
#pragma unroll
  for (int s = 0; s < R; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (!LAST_STRIP) {
        if (full) *(glb_u4a4*)(qbase[s][i] + 16 * k) = v[s][i];
      } else {
        const int rho = R * (16 * i + (lane >> 2)) + s;
        const int64_t row = B.row0 + rho;
        if (row < B.m && full) *(glb_u4a4*)(qbase[s][i] + 16 * k) = v[s][i];
        if (row == B.m - 1 && g.last_row)
          *(glb_u4a4*)(G32((uint32_t*)g.last_row) + 16 * (int64_t)k + 4 * lq - rho) = v[s][i];
      }
    }
}

template <int R>
__device__ __forceinline__ void store_chunk(const GridDesc& g, const BandGeom& B, const unsigned char* hring, int k,
                                            int lane) {
  u4 v[R][4];
#pragma unroll
  for (int s = 0; s < R; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      v[s][i] = lds_ld4(L8(hring) + (k % H_SLOTS) * (R * SLAB) + SLAB * s + 1024 * i + 16 * lane);
  const bool full = g.mode == 0;
  const int lq = io_quad(lane);
#pragma unroll
  for (int s = 0; s < R; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rho = R * (16 * i + (lane >> 2)) + s;
      const int64_t row = B.row0 + rho;
      const int64_t col = 16 * k + 4 * lq - rho;
      if (row >= B.m || col > B.n - 1 || col + 3 < 0) continue;
      const u4 x = v[s][i];
      if (full) {
        glb_u32* op = G32((uint32_t*)g.out + row * g.ld_out);
        if (col >= 0 && col + 3 <= B.n - 1) {
          *(glb_u4a4*)(op + col) = x;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (col + e >= 0 && col + e <= B.n - 1) op[col + e] = pick(x, e);
        }
      }
      const bool has_last = col <= B.n - 1 && col + 3 >= B.n - 1;
      if (has_last && g.last_col) G32((uint32_t*)g.last_col)[row] = pick(x, (int)(B.n - 1 - col));
      if (row == B.m - 1) {
        if (g.last_row) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (col + e >= 0 && col + e <= B.n - 1) G32((uint32_t*)g.last_row)[col + e] = pick(x, e);
        }
        if (has_last && g.final_cell) *G32((uint32_t*)g.final_cell) = pick(x, (int)(B.n - 1 - col));
      }
    }
}

// Storer s serves compute wave s.
template <typename T, int W, int R>
__device__ __forceinline__ void storer_band(const GridDesc& g, int band, WaveLds* lds, WaveRings<R>* rings, int s,
                                            int lane, const KArgs& a, uint32_t item) {
  const uint32_t SENT = Num<T>::SENT;
  const BandGeom B = band_geom<W, R>(g, band, s);
  const bool active = B.row0 < B.m;
  WaveLds& L = lds[s];
  const unsigned char* hring = rings[s].hring;
  int ks = 0;
  glb_u32* qbase[R][4];
  const int lq = io_quad(lane);
#pragma unroll
  for (int sr = 0; sr < R; ++sr)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rho = R * (16 * i + (lane >> 2)) + sr;
      // Only dereferenced on the fast path, where the strip is full and the quad interior.
      qbase[sr][i] = G32((uint32_t*)g.out) + (B.row0 + rho) * g.ld_out + 4 * lq - rho;
    }
  // Handoff-row re-arming: only the storer of compute wave 0, only below band 0.
  const bool rearm_hand = s == 0 && band > 0;
  __amdgpu_buffer_rsrc_t hand_in =
      make_rsrc(g.hand + (band > 0 ? (int64_t)(band - 1) * g.hand_ld : 0), (uint32_t)(g.hand_ld * 4));
  int hr = t_first(R);
  const int hand_end = B.T_END;
  const bool full_strip = B.row0 + 64 * R < B.m;
  Watch t_idle;
  uint32_t polls = 0;
  for (;;) {
    bool did = false, done = true;
    if (active) {
      // Store every chunk the compute wave has finished (progress >= 16 (k+1), or the
      // end of the walk), then release their H slots at once.
      const int prog = (int)ld_ctl(&L.progress);
      CBAR();
      const int k0 = ks;
      while (ks < B.NC && prog >= (16 * (ks + 1) < B.T_END ? 16 * (ks + 1) : B.T_END)) {
        if (glb_u64* r = chunk_rec(a, item, W, s, ks))
          if (lane == 0) r[6] = wall_clock64();
        if (!store_interior<R>(B, ks)) store_chunk<R>(g, B, hring, ks, lane);
        else if (full_strip) store_chunk_fast<R, false>(g, B, hring, ks, lane, qbase);
        else store_chunk_fast<R, true>(g, B, hring, ks, lane, qbase);
        ++ks;
      }
      if (ks > k0) {
        __builtin_amdgcn_s_waitcnt(0xc07f);  // the ring reads are done before the slots are released
        CBAR();
        if (lane == 0) st_ctl(&L.h_done, (uint32_t)(16 * ks));
        if (a.ctrace && lane == 0) {
          const uint64_t now = wall_clock64();
          for (int kk = k0; kk < ks; ++kk)
            if (glb_u64* r = chunk_rec(a, item, W, s, kk)) r[7] = now;
        }
        did = true;
      }
      if (ks < B.NC) done = false;
    }
    if (rearm_hand) {
      int fed = (int)ld_ctl(&lds[0].t_fed);
      if (fed > hand_end) fed = hand_end;  // positions past the handoff row are padding
      if (fed > hr) {
        const int nq = (fed - hr) / 4;
        for (int base = 0; base < nq; base += 64) {
          if (base + lane < nq) {
            const int p = hr + 4 * (base + lane);
            u4 s4 = {SENT, SENT, SENT, SENT};
            // Device-coherent like every other access to the handoff rows: a plain store
            // could linger in this XCD's L2 and reach memory after the next launch's data.
            __builtin_amdgcn_raw_buffer_store_b128(s4, hand_in, p * 4, 0, CPOL_SC1);
          }
        }
        hr = fed;
        did = true;
      }
      if (hr < hand_end) done = false;
    }
    if (done) break;
    if (did) {
      t_idle.reset();
      continue;
    }
    if (!io_idle<false>(lds, a, t_idle, polls)) return;
  }
}

// Feed the T ring of compute wave 0 (positions t_first(R) .. T_END) from the top
// boundary (band 0) or from the handoff row of the band above, then pad it with
// absent values up to t_pad_end(G, R), the last position the walk's chunks check.
//
// The handoff row is polled with two loads in flight, issued about half a round
// trip apart, so new quads are seen about half a round trip sooner than with one.
// A poll covers the next SMALL quads while the producer is ahead of it by less than
// that (the usual case); when a poll comes back wholly valid the producer is far
// ahead and the next poll covers up to 64 quads.
template <typename T, int RULE, int W, int R>
__device__ __forceinline__ void feeder_band(const GridDesc& g, int band, WaveLds* lds, int lane, const KArgs& a,
                                            uint32_t item) {
  const uint32_t SENT = Num<T>::SENT;
  const BandGeom B = band_geom<W, R>(g, band, 0);
  WaveLds& L = lds[0];
  int tw = t_first(R);
  Watch t_idle;
  uint32_t polls = 0;
  const int t_pad = t_pad_end(B.G, R);
  // Trace: the time each sampled chunk's T positions were all in the ring.
  int next_s = 0;
  auto note_fed = [&] {
    if (!a.ctrace || lane != 0) return;
    while (next_s < a.ctrace_nc && tw >= CHUNK * CTRACE_EVERY * next_s + 64 * R + CHUNK) {
      chunk_rec(a, item, W, 0, CTRACE_EVERY * next_s)[8] = wall_clock64();
      ++next_s;
    }
  };
  if (band == 0) {
    while (tw < t_pad) {
      int limit = (int)ld_ctl(&L.t_reset) + RING_T;
      if (limit > t_pad) limit = t_pad;
      CBAR();
      if (tw < limit) {
        const int nq = (limit - tw) / 4;
        const int p = tw + 4 * lane;
        if (lane < nq) {
          u4 v;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t ti = (int64_t)p + e - (64 * R - 2);  // index into top[] (= column + 1)
            T val = Num<T>::template absent<RULE>();
            if (ti >= 0 && ti <= B.n) {
              if (g.top) val = GC<T>(g.top)[ti];
              else if (ti == 0) val = (T)0;
            }
            v[e] = bits(val);
          }
          lds_st4(L8(L.tring) + (p & (RING_T - 1)) * 4, v);
        }
        tw += 4 * (nq < 64 ? nq : 64);
        note_fed();
        __builtin_amdgcn_s_waitcnt(0xc07f);
        CBAR();
        if (lane == 0) st_ctl(&L.t_fed, (uint32_t)tw);
        t_idle.reset();
        continue;
      }
      if (!io_idle<true>(lds, a, t_idle, polls)) return;
    }
    return;
  }
  constexpr int SMALL = 8;
  const __amdgpu_buffer_rsrc_t hand_in = make_rsrc(g.hand + (int64_t)(band - 1) * g.hand_ld, (uint32_t)(g.hand_ld * 4));
  int want = SMALL;
  // Poll: quads [base, base + 4 nq) of the handoff row (nq = 0: nothing issued).
  // How far the ring has room (t_reset + RING_T, at most t_pad), re-read from LDS only when
  // a poll would reach past the last value read: the ring is rarely that full, and a
  // poll issued behind an LDS read waits for it.
  int limit = t_first(R) + RING_T < t_pad ? t_first(R) + RING_T : t_pad;
  auto issue = [&](u4& v, int& base, int& nq) {
    if (tw + 4 * want > limit && limit < t_pad) {
      limit = (int)ld_ctl(&L.t_reset) + RING_T;
      if (limit > t_pad) limit = t_pad;
    }
    base = tw;
    nq = (limit - tw) / 4;
    if (nq > want) nq = want;
    if (nq < 0) nq = 0;
    // Every lane issues the load (lanes past nq or past the handoff row at an
    // out-of-range offset, which reads zeros without touching memory), so no branch
    // separates the two polls and the wait before a poll is used counts only the loads
    // issued after it.
    const int p = base + 4 * lane;
    const uint32_t off = lane < nq && p < B.T_END ? (uint32_t)(p * 4) : 0x80000000u;
    v = __builtin_amdgcn_raw_buffer_load_b128(hand_in, off, 0, CPOL_SC1);
    // Keep the other poll's checks below this load (else waiting for them would also
    // wait for this load).
    __builtin_amdgcn_sched_barrier(0);
  };
  // Take the leading run of valid quads at positions >= tw from a returned poll.
  auto consume = [&](u4& v, int base, int nq) -> int {
    const int off = (tw - base) / 4;  // quads of this poll already taken from the other one
    const bool pad = base + 4 * lane >= B.T_END;
    if (pad) v = absent4<T, RULE>();
    const bool valid = lane >= off && lane < nq && (pad || (v.x != SENT && v.y != SENT && v.z != SENT && v.w != SENT));
    const uint64_t m = __builtin_amdgcn_ballot_w64(valid) >> (off < 64 ? off : 63);
    if (off >= nq) return 0;
    // ~m is 0 only when all 64 lanes of the poll are valid (off = 0, nq = 64).
    const int nvalid = ~m == 0ull ? 64 : (int)__builtin_ctzll(~m);
    if (nvalid == 0) {
      want = SMALL;
      return 0;
    }
    if (lane >= off && lane < off + nvalid) lds_st4(L8(L.tring) + ((base + 4 * lane) & (RING_T - 1)) * 4, v);
    tw += 4 * nvalid;
    note_fed();
    want = nvalid == nq - off ? 64 : SMALL;
    // LDS accesses of one wave complete in order: a wave that sees the new count reads
    // the quads written before it.
    CBAR();
    if (lane == 0) st_ctl(&L.t_fed, (uint32_t)tw);
    return nvalid;
  };
  u4 vA, vB;
  int bA, nA, bB, nB;
  issue(vA, bA, nA);
  __builtin_amdgcn_s_sleep(8);
  for (;;) {
    issue(vB, bB, nB);
    int got = consume(vA, bA, nA);
    if (tw >= t_pad) break;
    issue(vA, bA, nA);
    got += consume(vB, bB, nB);
    if (tw >= t_pad) break;
    if (got) {
      t_idle.reset();
    } else if (!io_idle<true>(lds, a, t_idle, polls)) {
      break;
    }
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // no poll still landing in registers at exit
}

// ------------------------------------------------------------------ kernel
// One storer per compute wave: at full speed a compute wave finishes a chunk about as
// fast as one wave can issue that chunk's H stores while every strip is storing.
constexpr int storers_for(int W) { return W; }
constexpr int waves_for(int W) { return 2 * W + storers_for(W) + 1; }

// Wave index -> role.  A workgroup's waves are dealt over the four SIMDs of its compute
// unit in turn, so waves i and i + 4 share a SIMD.  A compute wave's walk is one
// dependent chain: a busy wave on the same SIMD lengthens every step, so the compute
// waves get the quietest places: alone at W = 1; at W = 2 one alone and one beside the
// feeder, while the loaders pair up and so do the storers.
enum RoleKind { R_COMPUTE = 0, R_LOADER = 1, R_STORER = 2, R_FEEDER = 3 };
struct Role {
  int kind, strip;
};
template <int W>
__device__ __forceinline__ Role role_of(int wave) {
  if constexpr (W == 1) {
    constexpr int kinds[4] = {R_COMPUTE, R_LOADER, R_STORER, R_FEEDER};
    return Role{kinds[wave & 3], 0};
  } else {
    static_assert(W == 2, "roles are laid out for one or two compute waves");
    switch (wave) {
      case 0: return Role{R_COMPUTE, 1};
      case 1: return Role{R_LOADER, 0};
      case 2: return Role{R_STORER, 0};
      case 3: return Role{R_COMPUTE, 0};
      case 4: return Role{R_FEEDER, 0};
      case 5: return Role{R_LOADER, 1};
      default: return Role{R_STORER, 1};
    }
  }
}

// Two waves per SIMD at most (the LDS rings allow two workgroups of one compute wave of
// one row per lane per compute unit, or one of two such waves or of one wave of two rows
// per lane), so up to 256 VGPRs each.  TR: the launch records traces; without it every
// trace branch is compiled out of the walk.
template <typename T, int RULE, int W, int R, bool TR>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * waves_for(W), 64 * waves_for(W)),
                          amdgpu_waves_per_eu(R == 2 ? 1 : 2, R == 2 ? 1 : 2)))
void wf_sweep_kernel(KArgs a_in) {
  KArgs a = a_in;
  if (!TR) {
    a.trace = nullptr;
    a.ctrace = nullptr;
    a.ctrace_nc = 0;
  }
  __shared__ WaveLds lds[W];
  __shared__ WaveRings<R> rings[W];
  __shared__ uint32_t s_item;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const Role role = role_of<W>(__builtin_amdgcn_readfirstlane(wave));
  const uint32_t nx = a.nx > 1 ? (uint32_t)a.nx : 1u, seg = a.seg > 0 ? (uint32_t)a.seg : 1u;
  // The queue of the XCD this workgroup runs on: every workgroup of a queue shares one L2.
  const uint32_t xq = nx > 1 ? xcc_id() % nx : 0u;
  for (;;) {
    if (threadIdx.x == 0) {
      uint32_t t;
      if (nx > 1) {
        const uint32_t q = atomicAdd(&a.ctl[CTL_QUEUE + xq], 1u);
        t = ((q / seg) * nx + xq) * seg + q % seg;
      } else {
        t = atomicAdd(&a.ctl[CTL_TICKET], 1u);
      }
      if (ld_dev(a.ctl + CTL_ABORT)) t = 0xFFFFFFFFu;
      s_item = t;
    }
    // Re-arm this workgroup's LDS state for the next band.
    if (role.kind == R_COMPUTE) {
      WaveLds& L = lds[role.strip];
      const uint32_t SENT = Num<T>::SENT;
      for (int i = lane; i < RING_T; i += 64) L.tring[i] = SENT;
      if (lane == 0) {
        L.c_ready = 0;
        L.h_done = 0;
        // -16: nothing computed and no T quad validated yet.  The compute wave publishes 0
        // only after it has validated the first quad (positions 60..63), so the storer
        // cannot re-arm, and the feeder cannot refill, that slot before it has been read.
        L.progress = (uint32_t)-16;
        L.t_reset = t_first(R);
        L.t_fed = t_first(R);
        L.abort = 0;
        L.tr_start = L.tr_first = L.tr_end = L.tr_wall = 0;
        L.tr_chunk_wait = L.tr_t_wait = L.tr_load_wait = 0;
      }
    }
    __syncthreads();
    const uint32_t t = __builtin_amdgcn_readfirstlane(s_item);
    if ((int64_t)t >= a.nitems) break;
    GridDesc gd;
    int band;
    if (a.grids) {
      const Item it = a.items[t];
      gd = a.grids[it.grid];
      band = (int)it.band;
    } else {
      gd = a.g0;
      band = (int)t;
    }
    if (role.kind == R_COMPUTE) {
      uint64_t* crec = a.ctrace ? a.ctrace + ((int64_t)t * W + role.strip) * a.ctrace_nc * CTRACE_WORDS : nullptr;
      // The next band (ticket t + 1 of a single grid) runs on this XCD when both tickets
      // fall in queue xq.
      const bool hand_local = nx > 1 && ((t + 1u) / seg) % nx == xq;
      compute_band<T, RULE, W, R>(gd, band, lds, rings, role.strip, lane, a, crec, hand_local);
    }
    else if (role.kind == R_LOADER) loader_band<W, R>(gd, band, lds, rings, role.strip, lane, a, t);
    else if (role.kind == R_STORER) storer_band<T, W, R>(gd, band, lds, rings, role.strip, lane, a, t);
    else feeder_band<T, RULE, W, R>(gd, band, lds, lane, a, t);
    __syncthreads();
    if (a.trace && role.kind == R_COMPUTE && lane == 0) {
      const WaveLds& L = lds[role.strip];
      uint64_t* r = a.trace + ((uint64_t)t * W + role.strip) * TRACE_WORDS;
      r[0] = ((uint64_t)(a.grids ? a.items[t].grid : 0) << 32) | ((uint64_t)band << 8) | (uint64_t)role.strip;
      r[1] = L.tr_start;
      r[2] = L.tr_first;
      r[3] = L.tr_end;
      r[4] = L.tr_chunk_wait;
      r[5] = L.tr_t_wait;
      r[6] = L.tr_load_wait;
      r[7] = L.tr_wall;
    }
  }
}

__global__ void xcc_probe_kernel(uint32_t* out) {
  if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

// Arm the handoff rows of every grid of a launch's descriptor table with the sentinel:
// grid g's (nbands - 1) rows of hand_ld words (blockIdx.y strides over the grids).
__global__ void arm_hand_kernel(const GridDesc* grids, int ngrids, uint32_t sent) {
  for (int gi = blockIdx.y; gi < ngrids; gi += gridDim.y) {
    uint32_t* hand = grids[gi].hand;
    const int64_t count = (int64_t)(grids[gi].nbands - 1) * grids[gi].hand_ld;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) hand[i] = sent;
  }
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

// ======================================================================= fp64
// The fp64 sweep: bands of 64 rows, one compute wave per workgroup (lane r owns row r),
// and the same four roles as the 4-byte kernel.  A chunk of 16 positions of one row is
// 128 bytes: two slab rows of 64 bytes (slab h holds positions 8h .. 8h + 7, a quad two
// positions), so a chunk slot is two slabs and the loader and storer move 16 bytes per
// lane as before.
//
// Top-boundary and handoff positions travel encoded in 16 bytes each: the high word,
// the low word's upper and lower 16 bits, the high word again.  Every word of a written
// position then differs from the all-ones sentinel (a high word of all ones is a NaN,
// which neither an input nor a sum of finite inputs and infinities produces), so a
// reader checks each 32-bit word on its own: an access that races a write may see any
// mix of old and new words, and the position is taken only when all four are new.
// The bottom row is handed on by the storer, which reads it from the H ring after
// storing a chunk, so the walk issues no memory instructions at all.
constexpr int RT64 = 128;       // positions of the fp64 T ring (16 bytes each)
constexpr int H64_SLOTS = 4;    // chunk slots of the fp64 H ring

__device__ __forceinline__ u4 enc64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t hi = (uint32_t)(b >> 32), lo = (uint32_t)b;
  return u4{hi, lo >> 16, lo & 0xFFFFu, hi};
}
__device__ __forceinline__ double dec64(const u4& q) {
  return __builtin_bit_cast(double, ((uint64_t)q.x << 32) | (uint64_t)((q.y << 16) | q.z));
}
// SENT_F32 iff some word of the position is still the sentinel.
__device__ __forceinline__ uint32_t probe_pos(const u4& q) {
  const uint32_t a = q.x > q.y ? q.x : q.y, b = q.z > q.w ? q.z : q.w;
  return a > b ? a : b;
}
template <int RULE> __device__ __forceinline__ double absent64() {
  return RULE == 0 ? __builtin_inf() : -__builtin_inf();
}
template <int RULE> __device__ __forceinline__ double op3_64(double a, double b, double c) {
  if constexpr (RULE == 0) return __builtin_fmin(__builtin_fmin(a, b), c);
  else return __builtin_fmax(__builtin_fmax(a, b), c);
}
// N for every lane: lane r receives lane r-1's `src`; lane 0 keeps `old`.
__device__ __forceinline__ double dpp_shr1_64(double old, double src) {
  const uint64_t o = __builtin_bit_cast(uint64_t, old), s = __builtin_bit_cast(uint64_t, src);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)s, 0x138, 0xf, 0xf, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(s >> 32), 0x138, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

struct alignas(16) WaveLds64 {
  u4 tring[RT64];     // encoded T positions
  uint32_t c_ready;   // chunks of c committed to the c ring (loader -> compute)
  uint32_t h_done;    // positions of H stored out of the H ring (storer -> compute)
  uint32_t progress;  // (signed) position of the chunk being computed (compute -> IO)
  uint32_t t_reset;   // T positions below this are re-armed (compute -> feeder)
  uint32_t abort;     // workgroup abort flag
  uint32_t t_fed;     // T positions written by the feeder (feeder -> storer)
  uint32_t pad[2];
};
struct alignas(16) WaveRings64 {
  unsigned char cring[C_SLOTS * 2 * SLAB];
  unsigned char hring[H64_SLOTS * 2 * SLAB];
};

// LDS offset of row r's position p (0..15) of a chunk inside a slot.
__device__ __forceinline__ int pos_off64(int r, int p) { return (p >> 3) * SLAB + quad_off(r, (p & 7) >> 1) + 8 * (p & 1); }

// Chunk k of the walk (16 steps): wait for the c chunk, a free H slot and the 16 T
// positions the chunk needs, re-arm those T slots, then run the 16 steps.
template <int RULE, int KIND>
__device__ __forceinline__ void compute_chunk64(int k, int NC, WaveLds64& L, WaveLds64* lds, const lds_u8* cslot0,
                                                lds_u8* hslot0, int lane, double& H, double& Np, double& tprev,
                                                const KArgs& a) {
  const int pos = CHUNK * k;
  CBAR();
  if (lane == 0) st_ctl(&L.progress, (uint32_t)pos);
  const int need_h = pos + CHUNK - H64_SLOTS * CHUNK;
  wait_until<false>([&] { return (int)ld_ctl(&L.c_ready) >= k + 1 && (int)ld_ctl(&L.h_done) >= need_h; }, lds, a);
  CBAR();
  // T positions pos + 64 .. pos + 79: lane j < 16 holds position pos + 64 + j.
  const int tslot = (pos + 64 + (lane & 15)) & (RT64 - 1);
  u4 tq = lds_ld4_fresh(L8(&L.tring[tslot]));
  {
    uint64_t t0 = 0;
    uint32_t spins = 0;
    for (;;) {
      const bool bad = lane < 16 && probe_pos(tq) == SENT_F32;
      if (__builtin_amdgcn_ballot_w64(bad) == 0ull) break;
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 2047u) == 0u && (t0 = spin_check(lds, a.ctl, a.watchdog_ticks, t0)) == 0) break;
      tq = lds_ld4_fresh(L8(&L.tring[tslot]));
    }
  }
  const double tv = dec64(tq);  // lane j: position pos + 64 + j
  CBAR();
  // Re-arm the chunk's T slots (every lane holds its value in a register now).
  if (lane < 16) lds_st4(L8(&L.tring[tslot]), u4{SENT_F32, SENT_F32, SENT_F32, SENT_F32});
  __builtin_amdgcn_s_waitcnt(0xc07f);
  CBAR();
  if (lane == 0) st_ctl(&L.t_reset, (uint32_t)(pos + 80));
  const lds_u8* cs = cslot0 + (k % C_SLOTS) * (2 * SLAB);
  lds_u8* hs = hslot0 + (k % H64_SLOTS) * (2 * SLAB);
  double c[16];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const u4 v = lds_ld4(cs + h * SLAB + quad_off(lane, q));
      c[8 * h + 2 * q] = __builtin_bit_cast(double, ((uint64_t)v.y << 32) | v.x);
      c[8 * h + 2 * q + 1] = __builtin_bit_cast(double, ((uint64_t)v.w << 32) | v.z);
    }
  double hv[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    // Lane 0's N at step pos + s is the row above at column pos + s: position pos + s + 63.
    const double tn = s == 0 ? tprev : __builtin_bit_cast(double, (uint64_t)__builtin_amdgcn_readlane(
                                                                       (int)(__builtin_bit_cast(uint64_t, tv) >> 32), s - 1)
                                                                       << 32 |
                                                                   (uint32_t)__builtin_amdgcn_readlane(
                                                                       (int)(uint32_t)__builtin_bit_cast(uint64_t, tv), s - 1));
    const double N = dpp_shr1_64(tn, H);
    double Hn = c[s] + op3_64<RULE>(N, Np, H);
    if (KIND == 0) Hn = (pos + s < lane) ? H : Hn;  // rows left of column 0 keep the left boundary
    Np = N;
    H = Hn;
    hv[s] = H;
  }
  tprev = __builtin_bit_cast(double, (uint64_t)__builtin_amdgcn_readlane((int)(__builtin_bit_cast(uint64_t, tv) >> 32), 15)
                                         << 32 |
                                     (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)__builtin_bit_cast(uint64_t, tv), 15));
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint64_t x = __builtin_bit_cast(uint64_t, hv[8 * h + 2 * q]), y = __builtin_bit_cast(uint64_t, hv[8 * h + 2 * q + 1]);
      lds_st4(hs + h * SLAB + quad_off(lane, q), u4{(uint32_t)x, (uint32_t)(x >> 32), (uint32_t)y, (uint32_t)(y >> 32)});
    }
  (void)NC;
}

template <int RULE>
__device__ __forceinline__ void compute_band64(const GridDesc& g, int band, WaveLds64* lds, WaveRings64* rings, int lane,
                                               const KArgs& a) {
  WaveLds64& L = lds[0];
  const int64_t m = g.m, n = g.n, row0 = (int64_t)band * 64;
  if (row0 >= m) return;
  __builtin_amdgcn_s_setprio(3);
  const int G = (int)groups_for(n, 1);
  const int NC = (4 * G + CHUNK - 1) / CHUNK;
  double H = absent64<RULE>();
  if (g.left && row0 + lane < m) H = GC<double>(g.left)[row0 + lane];
  // First T positions: 62 (column -1, the corner: NW of step 0) and 63 (column 0).
  u4 q62 = lds_ld4_fresh(L8(&L.tring[62])), q63 = lds_ld4_fresh(L8(&L.tring[63]));
  {
    uint64_t t0 = 0;
    uint32_t spins = 0;
    while (__builtin_amdgcn_readfirstlane(probe_pos(q62) == SENT_F32 || probe_pos(q63) == SENT_F32 ? 1 : 0)) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 2047u) == 0u && (t0 = spin_check(lds, a.ctl, a.watchdog_ticks, t0)) == 0) break;
      q62 = lds_ld4_fresh(L8(&L.tring[62]));
      q63 = lds_ld4_fresh(L8(&L.tring[63]));
    }
  }
  double Np = dec64(q62), tprev = dec64(q63);
  CBAR();
  if (lane < 4) lds_st4(L8(&L.tring[60 + lane]), u4{SENT_F32, SENT_F32, SENT_F32, SENT_F32});
  __builtin_amdgcn_s_waitcnt(0xc07f);
  const lds_u8* cs = L8(rings->cring);
  lds_u8* hs = L8(rings->hring);
  int k = 0;
  for (; k < 4; ++k) compute_chunk64<RULE, 0>(k, NC, L, lds, cs, hs, lane, H, Np, tprev, a);
  for (; k < NC; ++k) compute_chunk64<RULE, 1>(k, NC, L, lds, cs, hs, lane, H, Np, tprev, a);
  CBAR();
  if (lane == 0) {
    st_ctl(&L.progress, (uint32_t)(4 * G));
    st_ctl(&L.t_reset, (uint32_t)t_pad_end(G, 1));
  }
}

// Loader: chunk k of the strip into c-ring slot k % C_SLOTS with LDS-DMA loads; load
// (h, i) covers lane rows 16i .. 16i+15 of slab h, lane L reading row r = 16i + L/4 at
// positions 16k + 8h + 2q, +1 with q = io_quad(L): columns col, col+1, col = that - r.
__device__ __forceinline__ void loader_band64(const GridDesc& g, int band, WaveLds64* lds, WaveRings64* rings, int lane,
                                              const KArgs& a) {
  const int64_t m = g.m, n = g.n, row0 = (int64_t)band * 64;
  if (row0 >= m) return;
  WaveLds64& L = lds[0];
  const int G = (int)groups_for(n, 1);
  const int NC = (4 * G + CHUNK - 1) / CHUNK;
  const int64_t span = (m - 1 - row0) * g.ld_cost + n;  // elements from the strip's first row to the grid's end
  const uint32_t span_bytes = (uint32_t)(span * 8 < 0xFFFFFFF0ll ? span * 8 : 0xFFFFFFF0ll);
  const __amdgpu_buffer_rsrc_t rsrc = make_rsrc((const double*)g.cost + row0 * g.ld_cost, span_bytes);
  const int64_t last_r = m - 1 - row0;
  const int lq = io_quad(lane);
  int64_t rel[2][4];
  int rr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    rr[i] = 16 * i + (lane >> 2);
    const int64_t rc = rr[i] < last_r ? rr[i] : last_r;
#pragma unroll
    for (int h = 0; h < 2; ++h) rel[h][i] = rc * g.ld_cost + 8 * h + 2 * lq - rr[i];
  }
  int k_clean = 0;
  if (row0 + 63 <= m - 1) {
    const int64_t max_rel = 63 * g.ld_cost + 14 - 63;
    const int64_t room = span - 2 - max_rel;
    if (room >= 0) k_clean = (int)(room / 16 + 1 < NC ? room / 16 + 1 : NC);
  }
  const bool padded = g.ld_cost > n;
  if (padded) {
    const int k_pad = n >= 16 ? (int)((n - 16) / 16 + 1) : 0;
    if (k_clean > k_pad) k_clean = k_pad;
  }
  const uint32_t slot0 = (uint32_t)(uintptr_t)L8(rings->cring);
  int issued = 0, committed = 0;
  Watch t_idle;
  uint32_t polls = 0;
  for (;;) {
    while (issued < NC && (int)ld_ctl(&L.progress) >= 16 * (issued - C_SLOTS + 1)) {
      const uint32_t base = __builtin_amdgcn_readfirstlane(slot0 + (uint32_t)((issued % C_SLOTS) * (2 * SLAB)));
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t e = rel[h][i] + 16 * issued;
          const uint32_t voff = (issued < k_clean) ? (uint32_t)(e * 8)
                                                   : ((e < 0 || e + 2 > span) ? 0xFFFFFFFFu : (uint32_t)(e * 8));
          dma_quad16(rsrc, voff, base + (uint32_t)(SLAB * h + 1024 * i));
        }
      ++issued;
    }
    if (committed < issued) {
      const int k = committed;
      wait_dma<2>(issued - committed - 1);
      if (k >= k_clean) {
        // Quads that straddle the end of the grid or reach into row padding: element loads
        // for the columns of the row, zeros past it.
        bool fix[2][4];
        bool any = false;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int64_t col = 16 * k + 8 * h + 2 * lq - rr[i];
            const int64_t e = rel[h][i] + 16 * k;
            fix[h][i] = rr[i] <= last_r && col + 1 >= 0 && ((e + 2 > span && col <= n - 1) || (padded && col + 1 > n - 1));
            any |= fix[h][i];
          }
        if (__builtin_amdgcn_ballot_w64(any)) {
          typedef __attribute__((address_space(1))) const uint64_t g64;
          const g64* cb = (const g64*)(const void*)((const double*)g.cost + row0 * g.ld_cost);
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              if (!fix[h][i]) continue;
              const int64_t col = 16 * k + 8 * h + 2 * lq - rr[i];
              const uint64_t x = (col >= 0 && col <= n - 1) ? cb[(int64_t)rr[i] * g.ld_cost + col] : 0ull;
              const uint64_t y = (col + 1 >= 0 && col + 1 <= n - 1) ? cb[(int64_t)rr[i] * g.ld_cost + col + 1] : 0ull;
              lds_st4(L8(rings->cring) + (k % C_SLOTS) * (2 * SLAB) + SLAB * h + 1024 * i + 16 * lane,
                      u4{(uint32_t)x, (uint32_t)(x >> 32), (uint32_t)y, (uint32_t)(y >> 32)});
            }
          __builtin_amdgcn_s_waitcnt(0xc07f);
        }
      }
      CBAR();
      if (lane == 0) st_ctl(&L.c_ready, (uint32_t)(k + 1));
      ++committed;
      t_idle.reset();
      continue;
    }
    if (committed == NC) break;
    bool ok = true;
    while ((int)ld_ctl(&L.progress) < 16 * (issued - C_SLOTS + 1))
      if (!(ok = io_idle<false>(lds, a, t_idle, polls))) break;
    if (!ok) break;
  }
  wait_dma<2>(0);
}

// Storer: chunk k of H from the H ring to memory (full mode) or to the edge outputs, the
// bottom row's positions of the chunk to the handoff row (encoded), then the slot is
// released; the storer also re-arms the band above's handoff positions behind the feeder.
__device__ __forceinline__ void storer_band64(const GridDesc& g, int band, WaveLds64* lds, WaveRings64* rings, int lane,
                                              const KArgs& a, bool hand_local) {
  const int64_t m = g.m, n = g.n, row0 = (int64_t)band * 64;
  if (row0 >= m) return;
  WaveLds64& L = lds[0];
  const int G = (int)groups_for(n, 1);
  const int NC = (4 * G + CHUNK - 1) / CHUNK, T_END = 4 * G;
  const int lq = io_quad(lane);
  const bool full = g.mode == 0;
  const bool handoff = band + 1 < g.nbands && a.fault_band != (uint32_t)band + 1u;
  const __amdgpu_buffer_rsrc_t hand_out = make_rsrc(g.hand + (int64_t)band * g.hand_ld * 4, (uint32_t)(g.hand_ld * 16));
  const __amdgpu_buffer_rsrc_t hand_in =
      make_rsrc(g.hand + (band > 0 ? (int64_t)(band - 1) * g.hand_ld * 4 : 0), (uint32_t)(g.hand_ld * 16));
  int ks = 0, hr = 60;
  Watch t_idle;
  uint32_t polls = 0;
  for (;;) {
    bool did = false;
    const int prog = (int)ld_ctl(&L.progress);
    CBAR();
    while (ks < NC && prog >= (16 * (ks + 1) < T_END ? 16 * (ks + 1) : T_END)) {
      const int k = ks;
      const lds_u8* hs = L8(rings->hring) + (k % H64_SLOTS) * (2 * SLAB);
      // A chunk whose cells all lie inside the grid and left of the last column needs no
      // bounds checks and touches no edge output but the last row: all eight quads are
      // read from the ring first, then written with one 16-byte store each (full mode),
      // and lanes 60..63 (row 63) write theirs to the last-row output when the band ends
      // the grid.
      const bool clean = k >= 4 && 16 * k + 15 <= n - 2 && row0 + 63 <= m - 1;
      const bool to_last_row = row0 + 63 == m - 1 && g.last_row;
      if (clean) {
        if (full || to_last_row) {
          u4 v[2][4];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) v[h][i] = lds_ld4(hs + SLAB * h + 1024 * i + 16 * lane);
          if (full) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int r = 16 * i + (lane >> 2);
              double* op = (double*)g.out + (row0 + r) * g.ld_out + (16 * k + 2 * lq - r);
#pragma unroll
              for (int h = 0; h < 2; ++h) *(glb_u4a4*)(op + 8 * h) = v[h][i];
            }
          }
          if (to_last_row && lane >= 60) {
#pragma unroll
            for (int h = 0; h < 2; ++h) *(glb_u4a4*)((double*)g.last_row + (16 * k + 8 * h + 2 * lq - 63)) = v[h][3];
          }
        }
      } else {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const u4 v = lds_ld4(hs + SLAB * h + 1024 * i + 16 * lane);
          const int r = 16 * i + (lane >> 2);
          const int64_t row = row0 + r;
          const int64_t col = 16 * k + 8 * h + 2 * lq - r;
          if (row >= m || col > n - 1 || col + 1 < 0) continue;
          const uint64_t x[2] = {((uint64_t)v.y << 32) | v.x, ((uint64_t)v.w << 32) | v.z};
          typedef __attribute__((address_space(1))) uint64_t g64;
          if (full) {
            g64* op = (g64*)(void*)((double*)g.out + row * g.ld_out);
            if (col >= 0 && col + 1 <= n - 1) {
              *(glb_u4a4*)(op + col) = v;
            } else {
#pragma unroll
              for (int e = 0; e < 2; ++e)
                if (col + e >= 0 && col + e <= n - 1) op[col + e] = x[e];
            }
          }
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            if (col + e < 0 || col + e > n - 1) continue;
            if (col + e == n - 1 && g.last_col) ((g64*)(void*)g.last_col)[row] = x[e];
            if (row == m - 1) {
              if (g.last_row) ((g64*)(void*)g.last_row)[col + e] = x[e];
              if (col + e == n - 1 && g.final_cell) *(g64*)(void*)g.final_cell = x[e];
            }
          }
        }
      }
      if (handoff) {
        // Positions 16k .. 16k + 15 of the bottom row (lane 63's row), the ones in [60, T_END).
        const int p = 16 * k + (lane & 15);
        if (lane < 16 && p >= 60 && p < T_END) {
          const uint64_t x = *(const __attribute__((address_space(3))) uint64_t*)(hs + pos_off64(63, lane));
          // Plain stores when the band below runs on this XCD (same L2), system-coherent
          // ones otherwise.
          if (hand_local) __builtin_amdgcn_raw_buffer_store_b128(enc64(__builtin_bit_cast(double, x)), hand_out, p * 16, 0, 0);
          else __builtin_amdgcn_raw_buffer_store_b128(enc64(__builtin_bit_cast(double, x)), hand_out, p * 16, 0, CPOL_SC1);
        }
      }
      ++ks;
      __builtin_amdgcn_s_waitcnt(0xc07f);  // the ring reads are done before the slot is released
      CBAR();
      if (lane == 0) st_ctl(&L.h_done, (uint32_t)(16 * ks));
      did = true;
    }
    if (band > 0) {
      int fed = (int)ld_ctl(&L.t_fed);
      if (fed > T_END) fed = T_END;
      if (fed > hr) {
        for (int p = hr + lane; p < fed; p += 64)
          __builtin_amdgcn_raw_buffer_store_b128(u4{SENT_F32, SENT_F32, SENT_F32, SENT_F32}, hand_in, p * 16, 0, CPOL_SC1);
        hr = fed;
        did = true;
      }
    }
    if (ks >= NC && (band == 0 || hr >= T_END)) break;
    if (did) {
      t_idle.reset();
      continue;
    }
    if (!io_idle<false>(lds, a, t_idle, polls)) return;
  }
}

// Feeder: T positions 60 .. T_END of the walk from the top boundary (band 0) or the
// band above's handoff row, then absent values up to t_pad_end(G, 1).
template <int RULE>
__device__ __forceinline__ void feeder_band64(const GridDesc& g, int band, WaveLds64* lds, int lane, const KArgs& a) {
  const int64_t m = g.m, n = g.n, row0 = (int64_t)band * 64;
  if (row0 >= m) return;
  WaveLds64& L = lds[0];
  const int G = (int)groups_for(n, 1);
  const int T_END = 4 * G, t_pad = t_pad_end(G, 1);
  const __amdgpu_buffer_rsrc_t hand_in =
      make_rsrc(g.hand + (band > 0 ? (int64_t)(band - 1) * g.hand_ld * 4 : 0), (uint32_t)(g.hand_ld * 16));
  int tw = 60;
  Watch t_idle;
  uint32_t polls = 0;
  while (tw < t_pad) {
    int limit = (int)ld_ctl(&L.t_reset) + RT64;
    if (limit > t_pad) limit = t_pad;
    CBAR();
    int got = 0;
    if (tw < limit) {
      const int nq = limit - tw < 64 ? limit - tw : 64;
      const int p = tw + lane;
      u4 v = u4{SENT_F32, SENT_F32, SENT_F32, SENT_F32};
      bool valid = false;
      if (lane < nq) {
        if (band == 0 || p >= T_END) {
          double val = absent64<RULE>();
          const int64_t ti = (int64_t)p - 62;  // index into top[] (= column + 1)
          if (band == 0 && ti >= 0 && ti <= n) {
            if (g.top) val = GC<double>(g.top)[ti];
            else if (ti == 0) val = 0.0;
          }
          v = enc64(val);
          valid = true;
        } else {
          v = __builtin_amdgcn_raw_buffer_load_b128(hand_in, p * 16, 0, CPOL_SC1);
          valid = probe_pos(v) != SENT_F32;
        }
      }
      const uint64_t bal = __builtin_amdgcn_ballot_w64(valid);
      got = ~bal == 0ull ? 64 : (int)__builtin_ctzll(~bal);
      if (got > nq) got = nq;
      if (lane < got) lds_st4(L8(&L.tring[p & (RT64 - 1)]), v);
      if (got) {
        tw += got;
        __builtin_amdgcn_s_waitcnt(0xc07f);
        CBAR();
        if (lane == 0) st_ctl(&L.t_fed, (uint32_t)tw);
      }
    }
    if (got) {
      t_idle.reset();
      continue;
    }
    if (!io_idle<true>(lds, a, t_idle, polls)) break;
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Waves: 0 compute, 1 loader, 2 storer, 3 feeder (one per SIMD).
template <int RULE>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(1, 1)))
void wf_sweep64_kernel(KArgs a) {
  __shared__ WaveLds64 lds[1];
  __shared__ WaveRings64 rings;
  __shared__ uint32_t s_item;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  // Per-XCD ticket queues as in the fp32 kernel (single-grid launches only).
  const uint32_t nx = a.nx > 1 ? (uint32_t)a.nx : 1u, seg = a.seg > 0 ? (uint32_t)a.seg : 1u;
  const uint32_t xq = nx > 1 ? xcc_id() % nx : 0u;
  for (;;) {
    if (threadIdx.x == 0) {
      uint32_t t;
      if (nx > 1) {
        const uint32_t q = atomicAdd(&a.ctl[CTL_QUEUE + xq], 1u);
        t = ((q / seg) * nx + xq) * seg + q % seg;
      } else {
        t = atomicAdd(&a.ctl[CTL_TICKET], 1u);
      }
      if (ld_dev(a.ctl + CTL_ABORT)) t = 0xFFFFFFFFu;
      s_item = t;
    }
    if (wave == 0) {
      WaveLds64& L = lds[0];
      for (int i = lane; i < RT64; i += 64) L.tring[i] = u4{SENT_F32, SENT_F32, SENT_F32, SENT_F32};
      if (lane == 0) {
        L.c_ready = 0;
        L.h_done = 0;
        L.progress = (uint32_t)-16;
        L.t_reset = 60;
        L.t_fed = 60;
        L.abort = 0;
      }
    }
    __syncthreads();
    const uint32_t t = __builtin_amdgcn_readfirstlane(s_item);
    if ((int64_t)t >= a.nitems) break;
    GridDesc gd;
    int band;
    if (a.grids) {
      const Item it = a.items[t];
      gd = a.grids[it.grid];
      band = (int)it.band;
    } else {
      gd = a.g0;
      band = (int)t;
    }
    if (wave == 0) compute_band64<RULE>(gd, band, lds, &rings, lane, a);
    else if (wave == 1) loader_band64(gd, band, lds, &rings, lane, a);
    else if (wave == 2) storer_band64(gd, band, lds, &rings, lane, a, nx > 1 && ((t + 1u) / seg) % nx == xq);
    else feeder_band64<RULE>(gd, band, lds, lane, a);
    __syncthreads();
  }
}

// Traceback of a computed grid: from (m-1, n-1), step to the predecessor whose value the
// rule selects, NW before N before W on equal values, until that predecessor lies
// outside the grid.  One wave.  Lane b holds in registers column j0 - 1 + b of the
// 64 x 64 block whose bottom-right cell is the walk's current cell: rows i0 - 1 ..
// i0 + 62, i.e. 63 x 63 cells of H plus the row above and the column left of them (from
// H, or the boundary).  Each lane turns its column into predecessor codes (0: NW, 1: N,
// 2: W) with one DPP shift per row for the left neighbour's values, packed two bits per
// row, 16 rows per register.  The walk runs on the scalar unit: one lane read per step
// from the register of the current 16 rows, and the step's code shifted into a 64-bit
// move record; every 31 steps the wave turns the record into (i, j) pairs with a prefix
// sum over lanes and writes them out.
constexpr int TB = 64;  // staged block side (63 cells + one boundary row / column)

template <typename T> __device__ __forceinline__ T shr1_any(T x) {
  if constexpr (sizeof(T) == 8) return dpp_shr1_64(x, x);
  else return dpp_shr1<T>(x, x);
}

template <typename T, int RULE>
__global__ void __launch_bounds__(64) traceback_kernel(const T* H, int64_t ld, int64_t m, int64_t n, const T* top,
                                                       const T* left, int32_t* path, int64_t* length) {
  const int lane = threadIdx.x;
  const T absent = Num<T>::template absent<RULE>();
  int ci = (int)(m - 1), cj = (int)(n - 1);  // the walk's current cell
  int64_t k = 0;                             // path entries written
  // Codes of the pending steps, newest in the low bits, above a marker bit: with n steps
  // pending the marker is bit 2n, so it reaches bit 62 at 31 steps.
  uint64_t mv = 1;
  int fi = ci, fj = cj;  // cell of the first pending step
  // Write the pending steps: step e visited (fi, fj) minus the moves of steps 0 .. e-1.
  auto flush = [&]() {
    const int nmv = (63 - __builtin_clzll(mv)) >> 1;
    const uint32_t c = lane < nmv ? (uint32_t)(mv >> (2 * (nmv - 1 - lane))) & 3u : 3u;
    const uint32_t d = lane < nmv ? ((1u - (c >> 1)) << 16) | (1u - (c & 1u)) : 0u;  // (rows, cols) moved
    // Inclusive prefix sum over lanes 0 .. 31 with DPP: within rows of 16, then row 0's
    // total into row 1.
    uint32_t inc = d;
    inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x111, 0xf, 0xf, true);  // row_shr:1
    inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x112, 0xf, 0xf, true);  // row_shr:2
    inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x114, 0xf, 0xf, true);  // row_shr:4
    inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x118, 0xf, 0xf, true);  // row_shr:8
    inc += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)inc, 0x142, 0xa, 0xf, false); // row_bcast:15
    const uint32_t ex = inc - d;
    if (lane < nmv) {
      path[2 * (k + lane)] = fi - (int)(ex >> 16);
      path[2 * (k + lane) + 1] = fj - (int)(ex & 0xffffu);
    }
    const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)inc, 31);
    fi -= (int)(tot >> 16);
    fj -= (int)(tot & 0xffffu);
    k += nmv;
    mv = 1;
  };
  for (;;) {
    const int i0 = ci - (TB - 2) > 0 ? ci - (TB - 2) : 0;
    const int j0 = cj - (TB - 2) > 0 ? cj - (TB - 2) : 0;
    // Lane b loads column j0 - 1 + b of rows i0 - 1 .. i0 + 62 (all loads in flight at once);
    // cells below or right of the current cell are never read and stay absent.
    const int64_t col = j0 - 1 + lane;
    T v[TB];
    if (i0 >= 1 && j0 >= 1) {  // inside the grid and 63 x 63 cells up-left of the current cell
      const T* p = H + (int64_t)(i0 - 1) * ld + col;
#pragma unroll
      for (int a = 0; a < TB; ++a) v[a] = p[a * ld];
    } else {
#pragma unroll
      for (int a = 0; a < TB; ++a) {
        const int64_t r = i0 - 1 + a;
        T x = absent;
        if (r <= ci && col <= cj) {
          if (r < 0) x = top ? top[col + 1] : (col == -1 ? (T)0 : absent);
          else if (col < 0) x = left ? left[r] : absent;
          else x = H[r * ld + col];
        }
        v[a] = x;
      }
    }
    uint32_t pk[4] = {0u, 0u, 0u, 0u};  // code of row a at bits 2 (a % 16) of pk[a / 16]
    T wp = shr1_any(v[0]);                // the left neighbour's value in the previous row
#pragma unroll
    for (int a = 1; a < TB; ++a) {
      const T ww = shr1_any(v[a]);
      const bool n_lt = RULE == 0 ? v[a - 1] < wp : v[a - 1] > wp;
      const T best = n_lt ? v[a - 1] : wp;
      const bool w_lt = RULE == 0 ? ww < best : ww > best;
      pk[a >> 4] |= (w_lt ? 2u : (n_lt ? 1u : 0u)) << (2 * (a & 15));
      wp = ww;
    }
    // Row r of the block is tracked as the bit-field operand of s_bfe_u32: offset 2 r
    // (the hardware takes it modulo 32, which is the field of row r in its register),
    // width 2.
    constexpr int BFE2 = 2 << 16;
    int fo = BFE2 + 2 * __builtin_amdgcn_readfirstlane(ci - i0 + 1);
    int b = __builtin_amdgcn_readfirstlane(cj - j0 + 1);
#pragma unroll
    for (int q = 3; q >= 0; --q) {
      const int lo = BFE2 + 2 * (q == 0 ? 1 : 16 * q);  // stay while row >= 16 q (>= 1)
      const int cur = (int)pk[q];
      auto step = [&]() {
        const uint32_t w = (uint32_t)__builtin_amdgcn_readlane(cur, b);
        uint32_t c;
        asm("s_bfe_u32 %0, %1, %2" : "=s"(c) : "s"(w), "s"(fo));
        mv = (mv << 2) | c;
        uint32_t top = (uint32_t)(mv >> 32);
        asm("" : "+s"(top));  // a 32-bit scalar compare, not a 64-bit vector one
        if (__builtin_expect(top >= (1u << 30), 0)) flush();
        fo -= 2 - (int)(c & 2u);  // NW and N step up a row
        b -= 1 - (int)(c & 1u);   // NW and W step left a column
      };
      // Two steps per pass: one taken branch per two steps (four measure the same).
      while (((fo - lo) | (b - 1)) >= 0) {
        step();
        if (((fo - lo) | (b - 1)) < 0) break;
        step();
      }
    }
    ci = i0 - 1 + ((fo - BFE2) >> 1);
    cj = j0 - 1 + b;
    if (ci < 0 || cj < 0) break;
  }
  flush();
  // The outside predecessor the walk ended on follows the visited cells.
  if (lane == 0) {
    path[2 * k] = ci;
    path[2 * k + 1] = cj;
    *length = k;
  }
}

// Set-up of an allocation-free launch: zero the control words (the error word only when
// asked: it accumulates across launches until the host has seen it) and arm `count`
// handoff-row words with the sentinel.
__global__ void noalloc_prep_kernel(uint32_t* ctl, uint32_t reset_error, uint32_t* hand, uint32_t sent,
                                    int64_t count) {
  if (blockIdx.x == 0 && threadIdx.x < CTL_WORDS && (threadIdx.x != CTL_ERROR || reset_error != 0u))
    ctl[threadIdx.x] = 0u;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) hand[i] = sent;
}

template <typename T, int RULE, int W, int R>
hipError_t launch_t(int nwg, const KArgs& args, hipStream_t stream) {
  if (args.trace || args.ctrace)
    hipLaunchKernelGGL((wf_sweep_kernel<T, RULE, W, R, true>), dim3(nwg), dim3(64 * waves_for(W)), 0, stream, args);
  else
    hipLaunchKernelGGL((wf_sweep_kernel<T, RULE, W, R, false>), dim3(nwg), dim3(64 * waves_for(W)), 0, stream, args);
  return hipGetLastError();
}

// Band shapes: W compute waves of R rows per lane (64 R W rows per band).
template <typename T, int RULE>
hipError_t launch_w(int W, int R, int nwg, const KArgs& args, hipStream_t stream) {
  if (W == 1 && R == 1) return launch_t<T, RULE, 1, 1>(nwg, args, stream);
  if (W == 2 && R == 1) return launch_t<T, RULE, 2, 1>(nwg, args, stream);
  if (W == 1 && R == 2) return launch_t<T, RULE, 1, 2>(nwg, args, stream);
  return hipErrorInvalidValue;
}

}  // namespace
}  // namespace wfk

// Fixed workspace of the allocation-free entry point: control words, then handoff rows.
// Each device that loads the library holds its own copy until the process ends.  Host
// code must never pass `scratch` itself to a kernel (in host code the name is a
// host-side stand-in, not a device address): it uses the address that
// noalloc_scratch() returns for the current device.
static __device__ __align__(256) uint32_t scratch[wfk::NOALLOC_WORDS];

namespace wfk {

hipError_t noalloc_scratch(uint32_t** ptr) {
  *ptr = nullptr;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess) *ptr = (uint32_t*)p;
  return e;
}

size_t lds_bytes(int W, int R) {
  return (sizeof(WaveLds) + (size_t)(C_SLOTS + H_SLOTS) * R * SLAB) * (size_t)W + 16;
}

hipError_t launch_sweep(int dtype, int rule, int W, int R, int nwg, const KArgs& args, hipStream_t stream) {
  if (dtype == 2) {
    if (W != 1 || R != 1) return hipErrorInvalidValue;
    if (rule == 0) hipLaunchKernelGGL((wf_sweep64_kernel<0>), dim3(nwg), dim3(256), 0, stream, args);
    else hipLaunchKernelGGL((wf_sweep64_kernel<1>), dim3(nwg), dim3(256), 0, stream, args);
    return hipGetLastError();
  }
  if (dtype == 0)
    return rule == 0 ? launch_w<float, 0>(W, R, nwg, args, stream) : launch_w<float, 1>(W, R, nwg, args, stream);
  if (dtype == 1)
    return rule == 0 ? launch_w<int32_t, 0>(W, R, nwg, args, stream) : launch_w<int32_t, 1>(W, R, nwg, args, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_noalloc_prep(uint32_t* ctl, bool reset_error, uint32_t* hand, uint32_t sent, int64_t count,
                               hipStream_t stream) {
  int64_t blocks = (count + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(noalloc_prep_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, ctl,
                     reset_error ? 1u : 0u, hand, sent, count);
  return hipGetLastError();
}

hipError_t launch_traceback(int dtype, int rule, const void* H, int64_t ld, int64_t m, int64_t n, const void* top,
                            const void* left, int32_t* path, int64_t* length, hipStream_t stream) {
#define WF_TB(T, RL)                                                                                           \
  hipLaunchKernelGGL((traceback_kernel<T, RL>), dim3(1), dim3(64), 0, stream, (const T*)H, ld, m, n, (const T*)top, \
                     (const T*)left, path, length)
  if (dtype == 0) {
    if (rule == 0) WF_TB(float, 0);
    else WF_TB(float, 1);
  } else if (dtype == 1) {
    if (rule == 0) WF_TB(int32_t, 0);
    else WF_TB(int32_t, 1);
  } else if (dtype == 2) {
    if (rule == 0) WF_TB(double, 0);
    else WF_TB(double, 1);
  } else {
    return hipErrorInvalidValue;
  }
#undef WF_TB
  return hipGetLastError();
}

hipError_t launch_xcc_probe(uint32_t* out, int nwg, hipStream_t stream) {
  if (nwg <= 0) return hipSuccess;
  hipLaunchKernelGGL(xcc_probe_kernel, dim3((unsigned)nwg), dim3(64), 0, stream, out);
  return hipGetLastError();
}

hipError_t launch_arm_hand(const GridDesc* grids, int ngrids, uint32_t sent, hipStream_t stream) {
  if (ngrids <= 0) return hipSuccess;
  const dim3 grid(16, (unsigned)(ngrids < 1024 ? ngrids : 1024));
  hipLaunchKernelGGL(arm_hand_kernel, grid, dim3(256), 0, stream, grids, ngrids, sent);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, value, count);
  return hipGetLastError();
}

}  // namespace wfk
