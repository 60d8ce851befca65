// Internal definitions of libprune_hip shared by the host runtime and the
// HIP kernels: device-resident FIFO/actor/port tables, per-firing records,
// filter-bank frame descriptors, and the integer rules of the model of
// computation written once as __host__ __device__ functions (Eq. 2 capacity,
// the Fig. 6 slot rule, Eq. 1 decoding, the configuration actor's mapping).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "prune.h"
#include "prune_rules.h"

namespace prune {

// Samples read and written through pointers taken from descriptors in
// memory: the compiler cannot tell that they address global memory and
// would emit generic (flat) accesses, which also count against the LDS wait
// counter, so that every wait for an LDS read would also wait for them (a
// prefetch of the next tile would then end before the current tile's
// arithmetic starts).  These helpers make them global-memory accesses.
__device__ __forceinline__ float2 ld_global(const float2 *p) {
  typedef __attribute__((address_space(1))) const unsigned long long gword;
  return __builtin_bit_cast(float2, *(const gword *)(const unsigned long long *)p);
}

__device__ __forceinline__ void st_global(float2 *p, float2 v) {
  typedef __attribute__((address_space(1))) unsigned long long gword;
  *(gword *)(unsigned long long *)p = __builtin_bit_cast(unsigned long long, v);
}

constexpr int kMaxPorts = PRUNE_MAX_PORTS;   // ports per actor, control port included
constexpr int kMaxFanout = 4;         // FIFOs per output port (broadcast)
constexpr int kMaxIO = PRUNE_MAX_IO;         // data FIFO accesses per firing
constexpr uint32_t kNone = 0xffffffffu;

// Device error word bits (reported by prune_graph_sync).
enum : uint32_t {
  kErrToken = 1u,      // control value beyond its declared size
  kErrRate = 2u,       // rate parameter outside 1..atr
  kErrCount = 4u,      // block count differs from the firing's rate
  kErrTrace = 8u,      // trace buffer overflow
  kErrInvariant = 16u, // a FIFO's counters broke an invariant (PRUNE_DEBUG builds)
};

// Checks of the bookkeeping kernels that only PRUNE_DEBUG builds compile:
// a failed one sets kErrInvariant in the device error word.
#if defined(PRUNE_DEBUG)
#define PRUNE_DEBUG_CHECK(cond, err) \
  do {                               \
    if (!(cond)) atomicOr((err), ::prune::kErrInvariant); \
  } while (0)
constexpr bool kDebugBuild = true;
#else
#define PRUNE_DEBUG_CHECK(cond, err) \
  do {                               \
  } while (0)
constexpr bool kDebugBuild = false;
#endif

// ---------------------------------------------------------------- device tables
struct FifoDev {
  char *base;              // storage: borrowed data FIFO or library-owned control FIFO
  uint32_t *counts;        // per-block token counts (blocks of r slots)
  uint32_t r, Q, C, blocks;
  uint32_t token_bytes, param, halo, aligned;
  uint64_t writes, reads, tokens_written, tokens_read, max_occ, pad;
};

struct PortDev {
  uint32_t actor, dir, kind, atr;
  uint32_t param, halo, element;   // element: control-table entry of a DRP
  uint32_t n_fifos;
  uint32_t power;                  // POLY output k: basis |x|^k x (0 elsewhere)
  uint32_t fifo[kMaxFanout];
};

struct ActorDev {
  uint32_t kind, n_ports, cport_fifo, n_elements;  // cport_fifo = kNone if static
  uint32_t port[kMaxPorts];                        // PortDev indices (cport excluded)
  uint32_t first_in;                               // PortDev index of the first data input
  uint32_t cfg_mode, cfg_Kmax;                     // CONFIG
  uint32_t fb;                                     // FbParamsDev index for FILTERBANK
  uint32_t fixed_mask;                             // static filter bank
  uint32_t pix_w, pix_h, pix_t;                    // GAUSS5 / THRES / MED5
  uint32_t hist_len;                               // stream history kept by the actor
  float2 *history;                                 // [hist_len] library-owned
  uint64_t firings;                                // device firing counter
  void *queue;                                     // SOURCE: SrcIn ring; CONFIG: side-info ring
  uint64_t q_head, q_cap;                          // next entry to consume, ring size
  float2 *sink_out;                                // SINK: optional bound output
  uint64_t sink_pos, sink_cap;
};

struct FbParamsDev {
  uint32_t n_banks, Kmax, Lmax, windowed;
  uint32_t L[PRUNE_MAX_BANKS];
  float2 *taps;           // [n_banks][Kmax][Lmax]
  uint64_t *branch_firings;  // [n_banks*Kmax]
  uint64_t *branch_tokens;
  uint32_t elem[PRUNE_MAX_BRANCHES];  // control-table element of each branch DRP
};

// One firing's resolved data accesses (output of the bookkeeping step).
struct IoRec {
  char *ptr;               // first slot of the access
  uint32_t count, fifo;
};

constexpr int kMaxIn = PRUNE_MAX_IN;   // data inputs per actor

struct FiringRec {
  uint32_t fired, firing, mask, rate;
  uint32_t bitmap, n_io, pad0, pad1;
  IoRec in[kMaxIn];        // data inputs in port order
  IoRec out[kMaxIO];       // every (output port, fifo) access in port order
  uint32_t out_port[kMaxIO];
};

// Filter-bank firing descriptor consumed by the forward kernels.
struct FbFrameDesc {
  const float2 *x;         // sample 0 of the frame
  const float2 *halo;      // sample -Hd (Hd = Lmax-1); halo[k] = sample k - Hd
  float2 *y[kMaxFanout];   // outputs (broadcast)
  const float2 *taps;      // [n_banks][Kmax][Lmax]
  uint32_t n, mask, halo_valid, n_y;
  uint32_t n_banks, Kmax, Lmax, route;  // route 1: passthrough copy
  uint32_t L[PRUNE_MAX_BANKS];
};

struct WorkItem {
  uint32_t frame, tile;
};

// Trace record as in prune.h.
struct TraceBuf {
  prune_trace_record *rec;
  uint64_t cap;
  unsigned long long *count;
};

}  // namespace prune
