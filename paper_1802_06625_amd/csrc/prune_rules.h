// The integer rules of the model of computation, written once for the host
// and the device: Eq. 2 capacity, the Fig. 6 slot rule, the blocking rules,
// Eq. 1 decoding and the configuration actor's mapping.  Plain C++ apart from
// the __host__ __device__ qualifiers, so a host compiler (the sanitizer
// builds of the CPU checks) takes it as it is.
#pragma once

#include <stdint.h>

#include "prune.h"

#if defined(__HIPCC__)
#define PRUNE_HD __host__ __device__
#else
#define PRUNE_HD
#endif

namespace prune {

// ---------------------------------------------------------------- Eq. 2
PRUNE_HD inline uint64_t fifo_capacity(uint32_t r, uint32_t Q, uint32_t C) {
  return (Q % r) ? (uint64_t)r * C + Q
                 : ((uint64_t)r * C > Q ? (uint64_t)r * C : (uint64_t)Q);
}

// ---------------------------------------------------------------- Fig. 6 rule
// Aligned (Q mod r == 0): ring of max(rC, Q) slots in blocks of r, Q/r blocks
// prefilled; write j -> block (Q/r + j) mod blocks, read i -> block i mod blocks.
// Unaligned: ring of rC slots plus a Q-slot overflow area; write j at
// Q + (j mod C) r (copied back to slot 0 when it runs past rC-1), read i at
// (i mod C) r.
PRUNE_HD inline uint64_t fifo_write_slot(uint32_t r, uint32_t Q, uint32_t C,
                                                     uint64_t j) {
  if (Q % r == 0) {
    uint64_t blocks = fifo_capacity(r, Q, C) / r;
    return ((Q / r + j) % blocks) * r;
  }
  return Q + (j % C) * (uint64_t)r;
}

PRUNE_HD inline uint64_t fifo_read_slot(uint32_t r, uint32_t Q, uint32_t C,
                                                    uint64_t i) {
  if (Q % r == 0) {
    uint64_t blocks = fifo_capacity(r, Q, C) / r;
    return (i % blocks) * r;
  }
  return (i % C) * (uint64_t)r;
}

// Blocking rules in terms of blocks in flight (writes - reads).
PRUNE_HD inline bool fifo_can_write(uint32_t r, uint32_t Q, uint32_t C,
                                               int64_t inflight) {
  if (Q % r == 0) return (int64_t)(Q / r) + inflight < (int64_t)(fifo_capacity(r, Q, C) / r);
  return (inflight + 1) * (int64_t)r <= (int64_t)r * C - (int64_t)Q;
}

PRUNE_HD inline bool fifo_can_read(uint32_t r, uint32_t Q, uint32_t /*C*/,
                                              int64_t inflight) {
  if (Q % r == 0) return (int64_t)(Q / r) + inflight > 0;
  return (int64_t)Q + inflight * (int64_t)r >= (int64_t)r;
}

// ---------------------------------------------------------------- Eq. 1
// tokrate(p, phi) = BTOI(v_phi[T[j][p]]) * atr(p): the element's bit.
PRUNE_HD inline uint32_t decode_bit(uint32_t mask, uint32_t element) {
  return element ? (mask >> (element - 1)) & 1u : 0u;
}

// Configuration actor mapping: external side-information -> control token.
PRUNE_HD inline prune_ctrl_token config_map(uint32_t mode, uint32_t Kmax,
                                                       prune_side_info s) {
  prune_ctrl_token t;
  if (mode == PRUNE_CONFIG_ROUTE) {
    t.mask = s.route < 32 ? (1u << s.route) : 0u;
  } else if (mode == PRUNE_CONFIG_MASK) {
    const uint32_t bank_bits = Kmax >= 32 ? 0xffffffffu : ((1u << Kmax) - 1u);
    const uint32_t sh = s.bank * Kmax;
    t.mask = sh < 32 ? ((s.K & bank_bits) << sh) : 0u;
  } else {
    uint32_t K = s.K > 31 ? 31 : s.K;
    uint32_t m = K ? ((K >= 32) ? 0xffffffffu : ((1u << K) - 1u)) : 0u;
    uint32_t sh = s.bank * Kmax;
    t.mask = sh < 32 ? (m << sh) : 0u;
  }
  t.rate = s.n;
  return t;
}

// ---------------------------------------------------------------- invariants
// What every FIFO state reachable under the blocking rules satisfies: the
// occupancy (delay + tokens written - tokens read, in whole blocks here)
// never exceeds the Eq. 2 capacity and never goes below zero.  Checked by the
// bookkeeping kernels in PRUNE_DEBUG builds and by the host rule checks.
PRUNE_HD inline bool fifo_state_ok(uint32_t r, uint32_t Q, uint32_t C, int64_t inflight) {
  const int64_t occ = (int64_t)Q + inflight * (int64_t)r;
  return inflight >= -(int64_t)(Q / r) && occ >= 0 && (uint64_t)occ <= fifo_capacity(r, Q, C);
}

// The four counters a FIFO keeps (block accesses written and read, tokens
// written and read) after a bookkeeping update: the block state is one the
// blocking rules reach (fifo_state_ok), no access carries more than r
// tokens, and the token occupancy Q + tokens written - tokens read lies in
// [0, Eq. 2 capacity].
PRUNE_HD inline bool fifo_counters_ok(uint32_t r, uint32_t Q, uint32_t C, uint64_t writes, uint64_t reads,
                                      uint64_t tokens_written, uint64_t tokens_read) {
  if (!fifo_state_ok(r, Q, C, (int64_t)writes - (int64_t)reads)) return false;
  if (tokens_written > writes * r || tokens_read > reads * r) return false;
  if (tokens_read > (uint64_t)Q + tokens_written) return false;
  return (uint64_t)Q + tokens_written - tokens_read <= fifo_capacity(r, Q, C);
}

// One update of a counter pair (accesses, tokens) from (n0, t0) to (n1, t1):
// neither goes back, and the new accesses carry at most r tokens each.
PRUNE_HD inline bool fifo_advance_ok(uint32_t r, uint64_t n0, uint64_t t0, uint64_t n1, uint64_t t1) {
  return n1 >= n0 && t1 >= t0 && t1 - t0 <= (n1 - n0) * r;
}

}  // namespace prune
