// End of a per-firing run: the classification of a state in which no actor
// can fire, on a plain view of the graph's state (host code, no device
// types), so the executor and the host checks share it.
#pragma once

#include <cstdint>
#include <vector>

namespace prune {

struct StopFifo {
  uint32_t src_port, dst_port, rate, delay;
  int64_t inflight;              // blocks written and not yet read
};

struct StopPort {
  uint32_t actor, dir, kind;     // PRUNE_IN/OUT, PRUNE_SRP/DRP/CPORT
  uint32_t element;              // DRP: its control-table element (1-based, 0 none)
  std::vector<uint32_t> fifos;
};

struct StopActor {
  uint32_t kind;
  bool exhausted;                // source / configuration actor with no input left
  int64_t cport_fifo;            // -1: static
  bool has_token;                // a control token is waiting on the control port
  uint32_t token_mask;           // that token's mask
  uint64_t firings;
  std::vector<uint32_t> ports;   // external ports
};

struct StopResult {
  std::vector<uint32_t> stuck, linked;   // both empty: a normal end
};

StopResult classify_stop_view(const std::vector<StopActor> &actors, const std::vector<StopPort> &ports,
                              const std::vector<StopFifo> &fifos, uint32_t C);

}  // namespace prune
