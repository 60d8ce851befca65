// Compile-time analysis of a PRUNE graph: the design rules of Sec. IV and
// the dynamic processing graph (DPG) analysis of Sec. V.  Host code; the
// graph is given as plain structure (actors, external ports, FIFOs, control
// table) so that it runs on graphs that are not finalized and on hosts
// without a GPU.
#pragma once

#include <array>
#include <cstdint>
#include <map>
#include <utility>
#include <vector>

namespace prune {

struct DesignPort {
  uint32_t actor, dir, kind;          // PRUNE_IN/OUT, PRUNE_SRP/DRP/CPORT
  std::vector<uint32_t> fifos;
};

struct DesignFifo {
  uint32_t src, dst, rate, delay;     // src/dst are port ids
};

struct DesignGraph {
  std::vector<uint32_t> kind;                      // per actor
  std::vector<std::vector<uint32_t>> ports;        // external ports per actor, creation order
  std::vector<DesignPort> port;                    // every port id (internal ones unused)
  std::vector<DesignFifo> fifo;
  std::map<std::pair<uint32_t, uint32_t>, uint32_t> table;   // (control port, DRP) -> element
};

// Violation codes, as in include/prune.h (PRUNE_RULE_*).
enum : int64_t {
  kRule1 = 1, kRule2 = 2, kRule3Kind = 31, kRule3Shared = 32, kRule4 = 4, kRule5 = 5,
  kDpgA = 10, kDpgBDc = 11, kDpgBCount = 12, kDpgC = 13,
  kDeadlockDc = 20, kDeadlockTop = 21, kPairing = 40, kUnpaired = 41,
};

struct DesignReport {
  std::vector<std::array<int64_t, 2>> linked;       // linked DRP pairs, p < p2, sorted
  std::vector<std::array<int64_t, 4>> dpgs;         // q, x, y, control output port
  struct Dc {
    int64_t dpg, element, direct_fifo;              // direct_fifo: dummy actor's FIFO or -1
    std::vector<uint32_t> actors;                   // sorted
  };
  std::vector<Dc> dcs;
  std::vector<int64_t> dc_of_actor;                 // DC index or -1
  std::vector<int64_t> beta;                        // buffer bound per FIFO, -1 if none
  std::vector<std::array<int64_t, 3>> violations;   // sorted, unique
};

DesignReport analyze_design(const DesignGraph &g);

}  // namespace prune
