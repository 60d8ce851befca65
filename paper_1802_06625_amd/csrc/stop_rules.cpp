// Classification of a stopped per-firing run (blocking reads and writes,
// Sec. III-A; linked DRPs, Sec. V).
//
// * Each actor that cannot fire waits on FIFOs: a blocking read on an input
//   holding less than a block (its writer must fire), a blocking write on an
//   output without room for one (its reader must fire).  A dynamic actor
//   without a control token waits on its control FIFO; with one, on the
//   FIFOs of the ports its token sets active (Eq. 1).
// * A source or configuration actor with no external input left is
//   exhausted.  An actor is starved when one of its waits has an exhausted or
//   starved actor at the FIFO's other end: it stopped because input ran out.
//   Every other actor is stuck: its waits only lead round a cycle, which no
//   further input can break.
// * A dynamic actor y that holds a token and waits to read an active DRP
//   input is followed upstream, through the read waits of the actors feeding
//   it, to the dynamic actor x whose DRP output starts the chain.  In a valid
//   DPG y's k-th firing lacks data from x only while x has not fired its k-th
//   (both counted from the first control token that is not a delay); if x
//   has, the two tokens set the linked DRPs differently (the deadlock of
//   Sec. V) and y is reported.
#include "stop_rules.h"

#include <algorithm>

#include "prune.h"
#include "prune_rules.h"

namespace prune {

namespace {
struct Wait {
  uint32_t fifo;
  bool read;
};
}  // namespace

StopResult classify_stop_view(const std::vector<StopActor> &actors, const std::vector<StopPort> &ports,
                              const std::vector<StopFifo> &fifos, uint32_t C) {
  const uint32_t na = (uint32_t)actors.size();
  std::vector<std::vector<Wait>> w(na);
  std::vector<char> starved(na, 0);
  for (uint32_t a = 0; a < na; ++a) {
    const StopActor &A = actors[a];
    if (A.exhausted) {
      starved[a] = 1;
      continue;
    }
    if (A.cport_fifo >= 0 && !A.has_token) {
      w[a].push_back({(uint32_t)A.cport_fifo, true});
      continue;
    }
    for (uint32_t p : A.ports) {
      const StopPort &P = ports[p];
      if (P.kind == PRUNE_CPORT) continue;
      if (P.kind == PRUNE_DRP && !(A.cport_fifo >= 0 && decode_bit(A.token_mask, P.element))) continue;
      for (uint32_t f : P.fifos) {
        const StopFifo &F = fifos[f];
        if (P.dir == PRUNE_IN) {
          if (!fifo_can_read(F.rate, F.delay, C, F.inflight)) w[a].push_back({f, true});
        } else if (!fifo_can_write(F.rate, F.delay, C, F.inflight)) {
          w[a].push_back({f, false});
        }
      }
    }
  }
  for (bool grown = true; grown;) {
    grown = false;
    for (uint32_t a = 0; a < na; ++a) {
      if (starved[a] || w[a].empty()) continue;
      for (const Wait &x : w[a]) {
        const StopFifo &F = fifos[x.fifo];
        if (starved[ports[x.read ? F.src_port : F.dst_port].actor]) {
          starved[a] = 1;
          grown = true;
          break;
        }
      }
    }
  }
  StopResult res;
  for (uint32_t a = 0; a < na; ++a)
    if (!starved[a]) res.stuck.push_back(a);
  auto token_index = [&](uint32_t a) {
    return (int64_t)actors[a].firings - (int64_t)fifos[actors[a].cport_fifo].delay;
  };
  std::vector<uint32_t> todo;
  std::vector<char> seen(na);
  for (uint32_t y = 0; y < na; ++y) {
    const StopActor &Y = actors[y];
    if (Y.cport_fifo < 0 || !Y.has_token || w[y].empty()) continue;
    todo.clear();
    std::fill(seen.begin(), seen.end(), 0);
    for (const Wait &x : w[y])
      if (x.read && ports[fifos[x.fifo].dst_port].kind == PRUNE_DRP) todo.push_back(x.fifo);
    bool hit = false;
    while (!todo.empty() && !hit) {
      const uint32_t f = todo.back();
      todo.pop_back();
      const StopPort &SP = ports[fifos[f].src_port];
      if (SP.kind == PRUNE_DRP) {
        hit = actors[SP.actor].cport_fifo >= 0 && token_index(SP.actor) > token_index(y);
        continue;
      }
      if (seen[SP.actor]) continue;
      seen[SP.actor] = 1;
      for (const Wait &x : w[SP.actor])
        if (x.read && (int64_t)x.fifo != actors[SP.actor].cport_fifo) todo.push_back(x.fifo);
    }
    if (hit) res.linked.push_back(y);
  }
  return res;
}

}  // namespace prune
