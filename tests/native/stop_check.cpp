// Host check of the per-firing stop classification (stop_rules.cpp, the code
// the library runs) on views read from stdin, one per case:
//   C na np nf
//   na lines: kind exhausted cport_fifo has_token token_mask firings n p...
//   np lines: actor dir kind element n f...
//   nf lines: src dst rate delay inflight
// Prints "stuck a..." and "linked y..." per case.  Built with ASan/UBSan.
#include <cstdio>
#include <vector>

#include "stop_rules.h"

using namespace prune;

int main() {
  unsigned C, na, np, nf;
  while (std::scanf("%u %u %u %u", &C, &na, &np, &nf) == 4) {
    std::vector<StopActor> a(na);
    std::vector<StopPort> p(np);
    std::vector<StopFifo> f(nf);
    for (auto &x : a) {
      unsigned kind, ex, tok, mask, n;
      long long cf;
      unsigned long long fir;
      if (std::scanf("%u %u %lld %u %u %llu %u", &kind, &ex, &cf, &tok, &mask, &fir, &n) != 7) return 2;
      x.kind = kind; x.exhausted = ex; x.cport_fifo = cf; x.has_token = tok; x.token_mask = mask;
      x.firings = fir;
      x.ports.resize(n);
      for (auto &q : x.ports)
        if (std::scanf("%u", &q) != 1) return 2;
    }
    for (auto &x : p) {
      unsigned n;
      if (std::scanf("%u %u %u %u %u", &x.actor, &x.dir, &x.kind, &x.element, &n) != 5) return 2;
      x.fifos.resize(n);
      for (auto &q : x.fifos)
        if (std::scanf("%u", &q) != 1) return 2;
    }
    for (auto &x : f) {
      long long inf;
      if (std::scanf("%u %u %u %u %lld", &x.src_port, &x.dst_port, &x.rate, &x.delay, &inf) != 5) return 2;
      x.inflight = inf;
    }
    const StopResult r = classify_stop_view(a, p, f, C);
    std::printf("stuck");
    for (unsigned v : r.stuck) std::printf(" %u", v);
    std::printf("\nlinked");
    for (unsigned v : r.linked) std::printf(" %u", v);
    std::printf("\n");
  }
  return 0;
}
