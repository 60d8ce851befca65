// Host check of the compile-time analysis (design_analysis.cpp, the code the
// library runs) on graph structures read from stdin, one per case:
//   na np nf nt
//   na kinds
//   np lines: actor dir kind        (external ports, in creation order)
//   nf lines: src dst rate delay
//   nt lines: control_port drp element
// Prints the report's tables one per line.  Built with ASan/UBSan.
#include <cstdio>

#include "design_analysis.h"

using namespace prune;

int main() {
  unsigned na, np, nf, nt;
  while (std::scanf("%u %u %u %u", &na, &np, &nf, &nt) == 4) {
    DesignGraph g;
    g.kind.resize(na);
    g.ports.resize(na);
    for (auto &k : g.kind)
      if (std::scanf("%u", &k) != 1) return 2;
    g.port.resize(np);
    for (unsigned i = 0; i < np; ++i) {
      DesignPort &P = g.port[i];
      if (std::scanf("%u %u %u", &P.actor, &P.dir, &P.kind) != 3 || P.actor >= na) return 2;
      g.ports[P.actor].push_back(i);
    }
    g.fifo.resize(nf);
    for (unsigned i = 0; i < nf; ++i) {
      DesignFifo &F = g.fifo[i];
      if (std::scanf("%u %u %u %u", &F.src, &F.dst, &F.rate, &F.delay) != 4 || F.src >= np || F.dst >= np)
        return 2;
      g.port[F.src].fifos.push_back(i);
      g.port[F.dst].fifos.push_back(i);
    }
    for (unsigned i = 0; i < nt; ++i) {
      unsigned c, p, e;
      if (std::scanf("%u %u %u", &c, &p, &e) != 3) return 2;
      g.table[{c, p}] = e;
    }
    const DesignReport r = analyze_design(g);
    std::printf("linked");
    for (auto &v : r.linked) std::printf(" %lld %lld", (long long)v[0], (long long)v[1]);
    std::printf("\ndpgs");
    for (auto &v : r.dpgs) std::printf(" %lld %lld %lld %lld", (long long)v[0], (long long)v[1], (long long)v[2], (long long)v[3]);
    std::printf("\ndcs");
    for (auto &d : r.dcs) {
      std::printf(" %lld %lld %lld %zu", (long long)d.dpg, (long long)d.element, (long long)d.direct_fifo, d.actors.size());
      for (unsigned a : d.actors) std::printf(" %u", a);
    }
    std::printf("\ndc_of_actor");
    for (auto v : r.dc_of_actor) std::printf(" %lld", (long long)v);
    std::printf("\nbeta");
    for (auto v : r.beta) std::printf(" %lld", (long long)v);
    std::printf("\nviolations");
    for (auto &v : r.violations) std::printf(" %lld %lld %lld", (long long)v[0], (long long)v[1], (long long)v[2]);
    std::printf("\n");
  }
  return 0;
}
