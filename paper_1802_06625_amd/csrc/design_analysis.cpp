// Compile-time analysis of a PRUNE graph (Sec. IV design rules, Sec. V DPG
// analysis).
//
// Adjacency and chains use data FIFOs only.  Two DRPs of different actors x
// and y are linked when they share a FIFO, or when the actors u and w at the
// far ends of their FIFOs are connected in the data graph with x and y
// removed; the actors of the connecting subchains are then exactly the
// vertices of every simple u-w path there, which is the biconnected block
// that holds an added u-w edge.  The same block query with an added x-y
// edge answers whether an actor lies on a chain connecting x and y (rule 5).
//
// DPGs pair an actor with output DRPs and an actor with input DRPs that
// have linked DRPs; their DCs are the components left after removing q, x
// and y, plus one dummy DC per FIFO joining a DRP of x to a DRP of y.  Each
// DC is scheduled once (x, its actors by id, y; every repetition count is
// one because FIFO rates are symmetric), which decides deadlock and gives
// the buffer bound beta(f) as the largest token count seen.  Actors outside
// every DC are scheduled the same way over the FIFOs among them.
#include "design_analysis.h"

#include <algorithm>
#include <set>

#include "prune.h"

namespace prune {
namespace {

struct Ctx {
  const DesignGraph &g;
  uint32_t na = 0, nf = 0;
  std::vector<char> is_ctrl;                  // FIFO ends in a control port
  std::vector<std::vector<uint32_t>> nb;      // data adjacency: sorted, unique, no self loops
  std::vector<std::vector<uint32_t>> drps;    // external DRPs per actor, creation order
  std::vector<int64_t> ctl, ctl_fifo;         // control output port feeding the actor, its FIFO
  std::vector<uint32_t> comp;                 // connected component of the data graph

  explicit Ctx(const DesignGraph &gr) : g(gr) {
    na = (uint32_t)g.kind.size();
    nf = (uint32_t)g.fifo.size();
    is_ctrl.assign(nf, 0);
    nb.assign(na, {});
    for (uint32_t f = 0; f < nf; ++f) {
      is_ctrl[f] = g.port[g.fifo[f].dst].kind == PRUNE_CPORT;
      if (is_ctrl[f]) continue;
      const uint32_t u = actor(g.fifo[f].src), v = actor(g.fifo[f].dst);
      if (u == v) continue;
      nb[u].push_back(v);
      nb[v].push_back(u);
    }
    for (auto &v : nb) {
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    drps.assign(na, {});
    ctl.assign(na, -1);
    ctl_fifo.assign(na, -1);
    for (uint32_t a = 0; a < na; ++a) {
      for (uint32_t p : g.ports[a]) {
        const DesignPort &P = g.port[p];
        if (P.kind == PRUNE_DRP) drps[a].push_back(p);
        if (ctl[a] < 0 && P.dir == PRUNE_IN && P.kind == PRUNE_CPORT && !P.fifos.empty()) {
          ctl_fifo[a] = P.fifos[0];
          ctl[a] = g.fifo[P.fifos[0]].src;
        }
      }
    }
    comp.assign(na, UINT32_MAX);
    std::vector<char> none(na, 0);
    for (uint32_t a = 0; a < na; ++a)
      if (comp[a] == UINT32_MAX) label(none, a, a, comp);
  }

  uint32_t actor(uint32_t p) const { return g.port[p].actor; }
  bool dynamic(uint32_t a) const { return !drps[a].empty(); }
  bool static_proc(uint32_t a) const { return !dynamic(a) && g.kind[a] != PRUNE_CONFIG; }
  uint32_t other_end(uint32_t f, uint32_t p) const {
    return g.fifo[f].src == p ? actor(g.fifo[f].dst) : actor(g.fifo[f].src);
  }
  int64_t element(uint32_t p) const {
    const int64_t c = ctl[actor(p)];
    if (c < 0) return 0;
    auto it = g.table.find({(uint32_t)c, p});
    return it == g.table.end() ? 0 : it->second;
  }

  // Mark every actor reachable from `a` in the data graph minus `banned`.
  void label(const std::vector<char> &banned, uint32_t a, uint32_t id, std::vector<uint32_t> &lab) const {
    std::vector<uint32_t> todo{a};
    lab[a] = id;
    while (!todo.empty()) {
      const uint32_t v = todo.back();
      todo.pop_back();
      for (uint32_t w : nb[v])
        if (!banned[w] && lab[w] == UINT32_MAX) {
          lab[w] = id;
          todo.push_back(w);
        }
    }
  }

  // Vertices of every simple s-t path in the data graph minus `banned`; false
  // if there is no such path.
  bool path_vertices(const std::vector<char> &banned, uint32_t s, uint32_t t,
                     std::vector<uint32_t> &out) const {
    out.clear();
    if (banned[s] || banned[t]) return false;
    if (s == t) {
      out.push_back(s);
      return true;
    }
    {
      std::vector<uint32_t> lab(na, UINT32_MAX);
      label(banned, s, 0, lab);
      if (lab[t] == UINT32_MAX) return false;
    }
    // Blocks of the graph plus a virtual s-t edge (Hopcroft-Tarjan, iterative,
    // edge stack); the virtual edge is the last neighbour of s and of t.
    struct Edge { uint32_t a, b; bool virt; };
    struct Frame { uint32_t v; int64_t parent; bool parent_virt; size_t k; };
    std::vector<int> disc(na, -1), low(na, 0);
    std::vector<Edge> est;
    std::vector<Frame> st;
    int timer = 0;
    disc[s] = low[s] = timer++;
    st.push_back({s, -1, false, 0});
    bool found = false;
    while (!st.empty()) {
      const uint32_t v = st.back().v;
      const std::vector<uint32_t> &nv = nb[v];
      const size_t deg = nv.size() + ((v == s || v == t) ? 1 : 0);
      if (st.back().k < deg) {
        const size_t k = st.back().k++;
        const bool virt = k == nv.size();
        const uint32_t w = virt ? (v == s ? t : s) : nv[k];
        if (banned[w]) continue;
        if ((int64_t)w == st.back().parent && virt == st.back().parent_virt) continue;
        if (disc[w] < 0) {
          est.push_back({v, w, virt});
          disc[w] = low[w] = timer++;
          st.push_back({w, (int64_t)v, virt, 0});
        } else if (disc[w] < disc[v]) {
          est.push_back({v, w, virt});
          low[v] = std::min(low[v], disc[w]);
        }
        continue;
      }
      const Frame done = st.back();
      st.pop_back();
      if (done.parent < 0) continue;
      const uint32_t p = (uint32_t)done.parent;
      low[p] = std::min(low[p], low[v]);
      if (low[v] >= disc[p]) {
        std::vector<uint32_t> verts;
        bool has_virt = false;
        for (;;) {
          const Edge e = est.back();
          est.pop_back();
          verts.push_back(e.a);
          verts.push_back(e.b);
          has_virt |= e.virt;
          if (e.a == p && e.b == v && e.virt == done.parent_virt) break;
        }
        if (has_virt) {
          std::sort(verts.begin(), verts.end());
          verts.erase(std::unique(verts.begin(), verts.end()), verts.end());
          out = verts;
          found = true;
        }
      }
    }
    return found;
  }

  // Fire each actor of `order` once, always the first fireable one, over the
  // FIFOs `H` (sorted ids).  bound[i] receives the largest count of H[i];
  // false on deadlock.
  bool schedule(const std::vector<uint32_t> &order, const std::vector<uint32_t> &H,
                std::vector<int64_t> &bound) const {
    const size_t n = order.size();
    std::vector<int64_t> tok(H.size());
    bound.assign(H.size(), 0);
    std::vector<std::vector<uint32_t>> ins(n), outs(n);
    std::vector<int64_t> pos(na, -1);
    for (size_t i = 0; i < n; ++i) pos[order[i]] = (int64_t)i;
    for (size_t i = 0; i < H.size(); ++i) {
      const DesignFifo &F = g.fifo[H[i]];
      tok[i] = bound[i] = F.delay;
      const int64_t ps = pos[actor(F.src)], pd = pos[actor(F.dst)];
      if (pd >= 0) ins[pd].push_back((uint32_t)i);
      if (ps >= 0) outs[ps].push_back((uint32_t)i);
    }
    std::vector<char> fired(n, 0);
    for (size_t step = 0; step < n; ++step) {
      size_t pick = n;
      for (size_t i = 0; i < n && pick == n; ++i) {
        if (fired[i]) continue;
        bool ok = true;
        for (uint32_t e : ins[i]) ok = ok && tok[e] >= (int64_t)g.fifo[H[e]].rate;
        if (ok) pick = i;
      }
      if (pick == n) return false;
      fired[pick] = 1;
      for (uint32_t e : ins[pick]) tok[e] -= g.fifo[H[e]].rate;
      for (uint32_t e : outs[pick]) tok[e] += g.fifo[H[e]].rate;
      for (uint32_t e : ins[pick]) bound[e] = std::max(bound[e], tok[e]);
      for (uint32_t e : outs[pick]) bound[e] = std::max(bound[e], tok[e]);
    }
    return true;
  }
};

}  // namespace

DesignReport analyze_design(const DesignGraph &g) {
  Ctx c(g);
  DesignReport R;
  std::set<std::array<int64_t, 3>> viol;
  const uint32_t na = c.na;

  // ---- linked DRPs and the actors of their connecting subchains
  std::vector<uint32_t> all;
  for (uint32_t a = 0; a < na; ++a) all.insert(all.end(), c.drps[a].begin(), c.drps[a].end());
  struct Link { uint32_t p, p2; std::vector<uint32_t> members; };
  std::vector<Link> links;
  std::vector<char> banned(na, 0);
  std::vector<uint32_t> verts;
  for (size_t i = 0; i < all.size(); ++i) {
    for (size_t j = i + 1; j < all.size(); ++j) {
      const uint32_t p = all[i], p2 = all[j];
      const uint32_t x = c.actor(p), y = c.actor(p2);
      if (x == y) continue;
      bool direct = false;
      for (uint32_t f : g.port[p].fifos)
        for (uint32_t f2 : g.port[p2].fifos) direct |= f == f2;
      // a chain needs x and y in one component of the data graph
      if (!direct && c.comp[x] != c.comp[y]) continue;
      std::vector<char> mem(na, 0);
      bool chain = false;
      banned[x] = banned[y] = 1;
      for (uint32_t f : g.port[p].fifos) {
        if (c.is_ctrl[f]) continue;
        const uint32_t u = c.other_end(f, p);
        for (uint32_t f2 : g.port[p2].fifos) {
          if (c.is_ctrl[f2] || f2 == f) continue;
          const uint32_t w = c.other_end(f2, p2);
          if (u == x || u == y || w == x || w == y) continue;
          if (c.path_vertices(banned, u, w, verts)) {
            chain = true;
            for (uint32_t v : verts) mem[v] = 1;
          }
        }
      }
      banned[x] = banned[y] = 0;
      if (!direct && !chain) continue;
      Link L{std::min(p, p2), std::max(p, p2), {}};
      for (uint32_t a = 0; a < na; ++a)
        if (mem[a]) L.members.push_back(a);
      links.push_back(std::move(L));
    }
  }
  std::sort(links.begin(), links.end(), [](const Link &a, const Link &b) {
    return a.p != b.p ? a.p < b.p : a.p2 < b.p2;
  });
  for (const Link &L : links) R.linked.push_back({L.p, L.p2});

  // ---- rule 1: linked DRPs share the control output port and the element
  for (const Link &L : links) {
    const int64_t cx = c.ctl[c.actor(L.p)], cy = c.ctl[c.actor(L.p2)];
    const int64_t ex = c.element(L.p), ey = c.element(L.p2);
    if (!(cx >= 0 && cx == cy && ex == ey && ex > 0)) viol.insert({kRule1, L.p, L.p2});
  }

  // ---- rule 2: one control output port reaches its dynamic actors with one delay
  {
    std::map<int64_t, std::vector<uint32_t>> by_port;
    for (uint32_t a = 0; a < na; ++a)
      if (c.dynamic(a) && c.ctl[a] >= 0) by_port[c.ctl[a]].push_back(a);
    for (auto &kv : by_port) {
      const uint32_t a0 = kv.second.front();
      const uint32_t d0 = g.fifo[c.ctl_fifo[a0]].delay;
      for (uint32_t a : kv.second)
        if (g.fifo[c.ctl_fifo[a]].delay != d0) viol.insert({kRule2, a0, a});
    }
  }

  // ---- rules 3 and 5 over the connecting subchains
  {
    std::map<uint32_t, std::set<std::pair<uint32_t, uint32_t>>> assoc;
    std::map<std::pair<uint32_t, uint32_t>, std::vector<char>> on_xy;   // cached per (x, y)
    std::vector<char> nobody(na, 0);
    for (const Link &L : links) {
      const uint32_t x = c.actor(L.p), y = c.actor(L.p2);
      const std::pair<uint32_t, uint32_t> key{std::min(x, y), std::max(x, y)};
      std::vector<char> in_s(na, 0);
      for (uint32_t a : L.members) {
        in_s[a] = 1;
        if (!c.static_proc(a)) viol.insert({kRule3Kind, a, -1});
        assoc[a].insert(key);
      }
      for (uint32_t a : L.members) {
        for (uint32_t p : g.ports[a]) {
          for (uint32_t f : g.port[p].fifos) {
            if (c.is_ctrl[f]) continue;
            const uint32_t bp = g.fifo[f].src == p ? g.fifo[f].dst : g.fifo[f].src;
            const uint32_t b = c.actor(bp);
            if (b == a || in_s[b] || g.port[bp].kind != PRUNE_SRP) continue;
            if (b == x || b == y) continue;
            auto it = on_xy.find(key);
            if (it == on_xy.end()) {
              std::vector<char> m(na, 0);
              if (c.path_vertices(nobody, key.first, key.second, verts))
                for (uint32_t v : verts) m[v] = 1;
              it = on_xy.emplace(key, std::move(m)).first;
            }
            if (!it->second[b]) viol.insert({kRule5, b, -1});
          }
        }
      }
    }
    for (auto &kv : assoc)
      if (kv.second.size() > 1) viol.insert({kRule3Shared, kv.first, -1});
  }

  // ---- rule 4: single-sided dynamism
  for (uint32_t a = 0; a < na; ++a) {
    bool in = false, out = false;
    for (uint32_t p : c.drps[a]) (g.port[p].dir == PRUNE_IN ? in : out) = true;
    if (in && out) viol.insert({kRule4, a, -1});
  }

  // ---- DPGs
  std::set<std::pair<uint32_t, uint32_t>> pairs;
  for (const Link &L : links) {
    const DesignPort &A = g.port[L.p], &B = g.port[L.p2];
    if (A.dir == PRUNE_OUT && B.dir == PRUNE_IN) pairs.insert({A.actor, B.actor});
    if (B.dir == PRUNE_OUT && A.dir == PRUNE_IN) pairs.insert({B.actor, A.actor});
  }
  {
    std::map<uint32_t, int> nx, ny;
    std::vector<char> in_dpg(na, 0);
    for (auto &pr : pairs) {
      ++nx[pr.first];
      ++ny[pr.second];
      in_dpg[pr.first] = in_dpg[pr.second] = 1;
    }
    for (auto &kv : nx)
      if (kv.second > 1) viol.insert({kPairing, kv.first, -1});
    for (auto &kv : ny)
      if (kv.second > 1) viol.insert({kPairing, kv.first, -1});
    for (uint32_t a = 0; a < na; ++a)
      if (c.dynamic(a) && !in_dpg[a]) viol.insert({kUnpaired, a, -1});
  }

  R.dc_of_actor.assign(na, -1);
  R.beta.assign(c.nf, -1);
  std::vector<char> dc_fifo(c.nf, 0);
  int64_t di = 0;
  for (auto &pr : pairs) {
    const uint32_t x = pr.first, y = pr.second;
    const int64_t cx = c.ctl[x];
    const int64_t q = cx >= 0 ? (int64_t)c.actor((uint32_t)cx) : -1;
    R.dpgs.push_back({q, x, y, cx});
    std::vector<char> removed(na, 0);
    removed[x] = removed[y] = 1;
    if (q >= 0) removed[q] = 1;
    // components left after removing q, x and y, named by their smallest actor
    std::vector<uint32_t> lab(na, UINT32_MAX);
    for (uint32_t a = 0; a < na; ++a)
      if (!removed[a] && lab[a] == UINT32_MAX) c.label(removed, a, a, lab);
    std::map<uint32_t, std::vector<uint32_t>> attach;
    std::vector<uint32_t> direct;
    std::vector<uint32_t> xy = c.drps[x];
    xy.insert(xy.end(), c.drps[y].begin(), c.drps[y].end());
    for (uint32_t p : xy) {
      for (uint32_t f : g.port[p].fifos) {
        if (c.is_ctrl[f]) continue;
        const uint32_t sa = c.actor(g.fifo[f].src), da = c.actor(g.fifo[f].dst);
        if ((sa == x && da == y) || (sa == y && da == x)) {
          if (g.port[g.fifo[f].src].kind == PRUNE_DRP && g.port[g.fifo[f].dst].kind == PRUNE_DRP &&
              std::find(direct.begin(), direct.end(), f) == direct.end())
            direct.push_back(f);
          continue;
        }
        const uint32_t o = c.other_end(f, p);
        if (!removed[o]) attach[lab[o]].push_back(p);
      }
    }
    std::sort(direct.begin(), direct.end());
    struct Local { std::vector<uint32_t> actors, ports; int64_t fifo; };
    std::vector<Local> local;
    for (auto &kv : attach) {
      Local l{{}, kv.second, -1};
      for (uint32_t a = 0; a < na; ++a)
        if (!removed[a] && lab[a] == kv.first) l.actors.push_back(a);
      local.push_back(std::move(l));
    }
    for (uint32_t f : direct) local.push_back({{}, {g.fifo[f].src, g.fifo[f].dst}, (int64_t)f});

    std::vector<int64_t> elements;
    for (const Local &l : local) {
      const int64_t idx = (int64_t)R.dcs.size();
      std::set<int64_t> E;
      bool to_x = false, to_y = false;
      for (uint32_t p : l.ports) {
        E.insert(c.element(p));
        to_x |= c.actor(p) == x;
        to_y |= c.actor(p) == y;
      }
      const int64_t el = E.size() == 1 ? *E.begin() : -1;
      if (el == -1) viol.insert({kDpgBDc, di, idx});
      if (!to_x || !to_y) viol.insert({kDpgA, di, idx});
      elements.push_back(el);
      R.dcs.push_back({di, el, l.fifo, l.actors});
      std::vector<char> mem(na, 0);
      for (uint32_t a : l.actors) {
        R.dc_of_actor[a] = idx;
        mem[a] = 1;
      }
      std::vector<uint32_t> H;
      if (l.fifo >= 0) H.push_back((uint32_t)l.fifo);
      for (uint32_t f = 0; f < c.nf; ++f) {
        if (c.is_ctrl[f] || (int64_t)f == l.fifo) continue;
        const uint32_t sp = g.fifo[f].src, dp = g.fifo[f].dst;
        const uint32_t u = c.actor(sp), w = c.actor(dp);
        if (!mem[u] && !mem[w]) continue;
        const bool inside = (mem[u] || u == x || u == y) && (mem[w] || w == x || w == y);
        if (inside) H.push_back(f);
        const bool ok = (mem[u] && mem[w]) ||
                        (u == x && mem[w] && g.port[sp].kind == PRUNE_DRP) ||
                        (w == y && mem[u] && g.port[dp].kind == PRUNE_DRP);
        if (!ok) viol.insert({kDpgC, di, (int64_t)f});
      }
      std::sort(H.begin(), H.end());
      std::vector<uint32_t> order{x};
      order.insert(order.end(), l.actors.begin(), l.actors.end());
      order.push_back(y);
      std::vector<int64_t> bound;
      const bool live = c.schedule(order, H, bound);
      if (!live) viol.insert({kDeadlockDc, di, idx});
      for (size_t i = 0; i < H.size(); ++i) {
        dc_fifo[H[i]] = 1;
        R.beta[H[i]] = live ? bound[i] : -1;
      }
    }
    std::set<int64_t> used;
    for (uint32_t p : xy) used.insert(c.element(p));
    std::set<int64_t> good;
    size_t n_good = 0;
    for (int64_t e : elements)
      if (e != -1) {
        good.insert(e);
        ++n_good;
      }
    if (good.size() != n_good || used.size() != local.size()) viol.insert({kDpgBCount, di, -1});
    ++di;
  }

  // ---- actors outside every DC and the FIFOs among them, control FIFOs included
  {
    std::vector<uint32_t> top;
    std::vector<char> in_top(na, 0);
    for (uint32_t a = 0; a < na; ++a)
      if (R.dc_of_actor[a] < 0) {
        top.push_back(a);
        in_top[a] = 1;
      }
    std::vector<uint32_t> T;
    for (uint32_t f = 0; f < c.nf; ++f)
      if (!dc_fifo[f] && in_top[c.actor(g.fifo[f].src)] && in_top[c.actor(g.fifo[f].dst)]) T.push_back(f);
    std::vector<int64_t> bound;
    const bool live = c.schedule(top, T, bound);
    if (!live) viol.insert({kDeadlockTop, -1, -1});
    for (size_t i = 0; i < T.size(); ++i) R.beta[T[i]] = live ? bound[i] : -1;
  }

  R.violations.assign(viol.begin(), viol.end());
  return R;
}

}  // namespace prune
