// Host runtime of libprune_hip: graph construction and validation (Sec. III,
// rule 4 of Sec. IV), FIFO sizing by Eq. 2, the per-firing executor (one
// launch sequence per firing, round-robin over actors as in Sec. VI-C), the
// batched executor (B graph iterations: one control launch, per-level copy
// and persistent filter-bank launches, one history launch) with optional
// hipGraph capture, and the direct filter-bank operations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "prune.h"
#include "design_analysis.h"
#include "stop_rules.h"
#include "prune_internal.h"
#include "runtime_kernels.h"

using namespace prune;

namespace {

thread_local std::string g_last_error;
thread_local float g_fb_ms = 0.f;
thread_local uint32_t g_fb_launches = 0;
thread_local bool g_timing = false;
std::atomic<bool> g_pipeline{true};   // batched firing: bookkeeping on a side stream

thread_local std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;
int g_variant_forced = 0;
}  // namespace

namespace prune {
int forced_variant() { return g_variant_forced; }
void set_last_error(const char *msg) { g_last_error = msg; }
// Kernel timing of the direct forward (prune_fb_forward) on this thread.
bool timing_on() { return g_timing; }
// A launch is timed only when both of its events exist.
void timing_push(hipEvent_t e0, hipEvent_t e1) {
  if (e0 && e1) {
    g_events.push_back({e0, e1});
    return;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
}
}  // namespace prune

namespace {

prune_status fail(prune_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

#define HIPCHECK(x)                                                                      \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      return fail(PRUNE_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_));          \
  } while (0)

#define TRY(x)                                                                           \
  do {                                                                                   \
    prune_status s_ = (x);                                                               \
    if (s_ != PRUNE_OK) return s_;                                                       \
  } while (0)

struct HPort {
  uint32_t actor, dir, kind, atr, token_bytes, flags, halo;
  bool internal = false;
  std::vector<uint32_t> fifos;
  uint32_t dev = kNone;    // PortDev index
};

struct HFifo {
  uint32_t src, dst, rate, delay, token_bytes;
  bool ctrl = false, param = false;
  uint64_t capacity = 0;   // tokens (Eq. 2)
  void *storage = nullptr;
  size_t bytes = 0;
  bool owned = false;
  uint32_t *counts = nullptr;
  int64_t inflight = 0;    // blocks written and not yet read (host view)
  std::deque<prune_ctrl_token> mirror;   // control FIFOs: tokens in flight
};

struct SrcPending {
  uint32_t count;
  const void *ptr;
};

struct HActor {
  uint32_t kind;
  std::vector<uint32_t> ports;      // external ports in creation order
  std::vector<uint32_t> branches;   // filter-bank branch DRPs
  prune_config_params cfg{};
  prune_fb_params fb{};
  prune_pixel_params pix{};
  uint32_t level = 0, comp = 0;
  uint64_t firings = 0;
  std::deque<SrcPending> src_q;
  std::deque<prune_side_info> side_q;
  void *q_dev = nullptr;
  uint64_t q_cap = 0, q_tail = 0, q_head = 0;
  // Queue entries below q_synced are known to be read by the device; those in
  // [q_synced, q_head) may still be read by bookkeeping in flight (fire calls
  // return before the device runs them).
  uint64_t q_synced = 0;
  float2 *history = nullptr;
  uint32_t hist_len = 0;
  float2 *taps = nullptr;
  uint64_t *bstats = nullptr;
  uint32_t fb_index = kNone;
  void *sink_out = nullptr;
  uint64_t sink_cap = 0;
};

}  // namespace

struct prune_graph {
  int device = 0;
  bool host_only = false;
  bool finalized = false;
  uint32_t C = 0;
  std::vector<HActor> actors;
  std::vector<HPort> ports;
  std::vector<HFifo> fifos;
  std::map<std::pair<uint32_t, uint32_t>, uint32_t> table;
  // compile-time analysis (Sec. IV-V)
  uint32_t checks = 0;
  bool analyzed = false;
  prune::DesignReport report;
  // device tables
  FifoDev *d_fifos = nullptr;
  PortDev *d_ports = nullptr;
  ActorDev *d_actors = nullptr;
  FbParamsDev *d_fbs = nullptr;
  uint32_t n_fb = 0;
  std::vector<PortDev> h_ports;
  // structure
  bool dag = true, has_delay = false, has_unaligned_delay = false;
  uint32_t n_comp = 0, n_levels = 0;
  std::vector<uint32_t> comp_off, comp_actors;
  uint32_t *d_comp_off = nullptr, *d_comp_actors = nullptr, *d_iota = nullptr,
           *d_single_off = nullptr;
  std::vector<char> level_fb, level_copy;
  std::vector<uint32_t> fb_item_off, fb_item_cap, copy_item_off, copy_item_cap, copy_max_total;
  std::vector<uint32_t> copy_pix_rows;   // per level: most rows of a pixel actor's frame
  std::vector<uint32_t> post_actors;
  uint32_t *d_post_actors = nullptr;
  // scratch
  uint32_t Bcap = 0;
  FiringRec *d_recs = nullptr;
  uint32_t *d_wrote = nullptr;
  FbFrameDesc *d_desc = nullptr;
  uint32_t *d_desc_off = nullptr;
  WorkItem *d_items = nullptr;
  uint32_t *d_item_off = nullptr;
  CopyItem *d_copy = nullptr;
  uint32_t *d_copy_off = nullptr;
  uint32_t *d_level_of = nullptr;
  float2 *d_halo_scratch = nullptr;
  uint32_t *d_halo_off = nullptr;
  uint32_t *d_ctr = nullptr;   // fb_count[nl], copy_count[nl], ticket[nl], gather_count[nl]
  GatherReq *d_gather = nullptr;
  bool fast_batch = true;
  BatchArgs bargs{};
  std::vector<uint32_t> fifo_local;
  uint32_t *d_gather_off = nullptr;
  std::vector<uint32_t> gather_off, gather_cap;
  uint32_t *d_err = nullptr;
  prune_trace_record *d_trace = nullptr;
  uint64_t trace_cap = 0;
  unsigned long long *d_trace_count = nullptr;
  std::map<uint64_t, hipGraphExec_t> graphs;
  std::map<uint64_t, hipGraph_t> graph_defs;
  // pipelined graph form: [set parity][0 bookkeeping, 1 data kernels]
  std::map<uint64_t, hipGraphExec_t> pgraphs[2][2];
  std::map<uint64_t, hipGraph_t> pgraph_defs[2][2];
  hipStream_t capture_stream = nullptr;
  int variant = 1;
  uint32_t tile = 2048;
  int ncu = 256;
  int fb_grid = 768;
  std::vector<void *> owned;
  // Per-batch buffers in two sets.  In stream mode the bookkeeping of batch
  // i (decode, scan, emit) runs on a side stream into set i%2 while the data
  // kernels of batch i-1 still read the other set on the caller's stream.
  struct BatchSet {
    FiringRec *recs; uint32_t *wrote; FbFrameDesc *desc; WorkItem *items; CopyItem *copy;
    float2 *halo_scratch; uint32_t *ctr; GatherReq *gather;
  };
  BatchSet sets[2]{};
  uint32_t parity = 0;
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_emit[2]{}, ev_done[2]{}, ev_sync = nullptr;
  bool done_valid[2]{};
  bool need_sync = true;    // the caller's stream has work the side stream must wait for

  ~prune_graph();
};

// Teardown reports nothing: errors here have no caller to go to.
prune_graph::~prune_graph() {
  if (side_stream) (void)hipStreamSynchronize(side_stream);
  for (hipEvent_t e : {ev_emit[0], ev_emit[1], ev_done[0], ev_done[1], ev_sync})
    if (e) (void)hipEventDestroy(e);
  if (side_stream) (void)hipStreamDestroy(side_stream);
  for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto &kv : graph_defs) (void)hipGraphDestroy(kv.second);
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < 2; ++k) {
      for (auto &kv : pgraphs[p][k]) (void)hipGraphExecDestroy(kv.second);
      for (auto &kv : pgraph_defs[p][k]) (void)hipGraphDestroy(kv.second);
    }
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
  for (void *p : owned) (void)hipFree(p);
  for (auto &a : actors)
    if (a.q_dev) (void)hipFree(a.q_dev);
  if (d_trace) (void)hipFree(d_trace);
  if (d_trace_count) (void)hipFree(d_trace_count);
}

namespace {

template <class T>
prune_status dalloc(prune_graph *g, T **p, size_t n) {
  if (n == 0) n = 1;
  HIPCHECK(hipMalloc((void **)p, n * sizeof(T)));
  HIPCHECK(hipMemset(*p, 0, n * sizeof(T)));
  g->owned.push_back((void *)*p);
  return PRUNE_OK;
}

template <class T>
prune_status upload(prune_graph *g, T **p, const std::vector<T> &v) {
  TRY(dalloc(g, p, v.size()));
  if (!v.empty()) HIPCHECK(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return PRUNE_OK;
}

int64_t cport_fifo(const prune_graph *g, const HActor &a) {
  for (uint32_t p : a.ports)
    if (g->ports[p].kind == PRUNE_CPORT) return g->ports[p].fifos.empty() ? -1 : g->ports[p].fifos[0];
  return -1;
}

uint32_t controller_port(const prune_graph *g, const HActor &a) {
  int64_t f = cport_fifo(g, a);
  return f < 0 ? kNone : g->fifos[f].src;
}

uint32_t n_elements_of(const prune_graph *g, const HActor &a) {
  uint32_t cp = controller_port(g, a);
  if (cp == kNone) return 32;
  const HActor &q = g->actors[g->ports[cp].actor];
  return q.cfg.n_elements ? q.cfg.n_elements : 32;
}

uint32_t fb_lmax(const prune_fb_params &p) {
  uint32_t m = 1;
  for (uint32_t b = 0; b < p.n_banks; ++b) m = std::max(m, p.L[b]);
  return m;
}

// ---------------------------------------------------------------- validation
prune_status validate_actor(prune_graph *g, uint32_t aid) {
  HActor &a = g->actors[aid];
  std::vector<HPort *> ins, outs, cps, din, in_drp, out_drp;
  for (uint32_t p : a.ports) {
    HPort &P = g->ports[p];
    if (P.dir == PRUNE_IN) {
      ins.push_back(&P);
      if (P.kind == PRUNE_CPORT) cps.push_back(&P);
      else din.push_back(&P);
      if (P.kind == PRUNE_DRP) in_drp.push_back(&P);
    } else {
      outs.push_back(&P);
      if (P.kind == PRUNE_DRP) out_drp.push_back(&P);
    }
  }
  char buf[160];
  auto err = [&](prune_status s, const char *m) {
    snprintf(buf, sizeof buf, "actor %u: %s", aid, m);
    return fail(s, buf);
  };
  for (HPort *p : cps)
    if (p->atr != 1) return err(PRUNE_E_PORT_KIND, "control port rate must be 1");
  if (a.kind == PRUNE_CONFIG) {
    if (!ins.empty()) return err(PRUNE_E_ARG, "configuration actors take external side-information only");
    if (outs.empty()) return err(PRUNE_E_ARG, "configuration actor without a control output port");
    for (HPort *p : outs) {
      if (p->kind != PRUNE_SRP || p->atr != 1)
        return err(PRUNE_E_PORT_KIND, "control output ports are SRPs of rate 1");
      for (uint32_t f : p->fifos)
        if (g->ports[g->fifos[f].dst].kind != PRUNE_CPORT)
          return err(PRUNE_E_PORT_KIND, "control output ports connect to control ports");
    }
    return PRUNE_OK;
  }
  const bool dyn_kind = a.kind == PRUNE_SWITCH || a.kind == PRUNE_POLY || a.kind == PRUNE_SELECT;
  // byte-token ports move whole 8-byte words
  for (HPort *p : din)
    if (p->token_bytes == 1 && (p->atr % 8 || (p->flags & PRUNE_PORT_PARAM) || p->halo))
      return err(PRUNE_E_UNSUPPORTED, "byte-token ports carry fixed blocks of a multiple of 8 bytes");
  for (HPort *p : outs)
    if (p->token_bytes == 1 && (p->atr % 8 || (p->flags & PRUNE_PORT_PARAM) || p->halo))
      return err(PRUNE_E_UNSUPPORTED, "byte-token ports carry fixed blocks of a multiple of 8 bytes");
  const bool dynamic = dyn_kind || (a.kind == PRUNE_FILTERBANK && !cps.empty());
  if (!dynamic) {
    if (!cps.empty() || !in_drp.empty() || !out_drp.empty())
      return err(PRUNE_E_PORT_KIND, "static actors have SRPs only");
  } else {
    if (cps.size() != 1) return err(PRUNE_E_PORT_KIND, "a dynamic actor has exactly one control port");
    if (a.kind != PRUNE_FILTERBANK && in_drp.empty() && out_drp.empty())
      return err(PRUNE_E_PORT_KIND, "a dynamic actor needs a DRP");
    if (!in_drp.empty() && !out_drp.empty())
      return err(PRUNE_E_RULE4, "dynamic inputs and outputs on one actor (rule 4)");
    uint32_t ctl = controller_port(g, a);
    if (ctl == kNone) return err(PRUNE_E_CONNECT, "control port not connected");
    const uint32_t nel = n_elements_of(g, a);
    std::vector<uint32_t> drps;
    if (a.kind == PRUNE_FILTERBANK) drps = a.branches;
    for (HPort *p : in_drp) drps.push_back((uint32_t)(p - g->ports.data()));
    for (HPort *p : out_drp) drps.push_back((uint32_t)(p - g->ports.data()));
    for (uint32_t d : drps) {
      auto it = g->table.find({ctl, d});
      uint32_t e = it == g->table.end() ? 0 : it->second;
      if (e < 1 || e > nel)
        return err(PRUNE_E_PORT_KIND, "DRP not controlled by the port feeding its actor");
    }
  }
  switch (a.kind) {
    case PRUNE_SOURCE:
      if (!ins.empty() || outs.size() != 1) return err(PRUNE_E_ARG, "one output port, no inputs");
      break;
    case PRUNE_SINK:
      if (din.size() != 1 || !outs.empty() || !cps.empty()) return err(PRUNE_E_ARG, "one input port");
      break;
    case PRUNE_PASSTHROUGH:
      if (din.size() != 1 || outs.size() != 1) return err(PRUNE_E_ARG, "one input and one output");
      if (din[0]->atr != outs[0]->atr || din[0]->flags != outs[0]->flags || din[0]->halo || outs[0]->halo)
        return err(PRUNE_E_RATE_MISMATCH, "input and output rates differ");
      break;
    case PRUNE_FILTERBANK: {
      if (din.size() != 1 || outs.size() != 1) return err(PRUNE_E_ARG, "one data input and one output");
      const uint32_t H = fb_lmax(a.fb) - 1;
      HPort *pi = din[0], *po = outs[0];
      if (pi->kind != PRUNE_SRP || po->kind != PRUNE_SRP)
        return err(PRUNE_E_PORT_KIND, "filter-bank data ports are SRPs");
      if ((pi->flags & PRUNE_PORT_PARAM) != (po->flags & PRUNE_PORT_PARAM))
        return err(PRUNE_E_RATE_MISMATCH, "parameterisation differs");
      if (a.fb.windowed) {
        if (pi->atr != po->atr + H || pi->halo != H || po->halo)
          return err(PRUNE_E_RATE_MISMATCH, "windowed input = output + Lmax-1");
      } else if (pi->atr != po->atr || pi->halo || po->halo) {
        return err(PRUNE_E_RATE_MISMATCH, "input and output rates differ");
      }
      if (!a.fb.windowed && H > 0 && cps.empty() && false)
        return err(PRUNE_E_ARG, "");
      break;
    }
    case PRUNE_SWITCH:
    case PRUNE_POLY:
      if (din.size() != 1 || din[0]->kind != PRUNE_SRP || outs.empty())
        return err(PRUNE_E_ARG, "one SRP input, DRP outputs");
      for (HPort *p : outs) {
        if (p->kind != PRUNE_DRP) return err(PRUNE_E_ARG, "switch outputs are DRPs");
        if (p->atr != din[0]->atr + p->halo || (p->flags & PRUNE_PORT_PARAM) != (din[0]->flags & PRUNE_PORT_PARAM))
          return err(PRUNE_E_RATE_MISMATCH, "output window = input + halo");
        if (p->halo > PRUNE_MAX_L - 1) return fail(PRUNE_E_UNSUPPORTED, "halo beyond 63 samples");
      }
      break;
    case PRUNE_GAUSS5:
    case PRUNE_THRES:
    case PRUNE_MED5: {
      const uint32_t npix = a.pix.W * a.pix.H;
      if (din.size() != (a.kind == PRUNE_THRES ? 2u : 1u) || outs.size() != 1)
        return err(PRUNE_E_ARG, "pixel actors: one input (two for THRES), one output");
      for (HPort *p : din)
        if (p->atr != npix || p->token_bytes != 1) return err(PRUNE_E_RATE_MISMATCH, "pixel ports carry one W*H frame");
      if (outs[0]->atr != npix || outs[0]->token_bytes != 1)
        return err(PRUNE_E_RATE_MISMATCH, "pixel ports carry one W*H frame");
      break;
    }
    case PRUNE_SELECT:
      if (outs.size() != 1 || outs[0]->kind != PRUNE_SRP || in_drp.empty() || in_drp.size() != din.size())
        return err(PRUNE_E_ARG, "DRP inputs, one SRP output");
      if (din.size() > (size_t)kMaxIn) return fail(PRUNE_E_UNSUPPORTED, "more than PRUNE_MAX_IN select inputs");
      for (HPort *p : din)
        if (p->atr != outs[0]->atr || (p->flags & PRUNE_PORT_PARAM) != (outs[0]->flags & PRUNE_PORT_PARAM) || p->halo)
          return err(PRUNE_E_RATE_MISMATCH, "input and output rates differ");
      break;
    default:
      return err(PRUNE_E_ARG, "unknown actor kind");
  }
  if (a.ports.size() > (size_t)kMaxPorts) return fail(PRUNE_E_UNSUPPORTED, "more than PRUNE_MAX_PORTS ports on an actor");
  size_t nio = 0;
  for (HPort *p : outs) {
    if (p->fifos.size() > (size_t)kMaxFanout) return fail(PRUNE_E_UNSUPPORTED, "more than 4 FIFOs on a port");
    nio += p->fifos.size();
  }
  if (nio > (size_t)kMaxIO) return fail(PRUNE_E_UNSUPPORTED, "more than PRUNE_MAX_IO output FIFO accesses");
  return PRUNE_OK;
}

// ---------------------------------------------------------------- device tables
prune_status sync_actor_dev(prune_graph *g, uint32_t aid);

prune_status build_device(prune_graph *g) {
  // ports
  g->h_ports.clear();
  for (uint32_t p = 0; p < g->ports.size(); ++p) {
    HPort &P = g->ports[p];
    if (P.internal) continue;
    PortDev d{};
    d.actor = P.actor; d.dir = P.dir; d.kind = P.kind; d.atr = P.atr;
    d.param = (P.flags & PRUNE_PORT_PARAM) ? 1 : 0; d.halo = P.halo;
    d.element = 0;
    if (P.kind == PRUNE_DRP) {
      uint32_t ctl = controller_port(g, g->actors[P.actor]);
      auto it = g->table.find({ctl, p});
      d.element = it == g->table.end() ? 0 : it->second;
    }
    d.n_fifos = (uint32_t)P.fifos.size();
    for (size_t k = 0; k < P.fifos.size(); ++k) d.fifo[k] = P.fifos[k];
    d.power = 0;
    if (g->actors[P.actor].kind == PRUNE_POLY && P.dir == PRUNE_OUT) {
      for (uint32_t q : g->actors[P.actor].ports) {
        if (q == p) break;
        if (g->ports[q].dir == PRUNE_OUT) ++d.power;
      }
    }
    P.dev = (uint32_t)g->h_ports.size();
    g->h_ports.push_back(d);
  }
  TRY(upload(g, &g->d_ports, g->h_ports));
  // FIFO slots within their component (for the parallel batch decode)
  g->fifo_local.assign(g->fifos.size(), 0);
  {
    std::vector<uint32_t> per_comp(g->n_comp, 0);
    for (uint32_t f = 0; f < g->fifos.size(); ++f) {
      const uint32_t cmp = g->actors[g->ports[g->fifos[f].src].actor].comp;
      g->fifo_local[f] = per_comp[cmp]++;
      if (g->fifo_local[f] >= (uint32_t)kMaxCompFifos) g->fast_batch = false;
    }
  }
  // fifos
  std::vector<FifoDev> hf(g->fifos.size());
  for (uint32_t f = 0; f < g->fifos.size(); ++f) {
    HFifo &F = g->fifos[f];
    FifoDev &d = hf[f];
    memset(&d, 0, sizeof d);
    d.r = F.rate; d.Q = F.delay; d.C = g->C;
    d.blocks = (uint32_t)(F.capacity / F.rate);
    d.token_bytes = F.token_bytes; d.param = F.param; d.halo = g->ports[F.src].halo;
    d.aligned = (F.delay % F.rate) == 0;
    d.max_occ = F.delay;
    if (F.ctrl) {
      TRY(dalloc(g, (char **)&F.storage, F.capacity * F.token_bytes));
      F.bytes = F.capacity * F.token_bytes;
      F.owned = true;
    }
    if (F.param) TRY(dalloc(g, &F.counts, d.blocks));
    d.base = (char *)F.storage;
    d.counts = F.counts;
    d.pad = g->fifo_local[f];
  }
  TRY(upload(g, &g->d_fifos, hf));
  // filter banks
  std::vector<FbParamsDev> hfb;
  for (uint32_t a = 0; a < g->actors.size(); ++a) {
    HActor &A = g->actors[a];
    if (A.kind != PRUNE_FILTERBANK) continue;
    FbParamsDev d{};
    d.n_banks = A.fb.n_banks; d.Kmax = A.fb.Kmax; d.Lmax = fb_lmax(A.fb); d.windowed = A.fb.windowed;
    for (int b = 0; b < PRUNE_MAX_BANKS; ++b) d.L[b] = b < (int)A.fb.n_banks ? A.fb.L[b] : 0;
    const size_t nt = (size_t)d.n_banks * d.Kmax * d.Lmax;
    TRY(dalloc(g, &A.taps, nt));
    TRY(dalloc(g, &A.bstats, 2 * PRUNE_MAX_BRANCHES));
    d.taps = A.taps;
    d.branch_firings = A.bstats;
    d.branch_tokens = A.bstats + PRUNE_MAX_BRANCHES;
    uint32_t ctl = controller_port(g, A);
    for (uint32_t k = 0; k < A.branches.size(); ++k) {
      auto it = g->table.find({ctl, A.branches[k]});
      d.elem[k] = it == g->table.end() ? 0 : it->second;
    }
    A.fb_index = (uint32_t)hfb.size();
    hfb.push_back(d);
  }
  g->n_fb = (uint32_t)hfb.size();
  TRY(upload(g, &g->d_fbs, hfb));
  // actors
  std::vector<ActorDev> ha(g->actors.size());
  for (uint32_t a = 0; a < g->actors.size(); ++a) {
    HActor &A = g->actors[a];
    ActorDev &d = ha[a];
    memset(&d, 0, sizeof d);
    d.kind = A.kind;
    int64_t cf = cport_fifo(g, A);
    d.cport_fifo = cf < 0 ? kNone : (uint32_t)cf;
    d.n_elements = n_elements_of(g, A);
    d.first_in = kNone;
    uint32_t np = 0;
    for (uint32_t p : A.ports) {
      if (g->ports[p].kind == PRUNE_CPORT) continue;
      d.port[np++] = g->ports[p].dev;
      if (g->ports[p].dir == PRUNE_IN && d.first_in == kNone) d.first_in = g->ports[p].dev;
    }
    d.n_ports = np;
    d.cfg_mode = A.cfg.mode; d.cfg_Kmax = A.cfg.Kmax;
    d.fb = A.fb_index;
    d.fixed_mask = A.fb.fixed_mask;
    d.pix_w = A.pix.W; d.pix_h = A.pix.H; d.pix_t = A.pix.threshold;
    if (A.kind == PRUNE_FILTERBANK && !A.fb.windowed) A.hist_len = fb_lmax(A.fb) - 1;
    if (A.kind == PRUNE_SWITCH || A.kind == PRUNE_POLY) {
      for (uint32_t p : A.ports)
        if (g->ports[p].dir == PRUNE_OUT) A.hist_len = std::max(A.hist_len, g->ports[p].halo);
    }
    if (A.hist_len) TRY(dalloc(g, &A.history, A.hist_len));
    d.hist_len = A.hist_len;
    d.history = A.history;
  }
  TRY(upload(g, &g->d_actors, ha));
  return PRUNE_OK;
}

// Update the host-controlled fields of one actor's device record.
prune_status sync_actor_dev(prune_graph *g, uint32_t aid) {
  HActor &A = g->actors[aid];
  ActorDev *d = g->d_actors + aid;
  HIPCHECK(hipMemcpy(&d->queue, &A.q_dev, sizeof(void *), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(&d->q_cap, &A.q_cap, sizeof(uint64_t), hipMemcpyHostToDevice));
  float2 *so = (float2 *)A.sink_out;
  HIPCHECK(hipMemcpy(&d->sink_out, &so, sizeof(void *), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(&d->sink_cap, &A.sink_cap, sizeof(uint64_t), hipMemcpyHostToDevice));
  return PRUNE_OK;
}

// ---------------------------------------------------------------- structure
prune_status analyse(prune_graph *g) {
  const uint32_t na = (uint32_t)g->actors.size();
  // components (union-find over FIFOs)
  std::vector<uint32_t> par(na);
  for (uint32_t a = 0; a < na; ++a) par[a] = a;
  auto find = [&](uint32_t x) {
    while (par[x] != x) x = par[x] = par[par[x]];
    return x;
  };
  for (auto &F : g->fifos) {
    uint32_t a = find(g->ports[F.src].actor), b = find(g->ports[F.dst].actor);
    if (a != b) par[a] = b;
    if (F.delay) g->has_delay = true;
    if (F.delay % F.rate) g->has_unaligned_delay = true;
  }
  // levels by longest path (Kahn)
  std::vector<uint32_t> indeg(na, 0), level(na, 0);
  std::vector<std::vector<uint32_t>> succ(na);
  for (auto &F : g->fifos) {
    uint32_t a = g->ports[F.src].actor, b = g->ports[F.dst].actor;
    succ[a].push_back(b);
    indeg[b]++;
  }
  std::vector<uint32_t> order;
  std::deque<uint32_t> q;
  for (uint32_t a = 0; a < na; ++a)
    if (!indeg[a]) q.push_back(a);
  while (!q.empty()) {
    uint32_t a = q.front();
    q.pop_front();
    order.push_back(a);
    for (uint32_t b : succ[a]) {
      level[b] = std::max(level[b], level[a] + 1);
      if (--indeg[b] == 0) q.push_back(b);
    }
  }
  g->dag = order.size() == na;
  g->n_levels = 1;
  for (uint32_t a = 0; a < na; ++a) {
    g->actors[a].level = level[a];
    g->n_levels = std::max(g->n_levels, level[a] + 1);
  }
  std::map<uint32_t, uint32_t> comp_id;
  for (uint32_t a = 0; a < na; ++a) {
    uint32_t r = find(a);
    if (!comp_id.count(r)) comp_id[r] = (uint32_t)comp_id.size();
    g->actors[a].comp = comp_id[r];
  }
  g->n_comp = (uint32_t)comp_id.size();
  std::vector<std::vector<uint32_t>> members(g->n_comp);
  std::vector<uint32_t> byl(na);
  for (uint32_t a = 0; a < na; ++a) byl[a] = a;
  std::stable_sort(byl.begin(), byl.end(),
                   [&](uint32_t x, uint32_t y) { return level[x] < level[y]; });
  for (uint32_t a : byl) members[g->actors[a].comp].push_back(a);
  g->comp_off.assign(1, 0);
  g->comp_actors.clear();
  for (auto &m : members) {
    g->comp_actors.insert(g->comp_actors.end(), m.begin(), m.end());
    g->comp_off.push_back((uint32_t)g->comp_actors.size());
  }
  return PRUNE_OK;
}

uint32_t in_atr(const prune_graph *g, const HActor &a) {
  for (uint32_t p : a.ports)
    if (g->ports[p].dir == PRUNE_IN && g->ports[p].kind != PRUNE_CPORT) return g->ports[p].atr;
  return 0;
}

uint32_t max_out_atr(const prune_graph *g, const HActor &a) {
  uint32_t m = 0;
  for (uint32_t p : a.ports)
    if (g->ports[p].dir == PRUNE_OUT) m = std::max(m, g->ports[p].atr);
  return m;
}

uint32_t out_accesses(const prune_graph *g, const HActor &a) {
  uint32_t n = 0;
  for (uint32_t p : a.ports)
    if (g->ports[p].dir == PRUNE_OUT) n += (uint32_t)g->ports[p].fifos.size();
  return n;
}

bool is_pixel_kind(uint32_t k) { return k == PRUNE_GAUSS5 || k == PRUNE_THRES || k == PRUNE_MED5; }

bool is_copy_kind(uint32_t k) {
  return k == PRUNE_SWITCH || k == PRUNE_POLY || k == PRUNE_SELECT || k == PRUNE_PASSTHROUGH || k == PRUNE_SOURCE ||
         k == PRUNE_GAUSS5 || k == PRUNE_THRES || k == PRUNE_MED5 ||
         k == PRUNE_SINK;
}

prune_status alloc_scratch(prune_graph *g) {
  const uint32_t na = (uint32_t)g->actors.size(), nl = g->n_levels;
  const uint32_t Bc = g->Bcap;
  const uint32_t min_tile = 512;
  g->level_fb.assign(nl, 0);
  g->level_copy.assign(nl, 0);
  g->fb_item_cap.assign(nl, 0);
  g->copy_item_cap.assign(nl, 0);
  g->copy_max_total.assign(nl, 0);
  g->copy_pix_rows.assign(nl, 0);
  std::vector<uint32_t> desc_off(na, 0), halo_off(na, 0), level_of(na, 0);
  g->gather_cap.assign(nl, 0);
  uint32_t ndesc = 0, nhalo = 0;
  g->post_actors.clear();
  for (uint32_t a = 0; a < na; ++a) {
    HActor &A = g->actors[a];
    level_of[a] = A.level;
    if (A.kind == PRUNE_FILTERBANK) {
      g->level_fb[A.level] = 1;
      desc_off[a] = ndesc;
      ndesc += Bc;
      const uint32_t n = in_atr(g, A);
      g->fb_item_cap[A.level] += Bc * ((n + min_tile - 1) / min_tile);
    }
    if (is_copy_kind(A.kind)) {
      g->level_copy[A.level] = 1;
      // a pixel firing is one item that stores to every FIFO of its output
      uint32_t items = is_pixel_kind(A.kind) ? 1 : std::max<uint32_t>(1, out_accesses(g, A));
      g->copy_item_cap[A.level] += Bc * items;
      if (is_pixel_kind(A.kind))
        g->copy_pix_rows[A.level] = std::max(g->copy_pix_rows[A.level], A.pix.H);
      else
        g->copy_max_total[A.level] = std::max(g->copy_max_total[A.level],
                                              std::max(max_out_atr(g, A), in_atr(g, A)));
    }
    if (A.hist_len) {
      halo_off[a] = nhalo;
      nhalo += Bc * A.hist_len;
      g->post_actors.push_back(a);
      g->gather_cap[A.level] += Bc;
    }
  }
  g->fb_item_off.assign(nl, 0);
  g->copy_item_off.assign(nl, 0);
  g->gather_off.assign(nl, 0);
  uint32_t fo = 0, co = 0, go = 0;
  for (uint32_t l = 0; l < nl; ++l) {
    g->gather_off[l] = go;
    go += g->gather_cap[l];
    g->fb_item_off[l] = fo;
    fo += g->fb_item_cap[l];
    g->copy_item_off[l] = co;
    co += g->copy_item_cap[l];
  }
  TRY(dalloc(g, &g->d_recs, (size_t)na * Bc));
  TRY(dalloc(g, &g->d_wrote, (size_t)g->fifos.size() * Bc));
  TRY(dalloc(g, &g->d_desc, ndesc));
  TRY(upload(g, &g->d_desc_off, desc_off));
  TRY(dalloc(g, &g->d_items, fo));
  TRY(upload(g, &g->d_item_off, g->fb_item_off));
  TRY(dalloc(g, &g->d_copy, co));
  TRY(upload(g, &g->d_copy_off, g->copy_item_off));
  TRY(upload(g, &g->d_level_of, level_of));
  TRY(dalloc(g, &g->d_halo_scratch, nhalo));
  TRY(upload(g, &g->d_halo_off, halo_off));
  TRY(dalloc(g, &g->d_ctr, 4 * nl));
  TRY(dalloc(g, &g->d_gather, go));
  g->sets[0] = {g->d_recs, g->d_wrote, g->d_desc, g->d_items, g->d_copy, g->d_halo_scratch, g->d_ctr, g->d_gather};
  {
    prune_graph::BatchSet &S = g->sets[1];
    TRY(dalloc(g, &S.recs, (size_t)na * Bc));
    TRY(dalloc(g, &S.wrote, (size_t)g->fifos.size() * Bc));
    TRY(dalloc(g, &S.desc, ndesc));
    TRY(dalloc(g, &S.items, fo));
    TRY(dalloc(g, &S.copy, co));
    TRY(dalloc(g, &S.halo_scratch, nhalo));
    TRY(dalloc(g, &S.ctr, 4 * nl));
    TRY(dalloc(g, &S.gather, go));
  }
  TRY(upload(g, &g->d_gather_off, g->gather_off));
  TRY(dalloc(g, &g->d_err, 1));
  TRY(upload(g, &g->d_post_actors, g->post_actors));
  TRY(upload(g, &g->d_comp_off, g->comp_off));
  TRY(upload(g, &g->d_comp_actors, g->comp_actors));
  std::vector<uint32_t> iota(na);
  for (uint32_t a = 0; a < na; ++a) iota[a] = a;
  TRY(upload(g, &g->d_iota, iota));
  std::vector<uint32_t> so = {0, 1};
  TRY(upload(g, &g->d_single_off, so));
  // access table and per-iteration arrays of the parallel batch bookkeeping
  std::vector<uint32_t> acc_off(na + 1, 0);
  std::vector<AccDev> acc;
  for (uint32_t a = 0; a < na; ++a) {
    acc_off[a] = (uint32_t)acc.size();
    uint32_t in_slot = 0, out_slot = 0, drp = 0;
    for (uint32_t p : g->actors[a].ports) {
      const HPort &P = g->ports[p];
      if (P.kind == PRUNE_CPORT) continue;
      const uint32_t my_drp = P.kind == PRUNE_DRP ? drp++ : kNone;
      if (P.dir == PRUNE_IN) {
        AccDev d{P.dev, P.fifos[0], PRUNE_IN, in_slot++, 1u, my_drp, g->fifo_local[P.fifos[0]], 0u};
        acc.push_back(d);
      } else {
        for (size_t k = 0; k < P.fifos.size(); ++k) {
          AccDev d{P.dev, P.fifos[k], PRUNE_OUT, out_slot++, k == 0 ? 1u : 0u, my_drp,
                   g->fifo_local[P.fifos[k]], 0u};
          acc.push_back(d);
        }
      }
    }
  }
  acc_off[na] = (uint32_t)acc.size();
  uint32_t max_acc = 0;
  for (uint32_t a = 0; a < na; ++a) max_acc = std::max(max_acc, acc_off[a + 1] - acc_off[a]);
  std::vector<uint32_t> fifo_wacc(g->fifos.size(), 0);
  for (uint32_t k = 0; k < acc.size(); ++k)
    if (acc[k].dir == PRUNE_OUT) fifo_wacc[acc[k].fifo] = k;
  const size_t nacc = acc.size();
  BatchArgs &b = g->bargs;
  b.max_acc = max_acc;
  TRY(upload(g, (uint32_t **)&b.acc_off, acc_off));
  TRY(upload(g, (AccDev **)&b.acc, acc));
  uint32_t **soa[] = {&b.s_fired, &b.s_mask, &b.s_rate, &b.s_bitmap, &b.s_firing, &b.s_aux,
                      &b.s_auxoff, &b.s_aux2};
  for (uint32_t **q : soa) TRY(dalloc(g, q, (size_t)na * Bc));
  TRY(dalloc(g, &b.s_cnt, nacc * Bc));
  TRY(dalloc(g, &b.s_pre, nacc * Bc));
  TRY(dalloc(g, &b.s_base, nacc));
  TRY(dalloc(g, &b.s_qbase, na));
  TRY(dalloc(g, &b.s_sink, na));
  TRY(dalloc(g, &b.s_rsnap, g->fifos.size()));
  TRY(upload(g, (uint32_t **)&b.fifo_wacc, fifo_wacc));
  return PRUNE_OK;
}

CtrlArgs make_args(prune_graph *g, uint32_t B) {
  CtrlArgs c;
  memset(&c, 0, sizeof c);
  c.fifos = g->d_fifos; c.ports = g->d_ports; c.actors = g->d_actors; c.fbs = g->d_fbs;
  c.comp_off = g->d_comp_off; c.comp_actors = g->d_comp_actors;
  c.B = B; c.Bcap = g->Bcap; c.tile = g->tile; c.clear_n = 0;
  c.n_fifos = (uint32_t)g->fifos.size();
  c.recs = g->d_recs; c.wrote = g->d_wrote;
  c.fb_desc = g->d_desc; c.desc_off = g->d_desc_off;
  c.fb_items = g->d_items; c.fb_item_off = g->d_item_off; c.fb_count = g->d_ctr;
  c.copy_items = g->d_copy; c.copy_item_off = g->d_copy_off; c.copy_count = g->d_ctr + g->n_levels;
  c.level_of = g->d_level_of;
  c.halo_scratch = g->d_halo_scratch; c.halo_off = g->d_halo_off;
  c.gather_items = g->d_gather; c.gather_off = g->d_gather_off;
  c.gather_count = g->d_ctr + 3 * g->n_levels;
  c.err = g->d_err; c.clear_ptr = g->d_ctr;
  c.trace.rec = g->d_trace; c.trace.cap = g->trace_cap; c.trace.count = g->d_trace_count;
  return c;
}

void fb_launch_timed(prune_graph *g, uint32_t level, uint32_t grid, hipStream_t s) {
  const uint32_t nl = g->n_levels;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (g_timing) {   // events that cannot be created leave the launch untimed
    if (hipEventCreate(&e0) != hipSuccess) e0 = nullptr;
    if (hipEventCreate(&e1) != hipSuccess) e1 = nullptr;
    if (!e0 || !e1) {
      timing_push(e0, e1);   // releases the one that exists
      e0 = e1 = nullptr;
    }
  }
  fb_forward_launch(g->variant, g->d_desc, g->d_items + g->fb_item_off[level], g->d_ctr + level,
                    (unsigned int *)(g->d_ctr + 2 * nl + level), grid, s, e0, e1);
  if (e0) timing_push(e0, e1);
}

void timing_reset() {
  for (auto &e : g_events) {
    if (e.first) (void)hipEventDestroy(e.first);
    if (e.second) (void)hipEventDestroy(e.second);
  }
  g_events.clear();
  g_fb_ms = 0.f;
  g_fb_launches = 0;
}

// ---------------------------------------------------------------- per-firing
bool port_active(const prune_graph *g, const HPort &p, const prune_ctrl_token *tok) {
  if (p.kind != PRUNE_DRP) return true;
  uint32_t ctl = controller_port(g, g->actors[p.actor]);
  auto it = g->table.find({ctl, (uint32_t)(&p - g->ports.data())});
  uint32_t e = it == g->table.end() ? 0 : it->second;
  return tok && decode_bit(tok->mask, e);
}

bool can_fire(prune_graph *g, uint32_t aid) {
  HActor &A = g->actors[aid];
  if (A.kind == PRUNE_SOURCE && A.src_q.empty()) return false;
  if (A.kind == PRUNE_CONFIG && A.side_q.empty()) return false;
  const prune_ctrl_token *tok = nullptr;
  int64_t cf = cport_fifo(g, A);
  if (cf >= 0) {
    HFifo &F = g->fifos[cf];
    if (F.mirror.empty()) return false;
    tok = &F.mirror.front();
  }
  for (uint32_t p : A.ports) {
    const HPort &P = g->ports[p];
    if (P.kind == PRUNE_CPORT) continue;
    if (!port_active(g, P, tok)) continue;
    for (uint32_t f : P.fifos) {
      const HFifo &F = g->fifos[f];
      if (P.dir == PRUNE_IN) {
        if (!fifo_can_read(F.rate, F.delay, g->C, F.inflight)) return false;
      } else if (!fifo_can_write(F.rate, F.delay, g->C, F.inflight)) {
        return false;
      }
    }
  }
  return true;
}

// ---------------------------------------------------------------- end of a run
// A per-firing run stopped (nothing can fire): classify the stop on a plain
// view of the graph's host state (stop_rules.cpp).  A normal end returns
// PRUNE_OK; actors stuck round a cycle of waits, or dynamic actors waiting on
// data their linked partner's firing did not send, give PRUNE_E_DEADLOCK.
prune_status classify_stop(prune_graph *g) {
  std::vector<StopActor> va(g->actors.size());
  std::vector<StopPort> vp(g->ports.size());
  std::vector<StopFifo> vf(g->fifos.size());
  for (uint32_t f = 0; f < g->fifos.size(); ++f) {
    const HFifo &F = g->fifos[f];
    vf[f] = {F.src, F.dst, F.rate, F.delay, F.inflight};
  }
  for (uint32_t p = 0; p < g->ports.size(); ++p) {
    const HPort &P = g->ports[p];
    vp[p].actor = P.actor;
    vp[p].dir = P.dir;
    vp[p].kind = P.kind;
    vp[p].fifos = P.fifos;
    vp[p].element = 0;
    if (P.kind == PRUNE_DRP && !P.internal) {
      auto it = g->table.find({controller_port(g, g->actors[P.actor]), p});
      if (it != g->table.end()) vp[p].element = it->second;
    }
  }
  for (uint32_t a = 0; a < g->actors.size(); ++a) {
    const HActor &A = g->actors[a];
    StopActor &V = va[a];
    V.kind = A.kind;
    V.exhausted = (A.kind == PRUNE_SOURCE && A.src_q.empty()) || (A.kind == PRUNE_CONFIG && A.side_q.empty());
    V.cport_fifo = cport_fifo(g, A);
    V.has_token = V.cport_fifo >= 0 && !g->fifos[V.cport_fifo].mirror.empty();
    V.token_mask = V.has_token ? g->fifos[V.cport_fifo].mirror.front().mask : 0u;
    V.firings = A.firings;
    V.ports = A.ports;
  }
  const StopResult r = classify_stop_view(va, vp, vf, g->C);
  if (r.stuck.empty() && r.linked.empty()) return PRUNE_OK;
  std::string msg = "no actor can fire;";
  if (!r.stuck.empty()) {
    msg += " actors waiting round a cycle:";
    for (uint32_t a : r.stuck) msg += " " + std::to_string(a);
    msg += ";";
  }
  if (!r.linked.empty()) {
    msg += " dynamic actors waiting on data their linked partner's firing did not send:";
    for (uint32_t a : r.linked) msg += " " + std::to_string(a);
  }
  return fail(PRUNE_E_DEADLOCK, msg);
}

prune_status fire_one(prune_graph *g, uint32_t aid, hipStream_t s) {
  HActor &A = g->actors[aid];
  const prune_ctrl_token *tok = nullptr;
  prune_ctrl_token tk{};
  int64_t cf = cport_fifo(g, A);
  if (cf >= 0) {
    tk = g->fifos[cf].mirror.front();
    g->fifos[cf].mirror.pop_front();
    g->fifos[cf].inflight--;
    tok = &tk;
  }
  uint32_t max_count = 0;
  for (uint32_t p : A.ports) {
    const HPort &P = g->ports[p];
    if (P.kind == PRUNE_CPORT) continue;
    if (!port_active(g, P, tok)) continue;
    max_count = std::max(max_count, P.atr);
    for (uint32_t f : P.fifos) g->fifos[f].inflight += P.dir == PRUNE_IN ? -1 : 1;
  }
  const void *src_ptr = nullptr;
  if (A.kind == PRUNE_SOURCE) {
    src_ptr = A.src_q.front().ptr;
    A.src_q.pop_front();
  }
  if (A.kind == PRUNE_CONFIG) {
    const prune_side_info side = A.side_q.front();
    A.side_q.pop_front();
    const prune_ctrl_token t = config_map(A.cfg.mode, A.cfg.Kmax, side);
    for (uint32_t p : A.ports)
      for (uint32_t f : g->ports[p].fifos) g->fifos[f].mirror.push_back(t);
  }
  A.firings++;
  A.q_head += (A.kind == PRUNE_SOURCE || A.kind == PRUNE_CONFIG) ? 1 : 0;
  // device work: bookkeeping of this single firing, then its data kernel
  CtrlArgs c = make_args(g, 1);
  c.comp_off = g->d_single_off;
  c.comp_actors = g->d_iota + aid;
  c.clear_n = 4 * g->n_levels;
  c.per_firing = 1;
  launch_control(c, 1, s);
  const uint32_t l = A.level;
  if (A.kind == PRUNE_FILTERBANK) {
    const uint32_t n = in_atr(g, A);
    fb_launch_timed(g, l, std::min<uint32_t>(g->fb_grid, (n + g->tile - 1) / g->tile), s);
  } else if (is_copy_kind(A.kind)) {
    const bool needs_copy = (A.kind != PRUNE_SOURCE && A.kind != PRUNE_SINK) ||
                            (A.kind == PRUNE_SINK && A.sink_out) ||
                            (A.kind == PRUNE_SOURCE && src_ptr != nullptr);
    if (needs_copy)
      launch_copy(g->d_copy + g->copy_item_off[l], g->d_ctr + g->n_levels + l,
                  std::max<uint32_t>(1, out_accesses(g, A)), is_pixel_kind(A.kind) ? 0 : max_count,
                  is_pixel_kind(A.kind) ? A.pix.H : 0, s);
  }
  if (A.hist_len) launch_post(c, g->d_iota + aid, 1, s);
  // FIFOs with an unaligned delay: copy the overflow of this write back
  uint32_t k = 0;
  for (uint32_t p : A.ports) {
    const HPort &P = g->ports[p];
    if (P.kind == PRUNE_CPORT || P.dir != PRUNE_OUT) continue;
    for (uint32_t f : P.fifos) {
      const HFifo &F = g->fifos[f];
      if (F.delay % F.rate) launch_copyback(c, aid, f, k, s);
      ++k;
    }
  }
  return PRUNE_OK;
}

}  // namespace

namespace prune {
void timing_restart() { timing_reset(); }
}  // namespace prune

// ======================================================================
// C ABI
// ======================================================================
namespace {

prune_status check_graph(prune_graph *g, bool need_final, bool need_device = true) {
  if (!g) return fail(PRUNE_E_ARG, "null graph");
  if (need_final && need_device && g->host_only) return fail(PRUNE_E_STATE, "host-only graph");
  if (need_final && !g->finalized) return fail(PRUNE_E_STATE, "graph not finalized");
  if (!need_final && g->finalized) return fail(PRUNE_E_STATE, "graph already finalized");
  return PRUNE_OK;
}

prune_status ensure_ring(prune_graph *g, HActor &A, size_t entry, uint64_t need) {
  (void)g;
  // a write that would reach ring positions of entries the device may not
  // have read yet waits for the device first
  if (A.q_dev && A.q_tail + need > A.q_synced + A.q_cap) {
    HIPCHECK(hipDeviceSynchronize());
    A.q_synced = A.q_head;
  }
  const uint64_t live = A.q_tail - A.q_head;
  if (A.q_dev && live + need <= A.q_cap) return PRUNE_OK;
  uint64_t cap = std::max<uint64_t>(1024, A.q_cap);
  while (cap < live + need) cap *= 2;
  char *nq = nullptr, *lin = nullptr;
  HIPCHECK(hipDeviceSynchronize());
  HIPCHECK(hipMalloc((void **)&nq, cap * entry));
  if (A.q_dev && live) {
    // linearise the live entries, then place them at their positions mod cap
    HIPCHECK(hipMalloc((void **)&lin, live * entry));
    const uint64_t h = A.q_head % A.q_cap;
    const uint64_t run1 = std::min<uint64_t>(live, A.q_cap - h);
    HIPCHECK(hipMemcpy(lin, (char *)A.q_dev + h * entry, run1 * entry, hipMemcpyDeviceToDevice));
    if (live > run1)
      HIPCHECK(hipMemcpy(lin + run1 * entry, A.q_dev, (live - run1) * entry, hipMemcpyDeviceToDevice));
    const uint64_t h2 = A.q_head % cap;
    const uint64_t run2 = std::min<uint64_t>(live, cap - h2);
    HIPCHECK(hipMemcpy(nq + h2 * entry, lin, run2 * entry, hipMemcpyDeviceToDevice));
    if (live > run2)
      HIPCHECK(hipMemcpy(nq, lin + run2 * entry, (live - run2) * entry, hipMemcpyDeviceToDevice));
    HIPCHECK(hipFree(lin));
  }
  if (A.q_dev) HIPCHECK(hipFree(A.q_dev));
  A.q_dev = nq;
  A.q_cap = cap;
  A.q_synced = A.q_head;   // the device was synchronized above
  return PRUNE_OK;
}

prune_status ring_write(HActor &A, size_t entry, const void *host, uint64_t n) {
  const char *src = (const char *)host;
  uint64_t k = 0;
  while (k < n) {
    const uint64_t pos = (A.q_tail + k) % A.q_cap;
    const uint64_t run = std::min<uint64_t>(n - k, A.q_cap - pos);
    HIPCHECK(hipMemcpy((char *)A.q_dev + pos * entry, src + k * entry, run * entry,
                       hipMemcpyHostToDevice));
    k += run;
  }
  A.q_tail += n;
  return PRUNE_OK;
}

// Levels whose copy kernel can have work in this batch, and levels whose
// stateful actors can see a previous frame shorter than their history.
void launch_masks(prune_graph *g, uint32_t B, uint64_t *copy_mask, uint64_t *gather_mask) {
  *copy_mask = 0;
  *gather_mask = 0;
  for (auto &A : g->actors) {
    const uint64_t bit = 1ull << std::min<uint32_t>(A.level, 63);
    if (A.kind == PRUNE_SWITCH || A.kind == PRUNE_POLY || A.kind == PRUNE_SELECT || A.kind == PRUNE_PASSTHROUGH ||
        A.kind == PRUNE_GAUSS5 || A.kind == PRUNE_THRES || A.kind == PRUNE_MED5)
      *copy_mask |= bit;
    if (A.kind == PRUNE_SINK && A.sink_out) *copy_mask |= bit;
    if (A.kind == PRUNE_SOURCE) {
      for (uint32_t k = 0; k < B && k < A.src_q.size(); ++k)
        if (A.src_q[k].ptr) { *copy_mask |= bit; break; }
    }
    if (A.hist_len && B > 1) {
      for (uint32_t p : A.ports) {
        const HPort &P = g->ports[p];
        if (P.dir == PRUNE_IN && P.kind == PRUNE_SRP &&
            ((P.flags & PRUNE_PORT_PARAM) || P.atr < A.hist_len))
          *gather_mask |= bit;
      }
    }
  }
}

// Point the graph's per-batch buffers at set p (kernels take the pointers by
// value at launch).
void use_set(prune_graph *g, uint32_t p) {
  const prune_graph::BatchSet &S = g->sets[p];
  g->d_recs = S.recs; g->d_wrote = S.wrote; g->d_desc = S.desc; g->d_items = S.items;
  g->d_copy = S.copy; g->d_halo_scratch = S.halo_scratch; g->d_ctr = S.ctr; g->d_gather = S.gather;
}

prune_status run_batch(prune_graph *g, uint32_t B, hipStream_t s, bool use_graph) {
  uint64_t cmask, gmask;
  launch_masks(g, B, &cmask, &gmask);
  auto bookkeeping = [&](hipStream_t st) {
    CtrlArgs c = make_args(g, B);
    if (g->fast_batch) {
      c.clear_n = 4 * g->n_levels;
      launch_batch(c, g->bargs, g->n_comp, (uint32_t)g->actors.size(), st);
    } else {
      launch_clear(g->d_ctr, 4 * g->n_levels, st);
      launch_control(c, g->n_comp, st);
    }
  };
  // the next batch's bookkeeping is issued beside this batch's data kernels
  const bool pipelined = g->fast_batch && g->side_stream && g_pipeline;
  auto data = [&](hipStream_t st) {
    CtrlArgs c = make_args(g, B);
    for (uint32_t l = 0; l < g->n_levels; ++l) {
      const uint64_t bit = 1ull << std::min<uint32_t>(l, 63);
      if ((gmask & bit) && g->gather_cap[l])
        launch_gather(make_args(g, B), l, std::min<uint32_t>(g->gather_cap[l], 256), st);
      if ((cmask & bit) && g->level_copy[l])
        launch_copy(g->d_copy + g->copy_item_off[l], g->d_ctr + g->n_levels + l,
                    g->copy_item_cap[l], g->copy_max_total[l], g->copy_pix_rows[l], st);
      if (g->level_fb[l]) fb_launch_timed(g, l, g->fb_grid, st);
    }
    launch_post(c, g->d_post_actors, (uint32_t)g->post_actors.size(), st);
  };
  auto enqueue = [&](hipStream_t st) {
    bookkeeping(st);
    data(st);
  };
  const uint64_t key = (uint64_t)B | (cmask << 20) | (gmask << 42);
  // capture fn's launches once into a graph kept in (execs, defs) under key
  auto captured = [&](std::map<uint64_t, hipGraphExec_t> &execs, std::map<uint64_t, hipGraph_t> &defs,
                      const std::function<void(hipStream_t)> &fn, hipGraphExec_t *out) -> prune_status {
    auto it = execs.find(key);
    if (it == execs.end()) {
      if (!g->capture_stream) HIPCHECK(hipStreamCreateWithFlags(&g->capture_stream, hipStreamNonBlocking));
      HIPCHECK(hipStreamSynchronize(s));
      const bool was = g_timing;
      g_timing = false;
      HIPCHECK(hipStreamBeginCapture(g->capture_stream, hipStreamCaptureModeRelaxed));
      fn(g->capture_stream);
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(g->capture_stream, &graph);
      g_timing = was;
      HIPCHECK(e);
      hipGraphExec_t exec = nullptr;
      HIPCHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      defs[key] = graph;
      it = execs.emplace(key, exec).first;
    }
    *out = it->second;
    return PRUNE_OK;
  };
  if (pipelined) {
    // pipelined: bookkeeping on the side stream into set p, data kernels on
    // the caller's stream once it is done; set p is reused only after the
    // data kernels of the batch that last used it.  The graph form replays
    // the same two parts as two captured graphs per set, in the same order.
    const uint32_t p = g->parity;
    use_set(g, p);
    hipStream_t b = g->side_stream;
    hipGraphExec_t gbk = nullptr, gdata = nullptr;
    if (use_graph) {
      TRY(captured(g->pgraphs[p][0], g->pgraph_defs[p][0], bookkeeping, &gbk));
      TRY(captured(g->pgraphs[p][1], g->pgraph_defs[p][1], data, &gdata));
    }
    if (g->need_sync) {
      HIPCHECK(hipEventRecord(g->ev_sync, s));
      HIPCHECK(hipStreamWaitEvent(b, g->ev_sync, 0));
      g->need_sync = false;
    } else if (g->done_valid[p]) {
      HIPCHECK(hipStreamWaitEvent(b, g->ev_done[p], 0));
    }
    if (use_graph)
      HIPCHECK(hipGraphLaunch(gbk, b));
    else
      bookkeeping(b);
    HIPCHECK(hipEventRecord(g->ev_emit[p], b));
    HIPCHECK(hipStreamWaitEvent(s, g->ev_emit[p], 0));
    if (use_graph)
      HIPCHECK(hipGraphLaunch(gdata, s));
    else
      data(s);
    HIPCHECK(hipEventRecord(g->ev_done[p], s));
    g->done_valid[p] = true;
    g->parity ^= 1u;
    HIPCHECK(hipGetLastError());
    return PRUNE_OK;
  }
  // single-stream forms use set 0; the next pipelined batch waits for them
  use_set(g, 0);
  g->need_sync = true;
  if (!use_graph) {
    enqueue(s);
    HIPCHECK(hipGetLastError());
    return PRUNE_OK;
  }
  hipGraphExec_t exec = nullptr;
  TRY(captured(g->graphs, g->graph_defs, enqueue, &exec));
  HIPCHECK(hipGraphLaunch(exec, s));
  return PRUNE_OK;
}

}  // namespace

// The graph's structure as the compile-time analysis reads it.
static void run_design_analysis(prune_graph *g) {
  prune::DesignGraph d;
  d.kind.reserve(g->actors.size());
  for (const HActor &A : g->actors) {
    d.kind.push_back(A.kind);
    d.ports.push_back(A.ports);
  }
  d.port.reserve(g->ports.size());
  for (const HPort &P : g->ports) d.port.push_back({P.actor, P.dir, P.kind, P.internal ? std::vector<uint32_t>{} : P.fifos});
  d.fifo.reserve(g->fifos.size());
  for (const HFifo &F : g->fifos) d.fifo.push_back({F.src, F.dst, F.rate, F.delay});
  d.table = g->table;
  g->report = prune::analyze_design(d);
  g->analyzed = true;
}

extern "C" {

prune_status prune_graph_set_checks(prune_graph_t g, uint32_t flags) {
  if (!g) return fail(PRUNE_E_ARG, "null graph");
  if (flags & ~(uint32_t)PRUNE_CHECK_RULES) return fail(PRUNE_E_ARG, "unknown check flags");
  g->checks = flags;
  return PRUNE_OK;
}

prune_status prune_graph_analyze(prune_graph_t g, prune_analysis_counts *counts) {
  if (!g) return fail(PRUNE_E_ARG, "null graph");
  run_design_analysis(g);
  if (counts) {
    counts->n_linked = (uint32_t)g->report.linked.size();
    counts->n_dpgs = (uint32_t)g->report.dpgs.size();
    counts->n_dcs = (uint32_t)g->report.dcs.size();
    counts->n_violations = (uint32_t)g->report.violations.size();
  }
  return PRUNE_OK;
}

prune_status prune_graph_analysis_table(prune_graph_t g, int table, int64_t *out, size_t cap,
                                        size_t *n) {
  if (!g || !n || (cap && !out)) return fail(PRUNE_E_ARG, "null argument");
  if (!g->analyzed) return fail(PRUNE_E_STATE, "no analysis yet");
  const prune::DesignReport &R = g->report;
  std::vector<int64_t> v;
  switch (table) {
    case PRUNE_AN_LINKED:
      for (auto &e : R.linked) v.insert(v.end(), e.begin(), e.end());
      break;
    case PRUNE_AN_DPGS:
      for (auto &e : R.dpgs) v.insert(v.end(), e.begin(), e.end());
      break;
    case PRUNE_AN_DCS:
      for (auto &e : R.dcs) v.insert(v.end(), {e.dpg, e.element, e.direct_fifo, (int64_t)e.actors.size()});
      break;
    case PRUNE_AN_DC_ACTORS:
      for (auto &e : R.dcs) v.insert(v.end(), e.actors.begin(), e.actors.end());
      break;
    case PRUNE_AN_ACTOR_DC:
      v = R.dc_of_actor;
      break;
    case PRUNE_AN_BETA:
      v = R.beta;
      break;
    case PRUNE_AN_VIOLATIONS:
      for (auto &e : R.violations) v.insert(v.end(), e.begin(), e.end());
      break;
    default:
      return fail(PRUNE_E_ARG, "unknown analysis table");
  }
  *n = v.size();
  std::copy(v.begin(), v.begin() + std::min(cap, v.size()), out);
  return PRUNE_OK;
}

prune_status prune_graph_create(int hip_device, prune_graph_t *out) {
  if (!out) return fail(PRUNE_E_ARG, "null output");
  if (hip_device < -1) return fail(PRUNE_E_ARG, "bad device");
  if (hip_device >= 0) HIPCHECK(hipSetDevice(hip_device));
  prune_graph *g = new prune_graph();
  g->device = hip_device;
  g->host_only = hip_device < 0;
  if (g->host_only) {
    *out = g;
    return PRUNE_OK;
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && ncu > 0)
    g->ncu = ncu;
  *out = g;
  return PRUNE_OK;
}

prune_status prune_graph_destroy(prune_graph_t g) {
  if (!g) return fail(PRUNE_E_ARG, "null graph");
  if (!g->host_only) (void)hipDeviceSynchronize();
  delete g;
  return PRUNE_OK;
}

prune_status prune_actor_create(prune_graph_t g, int kind, const void *params, size_t bytes,
                                prune_id *actor) {
  TRY(check_graph(g, false));
  if (!actor || kind < PRUNE_SOURCE || kind > PRUNE_MED5) return fail(PRUNE_E_ARG, "bad actor kind");
  HActor a;
  a.kind = (uint32_t)kind;
  if (kind == PRUNE_CONFIG) {
    if (!params || bytes != sizeof(prune_config_params)) return fail(PRUNE_E_ARG, "config params expected");
    a.cfg = *(const prune_config_params *)params;
    if (a.cfg.mode > PRUNE_CONFIG_MASK || a.cfg.n_elements > 32) return fail(PRUNE_E_ARG, "bad config params");
  } else if (kind == PRUNE_FILTERBANK) {
    if (!params || bytes != sizeof(prune_fb_params)) return fail(PRUNE_E_ARG, "filter-bank params expected");
    a.fb = *(const prune_fb_params *)params;
    if (a.fb.n_banks < 1 || a.fb.Kmax < 1) return fail(PRUNE_E_ARG, "filter bank needs banks and branches");
    if (a.fb.n_banks > PRUNE_MAX_BANKS || a.fb.Kmax > 10 || a.fb.n_banks * a.fb.Kmax > PRUNE_MAX_BRANCHES)
      return fail(PRUNE_E_UNSUPPORTED, "at most 4 banks of 10 branches (32 in total)");
    for (uint32_t b = 0; b < a.fb.n_banks; ++b)
      if (a.fb.L[b] < 1 || a.fb.L[b] > PRUNE_MAX_L) return fail(PRUNE_E_UNSUPPORTED, "taps per branch must be 1..64");
  } else if (kind == PRUNE_GAUSS5 || kind == PRUNE_THRES || kind == PRUNE_MED5) {
    if (!params || bytes != sizeof(prune_pixel_params)) return fail(PRUNE_E_ARG, "pixel params expected");
    a.pix = *(const prune_pixel_params *)params;
    if (a.pix.W < 1 || a.pix.H < 1 || (uint64_t)a.pix.W * a.pix.H > 0xffffffffull ||
        ((uint64_t)a.pix.W * a.pix.H) % 8)
      return fail(PRUNE_E_ARG, "frame sizes must be positive with W*H a multiple of 8");
    if (a.pix.W % 4) return fail(PRUNE_E_UNSUPPORTED, "frame width must be a multiple of 4");
  } else if (params && bytes) {
    return fail(PRUNE_E_ARG, "this actor kind takes no parameters");
  }
  const uint32_t id = (uint32_t)g->actors.size();
  if (kind == PRUNE_FILTERBANK) {
    for (uint32_t d = 0; d < a.fb.n_banks * a.fb.Kmax; ++d) {
      HPort p{};
      p.actor = id; p.dir = 2; p.kind = PRUNE_DRP; p.atr = 1; p.token_bytes = 8; p.flags = 0; p.halo = 0;
      p.internal = true;
      a.branches.push_back((uint32_t)g->ports.size());
      g->ports.push_back(p);
    }
  }
  g->actors.push_back(a);
  *actor = id;
  return PRUNE_OK;
}

prune_status prune_port_create(prune_graph_t g, prune_id actor, int dir, int kind, uint32_t atr,
                               uint32_t token_bytes, uint32_t flags, uint32_t halo, prune_id *port) {
  TRY(check_graph(g, false));
  if (!port || actor >= g->actors.size() || (dir != PRUNE_IN && dir != PRUNE_OUT) ||
      kind < PRUNE_SRP || kind > PRUNE_CPORT || atr == 0 || token_bytes == 0 || (flags & ~1u))
    return fail(PRUNE_E_ARG, "bad port arguments");
  if (kind == PRUNE_CPORT && (dir != PRUNE_IN || token_bytes != sizeof(prune_ctrl_token)))
    return fail(PRUNE_E_PORT_KIND, "a control port is an input of 8-byte control tokens");
  HActor &A = g->actors[actor];
  const bool byte_ok = A.kind == PRUNE_SOURCE || A.kind == PRUNE_SINK || A.kind == PRUNE_PASSTHROUGH ||
                       A.kind == PRUNE_GAUSS5 || A.kind == PRUNE_THRES || A.kind == PRUNE_MED5;
  if (A.kind != PRUNE_CONFIG && kind != PRUNE_CPORT && token_bytes != 8 && !(token_bytes == 1 && byte_ok))
    return fail(PRUNE_E_UNSUPPORTED, "data tokens are complex64 (8 bytes), or pixels (1 byte)");
  HPort p{};
  p.actor = actor; p.dir = (uint32_t)dir; p.kind = (uint32_t)kind; p.atr = atr;
  p.token_bytes = token_bytes; p.flags = flags; p.halo = halo;
  A.ports.push_back((uint32_t)g->ports.size());
  *port = (uint32_t)g->ports.size();
  g->ports.push_back(p);
  return PRUNE_OK;
}

prune_status prune_filterbank_branch(prune_graph_t g, prune_id fb, uint32_t d, prune_id *drp) {
  if (!g || !drp || fb >= g->actors.size() || g->actors[fb].kind != PRUNE_FILTERBANK ||
      d >= g->actors[fb].branches.size())
    return fail(PRUNE_E_ARG, "no such filter-bank branch");
  *drp = g->actors[fb].branches[d];
  return PRUNE_OK;
}

prune_status prune_fifo_connect(prune_graph_t g, prune_id src, prune_id dst, uint32_t rate,
                                uint32_t delay, prune_id *fifo) {
  TRY(check_graph(g, false));
  if (!fifo || src >= g->ports.size() || dst >= g->ports.size()) return fail(PRUNE_E_ARG, "unknown port");
  HPort &ps = g->ports[src], &pd = g->ports[dst];
  if (ps.internal || pd.internal || ps.dir != PRUNE_OUT || pd.dir != PRUNE_IN)
    return fail(PRUNE_E_CONNECT, "a FIFO runs from an output port to an input port");
  if (!pd.fifos.empty()) return fail(PRUNE_E_CONNECT, "an input port has exactly one FIFO");
  if (rate == 0) return fail(PRUNE_E_ARG, "fiforate must be positive");
  HFifo f{};
  f.src = src; f.dst = dst; f.rate = rate; f.delay = delay; f.token_bytes = ps.token_bytes;
  f.ctrl = pd.kind == PRUNE_CPORT;
  f.param = (ps.flags & PRUNE_PORT_PARAM) != 0;
  const uint32_t id = (uint32_t)g->fifos.size();
  ps.fifos.push_back(id);
  pd.fifos.push_back(id);
  g->fifos.push_back(f);
  *fifo = id;
  return PRUNE_OK;
}

prune_status prune_control_table_set(prune_graph_t g, prune_id ctl, prune_id drp, uint32_t element) {
  TRY(check_graph(g, false));
  if (ctl >= g->ports.size() || drp >= g->ports.size() || element > 32)
    return fail(PRUNE_E_ARG, "bad control-table entry");
  g->table[{ctl, drp}] = element;
  return PRUNE_OK;
}

prune_status prune_graph_finalize(prune_graph_t g, uint32_t C) {
  TRY(check_graph(g, false));
  if (C == 0) return fail(PRUNE_E_ARG, "C must be positive");
  // the batch kernels put actors (and components) on a grid's y dimension
  if (g->actors.size() > 65535) return fail(PRUNE_E_UNSUPPORTED, "at most 65535 actors per graph");
  if (g->checks & PRUNE_CHECK_RULES) {
    run_design_analysis(g);
    if (!g->report.violations.empty()) {
      const auto &v = g->report.violations.front();
      return fail(PRUNE_E_RULE, "design analysis: violation code " + std::to_string(v[0]) + " (" +
                                    std::to_string(v[1]) + ", " + std::to_string(v[2]) + "), " +
                                    std::to_string(g->report.violations.size()) + " in total");
    }
  }
  for (uint32_t p = 0; p < g->ports.size(); ++p) {
    const HPort &P = g->ports[p];
    if (P.internal) continue;
    if (P.dir == PRUNE_IN && P.fifos.size() != 1)
      return fail(PRUNE_E_CONNECT, "input port " + std::to_string(p) + " needs exactly one FIFO");
    if (P.dir == PRUNE_OUT && P.fifos.empty())
      return fail(PRUNE_E_CONNECT, "output port " + std::to_string(p) + " is not connected");
  }
  for (uint32_t f = 0; f < g->fifos.size(); ++f) {
    HFifo &F = g->fifos[f];
    const HPort &ps = g->ports[F.src], &pd = g->ports[F.dst];
    if (ps.atr != F.rate || pd.atr != F.rate)
      return fail(PRUNE_E_RATE_MISMATCH, "fifo " + std::to_string(f) + ": atr differs from fiforate");
    if (ps.flags != pd.flags || ps.halo != pd.halo || ps.token_bytes != pd.token_bytes)
      return fail(PRUNE_E_RATE_MISMATCH, "fifo " + std::to_string(f) + ": port parameterisation differs");
    if (F.param && F.delay) return fail(PRUNE_E_DELAY, "delay on a parameterised FIFO");
    const uint32_t r = F.rate, Q = F.delay;
    if ((Q % r) && (Q >= (uint64_t)r * C || (Q < r && Q + r > (uint64_t)r * C)))
      return fail(PRUNE_E_DELAY, "fifo " + std::to_string(f) + ": unaligned delay does not fit r*C");
    if (F.ctrl != (g->actors[ps.actor].kind == PRUNE_CONFIG))
      return fail(PRUNE_E_PORT_KIND, "control ports connect only to configuration actors");
    F.capacity = fifo_capacity(r, Q, C);
  }
  g->C = C;
  for (uint32_t a = 0; a < g->actors.size(); ++a) TRY(validate_actor(g, a));
  TRY(analyse(g));
  if (g->host_only) {
    g->finalized = true;
    return PRUNE_OK;
  }
  TRY(build_device(g));
  g->Bcap = std::max<uint32_t>(1, std::min<uint32_t>(C, 1u << 16));
  // A batch runs every iteration of one level before the next level, so a
  // FIFO with an aligned delay of Q/r blocks holds Q/r + B blocks at once.
  for (auto &F : g->fifos)
    if (F.delay && F.delay % F.rate == 0) {
      const uint64_t blocks = F.capacity / F.rate, pre = F.delay / F.rate;
      g->Bcap = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g->Bcap, blocks > pre ? blocks - pre : 1));
    }
  {
    // tuned on the structure of the filter bank with the most work per
    // sample (first such one): its banks, branch count and input rate
    const HActor *best = nullptr;
    for (auto &A : g->actors)
      if (A.kind == PRUNE_FILTERBANK &&
          (!best || fb_lmax(A.fb) * A.fb.Kmax > fb_lmax(best->fb) * best->fb.Kmax))
        best = &A;
    g->variant = 1;
    if (best) {
      bool param = false;
      for (uint32_t p : best->ports)
        if (g->ports[p].dir == PRUNE_IN && g->ports[p].kind != PRUNE_CPORT)
          param = (g->ports[p].flags & PRUNE_PORT_PARAM) != 0;
      const uint32_t n = std::max<uint32_t>(1, in_atr(g, *best) - (best->fb.windowed ? fb_lmax(best->fb) - 1 : 0));
      g->variant = choose_variant_graph(best->fb.n_banks, best->fb.L, best->fb.Kmax, n, param);
    }
  }
  g->tile = (uint32_t)fb_variant_tile(g->variant);
  g->fb_grid = g->ncu * (uint32_t)fb_variant_resident(g->variant);   // every workgroup slot
  TRY(alloc_scratch(g));
  if (g->fast_batch) {
    HIPCHECK(hipStreamCreateWithFlags(&g->side_stream, hipStreamNonBlocking));
    for (hipEvent_t *e : {&g->ev_emit[0], &g->ev_emit[1], &g->ev_done[0], &g->ev_done[1], &g->ev_sync})
      HIPCHECK(hipEventCreateWithFlags(e, hipEventDisableTiming));
  }
  g->finalized = true;
  return PRUNE_OK;
}

prune_status prune_fifo_required_bytes(prune_graph_t g, prune_id fifo, size_t *bytes) {
  TRY(check_graph(g, true, false));
  if (!bytes || fifo >= g->fifos.size()) return fail(PRUNE_E_ARG, "unknown fifo");
  *bytes = g->fifos[fifo].capacity * g->fifos[fifo].token_bytes;
  return PRUNE_OK;
}

prune_status prune_fifo_bind_storage(prune_graph_t g, prune_id fifo, void *dev_ptr, size_t bytes) {
  TRY(check_graph(g, true));
  if (fifo >= g->fifos.size() || !dev_ptr) return fail(PRUNE_E_ARG, "unknown fifo or null storage");
  HFifo &F = g->fifos[fifo];
  if (F.ctrl) return fail(PRUNE_E_ARG, "control FIFOs are library-owned");
  if (bytes < F.capacity * F.token_bytes) return fail(PRUNE_E_CAPACITY, "storage smaller than Eq. 2 capacity");
  F.storage = dev_ptr;
  F.bytes = bytes;
  char *b = (char *)dev_ptr;
  HIPCHECK(hipMemcpy(&g->d_fifos[fifo].base, &b, sizeof(char *), hipMemcpyHostToDevice));
  if (F.delay) HIPCHECK(hipMemset(dev_ptr, 0, F.capacity * F.token_bytes));   // delay tokens are zeros
  return PRUNE_OK;
}

prune_status prune_fifo_write_window(prune_graph_t g, prune_id fifo, uint32_t k, void **dev_ptr) {
  TRY(check_graph(g, true));
  if (fifo >= g->fifos.size() || !dev_ptr) return fail(PRUNE_E_ARG, "unknown fifo");
  HFifo &F = g->fifos[fifo];
  const HActor &w = g->actors[g->ports[F.src].actor];
  if (w.kind != PRUNE_SOURCE) return fail(PRUNE_E_ARG, "write windows are for source FIFOs");
  if (!F.storage) return fail(PRUNE_E_STATE, "storage not bound");
  const uint64_t j = w.firings + w.src_q.size() + k;
  *dev_ptr = (char *)F.storage + fifo_write_slot(F.rate, F.delay, g->C, j) * F.token_bytes;
  return PRUNE_OK;
}

prune_status prune_filterbank_set_taps(prune_graph_t g, prune_id fb, const void *dev_taps, size_t n,
                                       prune_stream_t stream) {
  TRY(check_graph(g, true));
  if (fb >= g->actors.size() || g->actors[fb].kind != PRUNE_FILTERBANK || !dev_taps)
    return fail(PRUNE_E_ARG, "not a filter bank");
  HActor &A = g->actors[fb];
  const size_t need = (size_t)A.fb.n_banks * A.fb.Kmax * fb_lmax(A.fb);
  if (n != need) return fail(PRUNE_E_ARG, "taps must be [n_banks][Kmax][Lmax]");
  HIPCHECK(hipMemcpyAsync(A.taps, dev_taps, n * sizeof(float2), hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
  return PRUNE_OK;
}

prune_status prune_actor_reset_history(prune_graph_t g, prune_id actor, prune_stream_t stream) {
  TRY(check_graph(g, true));
  if (actor >= g->actors.size()) return fail(PRUNE_E_ARG, "unknown actor");
  HActor &A = g->actors[actor];
  if (A.hist_len) HIPCHECK(hipMemsetAsync(A.history, 0, A.hist_len * sizeof(float2), (hipStream_t)stream));
  return PRUNE_OK;
}

prune_status prune_source_push(prune_graph_t g, prune_id src, const void *dev_samples,
                               const uint32_t *host_counts, uint32_t n) {
  TRY(check_graph(g, true));
  if (src >= g->actors.size() || g->actors[src].kind != PRUNE_SOURCE || (!host_counts && n))
    return fail(PRUNE_E_ARG, "not a source");
  HActor &A = g->actors[src];
  const HPort &P = g->ports[A.ports[0]];
  std::vector<SrcIn> ent(n);
  uint64_t off = 0;
  for (uint32_t f = 0; f < n; ++f) {
    const uint32_t c = host_counts[f];
    if ((P.flags & PRUNE_PORT_PARAM) ? (c < 1 || c > P.atr) : (c != P.atr))
      return fail(PRUNE_E_TOKEN, "frame length " + std::to_string(c) + " does not fit the source port");
    ent[f].count = c;
    ent[f].pad = 0;
    ent[f].ptr = dev_samples ? (const char *)dev_samples + off * P.token_bytes : nullptr;
    off += c;
  }
  TRY(ensure_ring(g, A, sizeof(SrcIn), n));
  TRY(ring_write(A, sizeof(SrcIn), ent.data(), n));
  TRY(sync_actor_dev(g, src));
  for (uint32_t f = 0; f < n; ++f) A.src_q.push_back({ent[f].count, ent[f].ptr});
  return PRUNE_OK;
}

prune_status prune_config_push(prune_graph_t g, prune_id cfg, const prune_side_info *side, uint32_t n,
                               prune_stream_t stream) {
  (void)stream;
  TRY(check_graph(g, true));
  if (cfg >= g->actors.size() || g->actors[cfg].kind != PRUNE_CONFIG || (!side && n))
    return fail(PRUNE_E_ARG, "not a configuration actor");
  HActor &A = g->actors[cfg];
  // side-information that addresses branches beyond a bank (the same records
  // the oracle's configuration actor rejects)
  for (uint32_t f = 0; f < n; ++f) {
    if (A.cfg.mode == PRUNE_CONFIG_PREFIX && side[f].K > A.cfg.Kmax)
      return fail(PRUNE_E_TOKEN, "record " + std::to_string(f) + ": K above the bank size");
    if (A.cfg.mode == PRUNE_CONFIG_MASK && A.cfg.Kmax < 32 && (side[f].K >> A.cfg.Kmax))
      return fail(PRUNE_E_TOKEN, "record " + std::to_string(f) + ": branch set beyond the bank size");
  }
  TRY(ensure_ring(g, A, sizeof(prune_side_info), n));
  TRY(ring_write(A, sizeof(prune_side_info), side, n));
  TRY(sync_actor_dev(g, cfg));
  for (uint32_t f = 0; f < n; ++f) A.side_q.push_back(side[f]);
  return PRUNE_OK;
}

prune_status prune_sink_bind_output(prune_graph_t g, prune_id snk, void *dev_out, uint64_t cap) {
  TRY(check_graph(g, true));
  if (snk >= g->actors.size() || g->actors[snk].kind != PRUNE_SINK) return fail(PRUNE_E_ARG, "not a sink");
  // batches in flight read the binding when their bookkeeping runs
  HIPCHECK(hipDeviceSynchronize());
  g->actors[snk].sink_out = dev_out;
  g->actors[snk].sink_cap = dev_out ? cap : 0;
  return sync_actor_dev(g, snk);
}

prune_status prune_graph_fire(prune_graph_t g, int mode, uint32_t max_firings, prune_stream_t stream,
                              uint64_t *fired) {
  TRY(check_graph(g, true));
  hipStream_t s = (hipStream_t)stream;
  for (uint32_t f = 0; f < g->fifos.size(); ++f)
    if (!g->fifos[f].storage) return fail(PRUNE_E_STATE, "fifo " + std::to_string(f) + " has no storage");
  uint64_t done = 0;
  if (mode == PRUNE_PER_FIRING) {
    // per-firing kernels update FIFO counters on the caller's stream: the
    // next pipelined batch's bookkeeping waits for them
    use_set(g, 0);
    g->need_sync = true;
    for (;;) {
      bool any = false;
      for (uint32_t a = 0; a < g->actors.size(); ++a) {
        if (max_firings && done >= max_firings) break;
        if (can_fire(g, a)) {
          TRY(fire_one(g, a, s));
          any = true;
          ++done;
        }
      }
      if (!any || (max_firings && done >= max_firings)) break;
    }
    HIPCHECK(hipGetLastError());
    if (fired) *fired = done;
    if (!max_firings || done < max_firings) return classify_stop(g);
    return PRUNE_OK;
  }
  if (mode != PRUNE_BATCHED && mode != PRUNE_BATCHED_GRAPH) return fail(PRUNE_E_ARG, "unknown mode");
  if (!g->dag || g->has_unaligned_delay)
    return fail(PRUNE_E_UNSUPPORTED, "batched firing needs a DAG whose delays are whole blocks");
  for (auto &F : g->fifos)
    if (F.inflight || !F.mirror.empty())
      return fail(PRUNE_E_STATE, "batched firing starts at an iteration boundary");
  for (;;) {
    uint64_t B = g->Bcap;
    bool any_src = false;
    for (auto &A : g->actors) {
      if (A.kind == PRUNE_SOURCE) { B = std::min<uint64_t>(B, A.src_q.size()); any_src = true; }
      if (A.kind == PRUNE_CONFIG) { B = std::min<uint64_t>(B, A.side_q.size()); any_src = true; }
    }
    if (!any_src) break;
    if (max_firings) B = std::min<uint64_t>(B, max_firings - done);
    if (B == 0) break;
    TRY(run_batch(g, (uint32_t)B, s, mode == PRUNE_BATCHED_GRAPH));
    for (auto &A : g->actors) {
      if (A.kind == PRUNE_SOURCE) {
        for (uint64_t k = 0; k < B; ++k) A.src_q.pop_front();
        A.firings += B;
        A.q_head += B;
      } else if (A.kind == PRUNE_CONFIG) {
        for (uint64_t k = 0; k < B; ++k) A.side_q.pop_front();
        A.firings += B;
        A.q_head += B;
      }
    }
    done += B;
    if (max_firings && done >= max_firings) break;
  }
  if (fired) *fired = done;
  return PRUNE_OK;
}

prune_status prune_graph_stream_host(prune_graph_t g, prune_id src, prune_id cfg, prune_id snk,
                                     const void *host_in, const prune_side_info *side, void *host_out,
                                     uint32_t n_frames, uint32_t batch, prune_stream_t stream) {
  TRY(check_graph(g, true));
  if (src >= g->actors.size() || g->actors[src].kind != PRUNE_SOURCE || cfg >= g->actors.size() ||
      g->actors[cfg].kind != PRUNE_CONFIG || snk >= g->actors.size() || g->actors[snk].kind != PRUNE_SINK)
    return fail(PRUNE_E_ARG, "src, cfg and snk must be a source, a configuration actor and a sink");
  if (n_frames && (!host_in || !side || !host_out)) return fail(PRUNE_E_ARG, "null host buffer");
  HActor &S = g->actors[src], &Q = g->actors[cfg], &K = g->actors[snk];
  const uint32_t fi = g->ports[S.ports[0]].fifos.at(0);
  uint32_t fo = kNone;
  for (uint32_t p : K.ports)
    if (g->ports[p].dir == PRUNE_IN && g->ports[p].kind != PRUNE_CPORT) fo = g->ports[p].fifos.at(0);
  if (fo == kNone || g->ports[S.ports[0]].fifos.size() != 1) return fail(PRUNE_E_ARG, "source or sink not connected");
  const HFifo &Fi = g->fifos[fi], &Fo = g->fifos[fo];
  if (Fi.param || Fo.param || Fi.delay || Fo.delay)
    return fail(PRUNE_E_UNSUPPORTED, "host streaming needs fixed-rate source and sink FIFOs without delay");
  if (!batch || g->C % batch || g->C < 2 * batch)
    return fail(PRUNE_E_ARG, "C must be a multiple of the batch and hold at least two batches");
  if (K.sink_out) return fail(PRUNE_E_STATE, "the sink must not have an output buffer bound");
  if (!S.src_q.empty() || !Q.side_q.empty()) return fail(PRUNE_E_STATE, "pending source or side input");
  if (!n_frames) return PRUNE_OK;
  hipStream_t s = (hipStream_t)stream;
  HIPCHECK(hipStreamSynchronize(s));
  HIPCHECK(hipDeviceSynchronize());
  FifoDev di, dout;
  HIPCHECK(hipMemcpy(&di, g->d_fifos + fi, sizeof di, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(&dout, g->d_fifos + fo, sizeof dout, hipMemcpyDeviceToHost));
  // every frame's side-information and (in-place) source entry up front
  std::vector<uint32_t> counts(n_frames, Fi.rate);
  TRY(prune_config_push(g, cfg, side, n_frames, stream));
  TRY(prune_source_push(g, src, nullptr, counts.data(), n_frames));

  const uint32_t depth = g->C / batch;   // batches the ring holds
  const uint32_t nb = (n_frames + batch - 1) / batch;
  const size_t bi = (size_t)Fi.rate * Fi.token_bytes, bo = (size_t)Fo.rate * Fo.token_bytes;
  hipStream_t h2d = nullptr, d2h = nullptr;
  std::vector<hipEvent_t> ev(3 * nb, nullptr);
  prune_status st = PRUNE_OK;
  auto cleanup = [&]() {
    if (h2d) (void)hipStreamSynchronize(h2d);
    if (d2h) (void)hipStreamSynchronize(d2h);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (h2d) (void)hipStreamDestroy(h2d);
    if (d2h) (void)hipStreamDestroy(d2h);
  };
  // Copies of a run of blocks of a ring, split where the ring wraps.
  auto copy_blocks = [&](char *ring, uint64_t first, uint32_t n, size_t blk, char *host, bool to_dev,
                         hipStream_t cs) -> hipError_t {
    uint32_t done = 0;
    while (done < n) {
      const uint64_t slot = (first + done) % g->C;
      const uint32_t run = (uint32_t)std::min<uint64_t>(n - done, g->C - slot);
      char *dev = ring + slot * blk;
      char *h = host + (size_t)done * blk;
      hipError_t e = to_dev ? hipMemcpyAsync(dev, h, (size_t)run * blk, hipMemcpyHostToDevice, cs)
                            : hipMemcpyAsync(h, dev, (size_t)run * blk, hipMemcpyDeviceToHost, cs);
      if (e != hipSuccess) return e;
      done += run;
    }
    return hipSuccess;
  };
  if (hipStreamCreateWithFlags(&h2d, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&d2h, hipStreamNonBlocking) != hipSuccess) {
    cleanup();
    return fail(PRUNE_E_HIP, "stream creation failed");
  }
  for (auto &e : ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      cleanup();
      return fail(PRUNE_E_HIP, "event creation failed");
    }
  for (uint32_t k = 0; k < nb && st == PRUNE_OK; ++k) {
    const uint32_t nk = std::min(batch, n_frames - k * batch);
    hipEvent_t e_in = ev[3 * k], e_fired = ev[3 * k + 1], e_out = ev[3 * k + 2];
    // frames of batch k into the source FIFO once the batch that last read
    // those blocks has fired
    if (k >= depth && hipStreamWaitEvent(h2d, ev[3 * (k - depth) + 1], 0) != hipSuccess) st = PRUNE_E_HIP;
    if (st == PRUNE_OK &&
        copy_blocks((char *)Fi.storage, di.writes + (uint64_t)k * batch, nk, bi,
                    (char *)host_in + (size_t)k * batch * bi, true, h2d) != hipSuccess)
      st = PRUNE_E_HIP;
    if (st == PRUNE_OK && hipEventRecord(e_in, h2d) != hipSuccess) st = PRUNE_E_HIP;
    // fire batch k once its frames are in and the output blocks it will
    // overwrite have been copied out
    if (st == PRUNE_OK && hipStreamWaitEvent(s, e_in, 0) != hipSuccess) st = PRUNE_E_HIP;
    if (st == PRUNE_OK && k >= depth && hipStreamWaitEvent(s, ev[3 * (k - depth) + 2], 0) != hipSuccess)
      st = PRUNE_E_HIP;
    uint64_t fired = 0;
    if (st == PRUNE_OK) st = prune_graph_fire(g, PRUNE_BATCHED, nk, stream, &fired);
    if (st == PRUNE_OK && fired != nk) st = fail(PRUNE_E_STATE, "a batch fired fewer iterations than queued");
    if (st == PRUNE_OK && hipEventRecord(e_fired, s) != hipSuccess) st = PRUNE_E_HIP;
    // outputs of batch k to the host
    if (st == PRUNE_OK && hipStreamWaitEvent(d2h, e_fired, 0) != hipSuccess) st = PRUNE_E_HIP;
    if (st == PRUNE_OK &&
        copy_blocks((char *)Fo.storage, dout.reads + (uint64_t)k * batch, nk, bo,
                    (char *)host_out + (size_t)k * batch * bo, false, d2h) != hipSuccess)
      st = PRUNE_E_HIP;
    if (st == PRUNE_OK && hipEventRecord(e_out, d2h) != hipSuccess) st = PRUNE_E_HIP;
  }
  cleanup();
  if (st == PRUNE_E_HIP) return fail(PRUNE_E_HIP, "host streaming: HIP call failed");
  if (st != PRUNE_OK) return st;
  HIPCHECK(hipStreamSynchronize(s));
  return PRUNE_OK;
}

prune_status prune_graph_sync(prune_graph_t g, prune_stream_t stream) {
  TRY(check_graph(g, true));
  HIPCHECK(hipStreamSynchronize((hipStream_t)stream));
  HIPCHECK(hipGetLastError());
  uint32_t e = 0;
  HIPCHECK(hipMemcpy(&e, g->d_err, sizeof e, hipMemcpyDeviceToHost));
  if (e) {
    uint32_t z = 0;
    HIPCHECK(hipMemcpy(g->d_err, &z, sizeof z, hipMemcpyHostToDevice));
    if (e & kErrToken) return fail(PRUNE_E_TOKEN, "control value with elements beyond its declared size");
    if (e & kErrRate) return fail(PRUNE_E_TOKEN, "rate parameter outside 1..atr");
    if (e & kErrCount) return fail(PRUNE_E_TOKEN, "block count differs from the firing's rate (or sink output full)");
    if (e & kErrTrace) return fail(PRUNE_E_CAPACITY, "trace buffer overflow");
    if (e & kErrInvariant)
      return fail(PRUNE_E_RULE, "bookkeeping broke a FIFO invariant (occupancy outside Eq. 2, or a counter going back)");
  }
  return PRUNE_OK;
}

prune_status prune_fifo_get_stats(prune_graph_t g, prune_id fifo, prune_fifo_stats *out) {
  TRY(check_graph(g, true));
  if (fifo >= g->fifos.size() || !out) return fail(PRUNE_E_ARG, "unknown fifo");
  HIPCHECK(hipDeviceSynchronize());
  FifoDev d;
  HIPCHECK(hipMemcpy(&d, g->d_fifos + fifo, sizeof d, hipMemcpyDeviceToHost));
  out->writes = d.writes; out->reads = d.reads;
  out->tokens_written = d.tokens_written; out->tokens_read = d.tokens_read;
  out->max_occ = d.max_occ; out->capacity = g->fifos[fifo].capacity;
  return PRUNE_OK;
}

prune_status prune_filterbank_branch_stats(prune_graph_t g, prune_id fb, uint64_t *firings,
                                           uint64_t *tokens, uint32_t n) {
  TRY(check_graph(g, true));
  if (fb >= g->actors.size() || g->actors[fb].kind != PRUNE_FILTERBANK) return fail(PRUNE_E_ARG, "not a filter bank");
  HActor &A = g->actors[fb];
  HIPCHECK(hipDeviceSynchronize());
  uint64_t buf[2 * PRUNE_MAX_BRANCHES];
  HIPCHECK(hipMemcpy(buf, A.bstats, sizeof buf, hipMemcpyDeviceToHost));
  for (uint32_t d = 0; d < n && d < PRUNE_MAX_BRANCHES; ++d) {
    if (firings) firings[d] = buf[d];
    if (tokens) tokens[d] = buf[PRUNE_MAX_BRANCHES + d];
  }
  return PRUNE_OK;
}

prune_status prune_actor_firings(prune_graph_t g, prune_id actor, uint64_t *firings) {
  TRY(check_graph(g, true));
  if (actor >= g->actors.size() || !firings) return fail(PRUNE_E_ARG, "unknown actor");
  HIPCHECK(hipDeviceSynchronize());
  HIPCHECK(hipMemcpy(firings, &g->d_actors[actor].firings, sizeof(uint64_t), hipMemcpyDeviceToHost));
  return PRUNE_OK;
}

prune_status prune_trace_enable(prune_graph_t g, size_t max_records) {
  TRY(check_graph(g, true));
  HIPCHECK(hipDeviceSynchronize());
  if (g->d_trace) { (void)hipFree(g->d_trace); g->d_trace = nullptr; }
  if (g->d_trace_count) { (void)hipFree(g->d_trace_count); g->d_trace_count = nullptr; }
  g->trace_cap = 0;
  // captured graphs hold the old trace pointers
  for (auto &kv : g->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto &kv : g->graph_defs) (void)hipGraphDestroy(kv.second);
  g->graphs.clear();
  g->graph_defs.clear();
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < 2; ++k) {
      for (auto &kv : g->pgraphs[p][k]) (void)hipGraphExecDestroy(kv.second);
      for (auto &kv : g->pgraph_defs[p][k]) (void)hipGraphDestroy(kv.second);
      g->pgraphs[p][k].clear();
      g->pgraph_defs[p][k].clear();
    }
  if (!max_records) return PRUNE_OK;
  HIPCHECK(hipMalloc((void **)&g->d_trace, max_records * sizeof(prune_trace_record)));
  HIPCHECK(hipMalloc((void **)&g->d_trace_count, sizeof(unsigned long long)));
  HIPCHECK(hipMemset(g->d_trace_count, 0, sizeof(unsigned long long)));
  g->trace_cap = max_records;
  return PRUNE_OK;
}

prune_status prune_trace_fetch(prune_graph_t g, void *host_buf, size_t bytes, size_t *used) {
  TRY(check_graph(g, true));
  if (!g->d_trace) return fail(PRUNE_E_STATE, "tracing is off");
  HIPCHECK(hipDeviceSynchronize());
  unsigned long long n = 0;
  HIPCHECK(hipMemcpy(&n, g->d_trace_count, sizeof n, hipMemcpyDeviceToHost));
  if (n > g->trace_cap) return fail(PRUNE_E_CAPACITY, "trace buffer overflowed");
  const size_t need = n * sizeof(prune_trace_record);
  if (used) *used = need;
  if (!host_buf) return PRUNE_OK;
  if (bytes < need) return fail(PRUNE_E_CAPACITY, "host buffer too small");
  if (need) HIPCHECK(hipMemcpy(host_buf, g->d_trace, need, hipMemcpyDeviceToHost));
  return PRUNE_OK;
}

prune_status prune_set_fb_variant(int v) {
  if (v < 0 || v > fb_variant_count()) return fail(PRUNE_E_ARG, "no such variant");
  g_variant_forced = v;
  return PRUNE_OK;
}

const char *prune_fb_variant_name(int v) { return fb_variant_name(v); }
int prune_fb_variant_count(void) { return fb_variant_count(); }

prune_status prune_set_batch_pipeline(int on) {
  g_pipeline = on != 0;
  return PRUNE_OK;
}

prune_status prune_timing_enable(int on) {
  g_timing = on != 0;
  timing_reset();
  return PRUNE_OK;
}

prune_status prune_last_fb_kernel_ms(float *ms, uint32_t *launches) {
  float tot = 0.f;
  for (auto &e : g_events) {
    HIPCHECK(hipEventSynchronize(e.second));
    float t = 0.f;
    HIPCHECK(hipEventElapsedTime(&t, e.first, e.second));
    tot += t;
  }
  if (ms) *ms = tot;
  if (launches) *launches = (uint32_t)g_events.size();
  return PRUNE_OK;
}

prune_status prune_rule_capacity(uint32_t r, uint32_t Q, uint32_t C, uint64_t *tokens) {
  if (!r || !C || !tokens) return fail(PRUNE_E_ARG, "rate and C must be positive");
  if ((Q % r) && (Q >= (uint64_t)r * C || (Q < r && Q + r > (uint64_t)r * C)))
    return fail(PRUNE_E_DELAY, "unaligned delay does not fit r*C");
  *tokens = fifo_capacity(r, Q, C);
  return PRUNE_OK;
}

prune_status prune_rule_slots(uint32_t r, uint32_t Q, uint32_t C, uint32_t n, uint64_t *ws,
                              uint64_t *rs) {
  uint64_t cap = 0;
  TRY(prune_rule_capacity(r, Q, C, &cap));
  for (uint32_t k = 0; k < n; ++k) {
    if (ws) ws[k] = fifo_write_slot(r, Q, C, k);
    if (rs) rs[k] = fifo_read_slot(r, Q, C, k);
  }
  return PRUNE_OK;
}

prune_status prune_rule_config_token(uint32_t mode, uint32_t Kmax, const prune_side_info *side,
                                     prune_ctrl_token *out) {
  if (!side || !out || mode > PRUNE_CONFIG_MASK) return fail(PRUNE_E_ARG, "bad arguments");
  *out = config_map(mode, Kmax, *side);
  return PRUNE_OK;
}

uint32_t prune_build_flags(void) { return kDebugBuild ? PRUNE_BUILD_DEBUG : 0u; }

const char *prune_status_string(prune_status s) {
  switch (s) {
    case PRUNE_OK: return "PRUNE_OK";
    case PRUNE_E_ARG: return "PRUNE_E_ARG";
    case PRUNE_E_STATE: return "PRUNE_E_STATE";
    case PRUNE_E_RATE_MISMATCH: return "PRUNE_E_RATE_MISMATCH";
    case PRUNE_E_PORT_KIND: return "PRUNE_E_PORT_KIND";
    case PRUNE_E_RULE4: return "PRUNE_E_RULE4";
    case PRUNE_E_CONNECT: return "PRUNE_E_CONNECT";
    case PRUNE_E_DELAY: return "PRUNE_E_DELAY";
    case PRUNE_E_TOKEN: return "PRUNE_E_TOKEN";
    case PRUNE_E_DEADLOCK: return "PRUNE_E_DEADLOCK";
    case PRUNE_E_CAPACITY: return "PRUNE_E_CAPACITY";
    case PRUNE_E_HIP: return "PRUNE_E_HIP";
    case PRUNE_E_UNSUPPORTED: return "PRUNE_E_UNSUPPORTED";
    case PRUNE_E_RULE: return "PRUNE_E_RULE";
    default: return "PRUNE_E_UNKNOWN";
  }
}

const char *prune_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
