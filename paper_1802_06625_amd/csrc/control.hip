// Control and bookkeeping kernels of the graph executor.
//
// k_control runs the bookkeeping of B graph iterations (B = 1 for the
// per-firing executor) for the actors of one connected component per
// workgroup, in topological order:
//  * configuration actors map side-information to control tokens and write
//    them into their control FIFOs (the control() half of Sec. VI-A lives in
//    the consumer: it reads the token back);
//  * dynamic actors read one token per firing from their control port and
//    decode every DRP per Eq. 1 (bit of element T[j][p] of the control value
//    times atr, or times the rate parameter for parameterised ports);
//  * each FIFO access gets its index by an exclusive scan over the batch of
//    the accesses that move tokens, its slot from the Eq. 2 / Fig. 6 rule,
//    and updates the device counters (writes, reads, tokens, occupancy);
//  * per-firing trace records, branch counters, filter-bank frame
//    descriptors and tile work lists, and copy work lists are produced for
//    the data kernels that follow.
// Static actors fire in an iteration exactly when their first input FIFO was
// written in that iteration (symmetric rates: one block per firing).
#include <algorithm>

#include "prune_internal.h"
#include "runtime_kernels.h"

namespace prune {

// ---------------------------------------------------------------- scans
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *total, uint32_t *sm) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sm[wid] = x;
  __syncthreads();
  if (wid == 0) {
    uint32_t w = lane < nw ? sm[lane] : 0u;
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t y = __shfl_up(w, o, 64);
      if (lane >= o) w += y;
    }
    if (lane < nw) sm[lane] = w;
  }
  __syncthreads();
  const uint32_t pre = (wid ? sm[wid - 1] : 0u) + x - v;
  *total = sm[nw - 1];
  __syncthreads();
  return pre;
}

__device__ uint64_t block_sum_u64(uint64_t v, unsigned long long *sm) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  uint64_t s = 0;
  for (int k = 0; k < nw; ++k) s += sm[k];
  __syncthreads();
  return s;
}

__device__ inline void trace_push(const CtrlArgs &c, uint32_t type, uint32_t a, uint32_t b,
                                  uint32_t cc, uint32_t d, uint32_t e, uint32_t f) {
  if (!c.trace.rec) return;
  unsigned long long k = atomicAdd(c.trace.count, 1ull);
  if (k < c.trace.cap) {
    prune_trace_record r;
    r.type = type; r.a = a; r.b = b; r.c = cc; r.d = d; r.e = e; r.f = f; r.pad = 0;
    c.trace.rec[k] = r;
  } else {
    atomicOr(c.err, kErrTrace);
  }
}

// Tokens moved through port p in a firing with the given rate and activity.
__device__ inline uint32_t port_count2(const CtrlArgs &c, const PortDev &p, uint32_t fired,
                                       uint32_t mask, uint32_t rate) {
  if (!fired) return 0;
  if (p.kind == PRUNE_DRP && !decode_bit(mask, p.element)) return 0;
  if (!p.param) return p.atr;
  if (rate < 1u || (uint64_t)rate + p.halo > p.atr) {
    atomicOr(c.err, kErrRate);
    return 0;
  }
  return rate + p.halo;
}

__device__ inline uint32_t port_count(const CtrlArgs &c, const PortDev &p, const FiringRec &r,
                                      uint32_t) {
  return port_count2(c, p, r.fired, r.mask, r.rate);
}

// Past samples of a stateful actor's stream before firing i of this batch:
// sample `e` positions before the frame (e = 1..H).
__device__ inline float2 past_sample(const CtrlArgs &c, uint32_t a, int i, uint32_t e) {
  const ActorDev &A = c.actors[a];
  const FiringRec *R = c.recs + (size_t)a * c.Bcap;
  for (int k = i - 1; k >= 0; --k) {
    const uint32_t cnt = R[k].in[0].count;
    if (e <= cnt) return ((const float2 *)R[k].in[0].ptr)[cnt - e];
    e -= cnt;
  }
  return e <= A.hist_len ? A.history[A.hist_len - e] : make_float2(0.f, 0.f);
}

// Resolve the H contiguous past samples of firing i: inside the previous
// block when it is long enough, the stored history for the first firing of
// the batch, otherwise a scratch copy that k_gather fills once the input
// blocks of this level have been written (after the upstream data kernels).
__device__ inline const float2 *resolve_halo(const CtrlArgs &c, uint32_t a, uint32_t i) {
  const ActorDev &A = c.actors[a];
  const uint32_t H = A.hist_len;
  const FiringRec *R = c.recs + (size_t)a * c.Bcap;
  if (i == 0) return A.history;
  const uint32_t cp = R[i - 1].in[0].count;
  if (cp >= H) return (const float2 *)R[i - 1].in[0].ptr + (cp - H);
  float2 *dst = c.halo_scratch + (size_t)c.halo_off[a] + (size_t)i * H;
  const uint32_t lev = c.level_of[a];
  const uint32_t k = atomicAdd(c.gather_count + lev, 1u);
  GatherReq g;
  g.actor = a; g.i = i; g.dst = dst;
  c.gather_items[c.gather_off[lev] + k] = g;
  return dst;
}

__device__ void actor_phase(const CtrlArgs &c, uint32_t a, uint32_t *sm32,
                            unsigned long long *sm64) {
  ActorDev &A = c.actors[a];
  const uint32_t B = c.B;
  const int tid = threadIdx.x, nt = blockDim.x;
  FiringRec *R = c.recs + (size_t)a * c.Bcap;
  const uint32_t kind = A.kind;
  const FbParamsDev *fb = kind == PRUNE_FILTERBANK ? &c.fbs[A.fb] : nullptr;

  // ---- step 1: firing, control value and rate of every iteration
  for (uint32_t i = tid; i < B; i += nt) {
    FiringRec r;
    r.fired = 1; r.firing = 0; r.mask = 0; r.rate = 0; r.bitmap = 0; r.n_io = 0;
    for (int s = 0; s < kMaxIn; ++s) { r.in[s].count = 0; r.in[s].ptr = nullptr; r.in[s].fifo = kNone; }
    if (kind == PRUNE_SOURCE) {
      const SrcIn s = ((const SrcIn *)A.queue)[(A.q_head + i) % A.q_cap];
      r.rate = s.count;
      r.in[0].ptr = (char *)s.ptr;      // copy-in source (null: frame written in place)
    } else if (kind == PRUNE_CONFIG) {
      const prune_side_info side = ((const prune_side_info *)A.queue)[(A.q_head + i) % A.q_cap];
      const prune_ctrl_token t = config_map(A.cfg_mode, A.cfg_Kmax, side);
      r.mask = t.mask; r.rate = t.rate;
    } else if (A.cport_fifo != kNone) {
      const FifoDev &f = c.fifos[A.cport_fifo];
      const uint64_t slot = fifo_read_slot(f.r, f.Q, f.C, f.reads + i);
      const prune_ctrl_token t = ((const prune_ctrl_token *)f.base)[slot];
      r.mask = t.mask; r.rate = t.rate;
      if (A.n_elements < 32 && (t.mask >> A.n_elements)) {
        atomicOr(c.err, kErrToken);
        r.mask &= (1u << A.n_elements) - 1u;
      }
    } else {
      // Static actor: in a batch it fires in the iterations whose input
      // block was written; a per-firing launch fires it once on the block
      // at its read index.  Its rate parameter is the block's count.
      const PortDev &p0 = c.ports[A.first_in];
      uint32_t w;
      if (c.per_firing) {
        const FifoDev &f = c.fifos[p0.fifo[0]];
        const uint64_t slot = fifo_read_slot(f.r, f.Q, f.C, f.reads);
        w = f.param ? f.counts[slot / f.r] : f.r;
      } else {
        w = c.wrote[(size_t)p0.fifo[0] * c.Bcap + i];
      }
      r.fired = w != 0;
      r.rate = w ? w - p0.halo : 0;
      r.mask = A.fixed_mask;
    }
    if (kind == PRUNE_FILTERBANK) {
      uint32_t eff = 0;
      if (A.cport_fifo != kNone) {
        for (uint32_t d = 0; d < fb->n_banks * fb->Kmax; ++d)
          eff |= decode_bit(r.mask, fb->elem[d]) << d;
      } else {
        eff = A.fixed_mask;
      }
      r.bitmap = eff;
    }
    R[i] = r;
  }
  __syncthreads();

  // ---- firing numbers and the control trace
  {
    uint32_t carry = 0;
    for (uint32_t base = 0; base < B; base += nt) {
      const uint32_t i = base + tid;
      const uint32_t fl = (i < B) ? R[i].fired : 0u;
      uint32_t tot;
      const uint32_t pre = block_excl_scan(fl, &tot, sm32);
      if (i < B) R[i].firing = (uint32_t)(A.firings + carry + pre);
      carry += tot;
    }
    __syncthreads();
    if (tid == 0) A.firings += carry;
  }

  // ---- step 2: FIFO accesses port by port
  uint32_t in_slot = 0, out_slot = 0;
  uint32_t drp_ord = 0;
  for (uint32_t q = 0; q < A.n_ports; ++q) {
    const PortDev &p = c.ports[A.port[q]];
    const bool is_in = p.dir == PRUNE_IN;
    const uint32_t my_drp = (p.kind == PRUNE_DRP) ? drp_ord++ : kNone;
    for (uint32_t fk = 0; fk < p.n_fifos; ++fk) {
      FifoDev &f = c.fifos[p.fifo[fk]];
      uint32_t carry = 0;
      uint64_t toks = 0;
      for (uint32_t base = 0; base < B; base += nt) {
        const uint32_t i = base + tid;
        uint32_t cnt = 0;
        if (i < B) {
          cnt = port_count(c, p, R[i], 0);
          if (my_drp != kNone && cnt && fk == 0) R[i].bitmap |= 1u << my_drp;
        }
        uint32_t tot;
        const uint32_t pre = block_excl_scan(cnt ? 1u : 0u, &tot, sm32);
        if (i < B) {
          if (!is_in) c.wrote[(size_t)p.fifo[fk] * c.Bcap + i] = cnt;
          if (cnt) {
            const uint64_t idx = (is_in ? f.reads : f.writes) + carry + pre;
            const uint64_t slot = is_in ? fifo_read_slot(f.r, f.Q, f.C, idx)
                                        : fifo_write_slot(f.r, f.Q, f.C, idx);
            const uint32_t blk = (uint32_t)(slot / f.r);
            char *ptr = f.base + slot * f.token_bytes;
            if (is_in) {
              if (f.param && f.counts[blk] != cnt) atomicOr(c.err, kErrCount);
              if (in_slot < (uint32_t)kMaxIn) { R[i].in[in_slot].ptr = ptr; R[i].in[in_slot].count = cnt;
                                                R[i].in[in_slot].fifo = p.fifo[fk]; }
            } else {
              if (f.param) f.counts[blk] = cnt;
              if (out_slot < (uint32_t)kMaxIO) {
                R[i].out[out_slot].ptr = ptr; R[i].out[out_slot].count = cnt;
                R[i].out[out_slot].fifo = p.fifo[fk]; R[i].out_port[out_slot] = q;
              }
            }
            trace_push(c, 0, p.fifo[fk], is_in ? 1u : 0u, R[i].firing, (uint32_t)idx,
                       (uint32_t)slot, cnt);
          } else if (is_in) {
            if (in_slot < (uint32_t)kMaxIn) { R[i].in[in_slot].ptr = nullptr; R[i].in[in_slot].count = 0; }
          } else if (out_slot < (uint32_t)kMaxIO) {
            R[i].out[out_slot].ptr = nullptr; R[i].out[out_slot].count = 0;
            R[i].out_port[out_slot] = q;
          }
        }
        toks += block_sum_u64(cnt, sm64);
        carry += tot;
      }
      if (tid == 0) {
        const uint64_t n0 = is_in ? f.reads : f.writes, t0 = is_in ? f.tokens_read : f.tokens_written;
        if (is_in) {
          f.reads += carry;
          f.tokens_read += toks;
        } else {
          f.writes += carry;
          f.tokens_written += toks;
          const uint64_t occ = f.Q + f.tokens_written - f.tokens_read;
          if (occ > f.max_occ) f.max_occ = occ;
        }
        PRUNE_DEBUG_CHECK(fifo_advance_ok(f.r, n0, t0, is_in ? f.reads : f.writes,
                                          is_in ? f.tokens_read : f.tokens_written) &&
                              fifo_counters_ok(f.r, f.Q, f.C, f.writes, f.reads, f.tokens_written, f.tokens_read),
                          c.err);
      }
      __syncthreads();
      if (is_in) { ++in_slot; break; }
      ++out_slot;
    }
  }
  // control-port read (one token per firing of a dynamic actor)
  if (A.cport_fifo != kNone) {
    FifoDev &f = c.fifos[A.cport_fifo];
    for (uint32_t i = tid; i < B; i += nt) {
      const uint64_t idx = f.reads + i;
      trace_push(c, 0, A.cport_fifo, 1u, R[i].firing, (uint32_t)idx,
                 (uint32_t)fifo_read_slot(f.r, f.Q, f.C, idx), 1u);
      trace_push(c, 1, a, 0u, R[i].firing, R[i].mask, R[i].rate, R[i].bitmap);
    }
    __syncthreads();
    if (tid == 0) {
      f.reads += B;
      f.tokens_read += B;
      PRUNE_DEBUG_CHECK(fifo_counters_ok(f.r, f.Q, f.C, f.writes, f.reads, f.tokens_written, f.tokens_read),
                        c.err);
    }
  }
  for (uint32_t i = tid; i < B; i += nt) R[i].n_io = out_slot;
  __syncthreads();
  if (tid == 0 && (kind == PRUNE_SOURCE || kind == PRUNE_CONFIG)) A.q_head += B;

  // ---- step 3: kind-specific products
  if (kind == PRUNE_CONFIG) {
    for (uint32_t i = tid; i < B; i += nt) {
      prune_ctrl_token t; t.mask = R[i].mask; t.rate = R[i].rate;
      for (uint32_t k = 0; k < out_slot; ++k)
        if (R[i].out[k].ptr) *(prune_ctrl_token *)R[i].out[k].ptr = t;
    }
  } else if (kind == PRUNE_FILTERBANK) {
    const uint32_t H = fb->Lmax - 1;
    FbFrameDesc *D = c.fb_desc + c.desc_off[a];
    for (uint32_t base = 0; base < B; base += nt) {
      const uint32_t i = base + tid;
      uint32_t tiles = 0;
      FbFrameDesc d;
      if (i < B && R[i].fired) {
        const char *xin = R[i].in[0].ptr;
        const uint32_t cin = R[i].in[0].count;
        d.n = fb->windowed ? cin - H : cin;
        d.x = (const float2 *)xin + (fb->windowed ? H : 0);
        if (fb->windowed) {
          d.halo = (const float2 *)xin;
          d.halo_valid = H;
        } else {
          d.halo = resolve_halo(c, a, i);
          d.halo_valid = H;
        }
        d.n_y = 0;
        for (uint32_t k = 0; k < out_slot && k < (uint32_t)kMaxFanout; ++k)
          if (R[i].out[k].ptr) d.y[d.n_y++] = (float2 *)R[i].out[k].ptr;
        d.taps = fb->taps;
        d.mask = R[i].bitmap;
        d.n_banks = fb->n_banks; d.Kmax = fb->Kmax; d.Lmax = fb->Lmax; d.route = 0;
        for (int b = 0; b < PRUNE_MAX_BANKS; ++b) d.L[b] = fb->L[b];
        tiles = (d.n + c.tile - 1) / c.tile;
        D[i] = d;
      }
      uint32_t tot;
      const uint32_t pre = block_excl_scan(tiles, &tot, sm32);
      __shared__ uint32_t s_res;
      if (tid == 0) s_res = atomicAdd(c.fb_count + c.level_of[a], tot);
      __syncthreads();
      const uint32_t off = c.fb_item_off[c.level_of[a]] + s_res + pre;
      for (uint32_t k = 0; k < tiles; ++k) {
        WorkItem w; w.frame = c.desc_off[a] + i; w.tile = k;
        c.fb_items[off + k] = w;
      }
      __syncthreads();
    }
    // branch counters
    const uint32_t Dn = fb->n_banks * fb->Kmax;
    for (uint32_t dd = 0; dd < Dn; ++dd) {
      uint64_t fi = 0, tk = 0;
      for (uint32_t base = 0; base < B; base += nt) {
        const uint32_t i = base + tid;
        uint32_t act = 0, n = 0;
        if (i < B && R[i].fired && ((R[i].bitmap >> dd) & 1u)) {
          act = 1;
          n = R[i].in[0].count - (fb->windowed ? H : 0);
        }
        fi += block_sum_u64(act, sm64);
        tk += block_sum_u64(n, sm64);
      }
      if (tid == 0) { fb->branch_firings[dd] += fi; fb->branch_tokens[dd] += tk; }
    }
  } else if (kind == PRUNE_SWITCH || kind == PRUNE_POLY || kind == PRUNE_SELECT ||
             kind == PRUNE_PASSTHROUGH || kind == PRUNE_SOURCE || kind == PRUNE_SINK ||
             kind == PRUNE_GAUSS5 || kind == PRUNE_THRES || kind == PRUNE_MED5) {
    // Items are counted first, then written in place at their scanned
    // offsets (a per-lane array of items, indexed by slot, would live in
    // scratch).
    CopyItem *CI = c.copy_items;
    for (uint32_t base = 0; base < B; base += nt) {
      const uint32_t i = base + tid;
      const bool fired = i < B && R[i].fired;
      uint32_t nitems = 0;
      if (fired) {
        if (kind == PRUNE_SWITCH || kind == PRUNE_POLY) {
          for (uint32_t k = 0; k < out_slot; ++k) nitems += R[i].out[k].ptr ? 1u : 0u;
        } else if (kind == PRUNE_SOURCE) {
          nitems = R[i].in[0].ptr ? out_slot : 0u;
        } else if (kind == PRUNE_SINK) {
          nitems = A.sink_out ? 1u : 0u;
        } else if (kind == PRUNE_GAUSS5 || kind == PRUNE_THRES || kind == PRUNE_MED5) {
          nitems = 1;
        } else {
          nitems = out_slot;
        }
      }
      // sink output offsets: running token offset over firings
      const uint32_t sink_tok = (kind == PRUNE_SINK && nitems) ? R[i].in[0].count : 0u;
      uint32_t tot_tok;
      const uint32_t pre_tok = block_excl_scan(sink_tok, &tot_tok, sm32);
      float2 *sink_dst = nullptr;
      if (kind == PRUNE_SINK && nitems) {
        const uint64_t off = A.sink_pos + pre_tok;
        const uint32_t tb = c.fifos[R[i].in[0].fifo].token_bytes;
        if (off + sink_tok <= A.sink_cap) sink_dst = (float2 *)((char *)A.sink_out + off * tb);
        else { nitems = 0; atomicOr(c.err, kErrCount); }
      }
      uint32_t tot;
      const uint32_t pre = block_excl_scan(nitems, &tot, sm32);
      __shared__ uint32_t s_cres;
      if (tid == 0) s_cres = atomicAdd(c.copy_count + c.level_of[a], tot);
      __syncthreads();
      const uint32_t off = c.copy_item_off[c.level_of[a]] + s_cres + pre;
      uint32_t w = 0;
      auto item = [&](const float2 *src, float2 *dst, uint32_t count) -> CopyItem & {
        CopyItem &ci = CI[off + w++];
        ci.n_src = src ? 1u : 0u;
        ci.src[0] = src;
        for (int q = 1; q < kMaxIn; ++q) ci.src[q] = nullptr;
        ci.dst = dst;
        ci.halo = nullptr;
        ci.halo_count = 0;
        ci.count = count;
        ci.pad = 0;
        ci.op = kOpCopy; ci.width = 0; ci.param = 0; ci.n_dst = 1;
        return ci;
      };
      auto words = [&](uint32_t fifo, uint32_t count) -> uint32_t {
        return fifo == kNone ? count : count * c.fifos[fifo].token_bytes / 8u;
      };
      if (nitems) {
        if (kind == PRUNE_SWITCH || kind == PRUNE_POLY) {
          const float2 *hp = resolve_halo(c, a, i);
          for (uint32_t k = 0; k < out_slot; ++k) {
            if (!R[i].out[k].ptr) continue;
            const PortDev &p = c.ports[A.port[R[i].out_port[k]]];
            CopyItem &ci = item((const float2 *)R[i].in[0].ptr, (float2 *)R[i].out[k].ptr, R[i].in[0].count);
            ci.halo = hp + (A.hist_len - p.halo);
            ci.halo_count = p.halo;
            ci.pad = p.power;
          }
        } else if (kind == PRUNE_SOURCE) {
          for (uint32_t k = 0; k < out_slot; ++k)
            item((const float2 *)R[i].in[0].ptr, (float2 *)R[i].out[k].ptr,
                 words(R[i].out[k].fifo, R[i].out[k].count));
        } else if (kind == PRUNE_SINK) {
          item((const float2 *)R[i].in[0].ptr, sink_dst, words(R[i].in[0].fifo, R[i].in[0].count));
        } else if (kind == PRUNE_GAUSS5 || kind == PRUNE_THRES || kind == PRUNE_MED5) {
          CopyItem &ci = item((const float2 *)R[i].in[0].ptr, (float2 *)R[i].out[0].ptr, A.pix_w * A.pix_h);
          ci.src[1] = kind == PRUNE_THRES ? (const float2 *)R[i].in[1].ptr : nullptr;
          ci.n_src = kind == PRUNE_THRES ? 2 : 1;
          for (uint32_t k = 1; k < out_slot && k + 1 < (uint32_t)kMaxIn; ++k)
            ci.src[k + 1] = (const float2 *)R[i].out[k].ptr;
          ci.n_dst = out_slot;
          ci.op = kind == PRUNE_GAUSS5 ? kOpGauss5 : (kind == PRUNE_THRES ? kOpThres : kOpMed5);
          ci.width = A.pix_w;
          ci.param = A.pix_t;
        } else {
          // SELECT sums its active inputs; PASSTHROUGH copies its input.
          for (uint32_t k = 0; k < out_slot; ++k) {
            CopyItem &ci = item(nullptr, (float2 *)R[i].out[k].ptr, words(R[i].out[k].fifo, R[i].out[k].count));
            uint32_t ns = 0;
            for (int q = 0; q < kMaxIn; ++q)
              if (R[i].in[q].ptr) ci.src[ns++] = (const float2 *)R[i].in[q].ptr;
            ci.n_src = ns;
          }
        }
      }
      if (tid == 0 && kind == PRUNE_SINK) A.sink_pos += tot_tok;
      __syncthreads();
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(1024) void k_control(CtrlArgs c) {
  __shared__ uint32_t sm32[32];
  __shared__ unsigned long long sm64[32];
  const uint32_t comp = blockIdx.x;
  if (c.clear_n && gridDim.x == 1) {
    for (uint32_t k = threadIdx.x; k < c.clear_n; k += blockDim.x) c.clear_ptr[k] = 0u;
    __syncthreads();
  }
  for (uint32_t k = c.comp_off[comp]; k < c.comp_off[comp + 1]; ++k) {
    actor_phase(c, c.comp_actors[k], sm32, sm64);
    __threadfence_block();
    __syncthreads();
  }
}

// Copy work: dst[0..halo_count) = halo, then dst[halo_count + k] = sum of
// the sources at k (zeros when there is none).  Grid: x over item slots of
// the level, y over chunks of kCopyChunk samples.
constexpr uint32_t kCopyChunk = 4096;

// ---- Motion Detection pixel actors on byte frames -------------------------
// Four pixels (one 32-bit word) per thread and row.  Two-lane arithmetic:
// bytes 0 and 2 of a word go to the 16-bit lanes of one register (even
// pixels), bytes 1 and 3 to another (odd pixels); sums that stay below 2^16
// per lane need no carry handling.
__device__ inline uint32_t lanes_even(uint32_t w) { return __builtin_amdgcn_perm(0u, w, 0x0c020c00u); }
__device__ inline uint32_t lanes_odd(uint32_t w) { return __builtin_amdgcn_perm(0u, w, 0x0c030c01u); }
// [hi lane of lo, lo lane of hi]: the lane pair one position to the left of hi
__device__ inline uint32_t lanes_shift(uint32_t hi, uint32_t lo) { return __builtin_amdgcn_alignbit(hi, lo, 16u); }
// bytes 0 of the even and odd lane registers back into one word
__device__ inline uint32_t lanes_pack(uint32_t ev, uint32_t od) { return __builtin_amdgcn_perm(od, ev, 0x06020400u); }
// the word's first (last) pixel in all four bytes: the columns beyond the
// left (right) frame edge repeat the edge pixel
__device__ inline uint32_t rep_first(uint32_t w) { return __builtin_amdgcn_perm(0u, w, 0x00000000u); }
__device__ inline uint32_t rep_last(uint32_t w) { return __builtin_amdgcn_perm(0u, w, 0x03030303u); }

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ inline uint32_t lanes_min(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                __builtin_bit_cast(u16x2, b)));
}
__device__ inline uint32_t lanes_max(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                __builtin_bit_cast(u16x2, b)));
}

// Median of five per lane: of the pairs (a, b) and (c, d), the smaller
// minimum and the larger maximum lie on either side of the median, so the
// median of five is the median of the larger minimum, the smaller maximum
// and e.
__device__ inline uint32_t lanes_median5(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t e) {
  const uint32_t x = lanes_max(lanes_min(a, b), lanes_min(c, d));
  const uint32_t y = lanes_min(lanes_max(a, b), lanes_max(c, d));
  return lanes_max(lanes_min(x, y), lanes_min(lanes_max(x, y), e));
}

// Vertical binomial [1 4 6 4 1] of one lane register over five rows:
// r0 + r4 + 4 (r1 + r2 + r3) + 2 r2, at most 16 * 255 per lane.
__device__ inline uint32_t lanes_binom(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3, uint32_t r4) {
  return r0 + r4 + (r2 << 1) + ((r1 + r2 + r3) << 2);
}

// Where a pixel item's word goes: the item's destination and, for a
// broadcast output, the further destinations listed after the two sources.
struct PixelDst {
  uint8_t *d0, *d1;
  const CopyItem *ci;   // LDS copy, for destinations beyond the second
  uint32_t nd;
  __device__ void store(size_t k, uint32_t v) const {
    *(uint32_t *)(d0 + k) = v;
    if (nd > 1) *(uint32_t *)(d1 + k) = v;
    for (uint32_t q = 2; q < nd; ++q) *(uint32_t *)((uint8_t *)ci->src[q + 1] + k) = v;
  }
};

// A thread takes its rows in steps of kPixRows output rows and issues every
// load of a step before using any of them, so that each wave keeps many
// loads in flight.  Rows outside the frame are clamped (in bounds; such rows
// only feed copied border rows).
constexpr int kPixRows = 8;
// Rows of a pixel frame per chunk of the grid's y dimension.
constexpr uint32_t kPixChunkRows = 16;

// Gauss 5x5 (binomial weights, (sum + 128) >> 8) of rows [ya, yb) at word
// column c.  Rows 0, 1, H-2 and H-1 are copied.  A step loads rows y0-2 ..
// y0+5, three words each (columns x-4 .. x+7 for x = 4c).  Vertical pass
// first, then the horizontal one on lane pairs shifted by one pixel
// position; every lane stays below 16 * 16 * 255 + 128 < 2^16.
__device__ void gauss_rows(const uint8_t *a, const PixelDst &out, int W, int H, uint32_t c, uint32_t G,
                           int ya, int yb) {
  const uint32_t xc = 4 * c, xl = c ? xc - 4 : xc, xr = c + 1 < G ? xc + 4 : xc;
  const bool at_left = c == 0, at_right = c + 1 == G;
  for (int y0 = ya; y0 < yb; y0 += kPixRows) {
    uint32_t wl[kPixRows + 4], wc[kPixRows + 4], wr[kPixRows + 4];
#pragma unroll
    for (int i = 0; i < kPixRows + 4; ++i) {
      const uint8_t *row = a + (size_t)min(max(y0 - 2 + i, 0), H - 1) * W;
      wl[i] = *(const uint32_t *)(row + xl);
      wc[i] = *(const uint32_t *)(row + xc);
      wr[i] = *(const uint32_t *)(row + xr);
    }
#pragma unroll
    for (int i = 0; i < kPixRows + 4; ++i) {
      if (at_left) wl[i] = rep_first(wc[i]);
      if (at_right) wr[i] = rep_last(wc[i]);
    }
#pragma unroll
    for (int j = 0; j < kPixRows; ++j) {
      const int y = y0 + j;
      if (y >= yb) break;
      uint32_t v = wc[j + 2];   // border rows are copied
      if (y >= 2 && y <= H - 3) {
        // vertical sums: [v(x-4), v(x-2)], [v(x-3), v(x-1)], [v(x), v(x+2)], ...
        const uint32_t ve0 = lanes_binom(lanes_even(wl[j]), lanes_even(wl[j + 1]), lanes_even(wl[j + 2]),
                                         lanes_even(wl[j + 3]), lanes_even(wl[j + 4]));
        const uint32_t vo0 = lanes_binom(lanes_odd(wl[j]), lanes_odd(wl[j + 1]), lanes_odd(wl[j + 2]),
                                         lanes_odd(wl[j + 3]), lanes_odd(wl[j + 4]));
        const uint32_t ve1 = lanes_binom(lanes_even(wc[j]), lanes_even(wc[j + 1]), lanes_even(wc[j + 2]),
                                         lanes_even(wc[j + 3]), lanes_even(wc[j + 4]));
        const uint32_t vo1 = lanes_binom(lanes_odd(wc[j]), lanes_odd(wc[j + 1]), lanes_odd(wc[j + 2]),
                                         lanes_odd(wc[j + 3]), lanes_odd(wc[j + 4]));
        const uint32_t ve2 = lanes_binom(lanes_even(wr[j]), lanes_even(wr[j + 1]), lanes_even(wr[j + 2]),
                                         lanes_even(wr[j + 3]), lanes_even(wr[j + 4]));
        const uint32_t vo2 = lanes_binom(lanes_odd(wr[j]), lanes_odd(wr[j + 1]), lanes_odd(wr[j + 2]),
                                         lanes_odd(wr[j + 3]), lanes_odd(wr[j + 4]));
        // even outputs (x, x+2) and odd outputs (x+1, x+3):
        // h(x) = v(x-2) + v(x+2) + 2 v(x) + 4 (v(x-1) + v(x) + v(x+1))
        const uint32_t e_m2 = lanes_shift(ve1, ve0);   // v(x-2) at the even pixels
        const uint32_t e_p2 = lanes_shift(ve2, ve1);   // v(x+2) at the even pixels = v(x+1) at the odd ones
        const uint32_t o_m1 = lanes_shift(vo1, vo0);   // v(x-1) at the even pixels = v(x-2) at the odd ones
        const uint32_t o_p2 = lanes_shift(vo2, vo1);   // v(x+2) at the odd pixels
        const uint32_t he = e_m2 + e_p2 + (ve1 << 1) + ((o_m1 + ve1 + vo1) << 2) + 0x00800080u;
        const uint32_t ho = o_m1 + o_p2 + (vo1 << 1) + ((ve1 + vo1 + e_p2) << 2) + 0x00800080u;
        v = __builtin_amdgcn_perm(ho, he, 0x07030501u);   // (h + 128) >> 8: each lane's high byte
      }
      out.store((size_t)y * W + xc, v);
    }
  }
}

// 5-pixel median (the pixel, up, down, left, right) of rows [ya, yb) at word
// column c.  Rows 0 and H-1 are copied.  A step loads the centre words of
// rows y0-1 .. y0+4 and the side words of rows y0 .. y0+3.
__device__ void med_rows(const uint8_t *a, const PixelDst &out, int W, int H, uint32_t c, uint32_t G,
                         int ya, int yb) {
  const uint32_t xc = 4 * c, xl = c ? xc - 4 : xc, xr = c + 1 < G ? xc + 4 : xc;
  const bool at_left = c == 0, at_right = c + 1 == G;
  for (int y0 = ya; y0 < yb; y0 += kPixRows) {
    uint32_t wc[kPixRows + 2], wl[kPixRows], wr[kPixRows];
#pragma unroll
    for (int i = 0; i < kPixRows + 2; ++i)
      wc[i] = *(const uint32_t *)(a + (size_t)min(max(y0 - 1 + i, 0), H - 1) * W + xc);
#pragma unroll
    for (int i = 0; i < kPixRows; ++i) {
      const uint8_t *row = a + (size_t)min(y0 + i, H - 1) * W;
      wl[i] = *(const uint32_t *)(row + xl);
      wr[i] = *(const uint32_t *)(row + xr);
    }
#pragma unroll
    for (int j = 0; j < kPixRows; ++j) {
      const int y = y0 + j;
      if (y >= yb) break;
      const uint32_t wu = wc[j], wm = wc[j + 1], wd = wc[j + 2];
      uint32_t v = wm;
      if (y >= 1 && y <= H - 2) {
        const uint32_t l = at_left ? rep_first(wm) : wl[j], r = at_right ? rep_last(wm) : wr[j];
        const uint32_t wlft = __builtin_amdgcn_alignbyte(wm, l, 3u);   // columns x-1 .. x+2
        const uint32_t wrgt = __builtin_amdgcn_alignbyte(r, wm, 1u);   // columns x+1 .. x+4
        const uint32_t me = lanes_median5(lanes_even(wu), lanes_even(wd), lanes_even(wlft), lanes_even(wrgt),
                                          lanes_even(wm));
        const uint32_t mo = lanes_median5(lanes_odd(wu), lanes_odd(wd), lanes_odd(wlft), lanes_odd(wrgt),
                                          lanes_odd(wm));
        v = lanes_pack(me, mo);
      }
      out.store((size_t)y * W + xc, v);
    }
  }
}

// Thres: 255 where |a - b| > T, else 0, of rows [ya, yb) at word column c.
// Per lane, d + (0x7fff - T) reaches bit 15 exactly when d > T (T clamped
// to 255, d <= 255).
__device__ void thres_rows(const uint8_t *a, const uint8_t *b, const PixelDst &out, int W, int H, uint32_t c,
                           int ya, int yb, uint32_t T) {
  const uint32_t bias = 0x7fffu - min(T, 255u), bias2 = bias | (bias << 16);
  for (int y0 = ya; y0 < yb; y0 += kPixRows) {
    uint32_t wa[kPixRows], wb[kPixRows];
#pragma unroll
    for (int i = 0; i < kPixRows; ++i) {
      const size_t k = (size_t)min(y0 + i, H - 1) * W + 4 * c;
      wa[i] = *(const uint32_t *)(a + k);
      wb[i] = *(const uint32_t *)(b + k);
    }
#pragma unroll
    for (int j = 0; j < kPixRows; ++j) {
      if (y0 + j >= yb) break;
      uint32_t r[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const uint32_t la = p ? lanes_odd(wa[j]) : lanes_even(wa[j]);
        const uint32_t lb = p ? lanes_odd(wb[j]) : lanes_even(wb[j]);
        const uint32_t d = lanes_max(la, lb) - lanes_min(la, lb);
        const uint32_t f = ((d + bias2) & 0x80008000u) >> 15;   // 0 or 1 per lane
        r[p] = (f << 8) - f;                                   // 0 or 255 per lane
      }
      out.store((size_t)(y0 + j) * W + 4 * c, lanes_pack(r[0], r[1]));
    }
  }
}

// Items with a nonzero power (POLY outputs) store |v|^power * v; pixel
// items (op != kOpCopy) run a Motion Detection actor over a byte frame.  The
// item is staged in LDS so that its source list is indexed there rather
// than in per-lane scratch.
// Instantiated with the pixel path only for levels that hold pixel actors:
// element copies keep the smaller register footprint (and occupancy).
template <bool kPixels>
__global__ __launch_bounds__(256) void k_copy(const CopyItem *__restrict__ items,
                                              const uint32_t *__restrict__ n_items) {
  __shared__ CopyItem s_ci;
  const uint32_t n = *n_items;
  for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
    __syncthreads();
    if (threadIdx.x == 0) s_ci = items[it];
    __syncthreads();
    if (kPixels && s_ci.op != kOpCopy) {
      // A pixel item covers a W x H byte frame (W a multiple of 4, frame
      // bases word aligned), in chunks of kPixChunkRows rows taken
      // grid-stride over blockIdx.y.  Threads split into P row groups of
      // G = W / 4 word columns; each thread runs down its column over its
      // run of the chunk's rows.
      const int W = (int)s_ci.width, H = (int)(s_ci.count / s_ci.width);
      const uint32_t G = (uint32_t)W / 4u;
      const uint32_t P = max(1u, blockDim.x / G);
      const uint32_t ty = threadIdx.x / G, tx = threadIdx.x - ty * G;
      if (ty >= P) continue;
      const uint8_t *a = (const uint8_t *)s_ci.src[0];
      const uint8_t *b = (const uint8_t *)s_ci.src[1];
      const uint32_t nd = s_ci.n_dst;
      const PixelDst out{(uint8_t *)s_ci.dst, nd > 1 ? (uint8_t *)s_ci.src[2] : nullptr, &s_ci, nd};
      const uint32_t cstep = P == 1 ? blockDim.x : G;
      for (int y_lo = (int)(blockIdx.y * kPixChunkRows); y_lo < H; y_lo += (int)(gridDim.y * kPixChunkRows)) {
        const int y_hi = min(H, y_lo + (int)kPixChunkRows);
        const int rpt = (y_hi - y_lo + (int)P - 1) / (int)P;
        const int ya = y_lo + (int)ty * rpt, yb = min(y_hi, ya + rpt);
        for (uint32_t c = tx; c < G && ya < yb; c += cstep) {
          if (s_ci.op == kOpGauss5) gauss_rows(a, out, W, H, c, G, ya, yb);
          else if (s_ci.op == kOpMed5) med_rows(a, out, W, H, c, G, ya, yb);
          else thres_rows(a, b, out, W, H, c, ya, yb, s_ci.param);
        }
      }
      continue;
    }
    const uint32_t halo_count = s_ci.halo_count, n_src = s_ci.n_src, power = s_ci.pad;
    const uint32_t total = halo_count + s_ci.count;
    float2 *dst = s_ci.dst;
    // chunks of kCopyChunk words, grid-stride over blockIdx.y
    for (uint64_t lo = (uint64_t)blockIdx.y * kCopyChunk; lo < total; lo += (uint64_t)gridDim.y * kCopyChunk) {
      const uint64_t hi = min((uint64_t)total, lo + kCopyChunk);
      for (uint64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
        float2 v;
        if (k < halo_count) {
          v = s_ci.halo[k];
        } else {
          const uint64_t s = k - halo_count;
          if (n_src == 1) {
            v = s_ci.src[0][s];   // a copy moves the bits (byte frames too), no arithmetic
          } else {
            v = make_float2(0.f, 0.f);
            for (uint32_t q = 0; q < n_src; ++q) {
              const float2 u = s_ci.src[q][s];
              v.x += u.x;
              v.y += u.y;
            }
          }
        }
        if (power) {
          const float r = sqrtf(v.x * v.x + v.y * v.y);
          float m = r;
          for (uint32_t e = 1; e < power; ++e) m *= r;
          v.x *= m;
          v.y *= m;
        }
        dst[k] = v;
      }
    }
  }
}

// Stream history update after a batch: the last H input samples of each
// stateful actor (stateful filter banks and switches).  One workgroup per
// actor listed in `actors`.
__global__ __launch_bounds__(256) void k_post(CtrlArgs c, const uint32_t *__restrict__ actors) {
  const uint32_t a = actors[blockIdx.x];
  ActorDev &A = c.actors[a];
  const uint32_t H = A.hist_len;
  const FiringRec *R = c.recs + (size_t)a * c.Bcap;
  int last = (int)c.B - 1;
  while (last >= 0 && !R[last].fired) --last;
  if (last < 0) return;
  __shared__ float2 tmp[PRUNE_MAX_L];
  for (uint32_t k = threadIdx.x; k < H; k += blockDim.x)
    tmp[k] = past_sample(c, a, last + 1, H - k);
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < H; k += blockDim.x) A.history[k] = tmp[k];
}

// Fill the halo copies requested by the control kernel for one level: one
// workgroup per request, after the level's inputs exist.
__global__ __launch_bounds__(64) void k_gather(CtrlArgs c, uint32_t level) {
  const uint32_t n = c.gather_count[level];
  for (uint32_t r = blockIdx.x; r < n; r += gridDim.x) {
    const GatherReq g = c.gather_items[c.gather_off[level] + r];
    const uint32_t H = c.actors[g.actor].hist_len;
    for (uint32_t k = threadIdx.x; k < H; k += blockDim.x)
      g.dst[k] = past_sample(c, g.actor, (int)g.i, H - k);
  }
}

// Copy-back of a FIFO with an unaligned delay (the access pattern of Fig. 6):
// after a write whose slots run past rC-1, the tokens in the overflow area
// [rC, end) are copied to [0, end-rC).  Per-firing launches only; `k` is the
// write's index among the actor's output accesses.
__global__ __launch_bounds__(256) void k_copyback(CtrlArgs c, uint32_t a, uint32_t fifo, uint32_t k) {
  const FiringRec &r = c.recs[(size_t)a * c.Bcap];
  if (!r.fired || k >= (uint32_t)kMaxIO || !r.out[k].ptr) return;
  const FifoDev &f = c.fifos[fifo];
  const uint64_t rc = (uint64_t)f.r * f.C;
  const uint64_t slot = (uint64_t)(r.out[k].ptr - f.base) / f.token_bytes;
  const uint64_t end = slot + f.r;
  if (end <= rc) return;
  const uint64_t nbytes = (end - rc) * f.token_bytes;
  for (uint64_t q = threadIdx.x; q < nbytes; q += blockDim.x) f.base[q] = f.base[rc * f.token_bytes + q];
}

// Zero the per-level counters and work tickets (a fill kernel rather than a
// memset so the sequence can be captured into a graph).
__global__ void k_clear_u32(uint32_t *p, uint32_t n) {
  for (uint32_t k = threadIdx.x + blockIdx.x * blockDim.x; k < n; k += blockDim.x * gridDim.x)
    p[k] = 0u;
}

// ---------------------------------------------------------------- launchers
void launch_control(const CtrlArgs &c, uint32_t n_comp, hipStream_t s) {
  hipLaunchKernelGGL(k_control, dim3(n_comp), dim3(1024), 0, s, c);
}

void launch_copy(const CopyItem *items, const uint32_t *n_items, uint32_t grid_x,
                 uint32_t max_total, uint32_t pix_rows, hipStream_t s) {
  // Element copies run up to 4096 workgroups that loop over the items.
  // Pixel frames take a workgroup per item and row chunk (as many as 64K):
  // their items are few and each stages its descriptor once.
  // both paths take their chunks grid-stride over y, so the grid's y extent
  // can stay within its limit
  const uint32_t gy = std::min<uint32_t>(65535u, std::max((max_total + kCopyChunk - 1) / kCopyChunk,
                                                          (pix_rows + kPixChunkRows - 1) / kPixChunkRows));
  if (!grid_x || !gy) return;
  const uint32_t budget = pix_rows ? 65536u : 4096u;
  const uint32_t gx = std::min<uint32_t>(grid_x, std::max<uint32_t>(1, budget / gy));
  if (pix_rows)
    hipLaunchKernelGGL(k_copy<true>, dim3(gx, gy), dim3(256), 0, s, items, n_items);
  else
    hipLaunchKernelGGL(k_copy<false>, dim3(gx, gy), dim3(256), 0, s, items, n_items);
}

void launch_post(const CtrlArgs &c, const uint32_t *actors, uint32_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_post, dim3(n), dim3(256), 0, s, c, actors);
}

void launch_gather(const CtrlArgs &c, uint32_t level, uint32_t grid, hipStream_t s) {
  if (!grid) return;
  hipLaunchKernelGGL(k_gather, dim3(grid), dim3(64), 0, s, c, level);
}

void launch_copyback(const CtrlArgs &c, uint32_t a, uint32_t fifo, uint32_t k, hipStream_t s) {
  hipLaunchKernelGGL(k_copyback, dim3(1), dim3(256), 0, s, c, a, fifo, k);
}

void launch_clear(uint32_t *p, uint32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(256), 0, s, p, n);
}

}  // namespace prune

// ======================================================================
// Parallel batch bookkeeping.  The per-firing path above runs one firing
// per launch; a batch of B iterations is split into three phases so that
// only the prefix sums run in one workgroup per component:
//   decode (thread per iteration): firing, control value, rate, the token
//     count of every FIFO access, tiles / copy items of the firing;
//   scan   (workgroup per component): exclusive prefix sums of the accesses
//     that move tokens (their FIFO indices), firing numbers, work-list
//     offsets, counters, branch statistics;
//   emit   (thread per iteration): slots from the indices, firing records,
//     trace, control tokens into control FIFOs, filter-bank descriptors and
//     tiles, copy items, halo gather requests.
// Within an iteration a thread walks the component's actors in topological
// order, so a static actor sees what its producer wrote in that iteration.
// ======================================================================

namespace prune {

// One wave per workgroup; each thread keeps the per-FIFO token counts of its
// iteration in LDS (a row of kMaxCompFifos + 1 words, an odd stride, so the
// lanes of an access hit distinct banks), which keeps the kernel at a few
// dozen registers: it runs beside the persistent filter-bank kernel of the
// previous batch in the room that kernel leaves free.
constexpr int kDecodeWG = 64;
__global__ __launch_bounds__(kDecodeWG) void k_batch_decode(CtrlArgs c, BatchArgs b) {
  __shared__ uint32_t s_wrote[kDecodeWG][kMaxCompFifos + 1];
  __shared__ uint32_t s_tmask[kDecodeWG][kMaxCompFifos + 1];
  __shared__ uint32_t s_trate[kDecodeWG][kMaxCompFifos + 1];
  const uint32_t comp = blockIdx.y;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  // per-level counters and work tickets start at zero for the later phases
  if (blockIdx.x == 0 && blockIdx.y == 0) {
    for (uint32_t k = threadIdx.x; k < c.clear_n; k += blockDim.x) c.clear_ptr[k] = 0u;
    for (uint32_t f = threadIdx.x; f < c.n_fifos; f += blockDim.x) b.s_rsnap[f] = c.fifos[f].tokens_read;
  }
  if (i >= c.B) return;
  const uint32_t Bc = c.Bcap;
  uint32_t *wrote = s_wrote[threadIdx.x], *tmask = s_tmask[threadIdx.x], *trate = s_trate[threadIdx.x];
  for (int k = 0; k < kMaxCompFifos; ++k) { wrote[k] = 0; tmask[k] = 0; trate[k] = 0; }
  for (uint32_t ka = c.comp_off[comp]; ka < c.comp_off[comp + 1]; ++ka) {
    const uint32_t a = c.comp_actors[ka];
    const ActorDev &A = c.actors[a];
    const uint32_t kind = A.kind;
    uint32_t fired = 1, mask = 0, rate = 0, bitmap = 0;
    const void *src_ptr = nullptr;
    if (kind == PRUNE_SOURCE) {
      const SrcIn sin = ((const SrcIn *)A.queue)[(A.q_head + i) % A.q_cap];
      rate = sin.count;
      src_ptr = sin.ptr;
    } else if (kind == PRUNE_CONFIG) {
      const prune_side_info side = ((const prune_side_info *)A.queue)[(A.q_head + i) % A.q_cap];
      const prune_ctrl_token t = config_map(A.cfg_mode, A.cfg_Kmax, side);
      mask = t.mask; rate = t.rate;
    } else if (A.cport_fifo != kNone) {
      // the control token this iteration's configuration firing wrote
      const uint32_t k2 = c.fifos[A.cport_fifo].pad;   // local slot of the control FIFO
      mask = tmask[k2]; rate = trate[k2];
      if (A.n_elements < 32 && (mask >> A.n_elements)) {
        atomicOr(c.err, kErrToken);
        mask &= (1u << A.n_elements) - 1u;
      }
    } else {
      const PortDev &p0 = c.ports[A.first_in];
      const uint32_t w = wrote[c.fifos[p0.fifo[0]].pad];
      fired = w != 0;
      rate = w ? w - p0.halo : 0;
      mask = A.fixed_mask;
    }
    const FbParamsDev *fb = kind == PRUNE_FILTERBANK ? &c.fbs[A.fb] : nullptr;
    if (fb) {
      if (A.cport_fifo != kNone) {
        for (uint32_t d = 0; d < fb->n_banks * fb->Kmax; ++d)
          bitmap |= decode_bit(mask, fb->elem[d]) << d;
      } else {
        bitmap = A.fixed_mask;
      }
    }
    uint32_t in0 = 0, n_out = 0, n_act_out = 0;
    bool first_in = true;
    for (uint32_t k2 = b.acc_off[a]; k2 < b.acc_off[a + 1]; ++k2) {
      const AccDev ac = b.acc[k2];
      const PortDev &p = c.ports[ac.port];
      const uint32_t cnt = port_count2(c, p, fired, mask, rate);
      if (p.kind == PRUNE_DRP && cnt && ac.first) bitmap |= 1u << ac.drp;
      b.s_cnt[(size_t)k2 * Bc + i] = cnt;
      if (ac.dir == PRUNE_OUT) {
        wrote[ac.local] = cnt;
        if (kind == PRUNE_CONFIG) { tmask[ac.local] = mask; trate[ac.local] = rate; }
        ++n_out;
        if (cnt) ++n_act_out;
      } else if (first_in) {
        in0 = cnt;
        first_in = false;
      }
    }
    uint32_t aux = 0;
    if (fired) {
      if (fb) {
        const uint32_t n = fb->windowed ? in0 - (fb->Lmax - 1) : in0;
        aux = in0 ? (n + c.tile - 1) / c.tile : 0;
      } else if (kind == PRUNE_SWITCH || kind == PRUNE_POLY) {
        aux = n_act_out;
      } else if (kind == PRUNE_SOURCE) {
        aux = src_ptr ? n_out : 0;
      } else if (kind == PRUNE_SINK) {
        aux = A.sink_out ? 1 : 0;
      } else if (kind == PRUNE_SELECT || kind == PRUNE_PASSTHROUGH) {
        aux = n_out;
      } else if (kind == PRUNE_GAUSS5 || kind == PRUNE_THRES || kind == PRUNE_MED5) {
        aux = 1;
      }
    }
    const size_t o = (size_t)a * Bc + i;
    b.s_fired[o] = fired;
    b.s_mask[o] = mask;
    b.s_rate[o] = rate;
    b.s_bitmap[o] = bitmap;
    b.s_aux[o] = aux;
    b.s_aux2[o] = (kind == PRUNE_SINK && fired && A.sink_out) ? in0 : 0;
  }
}

// Exclusive scan of v[0..B) into out[0..B) (out may alias v) by one
// workgroup: contiguous segments per thread, a block scan of their sums.
// Returns the total.
__device__ uint32_t seg_scan(const uint32_t *v, uint32_t *out, uint32_t B, bool flag,
                             uint32_t add, uint32_t *sm32) {
  const uint32_t nt = blockDim.x, tid = threadIdx.x;
  const uint32_t S = (B + nt - 1) / nt;
  const uint32_t lo = min(B, tid * S), hi = min(B, lo + S);
  uint32_t loc = 0;
  for (uint32_t i = lo; i < hi; ++i) loc += flag ? (v[i] != 0) : v[i];
  uint32_t tot;
  const uint32_t pre = block_excl_scan(loc, &tot, sm32);
  if (out) {
    uint32_t run = add + pre;
    for (uint32_t i = lo; i < hi; ++i) {
      const uint32_t x = flag ? (v[i] != 0) : v[i];
      out[i] = run;
      run += x;
    }
  }
  __syncthreads();
  return tot;
}

// Batch scans run one workgroup per actor.  Arrays are staged through LDS in
// chunks of kScanE * blockDim elements with coalesced loads and stores; each
// thread scans a contiguous run of kScanE elements of the chunk.
constexpr uint32_t kScanNT = 256, kScanE = 8;

// out[i] = base + exclusive prefix of (flag ? v != 0 : v); returns the total
// and adds the sum of the values to *sum.  out may alias v.
__device__ uint32_t chunk_scan(const uint32_t *v, uint32_t *out, uint32_t B, bool flag,
                               uint32_t base, uint64_t *sum, uint32_t *sh, uint32_t *sm32,
                               unsigned long long *sm64) {
  const uint32_t nt = blockDim.x, tid = threadIdx.x, CH = nt * kScanE;
  uint32_t carry = 0;
  uint64_t sv = 0;
  for (uint32_t c0 = 0; c0 < B; c0 += CH) {
#pragma unroll
    for (uint32_t k = 0; k < kScanE; ++k) {
      const uint32_t idx = c0 + k * nt + tid;
      sh[k * nt + tid] = idx < B ? v[idx] : 0u;
    }
    __syncthreads();
    uint32_t loc = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanE; ++k) {
      const uint32_t x = sh[tid * kScanE + k];
      loc += flag ? (x != 0) : x;
      sv += x;
    }
    uint32_t tot;
    const uint32_t pre = block_excl_scan(loc, &tot, sm32);
    uint32_t run = base + carry + pre;
#pragma unroll
    for (uint32_t k = 0; k < kScanE; ++k) {
      const uint32_t x = sh[tid * kScanE + k];
      sh[tid * kScanE + k] = run;
      run += flag ? (x != 0) : x;
    }
    __syncthreads();
    if (out) {
#pragma unroll
      for (uint32_t k = 0; k < kScanE; ++k) {
        const uint32_t idx = c0 + k * nt + tid;
        if (idx < B) out[idx] = sh[k * nt + tid];
      }
    }
    carry += tot;
    __syncthreads();
  }
  if (sum) *sum += block_sum_u64(sv, sm64);
  return carry;
}

// Phase 2 of the batch bookkeeping.  Workgroup (actor a, task t); the tasks
// of an actor are independent (each reads only phase-1 outputs and each
// counter has one writer task):
//   t = 0  firing numbers, queue/control-FIFO bases, firing counters;
//   t = 1  work-list region of the actor's data kernel (filter-bank tiles or
//          copy items) and per-iteration offsets in it;
//   t = 2  sink output offsets;
//   t = 3  branch statistics of a filter bank;
//   t >= kScanFixed  one FIFO access: scan of its per-iteration counts, the
//          FIFO's index and token counters, max occupancy.
constexpr uint32_t kScanFixed = 4;
__global__ __launch_bounds__(kScanNT) void k_batch_scan(CtrlArgs c, BatchArgs b) {
  __shared__ uint32_t sh[kScanNT * kScanE];
  __shared__ uint32_t sm32[32];
  __shared__ unsigned long long sm64[32];
  __shared__ unsigned long long s_bf[PRUNE_MAX_BRANCHES], s_bt[PRUNE_MAX_BRANCHES];
  // branch statistics: per wave, branch of a block of eight and lane (one pad
  // word per row, so that the eight summing lanes hit distinct banks)
  __shared__ uint32_t s_wf[kScanNT / 64][8][65];
  __shared__ unsigned long long s_wt[kScanNT / 64][8][65];
  __shared__ uint32_t s_res;
  const uint32_t a = blockIdx.x, task = blockIdx.y;
  const uint32_t B = c.B, Bc = c.Bcap, tid = threadIdx.x, nt = blockDim.x;
  ActorDev &A = c.actors[a];
  const uint32_t kind = A.kind;
  const size_t o = (size_t)a * Bc;
  // sources, configuration actors and dynamic actors fire every iteration
  const bool always = kind == PRUNE_SOURCE || kind == PRUNE_CONFIG || A.cport_fifo != kNone;

  if (task == 0) {
    uint32_t nf = B;
    if (always) {
      for (uint32_t i = tid; i < B; i += nt) b.s_firing[o + i] = i;
    } else {
      nf = chunk_scan(b.s_fired + o, b.s_firing + o, B, true, 0, nullptr, sh, sm32, sm64);
    }
    if (tid == 0) {
      b.s_qbase[a] = (kind == PRUNE_SOURCE || kind == PRUNE_CONFIG) ? A.q_head
                     : (A.cport_fifo != kNone ? c.fifos[A.cport_fifo].reads : 0);
      A.firings += nf;
      if (kind == PRUNE_SOURCE || kind == PRUNE_CONFIG) A.q_head += B;
      if (A.cport_fifo != kNone) {
        c.fifos[A.cport_fifo].reads += nf;
        c.fifos[A.cport_fifo].tokens_read += nf;
      }
    }
    return;
  }

  if (task >= kScanFixed) {
    const uint32_t k2 = b.acc_off[a] + (task - kScanFixed);
    if (k2 >= b.acc_off[a + 1]) return;
    const AccDev ac = b.acc[k2];
    FifoDev &f = c.fifos[ac.fifo];
    const uint32_t *cnt = b.s_cnt + (size_t)k2 * Bc;
    uint32_t *pre = b.s_pre + (size_t)k2 * Bc;
    uint32_t nacc;
    uint64_t toks = 0;
    if (always && c.ports[ac.port].kind != PRUNE_DRP) {
      // an SRP of an actor that fires every iteration is accessed every iteration
      uint64_t loc = 0;
#pragma unroll 8
      for (uint32_t i = tid; i < B; i += nt) {
        pre[i] = i;
        loc += cnt[i];
      }
      nacc = B;
      toks = block_sum_u64(loc, sm64);
    } else {
      nacc = chunk_scan(cnt, pre, B, true, 0, &toks, sh, sm32, sm64);
    }
    if (tid == 0) {
      // each FIFO has one writer access and one reader access: no other
      // workgroup updates these fields
      if (ac.dir == PRUNE_IN) {
        b.s_base[k2] = f.reads;
        const uint64_t t0 = f.tokens_read;
        f.reads += nacc;
        f.tokens_read += toks;
        PRUNE_DEBUG_CHECK(fifo_advance_ok(f.r, b.s_base[k2], t0, f.reads, f.tokens_read), c.err);
      } else {
        b.s_base[k2] = f.writes;
        const uint64_t t0 = f.tokens_written;
        f.writes += nacc;
        f.tokens_written += toks;
        PRUNE_DEBUG_CHECK(fifo_advance_ok(f.r, b.s_base[k2], t0, f.writes, f.tokens_written), c.err);
        // occupancy with all of this batch's tokens written, before its reads
        const uint64_t occ = f.Q + f.tokens_written - b.s_rsnap[ac.fifo];
        if (occ > f.max_occ) f.max_occ = occ;
      }
    }
    return;
  }

  if (task == 1) {
    if (!(kind == PRUNE_FILTERBANK || kind == PRUNE_SWITCH || kind == PRUNE_POLY || kind == PRUNE_SELECT ||
          kind == PRUNE_PASSTHROUGH || kind == PRUNE_SOURCE || kind == PRUNE_SINK || kind == PRUNE_GAUSS5 ||
          kind == PRUNE_THRES || kind == PRUNE_MED5))
      return;
    const uint32_t lev = c.level_of[a];
    const bool fbk = kind == PRUNE_FILTERBANK;
    // total first, then the region, then the offsets
    uint32_t loc = 0;
#pragma unroll 8
    for (uint32_t i = tid; i < B; i += nt) loc += b.s_aux[o + i];
    const uint64_t tot = block_sum_u64(loc, sm64);
    if (tid == 0) s_res = atomicAdd((fbk ? c.fb_count : c.copy_count) + lev, (uint32_t)tot);
    __syncthreads();
    const uint32_t base = (fbk ? c.fb_item_off[lev] : c.copy_item_off[lev]) + s_res;
    chunk_scan(b.s_aux + o, b.s_auxoff + o, B, false, base, nullptr, sh, sm32, sm64);
    return;
  }

  if (task == 2) {
    if (tid == 0) b.s_sink[a] = A.sink_pos;
    if (!(kind == PRUNE_SINK && A.sink_out)) return;
    __syncthreads();   // the sink base is read before it advances
    const uint32_t tot = chunk_scan(b.s_aux2 + o, b.s_aux2 + o, B, false, 0, nullptr, sh, sm32, sm64);
    if (tid == 0) A.sink_pos += tot;
    return;
  }

  if (task == 3 && kind == PRUNE_FILTERBANK) {
    // branch statistics: each thread loads its iterations' firing flag,
    // bitmap and input count once per pass; then per branch the firing
    // count and the tokens are summed over each wave through LDS, and one
    // shared-memory add per wave
    const FbParamsDev &fb = c.fbs[A.fb];
    const uint32_t D = fb.n_banks * fb.Kmax;
    for (uint32_t d = tid; d < D; d += nt) { s_bf[d] = 0; s_bt[d] = 0; }
    __syncthreads();
    uint32_t in_acc = b.acc_off[a];
    while (in_acc < b.acc_off[a + 1] && b.acc[in_acc].dir != PRUNE_IN) ++in_acc;
    const uint32_t *cin = b.s_cnt + (size_t)in_acc * Bc;
    const uint32_t H = fb.windowed ? fb.Lmax - 1 : 0;
    constexpr int kPer = 8;   // iterations per thread and pass
    for (uint32_t i0 = 0; i0 < B; i0 += kPer * nt) {
      uint32_t bm[kPer], nn[kPer];
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const uint32_t i = i0 + q * nt + tid;
        const bool ok = i < B;
        const uint32_t fz = ok ? b.s_fired[o + i] : 0u, bmv = ok ? b.s_bitmap[o + i] : 0u;
        const uint32_t cv = ok ? cin[i] : 0u;
        bm[q] = fz ? bmv : 0u;
        nn[q] = cv ? cv - H : 0u;
      }
      // eight branches at a time: every lane's counts go to LDS, then lane k
      // of each wave sums branch d0 + k over the wave's 64 lanes
      const uint32_t lane = tid & 63, w = tid >> 6;
      for (uint32_t d0 = 0; d0 < D; d0 += 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          uint32_t f = 0;
          unsigned long long tk = 0;
#pragma unroll
          for (int q = 0; q < kPer; ++q) {
            const uint32_t on = (bm[q] >> (d0 + k)) & 1u;   // d0 + k < 32
            f += on;
            tk += on ? nn[q] : 0u;
          }
          s_wf[w][k][lane] = f;
          s_wt[w][k][lane] = tk;
        }
        __syncthreads();
        if (lane < 8) {
          uint32_t sf = 0;
          unsigned long long st = 0;
#pragma unroll 8
          for (int j = 0; j < 64; ++j) {
            sf += s_wf[w][lane][j];
            st += s_wt[w][lane][j];
          }
          if (d0 + lane < D) {
            if (sf) atomicAdd(&s_bf[d0 + lane], (unsigned long long)sf);
            if (st) atomicAdd(&s_bt[d0 + lane], st);
          }
        }
        __syncthreads();   // the rows are rewritten for the next block
      }
    }
    __syncthreads();
    for (uint32_t d = tid; d < D; d += nt) {
      fb.branch_firings[d] += s_bf[d];
      fb.branch_tokens[d] += s_bt[d];
    }
  }
}

// Halo of firing i of a stateful actor from the batch's own records: the
// stored history for the first firing, the tail of the previous input block
// when it is long enough, else a gather request filled by k_gather.
__device__ inline const float2 *batch_halo(const CtrlArgs &c, const BatchArgs &b, uint32_t a,
                                           uint32_t in_acc, uint32_t i) {
  const ActorDev &A = c.actors[a];
  const uint32_t H = A.hist_len;
  if (i == 0) return A.history;
  const size_t q = (size_t)in_acc * c.Bcap + (i - 1);
  const uint32_t cp = b.s_cnt[q];
  if (cp >= H) {
    const AccDev ac = b.acc[in_acc];
    const FifoDev &f = c.fifos[ac.fifo];
    const uint64_t slot = fifo_read_slot(f.r, f.Q, f.C, b.s_base[in_acc] + b.s_pre[q]);
    return (const float2 *)(f.base + slot * f.token_bytes) + (cp - H);
  }
  float2 *dst = c.halo_scratch + (size_t)c.halo_off[a] + (size_t)i * H;
  const uint32_t lev = c.level_of[a];
  const uint32_t k = atomicAdd(c.gather_count + lev, 1u);
  GatherReq g;
  g.actor = a; g.i = i; g.dst = dst;
  c.gather_items[c.gather_off[lev] + k] = g;
  return dst;
}

__global__ __launch_bounds__(64) void k_batch_emit(CtrlArgs c, BatchArgs b) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (kDebugBuild && blockIdx.x == 0 && blockIdx.y == 0) {
    // every counter update of the batch is done (the scan precedes this
    // kernel): the final state is reachable, the batch's peak occupancy
    // (all writes before the reads) is within Eq. 2, and no counter went back
    for (uint32_t q = threadIdx.x; q < c.n_fifos; q += blockDim.x) {
      const FifoDev &f = c.fifos[q];
      const uint32_t wa = b.fifo_wacc[q];
      PRUNE_DEBUG_CHECK(fifo_counters_ok(f.r, f.Q, f.C, f.writes, f.reads, f.tokens_written, f.tokens_read) &&
                            f.max_occ <= fifo_capacity(f.r, f.Q, f.C) && f.tokens_read >= b.s_rsnap[q] &&
                            f.writes >= b.s_base[wa],
                        c.err);
    }
  }
  if (i >= c.B) return;
  const uint32_t Bc = c.Bcap, last = c.B - 1;
  {
    const uint32_t a = blockIdx.y;
    const ActorDev &A = c.actors[a];
    const uint32_t kind = A.kind;
    const size_t ab = (size_t)a * Bc, o = ab + i;
    // the firing record is written in place: a local copy indexed by access
    // slot would live in per-lane scratch
    FiringRec &r = c.recs[o];
    r.fired = b.s_fired[o];
    const uint32_t batch_fired = b.s_firing[ab + last] + b.s_fired[ab + last];
    r.firing = (uint32_t)(A.firings - batch_fired + b.s_firing[o]);
    r.mask = b.s_mask[o];
    r.rate = b.s_rate[o];
    r.bitmap = b.s_bitmap[o];
    r.pad0 = r.pad1 = 0;
    for (int s = 0; s < kMaxIn; ++s) { r.in[s].ptr = nullptr; r.in[s].count = 0; r.in[s].fifo = kNone; }
    uint32_t n_out = 0, in_acc = kNone;
    for (uint32_t k2 = b.acc_off[a]; k2 < b.acc_off[a + 1]; ++k2) {
      const AccDev ac = b.acc[k2];
      FifoDev &f = c.fifos[ac.fifo];
      const uint32_t cnt = b.s_cnt[(size_t)k2 * Bc + i];
      char *ptr = nullptr;
      if (cnt) {
        const uint64_t idx = b.s_base[k2] + b.s_pre[(size_t)k2 * Bc + i];
        const uint64_t slot = ac.dir == PRUNE_IN ? fifo_read_slot(f.r, f.Q, f.C, idx)
                                                 : fifo_write_slot(f.r, f.Q, f.C, idx);
        ptr = f.base + slot * f.token_bytes;
        const uint32_t blk = (uint32_t)(slot / f.r);
        if (f.param) {
          // in a batch the read of iteration i takes the block written in
          // iteration i: compare with the writer's count of that iteration
          if (ac.dir == PRUNE_OUT) f.counts[blk] = cnt;
          else if (b.s_cnt[(size_t)b.fifo_wacc[ac.fifo] * Bc + i] != cnt) atomicOr(c.err, kErrCount);
        }
        trace_push(c, 0, ac.fifo, ac.dir == PRUNE_IN ? 1u : 0u, r.firing, (uint32_t)idx,
                   (uint32_t)slot, cnt);
      }
      if (ac.dir == PRUNE_IN) {
        if (in_acc == kNone) in_acc = k2;
        if (ac.slot < (uint32_t)kMaxIn) {
          r.in[ac.slot].ptr = ptr; r.in[ac.slot].count = cnt; r.in[ac.slot].fifo = ac.fifo;
        }
      } else if (ac.slot < (uint32_t)kMaxIO) {
        r.out[ac.slot].ptr = ptr; r.out[ac.slot].count = cnt; r.out[ac.slot].fifo = ac.fifo;
        r.out_port[ac.slot] = ac.port;
        n_out = max(n_out, ac.slot + 1);
      }
    }
    r.n_io = n_out;
    if (A.cport_fifo != kNone && r.fired) {
      const FifoDev &f = c.fifos[A.cport_fifo];
      const uint64_t idx = b.s_qbase[a] + b.s_firing[o];
      trace_push(c, 0, A.cport_fifo, 1u, r.firing, (uint32_t)idx,
                 (uint32_t)fifo_read_slot(f.r, f.Q, f.C, idx), 1u);
      trace_push(c, 1, a, 0u, r.firing, r.mask, r.rate, r.bitmap);
    }
    if (!r.fired) return;

    if (kind == PRUNE_CONFIG) {
      prune_ctrl_token t;
      t.mask = r.mask;
      t.rate = r.rate;
      for (uint32_t k = 0; k < n_out; ++k)
        if (r.out[k].ptr) *(prune_ctrl_token *)r.out[k].ptr = t;
    } else if (kind == PRUNE_FILTERBANK) {
      const FbParamsDev &fb = c.fbs[A.fb];
      const uint32_t H = fb.Lmax - 1;
      const uint32_t di = c.desc_off[a] + i;
      FbFrameDesc &d = c.fb_desc[di];   // in place (its output list is indexed)
      const char *xin = r.in[0].ptr;
      const uint32_t cin = r.in[0].count;
      d.n = cin ? (fb.windowed ? cin - H : cin) : 0;
      d.x = (const float2 *)xin + (fb.windowed ? H : 0);
      d.halo = fb.windowed ? (const float2 *)xin : batch_halo(c, b, a, in_acc, i);
      d.halo_valid = H;
      d.n_y = 0;
      for (uint32_t k = 0; k < n_out && k < (uint32_t)kMaxFanout; ++k)
        if (r.out[k].ptr) d.y[d.n_y++] = (float2 *)r.out[k].ptr;
      d.taps = fb.taps;
      d.mask = r.bitmap;
      d.n_banks = fb.n_banks; d.Kmax = fb.Kmax; d.Lmax = fb.Lmax; d.route = 0;
      for (int q = 0; q < PRUNE_MAX_BANKS; ++q) d.L[q] = fb.L[q];
      const uint32_t tiles = b.s_aux[o], base = b.s_auxoff[o];
      for (uint32_t t = 0; t < tiles; ++t) {
        WorkItem w;
        w.frame = di;
        w.tile = t;
        c.fb_items[base + t] = w;
      }
    } else {
      // copy items are written in place (their source list is indexed)
      const uint32_t base = b.s_auxoff[o];
      uint32_t n = 0;
      auto item = [&](const float2 *src, float2 *dst, uint32_t count) -> CopyItem & {
        CopyItem &ci = c.copy_items[base + n++];
        ci.n_src = src ? 1u : 0u;
        ci.src[0] = src;
        for (int q = 1; q < kMaxIn; ++q) ci.src[q] = nullptr;
        ci.dst = dst;
        ci.halo = nullptr;
        ci.halo_count = 0;
        ci.count = count;
        ci.pad = 0;
        ci.op = kOpCopy; ci.width = 0; ci.param = 0; ci.n_dst = 1;
        return ci;
      };
      // copy items move 8-byte words: byte-token blocks are counted in words
      auto words = [&](uint32_t fifo, uint32_t count) -> uint32_t {
        return fifo == kNone ? count : count * c.fifos[fifo].token_bytes / 8u;
      };
      if (kind == PRUNE_SWITCH || kind == PRUNE_POLY) {
        const float2 *hp = batch_halo(c, b, a, in_acc, i);
        for (uint32_t k = 0; k < n_out; ++k) {
          if (!r.out[k].ptr) continue;
          const PortDev &p = c.ports[r.out_port[k]];
          CopyItem &ci = item((const float2 *)r.in[0].ptr, (float2 *)r.out[k].ptr, r.in[0].count);
          ci.halo = hp + (A.hist_len - p.halo);
          ci.halo_count = p.halo;
          ci.pad = p.power;
        }
      } else if (kind == PRUNE_SOURCE) {
        const SrcIn sin = ((const SrcIn *)A.queue)[(b.s_qbase[a] + i) % A.q_cap];
        if (sin.ptr)
          for (uint32_t k = 0; k < n_out; ++k)
            item((const float2 *)sin.ptr, (float2 *)r.out[k].ptr, words(r.out[k].fifo, r.out[k].count));
      } else if (kind == PRUNE_SINK) {
        if (A.sink_out) {
          const uint64_t off = b.s_sink[a] + b.s_aux2[o];
          const uint32_t cnt = r.in[0].count;
          const uint32_t tb = c.fifos[r.in[0].fifo].token_bytes;
          // sink_cap and sink_pos count tokens; the output is addressed in bytes
          if (off + cnt <= A.sink_cap) {
            item((const float2 *)r.in[0].ptr, (float2 *)((char *)A.sink_out + off * tb), words(r.in[0].fifo, cnt));
          } else {
            item(nullptr, A.sink_out, 0);
            atomicOr(c.err, kErrCount);
          }
        }
      } else if (kind == PRUNE_GAUSS5 || kind == PRUNE_THRES || kind == PRUNE_MED5) {
        // one item computes the frame once and stores it to every FIFO of the
        // (broadcast) output port: dst, then src[2..]
        CopyItem &ci = item((const float2 *)r.in[0].ptr, (float2 *)r.out[0].ptr, A.pix_w * A.pix_h);
        ci.src[1] = kind == PRUNE_THRES ? (const float2 *)r.in[1].ptr : nullptr;
        ci.n_src = kind == PRUNE_THRES ? 2 : 1;
        for (uint32_t k = 1; k < n_out && k + 1 < (uint32_t)kMaxIn; ++k) ci.src[k + 1] = (const float2 *)r.out[k].ptr;
        ci.n_dst = n_out;
        ci.op = kind == PRUNE_GAUSS5 ? kOpGauss5 : (kind == PRUNE_THRES ? kOpThres : kOpMed5);
        ci.width = A.pix_w;
        ci.param = A.pix_t;
      } else if (kind == PRUNE_SELECT || kind == PRUNE_PASSTHROUGH) {
        for (uint32_t k = 0; k < n_out; ++k) {
          CopyItem &ci = item(nullptr, (float2 *)r.out[k].ptr, words(r.out[k].fifo, r.out[k].count));
          uint32_t ns = 0;
          for (int q = 0; q < kMaxIn; ++q)
            if (r.in[q].ptr) ci.src[ns++] = (const float2 *)r.in[q].ptr;
          ci.n_src = ns;
        }
      }
    }
  }
}

void launch_batch(const CtrlArgs &c, const BatchArgs &b, uint32_t n_comp, uint32_t n_actors,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_batch_decode, dim3((c.B + kDecodeWG - 1) / kDecodeWG, n_comp), dim3(kDecodeWG), 0,
                     s, c, b);
  hipLaunchKernelGGL(k_batch_scan, dim3(n_actors, kScanFixed + b.max_acc), dim3(kScanNT), 0, s, c, b);
  hipLaunchKernelGGL(k_batch_emit, dim3((c.B + 63) / 64, n_actors), dim3(64), 0, s, c, b);
}

}  // namespace prune
