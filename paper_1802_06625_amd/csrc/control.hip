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
__device__ inline uint32_t port_count(const CtrlArgs &c, const PortDev &p, const FiringRec &r,
                                      uint32_t eff_bits) {
  if (!r.fired) return 0;
  if (p.kind == PRUNE_DRP && !decode_bit(r.mask, p.element)) return 0;
  (void)eff_bits;
  if (!p.param) return p.atr;
  if (r.rate < 1u || (uint64_t)r.rate + p.halo > p.atr) {
    atomicOr(c.err, kErrRate);
    return 0;
  }
  return r.rate + p.halo;
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
        if (is_in) {
          f.reads += carry;
          f.tokens_read += toks;
        } else {
          f.writes += carry;
          f.tokens_written += toks;
          const uint64_t occ = f.Q + f.tokens_written - f.tokens_read;
          if (occ > f.max_occ) f.max_occ = occ;
        }
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
    if (tid == 0) { f.reads += B; f.tokens_read += B; }
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
    uint32_t carry = 0;
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
      carry += tot;
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
  } else if (kind == PRUNE_SWITCH || kind == PRUNE_SELECT || kind == PRUNE_PASSTHROUGH ||
             kind == PRUNE_SOURCE || kind == PRUNE_SINK) {
    CopyItem *CI = c.copy_items;
    for (uint32_t base = 0; base < B; base += nt) {
      const uint32_t i = base + tid;
      uint32_t nitems = 0;
      CopyItem it[kMaxIO];
      if (i < B && R[i].fired) {
        if (kind == PRUNE_SWITCH) {
          const float2 *hp = resolve_halo(c, a, i);
          for (uint32_t k = 0; k < out_slot; ++k) {
            if (!R[i].out[k].ptr) continue;
            const PortDev &p = c.ports[A.port[R[i].out_port[k]]];
            CopyItem &ci = it[nitems++];
            ci.n_src = 1; ci.src[0] = (const float2 *)R[i].in[0].ptr;
            for (int s = 1; s < kMaxIn; ++s) ci.src[s] = nullptr;
            ci.dst = (float2 *)R[i].out[k].ptr;
            ci.halo = hp + (A.hist_len - p.halo); ci.halo_count = p.halo;
            ci.count = R[i].in[0].count;
          }
        } else if (kind == PRUNE_SOURCE) {
          if (R[i].in[0].ptr) {
            for (uint32_t k = 0; k < out_slot; ++k) {
              CopyItem &ci = it[nitems++];
              ci.n_src = 1; ci.src[0] = (const float2 *)R[i].in[0].ptr;
              for (int s = 1; s < kMaxIn; ++s) ci.src[s] = nullptr;
              ci.dst = (float2 *)R[i].out[k].ptr; ci.halo = nullptr; ci.halo_count = 0;
              ci.count = R[i].out[k].count;
            }
          }
        } else if (kind == PRUNE_SINK) {
          if (A.sink_out) {
            CopyItem &ci = it[nitems++];
            ci.n_src = 1; ci.src[0] = (const float2 *)R[i].in[0].ptr;
            for (int s = 1; s < kMaxIn; ++s) ci.src[s] = nullptr;
            ci.dst = nullptr;   // filled below with the running offset
            ci.halo = nullptr; ci.halo_count = 0; ci.count = R[i].in[0].count;
          }
        } else {
          // SELECT sums its active inputs; PASSTHROUGH copies its input.
          for (uint32_t k = 0; k < out_slot; ++k) {
            CopyItem &ci = it[nitems++];
            ci.n_src = 0;
            for (uint32_t s = 0; s < (uint32_t)kMaxIn; ++s)
              if (R[i].in[s].ptr) ci.src[ci.n_src++] = (const float2 *)R[i].in[s].ptr;
            for (uint32_t s = ci.n_src; s < (uint32_t)kMaxIn; ++s) ci.src[s] = nullptr;
            ci.dst = (float2 *)R[i].out[k].ptr; ci.halo = nullptr; ci.halo_count = 0;
            ci.count = R[i].out[k].count;
          }
        }
      }
      // sink output offsets: running token offset over firings
      uint32_t sink_tok = (kind == PRUNE_SINK && nitems) ? it[0].count : 0u;
      uint32_t tot_tok;
      const uint32_t pre_tok = block_excl_scan(sink_tok, &tot_tok, sm32);
      if (kind == PRUNE_SINK && nitems) {
        const uint64_t off = A.sink_pos + pre_tok;
        if (off + sink_tok <= A.sink_cap) it[0].dst = A.sink_out + off;
        else { nitems = 0; atomicOr(c.err, kErrCount); }
      }
      uint32_t tot;
      const uint32_t pre = block_excl_scan(nitems, &tot, sm32);
      __shared__ uint32_t s_cres;
      if (tid == 0) s_cres = atomicAdd(c.copy_count + c.level_of[a], tot);
      __syncthreads();
      const uint32_t off = c.copy_item_off[c.level_of[a]] + s_cres + pre;
      for (uint32_t k = 0; k < nitems; ++k) CI[off + k] = it[k];
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

__global__ __launch_bounds__(256) void k_copy(const CopyItem *__restrict__ items,
                                              const uint32_t *__restrict__ n_items) {
  const uint32_t it = blockIdx.x;
  if (it >= *n_items) return;
  const CopyItem ci = items[it];
  const uint32_t total = ci.halo_count + ci.count;
  const uint32_t lo = blockIdx.y * kCopyChunk;
  if (lo >= total) return;
  const uint32_t hi = min(total, lo + kCopyChunk);
  for (uint32_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
    float2 v;
    if (k < ci.halo_count) {
      v = ci.halo[k];
    } else {
      const uint32_t s = k - ci.halo_count;
      v = make_float2(0.f, 0.f);
      for (uint32_t q = 0; q < ci.n_src; ++q) {
        const float2 u = ci.src[q][s];
        v.x += u.x;
        v.y += u.y;
      }
    }
    ci.dst[k] = v;
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
                 uint32_t max_total, hipStream_t s) {
  const uint32_t gy = (max_total + kCopyChunk - 1) / kCopyChunk;
  if (!grid_x || !gy) return;
  hipLaunchKernelGGL(k_copy, dim3(grid_x, gy), dim3(256), 0, s, items, n_items);
}

void launch_post(const CtrlArgs &c, const uint32_t *actors, uint32_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_post, dim3(n), dim3(256), 0, s, c, actors);
}

void launch_gather(const CtrlArgs &c, uint32_t level, uint32_t grid, hipStream_t s) {
  if (!grid) return;
  hipLaunchKernelGGL(k_gather, dim3(grid), dim3(64), 0, s, c, level);
}

void launch_clear(uint32_t *p, uint32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(256), 0, s, p, n);
}

}  // namespace prune
