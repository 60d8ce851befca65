// Direct filter-bank operations over whole streams (prune_fb_forward) and
// the forward-kernel autotuner.  The direct forward builds one frame
// descriptor per frame and the tile work list on the device, then runs the
// same persistent forward kernel as the graph executor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "prune.h"
#include "prune_internal.h"
#include "runtime_kernels.h"

namespace prune {

__global__ __launch_bounds__(1024) void k_direct_prep(prune_fb_desc d, const float2 *x,
                                                      const float2 *taps,
                                                      const prune_fb_frame *frames, float2 *y,
                                                      uint32_t tile, FbFrameDesc *desc,
                                                      WorkItem *items, uint32_t *n_items,
                                                      unsigned int *ticket, uint32_t *err) {
  __shared__ uint32_t sm[32];
  __shared__ uint32_t s_carry;
  __shared__ uint32_t s_pre[1024], s_tl[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = max(Lmax, d.L[b]);
  const uint32_t H = Lmax - 1;
  const size_t tstride = (size_t)d.n_banks * d.Kmax * Lmax;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < d.n_frames; base += nt) {
    const uint32_t f = base + tid;
    uint32_t tiles = 0;
    if (f < d.n_frames) {
      const prune_fb_frame fr = frames[f];
      FbFrameDesc D;
      const bool ok = fr.stream < d.n_streams && (uint64_t)fr.t0 + fr.n <= d.stream_len &&
                      fr.n <= d.max_frame_len;
      if (!ok) atomicOr(err, 1u);
      const float2 *xs = x + (size_t)fr.stream * d.stream_len;
      D.x = xs + fr.t0;
      D.halo = xs + ((int64_t)fr.t0 - (int64_t)H);
      D.halo_valid = min(fr.t0, H);
      D.y[0] = y + (size_t)fr.stream * d.stream_len + fr.t0;
      D.y[1] = D.y[2] = D.y[3] = nullptr;
      D.n_y = 1;
      D.taps = taps + (size_t)fr.stream * tstride;
      D.n = ok ? fr.n : 0;
      D.mask = fr.mask;
      D.route = fr.route;
      D.n_banks = d.n_banks; D.Kmax = d.Kmax; D.Lmax = Lmax;
      for (int b = 0; b < PRUNE_MAX_BANKS; ++b) D.L[b] = b < (int)d.n_banks ? d.L[b] : 0;
      desc[f] = D;
      tiles = (D.n + tile - 1) / tile;
    }
    // block exclusive scan of tiles
    uint32_t v = tiles;
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t t = __shfl_up(v, o, 64);
      if (lane >= o) v += t;
    }
    if (lane == 63) sm[wid] = v;
    __syncthreads();
    if (wid == 0) {
      uint32_t w = lane < nw ? sm[lane] : 0u;
      for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(w, o, 64);
        if (lane >= o) w += t;
      }
      if (lane < nw) sm[lane] = w;
    }
    __syncthreads();
    const uint32_t pre = s_carry + (wid ? sm[wid - 1] : 0u) + v - tiles;
    s_pre[tid] = pre;
    s_tl[tid] = tiles;
    __syncthreads();
    // tiles of frame base+j written by wave j mod nw, lanes on consecutive items
    for (uint32_t j = wid; j < (uint32_t)nt && base + j < d.n_frames; j += nw) {
      const uint32_t p0 = s_pre[j], nj = s_tl[j];
      for (uint32_t k = lane; k < nj; k += 64) {
        WorkItem it;
        it.frame = base + j;
        it.tile = k;
        items[p0 + k] = it;
      }
    }
    __syncthreads();
    if (tid == 0) s_carry += sm[nw - 1];
    __syncthreads();
  }
  if (tid == 0) {
    *n_items = s_carry;
    *ticket = 0u;
  }
}

// One thread per frame: out-of-range frames and order violations.
__global__ __launch_bounds__(256) void k_check_frames(prune_fb_desc d, const prune_fb_frame *fr,
                                                      uint32_t *n_bad) {
  const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= d.n_frames) return;
  const prune_fb_frame q = fr[f];
  bool bad = q.stream >= d.n_streams || (uint64_t)q.t0 + q.n > d.stream_len || q.n > d.max_frame_len;
  if (f > 0) {
    const prune_fb_frame p = fr[f - 1];
    if (p.stream > q.stream || (p.stream == q.stream && (uint64_t)p.t0 + p.n > q.t0)) bad = true;
  }
  if (bad) atomicAdd(n_bad, 1u);
}

void launch_direct_prep(const prune_fb_desc &d, const float2 *x, const float2 *taps,
                        const prune_fb_frame *frames, float2 *y, uint32_t tile, FbFrameDesc *desc,
                        WorkItem *items, uint32_t *n_items, unsigned int *ticket, uint32_t *err,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_direct_prep, dim3(1), dim3(1024), 0, s, d, x, taps, frames, y, tile, desc,
                     items, n_items, ticket, err);
}

}  // namespace prune

using namespace prune;

namespace {

std::mutex g_mu;
thread_local bool g_tuning = false;   // autotuner launches are not timed
struct DirectScratch {
  FbFrameDesc *desc = nullptr;
  WorkItem *items = nullptr;
  uint32_t *ctr = nullptr;   // n_items, ticket, err
  size_t cap_frames = 0, cap_items = 0;
};
std::map<int, DirectScratch> g_scratch;
std::map<std::string, int> g_tuned;   // graph-path shape classes -> variant
// The direct forward's choices by (Lmax, Kmax, frame-length class), in a
// fixed table so that the allocation-free entry point can read them.
struct DirectChoice {
  uint32_t L, K, nc;
  int v;
};
constexpr int kMaxChoices = 64;
DirectChoice g_choice[kMaxChoices];
int g_n_choice = 0;
int g_ncu = 0;

prune_status check_desc(const prune_fb_desc *d) {
  if (!d || d->n_streams == 0 || d->n_banks < 1 || d->n_banks > PRUNE_MAX_BANKS || d->Kmax < 1 ||
      d->Kmax > 10 || d->n_banks * d->Kmax > PRUNE_MAX_BRANCHES)
    return PRUNE_E_UNSUPPORTED;
  for (uint32_t b = 0; b < d->n_banks; ++b)
    if (d->L[b] < 1 || d->L[b] > PRUNE_MAX_L) return PRUNE_E_UNSUPPORTED;
  return PRUNE_OK;
}

int ncu() {
  if (!g_ncu) {
    int dev = 0, n = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    g_ncu = n;
  }
  return g_ncu;
}

// Fixed workspace of prune_fb_forward_noalloc, one copy per device for the
// life of the process: frame descriptors, then work items, then the item
// count, ticket and error word.
constexpr size_t kNaDescBytes =
    ((size_t)PRUNE_NOALLOC_MAX_FRAMES * sizeof(FbFrameDesc) + 255) / 256 * 256;
constexpr size_t kNaItemBytes = (size_t)PRUNE_NOALLOC_MAX_ITEMS * sizeof(WorkItem);
constexpr size_t kNaBytes = kNaDescBytes + kNaItemBytes + 256;
static __device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
unsigned char *g_na_ptr[kNaMaxDevices] = {};

// Device address of the current device's copy of the workspace, looked up
// once per device with that device current.  In host code `scratch` names a
// host-side stand-in, never the device memory, so only this address is
// passed to kernels.
unsigned char *noalloc_workspace() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNaMaxDevices) {
    set_last_error("prune_fb_forward_noalloc: no current device, or device index beyond 63");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_last_error("prune_fb_forward_noalloc: hipGetSymbolAddress of the workspace failed");
      return nullptr;
    }
    g_na_ptr[dev] = (unsigned char *)p;
  }
  return g_na_ptr[dev];
}

}  // namespace

namespace prune {
int cached_variant(uint32_t L, uint32_t K, uint32_t n);
static int choose_direct_variant(const prune_fb_desc *desc, const void *x, const void *taps,
                                 const void *frames, void *y, prune_stream_t stream);

prune_status prune_fb_forward_variant(const prune_fb_desc *desc, const void *x, const void *taps,
                                      const void *frames, void *y, int variant,
                                      prune_stream_t stream) {
  prune_status st = check_desc(desc);
  if (st != PRUNE_OK) return st;
  if (!x || !taps || !frames || !y) return PRUNE_E_ARG;
  if (variant < 1 || variant > fb_variant_count()) return PRUNE_E_ARG;
  if (desc->n_frames == 0) return PRUNE_OK;
  const uint32_t tile = (uint32_t)fb_variant_tile(variant);
  const size_t per = ((size_t)desc->max_frame_len + tile - 1) / tile;
  const size_t items = (size_t)desc->n_frames * (per ? per : 1);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PRUNE_E_HIP;
  DirectScratch *sc;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    sc = &g_scratch[dev];
    if (sc->cap_frames < desc->n_frames || sc->cap_items < items) {
      if (hipDeviceSynchronize() != hipSuccess) return PRUNE_E_HIP;
      if (sc->desc) (void)hipFree(sc->desc);
      if (sc->items) (void)hipFree(sc->items);
      if (!sc->ctr && hipMalloc((void **)&sc->ctr, 4 * sizeof(uint32_t)) != hipSuccess) return PRUNE_E_HIP;
      sc->cap_frames = std::max<size_t>(desc->n_frames, 2 * sc->cap_frames);
      sc->cap_items = std::max<size_t>(items, 2 * sc->cap_items);
      if (hipMalloc((void **)&sc->desc, sc->cap_frames * sizeof(FbFrameDesc)) != hipSuccess ||
          hipMalloc((void **)&sc->items, sc->cap_items * sizeof(WorkItem)) != hipSuccess)
        return PRUNE_E_HIP;
      (void)hipMemset(sc->ctr, 0, 4 * sizeof(uint32_t));
    }
  }
  hipStream_t s = (hipStream_t)stream;
  launch_direct_prep(*desc, (const float2 *)x, (const float2 *)taps, (const prune_fb_frame *)frames,
                     (float2 *)y, tile, sc->desc, sc->items, sc->ctr, sc->ctr + 1, sc->ctr + 2, s);
  // the persistent grid: every workgroup slot of the chip, or one per tile
  const uint32_t grid = (uint32_t)std::min<size_t>((size_t)ncu() * fb_variant_resident(variant), items);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = timing_on() && !g_tuning;
  if (timed) {   // events that cannot be created leave the launch untimed
    if (hipEventCreate(&e0) != hipSuccess) e0 = nullptr;
    if (hipEventCreate(&e1) != hipSuccess) e1 = nullptr;
    if (!e0 || !e1) {
      timing_push(e0, e1);   // releases the one that exists
      e0 = e1 = nullptr;
    }
  }
  fb_forward_launch(variant, sc->desc, sc->items, sc->ctr, (unsigned int *)(sc->ctr + 1), grid, s, e0, e1);
  if (e0) timing_push(e0, e1);
  return hipGetLastError() == hipSuccess ? PRUNE_OK : PRUNE_E_HIP;
}
}  // namespace prune

extern "C" {

prune_status prune_fb_forward(const prune_fb_desc *desc, const void *x, const void *taps,
                              const void *frames, void *y, prune_stream_t stream) {
  prune_status st = check_desc(desc);
  if (st != PRUNE_OK) return st;
  if (!x || !taps || !frames || !y) return PRUNE_E_ARG;
  if (desc->n_frames == 0) return PRUNE_OK;
  const int v = choose_direct_variant(desc, x, taps, frames, y, stream);
  return prune_fb_forward_variant(desc, x, taps, frames, y, v, stream);
}

prune_status prune_fb_forward_noalloc(const prune_fb_desc *desc, const void *x, const void *taps,
                                      const void *frames, void *y, prune_stream_t stream) {
  prune_status st = check_desc(desc);
  if (st != PRUNE_OK) return st;
  if (!x || !taps || !frames || !y) return PRUNE_E_ARG;
  if (desc->n_frames == 0) return PRUNE_OK;
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < desc->n_banks; ++b) Lmax = std::max(Lmax, desc->L[b]);
  // never the autotuner (it allocates its trial batch): the forced variant,
  // else this process's choice for the shape class, else the first variant
  int variant = forced_variant();
  if (!variant) variant = cached_variant(Lmax, desc->Kmax, desc->max_frame_len);
  if (!variant) variant = 1;
  const uint32_t tile = (uint32_t)fb_variant_tile(variant);
  const size_t per = ((size_t)desc->max_frame_len + tile - 1) / tile;
  const size_t items = (size_t)desc->n_frames * (per ? per : 1);
  if (desc->n_frames > PRUNE_NOALLOC_MAX_FRAMES || items > PRUNE_NOALLOC_MAX_ITEMS) {
    set_last_error("prune_fb_forward_noalloc: more frames or tiles than its fixed workspace holds "
                   "(PRUNE_NOALLOC_MAX_FRAMES, PRUNE_NOALLOC_MAX_ITEMS)");
    return PRUNE_E_CAPACITY;
  }
  unsigned char *base = noalloc_workspace();
  if (!base) return PRUNE_E_HIP;
  FbFrameDesc *fd = (FbFrameDesc *)base;
  WorkItem *it = (WorkItem *)(base + kNaDescBytes);
  uint32_t *ctr = (uint32_t *)(base + kNaDescBytes + kNaItemBytes);   // n_items, ticket, err
  hipStream_t s = (hipStream_t)stream;
  // the prep kernel writes the item count and clears the ticket before the
  // forward kernel reads them; the error word is not read on this path
  launch_direct_prep(*desc, (const float2 *)x, (const float2 *)taps, (const prune_fb_frame *)frames,
                     (float2 *)y, tile, fd, it, ctr, ctr + 1, ctr + 2, s);
  const uint32_t grid = (uint32_t)std::min<size_t>((size_t)ncu() * fb_variant_resident(variant), items);
  fb_forward_launch(variant, fd, it, ctr, (unsigned int *)(ctr + 1), grid, s);
  return hipGetLastError() == hipSuccess ? PRUNE_OK : PRUNE_E_HIP;
}

prune_status prune_fb_check_frames(const prune_fb_desc *desc, const void *frames, uint32_t *n_bad,
                                   prune_stream_t stream) {
  if (!desc || !n_bad || (desc->n_frames && !frames)) return PRUNE_E_ARG;
  *n_bad = 0;
  if (desc->n_frames == 0) return PRUNE_OK;
  uint32_t *d_bad = nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (hipMalloc((void **)&d_bad, sizeof(uint32_t)) != hipSuccess) return PRUNE_E_HIP;
  prune_status st = PRUNE_OK;
  if (hipMemsetAsync(d_bad, 0, sizeof(uint32_t), s) != hipSuccess) st = PRUNE_E_HIP;
  if (st == PRUNE_OK) {
    hipLaunchKernelGGL(k_check_frames, dim3((desc->n_frames + 255) / 256), dim3(256), 0, s, *desc,
                       (const prune_fb_frame *)frames, d_bad);
    if (hipMemcpyAsync(n_bad, d_bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = PRUNE_E_HIP;
  }
  (void)hipFree(d_bad);
  return st;
}

prune_status prune_fb_tuned_variant(const prune_fb_desc *desc, int *variant) {
  prune_status st = check_desc(desc);
  if (st != PRUNE_OK) return st;
  if (!variant) return PRUNE_E_ARG;
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < desc->n_banks; ++b) Lmax = std::max(Lmax, desc->L[b]);
  const int f = forced_variant();
  *variant = f ? f : cached_variant(Lmax, desc->Kmax, desc->max_frame_len);
  return PRUNE_OK;
}

prune_status prune_autotune_fb(uint32_t L, uint32_t K, uint32_t n, int *variant) {
  if (L < 1 || L > PRUNE_MAX_L || K < 1 || K > 10 || n < 1) return PRUNE_E_ARG;
  const int v = choose_variant_graph(1, &L, K, n, false);
  if (variant) *variant = v;
  return PRUNE_OK;
}

}  // extern "C"

namespace prune {

static uint32_t length_class(uint32_t n) { return n >= 8192 ? 8192 : (n >= 2048 ? 2048 : 512); }

static std::string bank_list(uint32_t n_banks, const uint32_t *L) {
  std::string r;
  for (uint32_t b = 0; b < n_banks; ++b) r += (b ? "," : "") + std::to_string(L[b]);
  return r;
}

// The variant the autotuner already chose in this process for the direct
// forward's shape class, or 0; never tunes and never allocates.
int cached_variant(uint32_t L, uint32_t K, uint32_t n) {
  const uint32_t nc = length_class(n);
  std::lock_guard<std::mutex> lk(g_mu);
  for (int i = 0; i < g_n_choice; ++i)
    if (g_choice[i].L == L && g_choice[i].K == K && g_choice[i].nc == nc) return g_choice[i].v;
  return 0;
}

static int variant_index(const std::string &name) {
  for (int v = 1; v <= fb_variant_count(); ++v)
    if (name == fb_variant_name(v)) return v;
  return 0;
}

// Time every forward variant on one batch: a warm-up launch of each, then
// kRounds rounds that launch every variant once in turn, each launch timed
// by its own events on `stream`; the smallest median wins.  Returns 0 when
// events cannot be created.
static int time_variants(const prune_fb_desc *d, const void *x, const void *taps, const void *frames,
                         void *y, prune_stream_t stream, float *best_ms) {
  constexpr int kRounds = 5;
  const int nv = fb_variant_count();
  hipStream_t s = (hipStream_t)stream;
  std::vector<hipEvent_t> ev(2 * kRounds * nv, nullptr);
  bool ok = true;
  for (auto &e : ev) ok = ok && hipEventCreate(&e) == hipSuccess;
  int best = 0;
  if (ok) {
    g_tuning = true;
    for (int v = 1; v <= nv; ++v) prune_fb_forward_variant(d, x, taps, frames, y, v, stream);
    for (int r = 0; r < kRounds; ++r)
      for (int v = 1; v <= nv; ++v) {
        hipEvent_t *e = &ev[2 * (r * nv + v - 1)];
        (void)hipEventRecord(e[0], s);
        prune_fb_forward_variant(d, x, taps, frames, y, v, stream);
        (void)hipEventRecord(e[1], s);
      }
    g_tuning = false;
    if (hipStreamSynchronize(s) == hipSuccess) {
      float bm = 1e30f;
      for (int v = 1; v <= nv; ++v) {
        std::vector<float> t(kRounds);
        for (int r = 0; r < kRounds; ++r) {
          hipEvent_t *e = &ev[2 * (r * nv + v - 1)];
          if (hipEventElapsedTime(&t[r], e[0], e[1]) != hipSuccess) t[r] = 1e30f;
        }
        std::sort(t.begin(), t.end());
        if (t[kRounds / 2] < bm) {
          bm = t[kRounds / 2];
          best = v;
        }
      }
      *best_ms = bm;
    }
  }
  for (auto e : ev)
    if (e) (void)hipEventDestroy(e);
  return best;
}

// The direct forward tunes on the call's own frames, input and taps (the
// output is rewritten by the call that follows), once per shape class
// (Lmax, Kmax, frame-length class) and process, unless the cache file
// already holds a choice for the class on this architecture.
static int choose_direct_variant(const prune_fb_desc *desc, const void *x, const void *taps,
                                 const void *frames, void *y, prune_stream_t stream) {
  const int forced = forced_variant();
  if (forced) return forced;
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < desc->n_banks; ++b) Lmax = std::max(Lmax, desc->L[b]);
  const uint32_t K = desc->Kmax, nc = length_class(desc->max_frame_len);
  if (int v = cached_variant(Lmax, K, desc->max_frame_len)) return v;
  const std::string key = "fwd-direct|" + tune_arch() + "|L=" + bank_list(desc->n_banks, desc->L) +
                          "|K=" + std::to_string(K) + "|n=" + std::to_string(nc);
  int v = 0;
  std::string name;
  float ms = 0.f;
  if (tune_cache_lookup(key, &name)) v = variant_index(name);
  const char *env = getenv("PRUNE_AUTOTUNE");
  if (!v && env && env[0] == '0') return 1;
  const bool tuned = !v;
  if (!v) v = time_variants(desc, x, taps, frames, y, stream, &ms);
  if (!v) return 1;
  if (tuned) tune_cache_store(key, fb_variant_name(v), ms);
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_n_choice < kMaxChoices) g_choice[g_n_choice++] = {Lmax, K, nc, v};
  return v;
}

// A graph's filter banks are tuned at finalize, before any data exists, on
// a synthetic batch with the graph's own structure: its banks and tap
// counts, prefix masks of a uniform branch count in a uniform bank, and
// frame lengths of its rate (log-uniform from min(256, rate) up to the rate
// when the rate is a per-firing parameter), about 64K samples per CU.
int choose_variant_graph(uint32_t n_banks, const uint32_t *L, uint32_t K, uint32_t n, bool param) {
  const int forced = forced_variant();
  if (forced) return forced;
  const std::string key = "fwd-graph|" + tune_arch() + "|L=" + bank_list(n_banks, L) + "|K=" +
                          std::to_string(K) + "|n=" + std::to_string(n) + "|param=" +
                          std::to_string(param ? 1 : 0);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  std::string name;
  int v = 0;
  if (tune_cache_lookup(key, &name)) v = variant_index(name);
  const char *env = getenv("PRUNE_AUTOTUNE");
  if (!v && env && env[0] == '0') return 1;
  if (!v) {
    uint32_t Lmax = 1;
    for (uint32_t b = 0; b < n_banks; ++b) Lmax = std::max(Lmax, L[b]);
    const uint64_t target = (uint64_t)ncu() * 65536;
    std::vector<prune_fb_frame> hf;
    uint32_t st = 12345u;
    auto u01 = [&]() {
      st = st * 1664525u + 1013904223u;
      return ((st >> 8) & 0xffffff) / 16777216.0;
    };
    const double lo = std::log((double)std::min<uint32_t>(256, n)), hi = std::log((double)n);
    uint64_t N = 0;
    while (N < target && hf.size() < 65536) {
      prune_fb_frame f{};
      f.n = param ? (uint32_t)std::min<double>(n, std::max(1.0, std::rint(std::exp(lo + (hi - lo) * u01()))))
                  : n;
      const uint32_t k = 1 + (uint32_t)(u01() * K) % K, bank = (uint32_t)(u01() * n_banks) % n_banks;
      f.mask = (k >= 32 ? 0xffffffffu : ((1u << k) - 1u)) << (bank * K);
      f.t0 = (uint32_t)N;
      hf.push_back(f);
      N += f.n;
    }
    uint32_t mfl = 1;
    for (auto &f : hf) mfl = std::max(mfl, f.n);
    prune_fb_desc d{};
    d.n_streams = 1; d.n_frames = (uint32_t)hf.size(); d.stream_len = N; d.n_banks = n_banks;
    d.Kmax = K; d.max_frame_len = mfl;
    for (uint32_t b = 0; b < n_banks; ++b) d.L[b] = L[b];
    const size_t nt = (size_t)n_banks * K * Lmax;
    float2 *x = nullptr, *y = nullptr, *t = nullptr;
    prune_fb_frame *fr = nullptr;
    bool ok = hipMalloc((void **)&x, N * sizeof(float2)) == hipSuccess &&
              hipMalloc((void **)&y, N * sizeof(float2)) == hipSuccess &&
              hipMalloc((void **)&t, nt * sizeof(float2)) == hipSuccess &&
              hipMalloc((void **)&fr, hf.size() * sizeof(prune_fb_frame)) == hipSuccess;
    if (ok) {
      std::vector<float2> hx(N);
      for (auto &z : hx) z = make_float2((float)u01() - 0.5f, (float)u01() - 0.5f);
      std::vector<float2> ht(nt, make_float2(0.01f, -0.02f));
      ok = hipMemcpy(x, hx.data(), N * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(t, ht.data(), nt * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(fr, hf.data(), hf.size() * sizeof(prune_fb_frame), hipMemcpyHostToDevice) ==
               hipSuccess;
    }
    float ms = 0.f;
    if (ok) v = time_variants(&d, x, t, fr, y, nullptr, &ms);
    if (x) (void)hipFree(x);
    if (y) (void)hipFree(y);
    if (t) (void)hipFree(t);
    if (fr) (void)hipFree(fr);
    if (!v) return 1;
    tune_cache_store(key, fb_variant_name(v), ms);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_tuned[key] = v;
  return v;
}

}  // namespace prune
