// Direct filter-bank operations over whole streams (prune_fb_forward) and
// the forward-kernel autotuner.  The direct forward builds one frame
// descriptor per frame and the tile work list on the device, then runs the
// same persistent forward kernel as the graph executor.
#include <hip/hip_runtime.h>

#include <chrono>
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
std::map<std::tuple<uint32_t, uint32_t, uint32_t>, int> g_tuned;
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
int choose_variant(uint32_t L, uint32_t K, uint32_t n);
int cached_variant(uint32_t L, uint32_t K, uint32_t n);

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
  // four workgroups per CU, the residency of the J = 8, 256-thread forward kernels
  const uint32_t grid = (uint32_t)std::min<size_t>((size_t)ncu() * 4, items);
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
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < desc->n_banks; ++b) Lmax = std::max(Lmax, desc->L[b]);
  const int v = choose_variant(Lmax, desc->Kmax, desc->max_frame_len);
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
  const uint32_t grid = (uint32_t)std::min<size_t>((size_t)ncu() * 4, items);
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

prune_status prune_autotune_fb(uint32_t L, uint32_t K, uint32_t n, int *variant) {
  if (L < 1 || L > PRUNE_MAX_L || K < 1 || K > 10 || n < 1) return PRUNE_E_ARG;
  const int v = choose_variant(L, K, n);
  if (variant) *variant = v;
  return PRUNE_OK;
}

}  // extern "C"

namespace prune {

extern int forced_variant();

// Time each forward variant on a synthetic batch of the shape class and keep
// the fastest.  Key: (L, K, frame length class); L is exact because the
// kernels pad the tap count to different chunk sizes.
static uint32_t length_class(uint32_t n) { return n >= 8192 ? 8192 : (n >= 2048 ? 2048 : 512); }

// The variant the autotuner already chose in this process for the shape
// class, or 0; never tunes.
int cached_variant(uint32_t L, uint32_t K, uint32_t n) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tuned.find(std::make_tuple(L, K, length_class(n)));
  return it == g_tuned.end() ? 0 : it->second;
}

int choose_variant(uint32_t L, uint32_t K, uint32_t n) {
  const int forced = forced_variant();
  if (forced) return forced;
  const uint32_t Lc = L;
  const uint32_t nc = length_class(n);
  const auto key = std::make_tuple(Lc, K, nc);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  const char *env = getenv("PRUNE_AUTOTUNE");
  if (env && env[0] == '0') return 1;
  // synthetic problem: 64K samples per CU (16.7M on 256 CUs), long enough
  // that launch overhead and tail effects do not decide the ranking
  const uint32_t frames = std::max<uint32_t>(64, (uint32_t)((size_t)ncu() * 65536 / nc));
  const uint64_t N = (uint64_t)frames * nc;
  float2 *x = nullptr, *y = nullptr, *t = nullptr;
  prune_fb_frame *fr = nullptr;
  int best = 1;
  if (hipMalloc((void **)&x, N * sizeof(float2)) != hipSuccess) return 1;
  (void)hipMalloc((void **)&y, N * sizeof(float2));
  (void)hipMalloc((void **)&t, (size_t)K * Lc * sizeof(float2));
  (void)hipMalloc((void **)&fr, frames * sizeof(prune_fb_frame));
  {
    std::vector<float2> hx(N);
    uint32_t s = 12345u;
    for (auto &v : hx) {
      s = s * 1664525u + 1013904223u;
      v.x = ((s >> 8) & 0xffff) / 65536.f - 0.5f;
      s = s * 1664525u + 1013904223u;
      v.y = ((s >> 8) & 0xffff) / 65536.f - 0.5f;
    }
    (void)hipMemcpy(x, hx.data(), N * sizeof(float2), hipMemcpyHostToDevice);
    std::vector<float2> ht((size_t)K * Lc, make_float2(0.01f, -0.02f));
    (void)hipMemcpy(t, ht.data(), ht.size() * sizeof(float2), hipMemcpyHostToDevice);
    std::vector<prune_fb_frame> hf(frames);
    for (uint32_t f = 0; f < frames; ++f) {
      hf[f].stream = 0; hf[f].t0 = f * nc; hf[f].n = nc;
      hf[f].mask = K >= 32 ? 0xffffffffu : ((1u << K) - 1u); hf[f].route = 0;
      hf[f].pad[0] = hf[f].pad[1] = hf[f].pad[2] = 0;
    }
    (void)hipMemcpy(fr, hf.data(), frames * sizeof(prune_fb_frame), hipMemcpyHostToDevice);
  }
  prune_fb_desc d{};
  d.n_streams = 1; d.n_frames = frames; d.stream_len = N; d.n_banks = 1; d.Kmax = K;
  d.L[0] = Lc; d.max_frame_len = nc;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  float best_ms = 1e30f;
  g_tuning = true;
  for (int v = 1; v <= fb_variant_count(); ++v) {
    prune_fb_forward_variant(&d, x, t, fr, y, v, nullptr);   // warm-up
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < 3; ++r) prune_fb_forward_variant(&d, x, t, fr, y, v, nullptr);
    (void)hipEventRecord(e1, nullptr);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  g_tuning = false;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(x); (void)hipFree(y); (void)hipFree(t); (void)hipFree(fr);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned[key] = best;
  }
  if (const char *path = getenv("PRUNE_AUTOTUNE_CACHE")) {
    if (FILE *f = fopen(path, "a")) {
      fprintf(f, "{\"arch\": \"gfx950\", \"L\": %u, \"K\": %u, \"n\": %u, \"variant\": \"%s\", \"ms\": %.4f}\n",
              Lc, K, nc, fb_variant_name(best), best_ms);
      fclose(f);
    }
  }
  return best;
}

}  // namespace prune
