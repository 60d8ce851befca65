// Filter-bank forward kernels (the fused basis-generation + FIR + branch-sum
// actor of the DPD application, Sec. VII-A; the DPG of poly, FIR_b and add
// merged into one firing as in the actor merging of Sec. VII-A's DNN case).
//
// For one firing with branch mask m over banks of Kmax branches:
//   y[n] = sum_{d in m} sum_{l < L_d} h_d[l] |x[n-l]|^{p_d} x[n-l],  p_d = d mod Kmax
// Within one bank all branches share L, so the branch sum is rewritten per
// (n, l) as a polynomial in r = |x[n-l]| evaluated by Horner's rule:
//   y[n] = sum_l x[n-l] * P_l(r[n-l]),  P_l(r) = sum_{b active} h_b[l] r^{b-1}
// which costs 2(KH-1)+4 fp32 FMAs per (n, l) instead of 4 KH (KH = highest
// active branch + 1 of the bank; inactive lower branches get zero
// coefficients).  The arithmetic is fp32 with FMA contraction; r is the
// correctly rounded sqrtf(re^2 + im^2).
//
// Data layout: frames are complex64 (float2) blocks in HBM.  A work item is
// one tile of T = J*WG consecutive outputs of one frame.  The tile's input
// window [n0 - (Lpad-1), n0 + T) is staged in LDS as three fp32 planes (re,
// im, r) with one pad element per J: lane t reads at stride J+1 words (9 or
// 5, odd, so the lanes of a read fall in distinct banks), and every window
// and coefficient read of a chunk is a constant offset from one base.  At
// 12 bytes per window sample the J = 8, 256-thread kernel needs 33.6 KB of
// LDS, so four workgroups fit on a CU, as many as its registers allow.
// Window positions before the frame come from the frame's halo (the stream's
// past samples), positions after the frame are zero.  Each lane computes J
// consecutive outputs from a register window of 2J-1 samples per chunk of J
// taps; the tap coefficients of the chunk are LDS broadcasts.
#include <hip/hip_ext.h>

#include <algorithm>
#include <atomic>

#include "prune_internal.h"
#include "runtime_kernels.h"

namespace prune {

constexpr int kMaxKH = 10;

// Window layout: one pad element per J in each plane, so position t*J + k
// (k >= 0) is at t*(J+1) + k + k/J: a per-lane part plus a part uniform
// across lanes.  Lanes read words J+1 apart, an odd stride, so they hit
// distinct banks.
template <int J>
__device__ __forceinline__ int pidx(int i) { return i + i / J; }

// Coefficient table layout: tap-major, coef[l * kMaxKH + b], so the
// coefficients of a chunk are at constant offsets from one base.  Chunk c
// holds taps cJ .. cJ+J-1; the last one holds only L - (nchunks-1) J real
// taps (the rest are zero padding) and stops there.
template <int KH, int J, int G, bool PIPE>
__device__ __forceinline__ void horner_pass(const float *__restrict__ wre,
                                            const float *__restrict__ wim,
                                            const float *__restrict__ wrr,
                                            const float2 *__restrict__ coef, int Lpad, int L,
                                            int t, float *accr, float *acci) {
  const int nchunks = Lpad / J;
  for (int c = 0; c < nchunks; ++c) {
    // window positions t*J + k0 + w, k0 = Lpad - (c+1) J (a multiple of J)
    const int k0 = Lpad - c * J - J;
    const int wb = t * (J + 1) + k0 + k0 / J;   // this lane's part plus the chunk's
    const float2 *cb = coef + c * J * kMaxKH;
    float xr[2 * J - 1], xi[2 * J - 1], rr[2 * J - 1];
#pragma unroll
    for (int w = 0; w < 2 * J - 1; ++w) {
      const int q = wb + w + w / J;
      xr[w] = wre[q];
      xi[w] = wim[q];
      rr[w] = wrr[q];
    }
    // PIPE: the coefficients of tap i+1 are read from LDS while tap i
    // computes (every tap index below Lpad is in the table, zero-padded)
    float2 cn[KH];
    if (PIPE) {
#pragma unroll
      for (int b = 0; b < KH; ++b) cn[b] = cb[b];
    }
#pragma unroll
    for (int i = 0; i < J; ++i) {
      if (c * J + i >= L) break;   // uniform: zero-padded taps of the last chunk
      float2 cf[KH];
#pragma unroll
      for (int b = 0; b < KH; ++b) cf[b] = PIPE ? cn[b] : cb[i * kMaxKH + b];
      if (PIPE && i + 1 < J) {
#pragma unroll
        for (int b = 0; b < KH; ++b) cn[b] = cb[(i + 1) * kMaxKH + b];
      }
      // the Horner chains of G outputs advance together, one branch at a
      // time, so a wave has 2G independent FMAs in flight
#pragma unroll
      for (int j0 = 0; j0 < J; j0 += G) {
        float ar[G], ai[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          ar[g] = cf[KH - 1].x;
          ai[g] = cf[KH - 1].y;
        }
#pragma unroll
        for (int b = KH - 2; b >= 0; --b) {
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const int w = j0 + g - i + J - 1;
            ar[g] = fmaf(ar[g], rr[w], cf[b].x);
            ai[g] = fmaf(ai[g], rr[w], cf[b].y);
          }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int j = j0 + g, w = j - i + J - 1;
          accr[j] = fmaf(xr[w], ar[g], accr[j]);
          accr[j] = fmaf(-xi[w], ai[g], accr[j]);
          acci[j] = fmaf(xr[w], ai[g], acci[j]);
          acci[j] = fmaf(xi[w], ar[g], acci[j]);
        }
      }
    }
  }
}

template <int J, int G, bool PIPE>
__device__ __forceinline__ void horner_dispatch(int KH, const float *wre, const float *wim,
                                                const float *wrr, const float2 *coef, int Lpad,
                                                int L, int t, float *accr, float *acci) {
#define PRUNE_HP(k) horner_pass<k, J, G, PIPE>(wre, wim, wrr, coef, Lpad, L, t, accr, acci)
  switch (KH) {
    case 0: break;
    case 1: PRUNE_HP(1); break;
    case 2: PRUNE_HP(2); break;
    case 3: PRUNE_HP(3); break;
    case 4: PRUNE_HP(4); break;
    case 5: PRUNE_HP(5); break;
    case 6: PRUNE_HP(6); break;
    case 7: PRUNE_HP(7); break;
    case 8: PRUNE_HP(8); break;
    case 9: PRUNE_HP(9); break;
    default: PRUNE_HP(10); break;
  }
#undef PRUNE_HP
}

// Persistent forward kernel: each workgroup takes tiles blockIdx.x and
// blockIdx.x + gridDim.x, then further tiles from the item list with an
// atomic ticket (offset by twice the grid size) until the list is
// exhausted.  *ticket must be zero at launch (the producer of the item list
// clears it).
template <int J, int WG, int WAVES, int G, bool PIPE>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(WAVES)))
void k_fb_forward(const FbFrameDesc *__restrict__ frames,
                                                   const WorkItem *__restrict__ items,
                                                   const uint32_t *__restrict__ n_items_ptr,
                                                   unsigned int *__restrict__ ticket) {
  constexpr int T = J * WG;
  constexpr int WMAX = T + PRUNE_MAX_L - 1;
  constexpr int NIT = (WMAX + WG - 1) / WG;   // window elements per thread
  constexpr int WP = WMAX + WMAX / J + 1;   // window length with the pads
  __shared__ float wre[WP], wim[WP], wrr[WP];
  __shared__ float2 coef[kMaxKH * PRUNE_MAX_L];
  __shared__ uint32_t s_next[2];
  const int t = threadIdx.x;
  const uint32_t n_items = *n_items_ptr;
  // the coefficient table in LDS is kept while consecutive tiles share it
  const float2 *tab_taps = nullptr;
  uint32_t tab_key = 0xffffffffu;

  // Window elements k = t + i*WG of the window [n0-(Lpad-1), n0+T) of a tile:
  // positions before the frame come from its halo, after it are zero.
  auto load_window = [&](const FbFrameDesc &dd, int n0x, int Lpadx, float2 *v) {
    const int WN = T + Lpadx - 1, Hx = (int)dd.Lmax - 1, nx = (int)dd.n;
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
      const int k = t + i * WG, p = n0x - (Lpadx - 1) + k;
      v[i] = make_float2(0.f, 0.f);
      if (k < WN) {
        if (p >= 0) {
          if (p < nx) v[i] = dd.x[p];
        } else if (-p <= (int)dd.halo_valid) {
          v[i] = dd.halo[Hx + p];
        }
      }
    }
  };
  // The next tile's window (its first active bank) is loaded into registers
  // while the current tile computes; pv_bank = -1 when nothing is prefetched.
  float2 pv[NIT];
  int pv_bank = -1;
  auto prefetch = [&](uint32_t itx) {
    pv_bank = -1;
    if (itx >= n_items) return;
    const WorkItem wx = items[itx];
    const FbFrameDesc &dx = frames[wx.frame];
    if (dx.route) return;
    const uint32_t kf = dx.Kmax >= 32 ? 0xffffffffu : ((1u << dx.Kmax) - 1u);
    for (uint32_t bank = 0; bank < dx.n_banks; ++bank) {
      if ((dx.mask >> (bank * dx.Kmax)) & kf) {
        const int Lp = ((int)dx.L[bank] + J - 1) / J * J;
        load_window(dx, (int)wx.tile * T, Lp, pv);
        pv_bank = (int)bank;
        return;
      }
    }
  };

  // the first two tiles by workgroup index, later ones by ticket (offset by
  // twice the grid).  Thread 0 takes the ticket of the tile after next at the
  // start of a tile and keeps it in a register, so that its round trip (every
  // workgroup hits the one counter at about the same time) overlaps a whole
  // tile; a list of at most two rounds takes no ticket at all.
  uint32_t it = blockIdx.x;
  uint32_t par = 0;
  uint32_t tk = blockIdx.x + gridDim.x;   // thread 0: the next tile
  const bool tickets = 2ull * gridDim.x < n_items;
  prefetch(it);
  for (;;) {
    if (it >= n_items) break;
    // the next tile, read by all threads after this tile's first barrier
    if (t == 0) {
      s_next[par ^ 1u] = tk;
      tk = tickets ? 2u * gridDim.x + atomicAdd(ticket, 1u) : n_items;
    }
    const WorkItem wi = items[it];
    const FbFrameDesc &d = frames[wi.frame];
    const int n = (int)d.n;
    const int n0 = (int)wi.tile * T;
    const int cur_bank = pv_bank;
    bool fetched = false;
    uint32_t it_next = 0;

    if (d.route) {
      // passthrough-routed frame: y = x over the tile
      for (int k = t; k < T; k += WG) {
        const int p = n0 + k;
        if (p < n) {
          const float2 v = d.x[p];
          for (uint32_t o = 0; o < d.n_y; ++o) d.y[o][p] = v;
        }
      }
    } else {
      float accr[J], acci[J];
#pragma unroll
      for (int j = 0; j < J; ++j) accr[j] = acci[j] = 0.f;
      const uint32_t kfull = d.Kmax >= 32 ? 0xffffffffu : ((1u << d.Kmax) - 1u);
      for (uint32_t bank = 0; bank < d.n_banks; ++bank) {
        const uint32_t bmask = (d.mask >> (bank * d.Kmax)) & kfull;
        if (!bmask) continue;
        const int KH = 32 - __clz(bmask);
        const int L = (int)d.L[bank];
        const int Lpad = (L + J - 1) / J * J;
        float2 v[NIT];
        if ((int)bank == cur_bank) {
#pragma unroll
          for (int i = 0; i < NIT; ++i) v[i] = pv[i];
        } else {
          load_window(d, n0, Lpad, v);
        }
        __syncthreads();   // earlier readers of win / coef are done
        {
          const int WN = T + Lpad - 1;
#pragma unroll
          for (int i = 0; i < NIT; ++i) {
            const int k = t + i * WG;
            if (k < WN) {
              const int q = pidx<J>(k);
              wre[q] = v[i].x;
              wim[q] = v[i].y;
              wrr[q] = sqrtf(v[i].x * v[i].x + v[i].y * v[i].y);
            }
          }
        }
        const float2 *tb = d.taps + (size_t)bank * d.Kmax * d.Lmax;
        const uint32_t key = bmask | ((uint32_t)L << 16) | (bank << 24);
        if (tb != tab_taps || key != tab_key) {   // uniform: same frame descriptor for all threads
          tab_taps = tb;
          tab_key = key;
          for (int k = t; k < KH * Lpad; k += WG) {
            const int b = k / Lpad, l = k - b * Lpad;
            float2 c = make_float2(0.f, 0.f);
            if (((bmask >> b) & 1u) && l < L) c = tb[(size_t)b * d.Lmax + l];
            coef[l * kMaxKH + b] = c;
          }
        }
        __syncthreads();
        if (!fetched) {
          fetched = true;
          it_next = s_next[par ^ 1u];
          prefetch(it_next);   // in flight during the compute below
        }
        // a wave whose outputs all lie beyond the frame's end (the last tile
        // of a frame) stores nothing and skips the arithmetic (KH 0); the
        // condition is uniform across the wave
        horner_dispatch<J, G, PIPE>(n0 + (t & ~63) * J < n ? KH : 0, wre, wim, wrr, coef, Lpad, L,
                                    t, accr, acci);
      }
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int p = n0 + t * J + j;
        if (p < n) {
          const float2 v = make_float2(accr[j], acci[j]);
          for (uint32_t o = 0; o < d.n_y; ++o) d.y[o][p] = v;
        }
      }
    }
    __syncthreads();
    if (!fetched) {
      it_next = s_next[par ^ 1u];
      prefetch(it_next);
    }
    it = it_next;
    par ^= 1u;
  }
}

// ---------------------------------------------------------------- variants
struct FbVariant {
  const char *name;
  int tile, WG;   // outputs per work item, threads per workgroup
  void (*launch)(const FbFrameDesc *, const WorkItem *, const uint32_t *, unsigned int *,
                 uint32_t grid, hipStream_t, hipEvent_t, hipEvent_t);
  int (*resident)();   // workgroups of the kernel resident per CU
};

template <int J, int WG, int WAVES, int G = J, bool PIPE = false>
static int fwd_resident() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(
                                                           &k_fb_forward<J, WG, WAVES, G, PIPE>),
                                                   WG, 0) != hipSuccess)
    n = 0;
  return n;
}

// With events, the dispatch itself records the kernel's start and end
// (hipExtLaunchKernelGGL): no marker packets, no gaps around the kernel.
template <int J, int WG, int WAVES, int G = J, bool PIPE = false>
static void launch_fwd(const FbFrameDesc *f, const WorkItem *it, const uint32_t *n,
                       unsigned int *ticket, uint32_t grid, hipStream_t s, hipEvent_t e0,
                       hipEvent_t e1) {
  if (e0 || e1)
    hipExtLaunchKernelGGL((k_fb_forward<J, WG, WAVES, G, PIPE>), dim3(grid), dim3(WG), 0, s, e0, e1, 0,
                          f, it, n, ticket);
  else
    hipLaunchKernelGGL((k_fb_forward<J, WG, WAVES, G, PIPE>), dim3(grid), dim3(WG), 0, s, f, it, n,
                       ticket);
}

static const FbVariant kVariants[] = {
    // vector Horner kernels: J outputs per lane, WG threads, waves-per-EU
    // hint, Horner chains of G outputs advanced together, next tap's
    // coefficients read ahead (p) or not (g)
    {"valu_horner_J8_WG256_p4", 8 * 256, 256, launch_fwd<8, 256, 1, 4, true>,
      fwd_resident<8, 256, 1, 4, true>},
    {"valu_horner_J4_WG256_w3", 4 * 256, 256, launch_fwd<4, 256, 3>,
      fwd_resident<4, 256, 3>},
    {"valu_horner_J8_WG128_w2", 8 * 128, 128, launch_fwd<8, 128, 2>,
      fwd_resident<8, 128, 2>},
    {"valu_horner_J4_WG128_w4", 4 * 128, 128, launch_fwd<4, 128, 4>,
      fwd_resident<4, 128, 4>},
    {"valu_horner_J8_WG256_p2", 8 * 256, 256, launch_fwd<8, 256, 1, 2, true>,
      fwd_resident<8, 256, 1, 2, true>},
    // matrix-core block-Toeplitz kernels: NT result tiles per wave, NW waves
    {"mfma_toeplitz_NT4_W4", 4 * 256 * 4, 256, launch_fb_mfma<4, 4>,
      fb_mfma_resident<4, 4>},
    {"mfma_toeplitz_NT2_W4", 2 * 256 * 4, 256, launch_fb_mfma<2, 4>,
      fb_mfma_resident<2, 4>},
    {"mfma_toeplitz_NT4_W2", 4 * 256 * 2, 128, launch_fb_mfma<4, 2>,
      fb_mfma_resident<4, 2>},
};

int fb_variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
const char *fb_variant_name(int v) {
  return (v >= 1 && v <= fb_variant_count()) ? kVariants[v - 1].name : "auto";
}
int fb_variant_tile(int v) { return kVariants[v - 1].tile; }
int fb_variant_wg(int v) { return kVariants[v - 1].WG; }

// Queried once per variant (on the current device; every device here is
// the same gfx950 part).
int fb_variant_resident(int v) {
  static std::atomic<int> cache[sizeof(kVariants) / sizeof(kVariants[0])] = {};
  int n = cache[v - 1].load();
  if (n <= 0) {
    n = std::max(1, kVariants[v - 1].resident());
    cache[v - 1].store(n);
  }
  return n;
}

void fb_forward_launch(int v, const FbFrameDesc *frames, const WorkItem *items,
                       const uint32_t *n_items, unsigned int *ticket, uint32_t grid,
                       hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  kVariants[v - 1].launch(frames, items, n_items, ticket, grid, s, e0, e1);
}

}  // namespace prune
