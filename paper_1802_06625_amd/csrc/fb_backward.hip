// Adjoint of the filter bank over whole streams (prune_fb_backward).
//
// For a real loss with grad = dL/dRe + i dL/dIm, cotangent g = grad_y,
// p = b-1, r = |x|, and G_b[m] = sum_l conj(h_b[l]) g[m+l] over outputs of
// frames where branch b is active:
//   grad_h_b[l] = sum_n g[n] conj(x[n-l]) r[n-l]^p
//   grad_x[m]   = sum_b (p/2+1) r^p G_b + (p/2) r^(p-2) x^2 conj(G_b)
//               = S1 + (x^2 / r^2) S2,
//   S1 = sum_l g[m+l]       Q_l(r),  Q_l(r) = sum_b (p/2+1) conj(h_b[l]) r^p
//   S2 = sum_l conj(g[m+l]) T_l(r),  T_l(r) = sum_b (p/2)   h_b[l]       r^p
// Q_l and T_l are evaluated by Horner's rule in r (the |x|^p basis is
// recomputed, never stored); S2 carries r^p with p >= 1, so the term is zero
// at r = 0 and x^2/r^2 has magnitude 1.  Passthrough frames pass g through.
//
// Kernels (one tile = T consecutive outputs of one frame, as in the forward):
//  k_bwd_prep   frame descriptors, tile list, per-stream tile ranges;
//  k_bwd_main   per tile: grad_x at the tile's inputs from the frame's own
//               outputs, and the tile's grad_h partial (fp32, reduced over
//               the tile in a fixed order);
//  k_bwd_halo   per frame: gradient of the Lmax-1 past samples its window
//               reads (contributions that belong to earlier frames);
//  k_bwd_fix    adds those halo gradients into the earlier frames' grad_x
//               (each element written by exactly one thread); when the tap
//               gradient is wanted too, the same work runs in the first
//               workgroups of k_bwd_reduce1;
//  k_bwd_reduce1/2  fixed-order float64 sums of the tile partials per stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "prune.h"
#include "prune_internal.h"
#include "runtime_kernels.h"
#include "bwd_common.h"

namespace prune {

constexpr int kBJ = 4;          // inputs per lane for grad_x
constexpr int kBWG = 256;
static_assert(kBJ * kBWG == kBT, "vector backward tile");

__device__ __forceinline__ int bidx(int i) { return i + (i >> 3); }

// Per-stream sums of covered samples are kept in LDS for up to this many
// streams (global atomics beyond).
constexpr uint32_t kPrepCovLds = 1024;

__global__ __launch_bounds__(1024) void k_bwd_prep(prune_fb_desc d, const float2 *x,
                                                   const float2 *taps, const prune_fb_frame *fr,
                                                   const float2 *g, float2 *gx, BwdFrame *bf,
                                                   WorkItem *items, uint32_t *n_items,
                                                   uint32_t *s_begin, uint32_t *s_end,
                                                   unsigned long long *cov, uint32_t *sfirst,
                                                   uint32_t tile) {
  __shared__ uint32_t sm[32];
  __shared__ uint32_t s_carry;
  __shared__ uint32_t s_pre[1024], s_tl[1024];
  __shared__ unsigned long long s_cov[kPrepCovLds];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = max(Lmax, d.L[b]);
  const size_t tstride = (size_t)d.n_banks * d.Kmax * Lmax;
  const bool lds_cov = d.n_streams <= kPrepCovLds;
  for (uint32_t s = tid; s < d.n_streams; s += nt) {
    s_begin[s] = 0; s_end[s] = 0; cov[s] = 0ull; sfirst[s] = 0xffffffffu;
    if (lds_cov) s_cov[s] = 0ull;
  }
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < d.n_frames; base += nt) {
    const uint32_t f = base + tid;
    uint32_t tiles = 0;
    prune_fb_frame q;
    if (f < d.n_frames) {
      q = fr[f];
      const bool ok = q.stream < d.n_streams && (uint64_t)q.t0 + q.n <= d.stream_len &&
                      q.n <= d.max_frame_len;
      BwdFrame b;
      const size_t so = (size_t)q.stream * d.stream_len + q.t0;
      b.x = x + so; b.g = g + so; b.gx = gx + so;
      b.taps = taps + (size_t)q.stream * tstride;
      b.n = ok ? q.n : 0; b.mask = q.mask; b.route = q.route; b.t0 = q.t0; b.stream = q.stream;
      b.pad0 = b.pad1 = b.pad2 = 0;
      bf[f] = b;
      tiles = (b.n + tile - 1) / tile;
      if (b.n) {   // samples covered
        if (lds_cov) atomicAdd(&s_cov[q.stream], (unsigned long long)b.n);
        else atomicAdd(&cov[q.stream], (unsigned long long)b.n);
      }
      if (q.stream < d.n_streams && (f == 0 || fr[f - 1].stream != q.stream)) sfirst[q.stream] = f;
    }
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
    if (f < d.n_frames) {
      if (q.stream < d.n_streams) {
        if (f == 0 || fr[f - 1].stream != q.stream) s_begin[q.stream] = pre;
        if (f + 1 == d.n_frames || fr[f + 1].stream != q.stream) s_end[q.stream] = pre + tiles;
      }
    }
    __syncthreads();
    if (tid == 0) s_carry += sm[nw - 1];
    __syncthreads();
  }
  if (tid == 0) {
    n_items[0] = s_carry;
    n_items[1] = 0u;   // work tickets of the matrix-core adjoint kernels
    n_items[2] = 0u;
  }
  __syncthreads();
  if (lds_cov)
    for (uint32_t s = tid; s < d.n_streams; s += nt) cov[s] = s_cov[s];
}

// Zero grad_x of streams whose frames do not cover every sample (the
// kernels write grad_x only inside frames).  Workgroup (stream, chunk).
__global__ __launch_bounds__(256) void k_bwd_gapfill(prune_fb_desc d, const unsigned long long *cov,
                                                     float2 *gx) {
  const uint32_t s = blockIdx.x;
  if (cov[s] == (unsigned long long)d.stream_len) return;
  const uint64_t per = (d.stream_len + gridDim.y - 1) / gridDim.y;
  const uint64_t lo = (uint64_t)blockIdx.y * per, hi = min(lo + per, (uint64_t)d.stream_len);
  float2 *row = gx + (size_t)s * d.stream_len;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) row[i] = make_float2(0.f, 0.f);
}

// grad_x of the J inputs a lane owns for one chunk of J taps.
template <int KH>
__device__ __forceinline__ void gx_pass(const float2 *__restrict__ gw, const float2 *__restrict__ cq,
                                        const float2 *__restrict__ ct, int Lpad, int t,
                                        const float *rm, float *s1r, float *s1i, float *s2r,
                                        float *s2i) {
  for (int c = 0; c < Lpad / kBJ; ++c) {
    float gr[2 * kBJ - 1], gi[2 * kBJ - 1];
#pragma unroll
    for (int w = 0; w < 2 * kBJ - 1; ++w) {
      const float2 v = gw[bidx(t * kBJ + c * kBJ + w)];
      gr[w] = v.x;
      gi[w] = v.y;
    }
#pragma unroll
    for (int i = 0; i < kBJ; ++i) {
      const int l = c * kBJ + i;
      float2 q[KH], tt[KH];
#pragma unroll
      for (int b = 0; b < KH; ++b) {
        q[b] = cq[b * Lpad + l];
        tt[b] = ct[b * Lpad + l];
      }
#pragma unroll
      for (int j = 0; j < kBJ; ++j) {
        const int w = j + i;
        float qr = q[KH - 1].x, qi = q[KH - 1].y, tr = tt[KH - 1].x, ti = tt[KH - 1].y;
#pragma unroll
        for (int b = KH - 2; b >= 0; --b) {
          qr = fmaf(qr, rm[j], q[b].x);
          qi = fmaf(qi, rm[j], q[b].y);
          tr = fmaf(tr, rm[j], tt[b].x);
          ti = fmaf(ti, rm[j], tt[b].y);
        }
        // S1 += g * Q ; S2 += conj(g) * T
        s1r[j] = fmaf(gr[w], qr, s1r[j]);
        s1r[j] = fmaf(-gi[w], qi, s1r[j]);
        s1i[j] = fmaf(gr[w], qi, s1i[j]);
        s1i[j] = fmaf(gi[w], qr, s1i[j]);
        s2r[j] = fmaf(gr[w], tr, s2r[j]);
        s2r[j] = fmaf(gi[w], ti, s2r[j]);
        s2i[j] = fmaf(gr[w], ti, s2i[j]);
        s2i[j] = fmaf(-gi[w], tr, s2i[j]);
      }
    }
  }
}

__device__ __forceinline__ void gx_dispatch(int KH, const float2 *gw, const float2 *cq,
                                            const float2 *ct, int Lpad, int t, const float *rm,
                                            float *a, float *b, float *c, float *d) {
  switch (KH) {
    case 1: gx_pass<1>(gw, cq, ct, Lpad, t, rm, a, b, c, d); break;
    case 2: gx_pass<2>(gw, cq, ct, Lpad, t, rm, a, b, c, d); break;
    case 3: gx_pass<3>(gw, cq, ct, Lpad, t, rm, a, b, c, d); break;
    case 4: gx_pass<4>(gw, cq, ct, Lpad, t, rm, a, b, c, d); break;
    case 5: gx_pass<5>(gw, cq, ct, Lpad, t, rm, a, b, c, d); break;
    case 6: gx_pass<6>(gw, cq, ct, Lpad, t, rm, a, b, c, d); break;
    case 7: gx_pass<7>(gw, cq, ct, Lpad, t, rm, a, b, c, d); break;
    case 8: gx_pass<8>(gw, cq, ct, Lpad, t, rm, a, b, c, d); break;
    case 9: gx_pass<9>(gw, cq, ct, Lpad, t, rm, a, b, c, d); break;
    default: gx_pass<10>(gw, cq, ct, Lpad, t, rm, a, b, c, d); break;
  }
}

// Coefficients of Q_l and T_l for one bank of a frame (zero for inactive branches).
__device__ inline void load_coefs(const float2 *tb, uint32_t Lmax, uint32_t bmask, int KH, int L,
                                  int Lpad, float2 *cq, float2 *ct) {
  for (int k = threadIdx.x; k < KH * Lpad; k += blockDim.x) {
    const int b = k / Lpad, l = k - b * Lpad;
    float2 h = make_float2(0.f, 0.f);
    if (((bmask >> b) & 1u) && l < L) h = tb[(size_t)b * Lmax + l];
    const float al = 0.5f * (float)b + 1.f, be = 0.5f * (float)b;
    cq[k] = make_float2(al * h.x, -al * h.y);
    ct[k] = make_float2(be * h.x, be * h.y);
  }
}

__global__ __launch_bounds__(kBWG) void k_bwd_main(prune_fb_desc d, const BwdFrame *__restrict__ bf,
                                                  const WorkItem *__restrict__ items,
                                                  const uint32_t *__restrict__ n_items,
                                                  float2 *__restrict__ partial) {
  constexpr int WM = kBT + PRUNE_MAX_L - 1;
  __shared__ float4 xw[WM + (WM >> 3) + 1];   // x window {re, im, r, 0}, positions n0-(Lpad-1) ..
  __shared__ float2 gw[WM + (WM >> 3) + 1];   // g window, positions n0 .. n0+T+Lpad-2
  __shared__ float2 cq[10 * PRUNE_MAX_L], ct[10 * PRUNE_MAX_L];
  __shared__ float2 red[kBWG];                // grad_h chunk partials
  const int t = threadIdx.x;
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = max(Lmax, d.L[b]);
  const uint32_t D = d.n_banks * d.Kmax;
  const uint32_t ni = *n_items;
  for (uint32_t it = blockIdx.x; it < ni; it += gridDim.x) {
    const WorkItem wi = items[it];
    const BwdFrame F = bf[wi.frame];
    const int n = (int)F.n, n0 = (int)wi.tile * kBT;
    float2 *prow = partial + (size_t)it * D * Lmax;
    if (F.route) {
      for (int k = t; k < kBT; k += kBWG)
        if (n0 + k < n) F.gx[n0 + k] = F.g[n0 + k];
      for (uint32_t k = t; k < D * Lmax; k += kBWG) prow[k] = make_float2(0.f, 0.f);
      __syncthreads();
      continue;
    }
    float s1r[kBJ], s1i[kBJ], s2r[kBJ], s2i[kBJ], xr[kBJ], xi[kBJ], rm[kBJ];
#pragma unroll
    for (int j = 0; j < kBJ; ++j) s1r[j] = s1i[j] = s2r[j] = s2i[j] = xr[j] = xi[j] = rm[j] = 0.f;
    const uint32_t kfull = (1u << d.Kmax) - 1u;
    for (uint32_t bank = 0; bank < d.n_banks; ++bank) {
      const uint32_t bmask = (F.mask >> (bank * d.Kmax)) & kfull;
      float2 *brow = prow + (size_t)bank * d.Kmax * Lmax;
      if (!bmask) {
        for (uint32_t k = t; k < d.Kmax * Lmax; k += kBWG) brow[k] = make_float2(0.f, 0.f);
        continue;
      }
      const int KH = 32 - __clz(bmask);
      const int L = (int)d.L[bank];
      const int Lpad = (L + kBJ - 1) / kBJ * kBJ;
      __syncthreads();
      for (int k = t; k < kBT + Lpad - 1; k += kBWG) {
        const int p = n0 - (Lpad - 1) + k;   // x window
        float2 v = make_float2(0.f, 0.f);
        if (p < n && p >= -(int)F.t0) v = F.x[p];
        xw[bidx(k)] = make_float4(v.x, v.y, sqrtf(v.x * v.x + v.y * v.y), 0.f);
        const int q = n0 + k;                // g window (outputs of this frame only)
        gw[bidx(k)] = q < n ? F.g[q] : make_float2(0.f, 0.f);
      }
      load_coefs(F.taps + (size_t)bank * d.Kmax * Lmax, Lmax, bmask, KH, L, Lpad, cq, ct);
      __syncthreads();
      // ---- grad_x of inputs n0 + t*J + j
#pragma unroll
      for (int j = 0; j < kBJ; ++j) {
        const float4 v = xw[bidx(t * kBJ + j + Lpad - 1)];
        xr[j] = v.x; xi[j] = v.y; rm[j] = v.z;
      }
      gx_dispatch(KH, gw, cq, ct, Lpad, t, rm, s1r, s1i, s2r, s2i);
      // ---- grad_h partial of this tile: lane l = t % Lpad, chunk = t / Lpad
      if (Lpad <= kBWG) {
        const int nch = kBWG / Lpad, l = t % Lpad, ch = t / Lpad;
        const int per = (kBT + nch - 1) / nch;
        float ar[10], ai[10];
#pragma unroll
        for (int b = 0; b < 10; ++b) ar[b] = ai[b] = 0.f;
        if (ch < nch) {
          const int hi = min(kBT, (ch + 1) * per);
#pragma unroll 4
          for (int k = ch * per; k < hi; ++k) {
            const float2 gv = gw[bidx(k)];
            const float4 xv = xw[bidx(k - l + Lpad - 1)];
            // w = g * conj(x)
            const float wr = gv.x * xv.x + gv.y * xv.y;
            const float wi2 = gv.y * xv.x - gv.x * xv.y;
            float rp = 1.f;
#pragma unroll
            for (int b = 0; b < 10; ++b) {
              if (b < KH) {
                ar[b] = fmaf(wr, rp, ar[b]);
                ai[b] = fmaf(wi2, rp, ai[b]);
                rp *= xv.z;
              }
            }
          }
        }
        // fixed-order reduction over the chunks of each (b, l)
        for (int b = 0; b < KH; ++b) {
          __syncthreads();
          if (ch < nch) red[ch * Lpad + l] = make_float2(ar[b], ai[b]);
          __syncthreads();
          if (t < Lpad) {
            float sr = 0.f, si = 0.f;
            for (int q = 0; q < nch; ++q) {
              sr += red[q * Lpad + t].x;
              si += red[q * Lpad + t].y;
            }
            const bool act = ((bmask >> b) & 1u) && t < L;
            if (t < (int)Lmax) brow[(size_t)b * Lmax + t] = act ? make_float2(sr, si) : make_float2(0.f, 0.f);
          }
        }
        for (uint32_t k = t; k < d.Kmax * Lmax; k += kBWG) {
          const uint32_t b = k / Lmax, l2 = k - b * Lmax;
          if ((int)b >= KH || (int)l2 >= Lpad) brow[k] = make_float2(0.f, 0.f);
        }
      }
    }
    // ---- grad_x = S1 + (x^2/r^2) S2 for the inputs of this tile
#pragma unroll
    for (int j = 0; j < kBJ; ++j) {
      const int m = n0 + t * kBJ + j;
      if (m < n) {
        float gr = s1r[j], gi = s1i[j];
        const float r2 = xr[j] * xr[j] + xi[j] * xi[j];
        if (r2 > 0.f) {
          const float er = (xr[j] * xr[j] - xi[j] * xi[j]) / r2, ei = 2.f * xr[j] * xi[j] / r2;
          gr += er * s2r[j] - ei * s2i[j];
          gi += er * s2i[j] + ei * s2r[j];
        }
        F.gx[m] = make_float2(gr, gi);
      }
    }
    __syncthreads();
  }
}

// Gradient of the Lmax-1 stream samples before each filter-bank frame (its
// window's halo) from that frame's outputs: one workgroup per frame.
__global__ __launch_bounds__(64) void k_bwd_halo(prune_fb_desc d, const BwdFrame *__restrict__ bf,
                                                 float2 *__restrict__ hg) {
  const uint32_t f = blockIdx.x;
  if (f >= d.n_frames) return;
  const BwdFrame F = bf[f];
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = max(Lmax, d.L[b]);
  const int H = (int)Lmax - 1;
  const int k = threadIdx.x;
  __shared__ float2 tl[PRUNE_MAX_BRANCHES * PRUNE_MAX_L];
  __shared__ float2 gl[PRUNE_MAX_L];       // the frame's first H outputs' cotangent
  const uint32_t E = d.n_banks * d.Kmax * Lmax;
  if (!F.route && F.n) {
    for (uint32_t e = threadIdx.x; e < E; e += blockDim.x) tl[e] = F.taps[e];
    for (int e = threadIdx.x; e < H; e += blockDim.x)
      gl[e] = e < (int)F.n ? F.g[e] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  if (k >= H) return;
  const int m = k - H;                     // position relative to the frame start
  float2 out = make_float2(0.f, 0.f);
  if (!F.route && F.n && (int)F.t0 + m >= 0) {
    const float2 xv = F.x[m];
    const float r = sqrtf(xv.x * xv.x + xv.y * xv.y);
    float s1r = 0.f, s1i = 0.f, s2r = 0.f, s2i = 0.f;
    const uint32_t kfull = (1u << d.Kmax) - 1u;
    for (uint32_t bank = 0; bank < d.n_banks; ++bank) {
      const uint32_t bmask = (F.mask >> (bank * d.Kmax)) & kfull;
      if (!bmask) continue;
      const int KH = 32 - __clz(bmask);
      const int L = (int)d.L[bank];
      const float2 *tb = tl + (size_t)bank * d.Kmax * Lmax;
      for (int l = -m; l < L && m + l < (int)F.n; ++l) {
        float qr = 0.f, qi = 0.f, tr = 0.f, ti = 0.f;
        for (int b = KH - 1; b >= 0; --b) {
          float2 h = make_float2(0.f, 0.f);
          if ((bmask >> b) & 1u) h = tb[(size_t)b * Lmax + l];
          const float al = 0.5f * (float)b + 1.f, be = 0.5f * (float)b;
          qr = fmaf(qr, r, al * h.x);
          qi = fmaf(qi, r, -al * h.y);
          tr = fmaf(tr, r, be * h.x);
          ti = fmaf(ti, r, be * h.y);
        }
        const float2 gv = gl[m + l];
        s1r += gv.x * qr - gv.y * qi;
        s1i += gv.x * qi + gv.y * qr;
        s2r += gv.x * tr + gv.y * ti;
        s2i += gv.x * ti - gv.y * tr;
      }
    }
    const float r2 = xv.x * xv.x + xv.y * xv.y;
    out = make_float2(s1r, s1i);
    if (r2 > 0.f) {
      const float er = (xv.x * xv.x - xv.y * xv.y) / r2, ei = 2.f * xv.x * xv.y / r2;
      out.x += er * s2r - ei * s2i;
      out.y += er * s2i + ei * s2r;
    }
  }
  hg[(size_t)f * H + k] = out;
}

// Add the halo gradients into grad_x.  Stream sample q before a frame start
// (q in [t0 - H, t0)) is owned by the first frame of its stream that starts
// after q; that frame's thread (frame, q - (t0 - H)) adds, in frame order,
// the halo gradients of every frame whose window covers q.  Samples inside an
// earlier frame already hold that frame's own contribution; samples in a gap
// between frames hold zero.  Each sample is written by one thread, no atomics.
__device__ void bwd_fix_frame(const prune_fb_desc &d, const prune_fb_frame *__restrict__ fr,
                              const BwdFrame *__restrict__ bf, const float2 *__restrict__ hg,
                              float2 *__restrict__ gx, uint32_t f) {
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = max(Lmax, d.L[b]);
  const int H = (int)Lmax - 1;
  const int k = threadIdx.x;
  const prune_fb_frame G = fr[f];
  if (k >= H || G.stream >= d.n_streams) return;
  const int64_t q = (int64_t)G.t0 - H + k;
  if (q < 0) return;
  if (f > 0 && fr[f - 1].stream == G.stream && q < (int64_t)fr[f - 1].t0) return;   // not the owner
  float2 acc = make_float2(0.f, 0.f);
  for (uint32_t f2 = f; f2 < d.n_frames; ++f2) {
    const prune_fb_frame G2 = fr[f2];
    if (G2.stream != G.stream || (int64_t)G2.t0 - H > q) break;
    if (G2.route || !bf[f2].n) continue;
    const float2 v = hg[(size_t)f2 * H + (size_t)(q - ((int64_t)G2.t0 - H))];
    acc.x += v.x;
    acc.y += v.y;
  }
  float2 &out = gx[(size_t)G.stream * d.stream_len + (size_t)q];
  out = make_float2(out.x + acc.x, out.y + acc.y);
}

__global__ __launch_bounds__(64) void k_bwd_fix(prune_fb_desc d, const prune_fb_frame *__restrict__ fr,
                                                const BwdFrame *__restrict__ bf,
                                                const float2 *__restrict__ hg, float2 *__restrict__ gx) {
  if (blockIdx.x < d.n_frames) bwd_fix_frame(d, fr, bf, hg, gx, blockIdx.x);
}

// The two reduction stages (bwd_common.h) as kernels: workgroup (stream,
// entry block, chunk) and (stream, entry block).
// Stage 1, one workgroup per (chunk, entry block, stream) in that order
// along x; the first n_fix workgroups do the halo fix-up of frames 0 ..
// n_fix-1 instead (they write grad_x, stage 1 reads the tile partials).
__global__ __launch_bounds__(256) void k_bwd_reduce1(prune_fb_desc d, const float2 *__restrict__ partial,
                                                     const uint32_t *__restrict__ s_begin,
                                                     const uint32_t *__restrict__ s_end,
                                                     double2 *__restrict__ part2, uint32_t eblocks,
                                                     uint32_t n_fix, const prune_fb_frame *__restrict__ fr,
                                                     const BwdFrame *__restrict__ bf,
                                                     const float2 *__restrict__ hg, float2 *__restrict__ gx) {
  __shared__ double2 red[kRedQ][64];
  if (blockIdx.x < n_fix) {
    bwd_fix_frame(d, fr, bf, hg, gx, blockIdx.x);
    return;
  }
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = max(Lmax, d.L[b]);
  const uint32_t E = d.n_banks * d.Kmax * Lmax;
  const uint32_t r = blockIdx.x - n_fix, c = r % kRedG, se = r / kRedG, s = se / eblocks, eb = se - s * eblocks;
  red_chunk_block(E, partial, s_begin[s], s_end[s], s, c, eb, part2, red);
}

__global__ __launch_bounds__(256) void k_bwd_reduce2(prune_fb_desc d, const double2 *__restrict__ part2,
                                                     float2 *__restrict__ gtaps) {
  __shared__ double2 red[kRedQ][64];
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = max(Lmax, d.L[b]);
  const uint32_t E = d.n_banks * d.Kmax * Lmax;
  red_stream_block(E, part2, blockIdx.x, kRedG, blockIdx.y, gtaps, red);   // stage 1 wrote every chunk
}

struct BwdLayout {
  size_t frames, items, partial, part2, hg, sbeg, send, cov, sfirst, cnt, total;
  // work items at most: in kBT tiles, and in the plain-product form's tiles
  // (the item list and the partial rows are sized for the larger count)
  uint32_t max_items, max_items_gemm, E, H;
};

static BwdLayout bwd_layout(const prune_fb_desc &d) {
  BwdLayout L{};
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = std::max(Lmax, d.L[b]);
  L.E = d.n_banks * d.Kmax * Lmax;
  L.H = Lmax - 1;
  auto count = [&](uint32_t tile) {
    const size_t per = ((size_t)d.max_frame_len + tile - 1) / tile;
    return (uint32_t)std::max<size_t>(1, (size_t)d.n_frames * std::max<size_t>(per, 1));
  };
  L.max_items = count(kBT);
  L.max_items_gemm = count(bwd_gemm_tile(d));
  const uint32_t rows = std::max(L.max_items, L.max_items_gemm);
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t o = 0;
  L.frames = o; o = al(o + (size_t)d.n_frames * sizeof(BwdFrame));
  L.items = o; o = al(o + (size_t)rows * sizeof(WorkItem));
  L.partial = o; o = al(o + (size_t)rows * L.E * sizeof(float2));
  L.part2 = o; o = al(o + (size_t)d.n_streams * kRedG * L.E * sizeof(double2));
  L.hg = o; o = al(o + (size_t)d.n_frames * std::max<uint32_t>(L.H, 1) * sizeof(float2));
  L.sbeg = o; o = al(o + (size_t)d.n_streams * sizeof(uint32_t));
  L.send = o; o = al(o + (size_t)d.n_streams * sizeof(uint32_t));
  L.cov = o; o = al(o + (size_t)d.n_streams * sizeof(unsigned long long));
  L.sfirst = o; o = al(o + (size_t)d.n_streams * sizeof(uint32_t));
  L.cnt = o; o = al(o + 16);
  L.total = o;
  return L;
}

static prune_status check_bwd_desc(const prune_fb_desc *d) {
  if (!d || d->n_streams == 0 || d->n_banks < 1 || d->n_banks > PRUNE_MAX_BANKS || d->Kmax < 1 ||
      d->Kmax > 10 || d->n_banks * d->Kmax > PRUNE_MAX_BRANCHES)
    return PRUNE_E_UNSUPPORTED;
  for (uint32_t b = 0; b < d->n_banks; ++b)
    if (d->L[b] < 1 || d->L[b] > PRUNE_MAX_L) return PRUNE_E_UNSUPPORTED;
  return PRUNE_OK;
}

// 1: vector Horner kernel, 2: matrix-core block-Toeplitz kernels, 3: one
// matrix-core kernel of plain products for both gradients
constexpr int kBwdVariants = 3;
static std::atomic<int> g_bwd_forced{0};
static std::mutex g_bwd_mu;
static std::map<std::string, int> g_bwd_tuned;
static int choose_bwd_variant(const prune_fb_desc *desc, const void *x, const void *taps,
                              const void *frames, const void *gy, void *gx, void *gtaps,
                              void *workspace, size_t workspace_bytes, prune_stream_t stream);
static prune_status fb_backward_variant(const prune_fb_desc *desc, const void *x, const void *taps,
                                        const void *frames, const void *gy, void *gx, void *gtaps,
                                        void *workspace, size_t workspace_bytes, int variant,
                                        prune_stream_t stream);

}  // namespace prune

using namespace prune;

extern "C" {

prune_status prune_fb_workspace_bytes(const prune_fb_desc *desc, size_t *bytes) {
  prune_status st = check_bwd_desc(desc);
  if (st != PRUNE_OK) return st;
  if (!bytes) return PRUNE_E_ARG;
  *bytes = bwd_layout(*desc).total;
  return PRUNE_OK;
}

prune_status prune_fb_backward(const prune_fb_desc *desc, const void *x, const void *taps,
                               const void *frames, const void *gy, void *gx, void *gtaps,
                               void *workspace, size_t workspace_bytes, prune_stream_t stream) {
  prune_status st = check_bwd_desc(desc);
  if (st != PRUNE_OK) return st;
  if (!x || !taps || !frames || !gy || (!gx && !gtaps) || !workspace) return PRUNE_E_ARG;
  const int v = choose_bwd_variant(desc, x, taps, frames, gy, gx, gtaps, workspace, workspace_bytes,
                                   stream);
  return fb_backward_variant(desc, x, taps, frames, gy, gx, gtaps, workspace, workspace_bytes, v,
                             stream);
}

prune_status prune_set_bwd_variant(int variant) {
  if (variant < 0 || variant > kBwdVariants) return PRUNE_E_ARG;
  g_bwd_forced.store(variant);
  return PRUNE_OK;
}

const char *prune_bwd_variant_name(int variant) {
  switch (variant) {
    case 1: return "valu_horner";
    case 2: return "mfma_toeplitz";
    case 3: return "mfma_gemm";
    default: return "auto";
  }
}

prune_status prune_autotune_bwd(uint32_t L, uint32_t K, uint32_t n, int *variant) {
  if (L < 1 || L > PRUNE_MAX_L || K < 1 || K > 10 || n < 1) return PRUNE_E_ARG;
  // a synthetic batch of the shape class: uniform frames of length n,
  // every branch active, about 16K samples per CU
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const uint32_t frames = std::max<uint32_t>(64, (uint32_t)((size_t)ncu * 16384 / n));
  const uint64_t N = (uint64_t)frames * n;
  prune_fb_desc d{};
  d.n_streams = 1; d.n_frames = frames; d.stream_len = N; d.n_banks = 1; d.Kmax = K;
  d.L[0] = L; d.max_frame_len = n;
  const size_t ws = bwd_layout(d).total;
  float2 *x = nullptr, *g = nullptr, *gx = nullptr, *t = nullptr, *gt = nullptr;
  prune_fb_frame *fr = nullptr;
  void *work = nullptr;
  bool ok = hipMalloc((void **)&x, N * sizeof(float2)) == hipSuccess &&
            hipMalloc((void **)&g, N * sizeof(float2)) == hipSuccess &&
            hipMalloc((void **)&gx, N * sizeof(float2)) == hipSuccess &&
            hipMalloc((void **)&t, (size_t)K * L * sizeof(float2)) == hipSuccess &&
            hipMalloc((void **)&gt, (size_t)K * L * sizeof(float2)) == hipSuccess &&
            hipMalloc((void **)&fr, frames * sizeof(prune_fb_frame)) == hipSuccess &&
            hipMalloc(&work, ws) == hipSuccess;
  if (ok) {
    std::vector<float2> hx(N);
    uint32_t st = 2468u;
    for (auto &v : hx) {
      st = st * 1664525u + 1013904223u;
      v.x = ((st >> 8) & 0xffff) / 65536.f - 0.5f;
      st = st * 1664525u + 1013904223u;
      v.y = ((st >> 8) & 0xffff) / 65536.f - 0.5f;
    }
    std::vector<float2> ht((size_t)K * L, make_float2(0.01f, -0.02f));
    std::vector<prune_fb_frame> hf(frames);
    for (uint32_t f = 0; f < frames; ++f) {
      hf[f] = prune_fb_frame{};
      hf[f].t0 = f * n; hf[f].n = n; hf[f].mask = (1u << K) - 1u;
    }
    ok = hipMemcpy(x, hx.data(), N * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(g, hx.data(), N * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(t, ht.data(), ht.size() * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(fr, hf.data(), frames * sizeof(prune_fb_frame), hipMemcpyHostToDevice) == hipSuccess;
  }
  const int v = ok ? choose_bwd_variant(&d, x, t, fr, g, gx, gt, work, ws, nullptr) : 1;
  if (x) (void)hipFree(x);
  if (g) (void)hipFree(g);
  if (gx) (void)hipFree(gx);
  if (t) (void)hipFree(t);
  if (gt) (void)hipFree(gt);
  if (fr) (void)hipFree(fr);
  if (work) (void)hipFree(work);
  if (!ok) return PRUNE_E_HIP;
  if (variant) *variant = v;
  return PRUNE_OK;
}

}  // extern "C"

namespace prune {

static prune_status fb_backward_variant(const prune_fb_desc *desc, const void *x, const void *taps,
                                        const void *frames, const void *gy, void *gx, void *gtaps,
                                        void *workspace, size_t workspace_bytes, int variant,
                                        prune_stream_t stream) {
  // either gradient may be skipped (a null output), not both
  if (!x || !taps || !frames || !gy || (!gx && !gtaps) || !workspace) return PRUNE_E_ARG;
  const BwdLayout L = bwd_layout(*desc);
  if (workspace_bytes < L.total) return PRUNE_E_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  char *w = (char *)workspace;
  BwdFrame *bf = (BwdFrame *)(w + L.frames);
  WorkItem *items = (WorkItem *)(w + L.items);
  float2 *partial = (float2 *)(w + L.partial);
  double2 *part2 = (double2 *)(w + L.part2);
  float2 *hg = (float2 *)(w + L.hg);
  uint32_t *sb = (uint32_t *)(w + L.sbeg), *se = (uint32_t *)(w + L.send);
  uint32_t *cnt = (uint32_t *)(w + L.cnt);
  unsigned long long *cov = (unsigned long long *)(w + L.cov);
  uint32_t *sfirst = (uint32_t *)(w + L.sfirst);
  const prune_fb_desc d = *desc;
  if (d.n_frames == 0) {
    if (gx && hipMemsetAsync(gx, 0, (size_t)d.n_streams * d.stream_len * sizeof(float2), s) != hipSuccess)
      return PRUNE_E_HIP;
    if (gtaps && hipMemsetAsync(gtaps, 0, (size_t)d.n_streams * L.E * sizeof(float2), s) != hipSuccess)
      return PRUNE_E_HIP;
    return PRUNE_OK;
  }
  // Without grad_x the vector form runs the block-Toeplitz grad_h kernel
  // (the vector kernel computes both gradients in one pass).
  const bool gemm = variant == 3;
  const bool mfma = !gemm && (variant == 2 || !gx);
  hipLaunchKernelGGL(k_bwd_prep, dim3(1), dim3(1024), 0, s, d, (const float2 *)x, (const float2 *)taps,
                     (const prune_fb_frame *)frames, (const float2 *)gy, (float2 *)gx, bf, items, cnt,
                     sb, se, cov, sfirst, gemm ? bwd_gemm_tile(d) : (uint32_t)kBT);
  // grad_x starts as zero outside the frames' coverage (the matrix-core
  // grad_x kernel zeroes those samples itself)
  if (gx && !mfma && !gemm)
    hipLaunchKernelGGL(k_bwd_gapfill, dim3(d.n_streams, 64), dim3(256), 0, s, d, cov, (float2 *)gx);
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const uint32_t grid = std::min<uint32_t>(L.max_items, (uint32_t)ncu * 2);
  if (gemm) {
    // one dynamic work ticket (cnt[1], cleared by k_bwd_prep)
    launch_bwd_gemm(d, bf, items, cnt, (unsigned int *)(cnt + 1), hg, gtaps ? partial : nullptr, L.max_items_gemm,
                    (uint32_t)ncu, sfirst, (float2 *)gx, s);
  } else if (mfma) {
    // dynamic work tickets (cnt[1], cnt[2], cleared by k_bwd_prep); grids of
    // 3 and 2 workgroups per CU, the fastest measured (at their register use
    // the kernels keep 2 and 1 workgroups resident per CU)
    if (gx)
      launch_bwd_gu_mfma(d, bf, items, cnt, (unsigned int *)(cnt + 1), hg,
                         std::min<uint32_t>(L.max_items + d.n_frames, (uint32_t)ncu * 3), sfirst,
                         (float2 *)gx, s);
    if (gtaps)
      launch_bwd_gh_mfma(d, bf, items, cnt, (unsigned int *)(cnt + 2), partial, L.max_items,
                         (uint32_t)ncu * 2, s);
  } else {
    hipLaunchKernelGGL(k_bwd_main, dim3(grid), dim3(kBWG), 0, s, d, bf, items, cnt, partial);
  }
  if (gx && L.H && !mfma && !gemm)   // the matrix-core grad_x kernels compute the halo rows themselves
    hipLaunchKernelGGL(k_bwd_halo, dim3(d.n_frames), dim3(64), 0, s, d, bf, hg);
  // the halo fix-up rides in front of the first reduction stage when both run
  const uint32_t n_fix = (gx && L.H) ? d.n_frames : 0u;
  if (!gtaps) {
    if (n_fix)
      hipLaunchKernelGGL(k_bwd_fix, dim3(d.n_frames), dim3(64), 0, s, d, (const prune_fb_frame *)frames,
                         bf, hg, (float2 *)gx);
    return hipGetLastError() == hipSuccess ? PRUNE_OK : PRUNE_E_HIP;
  }
  const uint32_t eblocks = (L.E + 63) / 64;
  hipLaunchKernelGGL(k_bwd_reduce1, dim3(n_fix + d.n_streams * eblocks * kRedG), dim3(256), 0, s, d, partial,
                     sb, se, part2, eblocks, n_fix, (const prune_fb_frame *)frames, bf, hg, (float2 *)gx);
  hipLaunchKernelGGL(k_bwd_reduce2, dim3(d.n_streams, eblocks), dim3(256), 0, s, d, part2,
                     (float2 *)gtaps);
  return hipGetLastError() == hipSuccess ? PRUNE_OK : PRUNE_E_HIP;
}

// Both backward forms timed on the call's own inputs (the gradients and
// workspace are rewritten by the call that follows): a warm-up of each,
// then five rounds launching each form once in turn, each launch timed by
// its own events; the smaller median wins.  Once per shape class (banks,
// Kmax, frame-length class, whether grad_x is wanted) and process, unless
// PRUNE_AUTOTUNE_CACHE already holds a choice for it on this architecture.
static int choose_bwd_variant(const prune_fb_desc *desc, const void *x, const void *taps,
                              const void *frames, const void *gy, void *gx, void *gtaps,
                              void *workspace, size_t workspace_bytes, prune_stream_t stream) {
  const int forced = g_bwd_forced.load();
  if (forced) return forced;
  const uint32_t n = desc->max_frame_len;
  const uint32_t nc = n >= 8192 ? 8192 : (n >= 2048 ? 2048 : 512);
  std::string key = "bwd|" + tune_arch() + "|L=";
  for (uint32_t b = 0; b < desc->n_banks; ++b) key += (b ? "," : "") + std::to_string(desc->L[b]);
  key += "|K=" + std::to_string(desc->Kmax) + "|n=" + std::to_string(nc) + "|gx=" + (gx ? "1" : "0");
  {
    std::lock_guard<std::mutex> lk(g_bwd_mu);
    auto it = g_bwd_tuned.find(key);
    if (it != g_bwd_tuned.end()) return it->second;
  }
  int best = 0;
  std::string name;
  if (tune_cache_lookup(key, &name))
    for (int v = 1; v <= kBwdVariants; ++v)
      if (name == prune_bwd_variant_name(v)) best = v;
  const char *env = getenv("PRUNE_AUTOTUNE");
  if (!best && env && env[0] == '0') return 1;
  if (!best) {
    constexpr int kRounds = 5;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t ev[2 * kRounds * kBwdVariants] = {};
    bool ok = true;
    for (auto &e : ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    float best_ms = 1e30f;
    if (ok) {
      for (int v = 1; v <= kBwdVariants; ++v)
        fb_backward_variant(desc, x, taps, frames, gy, gx, gtaps, workspace, workspace_bytes, v, stream);
      for (int r = 0; r < kRounds; ++r)
        for (int v = 1; v <= kBwdVariants; ++v) {
          hipEvent_t *e = &ev[2 * (r * kBwdVariants + v - 1)];
          (void)hipEventRecord(e[0], s);
          fb_backward_variant(desc, x, taps, frames, gy, gx, gtaps, workspace, workspace_bytes, v,
                              stream);
          (void)hipEventRecord(e[1], s);
        }
      if (hipStreamSynchronize(s) == hipSuccess)
        for (int v = 1; v <= kBwdVariants; ++v) {
          float t[kRounds];
          for (int r = 0; r < kRounds; ++r) {
            hipEvent_t *e = &ev[2 * (r * kBwdVariants + v - 1)];
            if (hipEventElapsedTime(&t[r], e[0], e[1]) != hipSuccess) t[r] = 1e30f;
          }
          std::sort(t, t + kRounds);
          if (t[kRounds / 2] < best_ms) {
            best_ms = t[kRounds / 2];
            best = v;
          }
        }
    }
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
    if (!best) return 1;
    tune_cache_store(key, prune_bwd_variant_name(best), best_ms);
  }
  std::lock_guard<std::mutex> lk(g_bwd_mu);
  g_bwd_tuned[key] = best;
  return best;
}

}  // namespace prune
