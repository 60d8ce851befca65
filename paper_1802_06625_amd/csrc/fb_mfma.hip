// Filter-bank forward on the matrix cores: the block-Toeplitz form of the
// fused basis + FIR + branch-sum firing (Sec. VII-A), for wide filters.
//
// Outputs of a tile are grouped in blocks of P = 16 consecutive samples.  For
// a bank with L taps and an output block starting at q:
//   y[q + i] = sum_b sum_{m < L+15} H_b[i][m] U_b[m][q],       i = 0..15
//   H_b[i][m] = h_b[i + L-1 - m]   (zero unless 0 <= i+L-1-m < L)   Toeplitz
//   U_b[m][q] = u_b[q + m - (L-1)],  u_b = |x|^{b-1} x              Hankel
// Sixteen output blocks form one 16x16 result tile of H_b (16 x (L+15)) times
// U_b ((L+15) x 16), summed over the active branches; the contraction over m
// runs on v_mfma_f32_16x16x4_f32 in steps of 4.  The complex products use
// three real products (Gauss): T1 = Hr Ur, T2 = Hi Ui, T3 = (Hr+Hi)(Ur+Ui),
// Re y = T1 - T2, Im y = T3 - T1 - T2.  Per output and active branch this is
// 24 (L+15)/4 real multiply-adds, against 4 L for the direct form.
//
// Operand layout of the 16x16x4 fp32 instruction for lane l (li = l mod 16,
// lk = l / 16): A[i = li][k = lk], B[k = lk][j = li], and element e of the
// result is D[4 lk + e][li].  A lane therefore holds output rows 4lk..4lk+3
// of block li: four consecutive samples.
//
// A tile is NW waves x NT result tiles x 256 outputs.  LDS holds the tile's
// input window as three fp32 planes (re, im, r = |x|) with one pad float per
// 16 (the 16 lanes of a B fragment read 16 samples apart; an odd stride of
// 17 puts them in distinct banks), and each active branch's taps as
// {hr, hi, hr + hi, 0} with zeros on both sides, so every Toeplitz element is
// one table read.  u_b is formed in registers from the window by repeated
// multiplication with r.  Workgroups take tiles from the item list with an
// atomic ticket, as the vector kernels do.
#include <hip/hip_ext.h>

#include "prune_internal.h"
#include "runtime_kernels.h"

namespace prune {

namespace {
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kHOff = 20;                  // table index of tap l = 0
constexpr int kHQ = PRUNE_MAX_L + 36;      // table entries per branch: l = -20 .. L+15
constexpr int kMKH = 10;                   // branches per bank

__device__ __forceinline__ int widx(int k) { return k + (k >> 4); }

// One bank: S steps of 4 along m for the NT result tiles of this wave.
//  kb: window index of B element (m = 0, tile 0) for this lane;
//  hb: table entry of A element (m = 0, branch 0) for this lane.
template <int KH, int NT>
__device__ __forceinline__ void mfma_bank(const float *__restrict__ wr, const float *__restrict__ wi,
                                          const float *__restrict__ wm, const float4 *__restrict__ hb,
                                          int S, int kb, floatx4 *a1, floatx4 *a2,
                                          floatx4 *a3) {
  for (int s = 0; s < S; ++s) {
    float ur[NT], ui[NT], rr[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int q = widx(kb + 256 * j + 4 * s);
      ur[j] = wr[q];
      ui[j] = wi[q];
      rr[j] = wm[q];
    }
    float4 h[KH];
#pragma unroll
    for (int b = 0; b < KH; ++b) h[b] = hb[b * kHQ - 4 * s];
    // Every branch below KH is issued: an inactive branch has zero taps in
    // the table and adds exact zeros.  (A mask test here would split the
    // products into separate blocks and move the accumulators out of the
    // matrix registers around every instruction.)
#pragma unroll
    for (int b = 0; b < KH; ++b) {
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const float us = ur[j] + ui[j];
        a1[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(h[b].x, ur[j], a1[j], 0, 0, 0);
        a2[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(h[b].y, ui[j], a2[j], 0, 0, 0);
        a3[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(h[b].z, us, a3[j], 0, 0, 0);
      }
      if (b + 1 < KH) {
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          ur[j] *= rr[j];
          ui[j] *= rr[j];
        }
      }
    }
  }
}

template <int NT>
__device__ __forceinline__ void mfma_dispatch(int KH, const float *wr, const float *wi,
                                              const float *wm, const float4 *hb, int S, int kb, floatx4 *a1, floatx4 *a2,
                                              floatx4 *a3) {
  switch (KH) {
    case 1: mfma_bank<1, NT>(wr, wi, wm, hb, S, kb, a1, a2, a3); break;
    case 2: mfma_bank<2, NT>(wr, wi, wm, hb, S, kb, a1, a2, a3); break;
    case 3: mfma_bank<3, NT>(wr, wi, wm, hb, S, kb, a1, a2, a3); break;
    case 4: mfma_bank<4, NT>(wr, wi, wm, hb, S, kb, a1, a2, a3); break;
    case 5: mfma_bank<5, NT>(wr, wi, wm, hb, S, kb, a1, a2, a3); break;
    case 6: mfma_bank<6, NT>(wr, wi, wm, hb, S, kb, a1, a2, a3); break;
    case 7: mfma_bank<7, NT>(wr, wi, wm, hb, S, kb, a1, a2, a3); break;
    case 8: mfma_bank<8, NT>(wr, wi, wm, hb, S, kb, a1, a2, a3); break;
    case 9: mfma_bank<9, NT>(wr, wi, wm, hb, S, kb, a1, a2, a3); break;
    default: mfma_bank<10, NT>(wr, wi, wm, hb, S, kb, a1, a2, a3); break;
  }
}
}  // namespace

// *ticket must be zero at launch (the producer of the item list clears it).
template <int NT, int NW>
__global__ __launch_bounds__(64 * NW) void k_fb_mfma(const FbFrameDesc *__restrict__ frames,
                                                    const WorkItem *__restrict__ items,
                                                    const uint32_t *__restrict__ n_items_ptr,
                                                    unsigned int *__restrict__ ticket) {
  constexpr int WG = 64 * NW;
  constexpr int TW = 256 * NT;               // outputs per wave
  constexpr int T = TW * NW;                 // outputs per tile
  // Window positions: the last B element read is at T + Lmax + 1 (m runs to
  // 4 ceil((L+15)/4) - 1 <= L + 17), so T + PRUNE_MAX_L + 2 covers it.
  constexpr int WN = T + PRUNE_MAX_L + 2;
  constexpr int WS = WN + (WN >> 4) + 1;
  __shared__ float s_wr[WS], s_wi[WS], s_wm[WS];
  __shared__ float4 s_h[kMKH * kHQ];
  __shared__ uint32_t s_item;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const uint32_t n_items = *n_items_ptr;
  // the tap table in LDS is kept while consecutive tiles share it
  const float2 *tab_taps = nullptr;
  uint32_t tab_key = 0xffffffffu;

  bool first = true;   // first tile by workgroup index, later ones by ticket
  for (;;) {
    // (no ticket when the grid covers the list: every tile is some
    // workgroup's first)
    if (t == 0) s_item = first ? blockIdx.x : gridDim.x >= n_items ? n_items : gridDim.x + atomicAdd(ticket, 1u);
    first = false;
    __syncthreads();
    const uint32_t it = s_item;
    if (it >= n_items) break;
    const WorkItem wi = items[it];
    const FbFrameDesc &d = frames[wi.frame];
    const int n = (int)d.n;
    const int n0 = (int)wi.tile * T;

    if (d.route) {
      for (int k = t; k < T; k += WG) {
        const int p = n0 + k;
        if (p < n) {
          const float2 v = d.x[p];
          for (uint32_t o = 0; o < d.n_y; ++o) d.y[o][p] = v;
        }
      }
      __syncthreads();
      continue;
    }

    // Window index k holds stream position n0 - (Lw-1) + k.
    const int Lw = (int)d.Lmax;
    {
      // all of this thread's loads first, then the stores (one memory latency)
      constexpr int NIT = (WN + WG - 1) / WG;
      float2 v[NIT];
#pragma unroll
      for (int i = 0; i < NIT; ++i) {
        const int k = t + i * WG, p = n0 - (Lw - 1) + k;
        v[i] = make_float2(0.f, 0.f);
        if (k < WN) {
          if (p >= 0) {
            if (p < n) v[i] = d.x[p];
          } else if (-p <= (int)d.halo_valid) {
            v[i] = d.halo[Lw - 1 + p];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < NIT; ++i) {
        const int k = t + i * WG;
        if (k < WN) {
          const int q = widx(k);
          s_wr[q] = v[i].x;
          s_wi[q] = v[i].y;
          s_wm[q] = sqrtf(v[i].x * v[i].x + v[i].y * v[i].y);
        }
      }
    }

    floatx4 a1[NT], a2[NT], a3[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) a1[j] = a2[j] = a3[j] = floatx4{0.f, 0.f, 0.f, 0.f};

    const uint32_t kfull = d.Kmax >= 32 ? 0xffffffffu : ((1u << d.Kmax) - 1u);
    for (uint32_t bank = 0; bank < d.n_banks; ++bank) {
      const uint32_t bmask = (d.mask >> (bank * d.Kmax)) & kfull;
      if (!bmask) continue;
      const int KH = 32 - __clz(bmask);
      const int L = (int)d.L[bank];
      const int S = (L + 15 + 3) / 4;
      const float2 *tb = d.taps + (size_t)bank * d.Kmax * d.Lmax;
      const uint32_t key = bmask | ((uint32_t)L << 16) | (bank << 24);
      if (tb != tab_taps || key != tab_key) {   // uniform across the workgroup
        __syncthreads();   // earlier readers of s_h are done
        tab_taps = tb;
        tab_key = key;
        for (int k = t; k < KH * kHQ; k += WG) {
          const int b = k / kHQ, l = k - b * kHQ - kHOff;
          float2 h = make_float2(0.f, 0.f);
          if (((bmask >> b) & 1u) && l >= 0 && l < L) h = tb[(size_t)b * d.Lmax + l];
          s_h[k] = make_float4(h.x, h.y, h.x + h.y, 0.f);
        }
      }
      __syncthreads();
      // B(m, block li) of result tile j reads window index
      //   w TW + 256 j + 16 li + m + (Lw - L),  m = 4 s + lk;
      // A(row li, m) reads tap l = li + L-1 - m.
      const int kb = w * TW + 16 * li + lk + (Lw - L);
      const float4 *hb = s_h + (li + L - 1 - lk + kHOff);
      mfma_dispatch<NT>(KH, s_wr, s_wi, s_wm, hb, S, kb, a1, a2, a3);
    }

#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int p0 = n0 + w * TW + 256 * j + 16 * li + 4 * lk;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int p = p0 + e;
        if (p < n) {
          const float2 v = make_float2(a1[j][e] - a2[j][e], a3[j][e] - a1[j][e] - a2[j][e]);
          for (uint32_t o = 0; o < d.n_y; ++o) d.y[o][p] = v;
        }
      }
    }
    __syncthreads();
  }
}

template <int NT, int NW>
void launch_fb_mfma(const FbFrameDesc *f, const WorkItem *it, const uint32_t *n,
                    unsigned int *ticket, uint32_t grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (e0 || e1)
    hipExtLaunchKernelGGL((k_fb_mfma<NT, NW>), dim3(grid), dim3(64 * NW), 0, s, e0, e1, 0, f, it, n, ticket);
  else
    hipLaunchKernelGGL((k_fb_mfma<NT, NW>), dim3(grid), dim3(64 * NW), 0, s, f, it, n, ticket);
}

template <int NT, int NW>
int fb_mfma_resident() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_fb_mfma<NT, NW>),
                                                   64 * NW, 0) != hipSuccess)
    n = 0;
  return n;
}
template int fb_mfma_resident<4, 4>();
template int fb_mfma_resident<2, 4>();
template int fb_mfma_resident<4, 2>();

template void launch_fb_mfma<4, 4>(const FbFrameDesc *, const WorkItem *, const uint32_t *,
                                   unsigned int *, uint32_t, hipStream_t, hipEvent_t,
                                   hipEvent_t);
template void launch_fb_mfma<2, 4>(const FbFrameDesc *, const WorkItem *, const uint32_t *,
                                   unsigned int *, uint32_t, hipStream_t, hipEvent_t,
                                   hipEvent_t);
template void launch_fb_mfma<4, 2>(const FbFrameDesc *, const WorkItem *, const uint32_t *,
                                   unsigned int *, uint32_t, hipStream_t, hipEvent_t,
                                   hipEvent_t);

}  // namespace prune
