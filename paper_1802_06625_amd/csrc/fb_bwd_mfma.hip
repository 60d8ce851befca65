// Adjoint of the filter bank on the matrix cores (prune_fb_backward).
//
// With g = grad_y, u_b = r^{b-1} x, p = b-1 and r = |x| (1-based b):
//   grad_u_b[m] = sum_l conj(h_b[l]) g[m+l]           (outputs of the frame)
//   grad_x[m]   = sum_b (p/2+1) r^p grad_u_b[m] + (p/2) r^p (x^2/r^2) conj(grad_u_b[m])
//   grad_h_b[l] = sum_n g[n] conj(u_b[n-l])
// Both sums over l are contractions that take block form with blocks of 16
// samples:
//  * grad_u: for the input block at q, GU_b[i][q] = sum_{m < L+15} Hc_b[i][m]
//    G[m][q], with Hc_b[i][m] = conj(h_b[m-i]) (zero unless 0 <= m-i < L) and
//    the Hankel matrix G[m][q] = g[q+m].  As in the forward, a 16x16 result
//    tile covers 16 blocks and the contraction runs in steps of 4 on
//    v_mfma_f32_16x16x4_f32, three real products per complex one (Gauss).
//    G is shared by all branches: a pass over the steps serves four branches
//    (one g value per lane and step, and each branch's taps), which bounds
//    the accumulators at 48 registers for any branch count.
//  * grad_h: over the 64 blocks c of a tile, W_b[i][m] = sum_c g[16c+i]
//    conj(u_b[16c+m-(L-1)]) for i < 16, m < 16*ceil((L+15)/16); tap l
//    collects the diagonal m = i + L-1 - l:  grad_h_b[l] = sum_i W_b[i][i+L-1-l].
//    The contraction over c runs in steps of 4 blocks.  Each wave takes
//    (16-column slab of m, pair of branches) units, the pair sharing one
//    power of r per element; a branch's 16x16 W tile goes through
//    the wave's LDS scratch and its diagonals are summed in a fixed order,
//    then the (at most two) slabs of each tap are added in a fixed order: the tile's grad_h
//    partial is deterministic, and the per-stream float64 reduction of the
//    partials is shared with the vector kernel.
// Halo contributions (inputs before a frame that its outputs read) are
// added by the same halo/fix kernels as for the vector form.
#include "bwd_common.h"
#include "runtime_kernels.h"

namespace prune {

namespace {
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kNW = 4;                      // waves per workgroup
constexpr int kWG = 64 * kNW;
constexpr int kMKH = 10;                    // branches per bank
constexpr int kHQ = PRUNE_MAX_L + 36;       // conj-tap table entries per branch
constexpr int kHOff = 16;                   // table index of tap l = 0
constexpr int kGB = 4;                      // branches per grad_u pass

__device__ __forceinline__ int widx(int k) { return k + 4 * (k >> 4); }

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// r^e for 0 <= e < 16 by binary powering, without branches.
__device__ __forceinline__ float ipow(float r, int e) {
  float p = 1.f, q = r;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    p *= ((e >> k) & 1) ? q : 1.f;
    q *= q;
  }
  return p;
}

// W tiles of branches b0..b0+NB-1 for slab mt over the tile's 64 blocks.
//  gb: g-window index of A(row li, block lk); xb: x-window index of
//  B(block lk, column li of slab mt).
template <int NB>
__device__ __forceinline__ void gh_unit(const float2 *__restrict__ gw, const float4 *__restrict__ xw,
                                        int gb, int xb, int b0, floatx4 (&acc)[2][3]) {
#pragma unroll 2
  for (int s = 0; s < kBT / 64; ++s) {
    const float2 gv = gw[gb + 64 * s];
    const float4 xv = xw[xb + 64 * s];
    const float gs = gv.x + gv.y;
    float rp = ipow(xv.z, b0);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const float ur = xv.x * rp, ui = -(xv.y * rp);   // conj(u_b)
      acc[j][0] = mfma4(gv.x, ur, acc[j][0]);
      acc[j][1] = mfma4(gv.y, ui, acc[j][1]);
      acc[j][2] = mfma4(gs, ur + ui, acc[j][2]);
      rp *= xv.z;
    }
  }
}

// grad_u of branches b0..b0+NB-1 of one bank for this wave's 16x16 result
// tile: acc[j][0..2] hold the Gauss products of branch b0+j.  Inactive
// branches have zero taps in the table and add exact zeros: the products are
// issued unconditionally so the accumulators stay in the matrix registers.
// kb: window index of G(m = 0) for this lane; hb: table entry of
// Hc(row li, m = 0) of branch 0.
template <int NB>
__device__ __forceinline__ void gu_group(const float2 *__restrict__ gw, const float4 *__restrict__ hb,
                                         int b0, int S, int kb, floatx4 (&acc)[kGB][3]) {
  for (int s = 0; s < S; ++s) {
    const float2 gv = gw[widx(kb + 4 * s)];
    const float gs = gv.x + gv.y;
    float4 h[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) h[j] = hb[(b0 + j) * kHQ + 4 * s];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      acc[j][0] = mfma4(h[j].x, gv.x, acc[j][0]);
      acc[j][1] = mfma4(h[j].y, gv.y, acc[j][1]);
      acc[j][2] = mfma4(h[j].z, gs, acc[j][2]);
    }
  }
}
}  // namespace

// ------------------------------------------------------------------ grad_x
__global__ __launch_bounds__(kWG) void k_bwd_gu_mfma(prune_fb_desc d, const BwdFrame *__restrict__ bf,
                                                    const WorkItem *__restrict__ items,
                                                    const uint32_t *__restrict__ n_items) {
  // G window: index k holds g at tile position k; the last one read is
  // 256*3 + 16*15 + 3 + 4*(S-1) <= kBT + L + 1.
  constexpr int WN = kBT + PRUNE_MAX_L + 2;
  constexpr int WS = WN + 4 * (WN >> 4) + 4;
  __shared__ float2 s_g[WS];
  __shared__ float4 s_h[kMKH * kHQ];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = max(Lmax, d.L[b]);
  const uint32_t ni = *n_items;
  for (uint32_t it = blockIdx.x; it < ni; it += gridDim.x) {
    const WorkItem wi = items[it];
    const BwdFrame F = bf[wi.frame];
    const int n = (int)F.n, n0 = (int)wi.tile * kBT;
    if (F.route) {
      for (int k = t; k < kBT; k += kWG)
        if (n0 + k < n) F.gx[n0 + k] = F.g[n0 + k];
      continue;
    }
    for (int k = t; k < WN; k += kWG) {
      const int q = n0 + k;                  // outputs of this frame only
      s_g[widx(k)] = q < n ? F.g[q] : make_float2(0.f, 0.f);
    }
    // this lane's inputs: rows 4lk..4lk+3 of block li of the wave's tile
    const int m0 = n0 + 256 * w + 16 * li + 4 * lk;
    float xr[4], xi[4], rr[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float2 v = m0 + e < n ? F.x[m0 + e] : make_float2(0.f, 0.f);
      xr[e] = v.x;
      xi[e] = v.y;
      rr[e] = sqrtf(v.x * v.x + v.y * v.y);
    }
    float s1r[4] = {0.f, 0.f, 0.f, 0.f}, s1i[4] = {0.f, 0.f, 0.f, 0.f};
    float s2r[4] = {0.f, 0.f, 0.f, 0.f}, s2i[4] = {0.f, 0.f, 0.f, 0.f};
    const uint32_t kfull = (1u << d.Kmax) - 1u;
    for (uint32_t bank = 0; bank < d.n_banks; ++bank) {
      const uint32_t bmask = (F.mask >> (bank * d.Kmax)) & kfull;
      if (!bmask) continue;
      const int KH = 32 - __clz(bmask);
      const int L = (int)d.L[bank];
      const int S = (L + 15 + 3) / 4;
      __syncthreads();   // s_g written; earlier readers of s_h done
      const float2 *tb = F.taps + (size_t)bank * d.Kmax * Lmax;
      for (int k = t; k < KH * kHQ; k += kWG) {
        const int b = k / kHQ, l = k - b * kHQ - kHOff;
        float2 h = make_float2(0.f, 0.f);
        if (((bmask >> b) & 1u) && l >= 0 && l < L) h = tb[(size_t)b * Lmax + l];
        s_h[k] = make_float4(h.x, -h.y, h.x - h.y, 0.f);   // conj(h), Gauss sum
      }
      __syncthreads();
      // A(row li, m) = Hc[li][m] = conj(h[m - li]);  B(m, block li) = g[16 li + m]
      const int kb = 256 * w + 16 * li + lk;
      const float4 *hb = s_h + (lk - li + kHOff);
      float rp[4] = {1.f, 1.f, 1.f, 1.f};   // r^b of the group's next branch
      for (int b0 = 0; b0 < KH; b0 += kGB) {
        floatx4 acc[kGB][3];
#pragma unroll
        for (int j = 0; j < kGB; ++j) acc[j][0] = acc[j][1] = acc[j][2] = floatx4{0.f, 0.f, 0.f, 0.f};
        switch (min(kGB, KH - b0)) {   // branches b0.. below KH only
          case 1: gu_group<1>(s_g, hb, b0, S, kb, acc); break;
          case 2: gu_group<2>(s_g, hb, b0, S, kb, acc); break;
          case 3: gu_group<3>(s_g, hb, b0, S, kb, acc); break;
          default: gu_group<4>(s_g, hb, b0, S, kb, acc); break;
        }
        // S1 += (p/2+1) r^p GU_b ; S2 += (p/2) r^p conj(GU_b)
#pragma unroll
        for (int j = 0; j < kGB; ++j) {
          const int b = b0 + j;
          if (b < KH) {
            const bool act = (bmask >> b) & 1u;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              if (act) {
                const float gr = acc[j][0][e] - acc[j][1][e];
                const float gi = acc[j][2][e] - acc[j][0][e] - acc[j][1][e];
                const float al = (0.5f * (float)b + 1.f) * rp[e], be = 0.5f * (float)b * rp[e];
                s1r[e] = fmaf(al, gr, s1r[e]);
                s1i[e] = fmaf(al, gi, s1i[e]);
                s2r[e] = fmaf(be, gr, s2r[e]);
                s2i[e] = fmaf(-be, gi, s2i[e]);
              }
              rp[e] *= rr[e];
            }
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = m0 + e;
      if (m < n) {
        float gr = s1r[e], gi = s1i[e];
        const float r2 = xr[e] * xr[e] + xi[e] * xi[e];
        if (r2 > 0.f) {
          const float er = (xr[e] * xr[e] - xi[e] * xi[e]) / r2, ei = 2.f * xr[e] * xi[e] / r2;
          gr += er * s2r[e] - ei * s2i[e];
          gi += er * s2i[e] + ei * s2r[e];
        }
        F.gx[m] = make_float2(gr, gi);
      }
    }
    __syncthreads();   // s_g and s_h are rewritten by the next item
  }
}

// ------------------------------------------------------------------ grad_h
__global__ __launch_bounds__(kWG) void k_bwd_gh_mfma(prune_fb_desc d, const BwdFrame *__restrict__ bf,
                                                    const WorkItem *__restrict__ items,
                                                    const uint32_t *__restrict__ n_items,
                                                    float2 *__restrict__ partial) {
  // X window: index k holds x at tile position k - (Lmax-1); the last one
  // read is 16*63 + 16*MT - 1 + (Lmax - L) <= kBT + Lmax + 14.
  constexpr int WX = kBT + PRUNE_MAX_L + 16;
  __shared__ float2 s_g[kBT];
  __shared__ float4 s_x[WX];
  __shared__ float2 s_w[kNW][16][17];
  // Slab partials of each tap: tap l collects diagonals of at most two
  // adjacent slabs (mt with 16 mt in [L-1-l-15, L-1-l+15]), which differ in
  // parity, so they are kept by slab parity and added in parity order.
  __shared__ float2 s_pd[kMKH][2][PRUNE_MAX_L];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
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
      for (uint32_t k = t; k < D * Lmax; k += kWG) prow[k] = make_float2(0.f, 0.f);
      continue;
    }
    for (int k = t; k < kBT; k += kWG) s_g[k] = n0 + k < n ? F.g[n0 + k] : make_float2(0.f, 0.f);
    for (int k = t; k < WX; k += kWG) {
      const int p = n0 - ((int)Lmax - 1) + k;
      float2 v = make_float2(0.f, 0.f);
      if (p < n && p >= -(int)F.t0) v = F.x[p];
      s_x[k] = make_float4(v.x, v.y, sqrtf(v.x * v.x + v.y * v.y), 0.f);
    }
    const uint32_t kfull = (1u << d.Kmax) - 1u;
    for (uint32_t bank = 0; bank < d.n_banks; ++bank) {
      const uint32_t bmask = (F.mask >> (bank * d.Kmax)) & kfull;
      float2 *brow = prow + (size_t)bank * d.Kmax * Lmax;
      if (!bmask) {
        for (uint32_t k = t; k < d.Kmax * Lmax; k += kWG) brow[k] = make_float2(0.f, 0.f);
        continue;
      }
      const int KH = 32 - __clz(bmask);
      const int L = (int)d.L[bank];
      const int MT = (L + 15 + 15) / 16;
      for (int k = t; k < kMKH * 2 * PRUNE_MAX_L; k += kWG) (&s_pd[0][0][0])[k] = make_float2(0.f, 0.f);
      __syncthreads();   // windows written, s_pd cleared
      // units: (slab mt, branches 2q and 2q+1)
      const int NQ = (KH + 1) / 2;
      const int units = NQ * MT;
      for (int u = w; u < units; u += kNW) {
        const int q = u / MT, mt = u - q * MT;
        const int b0 = 2 * q, nb = min(2, KH - b0);
        const uint32_t um = (bmask >> b0) & ((1u << nb) - 1u);
        if (!um) continue;
        floatx4 acc[2][3];
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[j][0] = acc[j][1] = acc[j][2] = floatx4{0.f, 0.f, 0.f, 0.f};
        // A(row li, block 4s+lk) = g[16(4s+lk) + li];
        // B(block 4s+lk, column li of slab mt) = conj u_b at x-window index
        //   16(4s+lk) + 16 mt + li + (Lmax - L)
        const int xb = 16 * lk + 16 * mt + li + ((int)Lmax - L);
        const int gb = 16 * lk + li;
        if (nb == 2) gh_unit<2>(s_g, s_x, gb, xb, b0, acc);
        else gh_unit<1>(s_g, s_x, gb, xb, b0, acc);
        for (int j = 0; j < nb; ++j) {
          const int b = b0 + j;
          if (!((bmask >> b) & 1u)) continue;
          // W tile (rows 4lk+e, column li) to the wave's scratch
#pragma unroll
          for (int e = 0; e < 4; ++e)
            s_w[w][4 * lk + e][li] =
                make_float2(acc[j][0][e] - acc[j][1][e], acc[j][2][e] - acc[j][0][e] - acc[j][1][e]);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          // lane 0..30: diagonal j - i = lane - 15, tap l = L-1 - 16 mt - (j - i)
          if (lane < 31) {
            const int dl = lane - 15;
            const int l = L - 1 - 16 * mt - dl;
            if (l >= 0 && l < L) {
              float sr = 0.f, si = 0.f;
              for (int i = max(0, -dl); i < min(16, 16 - dl); ++i) {
                const float2 v = s_w[w][i][i + dl];
                sr += v.x;
                si += v.y;
              }
              s_pd[b][mt & 1][l] = make_float2(sr, si);
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
      __syncthreads();
      for (uint32_t k = t; k < d.Kmax * Lmax; k += kWG) {
        const int b = (int)(k / Lmax), l = (int)(k - b * Lmax);
        float2 v = make_float2(0.f, 0.f);
        if (b < KH && ((bmask >> b) & 1u) && l < L) {
          v.x = s_pd[b][0][l].x + s_pd[b][1][l].x;
          v.y = s_pd[b][0][l].y + s_pd[b][1][l].y;
        }
        brow[k] = v;
      }
      __syncthreads();   // s_pd is cleared for the next bank
    }
    __syncthreads();     // windows are rewritten by the next item
  }
}

void launch_bwd_gu_mfma(const prune_fb_desc &d, const BwdFrame *bf, const WorkItem *items,
                        const uint32_t *n_items, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_bwd_gu_mfma, dim3(grid), dim3(kWG), 0, s, d, bf, items, n_items);
}

void launch_bwd_gh_mfma(const prune_fb_desc &d, const BwdFrame *bf, const WorkItem *items,
                        const uint32_t *n_items, float2 *partial, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_bwd_gh_mfma, dim3(grid), dim3(kWG), 0, s, d, bf, items, n_items, partial);
}

}  // namespace prune
