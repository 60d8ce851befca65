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
// added by the same fix-up kernel as for the vector form, and the tile
// partials of grad_h by the same reduction kernels.  The grad_x kernel
// zeroes the samples outside every frame after its items (no separate gap
// kernel).
#include <algorithm>

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

__device__ __forceinline__ int widx(int k) { return k + (k >> 4); }

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
// Tickets 0 .. n_items-1 are the tiles; tickets n_items .. n_items+n_frames-1
// are halo items: the gradient of the H = Lmax-1 stream samples before frame
// f from f's own outputs (positions -64 .. -1 of a tile at -64, computed by
// wave 0), written to hg[f][0 .. H) for the fix-up kernel.
__global__ __launch_bounds__(kWG) void k_bwd_gu_mfma(prune_fb_desc d, const BwdFrame *__restrict__ bf,
                                                    const WorkItem *__restrict__ items,
                                                    const uint32_t *__restrict__ n_items,
                                                    unsigned int *__restrict__ ticket,
                                                    float2 *__restrict__ hg,
                                                    const uint32_t *__restrict__ sfirst,
                                                    float2 *__restrict__ gxs) {
  // G window: index k holds g at tile position k; the last one read is
  // 256*3 + 16*15 + 3 + 4*(S-1) <= kBT + L + 1.
  constexpr int WN = kBT + PRUNE_MAX_L + 2;
  constexpr int WS = WN + (WN >> 4) + 1;
  __shared__ float2 s_g[WS];
  __shared__ float4 s_h[kMKH * kHQ];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = max(Lmax, d.L[b]);
  __shared__ uint32_t s_item;
  const uint32_t ni = *n_items;
  const int H = (int)Lmax - 1;
  // the conjugate-tap table in LDS is kept while consecutive items share it
  const float2 *tab_taps = nullptr;
  uint32_t tab_key = 0xffffffffu;
  const uint32_t nh = H > 0 ? d.n_frames : 0u;
  bool first = true;   // first item by workgroup index, later ones by ticket
  for (;;) {
    // (no ticket when the grid covers the list: every item is some
    // workgroup's first)
    if (t == 0) s_item = first ? blockIdx.x : gridDim.x >= ni + nh ? ni + nh : gridDim.x + atomicAdd(ticket, 1u);
    first = false;
    __syncthreads();
    const uint32_t it = s_item;
    __syncthreads();   // s_item is rewritten by the next ticket
    if (it >= ni + nh) break;
    const bool halo = it >= ni;
    const uint32_t frame = halo ? it - ni : items[it].frame;
    const BwdFrame F = bf[frame];
    const int n = (int)F.n, n0 = halo ? -64 : (int)items[it].tile * kBT;
    if (halo && (F.route || n == 0)) continue;   // the fix-up skips these frames
    if (F.route) {
      for (int k = t; k < kBT; k += kWG)
        if (n0 + k < n) st_global(F.gx + n0 + k, ld_global(F.g + n0 + k));
      continue;
    }
    const bool work = !halo || w == 0;   // a halo item needs wave 0's block only
    {
      // all of this thread's loads first, then the stores (one memory latency)
      constexpr int NIT = (WN + kWG - 1) / kWG;
      float2 v[NIT];
#pragma unroll
      for (int i = 0; i < NIT; ++i) {
        const int k = t + i * kWG, q = n0 + k;   // outputs of this frame only
        v[i] = (k < WN && q >= 0 && q < n) ? ld_global(F.g + q) : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int i = 0; i < NIT; ++i) {
        const int k = t + i * kWG;
        if (k < WN) s_g[widx(k)] = v[i];
      }
    }
    // this lane's inputs: rows 4lk..4lk+3 of block li of the wave's tile
    const int m0 = n0 + 256 * w + 16 * li + 4 * lk;
    float xr[4], xi[4], rr[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = m0 + e;   // stream history before the frame: m >= -t0
      const float2 v = (m < n && m >= -(int)F.t0) ? ld_global(F.x + m) : make_float2(0.f, 0.f);
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
      const float2 *tb = F.taps + (size_t)bank * d.Kmax * Lmax;
      const uint32_t key = bmask | ((uint32_t)L << 16) | (bank << 24);
      __syncthreads();   // s_g written; earlier readers of s_h done
      if (tb != tab_taps || key != tab_key) {   // uniform across the workgroup
        tab_taps = tb;
        tab_key = key;
        constexpr int NIT = (kMKH * kHQ + kWG - 1) / kWG;
        float2 hv[NIT];
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
          const int k = t + i * kWG;
          const int b = k / kHQ, l = k - b * kHQ - kHOff;
          hv[i] = (k < KH * kHQ && ((bmask >> b) & 1u) && l >= 0 && l < L) ? ld_global(tb + (size_t)b * Lmax + l)
                                                                            : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
          const int k = t + i * kWG;
          if (k < KH * kHQ) s_h[k] = make_float4(hv[i].x, -hv[i].y, hv[i].x - hv[i].y, 0.f);  // conj(h)
        }
      }
      __syncthreads();
      // A(row li, m) = Hc[li][m] = conj(h[m - li]);  B(m, block li) = g[16 li + m]
      const int kb = 256 * w + 16 * li + lk;
      const float4 *hb = s_h + (lk - li + kHOff);
      float rp[4] = {1.f, 1.f, 1.f, 1.f};   // r^b of the group's next branch
      for (int b0 = 0; work && b0 < KH; b0 += kGB) {
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
      if (halo ? (w == 0 && m >= -H && m < 0) : m < n) {
        float gr = s1r[e], gi = s1i[e];
        const float r2 = xr[e] * xr[e] + xi[e] * xi[e];
        if (r2 > 0.f) {
          const float er = (xr[e] * xr[e] - xi[e] * xi[e]) / r2, ei = 2.f * xr[e] * xi[e] / r2;
          gr += er * s2r[e] - ei * s2i[e];
          gi += er * s2i[e] + ei * s2r[e];
        }
        if (halo) hg[(size_t)frame * H + (m + H)] = make_float2(gr, gi);
        else st_global(F.gx + m, make_float2(gr, gi));
      }
    }
    __syncthreads();   // s_g and s_h are rewritten by the next item
  }
  if (sfirst) bwd_zero_gaps(d, bf, sfirst, gxs);
}

// ------------------------------------------------------------------ grad_h
namespace {
constexpr int kGH = 4;                       // branches per staged group
constexpr int kUMax = 5;                     // units per wave: 5 slabs x 4 branches / 4 waves
constexpr int kWX = kBT + PRUNE_MAX_L + 16;  // basis-plane positions per tile
constexpr int kMaxRun = 8;                   // tiles accumulated before the diagonal sums

// The contributions of one tile to NU units of this wave: 16 steps of 4
// blocks.  The A operand (cotangent) is the same for every unit, so each
// step loads it once and issues 3 NU independent products.
//  gb: g-plane index of A(row li, block lk); ub[k]: u-plane offset (plane
//  and column) of B(block lk, column li of unit k's slab).
template <int NU>
__device__ __forceinline__ void gh_tile(const float4 *__restrict__ gp, const float2 *__restrict__ up,
                                        int gb, const int *ub, floatx4 (*acc)[3]) {
#pragma unroll
  for (int s = 0; s < kBT / 64; ++s) {
    const float4 gv = gp[gb + 64 * s];
    float2 uv[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) uv[k] = up[ub[k] + 64 * s];
#pragma unroll
    for (int k = 0; k < NU; ++k) {
      acc[k][0] = mfma4(gv.x, uv[k].x, acc[k][0]);
      acc[k][1] = mfma4(gv.y, uv[k].y, acc[k][1]);
      acc[k][2] = mfma4(gv.z, uv[k].x + uv[k].y, acc[k][2]);
    }
  }
}
}  // namespace

// grad_h partials.  Work: runs of up to `run` consecutive tiles of one frame
// (item groups [g*run, g*run+run) split where the frame changes).  A run's
// W tiles are accumulated over all its tiles, then reduced once; the sum is
// the partial row of the run's first item and the other items' rows are
// zero.  Per tile and group of up to four branches, LDS holds the cotangent
// as {gr, gi, gr+gi} and the planes conj(u_b) = {ur, -ui} of the group's
// branches over the tile's window.
__global__ __launch_bounds__(kWG) void k_bwd_gh_mfma(prune_fb_desc d, const BwdFrame *__restrict__ bf,
                                                    const WorkItem *__restrict__ items,
                                                    const uint32_t *__restrict__ n_items,
                                                    unsigned int *__restrict__ ticket,
                                                    float2 *__restrict__ partial, uint32_t run) {
  __shared__ float4 s_g[kBT];
  // basis planes; after a run's tiles the same memory is the waves' W scratch
  __shared__ float2 s_u[kGH][kWX];
  __shared__ float2 s_pd[kMKH][2][PRUNE_MAX_L];
  float2 (*s_w)[16][17] = reinterpret_cast<float2 (*)[16][17]>(&s_u[0][0]);
  static_assert(kNW * 16 * 17 <= kGH * kWX, "W scratch fits in the basis planes");
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = max(Lmax, d.L[b]);
  const uint32_t D = d.n_banks * d.Kmax;
  const uint32_t ni = *n_items;
  const uint32_t R = min(max(run, 1u), (uint32_t)kMaxRun);
  const uint32_t ng = (ni + R - 1) / R;
  const uint32_t kfull = (1u << d.Kmax) - 1u;
  __shared__ uint32_t s_grp;
  bool first = true;   // first run group by workgroup index, later ones by ticket
  for (;;) {
    if (t == 0) s_grp = first ? blockIdx.x : gridDim.x >= ng ? ng : gridDim.x + atomicAdd(ticket, 1u);
    first = false;
    __syncthreads();
    const uint32_t grp = s_grp;
    __syncthreads();   // s_grp is rewritten by the next ticket
    if (grp >= ng) break;
    const uint32_t i1 = min(ni, (grp + 1) * R);
    for (uint32_t r0 = grp * R; r0 < i1;) {
      const WorkItem w0 = items[r0];
      uint32_t r1 = r0 + 1;
      while (r1 < i1 && items[r1].frame == w0.frame) ++r1;
      const BwdFrame F = bf[w0.frame];
      const int n = (int)F.n;
      // rows of the run's later items are zero
      for (uint32_t k = t; k < (r1 - r0 - 1) * D * Lmax; k += kWG)
        partial[(size_t)(r0 + 1) * D * Lmax + k] = make_float2(0.f, 0.f);
      float2 *prow = partial + (size_t)r0 * D * Lmax;
      if (F.route) {
        for (uint32_t k = t; k < D * Lmax; k += kWG) prow[k] = make_float2(0.f, 0.f);
        r0 = r1;
        continue;
      }
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
        __syncthreads();   // earlier readers of s_pd are done
        for (int k = t; k < kMKH * 2 * PRUNE_MAX_L; k += kWG) (&s_pd[0][0][0])[k] = make_float2(0.f, 0.f);
        // This thread's share of a tile's cotangent and inputs, loaded into
        // registers one tile ahead: the loads of the next tile are in flight
        // while the current one is on the matrix cores.
        constexpr int NG = kBT / kWG, NX = (kWX + kWG - 1) / kWG;
        float2 gv[NG], xv[NX];
        auto load_tile = [&](uint32_t itx) {
          const int n0 = (int)items[itx].tile * kBT;
#pragma unroll
          for (int i = 0; i < NG; ++i) {
            const int k = t + i * kWG;
            gv[i] = n0 + k < n ? ld_global(F.g + n0 + k) : make_float2(0.f, 0.f);
          }
          // u-plane index k holds position n0 - (Lmax-1) + k
#pragma unroll
          for (int i = 0; i < NX; ++i) {
            const int k = t + i * kWG, p = n0 - ((int)Lmax - 1) + k;
            xv[i] = (k < kWX && p < n && p >= -(int)F.t0) ? ld_global(F.x + p) : make_float2(0.f, 0.f);
          }
        };
        load_tile(r0);
        for (int b0 = 0; b0 < KH; b0 += kGH) {
          const int nb = min(kGH, KH - b0);
          const int units = MT * nb;   // unit u: slab u / nb, branch b0 + u % nb
          floatx4 acc[kUMax][3];
#pragma unroll
          for (int k = 0; k < kUMax; ++k) acc[k][0] = acc[k][1] = acc[k][2] = floatx4{0.f, 0.f, 0.f, 0.f};
          for (uint32_t it = r0; it < r1; ++it) {
            __syncthreads();   // earlier readers of s_g / s_u are done
            {
#pragma unroll
              for (int i = 0; i < NG; ++i)
                s_g[t + i * kWG] = make_float4(gv[i].x, gv[i].y, gv[i].x + gv[i].y, 0.f);
#pragma unroll
              for (int i = 0; i < NX; ++i) {
                const int k = t + i * kWG;
                if (k < kWX) {
                  const float r = sqrtf(xv[i].x * xv[i].x + xv[i].y * xv[i].y);
                  float rp = ipow(r, b0);
#pragma unroll
                  for (int j = 0; j < kGH; ++j) {
                    if (j < nb) s_u[j][k] = make_float2(xv[i].x * rp, -(xv[i].y * rp));
                    rp *= r;
                  }
                }
              }
            }
            // the next tile of this bank: the run's next one, else the run's
            // first one for the next branch group
            if (it + 1 < r1) load_tile(it + 1);
            else if (b0 + kGH < KH) load_tile(r0);
            __syncthreads();
            // this wave's units u = w + kNW k (slab u / nb, branch b0 + u % nb),
            // all at once; an inactive branch's unit is computed and discarded
            {
              int ub[kUMax];
#pragma unroll
              for (int k = 0; k < kUMax; ++k) {
                const int u = w + kNW * k;
                const int mt = u / nb, j = u - mt * nb;
                ub[k] = u < units ? j * kWX + 16 * lk + 16 * mt + li + ((int)Lmax - L) : 0;
              }
              const int nu = units > w ? (units - w + kNW - 1) / kNW : 0;
              const int gb = 16 * lk + li;
              switch (nu) {
                case 1: gh_tile<1>(s_g, &s_u[0][0], gb, ub, acc); break;
                case 2: gh_tile<2>(s_g, &s_u[0][0], gb, ub, acc); break;
                case 3: gh_tile<3>(s_g, &s_u[0][0], gb, ub, acc); break;
                case 4: gh_tile<4>(s_g, &s_u[0][0], gb, ub, acc); break;
                case 5: gh_tile<5>(s_g, &s_u[0][0], gb, ub, acc); break;
                default: break;
              }
            }
          }
          __syncthreads();   // the basis planes become the W scratch
#pragma unroll
          for (int k = 0; k < kUMax; ++k) {
            const int u = w + kNW * k;
            if (u >= units) continue;
            const int mt = u / nb, j = u - mt * nb, b = b0 + j;
            if (!((bmask >> b) & 1u)) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e)
              s_w[w][4 * lk + e][li] =
                  make_float2(acc[k][0][e] - acc[k][1][e], acc[k][2][e] - acc[k][0][e] - acc[k][1][e]);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // lane 0..30: diagonal j - i = lane - 15, tap l = L-1 - 16 mt - (j - i),
            // 16 predicated reads in a fixed order
            if (lane < 31) {
              const int dl = lane - 15;
              const int l = L - 1 - 16 * mt - dl;
              if (l >= 0 && l < L) {
                float2 v[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                  const int jj = i + dl;
                  v[i] = s_w[w][i][min(15, max(0, jj))];
                  if (jj < 0 || jj > 15) v[i] = make_float2(0.f, 0.f);
                }
                float sr = 0.f, si = 0.f;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                  sr += v[i].x;
                  si += v[i].y;
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
      }
      __syncthreads();   // LDS is rewritten by the next run
      r0 = r1;
    }
  }
}

void launch_bwd_gu_mfma(const prune_fb_desc &d, const BwdFrame *bf, const WorkItem *items,
                        const uint32_t *n_items, unsigned int *ticket, float2 *hg, uint32_t grid,
                        const uint32_t *sfirst, float2 *gx, hipStream_t s) {
  hipLaunchKernelGGL(k_bwd_gu_mfma, dim3(grid), dim3(kWG), 0, s, d, bf, items, n_items, ticket, hg,
                     sfirst, gx);
}

void launch_bwd_gh_mfma(const prune_fb_desc &d, const BwdFrame *bf, const WorkItem *items,
                        const uint32_t *n_items, unsigned int *ticket, float2 *partial,
                        uint32_t max_items, uint32_t grid, hipStream_t s) {
  // tiles per run: up to kMaxRun, about one run per workgroup of the grid
  const uint32_t run =
      std::max<uint32_t>(1, std::min<uint32_t>(kMaxRun, max_items / std::max(1u, grid)));
  hipLaunchKernelGGL(k_bwd_gh_mfma, dim3(grid), dim3(kWG), 0, s, d, bf, items, n_items, ticket,
                     partial, run);
}

}  // namespace prune
