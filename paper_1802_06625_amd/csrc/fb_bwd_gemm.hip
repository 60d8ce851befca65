// Adjoint of the filter bank as plain matrix products on the matrix cores
// (prune_fb_backward, form 3: both gradients from one pass over each tile).
//
// Notation as in the other adjoint kernels: g = grad_y, p = b-1 the power of
// branch b, r = |x|, u_p = r^p x.  Per frame, the active branches of every
// bank fold into one table of taps per power,
//   C_p[l] = sum of h_{k,p}[l] over banks k with branch (k, p) active and l < L_k,
// because grad_x depends on the branches only through that sum, and the tap
// gradient of branch (k, p) at tap l is the same correlation for every bank:
//   G_p[m]          = sum_l conj(C_p[l]) g[m+l]
//   grad_x[m]       = sum_p (p/2+1) r^p G_p[m] + (p/2) r^p (x^2/r^2) conj(G_p[m])
//   W[l][p]         = sum_m g[m+l] conj(u_p[m])
//   grad_h_{k,p}[l] = W[l][p]   where (k, p) is active and l < L_k.
// Both cores are real products on v_mfma_f32_16x16x4_f32 with complex values
// split into (re, im) along the contraction and along the result:
//  * grad_x, per block of 16 positions m: result rows (p, re|im), columns m,
//    contraction (l, re|im) in steps of two taps; the row operand is the
//    frame's tap table (conj(C) as a real 2x2 block per (p, l)), the column
//    operand is the cotangent's Hankel matrix g[m+l] read from LDS.
//  * W: result rows l, columns (p, re|im), contraction (m, re|im) over the
//    tile's positions; the row operand is the same Hankel matrix, the column
//    operand the basis planes u_p (re, im) of 64 positions at a time.
// With up to 8 powers and 16 taps no matrix-core product is padding.
//
// Work: a tile is kBT consecutive input positions m of one frame (items from
// the same preparation kernel as the other forms), taken with an atomic
// ticket; a frame's first tile also takes the 64 positions before the frame
// (the stream's history): grad_x there is the frame's halo row for the
// fix-up kernel, and its W terms are the pairs whose input precedes the
// frame.  Each wave takes 64-position steps of the tile, builds their basis
// planes in its own LDS area, and accumulates its share of W; the four
// waves' W are added in a fixed order and written as the tile's partial row
// (the per-stream float64 reduction is shared with the other forms).  After
// its items the kernel zeroes the samples of grad_x outside every frame.
#include <algorithm>
#include <atomic>

#include "bwd_common.h"
#include "runtime_kernels.h"

namespace prune {

namespace {
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kGW = 4;                             // waves per workgroup
constexpr int kGWG = 64 * kGW;
constexpr int kPre = 64;                           // history positions of a frame's first tile
constexpr int kMaxP = 10;                          // powers per bank
constexpr int kGWin = kPre + kBT + PRUNE_MAX_L;    // cotangent window positions
constexpr int kUPlane = 2 * 64 + 4;                // words per basis plane (planes 4 banks apart)
constexpr int kAxSteps = PRUNE_MAX_L / 2;          // grad_x contraction steps (two taps each)
constexpr int kChunks = kBT / 64 + 1;              // 64-position steps of a tile, history first

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Powers and taps that a frame's active branches reach over all banks.
struct FrameShape {
  int KH;   // highest active power + 1 (0: no active branch)
  int Lf;   // most taps of a bank with an active branch
};

__device__ __forceinline__ FrameShape frame_shape(const prune_fb_desc &d, uint32_t mask) {
  const uint32_t kfull = (1u << d.Kmax) - 1u;
  FrameShape s{0, 0};
  for (uint32_t bank = 0; bank < d.n_banks; ++bank) {
    const uint32_t bm = (mask >> (bank * d.Kmax)) & kfull;
    if (!bm) continue;
    s.KH = max(s.KH, 32 - __clz(bm));
    s.Lf = max(s.Lf, (int)d.L[bank]);
  }
  return s;
}
}  // namespace

// RT: 16-row tiles of (power, re|im) (1 for up to 8 powers, 2 for 10);
// LT: 16-row tiles of taps in W (up to 4 for 64 taps).
template <int RT, int LT>
__global__ __launch_bounds__(kGWG) __attribute__((amdgpu_waves_per_eu(RT == 1 ? (LT == 1 ? 4 : 3) : 2))) void k_bwd_gemm(prune_fb_desc d, const BwdFrame *__restrict__ bf,
                                                  const WorkItem *__restrict__ items,
                                                  const uint32_t *__restrict__ n_items,
                                                  unsigned int *__restrict__ ticket,
                                                  float2 *__restrict__ hg, float2 *__restrict__ partial,
                                                  uint32_t run, const uint32_t *__restrict__ sfirst,
                                                  float2 *__restrict__ gxs) {
  // cotangent window of the tile: position n0 - kPre + k at words 2k, 2k+1;
  // at the end of a run of tiles it holds W[l][p] for the partial row
  __shared__ float2 s_g[kGWin];
  // per-wave basis planes u_p of the current 64 positions (word p*kUPlane +
  // 2q + re|im); at the end of a run, the waves' W for the fixed-order sum
  __shared__ float s_u[kGW * kMaxP * kUPlane];
  __shared__ float s_r[kGW * 64];               // r of each wave's current 64 positions
  __shared__ float s_ax[RT * kAxSteps * 64];    // grad_x row operand per (row tile, step, lane)
  __shared__ uint32_t s_next[2];
  static_assert(kGW * LT * 4 * 64 <= kGW * kMaxP * kUPlane, "W sum fits in the basis planes");
  static_assert(PRUNE_MAX_L * kMaxP <= kGWin, "W table fits in the window");
  constexpr int NH = (LT * RT <= 2) ? 2 : 1;   // W accumulator sets (alternate steps)
  constexpr bool ACACHE = 8 * LT * RT <= 16;   // grad_x row operand kept in registers
  constexpr int WU = LT * RT <= 2 ? 4 : 1;       // W group pairs unrolled (all of them when small)
  constexpr int NGW = (kGWin + kGWG - 1) / kGWG;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int j16 = lane & 15, q4 = lane >> 4;
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = max(Lmax, d.L[b]);
  const int H = (int)Lmax - 1;
  const uint32_t E = d.n_banks * d.Kmax * Lmax;
  const uint32_t ni = *n_items;
  const uint32_t R = min(max(run, 1u), 8u), ng = (ni + R - 1) / R;
  const bool want_x = gxs != nullptr, want_h = partial != nullptr;
  float *const su = s_u + w * kMaxP * kUPlane;
  float *const sr = s_r + w * 64;
  const float *const sg = reinterpret_cast<const float *>(s_g);
  // the grad_x weights (p/2 + 1) and p/2 of this lane's powers p = 8 rt + 2 q4 + e2
  float c_al[RT][2], c_be[RT][2];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int e2 = 0; e2 < 2; ++e2) {
      c_be[rt][e2] = 0.5f * (float)(8 * rt + 2 * q4 + e2);
      c_al[rt][e2] = c_be[rt][e2] + 1.f;
    }
  // this lane's column-operand offsets into the basis planes (W):
  // column (p, c) = (8 ct + j16/2, j16&1), contraction (q, c') = (2s + q4/2, q4&1):
  // g conj(u) = (gr ur + gi ui) + i (gi ur - gr ui)
  int uoff[RT];
  float usgn[RT];
#pragma unroll
  for (int ct = 0; ct < RT; ++ct) {
    const int p = min(8 * ct + (j16 >> 1), kMaxP - 1), c = j16 & 1, cp = q4 & 1;
    uoff[ct] = p * kUPlane + 2 * (q4 >> 1) + (cp ^ c);
    usgn[ct] = (c && !cp) ? -1.f : 1.f;
  }
  // the 64-position steps of a tile: ci = 0 is the history before the frame
  // (first tile only), ci = 1 + k covers positions n0 + 64k; wave w takes
  // ci = w+1, w+5, ... (and the history step, on wave 3)
  auto first_ci = [&](uint32_t tile) {
    const int c = (w + 1) & 3;
    return (c == 0 && (tile != 0 || H == 0)) ? kGW : c;
  };
  auto x_at = [&](const BwdFrame &F, int m) {   // inputs of the frame or the stream's history
    return (!F.route && m < (int)F.n && m >= -(int)F.t0) ? ld_global(F.x + m) : make_float2(0.f, 0.f);
  };

  // a tile's cotangent window and this wave's first input sample, loaded
  // into registers one tile ahead
  float2 gv[NGW], xn;
  auto prefetch = [&](uint32_t itx) {
    const WorkItem wi = items[itx];
    const BwdFrame F = bf[wi.frame];
    const int n = F.route ? 0 : (int)F.n, base = (int)wi.tile * kBT - kPre;
#pragma unroll
    for (int i = 0; i < NGW; ++i) {
      const int k = t + i * kGWG, p = base + k;
      gv[i] = (k < kGWin && p >= 0 && p < n) ? ld_global(F.g + p) : make_float2(0.f, 0.f);
    }
    xn = x_at(F, base + 64 * first_ci(wi.tile) + lane);
  };

  uint32_t grp = blockIdx.x, par = 0, tab_frame = 0xffffffffu;
  if (grp < ng) prefetch(grp * R);
  for (;;) {
    if (grp >= ng) break;
    if (t == 0) s_next[par ^ 1u] = gridDim.x >= ng ? ng : gridDim.x + atomicAdd(ticket, 1u);
    const uint32_t i0 = grp * R, i1 = min(ni, i0 + R);
    uint32_t grp_next = 0;
    // W of the current segment (consecutive tiles of one frame in the run)
    floatx4 acc_h[NH][LT][RT];
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int lt = 0; lt < LT; ++lt)
#pragma unroll
        for (int ct = 0; ct < RT; ++ct) acc_h[h][lt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
    uint32_t seg0 = i0;
    for (uint32_t it = i0; it < i1; ++it) {
      const WorkItem wi = items[it];
      const BwdFrame F = bf[wi.frame];
      const int n = (int)F.n, n0 = (int)wi.tile * kBT;
      const FrameShape fs = F.route ? FrameShape{0, 0} : frame_shape(d, F.mask);
      const int RTf = (2 * fs.KH + 15) / 16, LTf = (fs.Lf + 15) / 16, Sf = (fs.Lf + 1) / 2;
      const bool seg_end = it + 1 == i1 || items[it + 1].frame != wi.frame;
      __syncthreads();   // the previous tile's readers of s_g, s_u and s_ax are done
#pragma unroll
      for (int i = 0; i < NGW; ++i) {
        const int k = t + i * kGWG;
        if (k < kGWin) s_g[k] = gv[i];
      }
      if (want_x && !F.route && wi.frame != tab_frame) {   // uniform: one frame per tile
        // row (p, re|im) = (8 rt + i/2, i&1), contraction (l, re|im) = (2s + kk/2, kk&1):
        // conj(C) g = (a gr + b gi) + i (a gi - b gr) for C = a + ib; rows of
        // powers no active branch has are zero
        for (int e = t; e < RT * Sf * 64; e += kGWG) {
          const int rt = e / (Sf * 64), s = (e / 64) % Sf, ln = e & 63;
          const int i = ln & 15, kk = ln >> 4;
          const int p = 8 * rt + (i >> 1), l = 2 * s + (kk >> 1);
          float a = 0.f, b = 0.f;
          if (p < (int)d.Kmax) {
            for (uint32_t bank = 0; bank < d.n_banks; ++bank) {
              if (((F.mask >> (bank * d.Kmax + p)) & 1u) && l < (int)d.L[bank]) {
                const float2 h = ld_global(F.taps + ((size_t)bank * d.Kmax + p) * Lmax + l);
                a += h.x;
                b += h.y;
              }
            }
          }
          s_ax[(rt * kAxSteps + s) * 64 + ln] = (i & 1) ? ((kk & 1) ? a : -b) : ((kk & 1) ? b : a);
        }
        tab_frame = wi.frame;
      }
      __syncthreads();
      // the grad_x row operand of every step in registers, when it fits
      float acache[ACACHE ? 8 * LT * RT : 1];
      if constexpr (ACACHE) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int s = 0; s < 8 * LT; ++s)
            acache[rt * 8 * LT + s] = s < Sf ? s_ax[(rt * kAxSteps + s) * 64 + lane] : 0.f;
      }
      // the ticket read from LDS is the same in every lane: readfirstlane
      // lets the compiler keep it, and all that depends on it, in scalars
      if (it == i0) grp_next = __builtin_amdgcn_readfirstlane(s_next[par ^ 1u]);
      const float2 x_first = xn;
      if (it + 1 < i1) prefetch(it + 1);   // in flight during the steps below
      else if (grp_next < ng) prefetch(grp_next * R);

      if (F.route) {
        // passthrough-routed frame: grad_x = g over the tile, no tap gradient
        if (want_x)
          for (int k = t; k < kBT; k += kGWG)
            if (n0 + k < n) st_global(F.gx + n0 + k, ld_global(F.g + n0 + k));
      } else {
        float2 xv = x_first;
        for (int ci = first_ci(wi.tile); ci < kChunks; ci += kGW) {
          const int m0 = n0 - kPre + 64 * ci;
          if (ci > 0 && m0 >= n) break;   // later steps lie further beyond the frame
          const float2 x_next = x_at(F, m0 + 64 * kGW + lane);   // the wave's next step
          {
            // basis planes of positions m0 .. m0+63 (zero past the frame and
            // before the stream)
            const float r = sqrtf(xv.x * xv.x + xv.y * xv.y);
            sr[lane] = r;
            float2 v = xv;
            for (int p = 0; p < fs.KH || p == 0; ++p) {
              *reinterpret_cast<float2 *>(su + p * kUPlane + 2 * lane) = v;
              v.x *= r;
              v.y *= r;
            }
          }
          wave_sync_lds();
          // Hankel operand offset of this lane: position m0 + j16 + q4/2 (+ l), word re|im = q4&1
          const int goff = 2 * (m0 - (n0 - kPre) + j16 + (q4 >> 1)) + (q4 & 1);
          // the step's work: grad_x products (ax), the W products, and the
          // grad_x epilogue; with both gradients wanted the W products and
          // the epilogue sit in one basic block, so that the scheduler can
          // issue the epilogue's vector instructions while the matrix cores
          // run
          floatx4 ax[4][RT];
          float gr = 0.f, gi = 0.f;
          auto gx_products = [&]() {
#pragma unroll
            for (int blk = 0; blk < 4; ++blk)
#pragma unroll
              for (int rt = 0; rt < RT; ++rt) ax[blk][rt] = floatx4{0.f, 0.f, 0.f, 0.f};
            if constexpr (ACACHE) {
              // row operand from registers (loaded once per tile), column
              // operands of step s + 1 read while step s is on the matrix cores
              float bn[4];
#pragma unroll
              for (int blk = 0; blk < 4; ++blk) bn[blk] = sg[goff + 32 * blk];
#pragma unroll
              for (int s = 0; s < 8 * LT; ++s) {
                if (s < Sf) {
                  float b[4];
#pragma unroll
                  for (int blk = 0; blk < 4; ++blk) b[blk] = bn[blk];
                  if (s + 1 < Sf) {
#pragma unroll
                    for (int blk = 0; blk < 4; ++blk) bn[blk] = sg[goff + 32 * blk + 4 * (s + 1)];
                  }
                  __builtin_amdgcn_sched_barrier(0);   // the next step's reads go first
#pragma unroll
                  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int blk = 0; blk < 4; ++blk)
                      ax[blk][rt] = mfma4(acache[rt * 8 * LT + s], b[blk], ax[blk][rt]);
                }
              }
            } else {
              // steps in pairs, each operand buffer keeping its role: the
              // reads of step s + 1 are issued before the products of step s
              // (the step index is clamped at the last step)
              float an[2][RT], bn[2][4];
              auto load1 = [&](int buf, int st) {
                st = min(st, Sf - 1);
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) an[buf][rt] = s_ax[(rt * kAxSteps + st) * 64 + lane];
#pragma unroll
                for (int blk = 0; blk < 4; ++blk) bn[buf][blk] = sg[goff + 32 * blk + 4 * st];
              };
              auto products1 = [&](int buf) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                  for (int blk = 0; blk < 4; ++blk) ax[blk][rt] = mfma4(an[buf][rt], bn[buf][blk], ax[blk][rt]);
              };
              load1(0, 0);
              for (int st = 0; st < Sf; st += 2) {
                load1(1, st + 1);
                __builtin_amdgcn_sched_barrier(0);
                products1(0);
                if (st + 1 < Sf) {
                  load1(0, st + 2);
                  __builtin_amdgcn_sched_barrier(0);
                  products1(1);
                }
              }
            }
          };
          // the grad_x epilogue in six pieces: lane (q4, j16) holds G_p at
          // position m0 + 16 blk + j16 for p = 8 rt + 2 q4 + e/2, re|im =
          // e&1; its shares of S1 = sum_p (p/2+1) r^p G_p and
          // S2 = sum_p (p/2) r^p conj(G_p) are summed over the four lane
          // groups so that lane group q4 keeps block q4 (blocks i and 2+i
          // across lanes 32 apart, then one block of the pair across lanes
          // 16 apart), and grad_x = S1 + (x^2/r^2) S2 at position m0 + lane
          float Pa[4], Pb[4], Q[2][4], S[4];
          auto share = [&](int blk, float (&P)[4]) {
            const float r = sr[16 * blk + j16], r2 = r * r, r4 = r2 * r2;
            const float pw0 = ((q4 & 1) ? r2 : 1.f) * ((q4 & 2) ? r4 : 1.f);   // r^(2 q4)
            P[0] = P[1] = P[2] = P[3] = 0.f;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
              float pw = rt ? pw0 * (r4 * r4) : pw0;
#pragma unroll
              for (int e2 = 0; e2 < 2; ++e2) {
                const float al = c_al[rt][e2] * pw, be = c_be[rt][e2] * pw;
                const float g_r = ax[blk][rt][2 * e2], g_i = ax[blk][rt][2 * e2 + 1];
                P[0] = fmaf(al, g_r, P[0]);
                P[1] = fmaf(al, g_i, P[1]);
                P[2] = fmaf(be, g_r, P[2]);
                P[3] = fmaf(-be, g_i, P[3]);
                pw *= r;
              }
            }
          };
          const bool hi2 = q4 & 2, hi1 = q4 & 1;
          auto epi_piece = [&](int k) {
            if (k == 0 || k == 2) {
              share(k >> 1, Pa);
            } else if (k == 1 || k == 3) {
              share(2 + (k >> 1), Pb);
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const float mine = hi2 ? Pb[v] : Pa[v], oth = hi2 ? Pa[v] : Pb[v];
                Q[k >> 1][v] = mine + __shfl_xor(oth, 32, 64);
              }
            } else if (k == 4) {
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const float mine = hi1 ? Q[1][v] : Q[0][v], oth = hi1 ? Q[0][v] : Q[1][v];
                S[v] = mine + __shfl_xor(oth, 16, 64);
              }
            } else if (k == 5) {
              // (x^2/r^2 is taken as zero at r = 0, where S2 is zero); no
              // contraction, so that every code path rounds the same way
#pragma clang fp contract(off)
              const float r2 = xv.x * xv.x + xv.y * xv.y;
              const float inv = r2 > 0.f ? 1.f / r2 : 0.f;
              const float er = (xv.x * xv.x - xv.y * xv.y) * inv, ei = 2.f * xv.x * xv.y * inv;
              gr = S[0] + (er * S[2] - ei * S[3]);
              gi = S[1] + (er * S[3] + ei * S[2]);
            }
          };
          auto gx_epilogue = [&]() {
#pragma unroll
            for (int k = 0; k < 6; ++k) epi_piece(k);
          };
          // hook(g) runs between the reads of group g+1 and the products of group g
          auto w_products = [&](auto hook) {
            // W over the 64 positions: rows l = 16 lt + j16, 32 steps of
            // (two positions, re|im); alternate accumulator sets when few.
            // Rows past the frame's taps and columns of powers beyond its
            // highest active one (stale planes) are computed and never written.
            // operands of four steps at a time, the next four read while
            // the current ones are on the matrix cores
            float ab[2][4][LT], bb[2][4][RT];
            auto load4 = [&](int buf, int s0) {
#pragma unroll
              for (int k = 0; k < 4; ++k) {
#pragma unroll
                for (int lt = 0; lt < LT; ++lt) ab[buf][k][lt] = sg[goff + 32 * lt + 4 * (s0 + k)];
#pragma unroll
                for (int ct = 0; ct < RT; ++ct) bb[buf][k][ct] = su[uoff[ct] + 4 * (s0 + k)];
              }
            };
            // groups in pairs, so that each buffer keeps its role (no copies
            // between them): the reads of group g+1 are issued before the
            // products of group g
            auto products4 = [&](int buf) {
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                const int h = NH == 2 ? (k & 1) : 0;
#pragma unroll
                for (int lt = 0; lt < LT; ++lt)
#pragma unroll
                  for (int ct = 0; ct < RT; ++ct)
                    acc_h[h][lt][ct] = mfma4(ab[buf][k][lt], usgn[ct] * bb[buf][k][ct], acc_h[h][lt][ct]);
              }
            };
            load4(0, 0);
#pragma unroll WU
            for (int g = 0; g < 8; g += 2) {
              load4(1, 4 * g + 4);
              __builtin_amdgcn_sched_barrier(0);
              hook(g);
              products4(0);
              if (g + 2 < 8) load4(0, 4 * g + 8);
              __builtin_amdgcn_sched_barrier(0);
              hook(g + 1);
              products4(1);
            }
          };
          if (want_x && want_h) {
            gx_products();
            if constexpr (LT * RT <= 2) {
              // W groups fully unrolled: the epilogue's pieces go between them
              w_products([&](int g) {
                if (g < 6) epi_piece(g);
              });
            } else {
              w_products([](int) {});
              gx_epilogue();
            }
          } else if (want_x) {
            gx_products();
            gx_epilogue();
          } else {
            w_products([](int) {});
          }
          if (want_x) {
            const int m = m0 + lane;
            if (ci == 0) {
              if (m >= -H) hg[(size_t)wi.frame * H + (m + H)] = make_float2(gr, gi);
            } else if (m < n) {
              st_global(F.gx + m, make_float2(gr, gi));
            }
          }
          wave_sync_lds();   // the planes are rewritten by the next step
          xv = x_next;
        }
      }
      if (want_h && seg_end) {
        // the segment's tiles seg0 .. it: W (summed over the four waves in a
        // fixed order, one column tile at a time, into the W table in s_g)
        // in the row of seg0, zero rows for the others
        float2 *const s_W = s_g;   // [l][p], PRUNE_MAX_L x kMaxP
        for (int ct = 0; ct < RTf; ++ct) {
          __syncthreads();   // every wave is done with s_g / s_u
#pragma unroll
          for (int lt = 0; lt < LT; ++lt) {
            if (lt < LTf) {
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                float v = 0.f;
#pragma unroll
                for (int h = 0; h < NH; ++h) v += acc_h[h][lt][ct][e];
                s_u[((w * LT + lt) * 4 + e) * 64 + lane] = v;
              }
            }
          }
          __syncthreads();
          // entry (l, pp, c): lane group (l%16)/4, register l%4, column 2 pp + c
          for (int k = t; k < LTf * 16 * 16; k += kGWG) {
            const int l = k >> 4, col = k & 15, p = 8 * ct + (col >> 1);
            const int src = (((l >> 4) * 4 + (l & 3)) * 64) + 16 * ((l & 15) >> 2) + col;
            float v = 0.f;
#pragma unroll
            for (int ww = 0; ww < kGW; ++ww) v += s_u[ww * LT * 4 * 64 + src];
            if (p < kMaxP) reinterpret_cast<float *>(&s_W[l * kMaxP + p])[col & 1] = v;
          }
        }
        __syncthreads();
        for (uint32_t k = t; k < (it + 1 - seg0) * E; k += kGWG) {
          const uint32_t e = k % E;
          const uint32_t bank = e / (d.Kmax * Lmax), p = (e / Lmax) % d.Kmax, l = e % Lmax;
          const bool act = k < E && !F.route && ((F.mask >> (bank * d.Kmax + p)) & 1u) && l < d.L[bank];
          partial[(size_t)seg0 * E + k] = act ? s_W[l * kMaxP + p] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
          for (int lt = 0; lt < LT; ++lt)
#pragma unroll
            for (int ct = 0; ct < RT; ++ct) acc_h[h][lt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
        seg0 = it + 1;
      }
    }
    grp = grp_next;
    par ^= 1u;
  }
  if (want_x && sfirst) bwd_zero_gaps(d, bf, sfirst, gxs);
}

// One-wave form for small shapes (at most 8 powers, at most 16 taps): the
// same products, with every wave on its own work (kWaveWG independent waves
// per workgroup) and no barriers, so that waves drift out of phase and one
// wave's loads overlap another's products.  Items are tiles of kWaveT positions (the preparation kernel's
// tile for this form); a frame's first tile also takes the 64 history
// positions.  Per 64-position step the wave stages the cotangent window
// (positions m0 .. m0+127) and the basis planes in its own LDS, the next
// step's inputs and window are read into registers meanwhile, and W is kept
// over a run of consecutive tiles of one frame (the run's first row holds
// it, the others are zero).  The grad_x row operand (the folded taps) lives
// in registers, rebuilt when the frame changes.  Work is assigned
// statically: with every wave resident and tiles of equal cost, a shared
// atomic ticket per group only adds its round trip (measured at twice the
// kernel time on 256 frames of 8192 samples).
constexpr int kWaveT = 512;
constexpr int kWWin = 128;   // cotangent window positions per step
// Waves per workgroup, each an independent worker: 1, 2, 4 and 8 measured
// 0.081, 0.080, 0.078 and 0.077 ms for the whole adjoint of 256 frames of
// 8192 samples (fewer workgroups to dispatch).
constexpr int kWaveWG = 8;

// NS: grad_x contraction steps (two taps each) taken for every frame: 4 when
// no bank has more than 8 taps, else 8 (the tap table is zero past a frame's
// own taps, so that the extra steps add zeros).
// WV: waves per workgroup, each an independent worker with its own LDS
// area (more waves per workgroup, fewer workgroups to dispatch).
template <int NS, int WV>
__global__ __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(4))) void k_bwd_gemm_wave(
    prune_fb_desc d, const BwdFrame *__restrict__ bf, const WorkItem *__restrict__ items,
    const uint32_t *__restrict__ n_items, float2 *__restrict__ hg, float2 *__restrict__ partial, uint32_t run,
    const uint32_t *__restrict__ sfirst, float2 *__restrict__ gxs) {
  __shared__ float2 s_gw_all[WV][kWWin];
  __shared__ float s_pl_all[WV][8 * kUPlane];
  __shared__ float s_rw_all[WV][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, j16 = lane & 15, q4 = lane >> 4;
  float2 *const s_gw = s_gw_all[wv];
  float *const s_pl = s_pl_all[wv];
  float *const s_rw = s_rw_all[wv];
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = max(Lmax, d.L[b]);
  const int H = (int)Lmax - 1;
  const uint32_t E = d.n_banks * d.Kmax * Lmax;
  const uint32_t ni = *n_items;
  const uint32_t R = min(max(run, 1u), 8u), ng = (ni + R - 1) / R;
  const bool want_x = gxs != nullptr, want_h = partial != nullptr;
  const float *const sg = reinterpret_cast<const float *>(s_gw);
  float c_al[2], c_be[2];
#pragma unroll
  for (int e2 = 0; e2 < 2; ++e2) {
    c_be[e2] = 0.5f * (float)(2 * q4 + e2);
    c_al[e2] = c_be[e2] + 1.f;
  }
  const int p_col = j16 >> 1, c_col = j16 & 1, cp = q4 & 1;
  const int uoff = p_col * kUPlane + 2 * (q4 >> 1) + (cp ^ c_col);
  const float usgn = (c_col && !cp) ? -1.f : 1.f;
  // the Hankel operand offset of this lane within the window (position
  // j16 + q4/2, word re|im = q4&1)
  const int goff = 2 * (j16 + (q4 >> 1)) + (q4 & 1);
  auto x_at = [&](const BwdFrame &F, int m) {
    return (!F.route && m < (int)F.n && m >= -(int)F.t0) ? ld_global(F.x + m) : make_float2(0.f, 0.f);
  };
  auto g_at = [&](const BwdFrame &F, int m) {
    return (!F.route && m >= 0 && m < (int)F.n) ? ld_global(F.g + m) : make_float2(0.f, 0.f);
  };
  float acache[8];
  uint32_t tab_frame = 0xffffffffu;
  // static assignment, one contiguous range of groups per XCD (workgroups
  // are dealt to the 8 XCDs round robin), so that neighbouring tiles, which
  // share cotangent samples, are read through one L2
  const uint32_t nx = (gridDim.x % 8u) ? 1u : 8u, per_x = gridDim.x / nx * WV;
  const uint32_t chunk = (ng + nx - 1) / nx, xcd = blockIdx.x % nx;
  const uint32_t g_end = min(ng, (xcd + 1) * chunk);
  for (uint32_t grp = xcd * chunk + blockIdx.x / nx * WV + wv; grp < g_end; grp += per_x) {
    const uint32_t i0 = grp * R, i1 = min(ni, i0 + R);
    floatx4 acc_h[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
    uint32_t seg0 = i0;
    for (uint32_t it = i0; it < i1; ++it) {
      const WorkItem wi = items[it];
      const BwdFrame F = bf[wi.frame];
      const int n = (int)F.n, n0 = (int)wi.tile * kWaveT;
      const FrameShape fs = F.route ? FrameShape{0, 0} : frame_shape(d, F.mask);
      const int Sf = (fs.Lf + 1) / 2;
      const bool seg_end = it + 1 == i1 || items[it + 1].frame != wi.frame;
      if (F.route) {
        if (want_x)
          for (int k = lane; k < kWaveT; k += 64)
            if (n0 + k < n) st_global(F.gx + n0 + k, ld_global(F.g + n0 + k));
      } else {
        if (want_x && wi.frame != tab_frame) {
          // row (p, re|im) = (i/2, i&1), contraction (l, re|im) = (2s + kk/2, kk&1);
          // a bank's eight taps of this lane are read together
          const int p = j16 >> 1;
          float a[8], b[8];
#pragma unroll
          for (int st = 0; st < 8; ++st) a[st] = b[st] = 0.f;
          for (uint32_t bank = 0; bank < d.n_banks; ++bank) {
            const bool on = p < (int)d.Kmax && ((F.mask >> (bank * d.Kmax + p)) & 1u);
            float2 h[8];
#pragma unroll
            for (int st = 0; st < 8; ++st) {
              const int l = 2 * st + (q4 >> 1);
              h[st] = (on && st < Sf && l < (int)d.L[bank])
                          ? ld_global(F.taps + ((size_t)bank * d.Kmax + p) * Lmax + l)
                          : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int st = 0; st < 8; ++st) {
              a[st] += h[st].x;
              b[st] += h[st].y;
            }
          }
#pragma unroll
          for (int st = 0; st < 8; ++st)
            acache[st] = (j16 & 1) ? ((q4 & 1) ? a[st] : -b[st]) : ((q4 & 1) ? b[st] : a[st]);
          tab_frame = wi.frame;
        }
        // steps: the history step first (first tile only), then 4 of 64
        const int c_first = (wi.tile == 0 && H > 0) ? 0 : 1;
        int m0 = n0 - 64 + 64 * c_first;
        float2 xv = x_at(F, m0 + lane);
        float2 gw0 = g_at(F, m0 + lane), gw1 = g_at(F, m0 + 64 + lane);
        for (int ci = c_first; ci <= kWaveT / 64; ++ci, m0 += 64) {
          if (ci > 0 && m0 >= n) break;
          {
            s_gw[lane] = gw0;
            s_gw[64 + lane] = gw1;
            const float r = sqrtf(xv.x * xv.x + xv.y * xv.y);
            s_rw[lane] = r;
            float2 v = xv;
            for (int p = 0; p < fs.KH || p == 0; ++p) {
              *reinterpret_cast<float2 *>(s_pl + p * kUPlane + 2 * lane) = v;
              v.x *= r;
              v.y *= r;
            }
          }
          wave_sync_lds();
          // the next step's inputs, in flight during this step's products
          const float2 x_cur = xv;
          xv = x_at(F, m0 + 64 + lane);
          gw0 = gw1;
          gw1 = g_at(F, m0 + 128 + lane);
          float gr = 0.f, gi = 0.f;
          if (want_x) {
            floatx4 ax[4] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f},
                             floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
            // column operands of step st + 1 read while step st is on the matrix cores
            float bn[2][4];
#pragma unroll
            for (int blk = 0; blk < 4; ++blk) bn[0][blk] = sg[goff + 32 * blk];
#pragma unroll
            for (int st = 0; st < NS; ++st) {
              if (st + 1 < NS) {
#pragma unroll
                for (int blk = 0; blk < 4; ++blk) bn[(st + 1) & 1][blk] = sg[goff + 32 * blk + 4 * (st + 1)];
              }
              __builtin_amdgcn_sched_barrier(0);
#pragma unroll
              for (int blk = 0; blk < 4; ++blk) ax[blk] = mfma4(acache[st], bn[st & 1][blk], ax[blk]);
            }
            float P[4][4];
#pragma unroll
            for (int blk = 0; blk < 4; ++blk) {
              const float r = s_rw[16 * blk + j16], r2 = r * r, r4 = r2 * r2;
              float pw = ((q4 & 1) ? r2 : 1.f) * ((q4 & 2) ? r4 : 1.f);   // r^(2 q4)
              P[blk][0] = P[blk][1] = P[blk][2] = P[blk][3] = 0.f;
#pragma unroll
              for (int e2 = 0; e2 < 2; ++e2) {
                const float al = c_al[e2] * pw, be = c_be[e2] * pw;
                const float g_r = ax[blk][2 * e2], g_i = ax[blk][2 * e2 + 1];
                P[blk][0] = fmaf(al, g_r, P[blk][0]);
                P[blk][1] = fmaf(al, g_i, P[blk][1]);
                P[blk][2] = fmaf(be, g_r, P[blk][2]);
                P[blk][3] = fmaf(-be, g_i, P[blk][3]);
                pw *= r;
              }
            }
            const bool hi2 = q4 & 2, hi1 = q4 & 1;
            float Q[2][4], S[4];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const float mine = hi2 ? P[2 + i][v] : P[i][v], oth = hi2 ? P[i][v] : P[2 + i][v];
                Q[i][v] = mine + __shfl_xor(oth, 32, 64);
              }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const float mine = hi1 ? Q[1][v] : Q[0][v], oth = hi1 ? Q[0][v] : Q[1][v];
              S[v] = mine + __shfl_xor(oth, 16, 64);
            }
            {
#pragma clang fp contract(off)
              const float r2 = x_cur.x * x_cur.x + x_cur.y * x_cur.y;
              const float inv = r2 > 0.f ? 1.f / r2 : 0.f;
              const float er = (x_cur.x * x_cur.x - x_cur.y * x_cur.y) * inv, ei = 2.f * x_cur.x * x_cur.y * inv;
              gr = S[0] + (er * S[2] - ei * S[3]);
              gi = S[1] + (er * S[3] + ei * S[2]);
            }
          }
          if (want_h) {
            // W over the 64 positions: rows l = j16, 32 steps of (two
            // positions, re|im), two accumulator sets
            // operands of four steps at a time, the next four read while the
            // current ones are on the matrix cores
            float ab[2][4], bb[2][4];
            auto load4 = [&](int buf, int s0) {
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                ab[buf][k] = sg[goff + 4 * (s0 + k)];
                bb[buf][k] = usgn * s_pl[uoff + 4 * (s0 + k)];
              }
            };
            auto prod4 = [&](int buf) {
#pragma unroll
              for (int k = 0; k < 4; ++k) acc_h[k & 1] = mfma4(ab[buf][k], bb[buf][k], acc_h[k & 1]);
            };
            load4(0, 0);
#pragma unroll
            for (int g8 = 0; g8 < 8; g8 += 2) {
              load4(1, 4 * g8 + 4);
              __builtin_amdgcn_sched_barrier(0);
              prod4(0);
              if (g8 + 2 < 8) load4(0, 4 * g8 + 8);
              __builtin_amdgcn_sched_barrier(0);
              prod4(1);
            }
          }
          if (want_x) {
            const int m = m0 + lane;
            if (ci == 0) {
              if (m >= -H) hg[(size_t)wi.frame * H + (m + H)] = make_float2(gr, gi);
            } else if (m < n) {
              st_global(F.gx + m, make_float2(gr, gi));
            }
          }
          wave_sync_lds();   // the window and planes are rewritten by the next step
        }
      }
      if (want_h && seg_end) {
        // rows seg0 .. it: W (lane (q4, j16) holds row l = 4 q4 + e, column
        // (p, re|im) = (j16/2, j16&1)) into the row of seg0, zero elsewhere;
        // every entry of a row belongs to one lane (p < 8, l < 16)
        const uint32_t p = j16 >> 1, c = j16 & 1;
        for (uint32_t row = seg0; row <= it; ++row) {
          float *prow = reinterpret_cast<float *>(partial + (size_t)row * E);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t l = 4 * q4 + e;
            const float w = acc_h[0][e] + acc_h[1][e];
            for (uint32_t bank = 0; bank < d.n_banks; ++bank) {
              if (p < d.Kmax && l < Lmax) {
                const bool act = row == seg0 && !F.route && ((F.mask >> (bank * d.Kmax + p)) & 1u) &&
                                 l < d.L[bank];
                prow[2 * (((size_t)bank * d.Kmax + p) * Lmax + l) + c] = act ? w : 0.f;
              }
            }
          }
        }
        acc_h[0] = acc_h[1] = floatx4{0.f, 0.f, 0.f, 0.f};
        seg0 = it + 1;
      }
    }
  }
  if (want_x && sfirst) bwd_zero_gaps(d, bf, sfirst, gxs);
}

namespace {
template <int RT, int LT>
int gemm_resident() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&k_bwd_gemm<RT, LT>),
                                                   kGWG, 0) != hipSuccess)
    n = 0;
  return std::max(n, 1);
}

template <int RT, int LT>
void launch_gemm(const prune_fb_desc &d, const BwdFrame *bf, const WorkItem *items, const uint32_t *n_items,
                 unsigned int *ticket, float2 *hg, float2 *partial, uint32_t max_items, uint32_t ncu,
                 const uint32_t *sfirst, float2 *gx, hipStream_t s) {
  static std::atomic<int> resident{0};
  int res = resident.load();
  if (res <= 0) {
    res = gemm_resident<RT, LT>();
    resident.store(res);
  }
  const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(max_items, ncu * (uint32_t)res));
  // tiles per ticket: up to 8, about one run per workgroup of the grid
  const uint32_t run = std::max<uint32_t>(1, std::min<uint32_t>(8, max_items / grid));
  hipLaunchKernelGGL((k_bwd_gemm<RT, LT>), dim3(grid), dim3(kGWG), 0, s, d, bf, items, n_items, ticket, hg,
                     partial, run, sfirst, gx);
}
}  // namespace

uint32_t bwd_gemm_tile(const prune_fb_desc &d) {
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = std::max(Lmax, d.L[b]);
  return (d.Kmax <= 8 && Lmax <= 16) ? (uint32_t)kWaveT : (uint32_t)kBT;
}

void launch_bwd_gemm(const prune_fb_desc &d, const BwdFrame *bf, const WorkItem *items,
                     const uint32_t *n_items, unsigned int *ticket, float2 *hg, float2 *partial,
                     uint32_t max_items, uint32_t ncu, const uint32_t *sfirst, float2 *gx, hipStream_t s) {
  uint32_t Lmax = 1;
  for (uint32_t b = 0; b < d.n_banks; ++b) Lmax = std::max(Lmax, d.L[b]);
  if (bwd_gemm_tile(d) == kWaveT) {
    auto launch = [&](auto kern, std::atomic<int> &resident) {
      int res = resident.load();
      if (res <= 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(kern), 64 * kWaveWG, 0) !=
            hipSuccess)
          nb = 0;
        res = std::max(nb, 1);
        resident.store(res);
      }
      // workers (waves): one per tile up to every resident wave
      const uint32_t grid = std::max<uint32_t>(
          1, std::min<uint32_t>((max_items + kWaveWG - 1) / kWaveWG, ncu * (uint32_t)res));
      const uint32_t run = std::max<uint32_t>(1, std::min<uint32_t>(8, max_items / (grid * kWaveWG)));
      hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * kWaveWG), 0, s, d, bf, items, n_items, hg, partial, run,
                         sfirst, gx);
    };
    static std::atomic<int> res4{0}, res8{0};
    if (Lmax <= 8) launch(&k_bwd_gemm_wave<4, kWaveWG>, res4);
    else launch(&k_bwd_gemm_wave<8, kWaveWG>, res8);
    return;
  }
  const int RT = d.Kmax > 8 ? 2 : 1, LT = (int)(Lmax + 15) / 16;
#define PRUNE_GEMM(rt, lt) \
  launch_gemm<rt, lt>(d, bf, items, n_items, ticket, hg, partial, max_items, ncu, sfirst, gx, s)
  if (RT == 1) {
    switch (LT) {
      case 1: PRUNE_GEMM(1, 1); break;
      case 2: PRUNE_GEMM(1, 2); break;
      case 3: PRUNE_GEMM(1, 3); break;
      default: PRUNE_GEMM(1, 4); break;
    }
  } else {
    switch (LT) {
      case 1: PRUNE_GEMM(2, 1); break;
      case 2: PRUNE_GEMM(2, 2); break;
      case 3: PRUNE_GEMM(2, 3); break;
      default: PRUNE_GEMM(2, 4); break;
    }
  }
#undef PRUNE_GEMM
}

}  // namespace prune
