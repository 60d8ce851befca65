// Definitions shared by the adjoint kernels (vector and matrix-core forms).
#pragma once
#include <hip/hip_runtime.h>

#include "prune_internal.h"

namespace prune {

constexpr int kBT = 1024;   // backward tile: outputs (and inputs) per work item

struct BwdFrame {
  const float2 *x;      // sample 0 of the frame (stream pointer + t0)
  const float2 *g;      // cotangent at sample 0
  float2 *gx;           // grad_x at sample 0
  const float2 *taps;   // [n_banks][Kmax][Lmax] of the frame's stream
  uint32_t n, mask, route, t0;
  uint32_t stream, pad0, pad1, pad2;
};

// Fixed-order float64 reduction of the grad_h tile partials of a stream
// (rows b0 .. b1 of partial, E entries each) in kRedG chunks.  Stage 1 sums
// chunk c of the stream: thread (q, el) of a 256-thread workgroup adds tiles
// q, q+4, ... of the chunk for entry eb*64 + el, and the four sub-sums are
// added in q order.  Stage 2 sums the chunk results the same way.  The order
// of every sum depends only on the item list, so results are reproducible.
constexpr int kRedG = 64;        // chunks per stream
constexpr int kRedQ = 4;         // sub-sums per entry

__device__ inline uint32_t red_per(uint32_t b0, uint32_t b1) {
  return (b1 - b0 + kRedG - 1) / kRedG;
}

// Stage 1, entries eb*64 .. eb*64+63 of chunk c of stream s.
__device__ inline void red_chunk_block(uint32_t E, const float2 *__restrict__ partial, uint32_t b0,
                                       uint32_t b1, uint32_t s, uint32_t c, uint32_t eb,
                                       double2 *__restrict__ part2, double2 (*red)[64]) {
  const uint32_t el = threadIdx.x & 63, q = threadIdx.x >> 6, e = eb * 64 + el;
  const uint32_t per = red_per(b0, b1);
  const uint32_t lo = min(b1, b0 + c * per), hi = min(b1, lo + per);
  double sr = 0.0, si = 0.0;
  if (e < E) {
    for (uint32_t t = lo + q; t < hi; t += kRedQ) {
      const float2 v = partial[(size_t)t * E + e];
      sr += v.x;
      si += v.y;
    }
  }
  red[q][el] = make_double2(sr, si);
  __syncthreads();
  if (q == 0 && e < E) {
    double2 a = red[0][el];
#pragma unroll
    for (int k = 1; k < kRedQ; ++k) {
      a.x += red[k][el].x;
      a.y += red[k][el].y;
    }
    part2[((size_t)s * kRedG + c) * E + e] = a;
  }
  __syncthreads();
}

// Stage 2, entries eb*64 .. eb*64+63 of stream s, over its chunks 0 .. nch-1
// (the chunks that hold tiles; later ones are empty).
__device__ inline void red_stream_block(uint32_t E, const double2 *__restrict__ part2, uint32_t s,
                                        uint32_t nch, uint32_t eb, float2 *__restrict__ gtaps,
                                        double2 (*red)[64]) {
  const uint32_t el = threadIdx.x & 63, q = threadIdx.x >> 6, e = eb * 64 + el;
  double sr = 0.0, si = 0.0;
  if (e < E) {
    for (uint32_t c = q; c < nch; c += kRedQ) {
      const double2 v = part2[((size_t)s * kRedG + c) * E + e];
      sr += v.x;
      si += v.y;
    }
  }
  red[q][el] = make_double2(sr, si);
  __syncthreads();
  if (q == 0 && e < E) {
    double2 a = red[0][el];
#pragma unroll
    for (int k = 1; k < kRedQ; ++k) {
      a.x += red[k][el].x;
      a.y += red[k][el].y;
    }
    gtaps[(size_t)s * E + e] = make_float2((float)a.x, (float)a.y);
  }
  __syncthreads();
}

// Samples of grad_x outside every frame get a zero gradient.  Run by every
// workgroup of a grid after its items: workgroup k takes frames k, k + grid,
// ... and zeroes the gap after each (up to the next frame of its stream or
// the stream's end) and, for a stream's first frame (sfirst), the samples
// before it; then streams without frames.  Frame samples are written by the
// items only, so the two never touch one sample.  (Positions are clamped to
// the stream: a frame out of range has n = 0.)
__device__ inline void bwd_zero_gaps(const prune_fb_desc &d, const BwdFrame *__restrict__ bf,
                                     const uint32_t *__restrict__ sfirst, float2 *__restrict__ gxs) {
  const uint64_t N = d.stream_len;
  const uint32_t t = threadIdx.x, nt = blockDim.x;
  for (uint32_t f = blockIdx.x; f < d.n_frames; f += gridDim.x) {
    const BwdFrame F = bf[f];
    if (F.stream >= d.n_streams) continue;
    float2 *row = gxs + (size_t)F.stream * N;
    const uint64_t end = min((uint64_t)F.t0 + F.n, N);
    uint64_t nxt = N;
    if (f + 1 < d.n_frames) {
      const BwdFrame G = bf[f + 1];
      if (G.stream == F.stream) nxt = min((uint64_t)G.t0, N);
    }
    for (uint64_t q = end + t; q < nxt; q += nt) row[q] = make_float2(0.f, 0.f);
    if (sfirst[F.stream] == f)
      for (uint64_t q = t; q < min((uint64_t)F.t0, N); q += nt) row[q] = make_float2(0.f, 0.f);
  }
  for (uint32_t st = blockIdx.x; st < d.n_streams; st += gridDim.x) {
    if (sfirst[st] != 0xffffffffu) continue;
    float2 *row = gxs + (size_t)st * N;
    for (uint64_t q = t; q < N; q += nt) row[q] = make_float2(0.f, 0.f);
  }
}

// Matrix-core adjoint over the same work items (one tile of kBT samples of
// one frame each) as the vector kernel:
//  grad_x at the tile's inputs from the frame's own outputs, and
//  the tile's grad_h partial, row (bank * Kmax + b) * Lmax + l of partial[item].
// Workgroups take work with an atomic ticket (*ticket zero at launch).
// The grad_x kernel also computes each frame's halo gradient into hg
// ([n_frames][Lmax-1], as the vector halo kernel does).
// With sfirst (first frame of each stream, 0xffffffff for none), the grad_x
// kernel also zeroes, after its items, the samples of grad_x that lie
// outside every frame (before a stream's first frame, between frames, after
// its last, or the whole stream when it has none).
void launch_bwd_gu_mfma(const prune_fb_desc &d, const BwdFrame *bf, const WorkItem *items,
                        const uint32_t *n_items, unsigned int *ticket, float2 *hg, uint32_t grid,
                        const uint32_t *sfirst, float2 *gx, hipStream_t s);
void launch_bwd_gh_mfma(const prune_fb_desc &d, const BwdFrame *bf, const WorkItem *items,
                        const uint32_t *n_items, unsigned int *ticket, float2 *partial,
                        uint32_t max_items, uint32_t grid, hipStream_t s);
// Tile (positions per work item) of the plain-product form for this shape:
// 512 for the one-wave kernel of small shapes (at most 8 powers, at most 16
// taps), kBT otherwise.  The preparation kernel cuts frames into these tiles.
uint32_t bwd_gemm_tile(const prune_fb_desc &d);
// Both gradients as plain matrix products in one pass over each tile
// (fb_bwd_gemm.hip): grad_x at the tile's inputs (a null gx skips it; the
// halo rows go to hg and the samples outside every frame are zeroed), and
// the tile's grad_h partial row (a null partial skips it).  The block kernel
// takes runs of tiles with the atomic ticket over every resident workgroup
// slot of ncu CUs; the one-wave kernel (small shapes) assigns its tiles
// statically to every resident wave and leaves the ticket alone.  max_items
// bounds the item count in this form's tiles.
void launch_bwd_gemm(const prune_fb_desc &d, const BwdFrame *bf, const WorkItem *items,
                     const uint32_t *n_items, unsigned int *ticket, float2 *hg, float2 *partial,
                     uint32_t max_items, uint32_t ncu, const uint32_t *sfirst, float2 *gx, hipStream_t s);

}  // namespace prune
