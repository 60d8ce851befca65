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

// Matrix-core adjoint over the same work items (one tile of kBT samples of
// one frame each) as the vector kernel:
//  grad_x at the tile's inputs from the frame's own outputs, and
//  the tile's grad_h partial, row (bank * Kmax + b) * Lmax + l of partial[item].
// Workgroups take work with an atomic ticket (*ticket zero at launch).
// The grad_x kernel also computes each frame's halo gradient into hg
// ([n_frames][Lmax-1], as the vector halo kernel does).
void launch_bwd_gu_mfma(const prune_fb_desc &d, const BwdFrame *bf, const WorkItem *items,
                        const uint32_t *n_items, unsigned int *ticket, float2 *hg, uint32_t grid,
                        hipStream_t s);
void launch_bwd_gh_mfma(const prune_fb_desc &d, const BwdFrame *bf, const WorkItem *items,
                        const uint32_t *n_items, unsigned int *ticket, float2 *partial,
                        uint32_t max_items, uint32_t grid, hipStream_t s);

}  // namespace prune
