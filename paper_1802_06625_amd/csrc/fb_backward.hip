// Adjoint of the filter-bank forward (placeholder until the adjoint kernels land).
#include "prune_internal.h"
#include "runtime_kernels.h"

extern "C" {
prune_status prune_fb_workspace_bytes(const prune_fb_desc *desc, size_t *bytes) {
  (void)desc;
  if (bytes) *bytes = 0;
  return PRUNE_E_UNSUPPORTED;
}
prune_status prune_fb_backward(const prune_fb_desc *desc, const void *x, const void *taps,
                               const void *frames, const void *gy, void *gx, void *gtaps,
                               void *workspace, size_t workspace_bytes, prune_stream_t stream) {
  (void)desc; (void)x; (void)taps; (void)frames; (void)gy; (void)gx; (void)gtaps;
  (void)workspace; (void)workspace_bytes; (void)stream;
  return PRUNE_E_UNSUPPORTED;
}
}
