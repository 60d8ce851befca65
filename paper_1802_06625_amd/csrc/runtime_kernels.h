// Kernel-side argument blocks and launchers shared by the host runtime and
// the kernel translation units.
#pragma once

#include <string>

#include "prune_internal.h"

namespace prune {

struct SrcIn {             // one queued source frame
  uint32_t count, pad;
  const void *ptr;         // copy-in source, or null when written in place
};

// Pixel operations of the Motion Detection actors, carried by copy items.
enum : uint32_t { kOpCopy = 0, kOpGauss5 = 1, kOpThres = 2, kOpMed5 = 3 };

struct CopyItem {          // dst = halo (halo_count samples), then sum of sources
  const float2 *src[kMaxIn];
  float2 *dst;
  const float2 *halo;
  uint32_t n_src, halo_count, count, pad;   // pad: POLY basis power
  uint32_t op, width, param, n_dst;         // pixel items: op, frame width, threshold and
                                            // destinations (dst, then src[2..]); count =
                                            // pixels; src[0..1] and the outputs are byte frames
};

struct GatherReq {         // fill dst[0..H) with the H stream samples before firing i
  uint32_t actor, i;
  float2 *dst;
};

struct CtrlArgs {
  FifoDev *fifos;
  PortDev *ports;
  ActorDev *actors;
  FbParamsDev *fbs;
  const uint32_t *comp_off;      // [n_comp + 1]
  const uint32_t *comp_actors;   // actors of each component in topological order
  uint32_t B, Bcap, tile, clear_n;
  uint32_t per_firing, n_fifos;
  FiringRec *recs;               // [n_actors][Bcap]
  uint32_t *wrote;               // [n_fifos][Bcap] tokens written per iteration
  FbFrameDesc *fb_desc;
  const uint32_t *desc_off;      // per actor
  WorkItem *fb_items;
  const uint32_t *fb_item_off;   // per level
  uint32_t *fb_count;            // per level
  CopyItem *copy_items;
  const uint32_t *copy_item_off; // per level
  uint32_t *copy_count;          // per level
  const uint32_t *level_of;      // per actor
  float2 *halo_scratch;
  const uint32_t *halo_off;      // per actor
  GatherReq *gather_items;
  const uint32_t *gather_off;    // per level
  uint32_t *gather_count;        // per level
  uint32_t *err;
  uint32_t *clear_ptr;           // zeroed by block 0 first when clear_n > 0 (single block)
  TraceBuf trace;
};

// Parallel bookkeeping of a batch (three phases): decode per (component,
// iteration), scans per component, emission per (component, iteration).
constexpr int kMaxCompFifos = 24;

struct AccDev {            // one (port, fifo) data access of an actor, in port order
  uint32_t port, fifo, dir, slot;   // slot: ordinal among the actor's inputs or outputs
  uint32_t first;                   // first FIFO of its port
  uint32_t drp;                     // DRP ordinal of its port, kNone otherwise
  uint32_t local;                   // FIFO slot within the component (< kMaxCompFifos)
  uint32_t pad;
};

struct BatchArgs {
  const uint32_t *acc_off;     // [n_actors + 1]
  const AccDev *acc;
  uint32_t *s_fired, *s_mask, *s_rate, *s_bitmap, *s_firing, *s_aux, *s_auxoff, *s_aux2;
  uint32_t *s_cnt, *s_pre;     // [n_acc][Bcap]
  uint64_t *s_base;            // [n_acc] FIFO index at batch start
  uint64_t *s_qbase;           // [n_actors] queue head / control-FIFO read index at batch start
  uint64_t *s_sink;            // [n_actors] sink output offset at batch start
  uint64_t *s_rsnap;           // [n_fifos] tokens read before the batch
  const uint32_t *fifo_wacc;   // [n_fifos] index of the FIFO's writer access
  uint32_t max_acc;            // most accesses of any actor (scan grid)
};

void launch_batch(const CtrlArgs &c, const BatchArgs &b, uint32_t n_comp, uint32_t n_actors,
                  hipStream_t s);
void launch_control(const CtrlArgs &c, uint32_t n_comp, hipStream_t s);
// Copy-kernel launch for one level: grid_x item slots, element chunks for
// copies of up to max_total 8-byte words, row chunks for pixel frames of up
// to pix_rows rows.
void launch_copy(const CopyItem *items, const uint32_t *n_items, uint32_t grid_x,
                 uint32_t max_total, uint32_t pix_rows, hipStream_t s);
void launch_post(const CtrlArgs &c, const uint32_t *actors, uint32_t n, hipStream_t s);
void launch_gather(const CtrlArgs &c, uint32_t level, uint32_t grid, hipStream_t s);
void launch_clear(uint32_t *p, uint32_t n, hipStream_t s);
void launch_copyback(const CtrlArgs &c, uint32_t a, uint32_t fifo, uint32_t k, hipStream_t s);

template <int NT, int NW>
void launch_fb_mfma(const FbFrameDesc *f, const WorkItem *it, const uint32_t *n,
                    unsigned int *ticket, uint32_t grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
int fb_variant_count();
const char *fb_variant_name(int v);
int fb_variant_tile(int v);
int fb_variant_wg(int v);
// Workgroups of variant v resident per CU: the persistent grid is this many
// per CU.
int fb_variant_resident(int v);
template <int NT, int NW>
int fb_mfma_resident();
// e0/e1 (may be null): events that receive the kernel's own start and end.
void fb_forward_launch(int v, const FbFrameDesc *frames, const WorkItem *items,
                       const uint32_t *n_items, unsigned int *ticket, uint32_t grid,
                       hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Direct-op helpers.
void launch_direct_prep(const prune_fb_desc &d, const float2 *x, const float2 *taps,
                        const prune_fb_frame *frames, float2 *y, uint32_t tile,
                        FbFrameDesc *desc, WorkItem *items, uint32_t *n_items,
                        unsigned int *ticket, uint32_t *err, hipStream_t s);
// Forward variant for a graph's filter banks (tuned on a synthetic batch of
// the graph's structure, cached per process and in PRUNE_AUTOTUNE_CACHE).
int choose_variant_graph(uint32_t n_banks, const uint32_t *L, uint32_t K, uint32_t n, bool param);
// Persistent autotuning choices (PRUNE_AUTOTUNE_CACHE), keyed by strings
// that name the kernel family, the architecture and the shape class.
std::string tune_arch();
bool tune_cache_lookup(const std::string &key, std::string *choice);
void tune_cache_store(const std::string &key, const char *choice, double ms);
void tune_cache_counts(uint32_t *runs, uint32_t *hits);
// Per-thread kernel timing (prune_timing_enable / prune_last_fb_kernel_ms).
bool timing_on();
void timing_restart();
void timing_push(hipEvent_t e0, hipEvent_t e1);
int forced_variant();
// Text returned by prune_last_error on this thread.
void set_last_error(const char *msg);

}  // namespace prune
