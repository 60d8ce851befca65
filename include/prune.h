/*
 * prune.h -- C ABI of libprune_hip: PRUNE dynamic dataflow graphs whose
 * signal-processing actors fire on an AMD Instinct MI355X (gfx950).
 *
 * Model of computation (Sec. III of Boutellier et al., "PRUNE: Dynamic and
 * Decidable Dataflow for Signal Processing on Heterogeneous Platforms"):
 * an application is a graph G = (A, F) of actors and FIFOs.  Ports are
 * control input ports (rate 1), static regular ports (SRP, one fixed rate) or
 * dynamic regular ports (DRP, rate atr or 0).  Each FIFO has one rate
 * (fiforate) that must equal the atr of both its ports, and a delay (initial
 * tokens).  A configuration actor emits control tokens; a dynamic actor
 * consumes one per firing and sets each DRP to atr or 0 per Eq. 1 through the
 * control table.  FIFO capacity is fixed by Eq. 2 with the compile-time
 * constant C (C = 2 double buffer, C = 3 triple buffer); channels with delay
 * follow the access pattern described with Fig. 6.
 *
 * Conventions for every entry point:
 *  - returns PRUNE_OK (0) or a negative prune_status; prune_last_error()
 *    gives a thread-local description of the last failure;
 *  - "device pointer" means memory on the graph's HIP device (for example a
 *    torch CUDA/HIP tensor's data_ptr()); "host pointer" means CPU memory;
 *  - host arrays are copied before the call returns; device buffers passed
 *    to *_bind_* calls are borrowed and must outlive the graph; buffers passed
 *    as sources of copies may be reused once the stream has passed the call;
 *  - all calls on one graph come from one host thread; device work is
 *    enqueued on the given hipStream_t (0 = the null stream) and asynchronous
 *    device errors surface at prune_graph_sync();
 *  - complex samples are complex64: interleaved (re, im) float32 pairs.
 */
#ifndef PRUNE_H
#define PRUNE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct prune_graph *prune_graph_t;
typedef int32_t prune_status;
typedef uint32_t prune_id;
typedef void *prune_stream_t; /* a hipStream_t */

/* ---- status codes ------------------------------------------------------ */
enum {
  PRUNE_OK = 0,
  PRUNE_E_ARG = -1,           /* bad argument or id                           */
  PRUNE_E_STATE = -2,         /* call not allowed in this state (e.g. edit
                                 after finalize, fire before finalize)        */
  PRUNE_E_RATE_MISMATCH = -3, /* atr(p) != fiforate(fifo(p)) (Sec. III-A), or
                                 an actor's rate relation does not hold       */
  PRUNE_E_PORT_KIND = -4,     /* control port rate != 1, control output port
                                 not an SRP of rate 1 feeding control ports,
                                 DRP on a static actor, dynamic actor without
                                 exactly one control port, DRP not controlled
                                 by the port feeding its actor (Sec. III-B/C) */
  PRUNE_E_RULE4 = -5,         /* dynamic inputs and outputs on one actor
                                 (single-sided dynamism rule, Sec. IV)        */
  PRUNE_E_CONNECT = -6,       /* input port without exactly one FIFO, output
                                 port without a FIFO, wrong direction         */
  PRUNE_E_DELAY = -7,         /* delay that the Eq. 2 buffer cannot hold     */
  PRUNE_E_TOKEN = -8,         /* control value with elements beyond its
                                 declared size, rate outside 1..atr, block
                                 count differing from the firing's rate      */
  PRUNE_E_DEADLOCK = -9,      /* stopped by a cycle of waits (Sec. III-A, V) */
  PRUNE_E_CAPACITY = -10,     /* bound storage smaller than Eq. 2's capacity */
  PRUNE_E_HIP = -11,          /* HIP runtime error (text in last_error)      */
  PRUNE_E_UNSUPPORTED = -12,  /* shape beyond the kernels' limits            */
  PRUNE_E_RULE = -13          /* design rule or DPG validity violated, or a
                                 dynamic component that deadlocks (only with
                                 PRUNE_CHECK_RULES, see prune_graph_analyze) */
};

enum { PRUNE_IN = 0, PRUNE_OUT = 1 };
enum { PRUNE_SRP = 0, PRUNE_DRP = 1, PRUNE_CPORT = 2 };

/* Port flags.  PRUNE_PORT_PARAM: the port moves the firing's rate parameter
 * (carried by the control token, or the frame length for a source) plus the
 * port's halo instead of its atr; atr is then the maximum.  With the
 * parameter equal to atr this is Eq. 1 unchanged. */
enum { PRUNE_PORT_PARAM = 1u };

/* Actor kinds.
 *  SOURCE      one output port; frames arrive through prune_source_push.
 *  CONFIG      configuration actor: control output ports (SRP, rate 1) that
 *              broadcast one control token per firing, computed from
 *              external side-information (prune_config_push).
 *  FILTERBANK  the merged dynamic processing graph of the DPD application
 *              (poly -> FIR_b -> add, Sec. VII-A): one data input, one data
 *              output, an optional control port.  Branch d is the DC whose
 *              DRPs are addressed by prune_filterbank_branch(); it computes
 *              sum_l h_d[l] |x[n-l]|^p x[n-l], p = d mod Kmax.
 *  SWITCH      dynamic actor x: one SRP input, DRP outputs; an active output
 *              port receives the frame preceded by `halo` past samples.
 *  SELECT      dynamic actor y: DRP inputs, one SRP output = sum of active
 *              inputs (the active input for one-hot control values).
 *  PASSTHROUGH static copy actor.
 *  SINK        one input port.
 *  POLY        dynamic actor x of the unfused DPD graph (Sec. VII-A, Fig. 8):
 *              a SWITCH whose k-th output port (creation order, k = 0..)
 *              carries the basis u_{k+1} = |x|^k x of the window (halo
 *              included), so output k feeds the FIR of branch k+1.
 *  GAUSS5, THRES, MED5  the static actors of the Motion Detection graph
 *              (Sec. VII-A, Fig. 7) on 8-bit frames (prune_pixel_params; a
 *              frame is W*H one-byte tokens, token_bytes 1, one frame per
 *              firing):
 *                GAUSS5 out = (sum_{dy,dx} w_dy w_dx in[y+dy][x+dx] + 128) >> 8
 *                       with w = (1 4 6 4 1), rows 2..H-3 (the two rows at
 *                       each end are copied), columns clamped at the edges;
 *                THRES  two inputs (current, previous frame): 255 where
 *                       |cur - prev| > threshold, else 0;
 *                MED5   median of the pixel and its up, down, left and right
 *                       neighbours, rows 1..H-2 (rows 0 and H-1 copied),
 *                       columns clamped.
 *              The previous frame reaches THRES through a FIFO with a delay
 *              of W*H tokens (one frame of zeros).  SOURCE and SINK carry
 *              such frames with token_bytes 1 (W*H a multiple of 8).
 * Limits: at most PRUNE_MAX_PORTS ports per actor, PRUNE_MAX_IN data
 * inputs, PRUNE_MAX_IO output FIFO accesses per firing. */
enum {
  PRUNE_SOURCE = 0,
  PRUNE_CONFIG = 1,
  PRUNE_FILTERBANK = 2,
  PRUNE_SWITCH = 3,
  PRUNE_SELECT = 4,
  PRUNE_PASSTHROUGH = 5,
  PRUNE_SINK = 6,
  PRUNE_POLY = 7,
  PRUNE_GAUSS5 = 8,
  PRUNE_THRES = 9,
  PRUNE_MED5 = 10
};
enum { PRUNE_MAX_PORTS = 14, PRUNE_MAX_IN = 10, PRUNE_MAX_IO = 12 };

/* Execution modes of prune_graph_fire. */
enum {
  PRUNE_PER_FIRING = 0,    /* one launch sequence per actor firing, in
                              round-robin actor order (the runtime model of
                              Sec. VI-C, one firing at a time)            */
  PRUNE_BATCHED = 1,       /* all firings of B graph iterations in a fixed
                              launch sequence with one persistent
                              filter-bank launch                          */
  PRUNE_BATCHED_GRAPH = 2  /* BATCHED, captured once per batch size as a
                              hipGraph and replayed                       */
};

/* Configuration actor modes (how side-information becomes a control value). */
enum {
  PRUNE_CONFIG_PREFIX = 0, /* mask = ((1 << K) - 1) << (bank * Kmax)        */
  PRUNE_CONFIG_ROUTE = 1,  /* mask = 1 << route (one-hot DC selection)     */
  PRUNE_CONFIG_MASK = 2    /* mask = (K & ((1 << Kmax) - 1)) << (bank * Kmax):
                              K carries any set of the bank's branches
                              (bit b-1 = branch b), not only a prefix      */
};

/* Control token (8 bytes): the control value v (bit e-1 = element e) and
 * the rate parameter of the firing. */
typedef struct {
  uint32_t mask;
  uint32_t rate;
} prune_ctrl_token;

/* External side-information of one configuration-actor firing. */
typedef struct {
  uint32_t K;     /* active branches (prefix mode)                          */
  uint32_t n;     /* frame length = rate parameter of the token             */
  uint32_t bank;  /* tap bank (prefix mode)                                 */
  uint32_t route; /* DC index (route mode)                                  */
} prune_side_info;

typedef struct {
  uint32_t mode;       /* PRUNE_CONFIG_PREFIX or PRUNE_CONFIG_ROUTE         */
  uint32_t Kmax;       /* branches per bank (prefix mode)                    */
  uint32_t n_elements; /* |v|: number of elements of the control value      */
} prune_config_params;

typedef struct {
  uint32_t W, H;        /* frame width and height in pixels (W*H = the rate)  */
  uint32_t threshold;   /* THRES: difference threshold (the paper's constant) */
} prune_pixel_params;

#define PRUNE_MAX_BANKS 4
#define PRUNE_MAX_BRANCHES 32 /* n_banks * Kmax <= 32 (one mask word)     */
#define PRUNE_MAX_L 64        /* taps per branch                           */

typedef struct {
  uint32_t n_banks;               /* 1..PRUNE_MAX_BANKS                     */
  uint32_t Kmax;                  /* branches per bank, 1..10               */
  uint32_t L[PRUNE_MAX_BANKS];    /* taps per branch of each bank, 1..64    */
  uint32_t windowed;              /* 0: stateful -- the actor keeps the
                                     last Lmax-1 input samples of its stream;
                                     1: stateless -- each input block holds
                                     Lmax-1 past samples, then the frame    */
  uint32_t fixed_mask;            /* branch mask used when the actor has no
                                     control port                          */
} prune_fb_params;

typedef struct {
  uint64_t writes, reads;                 /* firings that wrote / read     */
  uint64_t tokens_written, tokens_read;   /* tokens moved (delays excluded) */
  uint64_t max_occ;                       /* largest occupancy seen (tokens,
                                             delays included; depends on
                                             the schedule)                   */
  uint64_t capacity;                      /* Eq. 2 in tokens               */
} prune_fifo_stats;

/* Per-firing trace records (prune_trace_fetch), 8 x uint32 each.
 *  type 0 = FIFO access: a = fifo, b = op (0 write, 1 read), c = firing
 *           number of the accessing actor, d = write/read index, e = first
 *           slot, f = token count;
 *  type 1 = control decode of a dynamic actor: a = actor, c = firing,
 *           d = control value (mask), e = rate parameter, f = bitmap of
 *           DRPs set to atr (bit i = i-th DRP of the actor). */
typedef struct {
  uint32_t type, a, b, c, d, e, f, pad;
} prune_trace_record;

/* ---- graph construction (Sec. III-A/B) --------------------------------- */

/* Create an empty graph on HIP device `hip_device`.  *out receives the
 * handle.  E_HIP if the device cannot be selected.  hip_device = -1 creates
 * a host-only graph: construction, validation and Eq. 2 sizing work, device
 * calls (binding, pushing, firing) return E_STATE. */
prune_status prune_graph_create(int hip_device, prune_graph_t *out);

/* Free the graph's library-owned memory (metadata, taps, histories, work
 * lists).  Borrowed FIFO storage is not freed.  Waits for the device. */
prune_status prune_graph_destroy(prune_graph_t g);

/* Add an actor.  params: prune_config_params for CONFIG, prune_fb_params for
 * FILTERBANK, NULL for the other kinds; params_bytes its size.  *actor
 * receives the id.  E_ARG on unknown kinds or parameters out of range,
 * E_UNSUPPORTED beyond PRUNE_MAX_* limits, E_STATE after finalize. */
prune_status prune_actor_create(prune_graph_t g, int kind, const void *params,
                                size_t params_bytes, prune_id *actor);

/* Add a port to `actor`: dir PRUNE_IN/OUT, kind PRUNE_SRP/DRP/CPORT, active
 * token rate atr (> 0), token_bytes (8 for complex64 samples and control
 * tokens), flags (PRUNE_PORT_PARAM) and halo (extra past samples carried by
 * a window port, Sec. VII-A DPD windows).  *port receives the id. */
prune_status prune_port_create(prune_graph_t g, prune_id actor, int dir, int kind,
                               uint32_t atr, uint32_t token_bytes, uint32_t flags,
                               uint32_t halo, prune_id *port);

/* Id of branch d (0-based, d < n_banks*Kmax) of a filter bank: the DRP pair
 * of its DC d, addressable in the control table. */
prune_status prune_filterbank_branch(prune_graph_t g, prune_id fb, uint32_t d, prune_id *drp);

/* Connect output port src to input port dst with rate fiforate and `delay`
 * initial tokens (zeros).  *fifo receives the id.  E_CONNECT on wrong
 * directions or an input that already has its FIFO. */
prune_status prune_fifo_connect(prune_graph_t g, prune_id src_port, prune_id dst_port,
                                uint32_t fiforate, uint32_t delay, prune_id *fifo);

/* Control table entry T[ctrl_port][drp] = element (1-based element of the
 * control value; 0 = not controlled), Sec. III-C. */
prune_status prune_control_table_set(prune_graph_t g, prune_id ctrl_port, prune_id drp,
                                     uint32_t element);

/* Validate the graph (Sec. III local rules, rule 4 of Sec. IV, the actor
 * kinds' rate relations) and size every FIFO by Eq. 2 with constant C.
 * Allocates library-owned device state (counters, control FIFOs, histories,
 * taps, work lists).  Errors as listed with the status codes; E_UNSUPPORTED
 * for more than 65535 actors. */
prune_status prune_graph_finalize(prune_graph_t g, uint32_t C);

/* ---- compile-time analysis (Sec. IV design rules, Sec. V) --------------- */

/* Checks that finalize runs.  PRUNE_CHECK_RULES: prune_graph_finalize runs
 * prune_graph_analyze first and fails with E_RULE (the first violation in
 * prune_last_error) if the analysis reports any violation.  Default: off,
 * finalize applies the local checks only. */
enum { PRUNE_CHECK_RULES = 1u };
prune_status prune_graph_set_checks(prune_graph_t g, uint32_t flags);

/* Violation codes of the analysis, with the meaning of the two subjects
 * (a, b) of each record; -1 where unused.
 *  RULE1      (1)  linked DRPs not controlled by one control output port
 *                  and one element, T[p_q][p_x] = T[p_q][p_y] > 0 (Sec. IV,
 *                  linked port control rule); a, b: the two DRP ports.
 *  RULE2      (2)  one control output port reaches two dynamic actors
 *                  through FIFOs of different delay (balanced delay rule);
 *                  a: the lowest-id actor controlled by the port, b: the
 *                  other actor.
 *  RULE3_KIND (31) an actor on a connecting subchain is not a static
 *                  processing actor (connecting subchain rule, part 1); a.
 *  RULE3_SHARED (32) an actor lies on connecting subchains of two different
 *                  dynamic-actor pairs (part 2); a.
 *  RULE4      (4)  an actor with input and output DRPs (single-sided
 *                  dynamism); a.
 *  RULE5      (5)  an actor b next to a subchain through an SRP of b lies on
 *                  no chain connecting the pair (encapsulation rule); a = b.
 *  DPG_A      (10) a DC not attached to a DRP of both x and y (Sec. V,
 *                  validity a); a: DPG index, b: DC index.
 *  DPG_B_DC   (11) the DRPs attached to one DC use more than one element of
 *                  the control value (validity b); a: DPG, b: DC.
 *  DPG_B_COUNT (12) two DCs share an element, or the DRPs of x and y use a
 *                  number of elements other than the DC count M; a: DPG.
 *  DPG_C      (13) a FIFO with one end in a DC and the other not on a DRP of
 *                  x or y (a DC is entered and left only through the DPG's
 *                  DRPs); a: DPG, b: FIFO.
 *  DEADLOCK_DC (20) the periodic schedule of a DC cannot complete (Sec. V:
 *                  the DC, an SDF graph, is not consistent); a: DPG, b: DC.
 *  DEADLOCK_TOP (21) the actors outside every DC cannot complete one
 *                  period.
 *  PAIRING    (40) a dynamic actor is linked to more than one partner; a.
 *  UNPAIRED   (41) a dynamic actor belongs to no DPG; a. */
enum {
  PRUNE_RULE1 = 1, PRUNE_RULE2 = 2, PRUNE_RULE4 = 4, PRUNE_RULE5 = 5,
  PRUNE_DPG_A = 10, PRUNE_DPG_B_DC = 11, PRUNE_DPG_B_COUNT = 12, PRUNE_DPG_C = 13,
  PRUNE_DEADLOCK_DC = 20, PRUNE_DEADLOCK_TOP = 21,
  PRUNE_RULE3_KIND = 31, PRUNE_RULE3_SHARED = 32,
  PRUNE_PAIRING = 40, PRUNE_UNPAIRED = 41
};

typedef struct {
  uint32_t n_linked;       /* linked DRP pairs                                */
  uint32_t n_dpgs;         /* dynamic processing graphs                       */
  uint32_t n_dcs;          /* dynamic components over all DPGs (M per DPG)    */
  uint32_t n_violations;   /* 0 for a graph that passes every check           */
} prune_analysis_counts;

/* Analyse the graph as built so far (finalized or not; host-only graphs
 * included; nothing runs on a device) and keep the report in the graph
 * until the next call.  Adjacency and chains use data FIFOs (FIFOs into
 * control ports are left out).  A dynamic actor is one with an external
 * DRP: a filter bank, whose branch DRPs are internal, counts as a static
 * processing actor here.  Each DPG is (q, x, y) with x the actor with
 * output DRPs and y the actor with input DRPs of linked DRPs; its DCs are
 * the components left after removing q, x and y (Sec. V procedure), plus
 * one dummy DC per FIFO from a DRP of x to a DRP of y.  Each DC is scheduled
 * once (x, its actors in increasing id, y, always the first fireable one;
 * all repetition counts are one because a FIFO has one rate at both ends),
 * which decides its deadlock freedom and gives the buffer bound beta(f) of
 * each of its FIFOs: the largest token count over the initial state and the
 * state after each firing.  The actors outside every DC and the FIFOs among
 * them, control FIFOs included, are scheduled the same way in id order.
 * counts may be NULL. */
prune_status prune_graph_analyze(prune_graph_t g, prune_analysis_counts *counts);

/* Tables of the last analysis, as int64 values (-1 = none):
 *  PRUNE_AN_LINKED      2 per linked DRP pair: (p, p2), p < p2, sorted.
 *  PRUNE_AN_DPGS        4 per DPG: (q, x, y, control output port of x), in
 *                       increasing (x, y).
 *  PRUNE_AN_DCS         4 per DC: (DPG index, control-value element (1-based;
 *                       -1 if its DRPs disagree), FIFO of a dummy DC or -1,
 *                       number of actors), DCs of a DPG in increasing
 *                       smallest actor id, dummy DCs last in FIFO order.
 *  PRUNE_AN_DC_ACTORS   the actors of every DC in DC order, each DC's sorted.
 *  PRUNE_AN_ACTOR_DC    1 per actor: index of its DC, or -1.
 *  PRUNE_AN_BETA        1 per FIFO: its buffer bound, or -1 where a schedule
 *                       deadlocks or the FIFO joins a DC to an actor that is
 *                       not x or y.
 *  PRUNE_AN_VIOLATIONS  3 per violation: (code, a, b), sorted, unique.
 * *n receives the number of values of the table; min(cap, *n) are copied to
 * out (out may be NULL when cap is 0).  E_STATE before any analysis. */
enum {
  PRUNE_AN_LINKED = 0, PRUNE_AN_DPGS = 1, PRUNE_AN_DCS = 2, PRUNE_AN_DC_ACTORS = 3,
  PRUNE_AN_ACTOR_DC = 4, PRUNE_AN_BETA = 5, PRUNE_AN_VIOLATIONS = 6
};
prune_status prune_graph_analysis_table(prune_graph_t g, int table, int64_t *out, size_t cap,
                                        size_t *n);

/* Bytes of storage FIFO `fifo` needs: B * Gamma_f of Eq. 2. */
prune_status prune_fifo_required_bytes(prune_graph_t g, prune_id fifo, size_t *bytes);

/* Bind caller-owned device storage (borrowed) to a data FIFO.  Control FIFOs
 * are library-owned.  E_CAPACITY if bytes < prune_fifo_required_bytes. */
prune_status prune_fifo_bind_storage(prune_graph_t g, prune_id fifo, void *dev_ptr,
                                     size_t bytes);

/* Device address of the first slot of the k-th next write of `fifo` (for
 * writing frames in place, the fifoWriteStart window of Sec. VI). */
prune_status prune_fifo_write_window(prune_graph_t g, prune_id fifo, uint32_t k,
                                     void **dev_ptr);

/* Copy n_complex complex64 taps from device pointer dev_taps, laid out
 * [n_banks][Kmax][Lmax] (Lmax = largest L; entries beyond a bank's L
 * ignored), into the filter bank's library-owned tap buffer. */
prune_status prune_filterbank_set_taps(prune_graph_t g, prune_id fb, const void *dev_taps,
                                       size_t n_complex, prune_stream_t stream);

/* Zero the stream history of a stateful filter bank or a switch. */
prune_status prune_actor_reset_history(prune_graph_t g, prune_id actor, prune_stream_t stream);

/* ---- external input / output -------------------------------------------- */

/* Host actors beside device firings (the paper's heterogeneous execution,
 * Sec. VI-C, with a source and sink on the CPU): stream n_frames frames
 * from host memory through the graph and back, in batches of `batch`
 * iterations, with three stages in flight at once:
 *  - the frames of batch k+1 are copied from host_in into the source FIFO
 *    (in place, on a copy stream of the library's),
 *  - batch k fires (PRUNE_BATCHED on `stream`),
 *  - the outputs of batch k-1 are copied from the sink's input FIFO to
 *    host_out (on a second copy stream),
 * ordered by events: a batch's frames go into ring blocks only after the
 * batch that last read them has fired, and a batch fires only after the
 * output blocks it overwrites have been copied out.  The result equals
 * pushing every frame, firing and reading the sink.
 * host_in: n_frames x atr tokens of the source FIFO, back to back; side:
 * n_frames side-information records for `cfg`; host_out: n_frames x atr
 * tokens of the sink's FIFO.  Pinned host memory (hipHostMalloc, torch
 * pin_memory) lets the copies run concurrently with the firing; pageable
 * memory works but serialises them.  Requirements: fixed-rate source and
 * sink FIFOs without delay, the graph's C a multiple of `batch` holding at
 * least two batches, no sink output bound, no pending source or side input.
 * Returns when every output is on the host. */
prune_status prune_graph_stream_host(prune_graph_t g, prune_id src, prune_id cfg, prune_id snk,
                                     const void *host_in, const prune_side_info *side, void *host_out,
                                     uint32_t n_frames, uint32_t batch, prune_stream_t stream);

/* Queue n_frames firings of source `src`.  host_counts[f] = tokens of frame
 * f (equal to atr for an SRP, 1..atr for a PRUNE_PORT_PARAM port).
 * dev_samples: device pointer to the frames back to back (copied into the
 * FIFO when the source fires; must stay valid until then), or NULL when the
 * caller has already written frame f at prune_fifo_write_window(f).
 * Queued entries live in a device ring; a push that would overwrite entries
 * the device may not have read yet (fire calls return before the device
 * runs them) synchronizes the device first. */
prune_status prune_source_push(prune_graph_t g, prune_id src, const void *dev_samples,
                               const uint32_t *host_counts, uint32_t n_frames);

/* Queue n_frames firings of configuration actor `cfg` with host side-info
 * (same ring rule as prune_source_push).  E_TOKEN, with nothing queued, for
 * a record whose branches lie beyond the bank: K > Kmax in prefix mode, a
 * branch set with bits at or above Kmax in mask mode. */
prune_status prune_config_push(prune_graph_t g, prune_id cfg, const prune_side_info *host_side,
                               uint32_t n_frames, prune_stream_t stream);

/* Optional: every firing of sink `snk` copies its tokens to dev_out at the
 * running token offset (cap_tokens tokens available).  Without a bound
 * output the tokens stay in the FIFO storage.  Synchronizes the device
 * first: batches in flight read the binding. */
prune_status prune_sink_bind_output(prune_graph_t g, prune_id snk, void *dev_out,
                                    uint64_t cap_tokens);

/* ---- execution (Sec. VI-A actor functions, Sec. VI-C concurrency) -------- */

/* Fire the graph.  PER_FIRING: round-robin sweeps over actors in creation
 * order, each fireable actor firing at most once per sweep, until nothing
 * can fire or max_firings (0 = unlimited) firings were issued.  BATCHED /
 * BATCHED_GRAPH: graph iterations (one firing of every actor that is active
 * in the iteration) in batches as large as the pending input, the FIFO
 * capacities and max_firings (read as a cap on iterations per batch, 0 =
 * none) allow.  *fired (may be NULL) receives firings (PER_FIRING) or
 * iterations (BATCHED).  When PER_FIRING stops because nothing can fire, the
 * stop is classified by what each actor waits for (blocking reads and
 * writes, Sec. III-A): PRUNE_OK when every actor that cannot fire waits,
 * through the FIFOs it blocks on, on a source or configuration actor whose
 * pushed input is used up (more input may be pushed and fired later);
 * E_DEADLOCK when some actor's waits only lead round a cycle, or when a
 * dynamic actor waits on data that its linked partner's firing of the same
 * control-token index did not send (linked DRPs set differently, Sec. V).
 * The firings issued before the stop stay queued on `stream` either way.
 * E_UNSUPPORTED for batched mode on graphs with cycles or delays that are
 * not whole blocks. */
prune_status prune_graph_fire(prune_graph_t g, int mode, uint32_t max_firings,
                              prune_stream_t stream, uint64_t *fired);

/* Wait for `stream` and check the device error word (rates beyond atr,
 * control values beyond their size, block counts that differ from the
 * firing's rate).  Returns the first device-detected error. */
prune_status prune_graph_sync(prune_graph_t g, prune_stream_t stream);

/* Counters of a FIFO (synchronises the device). */
prune_status prune_fifo_get_stats(prune_graph_t g, prune_id fifo, prune_fifo_stats *out);

/* Per-branch counters of a filter bank: active firings and tokens of branch
 * d for d < n (synchronises). */
prune_status prune_filterbank_branch_stats(prune_graph_t g, prune_id fb, uint64_t *firings,
                                           uint64_t *tokens, uint32_t n);

/* Firings of an actor so far (host count). */
prune_status prune_actor_firings(prune_graph_t g, prune_id actor, uint64_t *firings);

/* Start recording per-firing trace records into a library-owned device
 * buffer of max_records entries (0 disables tracing and frees it). */
prune_status prune_trace_enable(prune_graph_t g, size_t max_records);

/* Copy the trace to host_buf (capacity `bytes`); *used receives the bytes
 * written.  E_CAPACITY if the device buffer overflowed. Synchronises. */
prune_status prune_trace_fetch(prune_graph_t g, void *host_buf, size_t bytes, size_t *used);

/* ---- direct filter-bank operations (same kernels as the graph path) ------ */

/* A batch of frames cut from S streams of N samples each.
 * frames: device array of n_frames prune_fb_frame, grouped by stream and in
 * stream order inside a stream; the frames of a stream tile [0, N) of it.
 * The Lmax-1 samples before t = 0 of every stream are zero. */
typedef struct {
  uint32_t n_streams;         /* S                                         */
  uint32_t n_frames;
  uint64_t stream_len;        /* N                                         */
  uint32_t n_banks, Kmax;
  uint32_t L[PRUNE_MAX_BANKS];
  uint32_t max_frame_len;     /* largest n of any frame                    */
  uint32_t reserved;
} prune_fb_desc;

typedef struct {
  uint32_t stream;  /* which stream and which tap set                      */
  uint32_t t0;      /* first sample of the frame within its stream         */
  uint32_t n;       /* samples                                             */
  uint32_t mask;    /* bit d: branch d active                              */
  uint32_t route;   /* 0: filter bank, 1: passthrough (y = x)              */
  uint32_t pad[3];
} prune_fb_frame;

/* y = filter bank of x (the forward of the merged DPG over whole streams,
 * including passthrough-routed frames).  x, y: device [S][N] complex64;
 * taps: device [S][n_banks][Kmax][Lmax] complex64; frames: device array.
 * Frames are sorted by stream, then by t0, and the frames of a stream do not
 * overlap; samples of y outside every frame are not written.  A frame whose
 * stream, extent or length is out of range is skipped (nothing of it is
 * written); prune_fb_check_frames reports such frames.
 * E_UNSUPPORTED beyond the limits, E_ARG on inconsistent descriptors. */
prune_status prune_fb_forward(const prune_fb_desc *desc, const void *x, const void *taps,
                              const void *frames, void *y, prune_stream_t stream);

/* prune_fb_forward without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result and errors as
 * prune_fb_forward.  Its frame descriptors and work list live in a fixed
 * device array of the library (about 2.9 MB per device, held until the
 * process ends) instead of library-allocated memory, so:
 *  - n_frames <= PRUNE_NOALLOC_MAX_FRAMES and n_frames * ceil(max_frame_len
 *    / tile) <= PRUNE_NOALLOC_MAX_ITEMS (tile: 1024 to 4096 outputs by
 *    variant), else E_CAPACITY (text in prune_last_error), nothing launched;
 *  - every call on one device uses the same array: calls that overlap in
 *    time on one device (different streams or threads) race and must be
 *    ordered by the caller.  The prep kernel of each call rewrites
 *    everything the forward kernel reads, so nothing carries over.
 * It never runs the autotuner (which allocates a trial batch): the variant
 * is the one set by prune_set_fb_variant, else the one the autotuner has
 * already chosen in this process for the shape class, else variant 1.
 * Launches are not timed (prune_timing_enable). */
#define PRUNE_NOALLOC_MAX_FRAMES 8192
#define PRUNE_NOALLOC_MAX_ITEMS 262144
prune_status prune_fb_forward_noalloc(const prune_fb_desc *desc, const void *x, const void *taps,
                                      const void *frames, void *y, prune_stream_t stream);


/* Validate a device frame table against `desc` (synchronous on `stream`):
 * *n_bad = number of frames with a stream index >= n_streams, t0 + n beyond
 * stream_len, n > max_frame_len, or that break the order (a frame of a lower
 * stream after a higher one, or overlapping / preceding the previous frame of
 * its stream).  The filter-bank operations skip out-of-range frames and
 * assume the order. */
prune_status prune_fb_check_frames(const prune_fb_desc *desc, const void *frames, uint32_t *n_bad,
                                   prune_stream_t stream);

/* Bytes of device workspace prune_fb_backward needs for `desc`. */
prune_status prune_fb_workspace_bytes(const prune_fb_desc *desc, size_t *bytes);

/* Adjoint of prune_fb_forward for a real loss (grad = dL/dRe + i dL/dIm):
 * gx [S][N] and gtaps [S][n_banks][Kmax][Lmax] (entries beyond a bank's L
 * are written as zero) from the cotangent gy [S][N].  The |x|^p basis is
 * recomputed, not stored.  workspace: device buffer of at least
 * prune_fb_workspace_bytes bytes (tile partials and halo gradients).
 * Either gx or gtaps may be NULL to skip that gradient (E_ARG if both are);
 * without gx only the matrix-core grad_h kernel and its reductions run,
 * whichever adjoint form is selected. */
prune_status prune_fb_backward(const prune_fb_desc *desc, const void *x, const void *taps,
                               const void *frames, const void *gy, void *gx, void *gtaps,
                               void *workspace, size_t workspace_bytes, prune_stream_t stream);

/* ---- tuning and diagnostics --------------------------------------------- */

/* Forward kernel variant: 0 = automatic (autotuned, cached), otherwise a
 * fixed variant index (see prune_fb_variant_name). */
prune_status prune_set_fb_variant(int variant);
const char *prune_fb_variant_name(int variant);
int prune_fb_variant_count(void);

/* Run the autotuner now for the given shape class (taps L, branches K,
 * frame length n) on a synthetic batch with a graph's structure (one bank,
 * every frame n samples, prefix masks of a uniform branch count) and report
 * the chosen variant: the one a graph with this filter bank uses.  Uses the
 * device's null stream.
 *
 * Autotuning in general: prune_fb_forward and prune_fb_backward tune on the
 * first call of a shape class (banks and tap counts, Kmax, frame-length
 * class; for the adjoint also whether grad_x is wanted) by timing every
 * variant on that call's own inputs, five alternating rounds of single
 * launches each timed by events, smallest median wins.  Graphs tune at
 * finalize on a synthetic batch of their own structure (banks, rate,
 * variable-rate ports drawing log-uniform frame lengths).  Choices are kept
 * per process and, when the environment variable PRUNE_AUTOTUNE_CACHE names
 * a file, appended to it as JSON lines {"key", "choice", "ms"} and read
 * back by later processes (keys include the device architecture), which
 * then run no tuning launches.  PRUNE_AUTOTUNE=0 disables tuning (variant 1
 * unless the cache file has a choice). */
prune_status prune_autotune_fb(uint32_t L, uint32_t K, uint32_t n, int *variant);

/* Autotuning in this process so far: tuning runs (forward or backward,
 * each one shape class) and choices taken from the PRUNE_AUTOTUNE_CACHE
 * file instead of tuning. */
prune_status prune_autotune_counts(uint32_t *tuning_runs, uint32_t *cache_hits);

/* The forward variant prune_fb_forward uses for desc's shape class: the
 * forced one, else the one tuned in this process, else 0 (not tuned yet). */
prune_status prune_fb_tuned_variant(const prune_fb_desc *desc, int *variant);

/* Backward form: 0 = automatic (autotuned per shape class like the forward,
 * cached per process), 1 = vector kernel (Horner form in r), 2 = matrix-core
 * kernels (block-Toeplitz grad_u and blocked grad_h, Gauss three-product
 * complex arithmetic), 3 = one matrix-core kernel computing both gradients
 * per tile as plain real products (taps of all banks folded per power, the
 * cotangent's Hankel matrix against the taps for grad_x and against the
 * basis planes for grad_h; with at most 8 powers and 16 taps every wave
 * works through its own 512-sample tiles).  All give the same result up to
 * fp32 rounding and the same deterministic float64 reduction of grad_h's
 * tile partials; the workspace size covers every form. */
prune_status prune_set_bwd_variant(int variant);
const char *prune_bwd_variant_name(int variant);
/* Run the backward autotuner now for (L, K, n) on a synthetic batch
 * (uniform frames of n samples, every branch, grad_x wanted) and report
 * the chosen form. */
prune_status prune_autotune_bwd(uint32_t L, uint32_t K, uint32_t n, int *variant);

/* Device-side timing of the filter-bank forward kernel launches made on this
 * thread by prune_graph_fire (stream modes) and prune_fb_forward since
 * timing was last switched on or off: HIP events recorded on the launch
 * stream around each launch, summed (milliseconds) with the launch count.
 * Autotuner launches and launches captured into hipGraphs are not timed. */
prune_status prune_timing_enable(int on);
prune_status prune_last_fb_kernel_ms(float *ms, uint32_t *launches);

/* Batched firing without hipGraph (PRUNE_BATCHED): with on != 0 (the
 * default) a graph's bookkeeping kernels (firing decode, index scans,
 * firing records and work lists) run on a stream the graph owns, ordered by
 * events, so that batch i+1's bookkeeping overlaps batch i's data kernels on
 * the caller's stream.  Two sets of per-batch buffers alternate.  Results
 * are identical either way; the caller's stream still completes after all
 * of a fire call's work.  Process-wide; takes effect at the next batch. */
prune_status prune_set_batch_pipeline(int on);

/* ---- ceiling probes (measurement, not an operation of the paper) --------- */
/* The rooflines the kernels are compared against, measured on the device
 * the library runs on instead of taken from its datasheet.
 *  COPY   float4 grid-stride copy between two device buffers of `size` bytes
 *         each, `waves` (0..32, 0 = 8) 256-thread workgroups per CU;
 *         work = bytes read + written (HBM bandwidth).
 *  FMA32  8 independent chains of unpacked fp32 FMAs per lane, `waves`
 *         waves (1..8) per SIMD, `size` trips of 64 FMAs; work = FMAs.
 *  FMAC32 16 accumulators per lane, acc += a * b with every operand in a
 *         register, `waves` waves per SIMD, `size` trips of 64 FMAs.
 *  FMA3V  8 chains v = v * a + b per lane, every operand in a register
 *         (three-operand encoding), `size` trips of 64 FMAs.
 *  FMAMIX 4 such chains beside 4 accumulators, `size` trips of 64 FMAs.
 *  MFMA32 4 independent 16x16x4 fp32 matrix-core chains per wave, `waves`
 *         waves per SIMD, `size` trips; work = flops (2048 per instruction).
 * One warm-up launch, then `reps` launches timed with HIP events on the
 * null stream.  The clock is the shader clock the launches ran at: core
 * cycles over real-time ticks read by each workgroup at its start and end.
 * The probe allocates and frees its own buffers.  E_ARG for sizes or wave
 * counts out of range, E_HIP when an allocation or launch fails. */
enum { PRUNE_PROBE_COPY = 0, PRUNE_PROBE_FMA32 = 1, PRUNE_PROBE_MFMA32 = 2, PRUNE_PROBE_FMAC32 = 3,
       PRUNE_PROBE_FMA3V = 4, PRUNE_PROBE_FMAMIX = 5 };
typedef struct {
  double seconds;     /* per launch */
  double work;        /* per launch: bytes, FMAs or flops */
  double rate;        /* work per second */
  double clock_ghz;   /* measured shader clock */
  uint32_t grid, block, n_cu, pad;
} prune_probe_result;
prune_status prune_probe_ceiling(int kind, uint32_t waves, uint64_t size, uint32_t reps,
                                 prune_probe_result *out);

/* ---- host evaluation of the integer rules -------------------------------- */
/* The kernels' integer rules compiled for the host from the same source:
 * Eq. 2 capacity (tokens), the first slots of writes and reads 0..n-1 of a
 * FIFO with rate r, delay Q and constant C (Fig. 6 access pattern), and the
 * configuration actor's control token for one side-information record.
 * E_DELAY for delays Eq. 2's buffer cannot hold. */
prune_status prune_rule_capacity(uint32_t r, uint32_t Q, uint32_t C, uint64_t *tokens);
prune_status prune_rule_slots(uint32_t r, uint32_t Q, uint32_t C, uint32_t n,
                              uint64_t *write_slots, uint64_t *read_slots);
prune_status prune_rule_config_token(uint32_t mode, uint32_t Kmax, const prune_side_info *side,
                                     prune_ctrl_token *out);

const char *prune_status_string(prune_status s);
const char *prune_last_error(void);

/* ---- build ----------------------------------------------------------------- */
/* Flags of the loaded library.  PRUNE_BUILD_DEBUG: a PRUNE_DEBUG build, whose
 * bookkeeping kernels check every FIFO after each counter update: the block
 * state is one the blocking rules reach, the token occupancy stays within
 * Eq. 2's capacity (Sec. IV), and no access or token counter goes back.  A
 * failed check makes the next prune_graph_sync return E_RULE. */
#define PRUNE_BUILD_DEBUG 1u
uint32_t prune_build_flags(void);

#ifdef __cplusplus
}
#endif
#endif /* PRUNE_H */
