/*
 * vibelsd.h -- C ABI of the MI355X (gfx950) VibeLSD decoder.
 *
 * VibeLSD (arXiv 2508.15743): every syndrome is decoded by an ensemble of L
 * min-sum belief-propagation decoders, each with its own serial-V schedule
 * (a fixed permutation of the columns, Sec. III.D.1 and Appendix A,
 * Algorithm 1).  Once M members have converged the rest are not needed; the
 * converged candidate of least prior weight is taken (Sec. III.D.2).  If no
 * member converges, the members' normalised posteriors are averaged and
 * localised statistics decoding (LSD-0, Sec. III.C) produces the correction.
 *
 * Conventions used by every entry point:
 *   - H is given in CSR form: row c (a detector) lists the columns (error
 *     mechanisms) it touches, strictly ascending.  Lobs (the k logical
 *     observables) likewise.  All host arrays are read during the call only.
 *   - Device pointers are caller-owned (for example allocated by PyTorch) and
 *     must stay valid until the work queued on `stream` has finished.  The
 *     library allocates its own device workspace, cached in the handle.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Decode calls
 *     are asynchronous: argument errors are reported synchronously before
 *     anything is queued, and nothing is written then; HIP launch errors are
 *     reported as VIBE_EHIP.
 *   - Calls on one handle must not overlap in time (they share its
 *     workspace): queue them on one stream, or use one handle per stream.
 *   - Every function returns VIBE_OK (0) or a negative status; the message
 *     of the last error on the calling thread is vibe_last_error().
 *   - Bit-packed vectors: bit j of a vector lives in word j / 64 at bit
 *     position j % 64 (little-endian uint64 words); a shot's vector occupies
 *     ceil(len / 64) words.
 */
#ifndef VIBELSD_H
#define VIBELSD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VIBE_OK 0
#define VIBE_EINVAL (-1)       /* bad argument; nothing was written */
#define VIBE_ENOMEM (-2)       /* a device or host allocation failed */
#define VIBE_EHIP (-3)         /* a HIP runtime call or launch failed */
#define VIBE_EUNSUPPORTED (-4) /* the graph exceeds a supported size limit */

/* per-shot flags */
#define VIBE_FLAG_BP_CONVERGED 1u /* the correction is a converged member's */
#define VIBE_FLAG_LSD_USED 2u     /* no member converged; LSD produced it */
#define VIBE_FLAG_LSD_FAILED 4u   /* some cluster could not be made valid */
#define VIBE_FLAG_SATURATED 8u    /* a message or posterior reached +-clamp: in the
                                     winning member's run, or in any member's
                                     run when LSD ran (members that stop early
                                     under the correction limit are not
                                     counted); never set for a zero syndrome
                                     decided without running BP */

typedef struct vibe_graph vibe_graph;

typedef struct vibe_config {
    uint32_t L;         /* ensemble size, 1..64 (Sec. III.D.1 step 1) */
    uint32_t M;         /* correction limit, 1..L (step 2) */
    uint32_t T_max;     /* iteration limit of every member, 1..64 */
    uint32_t lsd_order; /* 0 = LSD-0, the paper's setting (Sec. III.D.1 step
                           5); 1..64 adds, on every valid cluster, the
                           combination sweep of ordered statistics decoding
                           (the higher-order search that LSD-0 leaves out,
                           Sec. III.D.1 step 5): no non-pivot
                           column, each single one, each pair among the first
                           lsd_order in rank order; the candidate of least
                           prior weight wins, ties to the earlier.  Larger
                           values are VIBE_EINVAL. */
    double alpha;       /* min-sum scaling factor applied to every check message */
    double clamp;       /* bound on |messages|, |posteriors| and |lambda|; also
                           the magnitude sent by a check with no other
                           neighbour.  1e6 (exact in FP32) is the default. */
    uint32_t message_bits; /* BP arithmetic: 32 (or 0) = FP32 messages and
                              posteriors, the production setting; 64 = FP64,
                              in the same operation order as a plain
                              column-by-column FP64 decoder, for verification */
    uint32_t schedule;     /* 0 = serial-V (VibeLSD: each member updates the
                              columns one after another in its permutation
                              order, Algorithm 1 serial branch); 1 = parallel
                              (flooding: every message of an iteration is
                              formed from the previous iteration's, Algorithm
                              1 parallel branch; all members then agree, so
                              L = 1 gives the BP+LSD-0 baseline of Sec. IV.H);
                              2 = layered (check-serial, which Sec. V names as
                              future work: each member visits the checks one
                              at a time in its own order, every check working
                              from the latest posteriors, mu = L - r_own).
                              The gradient refuses layered graphs
                              (VIBE_EUNSUPPORTED); every decode path takes
                              them. */
} vibe_config;

typedef struct vibe_shot_stats {
    uint32_t flags;        /* VIBE_FLAG_* */
    int32_t winner;        /* member whose correction was taken, -1 if LSD ran */
    uint32_t t_win;        /* that member's convergence iteration, 0 if LSD ran */
    uint32_t n_conv;       /* members seen converged before the shot finished;
                              like member_iters it depends on timing (members
                              past the correction limit stop as soon as that is
                              known), unlike every other field and the
                              correction */
    uint32_t lsd_clusters; /* final LSD clusters (0 if LSD did not run) */
    uint32_t lsd_largest;  /* columns in the largest final cluster */
    uint32_t lsd_rounds;   /* LSD growth rounds */
    uint32_t member_iters; /* BP iterations run, summed over members */
} vibe_shot_stats;

typedef struct vibe_graph_info {
    uint32_t m, n, k, L, M, T_max;
    uint64_t nnz;          /* edges of the Tanner graph */
    uint32_t max_row_degree, max_col_degree;
    uint32_t levels_min, levels_max; /* dependency levels per member schedule */
    uint32_t chunks_min, chunks_max; /* parallel steps of one sweep per member */
    uint32_t message_bits;           /* 32 or 64 */
    uint32_t grad_width;             /* chunk width of the gradient schedule
                                        (16, 32 or 64; 0 before the first
                                        vibe_bp_grad call on the graph) */
    uint64_t device_bytes; /* graph + schedules resident on the device */
} vibe_graph_info_t;

/*
 * Offline stage (Sec. III.D.1): validate the detector error model, compute the
 * channel LLRs lambda_v = ln((1 - p_v) / p_v) in FP64 (clamped to
 * +-cfg->clamp), build the CSR/CSC copies and, for every member i, the
 * parallel steps of its serial schedule perms[i*n .. i*n+n-1] (a permutation
 * of 0..n-1; the paper draws them uniformly at random): columns that share no
 * check commute, so each step updates a set of mutually independent columns
 * while every row keeps the permutation's order.  Everything is uploaded to
 * the current HIP device, where it stays until vibe_graph_destroy.
 *
 *   m, n            detectors (rows) and error mechanisms (columns), n >= 1
 *   h_indptr        m + 1 entries, h_indptr[0] = 0, non-decreasing
 *   h_indices       h_indptr[m] column indices, < n, strictly ascending per row
 *   priors          n probabilities, each strictly between 0 and 1
 *   k, l_indptr, l_indices   the observable matrix in the same CSR form
 *   perms           L x n uint32 permutations of the columns (host); with
 *                   the layered schedule L x m permutations of the checks
 *                   (each member's check order)
 *   cfg             decoder settings (copied)
 *   out             receives the handle
 * Limits (VIBE_EUNSUPPORTED beyond them): m < 65536, n < 2^24, every column
 * in at most 15 checks, every row shorter than 65536, nnz < 2^31.
 */
int vibe_graph_create(uint32_t m, uint32_t n, const uint32_t* h_indptr, const uint32_t* h_indices,
                      const double* priors, uint32_t k, const uint32_t* l_indptr,
                      const uint32_t* l_indices, const uint32_t* perms, const vibe_config* cfg,
                      vibe_graph** out);

/* Frees the handle, its device copies and its workspace (synchronises the
   device first).  NULL is accepted. */
void vibe_graph_destroy(vibe_graph* g);

/* Sizes and footprint of a graph. */
int vibe_graph_info(const vibe_graph* g, vibe_graph_info_t* info);

/* One min-sum scaling factor per iteration (Algorithm 1 with alpha_t in
   place of a constant): alpha (host, count doubles, each in (0, 1e6]) gives
   alpha_1 .. alpha_count; iterations past count keep alpha_count.  count = 0
   returns to cfg->alpha for every iteration.  0..64 is accepted, anything
   else is VIBE_EINVAL.  The factors go to a new device table (512 bytes,
   freed by vibe_graph_destroy) and apply to later calls.  Work already
   queued and captured sequences (vibe_exec) keep the table they were given.
   A server reads the setting whenever it forms a batch, so change it only
   while no server holding the graph runs.  vibe_bp_grad takes its own
   factors and is not affected. */
int vibe_graph_set_alpha(vibe_graph* g, const double* alpha, uint32_t count);

/* Copies the member schedules the graph holds into perms (host, L x n
   uint32 column permutations, or L x m check orders for the layered
   schedule), so that a reference decoder can run the same members
   (Sec. III.D.1 step 1 draws them offline). */
int vibe_graph_get_schedules(const vibe_graph* g, uint32_t* perms);

/*
 * Online stage, batched (Sec. III.D.2): decode B syndromes in one launch
 * sequence on `stream`.
 *   syndromes    device, B x m uint8 (0/1), row-major
 *   corrections  device, B x ceil(n/64) uint64 words: the bit-packed e-hat,
 *                which always satisfies H e-hat = s for converged shots and
 *                for LSD shots without VIBE_FLAG_LSD_FAILED
 *   observables  device, B x k uint8: Lobs * e-hat mod 2
 *   stats        device, B records, or NULL
 * B = 0 is accepted and does nothing.
 */
int vibe_decode(vibe_graph* g, const uint8_t* syndromes, uint64_t B, uint64_t* corrections,
                uint8_t* observables, vibe_shot_stats* stats, void* stream);

/*
 * vibe_decode with bit-packed syndromes.  Not a separate operation of the
 * paper: the same online stage (Sec. III.D.2) taking the syndrome bits of
 * the decoding problem (Sec. II.B) eight times denser, for callers that
 * hold them packed.
 *   syndromes    device, B x ceil(m/64) uint64 words, row-major: check c of a
 *                shot is bit (c mod 64) of its word c / 64; bits past m in the
 *                last word are ignored
 * Outputs, results and errors are those of vibe_decode on the same
 * syndromes.  The words are expanded, one chunk of shots at a time, into a
 * buffer the handle keeps (one byte per check, grown on demand and freed by
 * vibe_graph_destroy); like vibe_decode's workspace it is shared by the
 * handle's calls, so calls on one handle must not overlap.
 */
int vibe_decode_packed(vibe_graph* g, const uint64_t* syndromes, uint64_t B, uint64_t* corrections,
                       uint8_t* observables, vibe_shot_stats* stats, void* stream);

/*
 * The same decoder with one launch sequence per shot: every shot is decoded
 * on its own (ensemble, selection, LSD if needed, observables) before the
 * next one starts.  Not a separate operation of the paper, which decodes one
 * shot at a time on a CPU (Sec. III.D.2): this is the per-shot-launch
 * baseline against which the batched form's throughput is measured.  Same
 * arguments, results and errors as vibe_decode.
 */
int vibe_decode_plain(vibe_graph* g, const uint8_t* syndromes, uint64_t B, uint64_t* corrections,
                      uint8_t* observables, vibe_shot_stats* stats, void* stream);

/*
 * vibe_decode for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as vibe_decode; the outputs equal
 * vibe_decode's on the same syndromes (every field but the timing-dependent
 * n_conv and member_iters of the stats).  Every buffer beyond the caller's
 * inputs and outputs is carved from one static device array of
 * VIBE_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs
 * on until the process ends; the call allocates nothing (no hipMalloc, no
 * events: kernel timing of vibe_profile_enable is not recorded).  The batch
 * is decoded in chunks of shots whose buffers fit the array, with a BP grid
 * cut to fit as well, so large graphs run with fewer resident wavefronts
 * than vibe_decode.  VIBE_EUNSUPPORTED (with nothing queued) when not even
 * one shot of the graph fits the array.  The packed input of
 * vibe_decode_packed is not offered here.  Every call on one device shares
 * that device's array, and each call overwrites it: calls that overlap in
 * time on one device (on any handles or streams) race and must not be
 * made.  The array is set up on the first call on each device (with the
 * graph's device made current for the lookup).
 */
#define VIBE_NOALLOC_SCRATCH_BYTES ((uint64_t)256 << 20)
int vibe_decode_noalloc(vibe_graph* g, const uint8_t* syndromes, uint64_t B, uint64_t* corrections,
                        uint8_t* observables, vibe_shot_stats* stats, void* stream);

/*
 * The BP ensemble alone (Algorithm 1, serial-V, every member), for B shots,
 * without the correction limit: every member runs until its own hard
 * decision satisfies the syndrome (if stop_on_converge) or for exactly
 * T_run iterations (1 <= T_run <= 64).
 *   t_conv       device, B x L int32: iteration at which the member's decision
 *                first satisfied the syndrome, 0 if it never did
 *   posteriors   device, B x L x n, or NULL: L_v after the member's last
 *                iteration; float when the graph has message_bits 32, double
 *                when it has 64
 *   ehat         device, B x L x ceil(n/64) uint64, or NULL: the member's
 *                decision after its last iteration
 */
int vibe_bp_ensemble(vibe_graph* g, const uint8_t* syndromes, uint64_t B, uint32_t T_run,
                     int stop_on_converge, int32_t* t_conv, void* posteriors, uint64_t* ehat,
                     void* stream);

/*
 * LSD alone (Sec. III.C), at the graph's lsd_order, on caller-given soft
 * information.
 *   soft         device, B x n float: lower = more likely flipped; columns are
 *                ranked by (soft, index) ascending
 *   corrections  device, B x ceil(n/64) uint64 (bit-packed e-hat)
 *   stats        device, B records or NULL (lsd_* fields and flags)
 */
int vibe_lsd(vibe_graph* g, const uint8_t* syndromes, const float* soft, uint64_t B,
             uint64_t* corrections, vibe_shot_stats* stats, void* stream);

/*
 * Ragged batching: several requests, possibly on graphs of different codes,
 * decoded with one persistent BP launch over all of their (shot, member)
 * items, then selection, LSD and observables per request.  Each request's
 * outputs are exactly those vibe_decode produces for it alone.  Graphs of
 * all three schedules can share one call and one launch.  All graphs of one
 * call must share message_bits and live on the runtime's device.  A runtime owns the device workspace of its calls;
 * calls on one runtime must not overlap in time.
 */
typedef struct vibe_runtime vibe_runtime;

typedef struct vibe_request {
    vibe_graph* graph;
    const uint8_t* syndromes;   /* device, B x m uint8 */
    uint64_t B;                 /* shots, may be 0 */
    uint64_t* corrections;      /* device, B x ceil(n/64) uint64 */
    uint8_t* observables;       /* device, B x k uint8 */
    vibe_shot_stats* stats;     /* device, B records, or NULL */
} vibe_request;

int vibe_runtime_create(vibe_runtime** out); /* on the current HIP device */
void vibe_runtime_destroy(vibe_runtime* rt); /* synchronises the device first; NULL accepted */
int vibe_decode_ragged(vibe_runtime* rt, const vibe_request* reqs, uint32_t n_reqs, void* stream);

/*
 * A captured launch sequence: vibe_exec_create records the kernels that
 * vibe_decode_ragged would queue for `reqs` into a HIP graph, with its own
 * workspace, after one eager run; vibe_exec_launch replays it on `stream`.
 * The requests' device pointers are fixed at creation: refill the syndrome
 * buffers and replay.  A replay writes the same outputs as an eager call on
 * the buffers' contents.  VIBE_EUNSUPPORTED if the requests need more than
 * one round of workspace (about 32 GB of per-shot buffers).
 */
typedef struct vibe_exec vibe_exec;
int vibe_exec_create(const vibe_request* reqs, uint32_t n_reqs, vibe_exec** out);
int vibe_exec_launch(vibe_exec* ex, void* stream);
void vibe_exec_destroy(vibe_exec* ex); /* synchronises the device first; NULL accepted */

/*
 * Launch settings of the BP ensemble (K1) for one graph.  The ensemble is
 * (shot, member) work items, each run by one wavefront in the paper's
 * layout (Sec. III.D.1: the hardware bounds how far the decoders run in
 * parallel).  Four settings map it onto the GPU; the decoder's results do
 * not depend on any of them:
 *   slab_in_lds     1: the member's message slab lives in LDS (only where
 *                   it fits, one shot per wavefront); 0: global memory.
 *                   Before any setting is applied: LDS where it fits and
 *                   lets as many wavefronts reside as a global slab.
 *   grid            persistent BP blocks (0 = as many as fit at once).
 *   shots_per_wave  1, 2 or 4: one wavefront runs P shots of a member side
 *                   by side on the member's schedule recut into chunks of
 *                   64 / P edges (serial schedule only).  On graphs whose
 *                   64-edge chunks are far from full (the sweep's
 *                   dependency chain, not its edge count, sets the chunk
 *                   count) this runs P times the shots per chunk step.
 *   decisions_global -1: automatic; 1: each wavefront keeps its hard
 *                   decisions in global memory (one mask per chunk, read
 *                   with the chunk, and a bitmap updated on flips) instead
 *                   of a bitmap in LDS (0).  On large graphs the bitmap
 *                   (n / 8 bytes per wavefront) caps how many wavefronts
 *                   fit in LDS; automatic takes global memory where that
 *                   lets more reside and the launch has more work items
 *                   than reside with the bitmap in LDS (a small batch is
 *                   bound by its serial chains, which the global masks
 *                   lengthen).  Not with the slab in LDS.
 * A launch whose work items all reside at once (no more than the grid)
 * runs a variant that loads more chunks ahead at fewer wavefronts per SIMD
 * (FP32, serial schedule, slab in global memory, one shot per wavefront,
 * decisions in LDS); its results are those of the persistent kernel.
 * vibe_set_launch applies settings (building the recut schedule on first
 * use: EUNSUPPORTED for the parallel and layered schedules); settings that
 * vibe_decode_noalloc uses must be applied before it is called.
 * vibe_get_launch reads them back (from_cache and ms are 0).
 */
typedef struct vibe_launch {
    int slab_in_lds;
    int grid;
    int shots_per_wave;
    int decisions_global;
    int from_cache;  /* vibe_autotune: 1 if taken from the shape cache untimed */
    double ms;       /* vibe_autotune: decode time of the sample (timed run) */
} vibe_launch_t;
int vibe_set_launch(vibe_graph* g, const vibe_launch_t* s);
int vibe_get_launch(const vibe_graph* g, vibe_launch_t* s);

/*
 * Autotuning: times vibe_decode of the given syndromes (device, B x m) with
 * the slab in LDS (where it fits), and in global memory with 1, 2 and 4
 * shots per wavefront and decisions in LDS or global memory, each at full
 * occupancy, then the best of those with the BP
 * grid at 7/8, 3/4, 5/8 and 1/2 of full; applies the fastest to the handle
 * and stores it in a process-wide cache keyed by the graph's shape (checks,
 * columns, edges, L, M, T, chunk and level counts, LSD order, precision,
 * schedule, device) and the batch size class (floor(log2 B)).  A graph of
 * a cached shape gets the stored settings without timing (from_cache = 1).
 * Synchronises `stream`.  out (may be NULL) receives the choice.
 */
int vibe_autotune(vibe_graph* g, const uint8_t* syndromes, uint64_t B, void* stream, vibe_launch_t* out);

/*
 * Serving: continuous batching over resident graphs, each request admitted
 * by its HBM footprint.  vibe_server_submit queues one request (any number
 * of shots, up to max_batch_shots) on graph graphs[graph_index] and returns
 * at once.  The server owns one device pool of hbm_budget bytes (0 = room
 * for `slots` full batches of the graph whose full batch is largest).  A
 * server thread keeps up to `slots` batches in flight, each on its own
 * stream; a batch holds requests on one graph, so small codes do not wait
 * for the long serial chains of large ones, and takes a block of the pool
 * sized by its own footprint (the decode buffers of its shots, BP slabs for
 * a grid no larger than its work items, staging, tables).  Whenever a slot
 * is free the thread takes the oldest queued request and, in order, the
 * later queued requests on the same graph while the batch still fits the
 * largest free block and the batch limits; an oldest request that does not
 * fit yet waits for batches to retire.  With two or more slots, the last
 * free slot only takes requests on the cheapest graphs (per-shot work
 * edges x T_max x L within twice the smallest of the server's graphs), so
 * their short batches never wait behind the long ones of large codes.  Requests arriving while others run
 * are so admitted as slots and memory free up, and their work overlaps on
 * the device.  Every request's outputs are exactly those of vibe_decode on
 * it alone.  vibe_server_wait blocks until the request is done and gives its
 * latency from submission to completion (host clock, ms).  Submit refuses a
 * request whose footprint alone exceeds the pool (VIBE_ENOMEM) or needs more
 * than one round of per-shot buffers (about 32 GB; VIBE_EINVAL).  A
 * request's syndromes must already be on the device when it is submitted
 * (the server's streams do not wait for the caller's), and its buffers must
 * stay valid until its wait returns.  Submit and wait may be called from
 * any thread.
 */
typedef struct vibe_server vibe_server;

typedef struct vibe_server_config {
    uint32_t slots;              /* batches in flight, 1..16 */
    uint32_t max_batch_requests; /* requests per batch */
    uint32_t max_batch_shots;    /* shots per batch (and per request) */
    uint32_t reserved;           /* set to 0 */
    uint64_t hbm_budget;         /* bytes of the device pool, 0 = see above */
} vibe_server_config;

int vibe_server_create(vibe_graph* const* graphs, uint32_t n_graphs, const vibe_server_config* cfg,
                       vibe_server** out);
int vibe_server_submit(vibe_server* s, uint32_t graph_index, const uint8_t* syndromes, uint64_t B,
                       uint64_t* corrections, uint8_t* observables, vibe_shot_stats* stats, uint64_t* ticket);
int vibe_server_wait(vibe_server* s, uint64_t ticket, double* latency_ms);
/* Batches launched, requests served, pool bytes, and the most pool bytes
   batches held at once (any output may be NULL). */
int vibe_server_info(vibe_server* s, uint64_t* batches, uint64_t* requests, uint64_t* pool_bytes,
                     uint64_t* peak_bytes);
void vibe_server_destroy(vibe_server* s); /* finishes every queued request first; NULL accepted */

/*
 * Differentiable decoder: gradient of the soft-syndrome loss of K unrolled
 * iterations (the paper defines no training objective; this one is ours).
 * Every member runs exactly K iterations of its schedule from the channel
 * LLRs lam (device, n values) and scaling factors alpha (device, K values;
 * alpha[t-1] in iteration t), both in the graph's message precision (float
 * for message_bits 32, double for 64) instead of the graph's own.  With the
 * final posteriors L_v, shat_c = (1 - prod_{v in N(c)} tanh(L_v / 2)) / 2 is
 * clamped to [eps, 1 - eps] and the loss is the binary cross-entropy of s_c
 * and shat_c summed over the checks.  Outputs (device, double): loss (1) =
 * sum over the B x L (shot, member) items, dlam (n) and dalpha (K) = its
 * gradient.  The gradient is exact wherever no argmin, sign or clamp changes
 * (a piecewise-smooth function).  Deterministic: the same inputs give the
 * same bits.  syndromes: device, B x m bytes, row-major.
 * Limits: 1 <= K <= 64, B >= 1, B x L <= 2^24, 0 < eps < 0.5, fewer than
 * 2^24 - 1 edges, and a per-wavefront row state that fits in 160 KB of LDS
 * (24 bytes per check in FP32, 36 in FP64, per shot of the wavefront: up
 * to ~6700 checks in FP32); VIBE_EINVAL / VIBE_EUNSUPPORTED otherwise.  The first call
 * on a graph builds its gradient schedule (device memory freed with the
 * graph); every call may grow the graph's workspace, like vibe_decode.
 * Calls on one graph must not overlap.
 */
/*
 * Chunk width of the gradient schedule: 16, 32 or 64 edges (64 / width
 * shots per wavefront), or 0 to let the library choose per graph (the
 * default).  Results per (shot, member) do not depend on it; only the
 * order of the final sums does.  Takes effect at the next vibe_bp_grad
 * call; waits for the device if a schedule must be dropped.
 * VIBE_EINVAL for other widths.  For measurements and tests.
 */
int vibe_grad_set_width(vibe_graph* g, uint32_t width);

int vibe_bp_grad(vibe_graph* g, const uint8_t* syndromes, uint64_t B, uint32_t K, const void* lam,
                 const void* alpha, double eps, double* loss, double* dlam, double* dalpha, void* stream);

/*
 * Kernel timing, for measurement: while enabled, every launch of the BP
 * ensemble kernel, of the selection kernel and of the LSD kernel made through
 * this handle is bracketed by HIP events recorded on the launch stream.
 * vibe_profile_read waits for those events and returns, per kernel, the
 * summed duration in milliseconds and the number of launches, then clears
 * the record.  Arrays are indexed 0 = BP ensemble, 1 = selection, 2 = LSD.
 */
int vibe_profile_enable(vibe_graph* g, int enable);
int vibe_profile_read(vibe_graph* g, double* ms /*[3]*/, uint64_t* launches /*[3]*/);

/*
 * Measurement of the HBM ceiling for the BP kernel's access pattern: `waves`
 * wavefronts each stream a private region of region_bytes of buf (device,
 * waves x region_bytes bytes, float data that is overwritten) `passes` times,
 * alternately up and down, reading and rewriting one 256-byte run per step
 * with loads three steps ahead, as the BP sweep and its backward pass move
 * a message slab.  Bytes moved = 2 x waves x region_bytes x passes; time it
 * with events on `stream`.  region_bytes: a positive multiple of 256.  For
 * the benchmark's roofline only; not part of the decode path.
 */
int vibe_measure_slab_stream(float* buf, uint64_t region_bytes, uint32_t waves, uint32_t passes, void* stream);

/* Message of the last failing call on this thread ("" if none). */
const char* vibe_last_error(void);

/* Library version string. */
const char* vibe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VIBELSD_H */
