/*
 * hookcc -- adaptive, work-efficient Hook-Compress connected components on
 * AMD Instinct MI355X (gfx950).  C ABI of libhookcc.so.
 *
 * The operation (Section 2 of the paper, definition of connected components):
 * for an undirected graph G = (V, E) with V = {0, ..., n-1}, give every vertex
 * the id of a representative vertex of its component.  The representative is
 * the SMALLEST vertex id of the component: every parent pointer the hooking
 * kernels write goes from a larger id to a smaller one (the global
 * high-to-low rule of Fig. 2 and Fig. 3), so each component tree's root is
 * its minimum, and after the final Multi-Jump every vertex points at it.
 * The result is therefore unique and exact: label[v] = min{ w : w ~ v }.
 *
 * Method (Section 3): the component-tree array pi (pi[v] = v initially) is
 * built by Atomic-Hook over edge-list segments, each followed by a full
 * Multi-Jump Compress (Fig. 3, Fig. 4), with s = max(1, round(m / n))
 * segments by default (the average-degree heuristic 2|E|/|V| of Section 3.B,
 * with m the number of edge entries passed: the average degree when the
 * list holds both orientations of every edge, half of it when each edge is
 * listed once).  The atomic-free Hook of Fig. 2 is the
 * alternative hook variant; its "repeat until Hook performs no change" loop
 * (Fig. 1) runs with the convergence test and the shrinking frontier of
 * still-active edges kept on the device.
 *
 * Conventions for every entry point:
 *  - Array pointers marked [device] are device (HBM) memory of the current
 *    HIP device, e.g. torch.Tensor.data_ptr() of a ROCm tensor.  The library
 *    does not probe pointer kinds.  Pointers marked [host] are host memory.
 *  - Vertex ids and labels are int32; edge counts and offsets are int64.
 *  - Edges are given as two parallel arrays (structure of arrays): entry i is
 *    the pair (edges_u[i], edges_v[i]).  Self-loops, repeated pairs and both
 *    orientations of a pair are allowed and mean the same undirected edge.
 *  - Input arrays are never written.  The caller owns every array it passes;
 *    the library keeps no pointer after a call returns, apart from its own
 *    cached workspace (freed by cc_release).
 *  - Errors are returned as status codes (no exceptions cross the ABI);
 *    cc_last_error() gives a message for the calling thread's last failure.
 *  - On any non-zero status the contents of out_label are unspecified.
 *  - Concurrent calls from different host threads are allowed; the library's
 *    workspace cache is guarded by a mutex and keyed by stream.
 */
#ifndef HOOKCC_H
#define HOOKCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define CC_OK 0
#define CC_ERR_ARG (-1)        /* null pointer with a non-zero length, n < 0, m < 0,
                                  bad offsets, or an unknown option value        */
#define CC_ERR_RANGE (-2)      /* an edge endpoint outside [0, n) (detected on the
                                  device during the first pass over the edges)    */
#define CC_ERR_NOMEM (-3)      /* workspace too small or device allocation failed */
#define CC_ERR_HIP (-4)        /* a HIP runtime error (message in cc_last_error)  */
#define CC_ERR_NOCONVERGE (-5) /* the atomic-free Hook hit opts->max_rounds       */

/* ---------------------------------------------------------------- options */
#define CC_HOOK_AUTO 0   /* library choice (the default): for lists of m >= 2^22
                            entries the Atomic-Hook with the giant filter when
                            m / n >= 8 and the hybrid plan below otherwise; the
                            atomic-free Hook for smaller lists (the hybrid plan for a
                            no-sync call); the Atomic-Hook with the symmetric flag    */
#define CC_HOOK_ATOMIC 1 /* Atomic-Hook (Fig. 3, CAS on roots) + segmentation (Fig. 4) */
#define CC_HOOK_PLAIN 2  /* atomic-free Hook (Fig. 2) rounds until no change (Fig. 1),
                            convergence test and active-edge frontier on the device   */
#define CC_HOOK_HYBRID 3 /* one atomic-free Hook round (Fig. 2) over all entries with its
                            Multi-Jump and frontier compaction, then Atomic-Hook (Fig. 3,
                            path halving) over the still-active root pairs and a final
                            Multi-Jump: a fixed launch sequence, no host read (the same
                            for CSR input)                                          */

#define CC_FILTER_OFF 0  /* Atomic-Hook only: hook every edge entry                   */
#define CC_FILTER_GIANT 1 /* Atomic-Hook only: after the first segment(s), sample the
                            labels, and when one component holds a large share of the
                            samples, keep a bitmap of its vertices and skip every later
                            edge whose two ends are both in it (exact: trees only
                            merge, so such an edge is already satisfied)               */
#define CC_FILTER_AUTO 2 /* library chooses (the default)                             */

typedef struct cc_options {
    int32_t hook;             /* CC_HOOK_AUTO (default), CC_HOOK_ATOMIC, CC_HOOK_PLAIN or
                                 CC_HOOK_HYBRID                                          */
    int32_t segments;         /* Atomic-Hook: number of edge segments s; 0 = default
                                 max(1, round(m / n)) (16x that when CC_HOOK_AUTO picks the
                                 filtered Atomic-Hook, so the first segment is ~n/16
                                 entries); clamped to [1, ceil(m / 4)]                  */
    int32_t filter;           /* CC_FILTER_* (Atomic-Hook only); default CC_FILTER_AUTO  */
    int32_t filter_after;     /* segments hooked before the giant-component sample
                                 (0 = default 1)                                        */
    int32_t block;            /* threads per workgroup for the edge kernels: 64..1024,
                                 multiple of 64; 0 = default: 256, 512 for the filtered
                                 plan CC_HOOK_AUTO picks, 1024 for the hybrid plan      */
    int32_t edges_per_thread; /* edge entries per thread in the edge kernels: 4, 8 or 16;
                                 0 = default                                            */
    int32_t max_rounds;       /* atomic-free Hook: round cap (0 = n + 1, which is never
                                 reached: every active round removes at least one root) */
    int32_t rounds_per_check; /* atomic-free Hook: rounds launched between two host reads
                                 of the device convergence word (0 = default 4)          */
    int32_t profile;          /* 1 = time every kernel with HIP events on the call's stream
                                 and report the phase times in cc_stats (adds a few
                                 microseconds per launch); 0 = off                      */
    int32_t host_loop;        /* hook = CC_HOOK_PLAIN only, for ablations of the paper's
                                 baseline (Fig. 1 as written, convergence read by the host
                                 after every launch): CC_HOST_LOOP_OFF (default: device-side
                                 convergence and compaction), CC_HOST_LOOP_JUMP (Compress as
                                 repeated single-level Jump launches, Fig. 2) or
                                 CC_HOST_LOOP_MULTIJUMP (Compress as one Multi-Jump)    */
    int32_t coherent_loads;   /* Atomic-Hook path: 1 = tree loads and stores are coherent
                                 across the XCDs (agent scope, served beyond the per-XCD
                                 L2); 0 (default) = cached loads, which may return an
                                 older ancestor -- always a valid one (kept for
                                 measurement; results are identical)                   */
    int32_t hot_cache;        /* giant filter only: answer the bit tests of the endpoints
                                 that a sample of the entries hits most often from a table
                                 in LDS.  CC_HOT_VERTEX: 81,920 two-way sets of one-byte
                                 vertex tags (160 KiB; set s holds the two most sampled
                                 vertices k * 81920 + s, k < 255, and answers for them
                                 while they are in the giant component); CC_HOT_LARGE:
                                 32,768 bitmap-word slots (160 KiB); CC_HOT_ON: 16,384
                                 word slots; CC_HOT_OFF: none.  CC_HOT_AUTO (default):
                                 CC_HOT_VERTEX for n <= 255 * 81920, else CC_HOT_LARGE  */
    int32_t path_halving;     /* Atomic-Hook climb: CC_HALVE_AUTO (default, on), CC_HALVE_ON
                                 or CC_HALVE_OFF (Fig. 3 exactly) -- re-point a non-root
                                 passed on the way up at its grandparent, on every 4th
                                 such step of a climb (every 8th in the giant-filtered
                                 and CSR kernels)                                       */
    int32_t symmetric;        /* 1 = the caller guarantees that every pair (u, v) of the list
                                 also appears as (v, u) (a symmetrised list); the Atomic-Hook
                                 then skips the entries with u > v, which changes nothing in
                                 the result for such lists and halves the tree accesses.
                                 Wrong labels if the guarantee does not hold.  Never on by
                                 default; with CC_HOOK_AUTO it forces the Atomic-Hook.    */
    int32_t graph;            /* 1 = capture the call's launch sequence in a hipGraph on the
                                 call's stream the first time and replay it on later
                                 calls with the same arrays, sizes and plan (Atomic-Hook
                                 single solves, graph lists and batches; for the
                                 atomic-free Hook, each block of rounds_per_check rounds
                                 between two host reads; needs a stream other than the
                                 null stream, else ignored; profile = 1 disables it)   */
    int32_t no_sync;          /* cc_labels_ex and cc_labels_csr only: 1 = enqueue the whole
                                 solve on the call's stream and return without waiting
                                 (Atomic-Hook only: CC_HOOK_AUTO then picks it, and
                                 CC_HOOK_PLAIN or profile = 1 is CC_ERR_ARG).  Argument
                                 errors still return at once; the device-detected status
                                 (CC_ERR_RANGE) is read with cc_stream_status.  The
                                 caller keeps every array alive and unchanged until the
                                 stream has passed the call.  0 = synchronous (default) */
    int32_t compact_threshold; /* atomic-free Hook: frontier compaction threshold tau in
                                 thousandths, 0..1000.  Every round counts the entries
                                 still active after its Compress; round 1 always writes
                                 them to a frontier of root pairs, and a later round
                                 rewrites them only when the previous round's surviving
                                 fraction (active entries / entries read) was below
                                 tau / 1000 -- otherwise the next round reads the same
                                 frontier again.  0 = default: rewrite every round     */
    int32_t reserved[1];      /* must be zero                                           */
} cc_options;

#define CC_HOT_AUTO 0
#define CC_HOT_ON 1
#define CC_HOT_OFF 2
#define CC_HOT_LARGE 3
#define CC_HOT_VERTEX 4

#define CC_HALVE_AUTO 0
#define CC_HALVE_ON 1
#define CC_HALVE_OFF 2

#define CC_HOST_LOOP_OFF 0
#define CC_HOST_LOOP_JUMP 1
#define CC_HOST_LOOP_MULTIJUMP 2

/* Fills *opts with the defaults (all fields zero = library choice). */
void cc_options_init(cc_options* opts);

/* Per-call statistics (optional output of cc_labels_ex). */
typedef struct cc_stats {
    int32_t hook;          /* variant that ran (CC_HOOK_ATOMIC or CC_HOOK_PLAIN)       */
    int32_t segments;      /* Atomic-Hook: segments used                               */
    int32_t filter_used;   /* 1 if the giant-component filter was active              */
    int32_t rounds;        /* atomic-free Hook: Hook rounds run until no change        */
    int64_t active_edges;  /* atomic-free Hook: edges still active after round 1       */
    int32_t giant_label;   /* filter: label of the sampled giant component (or -1)     */
    int32_t host_syncs;    /* host synchronisations made inside the call               */
    int32_t hook_launches; /* edge-pass kernels launched (Atomic-Hook / Hook / compaction) */
    int32_t compress_launches; /* Multi-Jump kernels launched                          */
    float hook_ms;         /* opts->profile: summed durations of the edge-pass kernels   */
    float compress_ms;     /* opts->profile: summed durations of the Multi-Jump kernels  */
    float other_ms;        /* opts->profile: init, sample and bitmap kernels             */
    int64_t reserved[4];
} cc_stats;

/* ------------------------------------------------------------- single graph */

/* Min-id component labels of one graph; synchronous.
 *   n          number of vertices (>= 0)
 *   edges_u    [device] int32[m], endpoint 0 of each entry, in [0, n)
 *   edges_v    [device] int32[m], endpoint 1 of each entry, in [0, n)
 *   m          number of edge entries (>= 0)
 *   out_label  [device] int32[n]; receives label[v] = min id of v's component
 * Runs on the null stream with default options and returns after the labels
 * are complete.  n == 0 returns CC_OK; m == 0 gives label[v] = v.
 * Returns CC_OK, CC_ERR_ARG, CC_ERR_RANGE, CC_ERR_NOMEM or CC_ERR_HIP. */
int32_t cc_labels(int32_t n, const int32_t* edges_u, const int32_t* edges_v, int64_t m,
                  int32_t* out_label);

/* As cc_labels, with options, caller workspace, stream and statistics.
 *   opts             [host] options, or NULL for the defaults
 *   workspace        [device] scratch of workspace_bytes bytes (256-byte aligned),
 *                    or NULL to use the library's cached pool for this stream
 *   workspace_bytes  size of workspace; must be >= cc_workspace_bytes(n, m, opts)
 *   stream           hipStream_t to run on (NULL = null stream)
 *   stats            [host] optional statistics output, or NULL
 * The call returns after the labels are complete on `stream` (it ends with
 * one stream synchronisation; the atomic-free Hook also reads the device
 * convergence word once every opts->rounds_per_check rounds), unless
 * opts->no_sync = 1: then it returns once the work is enqueued, and the
 * device-detected status is read with cc_stream_status. */
int32_t cc_labels_ex(int32_t n, const int32_t* edges_u, const int32_t* edges_v, int64_t m,
                     int32_t* out_label, const cc_options* opts, void* workspace,
                     size_t workspace_bytes, void* stream, cc_stats* stats);

/* Device-detected status of the last cc_labels_ex / cc_labels_csr call made on
 * `stream` (NULL = null stream) of the current device with opts->no_sync = 1:
 * CC_PENDING while that call's work has not finished, then CC_OK or
 * CC_ERR_RANGE (an endpoint outside [0, n) or a malformed row_ptr; the labels
 * are then unspecified).  Non-blocking.  CC_ERR_ARG when no such call was made
 * since the last cc_release.  Calls that fail before enqueuing work leave the
 * recorded status unchanged.  One status per stream: a later no-sync call on
 * the stream replaces it, so read it before the next one if it matters. */
#define CC_PENDING 1
int32_t cc_stream_status(void* stream);

/* Device scratch bytes cc_labels_ex needs for (n, m, opts); 0 on bad input. */
size_t cc_workspace_bytes(int32_t n, int64_t m, const cc_options* opts);

/* As cc_labels_ex, for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * call makes no device or host allocation.  Its workspace is a fixed device
 * array of CC_NOALLOC_SCRATCH_BYTES bytes inside the library, one per device,
 * held from the first call on a device until the process ends; the caller
 * still passes the edges and out_label.
 *   n, edges_u, edges_v, m, out_label   as cc_labels
 *   opts    [host] options or NULL; graph, no_sync and profile must be 0
 *           (CC_ERR_ARG otherwise)
 *   stream  hipStream_t to run on (NULL = null stream)
 *   stats   [host] optional statistics output, or NULL
 * Synchronous: returns after the labels are complete on `stream`.  With the
 * automatic hook (opts NULL or opts->hook = CC_HOOK_AUTO) a plan whose
 * workspace would exceed the array falls back to the Atomic-Hook (its
 * workspace: 256 bytes, plus n/8 bytes and the 20 MiB vertex table with the
 * giant filter, dropped when even that does not fit), so every size is
 * solved; an explicitly requested plan whose workspace (cc_workspace_bytes)
 * exceeds CC_NOALLOC_SCRATCH_BYTES returns CC_ERR_NOMEM with a message.
 * The array is shared by every call on a device and keeps the last call's
 * contents (each solve rewrites what it reads): calls on one device are
 * serialised by a host mutex, so two such calls never overlap on a GPU;
 * calls on different devices run independently.
 * Returns CC_OK, CC_ERR_ARG, CC_ERR_RANGE, CC_ERR_NOMEM, CC_ERR_NOCONVERGE
 * or CC_ERR_HIP. */
#define CC_NOALLOC_SCRATCH_BYTES (32 << 20)
int32_t cc_labels_noalloc(int32_t n, const int32_t* edges_u, const int32_t* edges_v, int64_t m,
                          int32_t* out_label, const cc_options* opts, void* stream,
                          cc_stats* stats);

/* ------------------------------------------------------------------ batches */

/* Min-id labels of many independent graphs packed back to back; synchronous.
 *   num_graphs  B >= 0
 *   vtx_off     [host] int64[B+1]; graph g owns vertices [vtx_off[g], vtx_off[g+1]);
 *               vtx_off[0] == 0, non-decreasing, each graph < 2^31 vertices
 *   edge_off    [host] int64[B+1]; graph g owns entries [edge_off[g], edge_off[g+1]);
 *               edge_off[0] == 0, non-decreasing
 *   edges_u/v   [device] int32[edge_off[B]]; LOCAL endpoint ids in [0, n_g)
 *   out_label   [device] int32[vtx_off[B]]; out_label[vtx_off[g] + x] receives the
 *               local label (min local id of x's component within graph g)
 * Graphs of at most CC_BATCH_LDS_MAX_N vertices are solved by one persistent
 * launch whose workgroups take graphs from a device work queue, largest first,
 * and keep each graph's tree array in LDS; larger graphs are solved in device
 * memory.  Returns after every label is complete (null stream).
 * Returns CC_OK, CC_ERR_ARG, CC_ERR_RANGE, CC_ERR_NOMEM or CC_ERR_HIP. */
#define CC_BATCH_LDS_MAX_N 65536
int32_t cc_labels_batch(int32_t num_graphs, const int64_t* vtx_off, const int64_t* edge_off,
                        const int32_t* edges_u, const int32_t* edges_v, int32_t* out_label);

/* As cc_labels_batch on `stream` (hipStream_t, NULL = null stream), using the
 * library's workspace pool; `opts` and `stats` may be NULL.  For the
 * LDS-solved graphs `opts` sets `path_halving` (CC_HALVE_AUTO / ON: the LDS
 * climb re-points passed non-roots at their grandparents; OFF: Fig. 3
 * exactly) and `segments`, a cap S on each graph's round(m_g / n_g) segments:
 * 0 = default, 2 with halving and no cap without it (in LDS a climb is
 * cheap, so fewer segments -- fewer Multi-Jump passes and barriers -- are
 * faster; the autotuner picks S) and `block`, the workgroup size of the LDS
 * solver (64..1024, multiple of 64; 0 = 1024; as many workgroups share a CU
 * as the LDS of the largest graph allows).  The LDS solver has no frontier
 * compaction and so no compaction threshold: each graph's entries are read
 * once per segment and hooked in LDS, with nothing left to compact.  `graph`
 * = 1 captures the launch sequence.  Larger graphs use the default
 * device-memory plan. */
int32_t cc_labels_batch_ex(int32_t num_graphs, const int64_t* vtx_off, const int64_t* edge_off,
                           const int32_t* edges_u, const int32_t* edges_v, int32_t* out_label,
                           const cc_options* opts, void* stream, cc_stats* stats);

/* As cc_labels_batch_ex with the offsets in DEVICE memory: the batch needs
 * no host pass at all.  Preparation launches of one thread per graph read
 * the offsets, check them, order the graphs largest first (a counting sort
 * on the size class of m_g + n_g, as the host-offset call does) and write
 * their descriptors; then the persistent LDS launch solves them.  A call is
 * three launches (four above 32,768 graphs, where a scan launch keeps the
 * ordering linear in the graph count) and one synchronisation on `stream`.
 *   vtx_off, edge_off  [device] int64[B+1], as for cc_labels_batch
 *   edges_u/v          [device] int32[edge_off[B]], local ids (NULL only if no graph
 *                      has entries)
 *   out_label          [device] int32[vtx_off[B]] (NULL only if no graph has vertices)
 *   max_n              an upper bound of every graph's vertex count, in
 *                      [1, CC_BATCH_LDS_MAX_N]: it sizes the launch's LDS (a
 *                      tight bound lets several workgroups share a CU)
 * Every graph is LDS-solved: offsets that do not start at 0, decrease, or
 * give a graph more than max_n vertices, and a NULL array that a graph
 * needs, are found on the device; then no
 * label is written for the offending graphs and the call returns
 * CC_ERR_ARG after the synchronisation.  `opts` (nullable) takes
 * `segments`, `path_halving`, `block` and `graph` as for cc_labels_batch_ex;
 * the device memory it needs (256 B, plus 40 B per graph, plus 1 KiB per
 * 1,024 graphs and 1 KiB) comes from the stream's pool.  Returns CC_OK, CC_ERR_ARG, CC_ERR_RANGE, CC_ERR_NOMEM or CC_ERR_HIP. */
int32_t cc_labels_batch_device(int32_t num_graphs, const int64_t* vtx_off,
                               const int64_t* edge_off, const int32_t* edges_u,
                               const int32_t* edges_v, int32_t* out_label, int32_t max_n,
                               const cc_options* opts, void* stream, cc_stats* stats);

/* Out-of-core solve: the edge lists stay in HOST memory and are streamed to
 * the device in chunks while earlier chunks are hooked.  The Atomic-Hook
 * reads every entry exactly once (Section 3.A), so each chunk is copied once
 * into one of two device staging buffers and hooked, followed by a
 * Multi-Jump (Fig. 4 with one segment per chunk; with the giant filter the
 * first chunk's labels are sampled and later chunks are filtered).  Device
 * memory holds only out_label, the bitmap and 2 x 2 x chunk_entries int32.
 *   host_u, host_v  [host] int32[m]; pinned memory (hipHostMalloc / torch
 *                   pin_memory) lets the copies overlap the hooks
 *   out_label       [device] int32[n]
 *   chunk_entries   entries per chunk (rounded down to a multiple of 4);
 *                   0 = 2^24
 *   opts            as cc_labels_ex; hook must be CC_HOOK_AUTO or CC_HOOK_ATOMIC
 *   stream          hipStream_t for the hooks (NULL = null stream); copies run
 *                   on a library stream ordered against it with events
 * Returns after the labels are complete; same status codes as cc_labels_ex. */
int32_t cc_labels_host(int32_t n, const int32_t* host_u, const int32_t* host_v, int64_t m,
                       int32_t* out_label, int64_t chunk_entries, const cc_options* opts,
                       void* stream, cc_stats* stats);

/* CSR adjacency input: entry i of row r is the pair (r, col[i]).  The
 * Atomic-Hook works on any subsets of E (Fig. 4), so the solve is the same as
 * for a pair list of m entries; the row of an entry is found on the fly (an
 * LDS window of row_ptr per tile), and with the giant filter the row's bit is
 * tested once per group of four consecutive entries.
 *   row_ptr    [device] int64[n+1]: row_ptr[0] == 0, non-decreasing, row_ptr[n] == m
 *   col        [device] int32[m], ids in [0, n)
 *   out_label  [device] int32[n]
 *   opts       as cc_labels_ex; hook CC_HOOK_AUTO, CC_HOOK_ATOMIC or CC_HOOK_HYBRID
 *              (AUTO: the hybrid plan for m >= 2^22 entries with m / n < 8, else
 *              the Atomic-Hook, filtered when m >= 2^22 and m / n >= 8);
 *              opts->symmetric = 1 promises a symmetric adjacency (every pair in
 *              both rows) and hooks only the entries with col > row
 * Synchronous on `stream` (NULL = null stream) unless opts->no_sync = 1 (as
 * for cc_labels_ex).  A malformed row_ptr or a column id outside [0, n)
 * returns CC_ERR_RANGE (checked on the device). */
int32_t cc_labels_csr(int32_t n, const int64_t* row_ptr, const int32_t* col, int64_t m,
                      int32_t* out_label, const cc_options* opts, void* stream, cc_stats* stats);

/* One graph of a graph list: its own device arrays, local ids in [0, n). */
typedef struct cc_graph {
    const int32_t* edges_u; /* [device] int32[m]                                          */
    const int32_t* edges_v; /* [device] int32[m]                                          */
    int32_t* out_label;     /* [device] int32[n]; receives local min-id labels            */
    int64_t m;              /* edge entries (>= 0)                                        */
    int32_t n;              /* vertices (>= 0)                                            */
    int32_t reserved;       /* must be zero                                               */
} cc_graph;

/* Labels of `count` independent graphs described by `graphs` ([host] array of
 * descriptors holding device pointers); synchronous on `stream` (NULL = null
 * stream).  Same solvers as cc_labels_batch: graphs of at most
 * CC_BATCH_LDS_MAX_N vertices share one persistent LDS launch, larger ones
 * are each solved in device memory on the same stream, and the call ends
 * with a single synchronisation.  Descriptors may point anywhere (the
 * graphs need not be packed).  `opts` as for cc_labels_batch_ex (nullable).
 * Returns CC_OK, CC_ERR_ARG, CC_ERR_RANGE, CC_ERR_NOMEM or CC_ERR_HIP. */
int32_t cc_labels_list(int32_t count, const cc_graph* graphs, const cc_options* opts, void* stream,
                       cc_stats* stats);

/* ------------------------------------------------------------------ serving */

/* A continuous-batching request server.  Requests (one graph each) are
 * admitted in arrival order while their HBM footprints fit a budget of
 * cfg->device_bytes.  A request's footprint is 8m bytes of edges, 4n bytes of
 * labels and the device workspace of its solve (256-byte granules), charged
 * whether its arrays are in host or device memory: a request of more than
 * CC_BATCH_LDS_MAX_N vertices brings its own Atomic-Hook workspace (bitmap
 * and vertex table of the giant filter), small requests share a fixed block
 * per worker, charged once at creation.  The server allocates one device
 * arena of cfg->device_bytes and carves from it everything it puts on the
 * device: copies of host edges and labels, and the workspaces, so the solves
 * of admitted requests never allocate.  Each of
 * cfg->workers host threads owns one HIP stream and, whenever it is free,
 * solves a wave taken from the head of the queue in arrival order (the
 * cc_labels_list solvers): the longest run of admitted small requests (at
 * most CC_BATCH_LDS_MAX_N vertices, one persistent LDS launch), or a single
 * large request on its own, so small requests never wait for a large one in
 * their wave.  Requests that arrive while other waves run join the next
 * wave, and waves overlap on the device.  Times are seconds on the clock of
 * cc_server_clock(). */
#define CC_REQ_HOST_EDGES 1  /* edges_u/edges_v are [host]: copied in at admission   */
#define CC_REQ_HOST_LABELS 2 /* out_label is [host]: labels copied back when done     */

typedef struct cc_server cc_server;

typedef struct cc_server_config {
    int64_t device_bytes;    /* footprint budget and arena size; 0 = a quarter of the
                                free device memory                                       */
    int32_t workers;         /* worker threads / streams, 1..16; 0 = 2                  */
    int32_t max_batch;       /* most requests in one wave; 0 = 1024                      */
    int64_t max_batch_edges; /* most edge entries in one wave (a larger single request
                                still runs alone); 0 = 2^28                              */
    int32_t reserved[8];     /* must be zero                                             */
} cc_server_config;

typedef struct cc_request_info {
    int32_t status;          /* CC_OK or the request's error code                        */
    int32_t batch_size;      /* requests in the wave that solved it                      */
    double t_submit;         /* cc_server_submit called                                  */
    double t_admit;          /* admitted: footprint charged, arena space granted         */
    double t_launch;         /* its wave started                                         */
    double t_device_done;    /* labels complete in device memory                         */
    double t_host_done;      /* labels copied back (== t_device_done without
                                CC_REQ_HOST_LABELS, up to the wave's final sync)         */
} cc_request_info;

/* Creates a server on the current device.  Returns CC_OK, CC_ERR_ARG,
 * CC_ERR_NOMEM (also when device_bytes cannot hold the workers' fixed
 * workspace) or CC_ERR_HIP; *out is NULL on failure. */
int32_t cc_server_create(const cc_server_config* cfg, cc_server** out);

/* Queues one request.  Pointers follow `flags` ([host] or [device]) and must
 * stay valid until the request is finished (cc_server_wait / poll).  Device
 * arrays are read (edges) and written (out_label) on a worker's stream, which
 * first waits for everything queued on `ready_stream` (hipStream_t of the
 * server's device; NULL = the null stream) at the time of this call: the work
 * that produces the edges, and earlier users of out_label's memory, may still
 * be running on that stream.  A request whose footprint exceeds the budget
 * left after the workers' fixed workspace finishes with CC_ERR_NOMEM; one
 * that fits waits in the queue until enough earlier requests have finished.
 * *ticket identifies it. */
int32_t cc_server_submit_on(cc_server* server, int32_t n, const int32_t* edges_u,
                            const int32_t* edges_v, int64_t m, int32_t* out_label, int32_t flags,
                            void* ready_stream, int64_t* ticket);

/* cc_server_submit_on with ready_stream = NULL (the null stream). */
int32_t cc_server_submit(cc_server* server, int32_t n, const int32_t* edges_u,
                         const int32_t* edges_v, int64_t m, int32_t* out_label, int32_t flags,
                         int64_t* ticket);

/* Blocks until the request is finished, fills *info (may be NULL) and forgets
 * the ticket.  Returns the request's status. */
int32_t cc_server_wait(cc_server* server, int64_t ticket, cc_request_info* info);

/* As cc_server_wait without blocking: returns 1 (and keeps the ticket) while
 * the request is still queued or running. */
int32_t cc_server_poll(cc_server* server, int64_t ticket, cc_request_info* info);

/* Requests waiting for admission, and footprint bytes charged against the
 * budget (admitted, unfinished requests plus the workers' fixed workspace);
 * either pointer may be NULL. */
int32_t cc_server_stats(cc_server* server, int64_t* pending, int64_t* arena_used);

/* Finishes every queued request, stops the workers and frees the arena. */
int32_t cc_server_destroy(cc_server* server);

/* The server's clock, in seconds. */
double cc_server_clock(void);

/* -------------------------------------------------------------- measurement */

/* Memory-ceiling probe (measurement only, no labels).  Streams the m entries
 * of edges_u/edges_v ([device], 16-byte aligned) with the tiling of the hook
 * kernels and, for mode 1, also gathers table[u] and table[v] from the
 * [device] int32[n] array `table`, or, for modes 2-4, tests bits u and v of
 * the [device] n-bit bitmap `table` (uint32 words) with cached loads (2),
 * non-temporal loads (3) or agent-scope atomic loads (4), or, for modes 5
 * and 6, makes one agent-scope compare-and-swap on table[u] per entry that
 * succeeds (5: swaps u for u) or fails (6: expects -1); `table` must then
 * hold table[x] = x and is left unchanged (the hooking atomic's ceiling).
 * Entries with an endpoint outside [0, n) are skipped by modes 1-6.
 * Modes 7-11 ignore the edges and probe the memory model behind the tree
 * array's write rule: `table` is [device] int32[n >= 128] with table[i] = i
 * for i < 32 and table[64] = 0.  Workgroup A (one XCD) loads table[1]
 * (modes 7-9 only), then stores table[0] = 100 with workgroup scope (7, 10),
 * agent scope (8, 11) or not at all (9); workgroup B (another XCD) then
 * swaps table[1] from 1 to 50 by an
 * agent-scope compare-and-swap; A then tries to swap table[1] from 1 to 70
 * the same way, which must fail.  table[96..97] receive the two XCD ids,
 * table[98..99] the polls of the two bounded waits (-1 = the wait ran out),
 * table[100] the value A loaded, table[101..102] the values A's and B's
 * compare-and-swap found (A's == 1: it ran on a stale copy of the line).
 * Asynchronous on `stream`.  Returns CC_OK, CC_ERR_ARG or CC_ERR_HIP. */
int32_t cc_probe(int32_t mode, const int32_t* edges_u, const int32_t* edges_v, int64_t m,
                 const void* table, int32_t n, void* stream);

/* ------------------------------------------------------------------ library */

/* Message for the calling thread's last non-zero status ("" if none). */
const char* cc_last_error(void);

/* Frees the library's cached device workspace (all streams).  Must not run
 * concurrently with another call (the workers of a running cc_server make
 * calls too). */
void cc_release(void);

/* Library version string. */
const char* cc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HOOKCC_H */
