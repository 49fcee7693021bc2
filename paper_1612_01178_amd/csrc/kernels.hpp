// Host-side launchers of the HIP kernels (internal to libhookcc).
#pragma once

#include "common.hpp"

namespace hookcc {

// pi[v] = v for v < n; resets the control block.  (Fig. 4, first step.)
hipError_t launch_init(int32_t* pi, int32_t n, Ctrl* ctrl, hipStream_t s);

// Atomic-Hook (Fig. 3) of entries [begin, end).  When `bits` is non-null the
// giant-component filter is applied (only if ctrl->filter_on is set);
// `halve` adds path halving to the climb; `sym` hooks only entries with
// u <= v (valid when every pair is present in both orientations).
hipError_t launch_ahook(const int32_t* u, const int32_t* v, int64_t begin, int64_t end,
                        int32_t* pi, int32_t n, Ctrl* ctrl, const uint32_t* bits, int block,
                        int ept, bool coherent, bool halve, bool sym, hipStream_t s);

// Multi-Jump (Fig. 3) over all n vertices.  When `gate` is non-null the
// kernel does nothing if *gate == 0.  `coherent` selects agent-scope tree
// loads and stores (see common.hpp).
hipError_t launch_mj(int32_t* pi, int32_t n, const uint32_t* gate, bool coherent, hipStream_t s);

// Multi-Jump for deep trees: pointer jumping within blocks of consecutive
// vertices in LDS, then a climb across blocks (the plain Multi-Jump for
// n < 2^22).  Postcondition as launch_mj: every tree is a star.
hipError_t launch_mj_deep(int32_t* pi, int32_t n, hipStream_t s);
// Multi-Jump with one vertex per thread (atomic-free path); does nothing when
// `gate` is non-null and *gate <= limit.
hipError_t launch_mj1(int32_t* pi, int32_t n, const uint32_t* gate, hipStream_t s,
                      uint32_t limit = 0);

// Giant-component sample: label of the component that holds the most of
// `samples` edge endpoints drawn across entries [0, m); sets ctrl->giant and
// ctrl->filter_on.  Requires pi to be a forest of stars (after Multi-Jump).
hipError_t launch_sample_giant(const int32_t* u, int64_t m, const int32_t* pi, int32_t n,
                               Ctrl* ctrl, int samples, hipStream_t s);

// bits[v] = (pi[v] == pi[ctrl->giant]) for v < n (stars required); no-op
// unless ctrl->filter_on.
hipError_t launch_bitmap(const int32_t* pi, int32_t n, Ctrl* ctrl, uint32_t* bits, hipStream_t s);
// Multi-Jump, then (when ctrl->filter_on) the giant bitmap and, when hot_tags
// is non-null, the cached words of the hot-word table, or when vtab is
// non-null, the bits of the vertex table, in one pass.
hipError_t launch_mj_bitmap(int32_t* pi, int32_t n, Ctrl* ctrl, uint32_t* bits,
                            const uint32_t* hot_tags, uint32_t* hot_vals, int slots, uint8_t* vtab,
                            hipStream_t s);

// Atomic-free Hook (Fig. 2) of round `round` (1-based).  Round 1 reads the
// input entries [0, m) and checks ranges; later rounds read the frontier of
// root pairs written by the previous round's compaction (size in ctrl->count).
hipError_t launch_hook_plain(int round, const int32_t* u, const int32_t* v, int64_t m,
                             const int2* f0, const int2* f1, int32_t* pi, int32_t n, Ctrl* ctrl,
                             int block, int ept, int grid_cap, hipStream_t s);

// Frontier compaction after the Compress of round `round`: keeps the entries
// whose endpoints still have different roots, written as root pairs to
// `dst` (capacity cap), size accumulated in ctrl->count[round & 1].
// Window round of the hybrid plan: an atomic-free Hook round over all m
// entries in which each workgroup first joins its chunk of entries inside an
// LDS window of consecutive vertices (see kernels_batch.hip).  Range-checks
// the entries.  Leaves pi a forest (not of stars).
hipError_t launch_hook_window(const int32_t* u, const int32_t* v, int64_t m, int32_t* pi,
                              int32_t n, Ctrl* ctrl, hipStream_t s);
// Atomic-Hook with path halving of the *count root pairs of a frontier.
hipError_t launch_ahook_pairs(const int2* fr, const uint32_t* count, int64_t cap, int32_t* pi,
                              bool halve, int grid_cap, hipStream_t s);

// tau: frontier rewrite threshold in thousandths (0xffffffff = every round).
hipError_t launch_compact(int round, const int32_t* u, const int32_t* v, int64_t m, int2* f0,
                          int2* f1, int64_t cap, const int32_t* pi, int32_t n, Ctrl* ctrl,
                          uint32_t tau, int block, int ept, int grid_cap, hipStream_t s);

// Fig. 1 as a host loop: a Hook pass over all m entries that sets
// ctrl->hook_changed when an entry's parents differ, and one level of Jump
// (Fig. 2) over all vertices that sets ctrl->jump_changed when it moves a
// pointer.
hipError_t launch_hook_flag(const int32_t* u, const int32_t* v, int64_t m, int32_t* pi, int32_t n,
                            Ctrl* ctrl, int block, int ept, hipStream_t s);
hipError_t launch_jump(int32_t* pi, int32_t n, Ctrl* ctrl, hipStream_t s);

// Hot-word LDS cache of the giant bitmap (kernels_hot.hip): `slots`
// direct-mapped slots (16384 or 32768); tags[t] = k means slot t caches bitmap
// word k * slots + t.  Global tag/value arrays hold kHotSlotsMax words.
constexpr int kHotSlotsMax = 32768;
// Vertex table: kVertSets sets of kVertWays one-byte slots; slot 2s + w holds
// the tag k of the vertex k * kVertSets + s (k < kVertTagNone; kVertTagNone
// marks an empty slot).  In device memory: the tags (kVertSlots bytes), then
// one member flag per slot (kVertSlots bytes; 1 = in the giant component).
constexpr int kVertSets = 5 << 14;  // 81,920
constexpr int kVertWays = 2;
constexpr int kVertSlots = kVertSets * kVertWays;  // 163,840 bytes = all 160 KiB of LDS
constexpr uint32_t kVertTagNone = 255;
// Selection sample: up to kVertRuns runs of 64 entries, kVRunsPerPart runs per
// workgroup part; sets grouped in kVBuckets buckets of kVBucketSets.
constexpr int64_t kVertRuns = int64_t(1) << 15;
constexpr int kVRunsPerPart = 128;
constexpr int kVPartsMax = (int)(kVertRuns / kVRunsPerPart);
constexpr int kVPartCap = kVRunsPerPart * 64 * 2;  // endpoints of one part
constexpr int kVBucketSets = 64;
constexpr int kVBuckets = kVertSets / kVBucketSets;
// Scratch words used by launch_hot_vprepare.
constexpr int64_t kVertScratchWords = (int64_t)kVPartsMax * kVPartCap + 2LL * kVPartsMax * kVBuckets;
// For every set, the kVertWays most sampled vertices (scratch:
// kVertScratchWords words); member flags are filled by launch_hot_vvalues.
hipError_t launch_hot_vprepare(const int32_t* u, const int32_t* v, int64_t m, int32_t n,
                               uint32_t* scratch, uint8_t* table, hipStream_t s);
// Every slot's member flag from the bitmap; no-op unless ctrl->filter_on.
hipError_t launch_hot_vvalues(const uint32_t* bits, uint8_t* table, const Ctrl* ctrl, hipStream_t s);
// Filtered Atomic-Hook of entries [begin, end) with the vertex table in LDS.
hipError_t launch_ahook_hotv(const int32_t* u, const int32_t* v, int64_t begin, int64_t end,
                             int32_t* pi, int32_t n, Ctrl* ctrl, const uint32_t* bits,
                             const uint8_t* table, bool halve, bool sym, hipStream_t s);
// Counts sampled endpoints per bitmap word (counts: ceil(n/32) words of
// scratch) and picks the hottest word for every slot.
hipError_t launch_hot_prepare(const int32_t* u, const int32_t* v, int64_t m, int32_t n,
                              uint32_t* counts, uint32_t* tags, int slots, hipStream_t s);
// vals[t] = bits[tags[t] * slots + t]; no-op unless ctrl->filter_on.
hipError_t launch_hot_values(const uint32_t* bits, const uint32_t* tags, uint32_t* vals,
                             const Ctrl* ctrl, int slots, hipStream_t s);
// Filtered Atomic-Hook of entries [begin, end) answering bit tests from the
// LDS copy of (tags, vals) when possible (persistent, one workgroup per CU).
hipError_t launch_ahook_hot(const int32_t* u, const int32_t* v, int64_t begin, int64_t end,
                            int32_t* pi, int32_t n, Ctrl* ctrl, const uint32_t* bits,
                            const uint32_t* tags, const uint32_t* vals, int ept, int slots,
                            bool halve, bool sym, hipStream_t s);

// CSR adjacency (kernels_csr.hip): Atomic-Hook of entries [begin, end) of
// col[], the first endpoint of entry i being its row; `bits` non-null applies
// the giant filter; `sym` hooks only col > row; `plain` runs the atomic-free
// Hook (Fig. 2) instead (no filter, no halving).
hipError_t launch_ahook_csr(const int64_t* row_ptr, const int32_t* col, int32_t n, int64_t begin,
                            int64_t end, int32_t* pi, Ctrl* ctrl, const uint32_t* bits, bool sym,
                            bool halve, bool plain, hipStream_t s);
// CSR hybrid: the entries whose endpoints' roots differ (pi a forest of stars)
// as root pairs in fr[0 .. *count) (capacity m; *count accumulated).
hipError_t launch_compact_csr(const int64_t* row_ptr, const int32_t* col, int32_t n, int64_t m,
                              const int32_t* pi, int2* fr, uint32_t* count, bool sym,
                              hipStream_t s);
// Sets the range bit unless row_ptr[0] == 0, row_ptr[n] == m and row_ptr is
// non-decreasing.
hipError_t launch_csr_check(const int64_t* row_ptr, int32_t n, int64_t m, Ctrl* ctrl,
                            hipStream_t s);

// Streaming and gather probes used to measure the memory ceilings.
hipError_t launch_probe_stream(const int32_t* u, const int32_t* v, int64_t m, uint32_t* sink,
                               hipStream_t s);
hipError_t launch_probe_gather(const int32_t* u, const int32_t* v, int64_t m, const int32_t* table,
                               int32_t n, uint32_t* sink, hipStream_t s);
// Stream + one agent-scope compare-and-swap per entry on table[u] (table
// must hold table[x] = x; it is left unchanged): succeeding or failing form.
hipError_t launch_probe_cas(const int32_t* u, const int32_t* v, int64_t m, int32_t* table,
                            int32_t n, bool fail, uint32_t* sink, hipStream_t s);
// Memory-model probe (modes 7-9, see kernels_probe.hip): t is int32[128].
hipError_t launch_probe_mm(int mode, int32_t* t, hipStream_t s);
hipError_t launch_probe_bitgather(const int32_t* u, const int32_t* v, int64_t m,
                                  const uint32_t* bits, int32_t n, int variant, uint32_t* sink,
                                  hipStream_t s);

// Batched solve: one workgroup per graph, tree array in LDS, graphs taken
// from a device work queue in the order of `descs`; `grid` = CU count, and
// each CU runs as many `block`-thread workgroups as the LDS allows.
hipError_t prepare_batch_lds();  // once per process, before the first launch
hipError_t launch_batch_lds(const GraphDesc* descs, int32_t count, int32_t max_n,
                            int32_t* queue_head, int32_t* status, bool halve, int grid,
                            hipStream_t s, int block = 1024);

// Descriptors of a batch with device offsets, largest first (two launches,
// one thread per graph, with a scan launch between them above 32,768
// graphs); `rows` is scratch of (ceil(B / 1024) + 1) x 256 int32.
// Clears ctrl->queue_head; status[1] / status[2] get kStatusBadGraph /
// kStatusRange for invalid graphs (status may be pinned host memory).
hipError_t launch_batch_prep(const int64_t* vo, const int64_t* eo, int32_t B, const int32_t* u,
                             const int32_t* v, int32_t* out, int32_t max_n, int32_t seg_cap,
                             GraphDesc* descs, int32_t* rows, Ctrl* ctrl, int32_t* status,
                             hipStream_t s);

// Zeroes `words` 32-bit words with a kernel (graph-capture friendly).
hipError_t launch_zero(void* p, int64_t words, hipStream_t s);

int device_cu_count();

}  // namespace hookcc
