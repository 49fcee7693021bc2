// Internal definitions shared by the HIP kernels and the host engine of
// libhookcc.  Not part of the public ABI (include/hookcc.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hookcc {

// Device control block, the first 256 bytes of every workspace.
// Written and read only by the kernels, except that the host zeroes it at the
// start of a solve (through the init kernel) and reads it once at the end.
struct Ctrl {
    int32_t status;       // bit 0: an endpoint outside [0, n); bit 1: frontier overflow
    int32_t giant;        // sampled giant-component label (-1 = none)
    int32_t filter_on;    // 1 when the giant-component bitmap is valid and worth using
    int32_t rounds;       // atomic-free Hook: rounds that found an active edge
    uint32_t count[2];    // atomic-free Hook: frontier sizes, ping-pong by round parity
    uint32_t nofilter;    // giant sample: 1 when no component is large enough to filter
    int32_t queue_head;   // batched solve: next position of the graph work queue
    int64_t active_round1;  // atomic-free Hook: frontier size after round 1
    int32_t hook_changed;   // host-loop form of Fig. 1: a Hook pass found an active edge
    int32_t jump_changed;   // host-loop form of Fig. 1: a Jump pass moved a pointer
    // atomic-free Hook, by round parity r & 1 (written by round r's compaction):
    int32_t fsel[2];        // where round r's source is: frontier buffer 0 / 1, or 2 = input lists
    uint32_t fsize[2];      // round r's source size
    int32_t fwrote[2];      // 1 = round r wrote its survivors to the other buffer
    uint32_t win_far;       // hybrid plan: entries the window round hooked outside LDS
    int32_t pad[45];
};
static_assert(sizeof(Ctrl) == 256, "control block is one 256-byte line");

constexpr int32_t kStatusRange = 1;
constexpr int32_t kStatusOverflow = 2;
constexpr int32_t kStatusBadGraph = 4;  // batch offsets: not from 0, decreasing, or n > max_n

// Graph descriptor used by the batched kernels (one per graph, in device
// memory).  Endpoints are local ids in [0, n); labels are local.
struct GraphDesc {
    const int32_t* u;
    const int32_t* v;
    int32_t* out;
    int64_t m;
    int32_t n;
    int32_t segments;
};
static_assert(sizeof(GraphDesc) == 40, "descriptor layout");

// Accesses of the tree array pi.
//
// The races on pi are part of the method (concurrent hooks and jumps,
// Section 3): every value pi[x] ever holds is x itself or a vertex of x's
// tree smaller than x (trees only merge), so a load that returns an
// out-of-date value still returns a valid pointer.  The climbing loops only
// need that (each kernel states why it stays correct and finite), so loads
// are relaxed atomics of WORKGROUP scope: ordinary cached accesses on gfx950
// that hit in L1 / the XCD's L2 and may not yet see a value another XCD wrote
// during the same kernel.  Kernel boundaries make every earlier write
// visible.  Stores are workgroup scope too in kernels where no thread takes
// a root by CAS (Multi-Jump, the atomic-free Hook).  In a kernel that hooks
// by CAS, every write is AGENT scope: the CAS itself and the path-halving
// store (halve_to).  COH = true makes the loads and stores agent scope as
// well (coherent across XCDs, served beyond the per-XCD L2); it is kept for
// measurement.
template <bool COH>
__device__ __forceinline__ int32_t ld_tree(const int32_t* p) {
    if (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <bool COH>
__device__ __forceinline__ void st_tree(int32_t* p, int32_t x) {
    if (COH) __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int32_t ld_rlx(const int32_t* p) { return ld_tree<false>(p); }
__device__ __forceinline__ void st_rlx(int32_t* p, int32_t x) { st_tree<false>(p, x); }
__device__ __forceinline__ int32_t cas_root(int32_t* p, int32_t expected, int32_t desired) {
    __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return expected;  // the value found (== the old expected on success)
}
// Path-halving re-point of a non-root x to a vertex a < x of its tree during
// a kernel that also hooks roots by cas_root.  Every write to pi in such a
// kernel is of agent scope, like the CAS: a workgroup-scope store there (a
// write-back line in one XCD's L2) races with the agent-scope CAS of other
// XCDs on the same words, and on gfx950 that mix has lost hooks (wrong
// labels, at random, on deep trees).  Concurrent re-points of one slot may
// land in any order: each value is in the slot's tree and below its index,
// so the partition into trees and the termination argument do not depend on
// which one stays.
__device__ __forceinline__ void halve_to(int32_t* p, int32_t a) {
    __hip_atomic_store(p, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// A climb re-points on one of every kHalveEvery* of its steps that can
// re-point (steps 1, 1 + k, 1 + 2k, ...): an agent-scope store goes past
// the L2, so fewer of them is faster until the trees grow deep enough to
// lengthen the climbs and the Multi-Jump.  Measured on gfx950: every 4th
// step for the unfiltered Atomic-Hook (percolated 4096^2 grid: 1.10 ms
// against 1.17 every 2nd and 1.33 every 16th), every 8th for the filtered
// kernels, whose climbs start from stars (R-MAT 24: 4.63 ms against 4.67).
constexpr uint32_t kHalveEveryCore = 4;
constexpr uint32_t kHalveEveryFiltered = 8;

}  // namespace hookcc
