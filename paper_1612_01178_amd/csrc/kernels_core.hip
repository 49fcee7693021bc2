// Core kernels of the adaptive Hook-Compress solver for CDNA4 (gfx950).
//
//   k_init        pi[v] = v                                   (Fig. 4, first step)
//   k_ahook       Atomic-Hook over an edge segment            (Fig. 3, top)
//   k_mj          Multi-Jump: a whole Compress in one launch  (Fig. 3, bottom)
//   k_sample      giant-component label from sampled endpoints
//   k_bitmap      bitmap of the giant component's vertices
//   k_hook_plain  atomic-free Hook                            (Fig. 2)
//   k_compact     frontier compaction of still-active edges
//
// Nothing here is a dense contraction, so there is no MFMA: the kernels are
// bound by the coalesced int32 edge stream from HBM and by random 4-byte
// gathers of the tree array pi (L2 / Infinity Cache).  Edge entries are read
// with 16-byte non-temporal vector loads so the stream does not evict pi from
// the caches; tree loads are cached relaxed atomics, and the scope of tree
// writes follows the rule stated in common.hpp.
#include "kernels.hpp"

namespace hookcc {

typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef uint32_t v2u __attribute__((ext_vector_type(2)));

// ----------------------------------------------------------------------------- helpers
// Number of set bits of `mask` in lanes below this one (wave64 lane prefix).
__device__ __forceinline__ uint32_t lane_prefix(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Loads EPT entries of one edge array for this thread: EPT/4 groups of 4
// consecutive entries, group k at e0 + k * stride.  Slots outside [.., end)
// read as vertex 0 and are reported in `valid`.
template <int EPT, bool VEC>
__device__ __forceinline__ void load_edges(const int32_t* __restrict__ p, int64_t e0, int64_t stride,
                                           int64_t end, int32_t (&x)[EPT]) {
#pragma unroll
    for (int k = 0; k < EPT / 4; ++k) {
        const int64_t e = e0 + k * stride;
        if (VEC && e + 3 < end) {
            v4i q = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(p + e));
            x[4 * k + 0] = q.x;
            x[4 * k + 1] = q.y;
            x[4 * k + 2] = q.z;
            x[4 * k + 3] = q.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                x[4 * k + j] = (e + j < end) ? __builtin_nontemporal_load(p + e + j) : 0;
        }
    }
}

// Atomic-Hook of one edge whose endpoints' current parents are (pu, pv)
// (Fig. 3, top; Section 3.A).  While the two parents differ, the larger one,
// H, is hooked under the smaller one, L, by a compare-and-swap that succeeds
// only if H is still a root (pi[H] == H), so no existing link is ever
// overwritten.  When H already has a parent, the pair to join becomes
// (parent of that parent, parent of L), one level up.  A cached read of pi[H]
// comes first: if it already shows a parent (values only decrease, so it
// cannot be wrong about that), the doomed CAS is skipped and the climb uses
// the value read; only apparent roots are CAS'd.  Every value written is
// smaller than the slot's index, so no cycle can form, and the loop ends
// because max(pu, pv) strictly decreases (every value read at a slot is at
// most the slot's index, and below it once the slot is not a root).
//
// HALVE (not in the paper): on the way up, a non-root H whose grandparent
// differs from its parent is re-pointed at the grandparent (path halving, as
// in sequential union-find; here on every kHalveEveryCore-th such step) by an
// agent-scope store (halve_to).  H
// is already a non-root, so no CAS on it can succeed any more, and the value
// written is in H's tree and smaller than H: the partition into trees is
// unchanged and later climbs through H are shorter.
template <bool COH, bool HALVE>
__device__ __forceinline__ void atomic_hook(int32_t* pi, int32_t pu, int32_t pv) {
    uint32_t step = 0;
    while (pu != pv) {
        const int32_t H = pu > pv ? pu : pv;
        const int32_t L = pu > pv ? pv : pu;
        int32_t found = ld_tree<COH>(pi + H);
        if (found == H) {
            found = cas_root(pi + H, H, L);
            if (found == H) return;
        }
        pu = ld_tree<COH>(pi + found);
        pv = ld_tree<COH>(pi + L);
        if (HALVE && pu != found && step++ % kHalveEveryCore == 0) halve_to(pi + H, pu);
    }
}

// ----------------------------------------------------------------------------- K-INIT
template <bool VEC>
__global__ __launch_bounds__(256) void k_init(int32_t* __restrict__ pi, int32_t n, Ctrl* ctrl) {
    const int64_t base = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (VEC && base + 3 < n) {
        v4i q = {(int32_t)base, (int32_t)base + 1, (int32_t)base + 2, (int32_t)base + 3};
        *reinterpret_cast<v4i*>(pi + base) = q;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (base + j < n) pi[base + j] = (int32_t)(base + j);
    }
    if (blockIdx.x == 0 && threadIdx.x < sizeof(Ctrl) / 4) {
        // status, giant (-1), filter_on, rounds, counts, ... all zero
        reinterpret_cast<int32_t*>(ctrl)[threadIdx.x] = (threadIdx.x == 1) ? -1 : 0;
    }
}

hipError_t launch_init(int32_t* pi, int32_t n, Ctrl* ctrl, hipStream_t s) {
    const int64_t groups = ((int64_t)n + 3) / 4;
    const int grid = (int)((groups + 255) / 256 > 0 ? (groups + 255) / 256 : 1);
    if (((uintptr_t)pi & 15) == 0)
        k_init<true><<<grid, 256, 0, s>>>(pi, n, ctrl);
    else
        k_init<false><<<grid, 256, 0, s>>>(pi, n, ctrl);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------- K-AHOOK
// Each thread takes EPT entries of [begin, end): EPT/4 groups of 4 consecutive
// entries, consecutive lanes on consecutive groups (fully coalesced 16-byte
// loads).  All 2*EPT parent gathers are issued before any climbing so that
// their latencies overlap.  Endpoints outside [0, n) raise the range bit of
// the status word and are skipped.
//
// FILTER: when ctrl->filter_on, bit v of `bits` says v's tree contained the
// giant component's sampled root g when the bitmap was built; trees only
// merge, so v stays joined to g.  An entry with both bits set is already
// satisfied and is skipped; an endpoint with its bit set starts its climb at
// g instead of gathering pi (any vertex of the endpoint's tree is a valid
// start for Atomic-Hook, since only tree membership matters).
template <int EPT, bool VEC, bool FILTER, bool COH, bool HALVE>
__global__ __launch_bounds__(1024) void k_ahook(const int32_t* __restrict__ eu,
                                                const int32_t* __restrict__ ev, int64_t begin,
                                                int64_t end, int32_t* pi, int32_t n, Ctrl* ctrl,
                                                const uint32_t* __restrict__ bits, bool sym) {
    const int64_t stride = (int64_t)blockDim.x * 4;
    const int64_t e0 = begin + (int64_t)blockIdx.x * blockDim.x * EPT + (int64_t)threadIdx.x * 4;
    int32_t a[EPT], b[EPT];
    load_edges<EPT, VEC>(eu, e0, stride, end, a);
    load_edges<EPT, VEC>(ev, e0, stride, end, b);

    uint32_t act = 0;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const bool in = (uint32_t)a[j] < (uint32_t)n && (uint32_t)b[j] < (uint32_t)n;
        bad |= !in;
        // sym: the caller's list holds every pair in both orientations; hook one
        if (in && a[j] != b[j] && !(sym && a[j] > b[j])) act |= 1u << j;
    }
    if (bad) atomicOr(&ctrl->status, kStatusRange);

    int32_t pa[EPT], pb[EPT];
    if (FILTER && ctrl->filter_on) {
        const int32_t g = ctrl->giant;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (act >> j & 1) {
                const uint32_t ba = bits[(uint32_t)a[j] >> 5] >> (a[j] & 31) & 1;
                const uint32_t bb = bits[(uint32_t)b[j] >> 5] >> (b[j] & 31) & 1;
                if (ba & bb) {
                    act &= ~(1u << j);
                } else {
                    pa[j] = ba ? g : ld_tree<COH>(pi + a[j]);
                    pb[j] = bb ? g : ld_tree<COH>(pi + b[j]);
                }
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (act >> j & 1) {
                pa[j] = ld_tree<COH>(pi + a[j]);
                pb[j] = ld_tree<COH>(pi + b[j]);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j)
        if (act >> j & 1) atomic_hook<COH, HALVE>(pi, pa[j], pb[j]);
}

template <int EPT, bool FILTER, bool COH>
static void ahook_dispatch(bool vec, bool halve, int grid, int block, hipStream_t s,
                           const int32_t* u, const int32_t* v, int64_t begin, int64_t end,
                           int32_t* pi, int32_t n, Ctrl* ctrl, const uint32_t* bits, bool sym) {
    if (vec && halve)
        k_ahook<EPT, true, FILTER, COH, true><<<grid, block, 0, s>>>(u, v, begin, end, pi, n, ctrl, bits, sym);
    else if (vec)
        k_ahook<EPT, true, FILTER, COH, false><<<grid, block, 0, s>>>(u, v, begin, end, pi, n, ctrl, bits, sym);
    else if (halve)
        k_ahook<EPT, false, FILTER, COH, true><<<grid, block, 0, s>>>(u, v, begin, end, pi, n, ctrl, bits, sym);
    else
        k_ahook<EPT, false, FILTER, COH, false><<<grid, block, 0, s>>>(u, v, begin, end, pi, n, ctrl, bits, sym);
}

template <int EPT>
static void ahook_dispatch2(bool vec, bool filter, bool coh, bool halve, int grid, int block,
                            hipStream_t s, const int32_t* u, const int32_t* v, int64_t begin,
                            int64_t end, int32_t* pi, int32_t n, Ctrl* ctrl, const uint32_t* bits,
                            bool sym) {
    if (filter) {
        if (coh) ahook_dispatch<EPT, true, true>(vec, halve, grid, block, s, u, v, begin, end, pi, n, ctrl, bits, sym);
        else ahook_dispatch<EPT, true, false>(vec, halve, grid, block, s, u, v, begin, end, pi, n, ctrl, bits, sym);
    } else {
        if (coh) ahook_dispatch<EPT, false, true>(vec, halve, grid, block, s, u, v, begin, end, pi, n, ctrl, bits, sym);
        else ahook_dispatch<EPT, false, false>(vec, halve, grid, block, s, u, v, begin, end, pi, n, ctrl, bits, sym);
    }
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

hipError_t launch_ahook(const int32_t* u, const int32_t* v, int64_t begin, int64_t end,
                        int32_t* pi, int32_t n, Ctrl* ctrl, const uint32_t* bits, int block,
                        int ept, bool coherent, bool halve, bool sym, hipStream_t s) {
    if (end <= begin) return hipSuccess;
    const int64_t tile = (int64_t)block * ept;
    const int64_t grid64 = (end - begin + tile - 1) / tile;
    if (grid64 > 0x7fffffff) return hipErrorInvalidValue;
    const int grid = (int)grid64;
    const bool vec = aligned16(u + begin) && aligned16(v + begin);
    const bool f = bits != nullptr;
    switch (ept) {
        case 4: ahook_dispatch2<4>(vec, f, coherent, halve, grid, block, s, u, v, begin, end, pi, n, ctrl, bits, sym); break;
        case 8: ahook_dispatch2<8>(vec, f, coherent, halve, grid, block, s, u, v, begin, end, pi, n, ctrl, bits, sym); break;
        case 16: ahook_dispatch2<16>(vec, f, coherent, halve, grid, block, s, u, v, begin, end, pi, n, ctrl, bits, sym); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ----------------------------------------------------------------------------- K-MJ
// 256-vertex chunks per wave in k_mj and k_mj_bitmap (two measured the same as
// one on R-MAT 24: the hoisted loads were what paid)
constexpr int kMjChunks = 1;

// Multi-Jump (Fig. 3, bottom): for every vertex, while its grandparent
// differs from its parent, replace the parent by the grandparent.  The new
// parent is stored on every step, not once at the end, so that other threads
// climbing through this vertex see the shortened path at once (the first of
// the two optimisations of Section 3.A).  Workgroups cover the vertex range in
// increasing id order, so the low ids near the roots are flattened first (the
// second optimisation; the hardware dispatches workgroups in index order).
// Each lane handles 4 consecutive vertices from one 16-byte load in each of CH
// chunks of 256 vertices per wave (wave w covers vertices [256 CH w,
// 256 CH (w + 1))); roots are skipped at once; the chunks' loads and their
// grandparent gathers are issued together (the pass is bound by the latency
// of these dependent loads, not by bandwidth).
//
// During a Multi-Jump no root changes (only non-roots are written, and only
// with ancestors), so "grandparent == parent" holds exactly when the parent is
// a root: on exit every vertex points at its tree's root, i.e. at the minimum
// id of its tree.
template <bool VEC, bool COH, int CH>
__global__ __launch_bounds__(256) void k_mj(int32_t* pi, int32_t n, const uint32_t* gate) {
    if (gate != nullptr && *gate == 0) return;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    int64_t base[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) base[c] = (wave * CH + c) * 256 + 4 * lane;
    int32_t p[CH][4];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        if (VEC && base[c] + 3 < n) {
            v4i q = *reinterpret_cast<const v4i*>(pi + base[c]);
            p[c][0] = q.x;
            p[c][1] = q.y;
            p[c][2] = q.z;
            p[c][3] = q.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                p[c][j] = (base[c] + j < n) ? ld_tree<COH>(pi + base[c] + j) : (int32_t)(base[c] + j);
        }
    }
    int32_t gp[CH][4];
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            gp[c][j] = (p[c][j] != base[c] + j) ? ld_tree<COH>(pi + p[c][j]) : p[c][j];
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int32_t q = p[c][j], g = gp[c][j];
            while (g != q) {
                st_tree<COH>(pi + base[c] + j, g);
                q = g;
                g = ld_tree<COH>(pi + q);
            }
        }
}

// Multi-Jump for deep trees (after an atomic-free Hook round every vertex
// points at a neighbour, and on a percolated grid the trees are chains of up
// to ~150 levels, which a per-vertex climb walks one dependent load at a
// time: 0.33 ms on a 4096^2 grid).  k_mj_local first takes kMjBlock
// consecutive vertices per workgroup into LDS and, in rounds, replaces every
// parent that lies inside the block by its own parent, until each vertex
// points at a root or outside the block, and writes back the changed
// entries; the Multi-Jump that follows then climbs across blocks only (a
// 4096^2 grid: 0.6 block exits per path on average).  Every value written
// is an ancestor, so pi stays a forest with pi[x] <= x.  No hook runs
// concurrently.
constexpr int kMjBlock = 16384;

__global__ __launch_bounds__(1024, 8) void k_mj_local(int32_t* pi, int32_t n) {
    __shared__ int32_t lp[kMjBlock];
    constexpr int kPer = kMjBlock / 1024;
    const int64_t base = (int64_t)blockIdx.x * kMjBlock;
    const int cnt = (int)min<int64_t>(kMjBlock, (int64_t)n - base);
    auto lds_ld = [&](int i) { return __hip_atomic_load(lp + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); };
    auto lds_st = [&](int i, int32_t x) { __hip_atomic_store(lp + i, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); };
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int i = k * 1024 + (int)threadIdx.x;
        if (i < cnt) lds_st(i, pi[base + i]);
    }
    __syncthreads();
    uint32_t dirty = 0;  // bit k: entry k of this thread changed
    constexpr int kGroup = 4;  // entries whose loads are in flight together
    while (true) {
        bool changed = false;
#pragma unroll
        for (int h = 0; h < kPer; h += kGroup) {
            int32_t pv[kGroup], gv[kGroup];
#pragma unroll
            for (int k = 0; k < kGroup; ++k) {
                const int i = (h + k) * 1024 + (int)threadIdx.x;
                pv[k] = i < cnt ? lds_ld(i) : (int32_t)(base + i);
            }
#pragma unroll
            for (int k = 0; k < kGroup; ++k) {
                const int i = (h + k) * 1024 + (int)threadIdx.x;
                const int64_t q = (int64_t)pv[k] - base;
                const bool inside = i < cnt && q >= 0 && q < cnt && q != i;
                gv[k] = lds_ld(inside ? (int)q : 0);
                if (!inside) gv[k] = pv[k];
            }
#pragma unroll
            for (int k = 0; k < kGroup; ++k) {
                if (gv[k] != pv[k]) {
                    lds_st((h + k) * 1024 + (int)threadIdx.x, gv[k]);
                    dirty |= 1u << (h + k);
                    changed = true;
                }
            }
        }
        if (!__syncthreads_or(changed)) break;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k)
        if (dirty >> k & 1) {
            const int i = k * 1024 + (int)threadIdx.x;
            st_tree<false>(pi + base + i, lds_ld(i));
        }
}

// Multi-Jump with one-word loads, for the atomic-free and hybrid paths:
// after k_mj_local, or after a round that hooked roots, most climbs are a
// dependent load or two, and k_mj's four consecutive vertices per thread
// would run their climbs one after the other (a 4096^2 grid: 0.575 -> 0.537
// ms; ER 2^16 rounds: 0.100 -> 0.090 ms); here a thread's V vertices climb
// interleaved.  The Atomic-Hook path keeps k_mj, whose 16-byte loads win on
// its shallow trees (R-MAT 24: 3.75 against 3.78 ms).
template <int V>
__global__ __launch_bounds__(256) void k_mj1(int32_t* pi, int32_t n, const uint32_t* gate,
                                             uint32_t limit) {
    if (gate != nullptr && *gate <= limit) return;
    // V vertices per thread and pass (v, v + blockDim.x, ...: every load
    // coalesced), their climbs interleaved so that each thread keeps V
    // dependent loads in flight; a finished climb stays on its root, whose
    // parent is itself.  Each vertex's root is stored once, if it is not
    // already its parent.
    const int64_t step = (int64_t)gridDim.x * blockDim.x * V;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x * V + threadIdx.x; v < n; v += step) {
        int32_t q[V], r[V], g[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const int64_t w = v + (int64_t)k * blockDim.x;
            // past n: vertex 0, always a root (pi[x] <= x), so that climb ends at once
            q[k] = w < n ? ld_tree<false>(pi + w) : 0;
        }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            r[k] = q[k];
            g[k] = ld_tree<false>(pi + r[k]);
        }
        bool more = false;
#pragma unroll
        for (int k = 0; k < V; ++k) more |= g[k] != r[k];
        while (more) {
            more = false;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                r[k] = g[k];
                g[k] = ld_tree<false>(pi + r[k]);
                more |= g[k] != r[k];
            }
        }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const int64_t w = v + (int64_t)k * blockDim.x;
            if (w < n && r[k] != q[k]) st_tree<false>(pi + w, r[k]);
        }
    }
}

// k_mj1 with V vertices per thread: four where that still gives every CU at
// least 8 workgroups (a 4096^2 grid's final Multi-Jump: 42 -> 35 us; eight
// per thread no better), else two (ER 2^16: four leaves 64 workgroups).
static hipError_t mj1_launch(int32_t* pi, int32_t n, const uint32_t* gate, uint32_t limit,
                             bool capped, hipStream_t s) {
    const int64_t cus = device_cu_count();
    const int V = (int64_t)n >= 256 * 4 * 8 * cus ? 4 : 2;
    int64_t grid = ((int64_t)n + 256 * V - 1) / (256 * V);
    if (capped) grid = std::min<int64_t>(grid, cus * 32);
    if (V == 4)
        k_mj1<4><<<(int)grid, 256, 0, s>>>(pi, n, gate, limit);
    else
        k_mj1<2><<<(int)grid, 256, 0, s>>>(pi, n, gate, limit);
    return hipGetLastError();
}

hipError_t launch_mj_deep(int32_t* pi, int32_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    // below ~256 blocks the GPU is not filled and the plain Multi-Jump wins
    if (n < (1 << 22)) return launch_mj1(pi, n, nullptr, s);
    const int grid = (int)(((int64_t)n + kMjBlock - 1) / kMjBlock);
    k_mj_local<<<grid, 1024, 0, s>>>(pi, n);
    return mj1_launch(pi, n, nullptr, 0, false, s);
}

hipError_t launch_mj1(int32_t* pi, int32_t n, const uint32_t* gate, hipStream_t s,
                      uint32_t limit) {
    if (n <= 0) return hipSuccess;
    // a gated launch may find nothing to do: a grid of at most 32 workgroups
    // per CU, each thread striding over vertices, exits in a few microseconds
    return mj1_launch(pi, n, gate, limit, gate != nullptr, s);
}

hipError_t launch_mj(int32_t* pi, int32_t n, const uint32_t* gate, bool coherent, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t waves = ((int64_t)n + 256 * kMjChunks - 1) / (256 * kMjChunks);
    const int grid = (int)((waves + 3) / 4);
    const bool vec = ((uintptr_t)pi & 15) == 0;
    if (vec && coherent) k_mj<true, true, kMjChunks><<<grid, 256, 0, s>>>(pi, n, gate);
    else if (vec) k_mj<true, false, kMjChunks><<<grid, 256, 0, s>>>(pi, n, gate);
    else if (coherent) k_mj<false, true, kMjChunks><<<grid, 256, 0, s>>>(pi, n, gate);
    else k_mj<false, false, kMjChunks><<<grid, 256, 0, s>>>(pi, n, gate);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------- giant sample
// One workgroup.  Sample i reads edge entry floor(i * m / S) (evenly spread
// over the list), takes the root of its first endpoint (pi is a forest of
// stars, so that is pi[u]), and counts roots in an LDS hash table
// (open addressing, 2*S slots).  The most frequent root is the giant label;
// the filter is switched on when it holds at least 1/8 of the samples.
constexpr int kSampleMax = 2048;

__global__ __launch_bounds__(1024) void k_sample(const int32_t* __restrict__ eu, int64_t m,
                                                 const int32_t* pi, int32_t n, Ctrl* ctrl, int S) {
    __shared__ int32_t keys[2 * kSampleMax];
    __shared__ int32_t cnts[2 * kSampleMax];
    __shared__ int32_t best_cnt[16];
    __shared__ int32_t best_key[16];
    constexpr int kSlots = 2 * kSampleMax;
    for (int i = threadIdx.x; i < kSlots; i += blockDim.x) {
        keys[i] = -1;
        cnts[i] = 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < S; i += blockDim.x) {
        const int64_t e = (int64_t)i * m / S;
        const int32_t x = eu[e];
        if ((uint32_t)x >= (uint32_t)n) continue;
        const int32_t r = ld_rlx(pi + x);
        uint32_t slot = ((uint32_t)r * 2654435761u) & (kSlots - 1);
        for (int probe = 0; probe < kSlots; ++probe) {
            const int32_t k = atomicCAS(&keys[slot], -1, r);
            if (k == -1 || k == r) {
                atomicAdd(&cnts[slot], 1);
                break;
            }
            slot = (slot + 1) & (kSlots - 1);
        }
    }
    __syncthreads();
    int bc = -1, bk = -1;
    for (int i = threadIdx.x; i < kSlots; i += blockDim.x) {
        if (cnts[i] > bc) {
            bc = cnts[i];
            bk = keys[i];
        }
    }
    // wave reduction (max count)
    for (int off = 32; off > 0; off >>= 1) {
        const int oc = __shfl_xor(bc, off);
        const int ok = __shfl_xor(bk, off);
        if (oc > bc) {
            bc = oc;
            bk = ok;
        }
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        best_cnt[wave] = bc;
        best_key[wave] = bk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int waves = (blockDim.x + 63) >> 6;
        int c = best_cnt[0], k = best_key[0];
        for (int w = 1; w < waves; ++w)
            if (best_cnt[w] > c) {
                c = best_cnt[w];
                k = best_key[w];
            }
        const bool on = k >= 0 && c * 8 >= S;
        ctrl->giant = on ? k : -1;
        ctrl->filter_on = on ? 1 : 0;
        ctrl->nofilter = on ? 0u : 1u;
    }
}

hipError_t launch_sample_giant(const int32_t* u, int64_t m, const int32_t* pi, int32_t n,
                               Ctrl* ctrl, int samples, hipStream_t s) {
    if (samples > kSampleMax) samples = kSampleMax;
    if (samples < 1 || m <= 0) return hipSuccess;
    k_sample<<<1, 1024, 0, s>>>(u, m, pi, n, ctrl, samples);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------- bitmap
// Each wave covers 256 consecutive vertices in 4 coalesced steps of 64; a
// ballot turns each step's predicate into 64 bits (2 words); lanes 0..7 store
// the wave's 8 words.  The giant's current root is re-read first (it may have
// been hooked under a smaller root since the sample), and stored back.
__global__ __launch_bounds__(256) void k_bitmap(const int32_t* pi, int32_t n, Ctrl* ctrl,
                                                uint32_t* __restrict__ bits) {
    if (!ctrl->filter_on) return;
    const int32_t g = ld_rlx(pi + ctrl->giant);
    const int lane = threadIdx.x & 63;
    const int64_t wave_base = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 256;
    uint64_t m4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t x = wave_base + 64 * k + lane;
        const bool in = x < n && ld_rlx(pi + x) == g;
        m4[k] = __ballot(in);
    }
    if (lane < 8) {
        const int64_t w = wave_base / 32 + lane;
        if (w * 32 < n) {
            const uint64_t mk = m4[lane >> 1];
            bits[w] = (lane & 1) ? (uint32_t)(mk >> 32) : (uint32_t)mk;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->giant = g;
}

hipError_t launch_bitmap(const int32_t* pi, int32_t n, Ctrl* ctrl, uint32_t* bits, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t waves = ((int64_t)n + 255) / 256;
    const int grid = (int)((waves + 3) / 4);
    k_bitmap<<<grid, 256, 0, s>>>(pi, n, ctrl, bits);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------- MJ + bitmap
// Bits 0..7 of x moved to bits 0, 4, 8, ..., 28.
__device__ __forceinline__ uint32_t spread4(uint32_t x) {
    x = (x | (x << 12)) & 0x000F000Fu;
    x = (x | (x << 6)) & 0x03030303u;
    x = (x | (x << 3)) & 0x11111111u;
    return x;
}

// Multi-Jump (as k_mj) and, when the filter is on, the giant bitmap rebuilt
// in the same pass (as k_bitmap) and the cached words of the hot-word table
// refreshed (as k_hot_values), instead of three passes over pi.  Each lane
// jumps 4 consecutive vertices in each of CH chunks of 256 vertices per wave
// (wave w covers vertices [256 CH w, 256 CH (w + 1))) to their roots; the
// giant's current root is found by climbing from the last giant label (other
// threads' jumps only move values up, and no hook runs, so the climb ends at
// the root); a vertex's bit is (its root == that root).  Per chunk, one
// ballot per slot j (bit l = vertex 4l + j of the chunk), and lane w < 8
// assembles word w of the chunk (its vertices 32w .. 32w + 31) from byte w of
// the four ballots.  The pass is bound by the latency of its dependent loads,
// so every load that does not depend on pi (the filter switch, the giant
// label and its parent, the vertex-table tags) is issued with the first pi
// load, and the CH chunks' loads and gathers are issued together.
template <bool VEC, int CH>
__global__ __launch_bounds__(256) void k_mj_bitmap(int32_t* pi, int32_t n, Ctrl* ctrl,
                                                   uint32_t* __restrict__ bits,
                                                   const uint32_t* __restrict__ hot_tags,
                                                   uint32_t* __restrict__ hot_vals, int slots,
                                                   uint8_t* vtab) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    int64_t base[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) base[c] = (wave * CH + c) * 256 + 4 * lane;
    const int32_t fon = ctrl->filter_on;
    int32_t groot = ctrl->giant;
    int32_t up = fon ? ld_tree<false>(pi + groot) : groot;
    uint64_t tags[CH];
    bool has_tags[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        // the sets of base .. base + 3 (same tag: kVertSets is a multiple of
        // 4) and their 8 tag bytes
        has_tags[c] = fon && vtab && base[c] < n && (uint32_t)base[c] / kVertSets < kVertTagNone;
        tags[c] = has_tags[c] ? *reinterpret_cast<const uint64_t*>(vtab + 2 * ((uint32_t)base[c] % kVertSets))
                              : 0;
    }
    int32_t p[CH][4];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        if (VEC && base[c] + 3 < n) {
            v4i q = *reinterpret_cast<const v4i*>(pi + base[c]);
            p[c][0] = q.x;
            p[c][1] = q.y;
            p[c][2] = q.z;
            p[c][3] = q.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                p[c][j] = (base[c] + j < n) ? ld_tree<false>(pi + base[c] + j) : (int32_t)(base[c] + j);
        }
    }
    int32_t gp[CH][4];
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            gp[c][j] = (p[c][j] != base[c] + j) ? ld_tree<false>(pi + p[c][j]) : p[c][j];
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int32_t q = p[c][j], g = gp[c][j];
            while (g != q) {
                st_tree<false>(pi + base[c] + j, g);
                q = g;
                g = ld_tree<false>(pi + q);
            }
            p[c][j] = q;  // the root
        }
    if (!fon) return;
    while (up != groot) {
        groot = up;
        up = ld_tree<false>(pi + groot);
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        uint64_t m4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) m4[j] = __ballot(base[c] + j < n && p[c][j] == groot);
        if (has_tags[c]) {
            // a member flag is written only by the vertex its slot holds
            const uint32_t k = (uint32_t)base[c] / kVertSets;
            uint8_t* mem = vtab + kVertSlots + 2 * ((uint32_t)base[c] % kVertSets);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int w = 0; w < kVertWays; ++w)
                    if (base[c] + j < n && (uint32_t)(tags[c] >> (8 * (2 * j + w)) & 0xffu) == k)
                        mem[2 * j + w] = p[c][j] == groot ? 1 : 0;
        }
        if (lane < 8) {
            const int64_t w = (wave * CH + c) * 8 + lane;  // word of vertices 32w .. 32w + 31
            if (w * 32 < n) {
                uint32_t word = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) word |= spread4((uint32_t)(m4[j] >> (8 * lane)) & 0xffu) << j;
                bits[w] = word;
                if (hot_tags) {
                    const uint32_t slot = (uint32_t)w & (uint32_t)(slots - 1);
                    if (hot_tags[slot] == (uint32_t)(w / slots)) hot_vals[slot] = word;
                }
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->giant = groot;
}

hipError_t launch_mj_bitmap(int32_t* pi, int32_t n, Ctrl* ctrl, uint32_t* bits,
                            const uint32_t* hot_tags, uint32_t* hot_vals, int slots, uint8_t* vtab,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (hot_tags && slots != 16384 && slots != 32768) return hipErrorInvalidValue;
    const int64_t waves = ((int64_t)n + 256 * kMjChunks - 1) / (256 * kMjChunks);
    const int grid = (int)((waves + 3) / 4);
    if (((uintptr_t)pi & 15) == 0)
        k_mj_bitmap<true, kMjChunks><<<grid, 256, 0, s>>>(pi, n, ctrl, bits, hot_tags, hot_vals, slots, vtab);
    else
        k_mj_bitmap<false, kMjChunks><<<grid, 256, 0, s>>>(pi, n, ctrl, bits, hot_tags, hot_vals, slots, vtab);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------- atomic-free Hook
// Source of round `round` of the atomic-free Hook, from the record the
// previous round's compaction left: the input lists in round 1; later, the
// frontier buffer that round wrote (its survivors, count[] entries) or, when
// it did not rewrite, the same buffer it read.  `total` is 0 once the
// previous round found no active entry (converged).
struct RoundSrc {
    int32_t sel;      // 0 / 1 = frontier buffer, 2 = input lists
    int64_t total;    // entries to read
};
__device__ __forceinline__ RoundSrc round_src(const Ctrl* ctrl, int round, int64_t m) {
    RoundSrc r{2, m};
    if (round == 1) return r;
    const int p = (round - 1) & 1;
    const int64_t active = ctrl->count[p];
    if (ctrl->fwrote[p]) {
        r.sel = ctrl->fsel[p] == 0 ? 1 : 0;
        r.total = active;
    } else {
        r.sel = ctrl->fsel[p];
        r.total = active ? (int64_t)ctrl->fsize[p] : 0;
    }
    r.total = min(r.total, m);
    return r;
}

// Fig. 2 Hook: H = max(pi[u], pi[v]), L = min(...), plain store pi[H] = L.
// Concurrent stores to one slot race and all but one are lost; the round
// loop (Fig. 1) repeats until no entry is active, and every store writes a
// smaller id than the slot's index, so no cycle forms.  Round 1 reads the
// input lists (range-checked); later rounds read the frontier of root pairs
// chosen by round_src (round 1 always writes one, so no later round reads
// the input lists).  Block 0 also clears the count the following compaction
// accumulates into, and records the round.
template <int EPT, bool VEC, bool FIRST>
__global__ __launch_bounds__(1024) void k_hook_plain(int round, const int32_t* __restrict__ eu,
                                                     const int32_t* __restrict__ ev, int64_t m,
                                                     const int2* f0, const int2* f1, int32_t* pi,
                                                     int32_t n, Ctrl* ctrl) {
    const RoundSrc rs = round_src(ctrl, round, m);
    const int64_t total = rs.total;
    const int2* fr = rs.sel == 0 ? f0 : f1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->count[round & 1] = 0;
        if (total > 0) ctrl->rounds = round;
        if (round == 2) ctrl->active_round1 = total;
    }
    if (total == 0) return;
    const int64_t tile = (int64_t)blockDim.x * EPT;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < total; t0 += (int64_t)gridDim.x * tile) {
        int32_t a[EPT], b[EPT];
        const int64_t e0 = t0 + (int64_t)threadIdx.x * 4;
        if (FIRST) {
            load_edges<EPT, VEC>(eu, e0, (int64_t)blockDim.x * 4, total, a);
            load_edges<EPT, VEC>(ev, e0, (int64_t)blockDim.x * 4, total, b);
        } else {
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const int64_t e = t0 + (int64_t)(j / 4) * blockDim.x * 4 + threadIdx.x * 4 + (j & 3);
                int2 q = e < total ? fr[e] : int2{0, 0};
                a[j] = q.x;
                b[j] = q.y;
            }
        }
        uint32_t act = 0;
        bool bad = false;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const bool in = (uint32_t)a[j] < (uint32_t)n && (uint32_t)b[j] < (uint32_t)n;
            bad |= !in;
            if (in && a[j] != b[j]) act |= 1u << j;
        }
        if (FIRST && bad) atomicOr(&ctrl->status, kStatusRange);
        int32_t pa[EPT], pb[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (act >> j & 1) {
                pa[j] = ld_rlx(pi + a[j]);
                pb[j] = ld_rlx(pi + b[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if ((act >> j & 1) && pa[j] != pb[j]) {
                const int32_t H = pa[j] > pb[j] ? pa[j] : pb[j];
                const int32_t L = pa[j] > pb[j] ? pb[j] : pa[j];
                st_rlx(pi + H, L);
            }
        }
    }
}

// ----------------------------------------------------------------------------- K-COMPACT
// After the Compress of a round, an entry is still active iff its endpoints'
// roots differ (pi is a forest of stars).  Trees only merge, so an inactive
// entry never becomes active again and can be dropped for good.  Every round
// counts its active entries (count[r & 1], the convergence test); it writes
// them, as root pairs, to the other frontier buffer only in round 1 and when
// the previous round's surviving fraction (its active entries over its
// source size) was below tau / 1000 -- otherwise the next round reads this
// round's source again, dead entries included, and the rewrite is saved.
// Per wave, one 64-bit ballot per slot j gives each lane its output position
// (mbcnt lane prefix plus the counts of earlier slots); the wave totals are
// scanned in LDS, the workgroup reserves its output range with one
// atomicAdd, and the survivors, staged in LDS in that order, are written out
// as one contiguous run.
template <int EPT, bool VEC, bool FIRST>
__global__ __launch_bounds__(256) void k_compact(int round, const int32_t* __restrict__ eu,
                                                 const int32_t* __restrict__ ev, int64_t m,
                                                 int2* f0, int2* f1, int64_t cap, const int32_t* pi,
                                                 int32_t n, Ctrl* ctrl, uint32_t tau) {
    __shared__ int2 stage[256 * EPT];
    __shared__ uint32_t wave_tot[4];
    __shared__ uint32_t wave_off[4];
    __shared__ uint32_t base_sh;
    const RoundSrc rs = round_src(ctrl, round, m);
    const int64_t total = rs.total;
    const int2* src = rs.sel == 0 ? f0 : f1;
    int2* dst = rs.sel == 0 ? f1 : f0;
    bool write = true;
    if (!FIRST) {
        const int p = (round - 1) & 1;
        write = (uint64_t)ctrl->count[p] * 1000u < (uint64_t)tau * ctrl->fsize[p];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->fsel[round & 1] = rs.sel;
        ctrl->fsize[round & 1] = (uint32_t)total;
        ctrl->fwrote[round & 1] = write ? 1 : 0;
    }
    if (total == 0) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t tile = (int64_t)blockDim.x * EPT;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < total; t0 += (int64_t)gridDim.x * tile) {
        int32_t a[EPT], b[EPT];
        const int64_t e0 = t0 + (int64_t)threadIdx.x * 4;
        if (FIRST) {
            load_edges<EPT, VEC>(eu, e0, (int64_t)blockDim.x * 4, total, a);
            load_edges<EPT, VEC>(ev, e0, (int64_t)blockDim.x * 4, total, b);
        } else {
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const int64_t e = t0 + (int64_t)(j / 4) * blockDim.x * 4 + threadIdx.x * 4 + (j & 3);
                int2 q = e < total ? src[e] : int2{0, 0};
                a[j] = q.x;
                b[j] = q.y;
            }
        }
        int32_t ra[EPT], rb[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const bool in = (uint32_t)a[j] < (uint32_t)n && (uint32_t)b[j] < (uint32_t)n && a[j] != b[j];
            ra[j] = in ? ld_rlx(pi + a[j]) : 0;
            rb[j] = in ? ld_rlx(pi + b[j]) : 0;
        }
        uint32_t pos[EPT];
        uint32_t run = 0;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const uint64_t mk = __ballot(ra[j] != rb[j]);
            pos[j] = run + lane_prefix(mk);
            run += (uint32_t)__popcll(mk);
        }
        if (lane == 0) wave_tot[wave] = run;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t acc = 0;
            const int waves = blockDim.x >> 6;
            for (int w = 0; w < waves; ++w) {
                wave_off[w] = acc;
                acc += wave_tot[w];
            }
            base_sh = acc ? (uint32_t)atomicAdd(&ctrl->count[round & 1], acc) : 0u;
            wave_tot[0] = acc;  // block total (read after the barrier)
        }
        __syncthreads();
        if (!write) {
            __syncthreads();  // wave_tot / wave_off are rewritten by the next tile
            continue;
        }
        const uint32_t woff = wave_off[wave];
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            if (ra[j] != rb[j]) stage[woff + pos[j]] = int2{ra[j], rb[j]};
        __syncthreads();
        const uint32_t cnt = wave_tot[0];
        const int64_t base = base_sh;
        if (base + cnt > cap) {
            if (threadIdx.x == 0) atomicOr(&ctrl->status, kStatusOverflow);
        } else {
            for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) dst[base + i] = stage[i];
        }
        __syncthreads();
    }
}

hipError_t launch_hook_plain(int round, const int32_t* u, const int32_t* v, int64_t m,
                             const int2* f0, const int2* f1, int32_t* pi, int32_t n, Ctrl* ctrl,
                             int block, int ept, int grid_cap, hipStream_t s) {
    const int64_t tile = (int64_t)block * ept;
    int64_t grid64 = (m + tile - 1) / tile;
    if (grid64 < 1) grid64 = 1;
    if (grid64 > grid_cap) grid64 = grid_cap;
    const int grid = (int)grid64;
    const bool vec = aligned16(u) && aligned16(v);
#define HP(EPT)                                                                                  \
    do {                                                                                         \
        if (round == 1) {                                                                        \
            if (vec)                                                                             \
                k_hook_plain<EPT, true, true><<<grid, block, 0, s>>>(round, u, v, m, f0, f1, pi, n, ctrl); \
            else                                                                                 \
                k_hook_plain<EPT, false, true><<<grid, block, 0, s>>>(round, u, v, m, f0, f1, pi, n, ctrl); \
        } else {                                                                                 \
            k_hook_plain<EPT, true, false><<<grid, block, 0, s>>>(round, u, v, m, f0, f1, pi, n, ctrl); \
        }                                                                                        \
    } while (0)
    switch (ept) {
        case 4: HP(4); break;
        case 8: HP(8); break;
        case 16: HP(16); break;
        default: return hipErrorInvalidValue;
    }
#undef HP
    return hipGetLastError();
}

hipError_t launch_compact(int round, const int32_t* u, const int32_t* v, int64_t m, int2* f0,
                          int2* f1, int64_t cap, const int32_t* pi, int32_t n, Ctrl* ctrl,
                          uint32_t tau, int block, int ept, int grid_cap, hipStream_t s) {
    (void)block;  // the compaction tile is fixed at 256 threads (LDS staging size)
    const int64_t tile = 256 * (int64_t)ept;
    int64_t grid64 = (m + tile - 1) / tile;
    if (grid64 < 1) grid64 = 1;
    if (grid64 > grid_cap) grid64 = grid_cap;
    const int grid = (int)grid64;
    const bool vec = aligned16(u) && aligned16(v);
#define CP(EPT)                                                                                  \
    do {                                                                                         \
        if (round == 1) {                                                                        \
            if (vec)                                                                             \
                k_compact<EPT, true, true><<<grid, 256, 0, s>>>(round, u, v, m, f0, f1, cap, pi, n, ctrl, tau); \
            else                                                                                 \
                k_compact<EPT, false, true><<<grid, 256, 0, s>>>(round, u, v, m, f0, f1, cap, pi, n, ctrl, tau); \
        } else {                                                                                 \
            k_compact<EPT, true, false><<<grid, 256, 0, s>>>(round, u, v, m, f0, f1, cap, pi, n, ctrl, tau); \
        }                                                                                        \
    } while (0)
    switch (ept) {
        case 4: CP(4); break;
        case 8: CP(8); break;
        case 16: CP(16); break;
        default: return hipErrorInvalidValue;
    }
#undef CP
    return hipGetLastError();
}

// ----------------------------------------------------------------------------- frontier Atomic-Hook
// Atomic-Hook (Fig. 3, with path halving) of a frontier of root pairs left
// by a compaction: *count pairs (at most cap), each a pair of roots at the
// time of the compaction, so the climb starts from the pair itself (values
// only ever name vertices of the same tree, smaller than the slot) without
// gathering pi first.  Persistent grid over the pairs, consecutive lanes on
// consecutive pairs.
template <int EPT, bool HALVE>
__global__ __launch_bounds__(256) void k_ahook_pairs(const int2* __restrict__ fr,
                                                     const uint32_t* count, int64_t cap,
                                                     int32_t* pi) {
    const int64_t total = min((int64_t)*count, cap);
    const int64_t tile = (int64_t)blockDim.x * EPT;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < total; t0 += (int64_t)gridDim.x * tile) {
        int2 q[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int64_t e = t0 + (int64_t)j * blockDim.x + threadIdx.x;
            q[j] = e < total ? fr[e] : int2{0, 0};
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            if (q[j].x != q[j].y) atomic_hook<false, HALVE>(pi, q[j].x, q[j].y);
    }
}

hipError_t launch_ahook_pairs(const int2* fr, const uint32_t* count, int64_t cap, int32_t* pi,
                              bool halve, int grid_cap, hipStream_t s) {
    constexpr int EPT = 8;
    const int64_t tile = 256 * EPT;
    int64_t grid64 = (cap + tile - 1) / tile;
    if (grid64 < 1) grid64 = 1;
    if (grid64 > grid_cap) grid64 = grid_cap;
    if (halve) k_ahook_pairs<EPT, true><<<(int)grid64, 256, 0, s>>>(fr, count, cap, pi);
    else k_ahook_pairs<EPT, false><<<(int)grid64, 256, 0, s>>>(fr, count, cap, pi);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------- Fig. 1 host loop
// Hook (Fig. 2) over every entry, raising ctrl->hook_changed (one store per
// wave that saw an active entry) -- the flag the host reads after the launch.
template <int EPT, bool VEC>
__global__ __launch_bounds__(1024) void k_hook_flag(const int32_t* __restrict__ eu,
                                                    const int32_t* __restrict__ ev, int64_t m,
                                                    int32_t* pi, int32_t n, Ctrl* ctrl) {
    const int64_t stride = (int64_t)blockDim.x * 4;
    const int64_t e0 = (int64_t)blockIdx.x * blockDim.x * EPT + (int64_t)threadIdx.x * 4;
    int32_t a[EPT], b[EPT];
    load_edges<EPT, VEC>(eu, e0, stride, m, a);
    load_edges<EPT, VEC>(ev, e0, stride, m, b);
    bool bad = false, changed = false;
    int32_t pa[EPT], pb[EPT];
    uint32_t act = 0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const bool in = (uint32_t)a[j] < (uint32_t)n && (uint32_t)b[j] < (uint32_t)n;
        bad |= !in;
        if (in && a[j] != b[j]) {
            act |= 1u << j;
            pa[j] = ld_rlx(pi + a[j]);
            pb[j] = ld_rlx(pi + b[j]);
        }
    }
    if (bad) atomicOr(&ctrl->status, kStatusRange);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        if ((act >> j & 1) && pa[j] != pb[j]) {
            st_rlx(pi + (pa[j] > pb[j] ? pa[j] : pb[j]), pa[j] > pb[j] ? pb[j] : pa[j]);
            changed = true;
        }
    }
    if (__ballot(changed) != 0 && (threadIdx.x & 63) == 0) ctrl->hook_changed = 1;
}

// One Jump (Fig. 2): pi(v) <- pi(pi(v)) for every vertex, raising
// ctrl->jump_changed when any pointer moved.
__global__ __launch_bounds__(256) void k_jump(int32_t* pi, int32_t n, Ctrl* ctrl) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool changed = false;
    if (x < n) {
        const int32_t p = ld_rlx(pi + x);
        const int32_t g = ld_rlx(pi + p);
        if (g != p) {
            st_rlx(pi + x, g);
            changed = true;
        }
    }
    if (__ballot(changed) != 0 && (threadIdx.x & 63) == 0) ctrl->jump_changed = 1;
}

hipError_t launch_hook_flag(const int32_t* u, const int32_t* v, int64_t m, int32_t* pi, int32_t n,
                            Ctrl* ctrl, int block, int ept, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const int64_t tile = (int64_t)block * ept;
    const int64_t grid64 = (m + tile - 1) / tile;
    if (grid64 > 0x7fffffff) return hipErrorInvalidValue;
    const int grid = (int)grid64;
    const bool vec = aligned16(u) && aligned16(v);
    switch (ept) {
        case 4:
            vec ? k_hook_flag<4, true><<<grid, block, 0, s>>>(u, v, m, pi, n, ctrl)
                : k_hook_flag<4, false><<<grid, block, 0, s>>>(u, v, m, pi, n, ctrl);
            break;
        case 8:
            vec ? k_hook_flag<8, true><<<grid, block, 0, s>>>(u, v, m, pi, n, ctrl)
                : k_hook_flag<8, false><<<grid, block, 0, s>>>(u, v, m, pi, n, ctrl);
            break;
        case 16:
            vec ? k_hook_flag<16, true><<<grid, block, 0, s>>>(u, v, m, pi, n, ctrl)
                : k_hook_flag<16, false><<<grid, block, 0, s>>>(u, v, m, pi, n, ctrl);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_jump(int32_t* pi, int32_t n, Ctrl* ctrl, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)(((int64_t)n + 255) / 256);
    k_jump<<<grid, 256, 0, s>>>(pi, n, ctrl);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------- zero fill
// Clears `words` 32-bit words (used instead of a memset so that a captured
// graph holds kernel nodes only).
__global__ __launch_bounds__(256) void k_zero(uint32_t* __restrict__ p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

hipError_t launch_zero(void* p, int64_t words, hipStream_t s) {
    if (words <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(1024, (words + 255) / 256);
    k_zero<<<grid, 256, 0, s>>>(static_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return cus;
}

}  // namespace hookcc
