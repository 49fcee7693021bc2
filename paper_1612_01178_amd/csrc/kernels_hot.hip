// Hot-word LDS cache for the giant-component filter (CDNA4).
//
// The filtered Atomic-Hook tests two bits of the giant bitmap (n/8 bytes,
// L2-resident) per edge entry; on skewed graphs those random L2 accesses,
// not the edge stream, bound the pass.  Endpoint frequencies are very
// skewed, so a small set of bitmap words takes a large share of the tests.
// This file keeps the hottest words in LDS:
//
//   k_hot_count   counts sampled endpoint occurrences per bitmap word
//   k_hot_select  for every LDS slot t (of `slots`, 16384 or 32768), picks the
//                 hottest word w = k * slots + t (direct-mapped; ties -> smallest k)
//   k_hot_values  copies the chosen words' current bits (after each bitmap build)
//   k_ahook_hot   the filtered Atomic-Hook, persistent: each workgroup loads
//                 the (tag, word) table into LDS once and answers a bit test
//                 from LDS when the word is cached, else from the bitmap
//
// The table holds copies of bitmap words taken after the bitmap was built,
// so a cached answer is exactly the bitmap's answer; the filter's exactness
// argument is unchanged.
//
// Vertex table (kVertSets two-way sets of one-byte slots, all 160 KiB of
// LDS): a hot vertex shares its bitmap word with 31 mostly cold ones, so word
// slots spend most of their bits on vertices that are rarely tested.  Set s
// caches up to two vertices v = k * kVertSets + s by their tags k; the LDS
// copy keeps a tag only while its vertex is in the giant component (else the
// slot reads as empty), so a tag match answers the test with 1 and anything
// else goes to the bitmap.  Membership only grows (trees only merge), and the
// hot vertices of a graph with a giant component are nearly all in it.
// Five times the hot vertices of the word table in the same LDS (R-MAT 24:
// 56 % of the bit tests answered in LDS, against 35 % for 32,768 word slots).
// Chosen from sampled endpoints (k_vsample, k_vselect); the fused
// Multi-Jump/bitmap pass refreshes the member flags in device memory with
// byte stores, each flag written only by its own vertex.
#include "kernels.hpp"

namespace hookcc {

typedef int32_t v4i __attribute__((ext_vector_type(4)));

constexpr uint32_t kHotNone = 0xffffffffu;

__global__ __launch_bounds__(256) void k_hot_zero(uint32_t* __restrict__ p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Sample i reads entry floor(i * m / S) and counts the words of both ends.
__global__ __launch_bounds__(256) void k_hot_count(const int32_t* __restrict__ eu,
                                                   const int32_t* __restrict__ ev, int64_t m,
                                                   int32_t n, int64_t S, uint32_t* counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    const int64_t e = i * m / S;
    const uint32_t a = (uint32_t)eu[e], b = (uint32_t)ev[e];
    if (a < (uint32_t)n) atomicAdd(counts + (a >> 5), 1u);
    if (b < (uint32_t)n) atomicAdd(counts + (b >> 5), 1u);
}

__global__ __launch_bounds__(256) void k_hot_select(const uint32_t* __restrict__ counts, int64_t nw,
                                                    uint32_t* __restrict__ tags, int slots) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= slots) return;
    uint32_t best_k = kHotNone, best_c = 0;
    for (int64_t w = t, k = 0; w < nw; w += slots, ++k) {
        const uint32_t c = counts[w];
        if (best_k == kHotNone || c > best_c) {
            best_k = (uint32_t)k;
            best_c = c;
        }
    }
    tags[t] = best_k;
}

__global__ __launch_bounds__(256) void k_hot_values(const uint32_t* __restrict__ bits,
                                                    const uint32_t* __restrict__ tags,
                                                    uint32_t* __restrict__ vals, const Ctrl* ctrl,
                                                    int slots) {
    if (!ctrl->filter_on) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= slots) return;
    const uint32_t k = tags[t];
    vals[t] = (k == kHotNone) ? 0u : bits[(int64_t)k * slots + t];
}

// Vertex table selection, without global atomics (random atomics over a
// per-vertex count array run at about 2 x 10^10/s here, 0.2 ms for 2^22
// endpoints).  Sampled entries: up to kVertRuns runs of 64 consecutive
// entries spread evenly over the list.  Endpoints x < n with tag
// x / kVertSets < kVertTagNone are candidates; bucket(x) is the range of
// kVBucketSets sets that holds set x mod kVertSets.
//   k_vsample  workgroup g takes kVRunsPerPart runs, histograms its
//              candidates by bucket in LDS, scans, and writes them grouped by
//              bucket into its own part of `region`, with the per-bucket
//              counts and offsets (cnt, off: [part][bucket]).
//   k_vselect  workgroup b gathers bucket b from every part, counts every
//              (set, tag) pair in LDS, and gives each set the kVertWays tags
//              with the largest counts (ties -> smaller tag).
// Entry of sample s: lane s % 64 of run s / 64, which starts at about
// (s / 64) * (m - 64) / runs (step = (m - 64) / runs; m >= 64).
__device__ __forceinline__ int64_t vsample_entry(int64_t s, int64_t m, double step) {
    const int64_t r0 = (int64_t)((double)(s >> 6) * step);
    return min(r0, m - 64) + (s & 63);
}

__device__ __forceinline__ bool vcandidate(uint32_t x, int32_t n) {
    return x < (uint32_t)n && x / kVertSets < kVertTagNone;
}

__device__ __forceinline__ uint32_t vbucket(uint32_t x) {
    return (x % kVertSets) / kVBucketSets;
}

// Exclusive scan of one value per thread over a 256-thread workgroup;
// returns this thread's base (the sum of the values of lower threads).
__device__ __forceinline__ uint32_t block_scan(uint32_t pair, uint32_t* wsum) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = pair;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t base = 0;
    for (int i = 0; i < w; ++i) base += wsum[i];
    return base + incl - pair;
}

constexpr int kVPerThread = kVRunsPerPart * 64 / 256;  // sampled entries per thread

__global__ __launch_bounds__(256) void k_vsample(const int32_t* __restrict__ eu,
                                                 const int32_t* __restrict__ ev, int64_t m,
                                                 int32_t n, int64_t runs, double step,
                                                 uint32_t* __restrict__ region,
                                                 uint32_t* __restrict__ cnt,
                                                 uint32_t* __restrict__ off) {
    constexpr int kPer = (kVBuckets + 255) / 256;  // buckets per thread in the scan
    __shared__ uint32_t hist[256 * kPer];
    __shared__ uint32_t cur[256 * kPer];
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t stage[kVPartCap];  // the part, grouped by bucket
    const int g = blockIdx.x;
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < kPer; ++q) hist[kPer * tid + q] = 0;
    // this thread's samples, all loads issued before any is used
    const int64_t s0 = (int64_t)g * kVRunsPerPart * 64;
    const int64_t s1 = min(runs, (int64_t)(g + 1) * kVRunsPerPart) * 64;
    uint32_t x[kVPerThread], y[kVPerThread];
#pragma unroll
    for (int i = 0; i < kVPerThread; ++i) {
        const int64_t s = s0 + tid + (int64_t)i * 256;
        const int64_t e = s < s1 ? vsample_entry(s, m, step) : 0;
        x[i] = s < s1 ? (uint32_t)eu[e] : 0xffffffffu;
        y[i] = s < s1 ? (uint32_t)ev[e] : 0xffffffffu;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kVPerThread; ++i) {
        if (vcandidate(x[i], n)) atomicAdd(&hist[vbucket(x[i])], 1u);
        if (vcandidate(y[i], n)) atomicAdd(&hist[vbucket(y[i])], 1u);
    }
    __syncthreads();
    // exclusive scan: thread tid owns buckets kPer * tid .. kPer * tid + kPer - 1
    uint32_t own = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) own += hist[kPer * tid + q];
    uint32_t at = block_scan(own, wsum);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int bk = kPer * tid + q;
        const uint32_t h = hist[bk];
        cur[bk] = at;
        if (bk < kVBuckets) {
            cnt[(int64_t)g * kVBuckets + bk] = h;
            off[(int64_t)g * kVBuckets + bk] = at;
        }
        at += h;
    }
    const uint32_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kVPerThread; ++i) {
        if (vcandidate(x[i], n)) stage[atomicAdd(&cur[vbucket(x[i])], 1u)] = x[i];
        if (vcandidate(y[i], n)) stage[atomicAdd(&cur[vbucket(y[i])], 1u)] = y[i];
    }
    __syncthreads();
    uint32_t* part = region + (int64_t)g * kVPartCap;
    for (uint32_t i = tid; i < total; i += 256) part[i] = stage[i];
}

__global__ __launch_bounds__(256) void k_vselect(const uint32_t* __restrict__ region,
                                                 const uint32_t* __restrict__ cnt,
                                                 const uint32_t* __restrict__ off, int parts,
                                                 int32_t n, uint8_t* __restrict__ tags) {
    constexpr int kTags = (int)kVertTagNone;  // candidate tags 0 .. kTags - 1
    // 16-bit counters, two per word (counter i in half i & 1 of word i / 2);
    // at most 65,535 endpoints of a bucket are counted, so none overflows
    __shared__ uint32_t c[kVBucketSets * kTags / 2 + 1];
    __shared__ uint32_t start[kVPartsMax + 1];  // first flat index of each part's piece
    __shared__ uint32_t src0[kVPartsMax];       // its offset in region
    __shared__ uint32_t wsum[4];
    static_assert(kVPartsMax == 256 && kVBucketSets <= 256, "one part per thread");
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    // the bucket's piece of every part, flattened: piece of part g holds the
    // flat indices [start[g], start[g + 1])
    const uint32_t k = tid < parts ? cnt[(int64_t)tid * kVBuckets + b] : 0u;
    src0[tid] = tid < parts ? (uint32_t)(tid * kVPartCap) + off[(int64_t)tid * kVBuckets + b] : 0u;
    for (int i = tid; i < kVBucketSets * kTags / 2 + 1; i += 256) c[i] = 0;
    const uint32_t st = block_scan(k, wsum);
    start[tid] = st;
    if (tid == 255) start[256] = st + k;
    __syncthreads();
    const uint32_t total = min(start[256], 65535u);
    constexpr int kUnroll = 8;  // independent gathers in flight per thread
    for (uint32_t j0 = 0; j0 < total; j0 += 256 * kUnroll) {
        uint32_t xs[kUnroll];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
            const uint32_t j = j0 + q * 256 + tid;
            // the last part g with start[g] <= j (start[0] = 0; parts past
            // the last non-empty piece start at total > j)
            uint32_t g = 0;
#pragma unroll
            for (uint32_t d = kVPartsMax / 2; d >= 1; d >>= 1)
                if (start[g + d] <= j) g += d;
            const uint32_t at = j < total ? src0[g] + (j - start[g]) : 0u;  // 0: in bounds
            xs[q] = j < total ? region[at] : 0xffffffffu;
        }
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
            if (xs[q] == 0xffffffffu) continue;
            const uint32_t i = (xs[q] % kVertSets % kVBucketSets) * kTags + xs[q] / kVertSets;
            atomicAdd(&c[i >> 1], 1u << (16 * (i & 1)));
        }
    }
    __syncthreads();
    // the two largest counts of set s (ties -> smaller tag); tags of vertices
    // past n are not candidates.  Threads 4i .. 4i + 3 scan a quarter of set
    // i's tags each, then merge their top two in two butterfly steps.
    static_assert(4 * kVBucketSets == 256 && kVertWays == 2, "four threads per set, two ways");
    constexpr int kQuarter = (kTags + 3) / 4;
    const int set = tid >> 2, part = tid & 3;
    const int64_t s = (int64_t)b * kVBucketSets + set;
    const int64_t tags_n = (int64_t)n > s ? ((int64_t)n - s + kVertSets - 1) / kVertSets : 0;
    const int q0 = part * kQuarter;
    const int q1 = (int)min<int64_t>(tags_n, min(kTags, (part + 1) * kQuarter));
    uint32_t k1 = kVertTagNone, c1 = 0, k2 = kVertTagNone, c2 = 0;
#pragma unroll 8
    for (int q = q0; q < q1; ++q) {
        const uint32_t i = set * kTags + q;
        const uint32_t cc = c[i >> 1] >> (16 * (i & 1)) & 0xffffu;
        if (k1 == kVertTagNone || cc > c1) {
            k2 = k1;
            c2 = c1;
            k1 = (uint32_t)q;
            c1 = cc;
        } else if (k2 == kVertTagNone || cc > c2) {
            k2 = (uint32_t)q;
            c2 = cc;
        }
    }
    // merge with the partner's list: the order is count descending, then tag
    // ascending (the same in every thread, so all four end with one result)
    auto before = [](uint32_t ka, uint32_t ca, uint32_t kb, uint32_t cb) {
        return ka != kVertTagNone && (kb == kVertTagNone || ca > cb || (ca == cb && ka < kb));
    };
#pragma unroll
    for (int d = 1; d <= 2; d <<= 1) {
        const uint32_t o1 = __shfl_xor(k1, d, 64), p1 = __shfl_xor(c1, d, 64);
        const uint32_t o2 = __shfl_xor(k2, d, 64), p2 = __shfl_xor(c2, d, 64);
        if (before(k1, c1, o1, p1)) {
            if (!before(k2, c2, o1, p1)) {
                k2 = o1;
                c2 = p1;
            }
        } else {
            if (!before(k1, c1, o2, p2)) {
                k2 = o2;
                c2 = p2;
            } else {
                k2 = k1;
                c2 = c1;
            }
            k1 = o1;
            c1 = p1;
        }
    }
    if (part == 0) {
        tags[2 * s] = (uint8_t)k1;
        tags[2 * s + 1] = (uint8_t)k2;
    }
}

// Member flag of every slot from the bitmap (0 for an empty slot); no-op
// unless ctrl->filter_on.
__global__ __launch_bounds__(256) void k_hot_vvalues(const uint32_t* __restrict__ bits,
                                                     uint8_t* __restrict__ vtab, const Ctrl* ctrl) {
    if (!ctrl->filter_on) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kVertSlots) return;
    const uint32_t k = vtab[t];
    uint8_t f = 0;
    if (k < kVertTagNone) {
        const int64_t v = (int64_t)k * kVertSets + t / kVertWays;
        f = (uint8_t)(bits[v >> 5] >> (v & 31) & 1u);
    }
    vtab[kVertSlots + t] = f;
}

template <int EPT>
__device__ __forceinline__ void load_tile(const int32_t* __restrict__ p, int64_t e0,
                                          int64_t stride, int64_t end, bool vec,
                                          int32_t (&x)[EPT]) {
#pragma unroll
    for (int k = 0; k < EPT / 4; ++k) {
        const int64_t e = e0 + k * stride;
        if (vec && e + 3 < end) {
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

// Atomic-Hook climb (Fig. 3, top), cached loads; see atomic_hook in
// kernels_core.hip for the argument.
__device__ __forceinline__ void hot_climb(int32_t* pi, int32_t pu, int32_t pv, bool halve) {
    uint32_t step = 0;
    while (pu != pv) {
        const int32_t H = pu > pv ? pu : pv;
        const int32_t L = pu > pv ? pv : pu;
        int32_t found = ld_tree<false>(pi + H);
        if (found == H) {
            found = cas_root(pi + H, H, L);
            if (found == H) return;
        }
        pu = ld_tree<false>(pi + found);
        pv = ld_tree<false>(pi + L);
        if (halve && pu != found && step++ % kHalveEveryFiltered == 0)
            halve_to(pi + H, pu);  // path halving
    }
}

// K climbs of hot_climb advanced together (a finished one has pu == pv):
// each step issues all their loads, then all their compare-and-swaps, then
// all their reloads, so a thread keeps K dependent chains of tree accesses in
// flight instead of one.  Every step of each climb is the step hot_climb
// takes, except that a climb whose bit is set in `root` starts at the
// compare-and-swap: the larger of its two starting values is an endpoint
// that was its own parent when its parent was gathered, so the load that
// would check that it is a root is skipped (if it no longer is one, the
// compare-and-swap fails and returns its parent, the value the load would
// have read, and the climb goes on from there as after that load).
template <int K>
__device__ __forceinline__ void hot_climb_k(int32_t* pi, int32_t* pu, int32_t* pv, bool halve,
                                            uint32_t root) {
    uint32_t step[K];
#pragma unroll
    for (int k = 0; k < K; ++k) step[k] = 0;
    while (true) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < K; ++k) any |= pu[k] != pv[k];
        if (!any) break;
        int32_t H[K], L[K], f[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            H[k] = pu[k] > pv[k] ? pu[k] : pv[k];
            L[k] = pu[k] > pv[k] ? pv[k] : pu[k];
            f[k] = pu[k] != pv[k] && !(root >> k & 1) ? ld_tree<false>(pi + H[k]) : H[k];
        }
        root = 0;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (pu[k] != pv[k] && f[k] == H[k]) f[k] = cas_root(pi + H[k], H[k], L[k]);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (pu[k] == pv[k]) continue;
            if (f[k] == H[k]) {
                pu[k] = pv[k] = L[k];  // hooked
            } else {
                pu[k] = ld_tree<false>(pi + f[k]);
                pv[k] = ld_tree<false>(pi + L[k]);
                if (halve && pu[k] != f[k] && step[k]++ % kHalveEveryFiltered == 0)
                    halve_to(pi + H[k], pu[k]);
            }
        }
    }
}

// SLOTS slots with tags of type TagT (16384 x uint16 = 96 KiB of LDS with the
// words, or 32768 x uint8 = 160 KiB); a tag equal to TagT's maximum marks an
// empty slot (also used for a word index too large for the tag type).
template <int EPT, int SLOTS, typename TagT>
__global__ __launch_bounds__(1024) void k_ahook_hot(const int32_t* __restrict__ eu,
                                                    const int32_t* __restrict__ ev, int64_t begin,
                                                    int64_t end, bool vec, int32_t* pi, int32_t n,
                                                    Ctrl* ctrl, const uint32_t* __restrict__ bits,
                                                    const uint32_t* __restrict__ gtags,
                                                    const uint32_t* __restrict__ gvals, bool halve,
                                                    bool sym) {
    constexpr uint32_t kEmpty = (uint32_t)(TagT)(~(TagT)0);
    __shared__ TagT ltag[SLOTS];
    __shared__ uint32_t lval[SLOTS];
    const bool filter = ctrl->filter_on != 0;
    const int32_t g = ctrl->giant;
    if (filter) {
        for (uint32_t t = threadIdx.x; t < (uint32_t)SLOTS; t += blockDim.x) {
            const uint32_t k = gtags[t];
            ltag[t] = (TagT)((k == kHotNone || k >= kEmpty) ? kEmpty : k);
            lval[t] = gvals[t];
        }
        __syncthreads();
    }
    const int64_t stride = (int64_t)blockDim.x * 4;
    const int64_t tile = (int64_t)blockDim.x * EPT;
    bool bad = false;
    for (int64_t t0 = begin + (int64_t)blockIdx.x * tile; t0 < end; t0 += (int64_t)gridDim.x * tile) {
        const int64_t e0 = t0 + (int64_t)threadIdx.x * 4;
        int32_t a[EPT], b[EPT];
        load_tile<EPT>(eu, e0, stride, end, vec, a);
        load_tile<EPT>(ev, e0, stride, end, vec, b);
        uint32_t act = 0;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const bool in = (uint32_t)a[j] < (uint32_t)n && (uint32_t)b[j] < (uint32_t)n;
            bad |= !in;
            if (in && a[j] != b[j] && !(sym && a[j] > b[j])) act |= 1u << j;
        }
        int32_t pa[EPT], pb[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (!(act >> j & 1)) continue;
            uint32_t ba = 0, bb = 0;
            if (filter) {
                const uint32_t wa = (uint32_t)a[j] >> 5, wb = (uint32_t)b[j] >> 5;
                const uint32_t sa = wa & (SLOTS - 1), sb = wb & (SLOTS - 1);
                const uint32_t ka = wa / SLOTS, kb = wb / SLOTS;
                // ka == kEmpty can never be cached (it is the empty marker).
                // Two separate (relaxed atomic) loads, the LDS one
                // unconditional: plain loads here are merged into one load
                // from a selected address, which is a flat load that also
                // waits on the LDS traffic.
                const bool hita = ka < kEmpty && (uint32_t)ltag[sa] == ka;
                const bool hitb = kb < kEmpty && (uint32_t)ltag[sb] == kb;
                uint32_t worda = __hip_atomic_load(lval + sa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                uint32_t wordb = __hip_atomic_load(lval + sb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (!hita) worda = __hip_atomic_load(bits + wa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (!hitb) wordb = __hip_atomic_load(bits + wb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                ba = worda >> (a[j] & 31) & 1;
                bb = wordb >> (b[j] & 31) & 1;
            }
            if (ba & bb) {
                act &= ~(1u << j);
            } else {
                pa[j] = ba ? g : ld_tree<false>(pi + a[j]);
                pb[j] = bb ? g : ld_tree<false>(pi + b[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            if (act >> j & 1) hot_climb(pi, pa[j], pb[j], halve);
    }
    if (bad) atomicOr(&ctrl->status, kStatusRange);
}

hipError_t launch_hot_prepare(const int32_t* u, const int32_t* v, int64_t m, int32_t n,
                              uint32_t* counts, uint32_t* tags, int slots, hipStream_t s) {
    if (slots != 16384 && slots != 32768) return hipErrorInvalidValue;
    const int64_t nw = ((int64_t)n + 31) / 32;
    k_hot_zero<<<1024, 256, 0, s>>>(counts, nw);
    const int64_t S = std::min<int64_t>(m, int64_t(1) << 19);
    if (S > 0) k_hot_count<<<(int)((S + 255) / 256), 256, 0, s>>>(u, v, m, n, S, counts);
    k_hot_select<<<slots / 256, 256, 0, s>>>(counts, nw, tags, slots);
    return hipGetLastError();
}

hipError_t launch_hot_values(const uint32_t* bits, const uint32_t* tags, uint32_t* vals,
                             const Ctrl* ctrl, int slots, hipStream_t s) {
    if (slots != 16384 && slots != 32768) return hipErrorInvalidValue;
    k_hot_values<<<slots / 256, 256, 0, s>>>(bits, tags, vals, ctrl, slots);
    return hipGetLastError();
}

// Filtered Atomic-Hook with the vertex table in LDS (loaded once per
// workgroup, a slot's tag kept only while its member flag is set).  A test of
// vertex x is answered with 1 in LDS when set x mod kVertSets holds the tag
// x / kVertSets, else from the bitmap.
template <int EPT>
__global__ __launch_bounds__(1024) void k_ahook_hotv(const int32_t* __restrict__ eu,
                                                     const int32_t* __restrict__ ev, int64_t begin,
                                                     int64_t end, bool vec, int32_t* pi, int32_t n,
                                                     Ctrl* ctrl, const uint32_t* __restrict__ bits,
                                                     const uint8_t* __restrict__ gtab, bool halve,
                                                     bool sym) {
    __shared__ uint32_t ltab[kVertSlots / 4];
    const bool filter = ctrl->filter_on != 0;
    const int32_t g = ctrl->giant;
    if (filter) {
        // tag | 0xff per byte whose member flag (0 or 1) is 0: bytes of
        // (0x01010101 - flags) are 1 - flag, times 0xff without carries
        const v4i* tg = reinterpret_cast<const v4i*>(gtab);
        const v4i* fl = reinterpret_cast<const v4i*>(gtab + kVertSlots);
        v4i* dst = reinterpret_cast<v4i*>(ltab);
        for (uint32_t i = threadIdx.x; i < (uint32_t)(kVertSlots / 16); i += blockDim.x) {
            const v4i t = tg[i], f = fl[i];
            v4i o;
            o.x = (int32_t)((uint32_t)t.x | (0x01010101u - (uint32_t)f.x) * 0xffu);
            o.y = (int32_t)((uint32_t)t.y | (0x01010101u - (uint32_t)f.y) * 0xffu);
            o.z = (int32_t)((uint32_t)t.z | (0x01010101u - (uint32_t)f.z) * 0xffu);
            o.w = (int32_t)((uint32_t)t.w | (0x01010101u - (uint32_t)f.w) * 0xffu);
            dst[i] = o;
        }
        __syncthreads();
    }
    const uint16_t* lset = reinterpret_cast<const uint16_t*>(ltab);
    const int64_t stride = (int64_t)blockDim.x * 4;
    const int64_t tile = (int64_t)blockDim.x * EPT;
    bool bad = false;
    for (int64_t t0 = begin + (int64_t)blockIdx.x * tile; t0 < end; t0 += (int64_t)gridDim.x * tile) {
        const int64_t e0 = t0 + (int64_t)threadIdx.x * 4;
        int32_t a[EPT], b[EPT];
        load_tile<EPT>(eu, e0, stride, end, vec, a);
        load_tile<EPT>(ev, e0, stride, end, vec, b);
        uint32_t act = 0;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const bool in = (uint32_t)a[j] < (uint32_t)n && (uint32_t)b[j] < (uint32_t)n;
            bad |= !in;
            if (in && a[j] != b[j] && !(sym && a[j] > b[j])) act |= 1u << j;
        }
        int32_t pa[EPT], pb[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (!(act >> j & 1)) continue;
            uint32_t ba = 0, bb = 0;
            if (filter) {
                const uint32_t xa = (uint32_t)a[j], xb = (uint32_t)b[j];
                // a tag of kVertTagNone or more never matches a stored byte's
                // tag (stored tags are below it or mark an empty slot)
                // a tag of kVertTagNone (the empty marker) or more never hits
                const uint32_t sa = lset[xa % kVertSets], sb = lset[xb % kVertSets];
                const uint32_t ka = xa / kVertSets, kb = xb / kVertSets;
                const bool hita = ka < kVertTagNone && ((sa & 0xffu) == ka || (sa >> 8) == ka);
                const bool hitb = kb < kVertTagNone && ((sb & 0xffu) == kb || (sb >> 8) == kb);
                uint32_t worda = 1, wordb = 1;
                if (!hita) worda = __hip_atomic_load(bits + (xa >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> (xa & 31);
                if (!hitb) wordb = __hip_atomic_load(bits + (xb >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> (xb & 31);
                ba = worda & 1;
                bb = wordb & 1;
            }
            if (ba & bb) {
                act &= ~(1u << j);
            } else {
                pa[j] = ba ? g : ld_tree<false>(pi + a[j]);
                pb[j] = bb ? g : ld_tree<false>(pi + b[j]);
            }
        }
        // the kept entries' climbs, kClimbs at a time (entries j, j + EPT /
        // kClimbs, ...; an entry not kept takes part as a finished climb)
        constexpr int kClimbs = 2;
#pragma unroll
        for (int j = 0; j < EPT / kClimbs; ++j) {
            int32_t cu[kClimbs], cv[kClimbs];
            bool anyk = false;
            // bit k of root: the larger start of climb k is an endpoint that
            // was its own parent (a wrong bit would only cost a failed CAS)
            uint32_t root = 0;
#pragma unroll
            for (int k = 0; k < kClimbs; ++k) {
                const int e = j + k * (EPT / kClimbs);
                const bool on = act >> e & 1;
                cu[k] = on ? pa[e] : 0;
                cv[k] = on ? pb[e] : 0;
                anyk |= on;
                const bool ra = cu[k] > cv[k] && cu[k] == a[e];
                const bool rb = cv[k] > cu[k] && cv[k] == b[e];
                root |= (uint32_t)(ra || rb) << k;
            }
            if (anyk) hot_climb_k<kClimbs>(pi, cu, cv, halve, root);
        }
    }
    if (bad) atomicOr(&ctrl->status, kStatusRange);
}

hipError_t launch_hot_vprepare(const int32_t* u, const int32_t* v, int64_t m, int32_t n,
                               uint32_t* scratch, uint8_t* table, hipStream_t s) {
    uint32_t* region = scratch;
    uint32_t* cnt = region + (int64_t)kVPartsMax * kVPartCap;
    uint32_t* off = cnt + kVPartsMax * kVBuckets;
    const int64_t runs = m >= 64 ? std::min<int64_t>(kVertRuns, m / 64) : 0;
    const int parts = (int)((runs + kVRunsPerPart - 1) / kVRunsPerPart);
    const double step = runs > 0 ? (double)(m - 64) / (double)runs : 0.0;
    if (parts > 0) k_vsample<<<parts, 256, 0, s>>>(u, v, m, n, runs, step, region, cnt, off);
    k_vselect<<<kVBuckets, 256, 0, s>>>(region, cnt, off, parts, n, table);  // tags
    return hipGetLastError();
}

hipError_t launch_hot_vvalues(const uint32_t* bits, uint8_t* table, const Ctrl* ctrl, hipStream_t s) {
    k_hot_vvalues<<<kVertSlots / 256, 256, 0, s>>>(bits, table, ctrl);
    return hipGetLastError();
}

hipError_t launch_ahook_hotv(const int32_t* u, const int32_t* v, int64_t begin, int64_t end,
                             int32_t* pi, int32_t n, Ctrl* ctrl, const uint32_t* bits,
                             const uint8_t* table, bool halve, bool sym, hipStream_t s) {
    if (end <= begin) return hipSuccess;
    constexpr int EPT = 8;
    const int block = 1024;
    const int64_t tile = (int64_t)block * EPT;
    const int64_t tiles = (end - begin + tile - 1) / tile;
    const int64_t cap = (int64_t)device_cu_count();  // one 1024-thread workgroup per CU (LDS)
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, cap));
    const bool vec = (((uintptr_t)(u + begin) | (uintptr_t)(v + begin)) & 15) == 0;
    k_ahook_hotv<EPT><<<grid, block, 0, s>>>(u, v, begin, end, vec, pi, n, ctrl, bits, table, halve,
                                             sym);
    return hipGetLastError();
}

template <int SLOTS, typename TagT>
static hipError_t ahook_hot_ept(int ept, int grid, int block, hipStream_t s, const int32_t* u,
                                const int32_t* v, int64_t begin, int64_t end, bool vec, int32_t* pi,
                                int32_t n, Ctrl* ctrl, const uint32_t* bits, const uint32_t* tags,
                                const uint32_t* vals, bool halve, bool sym) {
    switch (ept) {
        case 4: k_ahook_hot<4, SLOTS, TagT><<<grid, block, 0, s>>>(u, v, begin, end, vec, pi, n, ctrl, bits, tags, vals, halve, sym); break;
        case 8:
        case 16:  // the 16-entry tile does not fit the registers next to the LDS table; run 8
            k_ahook_hot<8, SLOTS, TagT><<<grid, block, 0, s>>>(u, v, begin, end, vec, pi, n, ctrl, bits, tags, vals, halve, sym); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ahook_hot(const int32_t* u, const int32_t* v, int64_t begin, int64_t end,
                            int32_t* pi, int32_t n, Ctrl* ctrl, const uint32_t* bits,
                            const uint32_t* tags, const uint32_t* vals, int ept, int slots,
                            bool halve, bool sym, hipStream_t s) {
    if (end <= begin) return hipSuccess;
    const int block = 1024;
    const int64_t tile = (int64_t)block * ept;
    const int64_t tiles = (end - begin + tile - 1) / tile;
    const int64_t cap = (int64_t)device_cu_count();  // one 1024-thread workgroup per CU (LDS)
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, cap));
    const bool vec = (((uintptr_t)(u + begin) | (uintptr_t)(v + begin)) & 15) == 0;
    if (slots == 16384)
        return ahook_hot_ept<16384, uint16_t>(ept, grid, block, s, u, v, begin, end, vec, pi, n,
                                              ctrl, bits, tags, vals, halve, sym);
    if (slots == 32768)
        return ahook_hot_ept<32768, uint8_t>(ept, grid, block, s, u, v, begin, end, vec, pi, n,
                                             ctrl, bits, tags, vals, halve, sym);
    return hipErrorInvalidValue;
}

}  // namespace hookcc
