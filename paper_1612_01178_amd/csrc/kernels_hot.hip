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
// Vertex table (kVertSlots one-byte slots, all 160 KiB of LDS): a hot vertex
// shares its bitmap word with 31 mostly cold ones, so word slots spend most
// of their bits on vertices that are rarely tested.  Slot t caches one vertex
// v = k * kVertSlots + t as the byte (k << 1) | bit(v): five times the hot
// vertices of the word table in the same LDS (R-MAT 24: about half of the
// bit tests answered in LDS, against 35 % for 32,768 word slots).  Chosen from sampled endpoints
// (k_vsample, k_vselect); the fused Multi-Jump/bitmap pass refreshes the
// bits with byte stores, each slot written only by its own vertex.
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
// x / kVertSlots < kVertTagNone are candidates; bucket(x) is the range of
// kVBucketSlots slots that holds slot x mod kVertSlots.
//   k_vsample  workgroup g takes kVRunsPerPart runs, histograms its
//              candidates by bucket in LDS, scans, and writes them grouped by
//              bucket into its own part of `region`, with the per-bucket
//              counts and offsets (cnt, off: [part][bucket]).
//   k_vselect  workgroup b gathers bucket b from every part, counts every
//              (slot, tag) pair in LDS, and gives each slot the tag with the
//              largest count (ties -> smallest tag).
// Entry of sample s: lane s % 64 of run s / 64, which starts at about
// (s / 64) * (m - 64) / runs (step = (m - 64) / runs; m >= 64).
__device__ __forceinline__ int64_t vsample_entry(int64_t s, int64_t m, double step) {
    const int64_t r0 = (int64_t)((double)(s >> 6) * step);
    return min(r0, m - 64) + (s & 63);
}

__device__ __forceinline__ bool vcandidate(uint32_t x, int32_t n) {
    return x < (uint32_t)n && x / kVertSlots < kVertTagNone;
}

__device__ __forceinline__ uint32_t vbucket(uint32_t x) {
    return (x % kVertSlots) / kVBucketSlots;
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
                                                 int32_t n, uint8_t* __restrict__ table) {
    constexpr int kTags = (int)kVertTagNone;  // candidate tags 0 .. kTags - 1
    // 16-bit counters, two per word (counter i in half i & 1 of word i / 2);
    // at most 65,535 endpoints of a bucket are counted, so none overflows
    __shared__ uint32_t c[kVBucketSlots * kTags / 2];
    __shared__ uint32_t start[kVPartsMax + 1];  // first flat index of each part's piece
    __shared__ uint32_t src0[kVPartsMax];       // its offset in region
    __shared__ uint32_t wsum[4];
    static_assert(kVBucketSlots == 256 && kVPartsMax == 256, "one slot and one part per thread");
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    // the bucket's piece of every part, flattened: piece of part g holds the
    // flat indices [start[g], start[g + 1])
    const uint32_t k = tid < parts ? cnt[(int64_t)tid * kVBuckets + b] : 0u;
    src0[tid] = tid < parts ? (uint32_t)(tid * kVPartCap) + off[(int64_t)tid * kVBuckets + b] : 0u;
    for (int i = tid; i < kVBucketSlots * kTags / 2; i += 256) c[i] = 0;
    const uint32_t st = block_scan(k, wsum);  // one value per thread here
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
            const uint32_t i = (xs[q] % kVertSlots % kVBucketSlots) * kTags + xs[q] / kVertSlots;
            atomicAdd(&c[i >> 1], 1u << (16 * (i & 1)));
        }
    }
    __syncthreads();
    const int64_t t = (int64_t)b * kVBucketSlots + tid;
    uint32_t best_k = kVertTagNone, best_c = 0;
    for (int q = 0; q < kTags && t + (int64_t)q * kVertSlots < n; ++q) {
        const uint32_t i = tid * kTags + q;
        const uint32_t cc = c[i >> 1] >> (16 * (i & 1)) & 0xffffu;
        if (best_k == kVertTagNone || cc > best_c) {
            best_k = (uint32_t)q;
            best_c = cc;
        }
    }
    table[t] = (uint8_t)(best_k << 1);
}

// Fills the bit of every slot from the bitmap; no-op unless ctrl->filter_on.
__global__ __launch_bounds__(256) void k_hot_vvalues(const uint32_t* __restrict__ bits,
                                                     uint8_t* __restrict__ table, const Ctrl* ctrl) {
    if (!ctrl->filter_on) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kVertSlots) return;
    const uint32_t k = table[t] >> 1;
    if (k >= kVertTagNone) return;
    const int64_t v = (int64_t)k * kVertSlots + t;
    table[t] = (uint8_t)((k << 1) | (bits[v >> 5] >> (v & 31) & 1u));
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

// Filtered Atomic-Hook with the vertex table in LDS (one byte per slot,
// loaded once per workgroup).  A test of vertex x is answered in LDS when
// slot x mod kVertSlots holds x (tag x / kVertSlots), else from the bitmap.
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
        const v4i* src = reinterpret_cast<const v4i*>(gtab);
        v4i* dst = reinterpret_cast<v4i*>(ltab);
        for (uint32_t i = threadIdx.x; i < (uint32_t)(kVertSlots / 16); i += blockDim.x) dst[i] = src[i];
        __syncthreads();
    }
    const uint8_t* lbyte = reinterpret_cast<const uint8_t*>(ltab);
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
                const uint32_t ca = lbyte[xa % kVertSlots];
                const uint32_t cb = lbyte[xb % kVertSlots];
                const bool hita = (ca >> 1) == xa / kVertSlots && xa / kVertSlots < kVertTagNone;
                const bool hitb = (cb >> 1) == xb / kVertSlots && xb / kVertSlots < kVertTagNone;
                uint32_t worda = ca, wordb = cb;
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
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            if (act >> j & 1) hot_climb(pi, pa[j], pb[j], halve);
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
    k_vselect<<<kVBuckets, 256, 0, s>>>(region, cnt, off, parts, n, table);
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
