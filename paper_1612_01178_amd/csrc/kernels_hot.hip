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
        if (halve && pu != found) st_tree<false>(pi + H, pu);  // path halving
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
    const int64_t step = (int64_t)gridDim.x * tile;
    bool bad = false;
    // Software pipelining: the next tile's entries are loaded while the
    // current tile's bit tests and climbs run.
    int32_t a[EPT], b[EPT], na[EPT], nb[EPT];
    int64_t t0 = begin + (int64_t)blockIdx.x * tile;
    if (t0 < end) {
        load_tile<EPT>(eu, t0 + (int64_t)threadIdx.x * 4, stride, end, vec, a);
        load_tile<EPT>(ev, t0 + (int64_t)threadIdx.x * 4, stride, end, vec, b);
    }
    for (; t0 < end; t0 += step) {
        const int64_t t1 = t0 + step;
        if (t1 < end) {
            load_tile<EPT>(eu, t1 + (int64_t)threadIdx.x * 4, stride, end, vec, na);
            load_tile<EPT>(ev, t1 + (int64_t)threadIdx.x * 4, stride, end, vec, nb);
        }
        uint32_t act = 0;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const bool in = (uint32_t)a[j] < (uint32_t)n && (uint32_t)b[j] < (uint32_t)n;
            bad |= !in;
            if (in && a[j] != b[j] && !(sym && a[j] > b[j])) act |= 1u << j;
        }
        // Bit tests, branch-free so that all of them are in flight at once:
        // every tag read, then every bitmap word load (an entry that is
        // inactive, or whose word is in LDS, loads word 0 instead, one hot
        // line), then the selection.
        uint32_t inga = 0, ingb = 0;  // giant-membership bits per entry
        if (filter) {
            uint32_t xa[EPT], xb[EPT], ta[EPT], tb[EPT];
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                xa[j] = (act >> j & 1) ? (uint32_t)a[j] : 0u;
                xb[j] = (act >> j & 1) ? (uint32_t)b[j] : 0u;
                ta[j] = ltag[(xa[j] >> 5) & (SLOTS - 1)];
                tb[j] = ltag[(xb[j] >> 5) & (SLOTS - 1)];
            }
            uint32_t wa[EPT], wb[EPT], la[EPT], lb[EPT], hit = 0;
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const uint32_t ka = (xa[j] >> 5) / SLOTS, kb = (xb[j] >> 5) / SLOTS;
                const bool ha = ka < kEmpty && ta[j] == ka, hb = kb < kEmpty && tb[j] == kb;
                hit |= (ha ? 1u : 0u) << (2 * j);
                hit |= (hb ? 1u : 0u) << (2 * j + 1);
                wa[j] = bits[ha ? 0u : (xa[j] >> 5)];
                wb[j] = bits[hb ? 0u : (xb[j] >> 5)];
                la[j] = lval[(xa[j] >> 5) & (SLOTS - 1)];
                lb[j] = lval[(xb[j] >> 5) & (SLOTS - 1)];
            }
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const uint32_t worda = (hit >> (2 * j) & 1) ? la[j] : wa[j];
                const uint32_t wordb = (hit >> (2 * j + 1) & 1) ? lb[j] : wb[j];
                inga |= (worda >> (xa[j] & 31) & 1u) << j;
                ingb |= (wordb >> (xb[j] & 31) & 1u) << j;
            }
            act &= ~(inga & ingb);  // both ends in the giant: already satisfied
        }
        // Parents of the endpoints outside the giant (again all issued at once;
        // an endpoint that needs none reads pi[0]).
        int32_t pa[EPT], pb[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const bool na_ = (act >> j & 1) && !(inga >> j & 1);
            const bool nb_ = (act >> j & 1) && !(ingb >> j & 1);
            const int32_t ra = ld_tree<false>(pi + (na_ ? a[j] : 0));
            const int32_t rb = ld_tree<false>(pi + (nb_ ? b[j] : 0));
            pa[j] = na_ ? ra : g;
            pb[j] = nb_ ? rb : g;
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            if (act >> j & 1) hot_climb(pi, pa[j], pb[j], halve);
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            a[j] = na[j];
            b[j] = nb[j];
        }
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

template <int SLOTS, typename TagT>
static hipError_t ahook_hot_ept(int ept, int grid, int block, hipStream_t s, const int32_t* u,
                                const int32_t* v, int64_t begin, int64_t end, bool vec, int32_t* pi,
                                int32_t n, Ctrl* ctrl, const uint32_t* bits, const uint32_t* tags,
                                const uint32_t* vals, bool halve, bool sym) {
    switch (ept) {
        case 4: k_ahook_hot<4, SLOTS, TagT><<<grid, block, 0, s>>>(u, v, begin, end, vec, pi, n, ctrl, bits, tags, vals, halve, sym); break;
        case 8:
        case 16:  // 16 would spill registers with the pipelined tile; run 8
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
