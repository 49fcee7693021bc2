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
