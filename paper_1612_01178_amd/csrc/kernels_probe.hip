// Memory-ceiling probes: the edge stream alone, the stream plus two random
// 4-byte gathers of an n-entry table per entry (the tree-array access
// pattern of a hook pass), the stream plus two bit lookups in an n-bit
// bitmap, and the stream plus one agent-scope compare-and-swap per entry on
// a random table slot (the hooking atomic; the table must hold t[x] = x: the
// succeeding form swaps x for x, the failing form expects -1, so the table
// never changes).  Each folds what it read into one word so nothing is
// optimised away.  Same tiling as the hook kernels: 16 entries per thread,
// 256 threads.
#include "kernels.hpp"

namespace hookcc {

typedef int32_t v4i __attribute__((ext_vector_type(4)));

template <int MODE>
__global__ __launch_bounds__(256) void k_probe(const int32_t* __restrict__ eu,
                                               const int32_t* __restrict__ ev, int64_t m,
                                               const int32_t* __restrict__ table,
                                               const uint32_t* __restrict__ bits, int32_t n,
                                               uint32_t* sink) {
    constexpr int EPT = 16;
    const int64_t stride = (int64_t)blockDim.x * 4;
    const int64_t e0 = (int64_t)blockIdx.x * blockDim.x * EPT + (int64_t)threadIdx.x * 4;
    uint32_t acc = 0;
    int32_t a[EPT], b[EPT];
#pragma unroll
    for (int k = 0; k < EPT / 4; ++k) {
        const int64_t e = e0 + k * stride;
        if (e + 3 < m) {
            v4i q = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(eu + e));
            v4i r = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(ev + e));
            a[4 * k] = q.x; a[4 * k + 1] = q.y; a[4 * k + 2] = q.z; a[4 * k + 3] = q.w;
            b[4 * k] = r.x; b[4 * k + 1] = r.y; b[4 * k + 2] = r.z; b[4 * k + 3] = r.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a[4 * k + j] = e + j < m ? eu[e + j] : 0;
                b[4 * k + j] = e + j < m ? ev[e + j] : 0;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const uint32_t x = (uint32_t)a[j], y = (uint32_t)b[j];
        uint32_t val;
        if (MODE == 0) {
            val = x + 3 * y;
        } else if (MODE == 1) {
            val = (x < (uint32_t)n && y < (uint32_t)n)
                      ? (uint32_t)table[x] + 3u * (uint32_t)table[y] : 0u;
        } else if (MODE == 2) {
            val = (x < (uint32_t)n && y < (uint32_t)n)
                      ? ((bits[x >> 5] >> (x & 31)) & 1u) | (((bits[y >> 5] >> (y & 31)) & 1u) << 1)
                      : 0u;
        } else if (MODE == 3) {  // bitmap words read with the non-temporal hint
            val = (x < (uint32_t)n && y < (uint32_t)n)
                      ? ((__builtin_nontemporal_load(bits + (x >> 5)) >> (x & 31)) & 1u) |
                            (((__builtin_nontemporal_load(bits + (y >> 5)) >> (y & 31)) & 1u) << 1)
                      : 0u;
        } else if (MODE == 4) {  // bitmap words read as agent-scope atomics (past the L1)
            val = (x < (uint32_t)n && y < (uint32_t)n)
                      ? ((__hip_atomic_load(bits + (x >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> (x & 31)) & 1u) |
                            (((__hip_atomic_load(bits + (y >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> (y & 31)) & 1u) << 1)
                      : 0u;
        } else {  // one agent-scope CAS on slot x: 5 succeeds (x -> x), 6 fails (expects -1)
            val = 0;
            if (x < (uint32_t)n) {
                int32_t expected = MODE == 5 ? (int32_t)x : -1;
                __hip_atomic_compare_exchange_strong(const_cast<int32_t*>(table) + x, &expected,
                                                     (int32_t)x, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                val = (uint32_t)expected + y;
            }
        }
        acc = ((acc << 5) | (acc >> 27)) ^ val;  // rotate-xor: every value matters
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;  // practically never taken
}

static hipError_t probe(int mode, const int32_t* u, const int32_t* v, int64_t m,
                        const int32_t* table, const uint32_t* bits, int32_t n, uint32_t* sink,
                        hipStream_t s) {
    if (m <= 0) return hipSuccess;
    if (((uintptr_t)u & 15) || ((uintptr_t)v & 15)) return hipErrorInvalidValue;
    const int64_t tile = 256 * 16;
    const int grid = (int)((m + tile - 1) / tile);
    switch (mode) {
        case 0: k_probe<0><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
        case 1: k_probe<1><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
        case 2: k_probe<2><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
        case 3: k_probe<3><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
        case 4: k_probe<4><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
        case 5: k_probe<5><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
        default: k_probe<6><<<grid, 256, 0, s>>>(u, v, m, table, bits, n, sink); break;
    }
    return hipGetLastError();
}

hipError_t launch_probe_stream(const int32_t* u, const int32_t* v, int64_t m, uint32_t* sink,
                               hipStream_t s) {
    return probe(0, u, v, m, nullptr, nullptr, 0, sink, s);
}
hipError_t launch_probe_gather(const int32_t* u, const int32_t* v, int64_t m, const int32_t* table,
                               int32_t n, uint32_t* sink, hipStream_t s) {
    return probe(1, u, v, m, table, nullptr, n, sink, s);
}
hipError_t launch_probe_cas(const int32_t* u, const int32_t* v, int64_t m, int32_t* table,
                            int32_t n, bool fail, uint32_t* sink, hipStream_t s) {
    return probe(fail ? 6 : 5, u, v, m, table, nullptr, n, sink, s);
}
hipError_t launch_probe_bitgather(const int32_t* u, const int32_t* v, int64_t m,
                                  const uint32_t* bits, int32_t n, int variant, uint32_t* sink,
                                  hipStream_t s) {
    return probe(2 + variant, u, v, m, nullptr, bits, n, sink, s);
}

}  // namespace hookcc
