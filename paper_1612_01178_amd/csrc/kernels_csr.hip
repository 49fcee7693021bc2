// Atomic-Hook over a CSR adjacency (row_ptr[n+1], col[m]): entry i of row r
// is the pair (r, col[i]).  The paper's hook works on any subsets of E
// (Fig. 4), so the solve is the same as for pair lists; only the way an
// entry's first endpoint is found differs.
//
// Row ids are expanded on the fly.  Each workgroup takes a tile of
// consecutive entries and finds the rows spanning it (row_ptr is int64 and
// non-decreasing) with a 32-ary search per tile end, both run at once by the
// first wave (half a wave each): 5 dependent rounds of loads for 16M rows
// instead of the 24 of a binary search, which at one tile per 2,048 entries
// otherwise dominate the pass.  The tile then loads that window of row_ptr
// into LDS, and every thread finds the row of its first entry by a binary
// search in LDS, advancing linearly for its following entries.  A tile whose
// window exceeds the LDS budget (many empty rows) searches row_ptr in device
// memory instead.
//
// With the giant filter, the row's bit is tested once per group of four
// consecutive entries (they nearly always share the row) instead of once
// per entry: on a skewed CSR graph the per-entry cost drops to one bit test.
// `sym`: the adjacency is symmetric (every pair stored in both rows), so
// only the entries with col > row are hooked: the copy of each pair kept is
// the one in the smaller endpoint's row, so the first segments (the first
// rows) already join the low ids to the whole graph and the giant component
// forms before the filter samples for it.  Keeping col < row instead hooks
// only pairs inside the row prefix seen so far, and the filter finds no
// giant until late.
//
// PLAIN: the atomic-free Hook (Fig. 2) instead of the CAS climb: where an
// entry's two parents differ, the larger is pointed at the smaller with a
// plain store.  Stores may overwrite each other, so this pass alone does not
// finish the solve: it is the first pass of the hybrid plan, whose closing
// Atomic-Hook pass over all entries restores every link lost here.  The
// kernel then has no CAS, so its stores may use workgroup scope.
#include "kernels.hpp"

namespace hookcc {

constexpr int kCsrWindow = 4096;  // rows of row_ptr held in LDS per tile

// Largest r in [0, n - 1] with rp[r] <= e, by lanes [half*32, half*32 + 32)
// of the calling wave (every lane of the wave must call it; each half-wave
// searches for its own e).  Each round, the half-wave's lanes probe 32
// evenly spaced rows of the current interval, and the interval shrinks to
// the gap after the last probe that is still <= e.
__device__ __forceinline__ int64_t upper_row32(const int64_t* __restrict__ rp, int32_t n, int64_t e) {
    const int lane = threadIdx.x & 63;
    const int sub = lane & 31;
    const int half = lane >> 5;
    int64_t lo = 0, hi = (int64_t)n - 1;  // answer in [lo, hi]; rp[0] <= e assumed
    while (true) {
        const int64_t span = hi - lo + 1;
        const bool last = span <= 32;
        // probe k (1..32) of this half-wave
        const int64_t probe = last ? lo + sub : lo + (span * (sub + 1)) / 33;
        const bool ok = probe <= hi && rp[probe] <= e;
        const uint64_t mk = __ballot(ok);
        const uint32_t mine = (uint32_t)(mk >> (32 * half));
        // rp is non-decreasing, so the probes that pass form a prefix
        const int cnt = __popc(mine);
        if (last) return lo + cnt - 1 < lo ? lo : lo + cnt - 1;
        // probes p_1 < ... < p_32; the answer lies in [p_cnt, p_{cnt+1} - 1]
        const int64_t nlo = cnt ? lo + (span * cnt) / 33 : lo;
        const int64_t nhi = cnt < 32 ? lo + (span * (cnt + 1)) / 33 - 1 : hi;
        lo = nlo;
        hi = nhi < lo ? lo : nhi;
    }
}

__device__ __forceinline__ int64_t upper_row(const int64_t* __restrict__ rp, int64_t lo, int64_t hi,
                                             int64_t e) {
    // largest r in [lo, hi] with rp[r] <= e (rp[lo] <= e assumed)
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (rp[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int EPT, bool PLAIN>
__global__ __launch_bounds__(512) void k_ahook_csr(const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col, int32_t n,
                                                   int64_t begin, int64_t end, int32_t* pi,
                                                   Ctrl* ctrl, const uint32_t* __restrict__ bits,
                                                   bool filter, bool sym, bool halve) {
    __shared__ int64_t win[kCsrWindow + 1];
    __shared__ int64_t r_lo_sh, r_hi_sh;
    const int64_t tile = (int64_t)blockDim.x * EPT;
    const int64_t t0 = begin + (int64_t)blockIdx.x * tile;
    const int64_t t1 = min(end, t0 + tile);  // exclusive
    if (threadIdx.x < 64) {
        // half-wave 0 finds the row of t0, half-wave 1 the row of t1 - 1
        const int64_t r = upper_row32(row_ptr, n, threadIdx.x < 32 ? t0 : t1 - 1);
        if (threadIdx.x == 0) r_lo_sh = r;
        if (threadIdx.x == 32) r_hi_sh = r;
    }
    __syncthreads();
    const int64_t r_lo = r_lo_sh;
    const int64_t r_hi = r_hi_sh < r_lo ? r_lo : r_hi_sh;  // only a malformed row_ptr inverts them
    const bool in_lds = r_hi - r_lo + 1 <= kCsrWindow;
    if (in_lds)
        for (int64_t r = r_lo + threadIdx.x; r <= r_hi + 1; r += blockDim.x) win[r - r_lo] = row_ptr[r];
    __syncthreads();
    const bool use_filter = !PLAIN && filter && ctrl->filter_on;
    const int32_t g = use_filter ? ctrl->giant : 0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < EPT / 4; ++k) {
        const int64_t e0 = t0 + (int64_t)k * blockDim.x * 4 + (int64_t)threadIdx.x * 4;
        if (e0 >= t1) continue;
        // row of e0, then of the next three entries
        int64_t r;
        if (in_lds) {
            int64_t lo = 0, hi = r_hi - r_lo;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (win[mid] <= e0) lo = mid;
                else hi = mid - 1;
            }
            r = r_lo + lo;
        } else {
            r = upper_row(row_ptr, r_lo, r_hi, e0);
        }
        int32_t a[4], b[4];
        uint32_t act = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t e = e0 + j;
            if (e >= t1) {
                a[j] = b[j] = 0;
                continue;
            }
            // advance to the row that owns e (rows may be empty); stays
            // inside the window even if row_ptr is malformed.  Two loops,
            // not one with a select between the LDS and the global row_ptr,
            // which would become flat loads.
            if (in_lds) {
                while (r < r_hi && win[r + 1 - r_lo] <= e) ++r;
            } else {
                while (r < (int64_t)n - 1 && row_ptr[r + 1] <= e) ++r;
            }
            a[j] = (int32_t)r;
            b[j] = __builtin_nontemporal_load(col + e);
            const bool in = (uint32_t)b[j] < (uint32_t)n;
            bad |= !in;
            if (in && a[j] != b[j] && !(sym && b[j] < a[j])) act |= 1u << j;
        }
        if (!act) continue;
        int32_t pa[4], pb[4];
        uint32_t inga = 0, ingb = 0;
        if (use_filter) {
            // the row's bit once per group (the group spans at most a few rows)
            const uint32_t ra = (uint32_t)a[0];
            const uint32_t ba0 = bits[ra >> 5] >> (ra & 31) & 1;
            uint32_t wb[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) wb[j] = bits[(act >> j & 1) ? ((uint32_t)b[j] >> 5) : 0u];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t x = (uint32_t)a[j];
                const uint32_t bax = (x == ra) ? ba0 : (bits[x >> 5] >> (x & 31) & 1);
                inga |= bax << j;
                ingb |= (wb[j] >> ((uint32_t)b[j] & 31) & 1u) << j;
            }
            act &= ~(inga & ingb);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool na = (act >> j & 1) && !(inga >> j & 1);
            const bool nb = (act >> j & 1) && !(ingb >> j & 1);
            const int32_t xa = ld_tree<false>(pi + (na ? a[j] : 0));
            const int32_t xb = ld_tree<false>(pi + (nb ? b[j] : 0));
            pa[j] = na ? xa : g;
            pb[j] = nb ? xb : g;
        }
        if (PLAIN) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if ((act >> j & 1) && pa[j] != pb[j])
                    st_rlx(pi + (pa[j] > pb[j] ? pa[j] : pb[j]), pa[j] > pb[j] ? pb[j] : pa[j]);
            }
            continue;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!(act >> j & 1)) continue;
            int32_t pu = pa[j], pv = pb[j];
            uint32_t step = 0;
            // Atomic-Hook climb (Fig. 3, top) with optional path halving; see
            // atomic_hook in kernels_core.hip for why it is correct and finite.
            while (pu != pv) {
                const int32_t H = pu > pv ? pu : pv;
                const int32_t L = pu > pv ? pv : pu;
                int32_t found = ld_tree<false>(pi + H);
                if (found == H) {
                    found = cas_root(pi + H, H, L);
                    if (found == H) break;
                }
                pu = ld_tree<false>(pi + found);
                pv = ld_tree<false>(pi + L);
                if (halve && pu != found && step++ % kHalveEveryFiltered == 0)
                    halve_to(pi + H, pu);
            }
        }
    }
    if (bad) atomicOr(&ctrl->status, kStatusRange);
}

// Frontier compaction of a CSR adjacency for the hybrid plan (after its
// atomic-free pass and a Multi-Jump, so pi is a forest of stars): the entries
// whose endpoints have different roots are written as root pairs to `fr`
// (capacity m), their number accumulated in *count.  Rows are found as in
// k_ahook_csr; positions come from wave ballots, per-wave totals in LDS and
// one atomicAdd per workgroup.
template <int EPT>
__global__ __launch_bounds__(512) void k_compact_csr(const int64_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col, int32_t n,
                                                     int64_t m, const int32_t* pi, int2* fr,
                                                     uint32_t* count, bool sym) {
    __shared__ int64_t win[kCsrWindow + 1];
    __shared__ int64_t r_sh[2];
    __shared__ uint32_t wave_off[512 / 64];
    __shared__ uint32_t base_sh;
    const int64_t tile = (int64_t)blockDim.x * EPT;
    const int64_t t0 = (int64_t)blockIdx.x * tile;
    const int64_t t1 = min(m, t0 + tile);  // exclusive
    if (threadIdx.x < 64) {
        const int64_t r = upper_row32(row_ptr, n, threadIdx.x < 32 ? t0 : t1 - 1);
        if (threadIdx.x == 0) r_sh[0] = r;
        if (threadIdx.x == 32) r_sh[1] = r;
    }
    __syncthreads();
    const int64_t r_lo = r_sh[0];
    const int64_t r_hi = r_sh[1] < r_lo ? r_lo : r_sh[1];
    const bool in_lds = r_hi - r_lo + 1 <= kCsrWindow;
    if (in_lds)
        for (int64_t r = r_lo + threadIdx.x; r <= r_hi + 1; r += blockDim.x) win[r - r_lo] = row_ptr[r];
    __syncthreads();
    int32_t qa[EPT], qb[EPT];
    uint32_t act = 0;
#pragma unroll
    for (int k = 0; k < EPT / 4; ++k) {
        const int64_t e0 = t0 + (int64_t)k * blockDim.x * 4 + (int64_t)threadIdx.x * 4;
        int64_t r = r_lo;
        if (e0 < t1) {
            if (in_lds) {
                int64_t lo = 0, hi = r_hi - r_lo;
                while (lo < hi) {
                    const int64_t mid = (lo + hi + 1) >> 1;
                    if (win[mid] <= e0) lo = mid;
                    else hi = mid - 1;
                }
                r = r_lo + lo;
            } else {
                r = upper_row(row_ptr, r_lo, r_hi, e0);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * k + j;
            const int64_t e = e0 + j;
            qa[i] = qb[i] = 0;
            if (e >= t1) continue;
            if (in_lds) {
                while (r < r_hi && win[r + 1 - r_lo] <= e) ++r;
            } else {
                while (r < (int64_t)n - 1 && row_ptr[r + 1] <= e) ++r;
            }
            const int32_t a = (int32_t)r, b = __builtin_nontemporal_load(col + e);
            if ((uint32_t)b >= (uint32_t)n || a == b || (sym && b < a)) continue;
            qa[i] = ld_tree<false>(pi + a);
            qb[i] = ld_tree<false>(pi + b);
            if (qa[i] != qb[i]) act |= 1u << i;
        }
    }
    // positions: per slot a wave ballot, lanes below counted with mbcnt
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t pos[EPT];
    uint32_t run = 0;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const uint64_t mk = __ballot((act >> i) & 1);
        pos[i] = run + __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
        run += (uint32_t)__popcll(mk);
    }
    if (lane == 0) wave_off[wave] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            const uint32_t t = wave_off[w];
            wave_off[w] = acc;
            acc += t;
        }
        base_sh = acc ? atomicAdd(count, acc) : 0u;
    }
    __syncthreads();
    const uint64_t at = (uint64_t)base_sh + wave_off[wave];
#pragma unroll
    for (int i = 0; i < EPT; ++i)
        if ((act >> i) & 1) fr[at + pos[i]] = int2{qa[i], qb[i]};
}

hipError_t launch_compact_csr(const int64_t* row_ptr, const int32_t* col, int32_t n, int64_t m,
                              const int32_t* pi, int2* fr, uint32_t* count, bool sym,
                              hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    constexpr int EPT = 8;
    constexpr int kBlock = 512;
    const int64_t grid64 = (m + kBlock * EPT - 1) / (kBlock * EPT);
    if (grid64 > 0x7fffffff) return hipErrorInvalidValue;
    k_compact_csr<EPT><<<(int)grid64, kBlock, 0, s>>>(row_ptr, col, n, m, pi, fr, count, sym);
    return hipGetLastError();
}

// Entry-count check of a CSR adjacency: status bit kStatusRange when
// row_ptr is not non-decreasing from 0 to m (done on the device, one pass).
__global__ __launch_bounds__(256) void k_csr_check(const int64_t* __restrict__ row_ptr, int32_t n,
                                                   int64_t m, Ctrl* ctrl) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n) return;
    bool bad = false;
    if (r == 0) bad = row_ptr[0] != 0;
    if (r == n) bad = row_ptr[n] != m;
    if (r < n) bad = bad || row_ptr[r + 1] < row_ptr[r];
    if (bad) atomicOr(&ctrl->status, kStatusRange);
}

hipError_t launch_csr_check(const int64_t* row_ptr, int32_t n, int64_t m, Ctrl* ctrl,
                            hipStream_t s) {
    const int grid = (int)(((int64_t)n + 1 + 255) / 256);
    k_csr_check<<<grid, 256, 0, s>>>(row_ptr, n, m, ctrl);
    return hipGetLastError();
}

hipError_t launch_ahook_csr(const int64_t* row_ptr, const int32_t* col, int32_t n, int64_t begin,
                            int64_t end, int32_t* pi, Ctrl* ctrl, const uint32_t* bits, bool sym,
                            bool halve, bool plain, hipStream_t s) {
    if (end <= begin || n <= 0) return hipSuccess;
    // 512 threads x 8 entries per tile: measured on R-MAT 24 (2^29 entries)
    // 4.97 ms against 5.86 (256 x 8), 5.49 (256 x 16), 5.13 (1024 x 8)
    constexpr int EPT = 8;
    constexpr int kBlock = 512;
    const int64_t tile = kBlock * EPT;
    const int64_t grid64 = (end - begin + tile - 1) / tile;
    if (grid64 > 0x7fffffff) return hipErrorInvalidValue;
    if (plain)
        k_ahook_csr<EPT, true><<<(int)grid64, kBlock, 0, s>>>(row_ptr, col, n, begin, end, pi, ctrl,
                                                           nullptr, false, sym, false);
    else
        k_ahook_csr<EPT, false><<<(int)grid64, kBlock, 0, s>>>(row_ptr, col, n, begin, end, pi, ctrl,
                                                            bits, bits != nullptr, sym, halve);
    return hipGetLastError();
}

}  // namespace hookcc
