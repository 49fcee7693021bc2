// Seeded synthetic graph generators (input plumbing shared by the tests, the
// CPU oracle and the GPU solver; holds none of the connected-components
// arithmetic).
//
// Every random number is a counter-based draw: the i-th output of a SplitMix64
// stream (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) whose starting state is itself derived from
// (seed, stream).  Draw i therefore does not depend on draws 0..i-1, so any
// slice of an edge list can be produced independently and in parallel, and the
// output is the same for any thread count.
//
// Built with g++ into libgraphgen.so and driven from graphgen/__init__.py.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ULL;

inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// Starting state of stream `stream` under `seed`: output number `stream` of a
// SplitMix64 generator started at `seed`.
inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return mix64(seed + (stream + 1) * kGamma);
}

// Output number `i` of the SplitMix64 generator started at `key`.
inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * kGamma); }

// Uniform integer in [0, k) for 0 < k <= 2^32 from the high 32 bits of a draw
// (multiply-shift; the bias is below 2^-32 * k and irrelevant here).
inline uint32_t below(uint64_t x, uint64_t k) { return (uint32_t)(((x >> 32) * k) >> 32); }

template <class F>
void parallel_for(int64_t count, int threads, F&& body) {
    if (threads <= 1 || count < (1 << 16)) {
        body(0, count);
        return;
    }
    std::vector<std::thread> pool;
    int64_t chunk = (count + threads - 1) / threads;
    for (int t = 0; t < threads; ++t) {
        int64_t lo = t * chunk, hi = std::min<int64_t>(count, lo + chunk);
        if (lo >= hi) break;
        pool.emplace_back([=, &body] { body(lo, hi); });
    }
    for (auto& th : pool) th.join();
}

}  // namespace

extern "C" {

// Raw draws `start .. start+count-1` of stream (seed, stream).
void gg_draws(uint64_t seed, uint64_t stream, int64_t start, int64_t count, uint64_t* out) {
    uint64_t key = stream_key(seed, stream);
    for (int64_t i = 0; i < count; ++i) out[i] = draw(key, (uint64_t)(start + i));
}

// Seeded uniform permutation of [0, n) by Fisher-Yates (Durstenfeld's
// descending form); swap partner for position i is draw i reduced to [0, i].
void gg_permutation(int32_t n, uint64_t seed, uint64_t stream, int32_t* perm) {
    uint64_t key = stream_key(seed, stream);
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    for (int64_t i = (int64_t)n - 1; i > 0; --i) {
        int64_t j = below(draw(key, (uint64_t)i), (uint64_t)i + 1);
        std::swap(perm[i], perm[j]);
    }
}

// m independent pairs with both ends uniform in [0, k): pair e uses draw e,
// high 32 bits -> u, low 32 bits -> v.
void gg_uniform_pairs(int64_t m, int64_t k, uint64_t seed, uint64_t stream, int32_t* u,
                      int32_t* v, int threads) {
    uint64_t key = stream_key(seed, stream);
    parallel_for(m, threads, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; ++e) {
            uint64_t x = draw(key, (uint64_t)e);
            u[e] = (int32_t)below(x, (uint64_t)k);
            v[e] = (int32_t)below(x << 32, (uint64_t)k);
        }
    });
}

// R-MAT pairs (Chakrabarti, Zhan and Faloutsos, SDM 2004) without noise: for
// each of `scale` levels, from the most significant bit down, a uniform
// 32-bit number r picks quadrant a (r < tA: bits 0,0), b (r < tAB: 0,1),
// c (r < tABC: 1,0) or d (1,1) for the (u, v) bit pair.  Edge e, level l uses
// half (l & 1) of draw e * ceil(scale/2) + l/2.
void gg_rmat_pairs(int32_t scale, int64_t m, uint32_t tA, uint32_t tAB, uint32_t tABC,
                   uint64_t seed, uint64_t stream, int32_t* u, int32_t* v, int threads) {
    uint64_t key = stream_key(seed, stream);
    const int64_t per_edge = (scale + 1) / 2;
    parallel_for(m, threads, [&](int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; ++e) {
            uint32_t a = 0, b = 0;
            uint64_t x = 0;
            for (int32_t l = 0; l < scale; ++l) {
                if ((l & 1) == 0) x = draw(key, (uint64_t)(e * per_edge + l / 2));
                uint32_t r = (l & 1) ? (uint32_t)x : (uint32_t)(x >> 32);
                uint32_t ub, vb;
                if (r < tA) { ub = 0; vb = 0; }
                else if (r < tAB) { ub = 0; vb = 1; }
                else if (r < tABC) { ub = 1; vb = 0; }
                else { ub = 1; vb = 1; }
                a = (a << 1) | ub;
                b = (b << 1) | vb;
            }
            u[e] = (int32_t)a;
            v[e] = (int32_t)b;
        }
    });
}

// x[i] = map[x[i]] for i < m (vertex relabelling by a permutation).
void gg_apply_map(int64_t m, const int32_t* map, int32_t* x, int threads) {
    parallel_for(m, threads, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) x[i] = map[x[i]];
    });
}

// Number of 4-neighbour lattice edges of a W x H grid.
int64_t gg_grid_edge_count(int32_t W, int32_t H) {
    return (int64_t)(W - 1) * H + (int64_t)W * (H - 1);
}

// W x H 4-neighbour lattice, vertex id = r * W + c (row-major, not permuted).
// Lattice edges are enumerated by lower endpoint in row-major order, the
// horizontal edge (v, v+1) before the vertical edge (v, v+W).  Exactly `ndel`
// of them, chosen by a seeded partial Fisher-Yates shuffle of the edge
// indices, are deleted; the rest are written in enumeration order.  Returns
// the number written (edge count - ndel), or -1 if ndel is out of range.
int64_t gg_grid(int32_t W, int32_t H, int64_t ndel, uint64_t seed, uint64_t stream, int32_t* u,
                int32_t* v) {
    const int64_t E = gg_grid_edge_count(W, H);
    if (ndel < 0 || ndel > E) return -1;
    uint64_t key = stream_key(seed, stream);
    std::vector<uint8_t> dead(E, 0);
    if (ndel > 0) {
        std::vector<int64_t> idx(E);
        for (int64_t i = 0; i < E; ++i) idx[i] = i;
        for (int64_t i = 0; i < ndel; ++i) {
            int64_t j = i + (int64_t)below(draw(key, (uint64_t)i), (uint64_t)(E - i));
            std::swap(idx[i], idx[j]);
            dead[idx[i]] = 1;
        }
    }
    int64_t e = 0, out = 0;
    for (int64_t r = 0; r < H; ++r) {
        for (int64_t c = 0; c < W; ++c) {
            int64_t x = r * W + c;
            if (c + 1 < W) {
                if (!dead[e]) { u[out] = (int32_t)x; v[out] = (int32_t)(x + 1); ++out; }
                ++e;
            }
            if (r + 1 < H) {
                if (!dead[e]) { u[out] = (int32_t)x; v[out] = (int32_t)(x + W); ++out; }
                ++e;
            }
        }
    }
    return out;
}

// Edges of many independent graphs packed back to back: graph g owns entries
// [edge_off[g], edge_off[g+1]) and its local endpoints are uniform in
// [0, nv[g]), drawn from stream stream_base + g.
void gg_batch_uniform_pairs(int32_t num_graphs, const int64_t* edge_off, const int32_t* nv,
                            uint64_t seed, uint64_t stream_base, int32_t* u, int32_t* v,
                            int threads) {
    parallel_for(num_graphs, threads, [&](int64_t lo, int64_t hi) {
        for (int64_t g = lo; g < hi; ++g) {
            uint64_t key = stream_key(seed, stream_base + (uint64_t)g);
            const int64_t base = edge_off[g], cnt = edge_off[g + 1] - edge_off[g];
            const uint64_t k = (uint64_t)nv[g];
            for (int64_t e = 0; e < cnt; ++e) {
                uint64_t x = draw(key, (uint64_t)e);
                u[base + e] = (int32_t)below(x, k);
                v[base + e] = (int32_t)below(x << 32, k);
            }
        }
    });
}

}  // extern "C"
