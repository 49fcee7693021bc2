/*
 * CPU oracle for connected-component labels.  TEST INFRASTRUCTURE ONLY:
 * used by tests/, the smoke check and the benchmark's CPU-baseline leg; the
 * GPU library never links, loads or calls it, and it shares no code with it.
 *
 * What it computes (Section 2, "Existing Approaches", definition of
 * connected components): every vertex of an undirected graph G = (V, E)
 * receives the id of a representative vertex of its component.  The
 * representative is the smallest vertex id of the component; this is the
 * root that the global high-to-low hooking rule (Fig. 2 Hook, Fig. 3
 * Atomic-Hook) leaves at the top of each component tree, since every parent
 * pointer it writes goes from a larger id to a smaller one.
 *
 *   label[v] = min { w in [0, n) : w and v are joined by a path of edges }
 *
 * with v joined to itself.  It is computed here by a plain sequential
 * union-find (one pass over the edges in input order, union by linking the
 * larger root under the smaller one, find with path halving), followed by a
 * single pass in increasing vertex order that resolves every vertex to its
 * root.  Nothing is parallel, blocked or reordered.
 *
 * Status values (same meaning as the GPU library's, defined separately):
 *   0  ok;  -1 bad argument;  -2 an endpoint outside [0, n).
 */
#include <stdint.h>
#include <stdlib.h>

#define ORACLE_OK 0
#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_RANGE (-2)
#define ORACLE_ERR_NOMEM (-3)

/* Root of x's tree; halves the path on the way (each visited vertex is
 * re-pointed at its grandparent), which never changes the set a vertex
 * belongs to. */
static int32_t find_root(int32_t* parent, int32_t x) {
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

/* Labels of one graph: n vertices, m edge entries (u[i], v[i]) with ids in
 * [0, n).  Self-loops and repeated pairs are allowed; either orientation of
 * an edge means the same undirected edge.  `label` receives n values. */
int32_t cc_oracle_labels(int32_t n, const int32_t* u, const int32_t* v, int64_t m,
                         int32_t* label) {
    if (n < 0 || m < 0) return ORACLE_ERR_ARG;
    if (m > 0 && (u == NULL || v == NULL)) return ORACLE_ERR_ARG;
    if (n > 0 && label == NULL) return ORACLE_ERR_ARG;
    for (int64_t i = 0; i < m; ++i) {
        if (u[i] < 0 || u[i] >= n || v[i] < 0 || v[i] >= n) return ORACLE_ERR_RANGE;
    }
    if (n == 0) return ORACLE_OK;

    int32_t* parent = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (parent == NULL) return ORACLE_ERR_NOMEM;
    for (int32_t x = 0; x < n; ++x) parent[x] = x;

    for (int64_t i = 0; i < m; ++i) {
        int32_t ru = find_root(parent, u[i]);
        int32_t rv = find_root(parent, v[i]);
        if (ru == rv) continue;
        /* Link the larger root under the smaller: every root stays the
         * minimum id of its tree. */
        if (ru < rv) parent[rv] = ru;
        else parent[ru] = rv;
    }

    /* parent[x] < x for every non-root x, so by the time x is reached its
     * parent's label is already final. */
    for (int32_t x = 0; x < n; ++x) {
        label[x] = (parent[x] == x) ? x : label[parent[x]];
    }
    free(parent);
    return ORACLE_OK;
}

/* Many independent graphs packed back to back: graph g has vertices
 * [vtx_off[g], vtx_off[g+1]) and edge entries [edge_off[g], edge_off[g+1]),
 * whose endpoints are local ids in [0, n_g).  label[vtx_off[g] + x] is the
 * local label of local vertex x.  Each graph is labelled on its own. */
int32_t cc_oracle_labels_batch(int32_t num_graphs, const int64_t* vtx_off, const int64_t* edge_off,
                               const int32_t* u, const int32_t* v, int32_t* label) {
    if (num_graphs < 0) return ORACLE_ERR_ARG;
    if (num_graphs == 0) return ORACLE_OK;
    if (vtx_off == NULL || edge_off == NULL) return ORACLE_ERR_ARG;
    if (vtx_off[0] != 0 || edge_off[0] != 0) return ORACLE_ERR_ARG;
    for (int32_t g = 0; g < num_graphs; ++g) {
        int64_t nv = vtx_off[g + 1] - vtx_off[g];
        int64_t ne = edge_off[g + 1] - edge_off[g];
        if (nv < 0 || ne < 0 || nv > INT32_MAX) return ORACLE_ERR_ARG;
    }
    for (int32_t g = 0; g < num_graphs; ++g) {
        int64_t nv = vtx_off[g + 1] - vtx_off[g];
        int64_t e0 = edge_off[g], ne = edge_off[g + 1] - edge_off[g];
        int32_t rc = cc_oracle_labels((int32_t)nv, ne ? u + e0 : NULL, ne ? v + e0 : NULL, ne,
                                      label + vtx_off[g]);
        if (rc != ORACLE_OK) return rc;
    }
    return ORACLE_OK;
}
