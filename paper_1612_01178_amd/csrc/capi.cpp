// C ABI of libhookcc (declared in include/hookcc.h): thin wrappers over the
// engine; no exception or C++ type crosses this boundary.
#include <cstring>

#include "engine.hpp"

using namespace hookcc;

extern "C" {

void cc_options_init(cc_options* opts) {
    if (!opts) return;
    std::memset(opts, 0, sizeof *opts);
    opts->filter = CC_FILTER_AUTO;
}

int32_t cc_labels(int32_t n, const int32_t* edges_u, const int32_t* edges_v, int64_t m,
                  int32_t* out_label) {
    return labels_impl(n, edges_u, edges_v, m, out_label, nullptr, nullptr, 0, nullptr, nullptr);
}

int32_t cc_labels_ex(int32_t n, const int32_t* edges_u, const int32_t* edges_v, int64_t m,
                     int32_t* out_label, const cc_options* opts, void* workspace,
                     size_t workspace_bytes, void* stream, cc_stats* stats) {
    return labels_impl(n, edges_u, edges_v, m, out_label, opts, workspace, workspace_bytes,
                       static_cast<hipStream_t>(stream), stats);
}

size_t cc_workspace_bytes(int32_t n, int64_t m, const cc_options* opts) {
    return workspace_bytes_impl(n, m, opts);
}

int32_t cc_labels_noalloc(int32_t n, const int32_t* edges_u, const int32_t* edges_v, int64_t m,
                          int32_t* out_label, const cc_options* opts, void* stream,
                          cc_stats* stats) {
    return labels_noalloc_impl(n, edges_u, edges_v, m, out_label, opts,
                               static_cast<hipStream_t>(stream), stats);
}

int32_t cc_labels_batch(int32_t num_graphs, const int64_t* vtx_off, const int64_t* edge_off,
                        const int32_t* edges_u, const int32_t* edges_v, int32_t* out_label) {
    return batch_impl(num_graphs, vtx_off, edge_off, edges_u, edges_v, out_label, nullptr, nullptr,
                      nullptr);
}

int32_t cc_labels_batch_ex(int32_t num_graphs, const int64_t* vtx_off, const int64_t* edge_off,
                           const int32_t* edges_u, const int32_t* edges_v, int32_t* out_label,
                           const cc_options* opts, void* stream, cc_stats* stats) {
    return batch_impl(num_graphs, vtx_off, edge_off, edges_u, edges_v, out_label, opts,
                      static_cast<hipStream_t>(stream), stats);
}

int32_t cc_labels_batch_device(int32_t num_graphs, const int64_t* vtx_off,
                               const int64_t* edge_off, const int32_t* edges_u,
                               const int32_t* edges_v, int32_t* out_label, int32_t max_n,
                               const cc_options* opts, void* stream, cc_stats* stats) {
    return batch_device_impl(num_graphs, vtx_off, edge_off, edges_u, edges_v, out_label, max_n,
                             opts, static_cast<hipStream_t>(stream), stats);
}

int32_t cc_labels_list(int32_t count, const cc_graph* graphs, const cc_options* opts, void* stream,
                       cc_stats* stats) {
    return list_impl(count, graphs, opts, static_cast<hipStream_t>(stream), stats, nullptr, 0,
                     nullptr);
}

int32_t cc_labels_host(int32_t n, const int32_t* host_u, const int32_t* host_v, int64_t m,
                       int32_t* out_label, int64_t chunk_entries, const cc_options* opts,
                       void* stream, cc_stats* stats) {
    return stream_impl(n, host_u, host_v, m, out_label, chunk_entries, opts,
                       static_cast<hipStream_t>(stream), stats);
}

int32_t cc_labels_csr(int32_t n, const int64_t* row_ptr, const int32_t* col, int64_t m,
                      int32_t* out_label, const cc_options* opts, void* stream, cc_stats* stats) {
    return csr_impl(n, row_ptr, col, m, out_label, opts, static_cast<hipStream_t>(stream), stats);
}

int32_t cc_probe(int32_t mode, const int32_t* edges_u, const int32_t* edges_v, int64_t m,
                 const void* table, int32_t n, void* stream) {
    return probe_impl(mode, edges_u, edges_v, m, table, n, static_cast<hipStream_t>(stream));
}

const char* cc_last_error(void) { return last_error(); }

void cc_release(void) { release_impl(); }

int32_t cc_stream_status(void* stream) { return stream_status_impl(static_cast<hipStream_t>(stream)); }

const char* cc_version(void) { return "hookcc 0.2 (gfx950)"; }

}  // extern "C"
