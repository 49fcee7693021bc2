// Host engine of libhookcc: plans, workspace cache, launch sequences.
// Internal; the public ABI is include/hookcc.h.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/hookcc.h"
#include "kernels.hpp"

namespace hookcc {

// Records `msg` as the calling thread's last error and returns `code`.
int32_t fail(int32_t code, const std::string& msg);
const char* last_error();

int32_t labels_impl(int32_t n, const int32_t* u, const int32_t* v, int64_t m, int32_t* out,
                    const cc_options* opts, void* workspace, size_t ws_bytes, hipStream_t s,
                    cc_stats* st);
size_t workspace_bytes_impl(int32_t n, int64_t m, const cc_options* opts);
// The same solve with the workspace in a fixed device array (cc_labels_noalloc).
int32_t labels_noalloc_impl(int32_t n, const int32_t* u, const int32_t* v, int64_t m,
                            int32_t* out, const cc_options* opts, hipStream_t s, cc_stats* st);

// Independent graphs given by descriptors (device arrays); synchronous on s.
// opts (nullable): `segments` (per-graph segment cap of the LDS solver),
// `path_halving` (in the LDS climb) and `graph` are used.  `workspace`
// (nullable, 256-byte aligned device memory of ws_bytes) replaces the
// stream's pool; with `ws_needed` non-null nothing runs and the workspace
// size the call needs is stored there.
int32_t list_impl(int32_t count, const cc_graph* graphs, const cc_options* opts, hipStream_t s,
                  cc_stats* st, void* workspace = nullptr, size_t ws_bytes = 0,
                  size_t* ws_needed = nullptr);
// Graphs packed back to back with host offsets; synchronous on s.
int32_t batch_impl(int32_t B, const int64_t* vo, const int64_t* eo, const int32_t* u,
                   const int32_t* v, int32_t* out, const cc_options* opts, hipStream_t s,
                   cc_stats* st);

// Graphs packed back to back with DEVICE offsets, all LDS-solved (n <= max_n
// <= CC_BATCH_LDS_MAX_N); ordered and described on the device; synchronous on s.
int32_t batch_device_impl(int32_t B, const int64_t* vo, const int64_t* eo, const int32_t* u,
                          const int32_t* v, int32_t* out, int32_t max_n, const cc_options* opts,
                          hipStream_t s, cc_stats* st);

// Edges in host memory, streamed in chunks (see engine.cpp).
int32_t stream_impl(int32_t n, const int32_t* hu, const int32_t* hv, int64_t m, int32_t* out,
                    int64_t chunk, const cc_options* opts, hipStream_t s, cc_stats* st);

// CSR adjacency input (see engine.cpp).
int32_t csr_impl(int32_t n, const int64_t* row_ptr, const int32_t* col, int64_t m, int32_t* out,
                 const cc_options* opts, hipStream_t s, cc_stats* st);

int32_t probe_impl(int32_t mode, const int32_t* u, const int32_t* v, int64_t m, const void* table,
                   int32_t n, hipStream_t s);
void release_impl();
// Status of the last no-sync call on s (see cc_stream_status).
int32_t stream_status_impl(hipStream_t s);

}  // namespace hookcc
