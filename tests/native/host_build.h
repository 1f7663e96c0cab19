// Test harness (CPU only): host construction of the library's graph layout.
#pragma once

#include <string>

#include "../../paper_2609_21848_amd/csrc/internal.h"

namespace dbbc {

// Build the relabelled CSR pair from an edge list (host memory).  Returns a
// DBBC status and fills err on failure.
int build_host_graph(int32_t n_u, int32_t n_v, int64_t m, const int32_t* u, const int32_t* v,
                     const int8_t* sign, uint32_t flags, HostGraph& g, std::string& err);

}  // namespace dbbc
