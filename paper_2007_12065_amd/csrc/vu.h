// Vertex update from filtered normals: internal interface between the C ABI
// and vertex.hip.
#pragma once

#include "common.h"

namespace pl {

size_t vertex_update_workspace(int M, int N, int iterations);
pl_status launch_vertex_update(const float *in, float *out, int M, int N, const void *normals,
                               pl_dtype ndt, int iterations, void *ws, hipStream_t s);

}  // namespace pl
