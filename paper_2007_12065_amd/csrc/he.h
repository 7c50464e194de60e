// Half-edges of a user-provided mesh (Sec. 4.3): internal interface between
// the C ABI and halfedges.hip.
#pragma once

#include "common.h"

namespace pl {

size_t user_halfedges_workspace(int cap);
pl_status launch_user_halfedges(const int32_t *tris, const int32_t *n_tri, int cap,
                                int32_t *he, void *ws, hipStream_t s);

}  // namespace pl
