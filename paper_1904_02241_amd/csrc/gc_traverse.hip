// Traversal (BFS / SSSP): not yet built.
#include "gc_internal.h"

namespace gcx {

hipError_t bfs_run(gc_graph, gc_tocab, int32_t, int32_t*, int32_t*, uint32_t, hipStream_t) {
  return hipErrorNotSupported;
}

hipError_t sssp_run(gc_graph, gc_tocab, int32_t, int32_t*, int32_t*, uint32_t, hipStream_t, bool*) {
  return hipErrorNotSupported;
}

}  // namespace gcx
