// Autotuner placeholder (filled in with the search below).
#include "bfs_internal.h"
namespace bfs {
void autotune(bfs_graph* g, const int32_t* roots, int32_t num_roots, int32_t mode, bfs_tunables* best) {
    (void)g; (void)roots; (void)num_roots; (void)mode; (void)best;
    fail(BFS_E_INTERNAL, "autotuner not built yet");
}
}  // namespace bfs
