// Server placeholder.
#include "bfs_internal.h"
extern "C" {
int bfs_server_create(const bfs_server_config*, bfs_server** out) { return out ? BFS_E_INTERNAL : BFS_E_INVALID_ARG; }
int bfs_server_add_graph(bfs_server* s, bfs_graph*, int32_t*) { return s ? BFS_E_INTERNAL : BFS_E_INVALID_ARG; }
int bfs_server_submit(bfs_server* s, int32_t, int32_t, uint64_t*) { return s ? BFS_E_INTERNAL : BFS_E_INVALID_ARG; }
int bfs_server_poll(bfs_server* s, uint64_t, int32_t*, int32_t*, bfs_request_stats*) { return s ? BFS_E_INTERNAL : BFS_E_INVALID_ARG; }
int bfs_server_destroy(bfs_server* s) { return s ? BFS_E_INTERNAL : BFS_OK; }
}
