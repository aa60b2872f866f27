// Entry points not built yet report themselves as unsupported.
#include "algos.hpp"

namespace gg {
[[noreturn]] static void todo(const char *what) { throw Error(GG_ERR_UNSUPPORTED_SCHEDULE, std::string(what) + " is not available"); }
void msbfs_run(Graph &, const int32_t *, int, const gg_schedule &, int32_t *, hipStream_t, gg_stats *) { todo("multi-source BFS"); }
void msbc_run(Graph &, const int32_t *, int, const gg_schedule &, uint64_t *, float *, hipStream_t, gg_stats *) { todo("multi-source BC"); }
}  // namespace gg
