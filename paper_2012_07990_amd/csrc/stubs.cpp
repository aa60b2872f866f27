// Entry points not built yet report themselves as unsupported.
#include "algos.hpp"

namespace gg {
[[noreturn]] static void todo(const char *what) { throw Error(GG_ERR_UNSUPPORTED_SCHEDULE, std::string(what) + " is not available"); }
}  // namespace gg
