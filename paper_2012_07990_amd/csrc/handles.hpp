// Opaque C handle types and the shared last-error slot of the C ABI.
#pragma once

#include <string>

#include "ops.hpp"

struct gg_graph {
    gg::Graph g;
};

namespace gg {
extern thread_local std::string g_last_error;  // message behind gg_last_error()
}
