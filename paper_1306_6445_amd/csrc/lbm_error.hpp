// Thread-local message of the most recent failure, shared by every C entry
// point of the library and read back through lbm_last_error().
#pragma once

#include <string>

namespace lbm {
void set_last_error(const std::string &msg);
}
