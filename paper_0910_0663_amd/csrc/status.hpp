// The calling thread's last error message (vtm_last_error) and the status that
// goes with it.
#pragma once

#include <string>

#include "vtm.h"

namespace vtm {

// Records msg as the calling thread's last error and returns s.
vtm_status fail(vtm_status s, const std::string& msg);

}  // namespace vtm
