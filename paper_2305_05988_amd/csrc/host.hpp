// Host-side helpers shared by the library's C ABI sources.
#pragma once

#include <string>

#include "../../include/itsolve.h"

// Records msg as the thread's last error (its_last_error) and returns st.
its_status its_fail(its_status st, const std::string &msg);
