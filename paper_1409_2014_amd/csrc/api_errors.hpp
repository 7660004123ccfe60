// Error reporting shared by the C-ABI sources: the message phi_last_error(NULL)
// returns for the calling thread.
#pragma once

#include <string>

#include "phi_solve.h"

namespace phi {

// Records msg as this thread's last error and returns st.
phi_status thread_error(phi_status st, const std::string& msg);

}  // namespace phi
