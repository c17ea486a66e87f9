// Error text behind dpso_last_error (thread-local) and the status helpers
// every entry point returns through.
#pragma once

#include "dpso.h"

namespace dpso {

// Records a printf-style message for dpso_last_error and returns `code`.
dpso_status fail(dpso_status code, const char *fmt, ...);
// Clears the message and returns DPSO_OK.
dpso_status ok();
// The message of this thread's last failed call ("" after a success).
const char *last_error();

}  // namespace dpso
