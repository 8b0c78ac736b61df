// Error text shared by the library's source files (vx_last_error).
#pragma once

namespace vxs {

// Sets the calling thread's vx_last_error() message.
void set_error(const char *msg);

}  // namespace vxs
