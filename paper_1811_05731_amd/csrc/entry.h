// Entry points of api.cpp that other translation units of the library call.
#pragma once

#include <cstddef>
#include <string>

#include "../../include/h2dlp.h"

namespace h2dlp {

// Record `msg` for h2dlp_last_error() and return `code`.
int set_error(int code, const std::string& msg);

// Device ordinal of a built handle; -1 for NULL or a handle from h2dlp_plan.
int handle_device(h2dlp_handle h);

// h2dlp_apply_ex.  workspace_is_library: the workspace is the library's own
// device array, so it is not looked up among the caller's allocations.
int apply_entry(h2dlp_handle h, const void* u1, void* u2, int nrhs, int io_dtype, void* stream, void* workspace,
                size_t workspace_bytes, bool workspace_is_library);

}  // namespace h2dlp
