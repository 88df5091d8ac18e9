// Entry points of api.cpp that other translation units of the library call.
#pragma once

#include <cstddef>
#include <string>

#include "../../include/h2dlp.h"

namespace h2dlp {

// Record `msg` for h2dlp_last_error() and return `code`.
int set_error(int code, const std::string& msg);

// `p` is device memory of GPU `dev` with at least `bytes` from it (else *why
// says what is wrong).
bool device_memory_ok(const void* p, size_t bytes, int dev, const char* name, std::string* why);

// *dev: a HIP ordinal or -1 (the current device), checked to be a gfx950;
// H2DLP_OK or an error code with its message recorded.
int gfx950_device(int* dev);

// Device ordinal of a built handle; -1 for NULL or a handle from h2dlp_plan.
int handle_device(h2dlp_handle h);

// h2dlp_apply_ex.  workspace_is_library: the workspace is the library's own
// device array, so it is not looked up among the caller's allocations.
int apply_entry(h2dlp_handle h, const void* u1, void* u2, int nrhs, int io_dtype, void* stream, void* workspace,
                size_t workspace_bytes, bool workspace_is_library);

}  // namespace h2dlp
