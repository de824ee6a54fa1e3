// fv_host.h -- host-side error reporting shared by the library's sources.
#pragma once

#include <string>

namespace fvh {
// Records `msg` as the thread's last error (fv_last_error) and returns `code`.
int fail(int code, const std::string& msg);
// FV_OK, or FV_E_HIP with the runtime's message if the last launch failed.
int launched(const char* what);
extern thread_local std::string g_last_error;
}  // namespace fvh
