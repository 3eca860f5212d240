// Error reporting and version of the meshrf C ABI.
#include <string>

#include "mr_common.h"

namespace mr {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
mr_status fail(mr_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}
}  // namespace mr

extern "C" const char* mr_last_error(void) { return mr::g_last_error.c_str(); }
extern "C" const char* mr_version(void) { return "meshrf 0.1 gfx950"; }
