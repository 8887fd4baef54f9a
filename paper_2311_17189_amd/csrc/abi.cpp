// Error reporting and version of the C ABI (include/amigpu.h).
#include <string>

#include "ami_internal.hpp"

namespace ami {

namespace {
thread_local std::string g_last_error;
}

AmiStatus fail(AmiStatus st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

void clear_error() { g_last_error.clear(); }

}  // namespace ami

extern "C" const char *amiLastError(void) { return ami::g_last_error.c_str(); }

extern "C" const char *amiVersion(void) { return "amigpu 0.1 (gfx950)"; }
