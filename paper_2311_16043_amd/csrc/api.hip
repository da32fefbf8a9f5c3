// api.hip -- error reporting and version of the visibility library.
#include "rv_internal.h"

namespace rv {

namespace {
thread_local std::string g_last_error;
}

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

rv_status check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: HIP error %d (%s)", what, (int)e, hipGetErrorString(e));
        return RV_ERR_HIP;
    }
    return RV_OK;
}

}  // namespace rv

extern "C" const char *rv_last_error(void) { return rv::g_last_error.c_str(); }

extern "C" const char *rv_version(void) { return "rvis 0.1 (gfx950)"; }
