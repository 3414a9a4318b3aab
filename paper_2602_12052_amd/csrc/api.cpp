// Status strings, per-thread error detail and shared argument validation.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "tred_internal.hpp"

static thread_local char g_err[512] = "";

tred_status tred_fail(tred_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

tred_status tred_check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return tred_fail(TRED_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return TRED_OK;
}

extern "C" const char* tred_status_string(int s) {
    switch (s) {
        case TRED_OK: return "ok";
        case TRED_EINVAL: return "invalid argument";
        case TRED_ECAPACITY: return "capacity too small";
        case TRED_EDEVICE: return "device error";
        case TRED_EUNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

extern "C" const char* tred_last_error(void) { return g_err; }

extern "C" int tred_abi_version(void) { return TRED_ABI_VERSION; }

#ifndef TRED_BUILD_ID
#define TRED_BUILD_ID "unversioned"
#endif

extern "C" const char* tred_build_id(void) { return TRED_BUILD_ID; }
