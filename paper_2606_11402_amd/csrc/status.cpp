// Thread-local last-error string of the C ABI.
#include <cstdarg>
#include <cstdio>
#include <string>

#include "status.h"
#include "vecchia.h"

static thread_local std::string g_last_error;

int vecchia_set_error(int code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void vecchia_clear_error() { g_last_error.clear(); }

extern "C" const char* vecchia_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* vecchia_version(void) { return "vecchia-mi355x 0.1 (gfx950)"; }

extern "C" int32_t vecchia_padded_k(int32_t k) {
    if (k < 1 || k > VECCHIA_KMAX) return -1;
    if (k <= 8) return 8;
    if (k <= 16) return 16;
    if (k <= 32) return 32;
    return 64;
}

extern "C" int vecchia_abi_sizes(size_t* view_bytes, size_t* kernel_bytes) {
    if (view_bytes) *view_bytes = sizeof(vecchia_view);
    if (kernel_bytes) *kernel_bytes = sizeof(vecchia_kernel);
    return VECCHIA_OK;
}
