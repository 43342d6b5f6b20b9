// Thread-local error message shared by every entry point of the C ABI.
#pragma once

int vecchia_set_error(int code, const char* fmt, ...)
#if defined(__GNUC__)
    __attribute__((format(printf, 2, 3)))
#endif
    ;
void vecchia_clear_error();
