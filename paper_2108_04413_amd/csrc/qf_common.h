// Internal helpers shared by the host builder and the device entry points:
// thread-local error text and status plumbing.  Not part of the public ABI.
#pragma once

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <exception>
#include <new>
#include <string>

#include "../../include/qforte_mi355x.h"

namespace qf {

std::string &last_error();

inline int fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    last_error() = buf;
    return status;
}

struct Error {
    int status;
    std::string msg;
};

[[noreturn]] inline void raise(int status, const std::string &msg) { throw Error{status, msg}; }

// Run f() and convert any exception into a status code.
template <class F> int guarded(F &&f)
{
    try {
        return f();
    } catch (const Error &e) {
        last_error() = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        return fail(QF_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(QF_E_ARG, "%s", e.what());
    } catch (...) {
        return fail(QF_E_ARG, "unknown error");
    }
}

inline int popc64(uint64_t v) { return __builtin_popcountll(v); }

} // namespace qf
