// Host-side guard of the C-ABI entry points of libuhnsw.
#pragma once
#include <exception>
#include <string>

#include "uhnsw.h"

namespace uhnsw {
// The body of an extern "C" entry point: a C++ exception raised inside it (a
// host container, string or thread that could not be created) ends the call
// with UHNSW_ENOMEM, its message handed to on_error, instead of crossing the
// C boundary.
template <typename Body, typename OnError>
int no_throw(const char *fn, Body &&body, OnError &&on_error) noexcept {
    const char *what = "unknown C++ exception";
    try {
        return body();
    } catch (const std::exception &e) {
        what = e.what();
    } catch (...) {
    }
    try {
        on_error((std::string(fn) + ": host resources exhausted (" + what + ")").c_str());
    } catch (...) {
    }
    return UHNSW_ENOMEM;
}

}  // namespace uhnsw
