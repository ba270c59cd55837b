// The calling thread's last error message (vtm_last_error) and the status that
// goes with it.
#pragma once

#include <exception>
#include <new>
#include <string>

#include "vtm.h"

namespace vtm {

// Records msg as the calling thread's last error and returns s (never throws:
// with no memory for the message, the message is left empty).
vtm_status fail(vtm_status s, const std::string& msg) noexcept;
vtm_status fail(vtm_status s, const char* msg) noexcept;

// Runs the body of a C ABI call so that no C++ exception leaves it: host memory
// exhaustion becomes VTM_E_OOM, any other exception VTM_E_UNSUPPORTED with its
// message.
template <typename F>
vtm_status guarded(F&& body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return fail(VTM_E_OOM, "host memory exhausted");
    } catch (const std::exception& e) {
        std::string msg;
        try {
            msg = std::string("internal error: ") + e.what();
        } catch (...) {
        }
        return fail(VTM_E_UNSUPPORTED, msg);
    } catch (...) {
        return fail(VTM_E_UNSUPPORTED, "internal error");
    }
}

}  // namespace vtm
