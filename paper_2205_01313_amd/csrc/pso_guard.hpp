// pso_guard.hpp -- keeps C++ exceptions from crossing the C ABI.
//
// Every entry point of include/pso.h returns a status and never aborts, but
// its body uses the C++ library (containers, threads, maps), which reports
// failure by throwing.  guarded() runs a body and turns whatever it throws
// into a status: std::bad_alloc (and std::length_error, a container size
// beyond what can be allocated) into PSO_ENOMEM, anything else into
// PSO_EDEVICE, each with a message for pso_last_error().
#pragma once

#include <exception>
#include <new>
#include <stdexcept>

#include "pso.h"

int pso_internal_fail(int code, const char *fmt, ...);

namespace pso {

template <class Body>
int guarded(Body &&body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return pso_internal_fail(PSO_ENOMEM, "host memory allocation failed");
    } catch (const std::length_error &e) {
        return pso_internal_fail(PSO_ENOMEM, "host container too large: %s", e.what());
    } catch (const std::exception &e) {
        return pso_internal_fail(PSO_EDEVICE, "internal error: %s", e.what());
    } catch (...) {
        return pso_internal_fail(PSO_EDEVICE, "internal error (unknown exception)");
    }
}

} // namespace pso
