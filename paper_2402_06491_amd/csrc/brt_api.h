// The C entry points' guard: the host code builds tables in standard containers, and a failed host
// allocation (std::bad_alloc) or any other C++ exception must come back as a status code instead of
// crossing the C ABI.
#pragma once

#include <exception>
#include <new>

#include "brt_internal.h"

namespace brt {

template <typename F>
int api_guard(const char* name, F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return set_error(BRT_E_NOMEM, "%s: host allocation failed", name);
  } catch (const std::exception& e) {
    return set_error(BRT_E_ARG, "%s: %s", name, e.what());
  } catch (...) {
    return set_error(BRT_E_ARG, "%s: internal error", name);
  }
}

}  // namespace brt
