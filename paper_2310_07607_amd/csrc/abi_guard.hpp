// abi_guard.hpp -- no C++ exception crosses the C ABI.  Every entry point of
// include/mdlts.h runs its body through abi_guard: a failed host allocation
// (std::bad_alloc, e.g. of a forest or table vector) becomes MDLTS_ENOMEM,
// any other exception MDLTS_EDEVICE, so that a caller in C (or through a
// foreign-function binding) always receives a status instead of a
// terminated process.
#pragma once
#include <new>

#include "mdlts.h"

namespace mdlts {

template <typename F>
inline mdlts_status abi_guard(F &&body) noexcept
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return MDLTS_ENOMEM;
    } catch (...) {
        return MDLTS_EDEVICE;
    }
}

}  // namespace mdlts
