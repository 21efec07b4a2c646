// Checks the exception-to-status mapping of the C ABI's guard: built and run
// by tests/test_abi_guard.py with the host compiler.
#include <cstdio>
#include <new>
#include <stdexcept>
#include <vector>

#include "abi_guard.hpp"

using mdlts::abi_guard;

int main()
{
    int bad = 0;
    if (abi_guard([]() -> mdlts_status { return MDLTS_EUNSTABLE; }) != MDLTS_EUNSTABLE) bad |= 1;
    if (abi_guard([]() -> mdlts_status { throw std::bad_alloc(); }) != MDLTS_ENOMEM) bad |= 2;
    if (abi_guard([]() -> mdlts_status {
            std::vector<double> v;
            v.reserve(v.max_size());  // length_error or bad_alloc, never returns
            return MDLTS_OK;
        }) == MDLTS_OK)
        bad |= 4;
    if (abi_guard([]() -> mdlts_status { throw std::runtime_error("x"); }) != MDLTS_EDEVICE) bad |= 8;
    if (abi_guard([]() -> mdlts_status { throw 7; }) != MDLTS_EDEVICE) bad |= 16;
    std::printf("abi_guard %s (%d)\n", bad ? "FAILED" : "ok", bad);
    return bad;
}
