// Internal error handling and small utilities shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "bcv.h"

namespace bcv {

struct Error : std::runtime_error {
    bcv_status code;
    Error(bcv_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(bcv_status c, const std::string &m) { throw Error(c, m); }

#define BCV_HIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            ::bcv::fail(BCV_EDEVICE, std::string(#call) + " failed: " + hipGetErrorString(e_));    \
    } while (0)

#define BCV_REQUIRE(cond, code, msg)                                                               \
    do {                                                                                           \
        if (!(cond)) ::bcv::fail(code, msg);                                                       \
    } while (0)

// Interleave the low `bits` bits of i, j, k: bit b of i -> 3b, of j -> 3b+1, of k -> 3b+2.
inline uint64_t morton3(uint32_t i, uint32_t j, uint32_t k, int bits)
{
    uint64_t key = 0;
    for (int b = 0; b < bits; ++b) {
        key |= uint64_t((i >> b) & 1u) << (3 * b);
        key |= uint64_t((j >> b) & 1u) << (3 * b + 1);
        key |= uint64_t((k >> b) & 1u) << (3 * b + 2);
    }
    return key;
}

}  // namespace bcv
