// CPU stand-in for the library internals that the request loop (csrc/serve.hip) uses, so that the
// loop can be compiled with g++ and run under AddressSanitizer and ThreadSanitizer without a GPU.
// The device calls become no-ops; build, solve and destroy come from stub_lib.cpp.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "wfq.h"

typedef int hipError_t;
constexpr hipError_t hipSuccess = 0;
inline hipError_t hipGetDeviceCount(int* c) {
    *c = 1;
    return hipSuccess;
}
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipMemGetInfo(size_t* free_b, size_t* total_b) {
    *free_b = size_t(1) << 34;
    *total_b = size_t(1) << 34;
    return hipSuccess;
}

namespace wfq {
constexpr int kPad = 256;
inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
struct Structure {
    int64_t n = 0;
    int64_t npad = 0;
};
uint64_t batch_bytes(const Structure& S, const wfq_solve_opts& o, int B, int n_dir);
void set_error(int code, const std::string& msg);
}  // namespace wfq
