// Measurement kernels that are not part of the method: a streaming probe with
// the access mix of one red-black half-sweep, to tell how close the sweep comes
// to what a plain streaming kernel with the same reads and writes achieves.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace hosc {

// The half-sweep moves 23 elements per updated node: 19 reads (seven row
// arrays, four right-hand sides, four own increments, four increments of the
// other colour) and 4 writes (the own increments, in place).  The probe has the
// same streams: 15 read-only arrays and 4 arrays read and rewritten in place,
// n 16-byte elements each, laid out one after another; thread t touches element
// t of every array, so the grid covers n threads and nothing else.
constexpr int kMixRead = 15, kMixInPlace = 4;

__global__ void __launch_bounds__(256) k_stream_mix(const double2 *__restrict__ rd, double2 *__restrict__ upd,
                                                    size_t n)
{
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n) return;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int q = 0; q < kMixRead; ++q) {
        const double2 v = rd[(size_t)q * n + t];
        sx += v.x;
        sy += v.y;
    }
#pragma unroll
    for (int q = 0; q < kMixInPlace; ++q) {
        double2 v = upd[(size_t)q * n + t];
        v.x = 0.5 * v.x + sx;
        v.y = 0.5 * v.y + sy;
        upd[(size_t)q * n + t] = v;
    }
}

}  // namespace hosc
