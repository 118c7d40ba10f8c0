// philox.hpp -- Philox4x32-10 counter-based generator (J. K. Salmon, M. A.
// Moraes, R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2,
// 3", SC'11), written from its published definition, plus the uniform and
// Box-Muller helpers used by the initial conditions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gl {

struct U4 {
    uint32_t v[4];
};

__host__ __device__ inline U4 philox4x32_10(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                            uint32_t c2, uint32_t c3) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        uint64_t a = (uint64_t)0xD2511F53u * c0;   // multiplies word 0
        uint64_t b = (uint64_t)0xCD9E8D57u * c2;   // multiplies word 2
        uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)b;
        uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)a;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;   // Weyl key schedule
        k1 += 0xBB67AE85u;
    }
    U4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// draw for counter (c0, c1, stream, 0) under a 64-bit seed
__host__ __device__ inline U4 draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t stream) {
    return philox4x32_10((uint32_t)seed, (uint32_t)(seed >> 32), c0, c1, stream, 0u);
}

// (2k+1) 2^-53 with k the top 52 bits of hi:lo -- exact, strictly inside (0, 1)
__host__ __device__ inline double uniform53(uint32_t lo, uint32_t hi) {
    uint64_t w = ((uint64_t)hi << 32) | lo;
    uint64_t k = ((w >> 12) << 1) | 1u;
    return (double)k * 1.1102230246251565404236316680908203125e-16;   // 2^-53
}

__device__ inline void box_muller(const U4 &w, double &g0, double &g1) {
    double r = sqrt(-2.0 * log(uniform53(w.v[0], w.v[1])));
    double s, c;
    sincos(6.283185307179586476925286766559 * uniform53(w.v[2], w.v[3]), &s, &c);
    g0 = r * c;
    g1 = r * s;
}

}  // namespace gl
