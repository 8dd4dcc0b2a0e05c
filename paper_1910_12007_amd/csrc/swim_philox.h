// swim_philox.h -- Philox4x32-10 counter-based generator (Salmon, Moraes,
// Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) and
// the uniform variates the ABC steps draw from it.  Host and device.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swim {

struct U4 {
    uint32_t v[4];
};

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.v[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.v[2];
        U4 n;
        n.v[0] = (uint32_t)(p1 >> 32) ^ c.v[1] ^ k0;
        n.v[1] = (uint32_t)p1;
        n.v[2] = (uint32_t)(p0 >> 32) ^ c.v[3] ^ k1;
        n.v[3] = (uint32_t)p0;
        c = n;
    }
    return c;
}

// two U(0,1) doubles for (seed, stream, index, draw), 53 bits each, never 0 or 1:
// counter = (index lo, index hi, draw, stream), key = (seed lo, seed hi)
__host__ __device__ inline void philox_uniforms2(uint64_t seed, uint32_t stream, uint64_t index, uint32_t draw,
                                                 double* u)
{
    U4 c;
    c.v[0] = (uint32_t)index;
    c.v[1] = (uint32_t)(index >> 32);
    c.v[2] = draw;
    c.v[3] = stream;
    const U4 w = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double sc = 1.0 / 9007199254740992.0;
    const uint64_t a = ((uint64_t)w.v[0] << 21) + (w.v[1] >> 11);
    const uint64_t b = ((uint64_t)w.v[2] << 21) + (w.v[3] >> 11);
    u[0] = ((double)a + 0.5) * sc;
    u[1] = ((double)b + 0.5) * sc;
}

}  // namespace swim
