// qt_philox.h -- the counter-based random numbers of the trajectories,
// usable from device and host code of the library.
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): key (seed, 0), counter (event + 1, trajectory
// id, 0, 0).  Event 0 is the start of a trajectory (word 2: its first
// threshold); event e >= 1 is its e-th jump (word 0: u_l, word 1: u_c,
// word 2: the next threshold).  A word w maps to ((w >> 12) + 0.5) 2^-52,
// strictly inside (0, 1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qt {

struct U4 { uint64_t w[4]; };

__host__ __device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b)
{
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

__host__ __device__ __forceinline__ U4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t lo0 = M0 * c0, hi0 = mulhi64(M0, c0);
        const uint64_t lo1 = M1 * c2, hi1 = mulhi64(M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    U4 o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

__host__ __device__ __forceinline__ double uniform01(uint64_t w)
{
    return ((double)(w >> 12) + 0.5) * (1.0 / 4503599627370496.0);
}

// Random block of event e (0 = start, e >= 1 = e-th jump) of a trajectory.
__host__ __device__ __forceinline__ U4 event_block(uint64_t seed, uint64_t traj_id, int64_t e)
{
    return philox4x64_10((uint64_t)e + 1u, traj_id, 0u, 0u, seed, 0u);
}

}  // namespace qt
