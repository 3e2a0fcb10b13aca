// Device-side helpers shared by the kernels: subspace table view and hash probe.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsd {

// Read-only view of a subspace's device tables, passed by value to kernels.
struct SubView {
    const uint64_t *__restrict__ keys;    // [Wp][N]
    const uint64_t *__restrict__ hkey;    // [N]
    const uint64_t *__restrict__ slots;   // [C]
    const uint32_t *__restrict__ bitmap;  // [C/32]
    int64_t N;
    uint32_t cmask;  // C - 1
};

// Hash probe: index of the string `col` (Wp words, known to hash to `h`) or -1.
// Linear probing; the occupancy bit of each slot is tested before the slot is read, so a
// probe that starts on an empty slot touches only the bitmap.  The table always has empty
// slots (load <= 1/2), so the loop ends.
template <int Wp>
__device__ __forceinline__ int64_t probe(const SubView &s, uint64_t h, const uint64_t (&col)[Wp]) {
    uint32_t pos = (uint32_t)h & s.cmask;
    const uint32_t tag = (uint32_t)(h >> 32);
    while (true) {
        const uint32_t word = s.bitmap[pos >> 5];
        if (!((word >> (pos & 31)) & 1u)) return -1;
        const uint64_t slot = s.slots[pos];
        if ((uint32_t)(slot >> 32) == tag) {
            const uint32_t r = (uint32_t)slot;
            bool eq = true;
#pragma unroll
            for (int w = 0; w < Wp; ++w) eq &= (s.keys[(int64_t)w * s.N + r] == col[w]);
            if (eq) return (int64_t)r;
        }
        pos = (pos + 1) & s.cmask;
    }
}

// Continues a probe at slot `pos` (known occupied or not) for a string with tag `tag`.
template <int Wp>
__device__ __forceinline__ int64_t probe_from(const SubView &s, uint32_t pos, uint32_t tag, const uint64_t (&col)[Wp]) {
    while (true) {
        const uint32_t word = s.bitmap[pos >> 5];
        if (!((word >> (pos & 31)) & 1u)) return -1;
        const uint64_t slot = s.slots[pos];
        if ((uint32_t)(slot >> 32) == tag) {
            const uint32_t r = (uint32_t)slot;
            bool eq = true;
#pragma unroll
            for (int w = 0; w < Wp; ++w) eq &= (s.keys[(int64_t)w * s.N + r] == col[w]);
            if (eq) return (int64_t)r;
        }
        pos = (pos + 1) & s.cmask;
    }
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

}  // namespace qsd
