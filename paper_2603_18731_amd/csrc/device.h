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
    uint32_t exact;  // slots carry the displacement: a tag match at the right displacement is the key
    const uint32_t *__restrict__ order;  // [N] row indices in the order of their slots in the table
    const uint64_t *__restrict__ okeys;  // [Wp][N] keys in that order
    const uint64_t *__restrict__ ohkey;  // [N] hashes in that order
    // part filters (NULL when the subspace has none): bit u of pfilt[0 .. 2047] is set when some
    // string's low-part index is u, bit u of pfilt[2048 .. 4095] when some string's high-part
    // index is u; pkey / opkey hold each row's packed part indices (high << 16 | low) in the
    // canonical and the slot order.  The indices are GF(2)-linear in the string, so a column's
    // are the row's XOR the group's.
    const uint32_t *__restrict__ pfilt;
    const uint32_t *__restrict__ pkey;
    const uint32_t *__restrict__ opkey;
    // product map (NULL when the subspace is not the Cartesian product of its two parts, or a
    // part has more than 16 qubits): prank[w] = set bits of pfilt's words before word w of the
    // same filter, and pna = the number of low parts.  Then the string (low l, high h) has
    // canonical index rank_high(h) * pna + rank_low(l).
    const uint16_t *__restrict__ prank;
    uint32_t pna;
};

constexpr int kPartBits = 16;                        // index bits of each part filter
constexpr int kPartWords = 2 << (kPartBits - 5);     // both filters, in 32-bit words (16 KB)

// Whether both parts of a string with packed part indices p occur in the subspace (a necessary
// condition for the string to be a member).
__device__ __forceinline__ bool part_pass(const uint32_t *pf, uint32_t p) {
    const uint32_t lo = p & 0xFFFFu, hi = p >> 16;
    return ((pf[lo >> 5] >> (lo & 31u)) & (pf[(kPartWords / 2) + (hi >> 5)] >> (hi & 31u)) & 1u) != 0u;
}

// Product map: the canonical index of the string with packed part indices p, or -1 when either
// part is absent.  Strings ascend by high part, then by low part, so when the subspace is the
// product of its low parts (pna of them) and high parts, the string (l, h) sits at
// rank(h) * pna + rank(l), each rank read off a filter as the set bits below the part's own.
// pf / pr are the filters and their word prefix counts (LDS or global copies).
// Rank of a part among the parts that occur (the set bits of its filter below its own bit);
// `half` 0 = low parts, 1 = high parts.
__device__ __forceinline__ uint32_t part_rank(const uint32_t *pf, const uint16_t *pr, int half, uint32_t q) {
    const uint32_t w = (uint32_t)half * (kPartWords / 2) + (q >> 5);
    return (uint32_t)pr[w] + (uint32_t)__popc(pf[w] & ((1u << (q & 31u)) - 1u));
}

__device__ __forceinline__ uint32_t product_rank(const uint32_t *pf, const uint16_t *pr, uint32_t pna, uint32_t p) {
    // the index of a string known to be present (both parts occur)
    return part_rank(pf, pr, 1, p >> 16) * pna + part_rank(pf, pr, 0, p & 0xFFFFu);
}

__device__ __forceinline__ int64_t product_index(const uint32_t *pf, const uint16_t *pr, uint32_t pna, uint32_t p) {
    const uint32_t lo = p & 0xFFFFu, hi = p >> 16;
    const uint32_t wl = pf[lo >> 5], wh = pf[(kPartWords / 2) + (hi >> 5)];
    const uint32_t bl = lo & 31u, bh = hi & 31u;
    // no branch: the prefix counts are read whether or not both parts occur (N < 2^32, so the
    // index fits 32 bits)
    const uint32_t rl = (uint32_t)pr[lo >> 5] + (uint32_t)__popc(wl & ((1u << bl) - 1u));
    const uint32_t rh = (uint32_t)pr[(kPartWords / 2) + (hi >> 5)] + (uint32_t)__popc(wh & ((1u << bh) - 1u));
    const bool ok = ((wl >> bl) & (wh >> bh) & 1u) != 0u;
    return ok ? (int64_t)(rh * pna + rl) : (int64_t)-1;
}

// Slot layout.  Default: tag (high 32 bits of the hash) | index (32 bits).  Exact mode (one-word
// keys, N < 2^26, and the map key -> (home slot, tag) proven injective when the table is built):
// tag | displacement from the home slot (6 bits, 63 = 63 or more) | index (26 bits).  Then a slot
// whose tag and displacement match the probe's holds the probed string itself, and the key
// compare is needed only for displacements of 63 or more.
constexpr int kExactIdxBits = 26;
constexpr uint32_t kExactIdxMask = (1u << kExactIdxBits) - 1u;

__device__ __forceinline__ uint32_t slot_index(const SubView &s, uint64_t slot) {
    return s.exact ? ((uint32_t)slot & kExactIdxMask) : (uint32_t)slot;
}

// Index of `col` if the occupied `slot` (tag already equal) holds it, probed at distance `dist`
// from col's home slot; -1 otherwise.
template <int Wp>
__device__ __forceinline__ int64_t slot_match(const SubView &s, uint64_t slot, uint32_t dist,
                                              const uint64_t (&col)[Wp]) {
    if (s.exact) {
        const uint32_t d = (uint32_t)(slot >> kExactIdxBits) & 63u;
        const uint32_t r = (uint32_t)slot & kExactIdxMask;
        if (d < 63u) return d == dist ? (int64_t)r : -1;
        if (dist < 63u) return -1;
        return s.keys[r] == col[0] ? (int64_t)r : -1;
    }
    const uint32_t r = (uint32_t)slot;
    bool eq = true;
#pragma unroll
    for (int w = 0; w < Wp; ++w) eq &= (s.keys[(int64_t)w * s.N + r] == col[w]);
    return eq ? (int64_t)r : -1;
}

// Hash probe: index of the string `col` (Wp words, known to hash to `h`) or -1.
// Linear probing; the occupancy bit of each slot is tested before the slot is read, so a
// probe that starts on an empty slot touches only the bitmap.  The table always has empty
// slots (load <= 1/2), so the loop ends.
template <int Wp>
__device__ __forceinline__ int64_t probe(const SubView &s, uint64_t h, const uint64_t (&col)[Wp]) {
    uint32_t pos = (uint32_t)h & s.cmask;
    const uint32_t tag = (uint32_t)(h >> 32);
    for (uint32_t dist = 0;; ++dist) {
        const uint32_t word = s.bitmap[pos >> 5];
        if (!((word >> (pos & 31)) & 1u)) return -1;
        const uint64_t slot = s.slots[pos];
        if ((uint32_t)(slot >> 32) == tag) {
            const int64_t r = slot_match<Wp>(s, slot, dist, col);
            if (r >= 0) return r;
        }
        pos = (pos + 1) & s.cmask;
    }
}

// Continues a probe at slot `pos`, `dist` slots after the string's home slot (known occupied or
// not), for a string with tag `tag`.
template <int Wp>
__device__ __forceinline__ int64_t probe_from(const SubView &s, uint32_t pos, uint32_t dist, uint32_t tag,
                                              const uint64_t (&col)[Wp]) {
    for (;; ++dist) {
        const uint32_t word = s.bitmap[pos >> 5];
        if (!((word >> (pos & 31)) & 1u)) return -1;
        const uint64_t slot = s.slots[pos];
        if ((uint32_t)(slot >> 32) == tag) {
            const int64_t r = slot_match<Wp>(s, slot, dist, col);
            if (r >= 0) return r;
        }
        pos = (pos + 1) & s.cmask;
    }
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

}  // namespace qsd
