// Row engine of the subspace Hamiltonian (Methods, Matrix evaluation), shared by the SpMV,
// the CSR passes and the work counter.
//
// Mapping.  One lane owns one row bit-string b_i (rows are consecutive in the canonical order).
// The off-diagonal groups are processed in chunks of kChunk:
//
//   scan   all 64 lanes walk the chunk's groups in lockstep (group descriptors are wave-uniform
//          scalar loads).  Each lane forms its ladder integer L from the row bits at the
//          group's ladder qubits and keeps the group iff some term has that ladder integer
//          (Methods, Fermionic Hamiltonians: an empty int_ptrs range needs no lookup).  The
//          surviving groups are recorded as one bit per group in a per-lane mask.
//   probe  each lane then pops its own set bits, lowest group first, kProbeBatch at a time, so
//          every probe instruction runs with (nearly) all lanes busy instead of with only the
//          lanes whose group happens to be live.  A probe forms hash(b_i ^ M_g) =
//          hash(b_i) ^ hash(M_g) (the hash is linear over GF(2)), tests the occupancy bit,
//          reads the {tag, index} slot and compares the key (Methods, Subspace data
//          structure).
//   hit    the terms of the group's ladder range are refined on their projector bits and
//          summed with popcount-parity signs; the caller's functor consumes (j, value).
//
// Each lane consumes its hits in increasing group order, so a row's sum is formed in a fixed
// order: results are bitwise reproducible and independent of how rows are batched.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"
#include "device.h"

namespace qsd {

constexpr int kChunk = 128;               // groups per chunk
constexpr int kMaskWords = kChunk / 32;   // per-lane live bits per chunk
constexpr int kProbeBatch = 2;            // probes in flight per lane

struct HamView {
    const uint64_t *__restrict__ g_mask;   // [G][Wp]
    const uint64_t *__restrict__ g_hash;   // [G]
    const uint64_t *__restrict__ g_pos;    // [G] four 16-bit ladder qubits
    const uint32_t *__restrict__ g_info;   // [G] k | ladder | care | live16 << 16
    const uint32_t *__restrict__ g_term0;  // [G]
    const uint32_t *__restrict__ g_nterm;  // [G]
    const uint16_t *__restrict__ g_iptr;   // [G][kIptr]
    const uint64_t *__restrict__ t_cws;    // [T][3][Wp] care, want, sign masks
    const void *__restrict__ t_coef;       // [T] double2 or float2
    int64_t G;
};

template <class ET>
struct C2;
template <>
struct C2<double> {
    using T = double2;
};
template <>
struct C2<float> {
    using T = float2;
};

template <int Wp>
__device__ __forceinline__ uint32_t row_bit(const uint64_t (&k)[Wp], uint32_t p) {
    uint64_t w = k[0];
#pragma unroll
    for (int i = 1; i < Wp; ++i)
        if ((p >> 6) == (uint32_t)i) w = k[i];
    const uint32_t half = (p & 32u) ? (uint32_t)(w >> 32) : (uint32_t)w;
    return (half >> (p & 31u)) & 1u;
}

template <int Wp>
__device__ __forceinline__ bool term_pass(const uint64_t (&k)[Wp], const uint64_t *__restrict__ cws) {
    bool ok = true;
#pragma unroll
    for (int w = 0; w < Wp; ++w) ok &= (k[w] & cws[w]) == cws[Wp + w];
    return ok;
}

template <int Wp>
__device__ __forceinline__ uint32_t term_parity(const uint64_t (&k)[Wp], const uint64_t *__restrict__ cws) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < Wp; ++w) c += (uint32_t)__popcll(k[w] & cws[2 * Wp + w]);
    return c & 1u;
}

template <int Wp>
__device__ __forceinline__ uint32_t ladder_int(const uint64_t (&k)[Wp], uint64_t pos, uint32_t kk) {
    uint32_t L = 0;
    for (uint32_t j = 0; j < kk; ++j) L |= row_bit<Wp>(k, (uint32_t)(pos >> (16 * j)) & 0xFFFFu) << j;
    return L;
}

// Term range of group g for a row: the ladder-integer range, or all terms.
template <int Wp>
__device__ __forceinline__ void term_range(const HamView &h, const uint64_t (&key)[Wp], int64_t g, uint32_t &lo,
                                           uint32_t &hi) {
    const uint32_t info = h.g_info[g];
    if (info & kInfoLadder) {
        const uint32_t L = ladder_int<Wp>(key, h.g_pos[g], info & kInfoKMask);
        lo = h.g_iptr[g * kIptr + L];
        hi = h.g_iptr[g * kIptr + L + 1];
    } else {
        lo = 0;
        hi = h.g_nterm[g];
    }
}

// Element value of group g for a row: sum over the range of c'_t (-1)^popcount(b & S_t) over the
// terms whose projector bits match.  Returns false when no term matches (no stored entry).
template <int Wp, class ET>
__device__ __forceinline__ bool group_value(const HamView &h, const uint64_t (&key)[Wp], int64_t g, ET &vre, ET &vim) {
    using CT = typename C2<ET>::T;
    const CT *__restrict__ coef = (const CT *)h.t_coef;
    uint32_t lo, hi;
    term_range<Wp>(h, key, g, lo, hi);
    const uint32_t t0 = h.g_term0[g];
    bool any = false;
    vre = 0;
    vim = 0;
    for (uint32_t t = lo; t < hi; ++t) {
        const uint64_t *cws = h.t_cws + (int64_t)(t0 + t) * 3 * Wp;
        if (!term_pass<Wp>(key, cws)) continue;
        any = true;
        const CT c = coef[t0 + t];
        if (term_parity<Wp>(key, cws)) {
            vre -= c.x;
            vim -= c.y;
        } else {
            vre += c.x;
            vim += c.y;
        }
    }
    return any;
}

// True iff some term of group g's range matches the row's projector bits.
template <int Wp>
__device__ __forceinline__ bool group_any(const HamView &h, const uint64_t (&key)[Wp], int64_t g) {
    uint32_t lo, hi;
    term_range<Wp>(h, key, g, lo, hi);
    if (!(h.g_info[g] & kInfoCare)) return lo < hi;
    const uint32_t t0 = h.g_term0[g];
    for (uint32_t t = lo; t < hi; ++t)
        if (term_pass<Wp>(key, h.t_cws + (int64_t)(t0 + t) * 3 * Wp)) return true;
    return false;
}

// LDS staging of one chunk: the group hashes and masks read by the probes.
template <int Wp>
struct ChunkLds {
    uint64_t hash[kChunk];
    uint64_t mask[kChunk][Wp];
    uint32_t live[kMaskWords][kBlock];  // per-lane live bits of the chunk
};

// Pops the lowest set bit of the lane's chunk mask (current word `cur`, index `qi`, later
// words in LDS); returns the chunk-relative group or -1.
__device__ __forceinline__ int pop_group(uint32_t &cur, int &qi, const uint32_t (*live)[kBlock]) {
    while (cur == 0 && qi + 1 < kMaskWords) {
        ++qi;
        cur = live[qi][threadIdx.x];
    }
    if (cur == 0) return -1;
    const int c = qi * 32 + __builtin_ctz(cur);
    cur &= cur - 1;
    return c;
}

// Walks all groups for the lane's row and calls on_hit(j, g) for every probe whose column
// b_i ^ M_g is in the subspace (j = its index), in increasing g.  All threads of the block
// must call it (it stages chunks through LDS with barriers).  `valid` = the lane owns a row.
template <int Wp, class OnHit>
__device__ __forceinline__ void row_engine(const SubView &s, const HamView &h, const uint64_t (&key)[Wp],
                                           uint64_t hrow, bool valid, ChunkLds<Wp> &lds, OnHit &&on_hit,
                                           unsigned long long *probes = nullptr) {
    for (int64_t g0 = 0; g0 < h.G; g0 += kChunk) {
        const int nc = (int)((h.G - g0) < kChunk ? (h.G - g0) : kChunk);
        __syncthreads();
        for (int c = threadIdx.x; c < nc; c += kBlock) {
            lds.hash[c] = h.g_hash[g0 + c];
#pragma unroll
            for (int w = 0; w < Wp; ++w) lds.mask[c][w] = h.g_mask[(g0 + c) * Wp + w];
        }
        // scan: one live bit per group
        uint32_t m0 = 0;
#pragma unroll
        for (int q = 0; q < kMaskWords; ++q) {
            uint32_t m = 0;
            const int cend = nc - 32 * q < 32 ? nc - 32 * q : 32;
            for (int b = 0; b < cend; ++b) {
                const int64_t g = g0 + 32 * q + b;
                const uint32_t info = h.g_info[g];
                uint32_t live = 1u;
                if (info & kInfoLadder) live = (info >> (16 + ladder_int<Wp>(key, h.g_pos[g], info & kInfoKMask))) & 1u;
                m |= live << b;
            }
            if (!valid) m = 0;
            if (q == 0)
                m0 = m;
            else
                lds.live[q][threadIdx.x] = m;
        }
        __syncthreads();
        if (probes) {
            unsigned long long cnt = __popc(m0);
            for (int q = 1; q < kMaskWords; ++q) cnt += __popc(lds.live[q][threadIdx.x]);
            *probes += cnt;
        }
        // probe: each lane pops its own live groups, kProbeBatch at a time
        uint32_t cur = m0;
        int qi = 0;
        while (true) {
            int c[kProbeBatch];
            bool anyc = false;
#pragma unroll
            for (int b = 0; b < kProbeBatch; ++b) {
                c[b] = pop_group(cur, qi, lds.live);
                anyc |= c[b] >= 0;
            }
            if (!__any(anyc)) break;
            uint64_t hh[kProbeBatch];
            uint32_t pos[kProbeBatch], word[kProbeBatch];
#pragma unroll
            for (int b = 0; b < kProbeBatch; ++b) {
                hh[b] = c[b] >= 0 ? (hrow ^ lds.hash[c[b]]) : 0ull;
                pos[b] = (uint32_t)hh[b] & s.cmask;
                word[b] = c[b] >= 0 ? s.bitmap[pos[b] >> 5] : 0u;
            }
            uint64_t slot[kProbeBatch];
            bool occ[kProbeBatch];
#pragma unroll
            for (int b = 0; b < kProbeBatch; ++b) {
                occ[b] = (word[b] >> (pos[b] & 31u)) & 1u;
                slot[b] = occ[b] ? s.slots[pos[b]] : ~0ull;
            }
#pragma unroll
            for (int b = 0; b < kProbeBatch; ++b) {
                if (!occ[b]) continue;
                const uint32_t tag = (uint32_t)(hh[b] >> 32);
                uint64_t col[Wp];
#pragma unroll
                for (int w = 0; w < Wp; ++w) col[w] = key[w] ^ lds.mask[c[b]][w];
                int64_t j = -1;
                if ((uint32_t)(slot[b] >> 32) == tag) {
                    const uint32_t r = (uint32_t)slot[b];
                    bool eq = true;
#pragma unroll
                    for (int w = 0; w < Wp; ++w) eq &= s.keys[(int64_t)w * s.N + r] == col[w];
                    if (eq) j = r;
                }
                if (j < 0) {
                    // first slot held another key: follow the run while slots stay occupied
                    const uint32_t nxt = (pos[b] + 1) & s.cmask;
                    const uint32_t nw = ((nxt >> 5) == (pos[b] >> 5)) ? word[b] : s.bitmap[nxt >> 5];
                    if ((nw >> (nxt & 31u)) & 1u) j = probe_from<Wp>(s, nxt, tag, col);
                }
                if (j >= 0) on_hit(j, g0 + c[b]);
            }
        }
    }
}

}  // namespace qsd
