// Row engine of the subspace Hamiltonian (Methods, Matrix evaluation), shared by the SpMV,
// the CSR passes and the work counter.
//
// Mapping.  One lane owns one row bit-string b_i (rows are consecutive in the canonical order,
// or in the order of their hash slots; the caller chooses).  The off-diagonal groups are
// processed in chunks of kChunk = 64:
//
//   scan   bit-sliced over the wave's 64 rows.  The rows' keys are transposed once into bit
//          planes (plane q = bit q of all 64 rows, one 64-bit word).  For the chunk, lane l
//          takes group l: its ladder-integer live table (Methods, Fermionic Hamiltonians: an
//          empty int_ptrs range needs no lookup) is evaluated as a boolean function of the four
//          planes of the group's ladder qubits, giving one 64-bit word of live rows.  A 64 x 64
//          bit transpose across the wave then hands every lane the live-group mask of its own
//          row.  This costs a few hundred wave instructions per chunk instead of a ladder
//          integer per (row, group).
//   probe  each lane then pops its own set bits, lowest group first, kProbeBatch at a time, so
//          every probe instruction runs with (nearly) all lanes busy instead of with only the
//          lanes whose group happens to be live.  A probe forms hash(b_i ^ M_g) =
//          hash(b_i) ^ hash(M_g) (the hash is linear over GF(2)), tests the occupancy bit,
//          reads the {tag, index} slot and compares the key (Methods, Subspace data
//          structure).  Two variants change only which probes share an instruction or a
//          batch: `lockstep` (the wave probes one group at a time) and `filter_first` (all
//          occupancy bits of a chunk's live groups first, then the slots of the occupied ones);
//          see row_engine.
//   hit    the row's ladder integer selects the group's term range; the terms are refined on
//          their projector bits and summed with popcount-parity signs; the caller's functor
//          consumes (j, value).
//
// Each lane consumes its hits in increasing group order, so a row's sum is formed in a fixed
// order: results are bitwise reproducible and independent of how rows are batched.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"
#include "device.h"

namespace qsd {

constexpr int kChunk = 64;      // groups per chunk (one 64-bit live mask per lane)
constexpr int kProbeBatch = 2;  // probes in flight per lane
constexpr int kLockBatch = 4;   // groups in flight per wave in lockstep mode
constexpr int kOccBatch = 8;    // occupancy-bit loads in flight per lane (filter-first mode)
constexpr int kSlotBatch = 4;   // slot loads in flight per lane (filter-first mode)
constexpr int kSlotBatchPM = 2; // hits per batch in filter-first mode with the product map
constexpr int kOccBatchPM = 1;  // filter tests per batch in filter-first mode with the product map

// One- and two-word keys copy the part filters into LDS; wider keys read them from memory.
template <int Wp>
struct PartLds {
    static constexpr int words = Wp <= 2 ? kPartWords : 1;
};

struct HamView {
    const uint64_t *__restrict__ g_mask;   // [G][Wp]
    const uint64_t *__restrict__ g_hash;   // [G]
    const uint64_t *__restrict__ g_pos;    // [G] four 16-bit ladder qubits
    const uint64_t *__restrict__ g_scan;   // [G padded to 8] live table | 4 x 12-bit shifts
    const uint32_t *__restrict__ g_info;   // [G] k | ladder | care | live16 << 16
    const uint32_t *__restrict__ g_term0;  // [G]
    const uint32_t *__restrict__ g_nterm;  // [G]
    const uint16_t *__restrict__ g_iptr;   // [G][kIptr]
    const uint64_t *__restrict__ t_cws;    // [T][3][Wp] care, want, sign masks
    const void *__restrict__ t_coef;       // [T] double2 or float2
    int64_t G;
    int coef_f32;                          // t_coef holds float2 (1) or double2 (0)
    const uint32_t *__restrict__ g_part;   // [G] packed part indices of the flip masks (with filters)
    const uint4 *__restrict__ t_cw32;      // [T] care, want, sign masks as 32-bit words (n <= 32), or NULL
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


// 4-bit ladder integer of a row from a scan record: bit j = row bit at qubit p_j = shift_j + j.
// One-word keys are shifted in registers (one 64-bit shift per bit); wider keys read the
// wave's bit planes in LDS (plane p_j, bit = the lane), which avoids indexing a register array
// with a run-time word number.  Unused positions are don't-cares of the replicated live table.
// (Product-map kernels take the positions decoded, see hit_range_pm.)
template <int Wp>
__device__ __forceinline__ uint32_t row_lint(const uint64_t (&key)[Wp], uint64_t rec, const uint64_t *planes,
                                             int lane) {
    uint32_t L = 0;
    if (Wp == 1) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t sh = (uint32_t)(rec >> (16 + 12 * j)) & 63u;
            L |= (uint32_t)(key[0] >> sh) & (1u << j);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t p = ((uint32_t)(rec >> (16 + 12 * j)) & 0xFFFu) + (uint32_t)j;
            L |= (uint32_t)((planes[p] >> lane) & 1ull) << j;
        }
    }
    return L;
}

// A 32-bit word of lane (lane ^ SH), without the LDS crossbar: half-wave and row swaps
// (permlane swaps) for SH = 32 and 16, row rotations and quad permutations (DPP) below.
template <int SH>
__device__ __forceinline__ uint32_t lane_xor32(uint32_t x, int lane) {
    if constexpr (SH == 32) {
        // vdst's upper half trades places with src0's lower half
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return lane < 32 ? r[1] : r[0];
    } else if constexpr (SH == 16) {
        // vdst's odd rows of 16 trade places with src0's even rows
        const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        return (lane & 16) ? r[0] : r[1];
    } else if constexpr (SH == 8) {
        return __builtin_amdgcn_update_dpp(0u, x, 0x128, 0xF, 0xF, false);  // row_ror:8
    } else if constexpr (SH == 4) {
        // lane l of a row of 16 reads lane l - 4 (row_ror:4) or l + 4 (row_ror:12)
        const uint32_t dn = __builtin_amdgcn_update_dpp(0u, x, 0x124, 0xF, 0xF, false);
        const uint32_t up = __builtin_amdgcn_update_dpp(0u, x, 0x12C, 0xF, 0xF, false);
        return (lane & 4) ? dn : up;
    } else if constexpr (SH == 2) {
        return __builtin_amdgcn_update_dpp(0u, x, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    } else {
        return __builtin_amdgcn_update_dpp(0u, x, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    }
}

template <int SH>
__device__ __forceinline__ uint64_t lane_xor64(uint64_t v, int lane) {
    const uint32_t lo = lane_xor32<SH>((uint32_t)v, lane);
    const uint32_t hi = lane_xor32<SH>((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

template <int K>
__device__ __forceinline__ uint64_t transpose_stage(uint64_t x, int lane) {
    constexpr int sh = 32 >> K;
    constexpr uint64_t M[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                               0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
    const uint64_t y = lane_xor64<sh>(x, lane);
    return (lane & sh) ? ((x & ~M[K]) | ((y & ~M[K]) >> sh)) : ((x & M[K]) | ((y & M[K]) << sh));
}

// 64 x 64 bit transpose across a wave: on return, bit j of lane i's word is bit i of lane j's
// input word.  Six butterfly stages, each exchanging words between lanes l and l ^ sh; every
// lane of the wave must take part.
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t x, int lane) {
    x = transpose_stage<0>(x, lane);
    x = transpose_stage<1>(x, lane);
    x = transpose_stage<2>(x, lane);
    x = transpose_stage<3>(x, lane);
    x = transpose_stage<4>(x, lane);
    return transpose_stage<5>(x, lane);
}

// Bit-sliced live test: bit r of the result = T[L_r], L_r = (a_r, b_r, c_r, d_r) as bits 0..3,
// for the 16-entry table T and the four planes a, b, c, d.
__device__ __forceinline__ uint64_t sliced_table(uint32_t T, uint64_t a, uint64_t b, uint64_t c, uint64_t d) {
    const uint64_t m[4] = {~a & ~b, a & ~b, ~a & b, a & b};
    const uint64_t u[4] = {~c & ~d, c & ~d, ~c & d, c & d};
    uint64_t f = 0;
#pragma unroll
    for (int hi = 0; hi < 4; ++hi) {
        uint64_t g = 0;
#pragma unroll
        for (int lo = 0; lo < 4; ++lo) g |= m[lo] & (0ull - (uint64_t)((T >> (4 * hi + lo)) & 1u));
        f |= g & u[hi];
    }
    return f;
}

// LDS staging of one chunk: what the probes and the hit ranges read, plus the bit planes of
// every wave's rows.
template <int Wp>
struct ChunkLds {
    // Hash-table kernels keep the groups' hashes and flip masks here.  Product-map kernels probe
    // no table; they keep the decoded ladder positions and the ranks of the block's shared high
    // part through each group's flips instead.
    union alignas(16) {
        struct {
            uint64_t hash[kChunk];
            uint64_t mask[kChunk][Wp];
        } t;
        struct {
            // packed part indices of the flips | rank of the high part reached times the number
            // of low parts (when the block's rows share their high part)
            uint2 gh[kChunk];
            // qubits of ladder bits 0..3 (5 bits each) | ladder mask << 20, first term
            uint2 rt[kChunk];
        } m;
    } u;
    uint64_t rec[kChunk];                // scan records (ladder positions for the hit ranges)
    uint32_t term0[kChunk];
    uint32_t nterm[kChunk];
    uint32_t lmask[kChunk];              // ladder-integer bits used for the range (0: all terms)
    uint16_t iptr[kChunk][kIptr];
    uint64_t planes[kBlock / 64][64 * Wp];
    uint8_t clist[kBlock / 64][kChunk];  // lockstep filter-first: the wave's k-th live group
    uint32_t gpart[kChunk];              // the chunk's groups' packed part indices
    uint32_t pf[PartLds<Wp>::words];     // part filters (one- and two-word keys)
    uint32_t whi[kBlock / 64];           // each wave's shared high part (see row_engine)
};

// Whether the row's bits under a term's care mask equal its want mask (projector and ladder
// bits), and the parity of the row's bits under its sign mask; cws = [care][want][sign] words.
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

// Sum over the terms [t0, t0 + len) that match the row's projector bits, with popcount-parity
// signs, in increasing t (the table kernels' walk): the care and want masks are read first, the
// sign mask and the coefficient only for a matching term.  Returns false when no term matches
// (no stored entry).
template <int Wp, class ET>
__device__ __forceinline__ bool range_value(const HamView &h, const uint64_t (&key)[Wp], uint32_t t0, uint32_t len,
                                            ET &vre, ET &vim) {
    using CT = typename C2<ET>::T;
    const CT *__restrict__ coef = (const CT *)h.t_coef;
    bool any = false;
    vre = 0;
    vim = 0;
    auto term = [&](uint32_t t) {
        const uint64_t *cws = h.t_cws + (int64_t)t * 3 * Wp;
        if (!term_pass<Wp>(key, cws)) return;
        any = true;
        const CT c = coef[t];
        if (term_parity<Wp>(key, cws)) {
            vre -= c.x;
            vim -= c.y;
        } else {
            vre += c.x;
            vim += c.y;
        }
    };
    // strings of at most 32 qubits: a projector tail (see range_sum) is visited only at the
    // qubits the row has set
    uint32_t t1 = t0 + len, R = 0, m = 0;
    if (Wp == 1 && h.t_cw32) {
        R = h.t_cw32[t0].w;
        t1 -= (uint32_t)__popc(R);
        m = (uint32_t)key[0] & R;
    }
    for (uint32_t t = t0; t < t1; ++t) term(t);
    for (; m; m &= m - 1u) term(t1 + (uint32_t)__popc(R & ((1u << __builtin_ctz(m)) - 1u)));
    return any;
}

// One term's care, want and sign masks and its coefficient c' (Methods, Matrix evaluation: a
// term contributes c' (-1)^{popcount(b & S)} to a row b whose bits under `care` equal `want`).
// NARROW: strings of at most 32 qubits, masks as 32-bit words (one 16-byte load).
template <int Wp, bool NARROW, class ET>
struct TermRec {
    uint64_t m[3][Wp];
    typename C2<ET>::T c;
};
template <int Wp, class ET>
struct TermRec<Wp, true, ET> {
    uint4 m;  // care, want, sign, unused
    typename C2<ET>::T c;
};

template <int Wp, bool NARROW, class ET>
__device__ __forceinline__ void load_term(const HamView &h, uint32_t t, TermRec<Wp, NARROW, ET> &r) {
    if constexpr (NARROW) {
        r.m = h.t_cw32[t];
    } else {
        const uint64_t *cw = h.t_cws + (int64_t)t * 3 * Wp;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int w = 0; w < Wp; ++w) r.m[k][w] = cw[k * Wp + w];
    }
    r.c = ((const typename C2<ET>::T *)h.t_coef)[t];
}

// Adds the term to (vre, vim) if the row's projector bits match.  A term that fails adds +0,
// which changes no sum (the sums start at +0 and are never -0), so there is no branch.
template <int Wp, bool NARROW, class ET>
__device__ __forceinline__ void add_term(const uint64_t (&key)[Wp], const TermRec<Wp, NARROW, ET> &r, ET &vre,
                                         ET &vim, bool &any) {
    bool ok;
    uint32_t par;
    if constexpr (NARROW) {
        const uint32_t k = (uint32_t)key[0];
        ok = (k & r.m.x) == r.m.y;
        par = (uint32_t)__popc(k & r.m.z);
    } else {
        ok = true;
        par = 0;
#pragma unroll
        for (int w = 0; w < Wp; ++w) {
            ok &= (key[w] & r.m[0][w]) == r.m[1][w];
            par += (uint32_t)__popcll(key[w] & r.m[2][w]);
        }
    }
    const ET re = (par & 1u) ? -r.c.x : r.c.x, im = (par & 1u) ? -r.c.y : r.c.y;
    vre += ok ? re : (ET)0;
    vim += ok ? im : (ET)0;
    any |= ok;
}

// Sum over the terms [t0, t0 + len), len >= 1, whose projector bits match the row, with
// popcount-parity signs, in increasing t; `first` holds term t0, already loaded.  The rest are
// loaded two at a time, both before either is tested.  Returns false when no term matches (no
// stored entry).  NARROW (strings of at most 32 qubits): the range may end in a projector tail,
// one term per qubit of the mask R that the first term carries, each wanting its qubit set and
// stored in increasing qubit order; only the tail terms of the qubits the row has set are
// visited (the others cannot match), so the matching terms are added in the same order.
template <int Wp, bool NARROW, class ET>
__device__ __forceinline__ bool range_sum(const HamView &h, const uint64_t (&key)[Wp], uint32_t t0, uint32_t len,
                                          const TermRec<Wp, NARROW, ET> &first, ET &vre, ET &vim) {
    bool any = false;
    vre = 0;
    vim = 0;
    add_term<Wp, NARROW, ET>(key, first, vre, vim, any);
    uint32_t t1 = t0 + len;  // end of the terms visited one by one
    uint32_t R = 0, m = 0;
    if constexpr (NARROW) {
        R = first.m.w;
        t1 -= (uint32_t)__popc(R);
        m = (uint32_t)key[0] & R;
        // a range of tail terms only: its first term (the lowest qubit of R) is summed already
        if (t1 == t0) m &= ~(R & (0u - R));
    }
    uint32_t t = t0 + 1u;
    for (; t + 1u < t1; t += 2u) {
        TermRec<Wp, NARROW, ET> a, b;
        load_term<Wp, NARROW, ET>(h, t, a);
        load_term<Wp, NARROW, ET>(h, t + 1u, b);
        add_term<Wp, NARROW, ET>(key, a, vre, vim, any);
        add_term<Wp, NARROW, ET>(key, b, vre, vim, any);
    }
    if (t < t1) {
        TermRec<Wp, NARROW, ET> a;
        load_term<Wp, NARROW, ET>(h, t, a);
        add_term<Wp, NARROW, ET>(key, a, vre, vim, any);
    }
    if constexpr (NARROW) {
        // the tail terms of the row's set qubits, two at a time
        const uint32_t base = t1;  // the first tail term
        while (m) {
            const uint32_t r0 = (uint32_t)__builtin_ctz(m);
            m &= m - 1u;
            const bool two = m != 0u;
            const uint32_t r1 = two ? (uint32_t)__builtin_ctz(m) : r0;
            m &= two ? m - 1u : m;
            TermRec<Wp, NARROW, ET> a, b;
            load_term<Wp, NARROW, ET>(h, base + (uint32_t)__popc(R & ((1u << r0) - 1u)), a);
            load_term<Wp, NARROW, ET>(h, base + (uint32_t)__popc(R & ((1u << r1) - 1u)), b);
            add_term<Wp, NARROW, ET>(key, a, vre, vim, any);
            if (two) add_term<Wp, NARROW, ET>(key, b, vre, vim, any);
        }
    }
    return any;
}

// Pops the lowest set bit of a 64-bit mask held as two words; -1 when empty.
__device__ __forceinline__ int pop_group(uint32_t &mlo, uint32_t &mhi) {
    const bool use_lo = mlo != 0u;
    const uint32_t w = use_lo ? mlo : mhi;
    const int c = w ? (int)__builtin_ctz(w) + (use_lo ? 0 : 32) : -1;
    const uint32_t nw = w & (w - 1u);
    mlo = use_lo ? nw : mlo;
    mhi = use_lo ? mhi : nw;
    return c;
}

// Highest qubit of a group's flip mask (its most significant off-diagonal bit).
template <int Wp>
__device__ __forceinline__ uint32_t group_msob(const uint64_t *__restrict__ mask) {
    uint32_t ms = 0;
    bool found = false;
#pragma unroll
    for (int w = Wp - 1; w >= 0; --w) {
        const uint64_t m = mask[w];
        if (!found && m) {
            ms = 64u * (uint32_t)w + 63u - (uint32_t)__clzll(m);
            found = true;
        }
    }
    return ms;
}

// A hit consumer: fetch(j) issues the loads a hit on column j needs (x_j, say) and returns them;
// use(j, vre, vim, pre) consumes a stored element H_ij = vre + i vim (the sum in ET of the
// row's matching terms) with what fetch returned.  The engine resolves a batch of groups, then
// fetches for all of the batch's hits and loads the first term of each, then evaluates and
// uses them in increasing group order, so the load latencies overlap while every row's sum
// keeps its fixed order.  Probes whose column is present but where no term matches the row's
// projector bits are not stored entries and are not handed over.
template <class ET, class Use, class Fetch>
struct HitSink {
    using value_type = ET;
    Use use;
    Fetch fetch;
};
struct NoFetch {
    __device__ __forceinline__ int operator()(int64_t) const { return 0; }
};
template <class ET, class Use>
__device__ __forceinline__ HitSink<ET, Use, NoFetch> sink(Use u) {
    return HitSink<ET, Use, NoFetch>{u, NoFetch{}};
}
template <class ET, class Use, class Fetch>
__device__ __forceinline__ HitSink<ET, Use, Fetch> sink(Use u, Fetch f) {
    return HitSink<ET, Use, Fetch>{u, f};
}

// Term range [t0, t0 + len) of chunk group cc for the row (its ladder integer selects it).
template <int Wp>
__device__ __forceinline__ void hit_range(const ChunkLds<Wp> &lds, const uint64_t (&key)[Wp], const uint64_t *planes,
                                          int lane, int cc, uint32_t &t0, uint32_t &len) {
    const uint32_t lm = lds.lmask[cc];
    const uint32_t L = row_lint<Wp>(key, lds.rec[cc], planes, lane) & lm;
    const uint32_t lo = lds.iptr[cc][L];
    const uint32_t hi = lm ? (uint32_t)lds.iptr[cc][L + 1] : lds.nterm[cc];
    t0 = lds.term0[cc] + lo;
    len = hi - lo;
}

// The same in product-map kernels (strings of at most 32 qubits, k = the row's bits): the ladder
// positions, the ladder mask and the first term come in one 8-byte record, and a group without
// ladder bits keeps its term count in its first two range pointers; no branch.
template <int Wp>
__device__ __forceinline__ void hit_range_rt(const ChunkLds<Wp> &lds, uint32_t k, int cc, uint2 rt, uint32_t &t0,
                                             uint32_t &len) {
    uint32_t L = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) L |= __builtin_amdgcn_ubfe(k, __builtin_amdgcn_ubfe(rt.x, 5u * j, 5u), 1u) << j;
    const uint32_t lm = __builtin_amdgcn_ubfe(rt.x, 20u, 4u);
    L &= lm;
    const uint32_t a = lds.iptr[cc][L], b = lds.iptr[cc][L + 1];
    const uint32_t lo = lm ? a : 0u, hi = lm ? b : (a | (b << 16));
    t0 = rt.y + lo;
    len = hi - lo;
}
template <int Wp>
__device__ __forceinline__ void hit_range_pm(const ChunkLds<Wp> &lds, uint32_t k, int cc, uint32_t &t0,
                                             uint32_t &len) {
    hit_range_rt<Wp>(lds, k, cc, lds.u.m.rt[cc], t0, len);
}

// Fetch, evaluate and use a batch whose columns are resolved (j[b] < 0: no hit).  A lane
// without a hit in the batch loads nothing.  Otherwise x_j (or what the sink fetches) is
// requested for every slot; in product-map kernels (PM: strings of at most 32 qubits, so 32-bit
// term masks) the term ranges of all slots are read and the first term of each is loaded before
// any is summed (term 0 for a slot without a hit, so no load needs a branch; an off-diagonal
// group always has a term).  The slots are summed and used in increasing b.
template <int Wp, int NB, bool PM, class Sink>
__device__ __forceinline__ void deliver(const HamView &h, const ChunkLds<Wp> &lds, const uint64_t (&key)[Wp],
                                        const uint64_t *planes, int lane, const int (&c)[NB], const int64_t (&j)[NB],
                                        Sink &on_hit) {
    using ET = typename Sink::value_type;
    bool any = false;
#pragma unroll
    for (int b = 0; b < NB; ++b) any |= j[b] >= 0;
    if (!any) return;  // most probes miss on sparse samples: no loads at all for them
    decltype(on_hit.fetch(0)) pre[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) pre[b] = on_hit.fetch(j[b]);
    if constexpr (PM) {
        // 32-bit masks: the records are small enough to hold one per slot
        uint32_t t0[NB], len[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            hit_range_pm<Wp>(lds, (uint32_t)key[0], c[b] & (kChunk - 1), t0[b], len[b]);
            if (j[b] < 0) len[b] = 0u;
        }
        TermRec<Wp, true, ET> first[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) load_term<Wp, true, ET>(h, len[b] ? t0[b] : 0u, first[b]);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (!len[b]) continue;
            ET vre, vim;
            if (range_sum<Wp, true, ET>(h, key, t0[b], len[b], first[b], vre, vim))
                on_hit.use(j[b], vre, vim, pre[b]);
        }
    } else {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (j[b] < 0) continue;
            uint32_t t0, len;
            hit_range<Wp>(lds, key, planes, lane, c[b], t0, len);
            ET vre, vim;
            if (range_value<Wp, ET>(h, key, t0, len, vre, vim)) on_hit.use(j[b], vre, vim, pre[b]);
        }
    }
}

// Probes NB groups for the lane's row: c[b] = chunk-local group, act[b] = whether the lane
// probes it.  All occupancy-bit loads are issued before the slot loads, and the slots before any
// hit is fetched; hits go to on_hit in increasing b (the caller passes increasing groups).
template <int Wp, int NB, bool PM, class OnHit>
__device__ __forceinline__ void probe_groups(const SubView &s, const HamView &h, const ChunkLds<Wp> &lds,
                                             const uint64_t (&key)[Wp],
                                             uint64_t hrow, uint32_t prow, const uint32_t *pf, const uint16_t *pr,
                                             bool hr, const uint64_t *planes, int lane, const int (&c)[NB],
                                             const bool (&act)[NB], OnHit &on_hit) {
    if (PM) {
        // product map: the column's index comes from its parts' ranks, no table access.  With
        // hr (the block's rows share their high part) the high rank comes with the chunk and the
        // scan has dropped the groups whose high part does not occur, so only the low part is
        // tested here.
        int64_t j[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int cc = c[b] & (kChunk - 1);
            const uint2 gh = lds.u.m.gh[cc];
            const uint32_t p = prow ^ gh.x, lo = p & 0xFFFFu;
            int64_t jb;
            if (hr)
                jb = ((pf[lo >> 5] >> (lo & 31u)) & 1u) ? (int64_t)(gh.y + part_rank(pf, pr, 0, lo)) : (int64_t)-1;
            else
                jb = product_index(pf, pr, s.pna, p);
            j[b] = act[b] ? jb : -1;
        }
        deliver<Wp, NB, PM>(h, lds, key, planes, lane, c, j, on_hit);
        return;
    }
    // unconditional loads: idle lanes read word 0 / slot 0 and ignore them
    uint64_t hh[NB];
    uint32_t pos[NB], word[NB];
    bool a[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        a[b] = act[b] && (!pf || part_pass(pf, prow ^ lds.gpart[c[b] & (kChunk - 1)]));
        hh[b] = hrow ^ lds.u.t.hash[c[b] & (kChunk - 1)];
        pos[b] = (uint32_t)hh[b] & s.cmask;
        word[b] = s.bitmap[a[b] ? (pos[b] >> 5) : 0u];
    }
    uint64_t slot[NB];
    bool occ[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        occ[b] = a[b] && ((word[b] >> (pos[b] & 31u)) & 1u);
        slot[b] = s.slots[occ[b] ? pos[b] : 0u];
    }
    int64_t j[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        j[b] = -1;
        if (!occ[b]) continue;
        const uint32_t tag = (uint32_t)(hh[b] >> 32);
        uint64_t col[Wp];
#pragma unroll
        for (int w = 0; w < Wp; ++w) col[w] = key[w] ^ lds.u.t.mask[c[b]][w];
        if ((uint32_t)(slot[b] >> 32) == tag) j[b] = slot_match<Wp>(s, slot[b], 0u, col);
        if (j[b] < 0) {
            // the home slot held another string: follow the run while slots stay occupied
            const uint32_t nxt = (pos[b] + 1) & s.cmask;
            const uint32_t nw = ((nxt >> 5) == (pos[b] >> 5)) ? word[b] : s.bitmap[nxt >> 5];
            if ((nw >> (nxt & 31u)) & 1u) j[b] = probe_from<Wp>(s, nxt, 1u, tag, col);
        }
    }
    deliver<Wp, NB, PM>(h, lds, key, planes, lane, c, j, on_hit);
}

// Filter-first mode with part filters, phase 1: a group whose column passes both part filters
// is marked for phase 2 (occ) with the run continued past an occupied home slot (occn); no
// occupancy bit is read (the slot itself shows whether it is empty), so a column that passes
// costs one slot read and one that fails costs nothing beyond LDS.
// hi_done: the wave's rows share their high part and the scan has already dropped the groups
// that flip it to an absent one, so only the low part is tested (wave-uniform).
template <int NB>
__device__ __forceinline__ void part_occupancy(const uint32_t *pf, const uint32_t *lpart, uint32_t prow, bool hi_done,
                                               const int (&c)[NB], const bool (&act)[NB], uint64_t &occ,
                                               uint64_t &occn) {
    if (hi_done) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uint32_t lo = (prow ^ lpart[c[b] & (kChunk - 1)]) & 0xFFFFu;
            const bool o = act[b] && ((pf[lo >> 5] >> (lo & 31u)) & 1u);
            occ |= (uint64_t)o << (c[b] & (kChunk - 1));
            occn |= (uint64_t)o << (c[b] & (kChunk - 1));
        }
        return;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const bool o = act[b] && part_pass(pf, prow ^ lpart[c[b] & (kChunk - 1)]);
        occ |= (uint64_t)o << (c[b] & (kChunk - 1));
        occn |= (uint64_t)o << (c[b] & (kChunk - 1));
    }
}

// Filter-first mode, phase 1: for the NB groups c[b] the lane probes (act[b]), sets bit c[b] of
// `occ` when the group's home slot is occupied, and of `occn` when the slot after it is occupied
// too (or lies in the next bitmap word, so is not known here).  All NB loads are in flight at once.
template <int NB>
__device__ __forceinline__ void occupancy(const SubView &s, const uint64_t *lhash, uint64_t hrow, const int (&c)[NB],
                                          const bool (&act)[NB], uint64_t &occ, uint64_t &occn) {
    // the loads are unconditional (idle lanes all read word 0 and ignore it), so they are issued
    // back to back without a branch per load
    uint32_t pos[NB], word[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        pos[b] = (uint32_t)(hrow ^ lhash[c[b] & (kChunk - 1)]) & s.cmask;
        word[b] = s.bitmap[act[b] ? (pos[b] >> 5) : 0u];
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const uint32_t sh = pos[b] & 31u;
        const uint32_t o = act[b] ? ((word[b] >> sh) & 1u) : 0u;
        const uint32_t n = sh == 31u ? 1u : ((word[b] >> (sh + 1u)) & 1u);
        occ |= (uint64_t)o << (c[b] & (kChunk - 1));
        occn |= (uint64_t)(o & n) << (c[b] & (kChunk - 1));
    }
}

// Filter-first mode, phase 2: resolves NB groups whose home slot is occupied: reads the slots,
// follows the run when the home slot holds another string and the next slot may be occupied
// (next[b]), and hands hits to on_hit in increasing b.
template <int Wp, int NB, bool PM, class OnHit>
__device__ __forceinline__ void resolve_groups(const SubView &s, const HamView &h, const ChunkLds<Wp> &lds,
                                               const uint64_t (&key)[Wp],
                                               uint64_t hrow, uint32_t prow, const uint32_t *pf, const uint16_t *pr,
                                               bool hr, const uint64_t *planes, int lane, const int (&c)[NB],
                                               const bool (&act)[NB], const bool (&next)[NB], OnHit &on_hit) {
    if (PM) {
        // product map: a group marked here passed both part filters, so its column is present
        // (with hr the high rank comes with the chunk)
        int64_t j[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int cc = c[b] & (kChunk - 1);
            const uint2 gh = lds.u.m.gh[cc];
            const uint32_t p = prow ^ gh.x;
            const uint32_t r = hr ? gh.y + part_rank(pf, pr, 0, p & 0xFFFFu) : product_rank(pf, pr, s.pna, p);
            j[b] = act[b] ? (int64_t)r : -1;
        }
        deliver<Wp, NB, PM>(h, lds, key, planes, lane, c, j, on_hit);
        return;
    }
    uint64_t hh[NB], slot[NB];
    uint32_t pos[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        hh[b] = hrow ^ lds.u.t.hash[c[b] & (kChunk - 1)];
        pos[b] = (uint32_t)hh[b] & s.cmask;
        slot[b] = s.slots[act[b] ? pos[b] : 0u];  // unconditional, as above
    }
    int64_t j[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        j[b] = -1;
        // with part filters the home slot was read without its occupancy bit: empty = absent
        if (!act[b] || slot[b] == ~0ull) continue;
        const uint32_t tag = (uint32_t)(hh[b] >> 32);
        uint64_t col[Wp];
#pragma unroll
        for (int w = 0; w < Wp; ++w) col[w] = key[w] ^ lds.u.t.mask[c[b]][w];
        if ((uint32_t)(slot[b] >> 32) == tag) j[b] = slot_match<Wp>(s, slot[b], 0u, col);
        if (j[b] < 0 && next[b]) j[b] = probe_from<Wp>(s, (pos[b] + 1) & s.cmask, 1u, tag, col);
    }
    deliver<Wp, NB, PM>(h, lds, key, planes, lane, c, j, on_hit);
}

// Filter-first phase 2 of product-map kernels, software-pipelined: while one batch's loads (x_j
// and the first term of each hit) are in flight, the next batch's groups are popped and their
// records and columns read from LDS.  `occ` holds the chunk's groups whose columns are present;
// every lane still sums and uses its hits in increasing group order, exactly as resolve_groups
// does.
template <int Wp, int NB, class OnHit>
__device__ __forceinline__ void pm_phase2(const SubView &s, const HamView &h, const ChunkLds<Wp> &lds,
                                          const uint64_t (&key)[Wp], uint32_t prow, const uint32_t *pf,
                                          const uint16_t *pr, bool hr, uint64_t occ, OnHit &on_hit) {
    using ET = typename OnHit::value_type;
    const uint32_t k = (uint32_t)key[0];
    // pops the next NB groups: chunk index, column (-1: none) and term record
    auto next = [&](int (&cb)[NB], int64_t (&jb)[NB], uint2 (&rb)[NB]) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int g = occ ? (int)__builtin_ctzll(occ) : -1;
            occ &= occ - 1ull;
            const int cc = g < 0 ? 0 : g;
            const uint2 gh = lds.u.m.gh[cc];
            rb[b] = lds.u.m.rt[cc];
            const uint32_t p = prow ^ gh.x;
            const uint32_t r = hr ? gh.y + part_rank(pf, pr, 0, p & 0xFFFFu) : product_rank(pf, pr, s.pna, p);
            cb[b] = cc;
            jb[b] = g >= 0 ? (int64_t)r : (int64_t)-1;
        }
    };
    int c[NB];
    int64_t j[NB];
    uint2 rt[NB];
    next(c, j, rt);
    while (__any(j[0] >= 0)) {  // a batch's slots fill in order: slot 0 empty = nothing left
        decltype(on_hit.fetch(0)) pre[NB];
        uint32_t t0[NB], len[NB];
        TermRec<Wp, true, ET> first[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) pre[b] = on_hit.fetch(j[b]);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            hit_range_rt<Wp>(lds, k, c[b], rt[b], t0[b], len[b]);
            if (j[b] < 0) len[b] = 0u;
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) load_term<Wp, true, ET>(h, len[b] ? t0[b] : 0u, first[b]);
        int cn[NB];
        int64_t jn[NB];
        uint2 rn[NB];
        next(cn, jn, rn);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (!len[b]) continue;
            ET vre, vim;
            if (range_sum<Wp, true, ET>(h, key, t0[b], len[b], first[b], vre, vim))
                on_hit.use(j[b], vre, vim, pre[b]);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            c[b] = cn[b];
            j[b] = jn[b];
            rt[b] = rn[b];
        }
    }
}

// Walks all groups for the lane's row and hands on_hit (a HitSink) every probe whose
// column b_i ^ M_g is in the subspace (j = its index; [t0, t0 + len) = the group's terms for
// the row's ladder integer), in increasing g.  All threads of the block must call it (chunks
// are staged through LDS with barriers).  `valid` = the lane owns a row.
//
// LOWER keeps only groups whose column sorts below the row (Methods, Lower / upper triangle
// evaluation): the flip changes the row's bit at the group's most significant off-diagonal
// bit, so the column is smaller exactly when that row bit is set, and in the ascending
// canonical order its index is smaller too.  One more plane test per group in the scan.
//
// `lockstep` changes only which probes share an instruction: the wave walks the groups that are
// live for any of its rows in increasing order, kLockBatch at a time, and every lane whose row
// has the group live probes it in the same instruction.  When the wave's rows sit in one
// stretch of the hash table (rows taken in slot order), the columns of one group, with hashes
// h(b_i) ^ h(M_g), land in one stretch as well, and the wave's occupancy-bit loads for the group
// touch one or two cache lines instead of one line per lane.  Each lane still meets its hits in
// increasing group order, so both modes give bitwise the same sums.
template <int Wp, bool LOWER = false, int PF = 1, class OnHit>
__device__ __forceinline__ void row_engine(const SubView &s, const HamView &h, const uint64_t (&key)[Wp],
                                           uint64_t hrow, uint32_t prow, bool valid, ChunkLds<Wp> &lds,
                                           OnHit &&on_hit, unsigned long long *probes = nullptr,
                                           bool lockstep = false, bool filter_first = false) {
    const int lane = threadIdx.x & 63;
    uint64_t *planes = lds.planes[threadIdx.x >> 6];
#pragma unroll
    for (int w = 0; w < Wp; ++w) planes[64 * w + lane] = wave_transpose64(valid ? key[w] : 0ull, lane);
    const uint64_t vrows = __ballot(valid);
    // part filters: one- and two-word keys read an LDS copy (visible after the first chunk's
    // barrier, before any probe)
    // PF = 0 compiles the engine without part filters (the launch checks that the subspace has
    // none); PF = 1 tests them when the subspace has them; PF = 2 is for subspaces with a product
    // map (one-word keys; the launch checks), whose columns take their index from it
    constexpr bool PM = PF == 2 && Wp == 1;
    const uint32_t *pf = nullptr;
    if (PF && s.pfilt) {
        if (PartLds<Wp>::words == kPartWords) {
            for (int k = threadIdx.x; k < kPartWords; k += kBlock) lds.pf[k] = s.pfilt[k];
            pf = lds.pf;
        } else {
            pf = s.pfilt;
        }
    }
    // the product map's prefix counts: an LDS array of their own, in product-map kernels only
    const uint16_t *pr = nullptr;
    if constexpr (PM) {
        __shared__ uint16_t pr_lds[kPartWords];
        for (int k = threadIdx.x; k < kPartWords; k += kBlock) pr_lds[k] = s.prank[k];
        pr = pr_lds;
    }
    // When every row of the wave has the same high (or low) part, as consecutive rows of an
    // alpha x beta product do, that part's filter test depends on the group only: the scan
    // applies it to the whole wave's live word before any lane probes.
    uint32_t uni_mask = 0u, uni_part = 0u;
    if (pf) {
        const int first = (int)__builtin_ctzll(vrows | (1ull << 63));
        const uint32_t p0 = (uint32_t)__shfl((int)prow, first, 64);
        if (__all(!valid || ((prow ^ p0) >> 16) == 0u)) uni_mask |= 0xFFFF0000u;
        if (__all(!valid || ((prow ^ p0) & 0xFFFFu) == 0u)) uni_mask |= 0x0000FFFFu;
        uni_part = p0;
    }
    // When all rows of the block share their high part (an alpha x beta product in canonical
    // order: 256 rows of one beta string, mostly), a chunk whose groups all flip it to a high
    // part that does not occur holds no live group for any row, and the whole block skips it
    // (bulk group rejection).  Each wave posts its shared high part; every wave then takes the
    // same decision per chunk, so the barriers stay matched.  Not for the work counter, which
    // counts the method's lookups.
    constexpr uint32_t kMixed = 0xFFFFFFFFu, kEmpty = 0xFFFFFFFEu;
    const bool bulk = pf && !probes;
    if (bulk && lane == 0)
        lds.whi[threadIdx.x >> 6] = vrows == 0ull ? kEmpty : ((uni_mask >> 16) ? (uni_part >> 16) : kMixed);
    uint32_t blk_hi = kMixed;
    constexpr int kSB = PM ? kSlotBatchPM : kSlotBatch;  // filter-first phase 2 batch
    for (int64_t g0 = 0; g0 < h.G; g0 += kChunk) {
        const int nc = (int)((h.G - g0) < kChunk ? (h.G - g0) : kChunk);
        __syncthreads();
        if (bulk) {
            if (g0 == 0) {
                uint32_t v = kEmpty;
#pragma unroll
                for (int w = 0; w < kBlock / 64; ++w) {
                    const uint32_t u = lds.whi[w];
                    v = u == kEmpty ? v : ((v == kEmpty || v == u) ? u : kMixed);
                }
                blk_hi = v;
            }
            if (blk_hi == kEmpty) break;  // a block without rows
            if (blk_hi != kMixed) {
                bool lv = false;
                if (lane < nc) {
                    const uint32_t q = blk_hi ^ (h.g_part[g0 + lane] >> 16);
                    lv = ((pf[kPartWords / 2 + (q >> 5)] >> (q & 31u)) & 1u) != 0u;
                }
                if (__ballot(lv) == 0ull) continue;
            }
        }
        // product-map kernels: whether the block's rows share their high part (then every
        // group's column has one high part for the whole block, and its rank comes with the chunk)
        const bool hr = PM && blk_hi < (1u << kPartBits);
        for (int c = threadIdx.x; c < nc; c += kBlock) {
            const int64_t g = g0 + c;
            const uint32_t info = h.g_info[g];
            const uint32_t lm = (info & kInfoLadder) ? ((1u << (info & kInfoKMask)) - 1u) : 0u;
            if constexpr (PM) {
                const uint64_t rec = h.g_scan[g];
                const uint32_t gp = h.g_part[g];
                uint32_t pk = lm << 20;
#pragma unroll
                for (int j = 0; j < 4; ++j) pk |= (((uint32_t)(rec >> (16 + 12 * j)) + (uint32_t)j) & 31u) << (5 * j);
                lds.u.m.rt[c] = make_uint2(pk, h.g_term0[g]);
                lds.u.m.gh[c] = make_uint2(gp, hr ? part_rank(pf, pr, 1, blk_hi ^ (gp >> 16)) * s.pna : 0u);
                if (lm) {
#pragma unroll
                    for (int q = 0; q < kIptr; ++q) lds.iptr[c][q] = h.g_iptr[g * kIptr + q];
                } else {
                    const uint32_t nt = h.g_nterm[g];
                    lds.iptr[c][0] = (uint16_t)(nt & 0xFFFFu);
                    lds.iptr[c][1] = (uint16_t)(nt >> 16);
                }
                lds.gpart[c] = gp;
            } else {
                lds.u.t.hash[c] = h.g_hash[g];
#pragma unroll
                for (int w = 0; w < Wp; ++w) lds.u.t.mask[c][w] = h.g_mask[g * Wp + w];
                lds.rec[c] = h.g_scan[g];
                lds.term0[c] = h.g_term0[g];
                lds.nterm[c] = h.g_nterm[g];
                lds.lmask[c] = lm;
#pragma unroll
                for (int q = 0; q < kIptr; ++q) lds.iptr[c][q] = h.g_iptr[g * kIptr + q];
                lds.gpart[c] = pf ? h.g_part[g] : 0u;
            }
        }
        // scan: lane l evaluates group g0 + l for the wave's 64 rows, then the masks are
        // transposed to one live-group mask per row
        uint64_t live = 0, live_method = 0;
        if (lane < nc) {
            const uint64_t rec = h.g_scan[g0 + lane];
            uint64_t P[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) P[j] = planes[((uint32_t)(rec >> (16 + 12 * j)) & 0xFFFu) + (uint32_t)j];
            live = sliced_table((uint32_t)rec & 0xFFFFu, P[0], P[1], P[2], P[3]) & vrows;
            if (LOWER) live &= planes[group_msob<Wp>(h.g_mask + (g0 + lane) * Wp)];
            live_method = live;  // the method's lookups, before the part filters answer some
            if (uni_mask) {
                // the part shared by the whole wave, through this group's flips
                const uint32_t q = uni_part ^ h.g_part[g0 + lane];
                const uint32_t lo = q & 0xFFFFu, hi = q >> 16;
                const bool lo_ok = !(uni_mask & 0xFFFFu) || ((pf[lo >> 5] >> (lo & 31u)) & 1u);
                const bool hi_ok = !(uni_mask >> 16) || ((pf[kPartWords / 2 + (hi >> 5)] >> (hi & 31u)) & 1u);
                if (!(lo_ok && hi_ok)) live = 0ull;
            }
        }
        uint64_t todo = __ballot(live != 0ull);  // groups live for some row of the wave
        live = wave_transpose64(live, lane);
        uint32_t mlo = (uint32_t)live, mhi = (uint32_t)(live >> 32);
        if (probes) *probes += (unsigned long long)__popcll(live_method);
        __syncthreads();
        if (filter_first && lockstep) {
            // phase 1, wave-uniform groups: bit k of occ / occn is for the wave's k-th live group,
            // whose chunk index is clist[k]
            uint8_t *clist = lds.clist[threadIdx.x >> 6];
            {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(todo >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)todo, 0u));
                if ((todo >> lane) & 1ull) clist[below] = (uint8_t)lane;
            }
            uint64_t occ = 0, occn = 0;
            for (int k0 = 0; todo; k0 += kOccBatch) {
                int c[kOccBatch];
#pragma unroll
                for (int b = 0; b < kOccBatch; ++b) {
                    c[b] = todo ? (int)__builtin_ctzll(todo) : -1;
                    todo &= todo - 1ull;
                }
                uint32_t po = 0, pn = 0;
                if (pf) {
                    // part filters instead of occupancy bits (see part_occupancy)
#pragma unroll
                    for (int b = 0; b < kOccBatch; ++b) {
                        const uint32_t a = c[b] >= 0 ? (uint32_t)(live >> (c[b] & (kChunk - 1))) & 1u : 0u;
                        const uint32_t t = a && part_pass(pf, prow ^ lds.gpart[c[b] & (kChunk - 1)]) ? 1u : 0u;
                        po |= t << b;
                        pn |= t << b;
                    }
                    occ |= (uint64_t)po << k0;
                    occn |= (uint64_t)pn << k0;
                    continue;
                }
                uint32_t pos[kOccBatch], word[kOccBatch];
#pragma unroll
                for (int b = 0; b < kOccBatch; ++b) {
                    pos[b] = (uint32_t)(hrow ^ lds.u.t.hash[c[b] & (kChunk - 1)]) & s.cmask;
                    word[b] = c[b] >= 0 ? s.bitmap[pos[b] >> 5] : 0u;  // uniform condition
                }
#pragma unroll
                for (int b = 0; b < kOccBatch; ++b) {
                    // a: the lane's row has the group live; t: bit 0 = home slot occupied,
                    // bit 1 = next slot occupied (or in the next bitmap word, so unknown).
                    // Past the end of the list (c < 0) the word is 0, so bit 0 of t is 0.
                    const uint32_t a = (uint32_t)(live >> (c[b] & (kChunk - 1))) & 1u;
                    const uint32_t t = __builtin_amdgcn_alignbit(1u, word[b], pos[b] & 31u);
                    po |= (t & a) << b;
                    pn |= ((t >> 1) & t & a) << b;
                }
                occ |= (uint64_t)po << k0;
                occn |= (uint64_t)pn << k0;
            }
            // phase 2: the slots of the occupied home slots, lowest group first
            while (__any(occ != 0ull)) {
                int c[kSB];
                bool act[kSB], nxt[kSB];
#pragma unroll
                for (int b = 0; b < kSB; ++b) {
                    const int k = occ ? (int)__builtin_ctzll(occ) : -1;
                    occ &= occ - 1ull;
                    act[b] = k >= 0;
                    c[b] = act[b] ? (int)clist[k] : 0;
                    nxt[b] = act[b] && ((occn >> k) & 1ull);
                }
                resolve_groups<Wp, kSB, PM>(s, h, lds, key, hrow, prow, pf, pr, hr, planes, lane, c, act, nxt, on_hit);
            }
            continue;
        }
        if (filter_first) {
            // phase 1: occupancy bits of the live groups' home slots (and of the slot after)
            constexpr int kOB = PM ? kOccBatchPM : kOccBatch;
            uint64_t occ = 0, occn = 0;
            uint64_t rem = live;
            while (__any(rem != 0ull)) {
                int c[kOB];
                bool act[kOB];
#pragma unroll
                for (int b = 0; b < kOB; ++b) {
                    c[b] = rem ? (int)__builtin_ctzll(rem) : -1;
                    rem &= rem - 1ull;
                    act[b] = c[b] >= 0;
                }
                if (pf)
                    part_occupancy<kOB>(pf, lds.gpart, prow, (uni_mask >> 16) != 0u, c, act, occ, occn);
                else
                    occupancy<kOB>(s, lds.u.t.hash, hrow, c, act, occ, occn);
            }
            if constexpr (PM) {
                // phase 2: the columns of the groups that passed, lowest group first
                pm_phase2<Wp, kSB>(s, h, lds, key, prow, pf, pr, hr, occ, on_hit);
                continue;
            }
            // phase 2: the slots of the occupied home slots, lowest group first
            while (__any(occ != 0ull)) {
                int c[kSB];
                bool act[kSB], nxt[kSB];
#pragma unroll
                for (int b = 0; b < kSB; ++b) {
                    c[b] = occ ? (int)__builtin_ctzll(occ) : -1;
                    occ &= occ - 1ull;
                    act[b] = c[b] >= 0;
                    nxt[b] = act[b] && ((occn >> c[b]) & 1ull);
                }
                resolve_groups<Wp, kSB, PM>(s, h, lds, key, hrow, prow, pf, pr, hr, planes, lane, c, act, nxt, on_hit);
            }
            continue;
        }
        if (lockstep) {
            while (todo) {
                int c[kLockBatch];
                bool act[kLockBatch];
#pragma unroll
                for (int b = 0; b < kLockBatch; ++b) {
                    c[b] = todo ? (int)__builtin_ctzll(todo) : -1;
                    todo &= todo - 1ull;
                    act[b] = c[b] >= 0 && ((live >> c[b]) & 1ull);
                }
                probe_groups<Wp, kLockBatch, PM>(s, h, lds, key, hrow, prow, pf, pr, hr, planes, lane, c, act, on_hit);
            }
            continue;
        }
        // probe: each lane pops its own live groups, kProbeBatch at a time
        while (true) {
            int c[kProbeBatch];
            bool anyc = false;
#pragma unroll
            for (int b = 0; b < kProbeBatch; ++b) {
                c[b] = pop_group(mlo, mhi);
                anyc |= c[b] >= 0;
            }
            if (!__any(anyc)) break;
            bool act[kProbeBatch];
#pragma unroll
            for (int b = 0; b < kProbeBatch; ++b) act[b] = c[b] >= 0;
            probe_groups<Wp, kProbeBatch, PM>(s, h, lds, key, hrow, prow, pf, pr, hr, planes, lane, c, act, on_hit);
        }
    }
}

}  // namespace qsd
