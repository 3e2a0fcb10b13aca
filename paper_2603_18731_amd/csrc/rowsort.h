// Per-row sort of CSR entries by column, shared by the two-pass CSR build and the stored-CSR
// (lower-triangle) build: one workgroup per row, columns distinct within a row.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "engine.h"

namespace qsd {

constexpr int kSortLds = 4096;  // columns of one row (or one chunk of a longer row) held in LDS

// Writes the row's (column, value) pairs [a, a + len) of the unsorted scratch (cols, vals) to
// out_idx / out_val in ascending column order.  A row of at most kSortLds entries is ranked in
// LDS (each element counts the smaller columns).  A longer row is taken in chunks of kSortLds:
// each chunk is ranked in LDS and written sorted to the output arrays; then every element's
// final position is the sum over chunks of the number of smaller columns, found by binary
// search in the sorted chunks, and is packed into its scratch column word (column < 2^32, rank
// < 2^32); last, the pairs move to their positions.  The cost is len * kSortLds comparisons in
// LDS plus len * chunks * log2(kSortLds) searches, not len^2 reads of global memory.  `sc` is
// the caller's LDS array of kSortLds words; all threads of the workgroup must call.
template <class ET, class IT, bool CPLX>
__device__ __forceinline__ void sort_row_entries(int64_t a, int64_t len, int64_t *__restrict__ cols,
                                                 const typename C2<ET>::T *__restrict__ vals, IT *__restrict__ out_idx,
                                                 ET *__restrict__ out_val, int64_t *sc) {
    auto put = [&](int64_t pos, int64_t c, const typename C2<ET>::T &v) {
        out_idx[pos] = (IT)c;
        if (CPLX) {
            out_val[2 * pos] = v.x;
            out_val[2 * pos + 1] = v.y;
        } else {
            out_val[pos] = v.x;
        }
    };
    if (len <= kSortLds) {
        for (int64_t e = threadIdx.x; e < len; e += kBlock) sc[e] = cols[a + e];
        __syncthreads();
        for (int64_t e = threadIdx.x; e < len; e += kBlock) {
            const int64_t c = sc[e];
            int64_t rank = 0;
            for (int64_t f = 0; f < len; ++f) rank += sc[f] < c;
            put(a + rank, c, vals[a + e]);
        }
        return;
    }
    const int64_t nch = (len + kSortLds - 1) / kSortLds;
    // 1. each chunk sorted into its own stretch of the output
    for (int64_t m = 0; m < nch; ++m) {
        const int64_t c0 = m * kSortLds, cl = (len - c0) < kSortLds ? (len - c0) : kSortLds;
        __syncthreads();  // the previous chunk's LDS reads are done
        for (int64_t e = threadIdx.x; e < cl; e += kBlock) sc[e] = cols[a + c0 + e];
        __syncthreads();
        for (int64_t e = threadIdx.x; e < cl; e += kBlock) {
            const int64_t c = sc[e];
            int64_t rank = 0;
            for (int64_t f = 0; f < cl; ++f) rank += sc[f] < c;
            put(a + c0 + rank, c, vals[a + c0 + e]);
        }
    }
    __threadfence();
    __syncthreads();
    // 2. final rank = smaller columns in every sorted chunk (the own chunk included)
    for (int64_t e = threadIdx.x; e < len; e += kBlock) {
        const int64_t c = cols[a + e];
        int64_t rank = 0;
        for (int64_t m = 0; m < nch; ++m) {
            const int64_t c0 = a + m * kSortLds, cl = (len - m * kSortLds) < kSortLds ? (len - m * kSortLds) : kSortLds;
            int64_t lo = 0, hi = cl;  // first position in the chunk whose column is >= c
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if ((int64_t)out_idx[c0 + mid] < c)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            rank += lo;
        }
        cols[a + e] = (int64_t)(((uint64_t)rank << 32) | (uint64_t)(uint32_t)c);
    }
    __threadfence();
    __syncthreads();
    // 3. every pair to its position (the sorted chunks are no longer read)
    for (int64_t e = threadIdx.x; e < len; e += kBlock) {
        const uint64_t pk = (uint64_t)cols[a + e];
        put(a + (int64_t)(pk >> 32), (int64_t)(uint32_t)pk, vals[a + e]);
    }
}

}  // namespace qsd
