// Bit-set subspace on the device: sort + deduplicate to the canonical index, GF(2)-linear
// hashing and an open-addressing table with an occupancy bitmap (Methods, Subspace data
// structure; Lower / upper triangle evaluation for the integer order).
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.h"
#include "device.h"

namespace qsd {
namespace {

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;  // 2048

// ------------------------------------------------------------------ exclusive scan (int64)

// Blocked per-thread sums, wave scan with shuffles, cross-wave scan through LDS.
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *total) {
    __shared__ int64_t wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wave) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int64_t *__restrict__ in, int64_t *__restrict__ out,
                                                       int64_t n, int64_t *__restrict__ tile_sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int64_t total;
    int64_t off = block_exclusive_scan(s, &total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = off;
        off += v[k];
    }
    if (threadIdx.x == 0 && tile_sums) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int64_t *__restrict__ out, int64_t n,
                                                     const int64_t *__restrict__ tile_offs) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int64_t add = tile_offs[blockIdx.x];
    for (int k = threadIdx.x; k < kScanTile; k += kBlock)
        if (base + k < n) out[base + k] += add;
}

// ------------------------------------------------------------------------ ingest

// Row-major [n][W] -> word planes [Wp][n] (padding words zero) and per-word OR / AND.
__global__ __launch_bounds__(kBlock) void k_ingest(const uint64_t *__restrict__ in, int64_t n, int W, int Wp,
                                                   uint64_t *__restrict__ planes, unsigned long long *__restrict__ or_and) {
    __shared__ unsigned long long s_or[kMaxWords], s_and[kMaxWords];
    if (threadIdx.x < kMaxWords) {
        s_or[threadIdx.x] = 0ull;
        s_and[threadIdx.x] = ~0ull;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int w = 0; w < Wp; ++w) {
        uint64_t v = 0, o = 0, a = ~0ull;
        if (i < n) {
            v = w < W ? in[i * W + w] : 0ull;
            planes[(int64_t)w * n + i] = v;
            o = v;
            a = v;
        }
        // wave reduce
        for (int d = 32; d >= 1; d >>= 1) {
            o |= __shfl_xor(o, d, 64);
            a &= __shfl_xor(a, d, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicOr(&s_or[w], (unsigned long long)o);
            atomicAnd(&s_and[w], (unsigned long long)a);
        }
    }
    __syncthreads();
    if (threadIdx.x < Wp) {
        atomicOr(&or_and[threadIdx.x], s_or[threadIdx.x]);
        atomicAnd(&or_and[kMaxWords + threadIdx.x], s_and[threadIdx.x]);
    }
}

// --------------------------------------------------------------- LSD radix sort (8-bit)
constexpr int kRsItems = 8;
constexpr int kRsTile = kBlock * kRsItems;  // 2048 keys, 512 per wave

__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint64_t *__restrict__ plane, int64_t n, int shift,
                                                    int64_t *__restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(plane[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one digit pass.  Each wave ranks its 512 keys in order, 64 at a time:
// lanes with the same digit are found with 8 ballots; the first of them advances the
// wave's running count for that digit.
template <int Wp>
__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst,
                                                       int64_t n, int word, int shift,
                                                       const int64_t *__restrict__ offs, int64_t nblocks) {
    __shared__ uint32_t wcnt[kBlock / 64][256];
    __shared__ int64_t gbase[256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < (kBlock / 64) * 256; k += kBlock) (&wcnt[0][0])[k] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)wave * (kRsTile / (kBlock / 64));
    uint32_t rank[kRsItems];
    uint32_t dig[kRsItems];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int c = 0; c < kRsItems; ++c) {
        const int64_t i = base + (int64_t)c * 64 + lane;
        const bool valid = i < n;
        const uint32_t d = valid ? (uint32_t)((src[(int64_t)word * n + i] >> shift) & 255u) : 0u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            m &= bit ? bal : ~bal;
        }
        const uint32_t prior = valid ? wcnt[wave][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        const int leader = m ? __builtin_ctzll(m) : 64;
        if (valid && lane == leader) wcnt[wave][d] = prior + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
        rank[c] = prior + (uint32_t)__popcll(m & lt);
        dig[c] = d;
    }
    __syncthreads();
    {
        const int d = threadIdx.x;  // kBlock == 256 digits
        uint32_t run = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            uint32_t c = wcnt[w][d];
            wcnt[w][d] = run;
            run += c;
        }
        gbase[d] = offs[(int64_t)d * nblocks + blockIdx.x];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kRsItems; ++c) {
        const int64_t i = base + (int64_t)c * 64 + lane;
        if (i < n) {
            const int64_t o = gbase[dig[c]] + wcnt[wave][dig[c]] + rank[c];
#pragma unroll
            for (int w = 0; w < Wp; ++w) dst[(int64_t)w * n + o] = src[(int64_t)w * n + i];
        }
    }
}

// ------------------------------------------------------------------------ unique

template <int Wp>
__global__ __launch_bounds__(kBlock) void k_unique_flags(const uint64_t *__restrict__ keys, int64_t n,
                                                         int64_t *__restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int64_t f = 1;
    if (i > 0) {
        bool same = true;
#pragma unroll
        for (int w = 0; w < Wp; ++w) same &= keys[(int64_t)w * n + i] == keys[(int64_t)w * n + i - 1];
        f = same ? 0 : 1;
    }
    flags[i] = f;
}

template <int Wp>
__global__ __launch_bounds__(kBlock) void k_compact(const uint64_t *__restrict__ keys, int64_t n,
                                                    const int64_t *__restrict__ flags, const int64_t *__restrict__ pos,
                                                    uint64_t *__restrict__ out, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n || !flags[i]) return;
#pragma unroll
    for (int w = 0; w < Wp; ++w) out[(int64_t)w * N + pos[i]] = keys[(int64_t)w * n + i];
}

// -------------------------------------------------------------------------- hash

template <int Wp>
__device__ __forceinline__ uint64_t tab_hash(const uint64_t (&k)[Wp], const uint64_t *__restrict__ ztab) {
    uint64_t h = 0;
#pragma unroll
    for (int w = 0; w < Wp; ++w)
#pragma unroll
        for (int c = 0; c < 8; ++c) h ^= ztab[(w * 8 + c) * 256 + ((k[w] >> (8 * c)) & 255u)];
    return h;
}

template <int Wp>
__global__ __launch_bounds__(kBlock) void k_hash_insert(SubView s, uint64_t *__restrict__ slots,
                                                        uint32_t *__restrict__ bitmap, uint64_t *__restrict__ hkey,
                                                        const uint64_t *__restrict__ ztab) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.N) return;
    uint64_t k[Wp];
#pragma unroll
    for (int w = 0; w < Wp; ++w) k[w] = s.keys[(int64_t)w * s.N + i];
    const uint64_t h = tab_hash<Wp>(k, ztab);
    hkey[i] = h;
    const unsigned long long base = ((unsigned long long)(h >> 32) << 32) | (unsigned long long)(uint32_t)i;
    uint32_t pos = (uint32_t)h & s.cmask;
    for (uint32_t step = 0; step <= s.cmask; ++step) {
        const unsigned long long val =
            s.exact ? (base | ((unsigned long long)(step < 63u ? step : 63u) << kExactIdxBits)) : base;
        unsigned long long prev = atomicCAS((unsigned long long *)&slots[pos], ~0ull, val);
        if (prev == ~0ull) {
            atomicOr(&bitmap[pos >> 5], 1u << (pos & 31));
            return;
        }
        pos = (pos + 1) & s.cmask;
    }
}

template <int Wp>
__global__ __launch_bounds__(kBlock) void k_lookup(SubView s, const uint64_t *__restrict__ q, int64_t n, int W,
                                                   uint64_t last_invalid, const uint64_t *__restrict__ ztab,
                                                   int64_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    uint64_t k[Wp];
#pragma unroll
    for (int w = 0; w < Wp; ++w) k[w] = w < W ? q[i * W + w] : 0ull;
    if (k[W - 1] & last_invalid) {
        out[i] = -1;
        return;
    }
    out[i] = probe<Wp>(s, tab_hash<Wp>(k, ztab), k);
}

__global__ __launch_bounds__(kBlock) void k_probe_len(SubView s, unsigned long long *__restrict__ acc) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    unsigned long long len = 0;
    if (i < s.N) {
        const uint64_t h = s.hkey[i];
        uint32_t pos = (uint32_t)h & s.cmask;
        while (true) {
            ++len;
            if (slot_index(s, s.slots[pos]) == (uint32_t)i) break;
            pos = (pos + 1) & s.cmask;
        }
    }
    unsigned long long sum = len, mx = len;
    for (int d = 32; d >= 1; d >>= 1) {
        sum += __shfl_xor(sum, d, 64);
        unsigned long long o = __shfl_xor(mx, d, 64);
        mx = o > mx ? o : mx;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&acc[0], sum);
        atomicMax(&acc[1], mx);
    }
}

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

inline unsigned grid_for(int64_t n, int per_block) { return (unsigned)((n + per_block - 1) / per_block); }

// ------------------------------------------------------------------- slot order of the rows

__global__ __launch_bounds__(kBlock) void k_word_counts(const uint32_t *__restrict__ bitmap, int64_t nw,
                                                        int64_t *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < nw) cnt[i] = __popc(bitmap[i]);
}

// order[base[i] + k] = index held by the k-th occupied slot of bitmap word i.  Every string
// occupies exactly one slot, so the bitmap holds N set bits and base[i] + popc(word i) <= N.
__global__ __launch_bounds__(kBlock) void k_slot_order(const uint32_t *__restrict__ bitmap,
                                                       const uint64_t *__restrict__ slots, int64_t nw,
                                                       const int64_t *__restrict__ base, uint32_t exact,
                                                       uint32_t *__restrict__ order) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nw) return;
    uint32_t w = bitmap[i];
    int64_t o = base[i];
    while (w) {
        const int b = __builtin_ctz(w);
        w &= w - 1u;
        const uint64_t slot = slots[i * 32 + b];
        order[o++] = exact ? ((uint32_t)slot & kExactIdxMask) : (uint32_t)slot;
    }
}

__global__ __launch_bounds__(kBlock) void k_gather_rows(const uint64_t *__restrict__ keys,
                                                        const uint64_t *__restrict__ hkey,
                                                        const uint32_t *__restrict__ pkey,
                                                        const uint32_t *__restrict__ order, int64_t N, int Wp,
                                                        uint64_t *__restrict__ okeys, uint64_t *__restrict__ ohkey,
                                                        uint32_t *__restrict__ opkey) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= N) return;
    const int64_t r = order[k];
    for (int w = 0; w < Wp; ++w) okeys[(int64_t)w * N + k] = keys[(int64_t)w * N + r];
    ohkey[k] = hkey[r];
    if (pkey) opkey[k] = pkey[r];
}

// Packed part indices of every row (byte tabulation of the part words) and both part filters:
// bit (low index) of the low filter and bit (high index) of the high filter, for every row.
template <int Wp>
__global__ __launch_bounds__(kBlock) void k_part_keys(const uint64_t *__restrict__ keys, int64_t N,
                                                      const uint32_t *__restrict__ ptab, uint32_t *__restrict__ pkey,
                                                      uint32_t *__restrict__ pfilt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    uint32_t p = 0;
#pragma unroll
    for (int w = 0; w < Wp; ++w) {
        const uint64_t k = keys[(int64_t)w * N + i];
#pragma unroll
        for (int c = 0; c < 8; ++c) p ^= ptab[(w * 8 + c) * 256 + ((k >> (8 * c)) & 255u)];
    }
    pkey[i] = p;
    atomicOr(&pfilt[(p & 0xFFFFu) >> 5], 1u << (p & 31u));
    atomicOr(&pfilt[kPartWords / 2 + (p >> 21)], 1u << ((p >> 16) & 31u));
}

// The rows listed in the order of their slots (a compaction of the occupancy bitmap), with
// their keys and hashes in that order.  A run of consecutive entries holds rows whose home slots
// share a stretch of the table, so for any group their columns b ^ M_g, whose hashes are
// h(b) ^ h(M_g), share a stretch too.
int build_order(const qsd_subspace *sub, const uint64_t *hkey, const uint32_t *pkey, int64_t C, bool exact,
                const uint64_t *slots, const uint32_t *bitmap, SlotRows *out, hipStream_t st) {
    const int64_t N = sub->N, nw = C / 32;
    int64_t *base = nullptr;
    SlotRows o;
    QSD_TRY(dev_alloc(&base, nw));
    int rc = dev_alloc(&o.order, N);
    if (rc == QSD_OK) rc = dev_alloc(&o.keys, (size_t)sub->Wp * N);
    if (rc == QSD_OK) rc = dev_alloc(&o.hkey, N);
    if (rc == QSD_OK && pkey) rc = dev_alloc(&o.pkey, N);
    if (rc == QSD_OK) {
        k_word_counts<<<grid_for(nw, kBlock), kBlock, 0, st>>>(bitmap, nw, base);
        rc = exclusive_scan_i64(base, base, nw, st);
    }
    if (rc == QSD_OK) {
        k_slot_order<<<grid_for(nw, kBlock), kBlock, 0, st>>>(bitmap, slots, nw, base, exact ? 1u : 0u, o.order);
        k_gather_rows<<<grid_for(N, kBlock), kBlock, 0, st>>>(sub->keys, hkey, pkey, o.order, N, sub->Wp, o.keys,
                                                              o.hkey, o.pkey);
        if (hipStreamSynchronize(st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "slot order failed: %s", hipGetErrorString(hipGetLastError()));
    }
    dev_free(base);
    if (rc != QSD_OK) {
        free_rows(o);
        return rc;
    }
    *out = o;
    return QSD_OK;
}

template <int Wp>
int build_impl(qsd_subspace *sub, const uint64_t *d_bits, int64_t n_in, uint32_t flags, double max_load,
               hipStream_t st) {
    const int W = sub->W;
    uint64_t *planes = nullptr, *tmp = nullptr;
    unsigned long long *or_and = nullptr;
    QSD_TRY(dev_alloc(&planes, (size_t)Wp * n_in));
    int rc = QSD_OK;
    auto cleanup = [&]() {
        dev_free(planes);
        dev_free(tmp);
        dev_free(or_and);
    };
    do {
        if ((rc = dev_alloc(&or_and, 2 * kMaxWords)) != QSD_OK) break;
        {
            std::vector<unsigned long long> init(2 * kMaxWords);
            for (int w = 0; w < kMaxWords; ++w) {
                init[w] = 0ull;
                init[kMaxWords + w] = ~0ull;
            }
            if (hipMemcpyAsync(or_and, init.data(), init.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess) {
                rc = fail(QSD_ERR_HIP, "copy failed");
                break;
            }
        }
        k_ingest<<<grid_for(n_in, kBlock), kBlock, 0, st>>>(d_bits, n_in, W, Wp, planes, or_and);
        std::vector<unsigned long long> oa(2 * kMaxWords);
        if (hipMemcpyAsync(oa.data(), or_and, oa.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(QSD_ERR_HIP, "ingest failed: %s", hipGetErrorString(hipGetLastError()));
            break;
        }
        const int nb = sub->n_qubits - 64 * (W - 1);
        const uint64_t valid_last = nb >= 64 ? ~0ull : ((1ull << nb) - 1ull);
        if (oa[W - 1] & ~valid_last) {
            rc = fail(QSD_ERR_INVALID_ARG, "a bit-string has a bit set at a position >= n_qubits (%d)", sub->n_qubits);
            break;
        }
        if ((rc = dev_alloc(&tmp, (size_t)Wp * n_in)) != QSD_OK) break;
        uint64_t *src = planes, *dst = tmp;
        if (!(flags & QSD_SUB_ASSUME_SORTED_UNIQUE)) {
            const int64_t nblocks = (n_in + kRsTile - 1) / kRsTile;
            int64_t *hist = nullptr;
            if ((rc = dev_alloc(&hist, (size_t)256 * nblocks)) != QSD_OK) break;
            for (int w = 0; w < W && rc == QSD_OK; ++w) {
                const uint64_t varies = oa[w] ^ oa[kMaxWords + w];
                for (int d = 0; d < 8; ++d) {
                    if (!((varies >> (8 * d)) & 255u)) continue;  // digit equal in every key
                    k_rs_hist<<<(unsigned)nblocks, kBlock, 0, st>>>(src + (int64_t)w * n_in, n_in, 8 * d, hist, nblocks);
                    if ((rc = exclusive_scan_i64(hist, hist, 256 * nblocks, st)) != QSD_OK) break;
                    k_rs_scatter<Wp><<<(unsigned)nblocks, kBlock, 0, st>>>(src, dst, n_in, w, 8 * d, hist, nblocks);
                    std::swap(src, dst);
                }
            }
            dev_free(hist);
            if (rc != QSD_OK) break;
        }
        // deduplicate
        int64_t *fl = nullptr, *pos = nullptr;
        if ((rc = dev_alloc(&fl, n_in)) != QSD_OK) break;
        if ((rc = dev_alloc(&pos, n_in)) != QSD_OK) {
            dev_free(fl);
            break;
        }
        k_unique_flags<Wp><<<grid_for(n_in, kBlock), kBlock, 0, st>>>(src, n_in, fl);
        rc = exclusive_scan_i64(fl, pos, n_in, st);
        int64_t last[2] = {0, 0};
        if (rc == QSD_OK) {
            if (hipMemcpyAsync(&last[0], pos + n_in - 1, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipMemcpyAsync(&last[1], fl + n_in - 1, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = fail(QSD_ERR_HIP, "sort failed: %s", hipGetErrorString(hipGetLastError()));
        }
        const int64_t N = last[0] + last[1];
        if (rc == QSD_OK && N >= 0xFFFFFFFFll) rc = fail(QSD_ERR_CAPACITY, "%lld unique strings exceed 2^32-2", (long long)N);
        if (rc == QSD_OK) rc = dev_alloc(&sub->keys, (size_t)Wp * N);
        if (rc == QSD_OK) k_compact<Wp><<<grid_for(n_in, kBlock), kBlock, 0, st>>>(src, n_in, fl, pos, sub->keys, N);
        if (rc == QSD_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(QSD_ERR_HIP, "compact failed");
        dev_free(fl);
        dev_free(pos);
        if (rc != QSD_OK) break;
        sub->N = N;
        // hash table
        int64_t C = 64;
        while ((double)N / (double)C > max_load) C <<= 1;
        if (C > (1ll << 32)) {
            rc = fail(QSD_ERR_CAPACITY, "hash table would exceed 2^32 slots");
            break;
        }
        sub->C = C;
        hash_words(sub->n_qubits, sub->z);
        sub->exact = exact_tags_ok(sub->z, sub->W, N, C);
        std::vector<uint64_t> tab;
        hash_byte_tables(Wp, sub->z, tab);
        if ((rc = dev_alloc(&sub->ztab, tab.size())) != QSD_OK) break;
        if ((rc = dev_alloc(&sub->slots, C)) != QSD_OK) break;
        if ((rc = dev_alloc(&sub->bitmap, C / 32)) != QSD_OK) break;
        if ((rc = dev_alloc(&sub->hkey, N)) != QSD_OK) break;
        if (hipMemcpyAsync(sub->ztab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess) {
            rc = fail(QSD_ERR_HIP, "copy failed");
            break;
        }
        k_fill_u64<<<1024, kBlock, 0, st>>>(sub->slots, C, ~0ull);
        k_fill_u32<<<256, kBlock, 0, st>>>(sub->bitmap, C / 32, 0u);
        SubView v{sub->keys, sub->hkey, sub->slots, sub->bitmap, N, (uint32_t)(C - 1), sub->exact ? 1u : 0u};
        k_hash_insert<Wp><<<grid_for(N, kBlock), kBlock, 0, st>>>(v, sub->slots, sub->bitmap, sub->hkey, sub->ztab);
        if (hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(QSD_ERR_HIP, "hash build failed: %s", hipGetErrorString(hipGetLastError()));
            break;
        }
        rc = build_order(sub, sub->hkey, nullptr, C, sub->exact, sub->slots, sub->bitmap, &sub->rows, st);
    } while (0);
    cleanup();
    return rc;
}

void free_sub(qsd_subspace *s) {
    if (!s) return;
    dev_free(s->keys);
    dev_free(s->hkey);
    dev_free(s->slots);
    dev_free(s->bitmap);
    dev_free(s->ztab);
    dev_free(s->pfilt);
    dev_free(s->pkey);
    dev_free(s->prank);
    free_rows(s->rows);
    delete s;
}

SubView view_of(const qsd_subspace *s) {
    return SubView{s->keys,       s->hkey,      s->slots,     s->bitmap, s->N, (uint32_t)(s->C - 1),
                   s->exact ? 1u : 0u, s->rows.order, s->rows.keys, s->rows.hkey, s->pfilt, s->pkey,
                   s->rows.pkey, s->prank,  s->pna};
}

}  // namespace

int exclusive_scan_i64(const int64_t *d_in, int64_t *d_out, int64_t n, hipStream_t st) {
    if (n <= 0) return QSD_OK;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 1) {
        k_scan_tiles<<<1, kBlock, 0, st>>>(d_in, d_out, n, nullptr);
        return hipGetLastError() == hipSuccess ? QSD_OK : fail(QSD_ERR_HIP, "scan launch failed");
    }
    int64_t *sums = nullptr;
    QSD_TRY(dev_alloc(&sums, tiles));
    k_scan_tiles<<<(unsigned)tiles, kBlock, 0, st>>>(d_in, d_out, n, sums);
    int rc = exclusive_scan_i64(sums, sums, tiles, st);
    if (rc == QSD_OK) k_scan_add<<<(unsigned)tiles, kBlock, 0, st>>>(d_out, n, sums);
    // the scratch must outlive the kernels that use it
    if (hipStreamSynchronize(st) != hipSuccess) rc = fail(QSD_ERR_HIP, "scan failed");
    dev_free(sums);
    return rc;
}

}  // namespace qsd

namespace qsd {
int rehash_split(qsd_subspace *sub, int split, hipStream_t st);
}

using namespace qsd;

extern "C" int qsd_subspace_build(const uint64_t *d_bits, int64_t n_in, int32_t n_qubits, uint32_t flags,
                                  double max_load, const qsd_allocator *alloc, void *stream, qsd_subspace **out) {
    clear_error();
    if (!out) return fail(QSD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!d_bits || n_in < 1) return fail(QSD_ERR_INVALID_ARG, "empty subspace (n_in = %lld)", (long long)n_in);
    if (n_qubits < 1) return fail(QSD_ERR_INVALID_ARG, "n_qubits must be >= 1");
    if (n_qubits > kMaxWords * 64) return fail(QSD_ERR_UNSUPPORTED, "n_qubits > %d", kMaxWords * 64);
    if (max_load == 0.0) max_load = 0.125;
    if (!(max_load > 0.0 && max_load <= 0.5)) return fail(QSD_ERR_INVALID_ARG, "max_load must be in (0, 0.5]");
    auto *sub = new (std::nothrow) qsd_subspace();
    if (!sub) return fail(QSD_ERR_OUT_OF_MEMORY, "host allocation failed");
    sub->alloc = keep_allocator(alloc);
    sub->stream = stream;
    AllocScope scope(&sub->alloc, stream);
    sub->n_qubits = n_qubits;
    sub->W = (n_qubits + 63) / 64;
    sub->Wp = padded_words(n_qubits);
    hipStream_t st = (hipStream_t)stream;
    int rc;
    switch (sub->Wp) {
        case 1: rc = build_impl<1>(sub, d_bits, n_in, flags, max_load, st); break;
        case 2: rc = build_impl<2>(sub, d_bits, n_in, flags, max_load, st); break;
        case 4: rc = build_impl<4>(sub, d_bits, n_in, flags, max_load, st); break;
        case 8: rc = build_impl<8>(sub, d_bits, n_in, flags, max_load, st); break;
        case 16: rc = build_impl<16>(sub, d_bits, n_in, flags, max_load, st); break;
        default: rc = fail(QSD_ERR_UNSUPPORTED, "unsupported width");
    }
    // a string of at most 32 qubits split in halves: when the subspace is the product of its
    // halves (an alpha x beta product), keep the part filters and the product map
    if (rc == QSD_OK && n_qubits >= 2 && n_qubits <= 32) {
        rc = rehash_split(sub, n_qubits / 2, st);
        if (rc == QSD_OK && !sub->prank) rc = rehash_split(sub, 0, st);
    }
    if (rc != QSD_OK) {
        free_sub(sub);
        return rc;
    }
    *out = sub;
    return QSD_OK;
}

namespace qsd {
namespace {

// Rebuilds, as needed, the table for C slots, the part filters for the split qubit (0 = none)
// and the slot order of the rows; the subspace keeps its old state until all of them are built.
// Operators bound to the subspace get their groups' part indices anew.  The hash words never
// change here, so row and group hashes stay valid (`new_words` keeps the path that rebuilds
// them for a table built under other words).
template <int Wp>
int rehash_impl(qsd_subspace *sub, int64_t C, int split, hipStream_t st) {
    const bool new_words = false;
    const bool new_table = new_words || C != sub->C;
    std::vector<uint64_t> z = sub->z;
    uint64_t *slots = sub->slots, *ztab = sub->ztab, *hkey = sub->hkey;
    uint32_t *bitmap = sub->bitmap;
    bool exact = sub->exact;
    uint32_t *pfilt = nullptr, *pkey = nullptr, *ptab_d = nullptr;
    uint16_t *prank = nullptr;
    uint32_t pna = 0;
    std::vector<uint32_t> pz;
    std::vector<uint64_t> tab;
    int rc = QSD_OK;
    if (new_words) {
        ztab = nullptr;
        hkey = nullptr;
        hash_words(sub->n_qubits, z);
        hash_byte_tables(Wp, z, tab);
        rc = dev_alloc(&ztab, tab.size());
        if (rc == QSD_OK) rc = dev_alloc(&hkey, sub->N);
        if (rc == QSD_OK && hipMemcpyAsync(ztab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "copy failed");
    }
    if (rc == QSD_OK && new_table) {
        slots = nullptr;
        bitmap = nullptr;
        exact = exact_tags_ok(z, sub->W, sub->N, C);
        rc = dev_alloc(&slots, C);
        if (rc == QSD_OK) rc = dev_alloc(&bitmap, C / 32);
        if (rc == QSD_OK) {
            k_fill_u64<<<1024, kBlock, 0, st>>>(slots, C, ~0ull);
            k_fill_u32<<<256, kBlock, 0, st>>>(bitmap, C / 32, 0u);
            // writes the row hashes (the same values when the words did not change)
            SubView v{sub->keys, hkey, slots, bitmap, sub->N, (uint32_t)(C - 1), exact ? 1u : 0u};
            k_hash_insert<Wp><<<grid_for(sub->N, kBlock), kBlock, 0, st>>>(v, slots, bitmap, hkey, ztab);
        }
    }
    if (rc == QSD_OK && split > 0) {
        part_words(sub->n_qubits, split, pz);
        std::vector<uint32_t> ptab((size_t)Wp * 8 * 256, 0u);
        for (int c = 0; c < Wp * 8; ++c)
            for (int v = 0; v < 256; ++v)
                for (int b = 0; b < 8; ++b)
                    if ((v >> b & 1) && 8 * c + b < sub->n_qubits) ptab[(size_t)c * 256 + v] ^= pz[8 * c + b];
        rc = dev_alloc(&pfilt, kPartWords);
        if (rc == QSD_OK) rc = dev_alloc(&pkey, sub->N);
        if (rc == QSD_OK) rc = dev_alloc(&ptab_d, ptab.size());
        if (rc == QSD_OK &&
            hipMemcpyAsync(ptab_d, ptab.data(), ptab.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "copy failed");
        if (rc == QSD_OK) {
            k_fill_u32<<<16, kBlock, 0, st>>>(pfilt, kPartWords, 0u);
            k_part_keys<Wp><<<grid_for(sub->N, kBlock), kBlock, 0, st>>>(sub->keys, sub->N, ptab_d, pkey, pfilt);
        }
        // the host tables must outlive their copies
        if (rc == QSD_OK && hipStreamSynchronize(st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "part filter build failed: %s", hipGetErrorString(hipGetLastError()));
        // product map: with parts of at most 16 qubits the filters are exact (a part's index is
        // its own bits), and the subspace is the product of its parts exactly when their counts
        // multiply to N (every row is one (low, high) pair, and rows are distinct)
        if (rc == QSD_OK && split <= 16 && sub->n_qubits - split <= 16) {
            std::vector<uint32_t> hf(kPartWords);
            if (hipMemcpyAsync(hf.data(), pfilt, kPartWords * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = fail(QSD_ERR_HIP, "copy failed");
            std::vector<uint16_t> pre(kPartWords);
            uint64_t cnt[2] = {0, 0};
            for (int f = 0; f < 2 && rc == QSD_OK; ++f)
                for (int w = 0; w < kPartWords / 2; ++w) {
                    pre[(size_t)f * (kPartWords / 2) + w] = (uint16_t)cnt[f];
                    cnt[f] += (uint64_t)__builtin_popcount(hf[(size_t)f * (kPartWords / 2) + w]);
                }
            if (rc == QSD_OK && cnt[0] * cnt[1] == (uint64_t)sub->N) {
                rc = dev_alloc(&prank, kPartWords);
                if (rc == QSD_OK &&
                    (hipMemcpyAsync(prank, pre.data(), kPartWords * 2, hipMemcpyHostToDevice, st) != hipSuccess ||
                     hipStreamSynchronize(st) != hipSuccess))
                    rc = fail(QSD_ERR_HIP, "copy failed");
                pna = (uint32_t)cnt[0];
            }
        }
    }
    if (rc == QSD_OK && hipStreamSynchronize(st) != hipSuccess)
        rc = fail(QSD_ERR_HIP, "hash rebuild failed: %s", hipGetErrorString(hipGetLastError()));
    SlotRows rows;
    if (rc == QSD_OK) rc = build_order(sub, hkey, pkey, C, exact, slots, bitmap, &rows, st);
    // the bound operators' group hashes (new words) and part indices (part filters)
    const size_t nb = sub->bound.size();
    std::vector<uint64_t *> ghash(nb, nullptr);
    std::vector<uint32_t *> gparts(nb, nullptr);
    std::vector<std::vector<uint64_t>> gh(nb);
    std::vector<std::vector<uint32_t>> gp(nb);
    for (size_t k = 0; k < nb && rc == QSD_OK; ++k) {
        const qsd_op *op = sub->bound[k]->op;
        AllocScope hscope(&sub->bound[k]->alloc, st);
        if (new_words) {
            gh[k] = group_hashes(op, z);
            rc = dev_alloc(&ghash[k], gh[k].size());
            if (rc == QSD_OK && !gh[k].empty() &&
                hipMemcpyAsync(ghash[k], gh[k].data(), gh[k].size() * 8, hipMemcpyHostToDevice, st) != hipSuccess)
                rc = fail(QSD_ERR_HIP, "copy failed");
        }
        if (rc == QSD_OK && split > 0) {
            gp[k] = group_parts(op, pz);
            rc = dev_alloc(&gparts[k], gp[k].size());
            if (rc == QSD_OK && !gp[k].empty() &&
                hipMemcpyAsync(gparts[k], gp[k].data(), gp[k].size() * 4, hipMemcpyHostToDevice, st) != hipSuccess)
                rc = fail(QSD_ERR_HIP, "copy failed");
        }
    }
    if (rc == QSD_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(QSD_ERR_HIP, "operator update failed");
    if (rc != QSD_OK) {
        for (size_t k = 0; k < nb; ++k) {
            AllocScope hscope(&sub->bound[k]->alloc, st);
            dev_free(ghash[k]);
            dev_free(gparts[k]);
        }
        free_rows(rows);
        if (new_words) {
            dev_free(ztab);
            dev_free(hkey);
        }
        if (new_table) {
            dev_free(slots);
            dev_free(bitmap);
        }
        dev_free(pfilt);
        dev_free(pkey);
        dev_free(prank);
        dev_free(ptab_d);
        return rc;
    }
    dev_free(ptab_d);
    if (new_words) {
        dev_free(sub->ztab);
        dev_free(sub->hkey);
    }
    if (new_table) {
        dev_free(sub->slots);
        dev_free(sub->bitmap);
    }
    dev_free(sub->pfilt);
    dev_free(sub->pkey);
    dev_free(sub->prank);
    free_rows(sub->rows);
    sub->z = z;
    sub->ztab = ztab;
    sub->hkey = hkey;
    sub->slots = slots;
    sub->bitmap = bitmap;
    sub->exact = exact;
    sub->C = C;
    sub->rows = rows;
    sub->pfilt = pfilt;
    sub->pkey = pkey;
    sub->prank = prank;
    sub->pna = pna;
    sub->pz = pz;
    sub->split = split;
    for (size_t k = 0; k < nb; ++k) {
        qsd_ham *h = sub->bound[k];
        AllocScope hscope(&h->alloc, st);
        if (new_words) {
            dev_free(h->g_hash);
            h->g_hash = ghash[k];
        }
        dev_free(h->g_part);
        h->g_part = gparts[k];
    }
    return QSD_OK;
}

}  // namespace

// New part filters (split 0: none) on the current table of a one-word subspace.
int rehash_split(qsd_subspace *sub, int split, hipStream_t st) {
    return rehash_impl<1>(sub, sub->C, split, st);
}

}  // namespace qsd

extern "C" int qsd_subspace_rehash(qsd_subspace *s, double max_load, int32_t split, void *stream) {
    clear_error();
    if (!s) return fail(QSD_ERR_INVALID_ARG, "subspace is NULL");
    AllocScope scope(&s->alloc, stream);
    if (max_load == 0.0) max_load = 0.125;
    if (!(max_load > 0.0 && max_load <= 0.5)) return fail(QSD_ERR_INVALID_ARG, "max_load must be in (0, 0.5]");
    if (split < 0 || split >= s->n_qubits)
        return fail(QSD_ERR_INVALID_ARG, "split qubit %d outside [0, %d)", split, s->n_qubits);
    int64_t C = 64;
    while ((double)s->N / (double)C > max_load) C <<= 1;
    if (C > (1ll << 32)) return fail(QSD_ERR_CAPACITY, "hash table would exceed 2^32 slots");
    if (C == s->C && split == s->split) return QSD_OK;
    hipStream_t st = (hipStream_t)stream;
    switch (s->Wp) {
        case 1: return rehash_impl<1>(s, C, split, st);
        case 2: return rehash_impl<2>(s, C, split, st);
        case 4: return rehash_impl<4>(s, C, split, st);
        case 8: return rehash_impl<8>(s, C, split, st);
        case 16: return rehash_impl<16>(s, C, split, st);
    }
    return fail(QSD_ERR_UNSUPPORTED, "unsupported width");
}

extern "C" int qsd_subspace_hash_info(const qsd_subspace *s, int32_t *split, int32_t *exact, int32_t *product) {
    clear_error();
    if (!s) return fail(QSD_ERR_INVALID_ARG, "subspace is NULL");
    if (split) *split = s->split;
    if (exact) *exact = s->exact ? 1 : 0;
    if (product) *product = s->prank ? 1 : 0;
    return QSD_OK;
}

extern "C" int qsd_subspace_info(const qsd_subspace *s, int64_t *N, int32_t *n_qubits, int32_t *W, int64_t *capacity) {
    clear_error();
    if (!s) return fail(QSD_ERR_INVALID_ARG, "subspace is NULL");
    if (N) *N = s->N;
    if (n_qubits) *n_qubits = s->n_qubits;
    if (W) *W = s->W;
    if (capacity) *capacity = s->C;
    return QSD_OK;
}

namespace {
__global__ __launch_bounds__(kBlock) void k_planes_to_rows(const uint64_t *__restrict__ planes, int64_t N, int W,
                                                           uint64_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    for (int w = 0; w < W; ++w) out[i * W + w] = planes[(int64_t)w * N + i];
}
}  // namespace

namespace {
__global__ __launch_bounds__(kBlock) void k_mask_to_i64(const uint8_t *__restrict__ m, int64_t N, int64_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < N) out[i] = m[i] ? 1 : 0;
    if (i == N) out[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_select_rows(const uint64_t *__restrict__ planes, int64_t N, int W,
                                                        const uint8_t *__restrict__ m, const int64_t *__restrict__ pos,
                                                        uint64_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= N || !m[i]) return;
    for (int w = 0; w < W; ++w) out[pos[i] * W + w] = planes[(int64_t)w * N + i];
}
}  // namespace

extern "C" int qsd_subspace_select(const qsd_subspace *s, const uint8_t *d_mask, double max_load, void *stream,
                                   qsd_subspace **out) {
    clear_error();
    if (!s || !d_mask || !out) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    AllocScope scope(&s->alloc, stream);
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = s->N;
    int64_t *flag = nullptr, *pos = nullptr;
    QSD_TRY(dev_alloc(&flag, N + 1));
    int rc = dev_alloc(&pos, N + 1);
    int64_t n = 0;
    if (rc == QSD_OK) {
        k_mask_to_i64<<<grid_for(N + 1, kBlock), kBlock, 0, st>>>(d_mask, N, flag);
        rc = exclusive_scan_i64(flag, pos, N + 1, st);
    }
    if (rc == QSD_OK && (hipMemcpyAsync(&n, pos + N, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                         hipStreamSynchronize(st) != hipSuccess))
        rc = fail(QSD_ERR_HIP, "selection count failed");
    if (rc == QSD_OK && n == 0) rc = fail(QSD_ERR_INVALID_ARG, "the mask selects no string");
    uint64_t *rows = nullptr;
    if (rc == QSD_OK) rc = dev_alloc(&rows, (size_t)n * s->W);
    if (rc == QSD_OK) {
        k_select_rows<<<grid_for(N, kBlock), kBlock, 0, st>>>(s->keys, N, s->W, d_mask, pos, rows);
        // the rows stay in ascending order and distinct
        rc = qsd_subspace_build(rows, n, s->n_qubits, QSD_SUB_ASSUME_SORTED_UNIQUE, max_load, &s->alloc, stream,
                                out);
    }
    dev_free(flag);
    dev_free(pos);
    dev_free(rows);
    return rc;
}

extern "C" int qsd_subspace_keys(const qsd_subspace *s, uint64_t *d_out, void *stream) {
    clear_error();
    if (!s || !d_out) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    k_planes_to_rows<<<grid_for(s->N, kBlock), kBlock, 0, (hipStream_t)stream>>>(s->keys, s->N, s->W, d_out);
    QSD_CHECK_HIP(hipGetLastError());
    return QSD_OK;
}

extern "C" int qsd_subspace_lookup(const qsd_subspace *s, const uint64_t *d_q, int64_t n, int64_t *d_idx,
                                   void *stream) {
    clear_error();
    if (!s || (n > 0 && (!d_q || !d_idx)) || n < 0) return fail(QSD_ERR_INVALID_ARG, "bad arguments");
    if (n == 0) return QSD_OK;
    const int nb = s->n_qubits - 64 * (s->W - 1);
    const uint64_t invalid = nb >= 64 ? 0ull : ~((1ull << nb) - 1ull);
    hipStream_t st = (hipStream_t)stream;
    SubView v = view_of(s);
    const unsigned g = grid_for(n, kBlock);
    switch (s->Wp) {
        case 1: k_lookup<1><<<g, kBlock, 0, st>>>(v, d_q, n, s->W, invalid, s->ztab, d_idx); break;
        case 2: k_lookup<2><<<g, kBlock, 0, st>>>(v, d_q, n, s->W, invalid, s->ztab, d_idx); break;
        case 4: k_lookup<4><<<g, kBlock, 0, st>>>(v, d_q, n, s->W, invalid, s->ztab, d_idx); break;
        case 8: k_lookup<8><<<g, kBlock, 0, st>>>(v, d_q, n, s->W, invalid, s->ztab, d_idx); break;
        case 16: k_lookup<16><<<g, kBlock, 0, st>>>(v, d_q, n, s->W, invalid, s->ztab, d_idx); break;
    }
    QSD_CHECK_HIP(hipGetLastError());
    return QSD_OK;
}

extern "C" int qsd_subspace_probe_stats(const qsd_subspace *s, double *mean_probe, int64_t *max_probe, void *stream) {
    clear_error();
    if (!s) return fail(QSD_ERR_INVALID_ARG, "subspace is NULL");
    AllocScope scope(&s->alloc, stream);
    hipStream_t st = (hipStream_t)stream;
    unsigned long long *acc = nullptr;
    QSD_TRY(dev_alloc(&acc, 2));
    unsigned long long h[2] = {0, 0};
    int rc = QSD_OK;
    if (hipMemcpyAsync(acc, h, 16, hipMemcpyHostToDevice, st) != hipSuccess) rc = fail(QSD_ERR_HIP, "copy failed");
    if (rc == QSD_OK) {
        k_probe_len<<<grid_for(s->N, kBlock), kBlock, 0, st>>>(view_of(s), acc);
        if (hipMemcpyAsync(h, acc, 16, hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "probe stats failed");
    }
    dev_free(acc);
    if (rc != QSD_OK) return rc;
    if (mean_probe) *mean_probe = (double)h[0] / (double)s->N;
    if (max_probe) *max_probe = (int64_t)h[1];
    return QSD_OK;
}

extern "C" int qsd_subspace_destroy(qsd_subspace *s) {
    clear_error();
    if (!s) return QSD_OK;
    AllocScope scope(&s->alloc, s->stream);
    free_sub(s);
    return QSD_OK;
}
