// SpMV of one block of 256 rows, shared by the single-operator kernel and the batched
// (serving) kernel.
#pragma once

#include "engine.h"

namespace qsd {

inline HamView ham_view(const qsd_ham *h, bool f32) {
    return HamView{h->g_mask, h->g_hash, h->g_pos,  h->g_scan, h->g_info, h->g_term0, h->g_nterm,
                   h->g_iptr, h->t_cws,  f32 ? (const void *)h->t_coef32 : (const void *)h->t_coef, h->G,
                   f32 ? 1 : 0, h->g_part, (const uint4 *)h->t_cw32};
}

inline SubView sub_view(const qsd_subspace *s) {
    return SubView{s->keys,       s->hkey,      s->slots,     s->bitmap, s->N, (uint32_t)(s->C - 1),
                   s->exact ? 1u : 0u, s->rows.order, s->rows.keys, s->rows.hkey, s->pfilt, s->pkey,
                   s->rows.pkey, s->prank,  s->pna};
}

// Row tile of workgroup b out of G.  Workgroups are dispatched round-robin over the 8 XCDs, so
// with `remap` the tiles of one XCD are made contiguous (XCD x takes the x-th eighth of the rows,
// in order): neighbouring rows, whose columns and hash probes overlap, then share one L2.
__device__ __forceinline__ int64_t tile_index(unsigned b, unsigned G, bool remap) {
    if (!remap) return b;
    const unsigned x = b & 7u, r = b >> 3, per = G >> 3, rem = G & 7u;
    return (int64_t)((x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + r);
}

// Loads the lane's row: position `row0 + lane` of the canonical order, or of the slot order
// with `by_slot` (clamped to a valid row for lanes past the end, or past `row_end` when given).
template <int Wp>
__device__ __forceinline__ int64_t load_row(const SubView &s, int64_t row0, uint64_t (&key)[Wp], uint64_t &hrow,
                                            uint32_t &prow, bool &valid, bool by_slot = false, int64_t row_end = -1) {
    const int64_t i = row0 + threadIdx.x;
    valid = i < (row_end < 0 ? s.N : row_end);
    const int64_t p = valid ? i : s.N - 1;
    if (by_slot) {
#pragma unroll
        for (int w = 0; w < Wp; ++w) key[w] = s.okeys[(int64_t)w * s.N + p];
        hrow = s.ohkey[p];
        prow = s.pfilt ? s.opkey[p] : 0u;
        return s.order[p];
    }
#pragma unroll
    for (int w = 0; w < Wp; ++w) key[w] = s.keys[(int64_t)w * s.N + p];
    hrow = s.hkey[p];
    prow = s.pfilt ? s.pkey[p] : 0u;
    return p;
}

// The diagonal term d_r x_r in FP64, with the same operations wherever it is formed.
template <bool CPLX>
__device__ __forceinline__ void diag_term(double dr, double di, double xr, double xi, double &re, double &im) {
    if (CPLX) {
        re = fma(dr, xr, -(di * xi));
        im = fma(dr, xi, di * xr);
    } else {
        re = dr * xr;
        im = 0.0;
    }
}

// Rows of rows row0 .. row0+255 (canonical order) that have no off-diagonal element (bit clear
// in `rowbits`): y[r] = d_r x[r].  The other part of the split SpMV (matvec_block with `split`)
// writes exactly the rows that have elements, so the two never write the same row.
template <int NV, class ET, bool CPLX>
__device__ __forceinline__ void diag_rows_block(const ET *__restrict__ dre, const ET *__restrict__ dim,
                                                const ET *__restrict__ x, int64_t ldx, ET *__restrict__ y, int64_t ldy,
                                                int nvec, int64_t N, const uint64_t *__restrict__ rowbits,
                                                int64_t row0) {
    const int64_t r = row0 + threadIdx.x;
    if (r >= N || ((rowbits[r >> 6] >> (r & 63)) & 1ull)) return;
    const double dr = (double)dre[r], di = CPLX ? (double)dim[r] : 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v < nvec) {
            double re, im;
            if (CPLX) {
                diag_term<true>(dr, di, (double)x[2 * (r * ldx + v)], (double)x[2 * (r * ldx + v) + 1], re, im);
                y[2 * (r * ldy + v)] = (ET)re;
                y[2 * (r * ldy + v) + 1] = (ET)im;
            } else {
                diag_term<false>(dr, 0.0, (double)x[r * ldx + v], 0.0, re, im);
                y[r * ldy + v] = (ET)re;
            }
        }
    }
}

// y[r] = d_r x[r] + sum over the row's present elements of H_rj x[j] for the rows at positions
// row0 .. row0+255 (of the canonical order, or of the slot order with `by_slot`), all `nvec`
// interleaved vectors; FP64 accumulation in group order.  With `split` a row forms d_r x[r] at
// its first off-diagonal element and writes y only if it has one (diag_rows_block writes the
// others), so rows without elements cost no random access to x, d or y.  Either way the sum is
// formed with the same operations in the same order.
template <int Wp, int NV, class ET, bool CPLX, int PF = 1>
__device__ __forceinline__ void matvec_block(const SubView &s, const HamView &h, const ET *__restrict__ dre,
                                             const ET *__restrict__ dim, const ET *__restrict__ x, int64_t ldx,
                                             ET *__restrict__ y, int64_t ldy, int nvec, int64_t row0,
                                             ChunkLds<Wp> &lds, bool by_slot = false, bool lockstep = false,
                                             bool filter_first = false, bool split = false, int64_t row_end = -1) {
    uint64_t key[Wp], hrow;
    uint32_t prow;
    bool valid;
    const int64_t r = load_row<Wp>(s, row0, key, hrow, prow, valid, by_slot, row_end);
    double acc_re[NV], acc_im[NV];
    bool have = !split;  // acc holds d_r x[r] (+ the elements so far)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc_re[v] = acc_im[v] = 0.0;
    if (!split) {
        const double dr = (double)dre[r];
        const double di = CPLX ? (double)dim[r] : 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (v < nvec) {
                if (CPLX)
                    diag_term<true>(dr, di, (double)x[2 * (r * ldx + v)], (double)x[2 * (r * ldx + v) + 1], acc_re[v],
                                    acc_im[v]);
                else
                    diag_term<false>(dr, 0.0, (double)x[r * ldx + v], 0.0, acc_re[v], acc_im[v]);
            }
        }
    }
    // one real vector: x_j is fetched for a whole batch of hits before any is consumed (a lane
    // without a hit loads x[0] and drops it, so the loads need no branch; ldx < 2^31)
    auto fetch = [&](int64_t j) -> double {
        if (CPLX || NV != 1) return 0.0;
        const uint32_t jj = j < 0 ? 0u : (uint32_t)j;
        const double v = (double)x[(uint64_t)jj * (uint32_t)ldx];
        return j < 0 ? 0.0 : v;
    };
    auto use = [&](int64_t j, ET vre, ET vim, double xj) {
        if (!have) {
            have = true;
            const double dr = (double)dre[r];
            const double di = CPLX ? (double)dim[r] : 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (v < nvec) {
                    if (CPLX)
                        diag_term<true>(dr, di, (double)x[2 * (r * ldx + v)], (double)x[2 * (r * ldx + v) + 1],
                                        acc_re[v], acc_im[v]);
                    else
                        diag_term<false>(dr, 0.0, (double)x[r * ldx + v], 0.0, acc_re[v], acc_im[v]);
                }
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (v < nvec) {
                if (CPLX) {
                    const double xr = (double)x[2 * (j * ldx + v)], xi = (double)x[2 * (j * ldx + v) + 1];
                    acc_re[v] += (double)vre * xr - (double)vim * xi;
                    acc_im[v] += (double)vre * xi + (double)vim * xr;
                } else {
                    acc_re[v] += (double)vre * (NV == 1 ? xj : (double)x[j * ldx + v]);
                }
            }
        }
    };
    row_engine<Wp, false, PF>(s, h, key, hrow, prow, valid, lds, sink<ET>(use, fetch), nullptr, lockstep, filter_first);
    if (!valid || !have) return;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v < nvec) {
            if (CPLX) {
                y[2 * (r * ldy + v)] = (ET)acc_re[v];
                y[2 * (r * ldy + v) + 1] = (ET)acc_im[v];
            } else {
                y[r * ldy + v] = (ET)acc_re[v];
            }
        }
    }
}

}  // namespace qsd
