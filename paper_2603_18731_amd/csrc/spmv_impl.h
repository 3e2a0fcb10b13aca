// The matrix-free SpMV kernel and its launch, instantiated for the key width QSD_SPMV_WP by the
// translation unit that includes this file (one per width, so they compile in parallel).
#include <type_traits>

#include "common.h"
#include "device.h"
#include "engine.h"
#include "matvec.h"
#include "spmv.h"

#ifndef QSD_SPMV_WP
#error "define QSD_SPMV_WP before including spmv_impl.h"
#endif

namespace qsd {
namespace {

inline unsigned grid_for(int64_t n, int per_block) { return (unsigned)((n + per_block - 1) / per_block); }

// Rows in slot order touch x, d and y at random positions.  With a slot-order schedule the launch
// is split by role: the first `nd` workgroups (a multiple of 8, so the XCD of a workgroup is still
// its index mod 8) write y = d x for the rows without off-diagonal elements in canonical order,
// the rest take the slot-order tiles and write only the rows with elements; no row is written
// twice, and each row's value is formed with the same operations as in every other schedule.
// Product-map kernels are never split (nd = 0: their rows find columns without the table, so a
// slot order gains them nothing), which drops the split's per-hit test from them.  With `tpb`
// (tiles per high part, for low-part counts of at least two tiles) their tiles follow the
// product's blocks of rows: tile (b, k) takes rows b |A| + 256 k .. of high part b only, so every
// workgroup's rows share their high part (bulk rejection and the once-per-chunk high rank
// apply to all of them), at the price of a partial last tile per high part.
// (Single-vector kernels for up to four key words are held to five waves per SIMD.)
template <int Wp, int NV, class ET, bool CPLX, int PF>
__global__ __launch_bounds__(kBlock, Wp <= 4 && NV == 1 ? 5 : 1) void k_matvec(
    SubView s, HamView h, const ET *__restrict__ dre,
                                                   const ET *__restrict__ dim, const ET *__restrict__ x, int64_t ldx,
                                                   ET *__restrict__ y, int64_t ldy, int nvec, uint32_t sched,
                                                   const uint64_t *__restrict__ rowbits, unsigned nd,
                                                   unsigned tpb = 0u) {
    __shared__ ChunkLds<Wp> lds;
    if (blockIdx.x < nd) {
        diag_rows_block<NV, ET, CPLX>(dre, dim, x, ldx, y, ldy, nvec, s.N, rowbits, (int64_t)blockIdx.x * kBlock);
        return;
    }
    const int64_t tile = tile_index(blockIdx.x - nd, gridDim.x - nd, (sched & QSD_SCHED_XCD_REMAP) != 0);
    int64_t row0 = tile * kBlock, row_end = -1;
    if (PF == 2 && tpb) {
        const int64_t b = tile / tpb;
        row0 = b * (int64_t)s.pna + (tile - b * tpb) * kBlock;
        row_end = (b + 1) * (int64_t)s.pna;
    }
    matvec_block<Wp, NV, ET, CPLX, PF>(s, h, dre, dim, x, ldx, y, ldy, nvec, row0, lds,
                                       (sched & QSD_SCHED_SLOT_ORDER) != 0, (sched & QSD_SCHED_LOCKSTEP) != 0,
                                       (sched & QSD_SCHED_FILTER_FIRST) != 0, PF != 2 && nd > 0, row_end);
}

template <int Wp, int NV, class ET, bool CPLX>
void launch_mv(const qsd_ham *h, const void *x, int64_t ldx, void *y, int64_t ldy, int nvec, hipStream_t st) {
    const bool f32 = std::is_same<ET, float>::value;
    const ET *dre = f32 ? (const ET *)h->diag32 : (const ET *)h->diag;
    const ET *dim = CPLX ? (f32 ? (const ET *)h->diag32_im : (const ET *)h->diag_im) : nullptr;
    const unsigned tiles = grid_for(h->N, kBlock);
    const bool split = (h->schedule & QSD_SCHED_SLOT_ORDER) && h->rowbits;
    const unsigned nd = split ? (tiles + 7u) & ~7u : 0u;
    // the part-filter variant only for subspaces that have filters (the other one carries no
    // filter code, so it keeps its registers), the product-map variant for one-word product
    // subspaces
    if constexpr (Wp == 1) {
        if (h->s->prank && !(h->schedule & QSD_SCHED_HASH_LOOKUP)) {
            // tiles within the product's blocks of rows when a block spans at least two tiles
            // (rows in canonical order: each high part's |A| rows are consecutive)
            const uint32_t pna = h->s->pna;
            const bool by_part = !(h->schedule & QSD_SCHED_SLOT_ORDER) && pna >= 2u * kBlock;
            const unsigned tpb = by_part ? (unsigned)((pna + kBlock - 1) / kBlock) : 0u;
            const unsigned grid = by_part ? (unsigned)(h->N / pna) * tpb : tiles;
            k_matvec<Wp, NV, ET, CPLX, 2><<<grid, kBlock, 0, st>>>(sub_view(h->s), ham_view(h, f32), dre, dim,
                                                                  (const ET *)x, ldx, (ET *)y, ldy, nvec,
                                                                  h->schedule, h->rowbits, 0u, tpb);
            return;
        }
    }
    if (h->s->pfilt)
        k_matvec<Wp, NV, ET, CPLX, 1><<<nd + tiles, kBlock, 0, st>>>(sub_view(h->s), ham_view(h, f32), dre, dim,
                                                                    (const ET *)x, ldx, (ET *)y, ldy, nvec,
                                                                    h->schedule, h->rowbits, nd);
    else
        k_matvec<Wp, NV, ET, CPLX, 0><<<nd + tiles, kBlock, 0, st>>>(sub_view(h->s), ham_view(h, f32), dre, dim,
                                                                    (const ET *)x, ldx, (ET *)y, ldy, nvec,
                                                                    h->schedule, h->rowbits, nd);
}

template <int Wp, class ET, bool CPLX>
void dispatch_nv(const qsd_ham *h, const void *x, int64_t ldx, void *y, int64_t ldy, int nvec, hipStream_t st) {
    if (nvec <= 1)
        launch_mv<Wp, 1, ET, CPLX>(h, x, ldx, y, ldy, nvec, st);
    else if (nvec <= 2)
        launch_mv<Wp, 2, ET, CPLX>(h, x, ldx, y, ldy, nvec, st);
    else if (nvec <= 4 || CPLX)
        launch_mv<Wp, 4, ET, CPLX>(h, x, ldx, y, ldy, nvec, st);
    else if (nvec <= 8)
        launch_mv<Wp, CPLX ? 4 : 8, ET, CPLX>(h, x, ldx, y, ldy, nvec, st);
    else
        launch_mv<Wp, CPLX ? 4 : 16, ET, CPLX>(h, x, ldx, y, ldy, nvec, st);
}


}  // namespace

template <int Wp, class ET, bool CPLX>
void spmv_dispatch(const qsd_ham *h, const void *x, int64_t ldx, void *y, int64_t ldy, int nvec, hipStream_t st) {
    dispatch_nv<Wp, ET, CPLX>(h, x, ldx, y, ldy, nvec, st);
}

template void spmv_dispatch<QSD_SPMV_WP, double, false>(const qsd_ham *, const void *, int64_t, void *, int64_t, int,
                                                        hipStream_t);
template void spmv_dispatch<QSD_SPMV_WP, float, false>(const qsd_ham *, const void *, int64_t, void *, int64_t, int,
                                                       hipStream_t);
template void spmv_dispatch<QSD_SPMV_WP, double, true>(const qsd_ham *, const void *, int64_t, void *, int64_t, int,
                                                       hipStream_t);
template void spmv_dispatch<QSD_SPMV_WP, float, true>(const qsd_ham *, const void *, int64_t, void *, int64_t, int,
                                                      hipStream_t);

}  // namespace qsd
