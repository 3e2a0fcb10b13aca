// Stored CSR operator: build (two-pass, or lower triangle with mirrored fill) and SpMV.
//
// The paper's primary output is a CSR matrix built in two passes over the rows (structure,
// then values; Methods, Matrix evaluation), and its CSR build evaluates only the lower
// triangle, recognised from the row bit at each group's most significant off-diagonal bit
// (Methods, Lower / upper triangle evaluation; Supplement, MSOB).  Here a qsd_csr handle keeps
// the matrix resident in HBM for repeated SpMVs (eigensolvers), trading memory for not
// re-evaluating matrix elements.
//
// Lower-triangle build: a row evaluates only the groups whose column sorts below it; every
// entry found is counted and written twice, into its own row and mirrored (conjugated) into
// the column's row, at positions taken from per-row atomic cursors.  Each row is then sorted
// by column, which makes the result independent of the atomic order.
//
// SpMV: LPR lanes per row (1, 4, 16 or 64, from the mean row length), entries strided over the
// row's lanes and summed by a fixed shuffle tree: bitwise reproducible.
#include <algorithm>
#include <vector>

#include "common.h"
#include "matvec.h"
#include "rowsort.h"

namespace qsd {
namespace {

inline unsigned grid_for_rows(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <int Wp>
__global__ __launch_bounds__(kBlock) void k_count_lower(SubView s, HamView h, unsigned long long *__restrict__ counts) {
    __shared__ ChunkLds<Wp> lds;
    uint64_t key[Wp], hrow;
    uint32_t prow;
    bool valid;
    const int64_t r = load_row<Wp>(s, (int64_t)blockIdx.x * kBlock, key, hrow, prow, valid);
    unsigned long long own = 1;  // diagonal
    row_engine<Wp, true>(s, h, key, hrow, prow, valid, lds, sink<double>([&](int64_t j, double, double, int) {
        ++own;
        atomicAdd(&counts[j], 1ull);  // the mirrored entry (r, j) -> (j, r)
    }), nullptr, false, true);
    if (valid) atomicAdd(&counts[r], own);
}

template <int Wp, class ET>
__global__ __launch_bounds__(kBlock) void k_fill_lower(SubView s, HamView h, const ET *__restrict__ dre,
                                                       const ET *__restrict__ dim, const int64_t *__restrict__ indptr,
                                                       unsigned long long *__restrict__ cursor,
                                                       int64_t *__restrict__ cols, typename C2<ET>::T *__restrict__ vals) {
    __shared__ ChunkLds<Wp> lds;
    uint64_t key[Wp], hrow;
    uint32_t prow;
    bool valid;
    const int64_t r = load_row<Wp>(s, (int64_t)blockIdx.x * kBlock, key, hrow, prow, valid);
    if (valid) {
        const int64_t o = indptr[r] + (int64_t)atomicAdd(&cursor[r], 1ull);
        typename C2<ET>::T d;
        d.x = dre[r];
        d.y = dim ? dim[r] : (ET)0;
        cols[o] = r;
        vals[o] = d;
    }
    row_engine<Wp, true>(s, h, key, hrow, prow, valid, lds, sink<ET>([&](int64_t j, ET vre, ET vim, int) {
        typename C2<ET>::T v;
        v.x = vre;
        v.y = vim;
        const int64_t o1 = indptr[r] + (int64_t)atomicAdd(&cursor[r], 1ull);
        cols[o1] = j;
        vals[o1] = v;
        const int64_t o2 = indptr[j] + (int64_t)atomicAdd(&cursor[j], 1ull);
        typename C2<ET>::T vc;
        vc.x = v.x;
        vc.y = -v.y;
        cols[o2] = r;
        vals[o2] = vc;
    }), nullptr, false, true);
}

// Sort each row's entries by column (one workgroup per row; see sort_row_entries).
template <class ET, class IT, bool CPLX>
__global__ __launch_bounds__(kBlock) void k_sort_rows(const int64_t *__restrict__ indptr, int64_t *__restrict__ cols,
                                                      const typename C2<ET>::T *__restrict__ vals, IT *__restrict__ out_idx,
                                                      ET *__restrict__ out_val) {
    __shared__ int64_t sc[kSortLds];
    const int64_t row = blockIdx.x;
    const int64_t a = indptr[row], b = indptr[row + 1];
    sort_row_entries<ET, IT, CPLX>(a, b - a, cols, vals, out_idx, out_val, sc);
}

__global__ void k_u64_to_i64(const unsigned long long *__restrict__ a, int64_t *__restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (int64_t)a[i];
}

__global__ void k_fill0_u64(unsigned long long *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// One stored entry's contribution to the row sums of `nvec` vectors.
template <int NV, class ET, bool CPLX>
__device__ __forceinline__ void csr_term(double vr, double vi, int64_t c, const ET *__restrict__ x, int64_t ldx,
                                         int nvec, double (&are)[NV], double (&aim)[NV]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v < nvec) {
            if (CPLX) {
                const double xr = (double)x[2 * (c * ldx + v)], xi = (double)x[2 * (c * ldx + v) + 1];
                are[v] += vr * xr - vi * xi;
                aim[v] += vr * xi + vi * xr;
            } else {
                are[v] += vr * (double)x[c * ldx + v];
            }
        }
    }
}

// stored entries in flight per lane: more for the long rows that get many lanes (LPR = 64 means a
// mean row length of 96 or more), two for the short rows
template <int LPR>
constexpr int csr_batch() {
    return LPR >= 64 ? 8 : LPR >= 16 ? 4 : 2;
}

// Index and value loads: non-temporal for long rows (streamed once, kept out of the caches that
// hold x), ordinary for short rows, whose neighbouring lanes share cache lines.
template <int LPR, class T>
__device__ __forceinline__ T stream_load(const T *p) {
    if (LPR >= 16) return __builtin_nontemporal_load(p);
    return *p;
}

// y[r] = sum over the row's entries of A_rc x[c] for `nvec` interleaved vectors; LPR lanes per
// row (consecutive lanes of one wave), FP64 accumulation, fixed reduction tree.  A lane takes
// entries a + sub, a + sub + LPR, ... in order, csr_batch<LPR>() at a time: the column indices and
// values of long rows are streamed once (non-temporal loads, so they do not evict x from the
// caches) and the x gathers of a batch are all in flight together.
template <int LPR, int NV, class IT, class ET, bool CPLX>
__global__ __launch_bounds__(256) void k_csr_spmv(const int64_t *__restrict__ indptr, const IT *__restrict__ idx,
                                                 const ET *__restrict__ val, int64_t N, const ET *__restrict__ x,
                                                 int64_t ldx, ET *__restrict__ y, int64_t ldy, int nvec) {
    const int sub = threadIdx.x % LPR;
    const int64_t row = ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPR;
    double are[NV], aim[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) are[v] = aim[v] = 0.0;
    constexpr int kCsrBatch = csr_batch<LPR>();
    if (row < N) {
        const int64_t a = indptr[row], b = indptr[row + 1];
        // batches of kCsrBatch entries per lane; past the row's end the loads repeat its last
        // entry (always valid) and the term is skipped, so the sum takes the entries in order
        for (int64_t e = a + sub; e < b; e += kCsrBatch * LPR) {
            int64_t c[kCsrBatch];
            double vr[kCsrBatch], vi[kCsrBatch];
#pragma unroll
            for (int k = 0; k < kCsrBatch; ++k) {
                const int64_t ek = min(e + (int64_t)k * LPR, b - 1);
                c[k] = (int64_t)stream_load<LPR>(&idx[ek]);
                if (CPLX) {
                    vr[k] = (double)stream_load<LPR>(&val[2 * ek]);
                    vi[k] = (double)stream_load<LPR>(&val[2 * ek + 1]);
                } else {
                    vr[k] = (double)stream_load<LPR>(&val[ek]);
                    vi[k] = 0.0;
                }
            }
            if (NV == 1 && !CPLX) {
                // one real vector: the batch's x gathers are issued together too
                double xv[kCsrBatch];
#pragma unroll
                for (int k = 0; k < kCsrBatch; ++k) xv[k] = (double)x[c[k] * ldx];
#pragma unroll
                for (int k = 0; k < kCsrBatch; ++k)
                    if (e + (int64_t)k * LPR < b) are[0] += vr[k] * xv[k];
            } else {
#pragma unroll
                for (int k = 0; k < kCsrBatch; ++k)
                    if (e + (int64_t)k * LPR < b) csr_term<NV, ET, CPLX>(vr[k], vi[k], c[k], x, ldx, nvec, are, aim);
            }
        }
    }
#pragma unroll
    for (int d = LPR / 2; d >= 1; d >>= 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            are[v] += __shfl_xor(are[v], d, 64);
            if (CPLX) aim[v] += __shfl_xor(aim[v], d, 64);
        }
    }
    if (sub == 0 && row < N) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (v < nvec) {
                if (CPLX) {
                    y[2 * (row * ldy + v)] = (ET)are[v];
                    y[2 * (row * ldy + v) + 1] = (ET)aim[v];
                } else {
                    y[row * ldy + v] = (ET)are[v];
                }
            }
        }
    }
}

template <int LPR, int NV, class IT, class ET, bool CPLX>
void launch_spmv(const qsd_csr *c, const void *x, int64_t ldx, void *y, int64_t ldy, int nvec, hipStream_t st) {
    const int64_t threads = c->N * LPR;
    const unsigned grid = (unsigned)((threads + 255) / 256);
    k_csr_spmv<LPR, NV, IT, ET, CPLX><<<grid, 256, 0, st>>>(c->indptr, (const IT *)c->indices, (const ET *)c->data,
                                                            c->N, (const ET *)x, ldx, (ET *)y, ldy, nvec);
}

template <int LPR, class IT, class ET, bool CPLX>
void spmv_nv(const qsd_csr *c, const void *x, int64_t ldx, void *y, int64_t ldy, int nvec, hipStream_t st) {
    if (nvec <= 1)
        launch_spmv<LPR, 1, IT, ET, CPLX>(c, x, ldx, y, ldy, nvec, st);
    else if (nvec <= 4 || CPLX)
        launch_spmv<LPR, 4, IT, ET, CPLX>(c, x, ldx, y, ldy, nvec, st);
    else if (nvec <= 8)
        launch_spmv<LPR, CPLX ? 4 : 8, IT, ET, CPLX>(c, x, ldx, y, ldy, nvec, st);
    else
        launch_spmv<LPR, CPLX ? 4 : 16, IT, ET, CPLX>(c, x, ldx, y, ldy, nvec, st);
}

template <class IT, class ET, bool CPLX>
void spmv_lpr(const qsd_csr *c, const void *x, int64_t ldx, void *y, int64_t ldy, int nvec, hipStream_t st) {
    switch (c->lpr) {
        case 1: spmv_nv<1, IT, ET, CPLX>(c, x, ldx, y, ldy, nvec, st); break;
        case 4: spmv_nv<4, IT, ET, CPLX>(c, x, ldx, y, ldy, nvec, st); break;
        case 16: spmv_nv<16, IT, ET, CPLX>(c, x, ldx, y, ldy, nvec, st); break;
        default: spmv_nv<64, IT, ET, CPLX>(c, x, ldx, y, ldy, nvec, st); break;
    }
}

template <class IT>
void spmv_dtype(const qsd_csr *c, const void *x, int64_t ldx, void *y, int64_t ldy, int nvec, hipStream_t st) {
    switch (c->dtype) {
        case QSD_F64: spmv_lpr<IT, double, false>(c, x, ldx, y, ldy, nvec, st); break;
        case QSD_F32: spmv_lpr<IT, float, false>(c, x, ldx, y, ldy, nvec, st); break;
        case QSD_C128: spmv_lpr<IT, double, true>(c, x, ldx, y, ldy, nvec, st); break;
        case QSD_C64: spmv_lpr<IT, float, true>(c, x, ldx, y, ldy, nvec, st); break;
    }
}

void free_csr(qsd_csr *c) {
    if (!c) return;
    dev_free(c->indptr);
    dev_free(c->indices);
    dev_free(c->data);
    dev_free(c->diag);
    delete c;
}

template <class ET>
void sort_into(qsd_csr *c, int64_t *cols, const void *vals, hipStream_t st) {
    const unsigned grid = (unsigned)c->N;
    const auto *v = (const typename C2<ET>::T *)vals;
    if (c->index_type == QSD_INDEX_I32) {
        if (c->cplx)
            k_sort_rows<ET, int32_t, true><<<grid, kBlock, 0, st>>>(c->indptr, cols, v, (int32_t *)c->indices, (ET *)c->data);
        else
            k_sort_rows<ET, int32_t, false><<<grid, kBlock, 0, st>>>(c->indptr, cols, v, (int32_t *)c->indices, (ET *)c->data);
    } else {
        if (c->cplx)
            k_sort_rows<ET, int64_t, true><<<grid, kBlock, 0, st>>>(c->indptr, cols, v, (int64_t *)c->indices, (ET *)c->data);
        else
            k_sort_rows<ET, int64_t, false><<<grid, kBlock, 0, st>>>(c->indptr, cols, v, (int64_t *)c->indices, (ET *)c->data);
    }
}

template <int Wp>
int build_lower(const qsd_ham *h, qsd_csr *c, hipStream_t st) {
    const int64_t N = h->N;
    const bool f32 = c->dtype == QSD_F32 || c->dtype == QSD_C64;
    unsigned long long *cnt = nullptr;
    QSD_TRY(dev_alloc(&cnt, N + 1));
    int64_t *tmp = nullptr;
    int rc = dev_alloc(&tmp, N + 1);
    if (rc == QSD_OK) {
        k_fill0_u64<<<1024, 256, 0, st>>>(cnt, N + 1);
        k_count_lower<Wp><<<grid_for_rows(N), kBlock, 0, st>>>(sub_view(h->s), ham_view(h, false), cnt);
        k_u64_to_i64<<<1024, 256, 0, st>>>(cnt, tmp, N + 1);
        rc = exclusive_scan_i64(tmp, c->indptr, N + 1, st);
    }
    int64_t nnz = 0;
    if (rc == QSD_OK && (hipMemcpyAsync(&nnz, c->indptr + N, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                         hipStreamSynchronize(st) != hipSuccess))
        rc = fail(QSD_ERR_HIP, "lower-triangle count failed: %s", hipGetErrorString(hipGetLastError()));
    dev_free(tmp);
    if (rc != QSD_OK) {
        dev_free(cnt);
        return rc;
    }
    c->nnz = nnz;
    int64_t *cols = nullptr;
    void *vals = nullptr;
    rc = dev_alloc(&cols, nnz);
    if (rc == QSD_OK) rc = f32 ? dev_alloc((float2 **)&vals, nnz) : dev_alloc((double2 **)&vals, nnz);
    const size_t isz = c->index_type == QSD_INDEX_I32 ? 4 : 8;
    const size_t vsz = (f32 ? 4 : 8) * (c->cplx ? 2 : 1);
    if (rc == QSD_OK) rc = dev_alloc((uint8_t **)&c->indices, nnz * isz);
    if (rc == QSD_OK) rc = dev_alloc((uint8_t **)&c->data, nnz * vsz);
    if (rc == QSD_OK) {
        k_fill0_u64<<<1024, 256, 0, st>>>(cnt, N + 1);
        const SubView sv = sub_view(h->s);
        if (f32)
            k_fill_lower<Wp, float><<<grid_for_rows(N), kBlock, 0, st>>>(
                sv, ham_view(h, true), h->diag32, h->is_complex ? h->diag32_im : nullptr, c->indptr, cnt, cols,
                (float2 *)vals);
        else
            k_fill_lower<Wp, double><<<grid_for_rows(N), kBlock, 0, st>>>(
                sv, ham_view(h, false), h->diag, h->is_complex ? h->diag_im : nullptr, c->indptr, cnt, cols,
                (double2 *)vals);
        if (f32)
            sort_into<float>(c, cols, vals, st);
        else
            sort_into<double>(c, cols, vals, st);
        if (hipStreamSynchronize(st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "lower-triangle fill failed: %s", hipGetErrorString(hipGetLastError()));
    }
    dev_free(cnt);
    dev_free(cols);
    dev_free(vals);
    return rc;
}

}  // namespace
}  // namespace qsd

using namespace qsd;

extern "C" int qsd_csr_create(const qsd_ham *h, int32_t index_type, int32_t dtype, uint32_t flags,
                              const qsd_allocator *alloc, void *stream, qsd_csr **out) {
    clear_error();
    if (!h || !out) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (flags & ~QSD_CSR_LOWER_MIRROR) return fail(QSD_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    if (index_type != QSD_INDEX_I32 && index_type != QSD_INDEX_I64)
        return fail(QSD_ERR_INVALID_ARG, "unknown index type %d", index_type);
    if (index_type == QSD_INDEX_I32 && h->N >= (1ll << 31))
        return fail(QSD_ERR_CAPACITY, "N = %lld does not fit int32 column indices", (long long)h->N);
    if (dtype < QSD_F64 || dtype > QSD_C64) return fail(QSD_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    if ((dtype == QSD_C128 || dtype == QSD_C64) != h->is_complex)
        return fail(QSD_ERR_DTYPE, "dtype %d does not match a %s operator", dtype, h->is_complex ? "complex" : "real");
    hipStream_t st = (hipStream_t)stream;
    auto *c = new (std::nothrow) qsd_csr();
    if (!c) return fail(QSD_ERR_OUT_OF_MEMORY, "host allocation failed");
    c->alloc = keep_allocator(alloc);
    c->stream = stream;
    AllocScope scope(&c->alloc, stream);
    c->N = h->N;
    c->index_type = index_type;
    c->dtype = dtype;
    c->cplx = h->is_complex;
    int rc = dev_alloc(&c->indptr, h->N + 1);
    if (rc == QSD_OK) rc = dev_alloc(&c->diag, h->N);
    if (rc == QSD_OK && hipMemcpyAsync(c->diag, h->diag, h->N * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
        rc = fail(QSD_ERR_HIP, "copy failed");
    if (rc == QSD_OK) {
        if (flags & QSD_CSR_LOWER_MIRROR) {
            switch (h->Wp) {
                case 1: rc = build_lower<1>(h, c, st); break;
                case 2: rc = build_lower<2>(h, c, st); break;
                case 4: rc = build_lower<4>(h, c, st); break;
                case 8: rc = build_lower<8>(h, c, st); break;
                case 16: rc = build_lower<16>(h, c, st); break;
            }
        } else {
            int64_t nnz = 0;
            rc = qsd_csr_build(h, c->indptr, nullptr, nullptr, index_type, dtype, &nnz, stream);
            const size_t isz = index_type == QSD_INDEX_I32 ? 4 : 8;
            const size_t vsz = ((dtype == QSD_F32 || dtype == QSD_C64) ? 4 : 8) * (c->cplx ? 2 : 1);
            if (rc == QSD_OK) rc = dev_alloc((uint8_t **)&c->indices, nnz * isz);
            if (rc == QSD_OK) rc = dev_alloc((uint8_t **)&c->data, nnz * vsz);
            if (rc == QSD_OK) rc = qsd_csr_build(h, c->indptr, c->indices, c->data, index_type, dtype, &nnz, stream);
            c->nnz = nnz;
        }
    }
    if (rc != QSD_OK) {
        free_csr(c);
        return rc;
    }
    const double mean = (double)c->nnz / (double)std::max<int64_t>(1, c->N);
    c->lpr = mean < 6.0 ? 1 : mean < 24.0 ? 4 : mean < 96.0 ? 16 : 64;
    *out = c;
    return QSD_OK;
}

extern "C" int qsd_csr_info(const qsd_csr *c, int64_t *N, int64_t *nnz, int64_t *bytes) {
    clear_error();
    if (!c) return fail(QSD_ERR_INVALID_ARG, "csr is NULL");
    if (N) *N = c->N;
    if (nnz) *nnz = c->nnz;
    if (bytes) {
        const int64_t isz = c->index_type == QSD_INDEX_I32 ? 4 : 8;
        const int64_t vsz = ((c->dtype == QSD_F32 || c->dtype == QSD_C64) ? 4 : 8) * (c->cplx ? 2 : 1);
        *bytes = (c->N + 1) * 8 + c->nnz * (isz + vsz);
    }
    return QSD_OK;
}

extern "C" int qsd_csr_export(const qsd_csr *c, int64_t *d_indptr, void *d_indices, void *d_data, void *stream) {
    clear_error();
    if (!c) return fail(QSD_ERR_INVALID_ARG, "csr is NULL");
    hipStream_t st = (hipStream_t)stream;
    const size_t isz = c->index_type == QSD_INDEX_I32 ? 4 : 8;
    const size_t vsz = ((c->dtype == QSD_F32 || c->dtype == QSD_C64) ? 4 : 8) * (c->cplx ? 2 : 1);
    if (d_indptr) QSD_CHECK_HIP(hipMemcpyAsync(d_indptr, c->indptr, (c->N + 1) * 8, hipMemcpyDeviceToDevice, st));
    if (d_indices && c->nnz)
        QSD_CHECK_HIP(hipMemcpyAsync(d_indices, c->indices, c->nnz * isz, hipMemcpyDeviceToDevice, st));
    if (d_data && c->nnz) QSD_CHECK_HIP(hipMemcpyAsync(d_data, c->data, c->nnz * vsz, hipMemcpyDeviceToDevice, st));
    return QSD_OK;
}

extern "C" int qsd_csr_matvec(const qsd_csr *c, int32_t nvec, const void *d_x, int64_t ldx, void *d_y, int64_t ldy,
                              int32_t dtype, void *stream) {
    clear_error();
    if (!c || !d_x || !d_y) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    if (nvec < 1 || nvec > 16) return fail(QSD_ERR_INVALID_ARG, "nvec must be in [1, 16]");
    if (ldx < nvec || ldy < nvec) return fail(QSD_ERR_INVALID_ARG, "leading dimension smaller than nvec");
    if (ldx > INT32_MAX || ldy > INT32_MAX) return fail(QSD_ERR_INVALID_ARG, "leading dimension of 2^31 or more");
    if (dtype != c->dtype) return fail(QSD_ERR_DTYPE, "vectors must have the matrix dtype %d", c->dtype);
    hipStream_t st = (hipStream_t)stream;
    const int chunk = c->cplx ? 4 : 16;
    const size_t esz = dtype == QSD_F64 ? 8 : dtype == QSD_F32 ? 4 : dtype == QSD_C128 ? 16 : 8;
    for (int v0 = 0; v0 < nvec; v0 += chunk) {
        const int nv = std::min(chunk, nvec - v0);
        const void *x = (const char *)d_x + v0 * esz;
        void *y = (char *)d_y + v0 * esz;
        if (c->index_type == QSD_INDEX_I32)
            spmv_dtype<int32_t>(c, x, ldx, y, ldy, nv, st);
        else
            spmv_dtype<int64_t>(c, x, ldx, y, ldy, nv, st);
    }
    QSD_CHECK_HIP(hipGetLastError());
    return QSD_OK;
}

extern "C" int qsd_csr_destroy(qsd_csr *c) {
    clear_error();
    if (!c) return QSD_OK;
    AllocScope scope(&c->alloc, c->stream);
    free_csr(c);
    return QSD_OK;
}
