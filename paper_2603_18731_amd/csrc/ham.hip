// Subspace Hamiltonian on the device: cached diagonal, matrix-free SpMV / SpMM and the
// two-pass CSR builder (Methods, Matrix evaluation).  The row walk itself is in engine.h.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "common.h"
#include "device.h"
#include "engine.h"
#include "matvec.h"
#include "rowsort.h"
#include "spmv.h"

namespace qsd {
namespace {

// ----------------------------------------------------------------------------- diagonal

template <int Wp>
__global__ __launch_bounds__(kBlock) void k_diag(SubView s, const uint64_t *__restrict__ cws,
                                                 const double *__restrict__ coef, int64_t Td, double *__restrict__ d_re,
                                                 double *__restrict__ d_im) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.N) return;
    uint64_t key[Wp];
#pragma unroll
    for (int w = 0; w < Wp; ++w) key[w] = s.keys[(int64_t)w * s.N + i];
    double re = 0.0, im = 0.0;
    for (int64_t t = 0; t < Td; ++t) {
        const uint64_t *c = cws + t * 3 * Wp;
        if (!term_pass<Wp>(key, c)) continue;  // projector pass-over before the sign
        const double cr = coef[2 * t], ci = coef[2 * t + 1];
        if (term_parity<Wp>(key, c)) {
            re -= cr;
            im -= ci;
        } else {
            re += cr;
            im += ci;
        }
    }
    d_re[i] = re;
    if (d_im) d_im[i] = im;
}

__global__ void k_to_f32(const double *__restrict__ in, float *__restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

// ------------------------------------------------------------------------------- matvec

// Bit r of `bits` = row r has an off-diagonal element (a probe whose column is present and
// whose term range has a term passing the row's projector bits).
template <int Wp>
__global__ __launch_bounds__(kBlock) void k_row_bits(SubView s, HamView h, uint64_t *__restrict__ bits) {
    __shared__ ChunkLds<Wp> lds;
    uint64_t key[Wp], hrow;
    uint32_t prow;
    bool valid;
    const int64_t row0 = (int64_t)blockIdx.x * kBlock;
    load_row<Wp>(s, row0, key, hrow, prow, valid);
    bool has = false;
    row_engine<Wp>(s, h, key, hrow, prow, valid, lds, sink<double>([&](int64_t, double, double, int) { has = true; }), nullptr, false, true);
    const uint64_t w = __ballot(has && valid);
    const int64_t word = (row0 >> 6) + (threadIdx.x >> 6);
    if ((threadIdx.x & 63) == 0 && word * 64 < s.N) bits[word] = w;
}

// ---------------------------------------------------------------------------------- CSR

template <int Wp>
__global__ __launch_bounds__(kBlock) void k_csr_count(SubView s, HamView h, int64_t *__restrict__ counts) {
    __shared__ ChunkLds<Wp> lds;
    uint64_t key[Wp], hrow;
    uint32_t prow;
    bool valid;
    const int64_t r = load_row<Wp>(s, (int64_t)blockIdx.x * kBlock, key, hrow, prow, valid);
    int64_t cnt = 1;  // diagonal
    row_engine<Wp>(s, h, key, hrow, prow, valid, lds, sink<double>([&](int64_t, double, double, int) { ++cnt; }), nullptr, false, true);
    if (valid) counts[r] = cnt;
}

// Work counters of one SpMV: probes (live groups that reach the hash table) and stored
// off-diagonal entries.
template <int Wp>
__global__ __launch_bounds__(kBlock) void k_probe_count(SubView s, HamView h, unsigned long long *__restrict__ acc) {
    __shared__ ChunkLds<Wp> lds;
    uint64_t key[Wp], hrow;
    uint32_t prow;
    bool valid;
    load_row<Wp>(s, (int64_t)blockIdx.x * kBlock, key, hrow, prow, valid);
    unsigned long long probes = 0, hits = 0;
    row_engine<Wp>(s, h, key, hrow, prow, valid, lds, sink<double>([&](int64_t, double, double, int) { ++hits; }), &probes, false, true);
    for (int d = 32; d >= 1; d >>= 1) {
        probes += __shfl_xor(probes, d, 64);
        hits += __shfl_xor(hits, d, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&acc[0], probes);
        atomicAdd(&acc[1], hits);
    }
}

// Unsorted fill into scratch: columns (int64) and values (double2 / float2).
template <int Wp, class ET>
__global__ __launch_bounds__(kBlock) void k_csr_fill(SubView s, HamView h, const ET *__restrict__ dre,
                                                     const ET *__restrict__ dim, const int64_t *__restrict__ indptr,
                                                     int64_t *__restrict__ cols, typename C2<ET>::T *__restrict__ vals) {
    __shared__ ChunkLds<Wp> lds;
    uint64_t key[Wp], hrow;
    uint32_t prow;
    bool valid;
    const int64_t r = load_row<Wp>(s, (int64_t)blockIdx.x * kBlock, key, hrow, prow, valid);
    int64_t o = indptr[r];
    if (valid) {
        cols[o] = r;
        typename C2<ET>::T d;
        d.x = dre[r];
        d.y = dim ? dim[r] : (ET)0;
        vals[o] = d;
    }
    ++o;
    row_engine<Wp>(s, h, key, hrow, prow, valid, lds, sink<ET>([&](int64_t j, ET vre, ET vim, int) {
        typename C2<ET>::T v;
        v.x = vre;
        v.y = vim;
        cols[o] = j;
        vals[o] = v;
        ++o;
    }), nullptr, false, true);
}

// Sort each row's entries by column (one workgroup per row; see sort_row_entries).
template <class ET, class IT, bool CPLX>
__global__ __launch_bounds__(kBlock) void k_csr_sort(const int64_t *__restrict__ indptr, int64_t *__restrict__ cols,
                                                     const typename C2<ET>::T *__restrict__ vals, IT *__restrict__ out_idx,
                                                     ET *__restrict__ out_val) {
    __shared__ int64_t sc[kSortLds];
    const int64_t row = blockIdx.x;
    const int64_t a = indptr[row], b = indptr[row + 1];
    sort_row_entries<ET, IT, CPLX>(a, b - a, cols, vals, out_idx, out_val, sc);
}

inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

inline HamView view_of(const qsd_ham *h, bool f32) { return ham_view(h, f32); }
inline SubView sview(const qsd_subspace *s) { return sub_view(s); }

template <class T>
int upload(T **dst, const std::vector<T> &src, hipStream_t st) {
    QSD_TRY(dev_alloc(dst, src.size()));
    if (!src.empty()) QSD_CHECK_HIP(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return QSD_OK;
}

void free_ham(qsd_ham *h) {
    if (!h) return;
    if (h->s) {
        auto &b = h->s->bound;
        b.erase(std::remove(b.begin(), b.end(), h), b.end());
    }
    dev_free(h->diag);
    dev_free(h->diag_im);
    dev_free(h->g_mask);
    dev_free(h->g_hash);
    dev_free(h->g_part);
    dev_free(h->g_pos);
    dev_free(h->g_scan);
    dev_free(h->g_info);
    dev_free(h->g_term0);
    dev_free(h->g_nterm);
    dev_free(h->g_iptr);
    dev_free(h->t_cws);
    dev_free(h->t_coef);
    dev_free(h->t_cw32);
    dev_free(h->t_coef32);
    dev_free(h->diag32);
    dev_free(h->diag32_im);
    dev_free(h->rowbits);
    delete h;
}

template <int Wp>
void launch_diag(const qsd_ham *h, const uint64_t *cws, const double *coef, int64_t Td,
                 hipStream_t st) {
    k_diag<Wp><<<grid_for(h->N, kBlock), kBlock, 0, st>>>(sview(h->s), cws, coef, Td, h->diag, h->diag_im);
}

int create_impl(qsd_ham *h, hipStream_t st) {
    const qsd_op *op = h->op;
    QSD_TRY(upload(&h->g_mask, op->g_mask, st));
    const std::vector<uint64_t> gh = group_hashes(op, h->s->z);  // alive until the synchronize below
    QSD_TRY(upload(&h->g_hash, gh, st));
    std::vector<uint32_t> gp;
    if (h->s->split > 0) {
        gp = group_parts(op, h->s->pz);
        QSD_TRY(upload(&h->g_part, gp, st));
    }
    QSD_TRY(upload(&h->g_pos, op->g_pos, st));
    QSD_TRY(upload(&h->g_scan, op->g_scan, st));
    QSD_TRY(upload(&h->g_info, op->g_info, st));
    QSD_TRY(upload(&h->g_term0, op->g_term0, st));
    QSD_TRY(upload(&h->g_nterm, op->g_nterm, st));
    QSD_TRY(upload(&h->g_iptr, op->g_iptr, st));
    QSD_TRY(upload(&h->t_cws, op->t_cws, st));
    std::vector<uint32_t> cw32;
    if (op->n_qubits <= 32) {
        // one-word keys of at most 32 qubits: the term masks fit 32 bits
        const size_t To = op->t_cws.size() / 3;
        cw32.assign(To * 4, 0u);
        for (size_t t = 0; t < To; ++t) {
            for (int k = 0; k < 3; ++k) cw32[t * 4 + k] = (uint32_t)op->t_cws[t * 3 + k];
            cw32[t * 4 + 3] = op->t_tail[t];
        }
        QSD_TRY(upload(&h->t_cw32, cw32, st));
    }
    QSD_TRY(upload(&h->t_coef, op->t_coef, st));
    std::vector<float> c32(op->t_coef.size());
    for (size_t k = 0; k < c32.size(); ++k) c32[k] = (float)op->t_coef[k];
    QSD_TRY(upload(&h->t_coef32, c32, st));
    QSD_TRY(dev_alloc(&h->diag, h->N));
    QSD_TRY(dev_alloc(&h->diag32, h->N));
    if (h->is_complex) {
        QSD_TRY(dev_alloc(&h->diag_im, h->N));
        QSD_TRY(dev_alloc(&h->diag32_im, h->N));
    }
    uint64_t *dcws = nullptr;
    double *dcoef = nullptr;
    const int64_t Td = (int64_t)op->diag_coef.size() / 2;
    QSD_TRY(upload(&dcws, op->diag_cws, st));
    int rc = upload(&dcoef, op->diag_coef, st);
    if (rc == QSD_OK) {
        switch (h->Wp) {
            case 1: launch_diag<1>(h, dcws, dcoef, Td, st); break;
            case 2: launch_diag<2>(h, dcws, dcoef, Td, st); break;
            case 4: launch_diag<4>(h, dcws, dcoef, Td, st); break;
            case 8: launch_diag<8>(h, dcws, dcoef, Td, st); break;
            case 16: launch_diag<16>(h, dcws, dcoef, Td, st); break;
        }
        k_to_f32<<<1024, kBlock, 0, st>>>(h->diag, h->diag32, h->N);
        if (h->is_complex) k_to_f32<<<1024, kBlock, 0, st>>>(h->diag_im, h->diag32_im, h->N);
        if (hipStreamSynchronize(st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "diagonal kernel failed: %s", hipGetErrorString(hipGetLastError()));
    }
    dev_free(dcws);
    dev_free(dcoef);
    return rc;
}

template <class ET, bool CPLX>
void dispatch_w(const qsd_ham *h, const void *x, int64_t ldx, void *y, int64_t ldy, int nvec, hipStream_t st) {
    switch (h->Wp) {
        case 1: spmv_dispatch<1, ET, CPLX>(h, x, ldx, y, ldy, nvec, st); break;
        case 2: spmv_dispatch<2, ET, CPLX>(h, x, ldx, y, ldy, nvec, st); break;
        case 4: spmv_dispatch<4, ET, CPLX>(h, x, ldx, y, ldy, nvec, st); break;
        case 8: spmv_dispatch<8, ET, CPLX>(h, x, ldx, y, ldy, nvec, st); break;
        case 16: spmv_dispatch<16, ET, CPLX>(h, x, ldx, y, ldy, nvec, st); break;
    }
}

template <int Wp>
void launch_count(const qsd_ham *h, int64_t *counts, hipStream_t st) {
    k_csr_count<Wp><<<grid_for(h->N, kBlock), kBlock, 0, st>>>(sview(h->s), view_of(h, false), counts);
}

template <int Wp, class ET>
void launch_fill(const qsd_ham *h, const int64_t *indptr, int64_t *cols, void *vals, hipStream_t st) {
    const bool f32 = std::is_same<ET, float>::value;
    const ET *dre = f32 ? (const ET *)h->diag32 : (const ET *)h->diag;
    const ET *dim = h->is_complex ? (f32 ? (const ET *)h->diag32_im : (const ET *)h->diag_im) : nullptr;
    k_csr_fill<Wp, ET><<<grid_for(h->N, kBlock), kBlock, 0, st>>>(sview(h->s), view_of(h, f32), dre, dim, indptr, cols,
                                                                   (typename C2<ET>::T *)vals);
}

template <class ET>
void fill_w(const qsd_ham *h, const int64_t *indptr, int64_t *cols, void *vals, hipStream_t st) {
    switch (h->Wp) {
        case 1: launch_fill<1, ET>(h, indptr, cols, vals, st); break;
        case 2: launch_fill<2, ET>(h, indptr, cols, vals, st); break;
        case 4: launch_fill<4, ET>(h, indptr, cols, vals, st); break;
        case 8: launch_fill<8, ET>(h, indptr, cols, vals, st); break;
        case 16: launch_fill<16, ET>(h, indptr, cols, vals, st); break;
    }
}

int check_dtype(const qsd_ham *h, int32_t dtype) {
    if (dtype < QSD_F64 || dtype > QSD_C64) return fail(QSD_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    const bool want_c = dtype == QSD_C128 || dtype == QSD_C64;
    if (want_c != h->is_complex)
        return fail(QSD_ERR_DTYPE, "dtype %d does not match a %s operator", dtype, h->is_complex ? "complex" : "real");
    return QSD_OK;
}

}  // namespace
}  // namespace qsd

using namespace qsd;

extern "C" int qsd_ham_create(const qsd_subspace *s, const qsd_op *op, uint32_t flags, const qsd_allocator *alloc,
                              void *stream, qsd_ham **out) {
    clear_error();
    if (!out) return fail(QSD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!s || !op) return fail(QSD_ERR_INVALID_ARG, "NULL subspace or operator");
    if (s->n_qubits != op->n_qubits)
        return fail(QSD_ERR_INVALID_ARG, "subspace has %d qubits, operator %d", s->n_qubits, op->n_qubits);
    (void)flags;
    auto *h = new (std::nothrow) qsd_ham();
    if (!h) return fail(QSD_ERR_OUT_OF_MEMORY, "host allocation failed");
    h->alloc = keep_allocator(alloc);
    h->stream = stream;
    AllocScope scope(&h->alloc, stream);
    h->s = s;
    h->op = op;
    h->N = s->N;
    h->G = (int64_t)op->g_info.size();
    h->Wp = s->Wp;
    h->is_complex = op->is_complex;
    int rc = create_impl(h, (hipStream_t)stream);
    if (rc != QSD_OK) {
        free_ham(h);
        return rc;
    }
    s->bound.push_back(h);
    *out = h;
    return QSD_OK;
}

extern "C" int qsd_ham_info(const qsd_ham *h, int64_t *N, int64_t *G, int32_t *is_complex) {
    clear_error();
    if (!h) return fail(QSD_ERR_INVALID_ARG, "ham is NULL");
    if (N) *N = h->N;
    if (G) *G = h->G + 1;
    if (is_complex) *is_complex = h->is_complex ? 1 : 0;
    return QSD_OK;
}

extern "C" int qsd_ham_diagonal(const qsd_ham *h, double *d_out, void *stream) {
    clear_error();
    if (!h || !d_out) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    QSD_CHECK_HIP(hipMemcpyAsync(d_out, h->diag, h->N * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return QSD_OK;
}

extern "C" int qsd_ham_destroy(qsd_ham *h) {
    clear_error();
    if (!h) return QSD_OK;
    AllocScope scope(&h->alloc, h->stream);
    free_ham(h);
    return QSD_OK;
}

extern "C" int qsd_matvec(const qsd_ham *h, int32_t nvec, const void *d_x, int64_t ldx, void *d_y, int64_t ldy,
                          int32_t dtype, void *stream) {
    clear_error();
    if (!h || !d_x || !d_y) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    if (nvec < 1 || nvec > 16) return fail(QSD_ERR_INVALID_ARG, "nvec must be in [1, 16]");
    if (ldx < nvec || ldy < nvec) return fail(QSD_ERR_INVALID_ARG, "leading dimension smaller than nvec");
    if (ldx > INT32_MAX || ldy > INT32_MAX) return fail(QSD_ERR_INVALID_ARG, "leading dimension of 2^31 or more");
    QSD_TRY(check_dtype(h, dtype));
    hipStream_t st = (hipStream_t)stream;
    const int chunk = (dtype == QSD_C128 || dtype == QSD_C64) ? 4 : 16;
    const size_t esz = dtype == QSD_F64 ? 8 : dtype == QSD_F32 ? 4 : dtype == QSD_C128 ? 16 : 8;
    for (int v0 = 0; v0 < nvec; v0 += chunk) {
        const int nv = std::min(chunk, nvec - v0);
        const void *x = (const char *)d_x + v0 * esz;
        void *y = (char *)d_y + v0 * esz;
        switch (dtype) {
            case QSD_F64: dispatch_w<double, false>(h, x, ldx, y, ldy, nv, st); break;
            case QSD_F32: dispatch_w<float, false>(h, x, ldx, y, ldy, nv, st); break;
            case QSD_C128: dispatch_w<double, true>(h, x, ldx, y, ldy, nv, st); break;
            case QSD_C64: dispatch_w<float, true>(h, x, ldx, y, ldy, nv, st); break;
        }
    }
    QSD_CHECK_HIP(hipGetLastError());
    return QSD_OK;
}

extern "C" int qsd_csr_build(const qsd_ham *h, int64_t *d_indptr, void *d_indices, void *d_data, int32_t index_type,
                             int32_t dtype, int64_t *nnz_out, void *stream) {
    clear_error();
    if (!h || !d_indptr) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    if (index_type != QSD_INDEX_I32 && index_type != QSD_INDEX_I64)
        return fail(QSD_ERR_INVALID_ARG, "unknown index type %d", index_type);
    if (index_type == QSD_INDEX_I32 && h->N >= (1ll << 31))
        return fail(QSD_ERR_CAPACITY, "N = %lld does not fit int32 column indices", (long long)h->N);
    QSD_TRY(check_dtype(h, dtype));
    AllocScope scope(&h->alloc, stream);
    hipStream_t st = (hipStream_t)stream;
    const bool fill = d_indices && d_data;
    if ((d_indices == nullptr) != (d_data == nullptr))
        return fail(QSD_ERR_INVALID_ARG, "indices and data must both be NULL (count) or both set (fill)");
    if (!fill) {
        int64_t *counts = nullptr;
        QSD_TRY(dev_alloc(&counts, h->N + 1));
        switch (h->Wp) {
            case 1: launch_count<1>(h, counts, st); break;
            case 2: launch_count<2>(h, counts, st); break;
            case 4: launch_count<4>(h, counts, st); break;
            case 8: launch_count<8>(h, counts, st); break;
            case 16: launch_count<16>(h, counts, st); break;
        }
        int64_t zero = 0;
        int rc = QSD_OK;
        if (hipMemcpyAsync(counts + h->N, &zero, 8, hipMemcpyHostToDevice, st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "copy failed");
        if (rc == QSD_OK) rc = exclusive_scan_i64(counts, d_indptr, h->N + 1, st);
        int64_t nnz = 0;
        if (rc == QSD_OK && (hipMemcpyAsync(&nnz, d_indptr + h->N, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                             hipStreamSynchronize(st) != hipSuccess))
            rc = fail(QSD_ERR_HIP, "CSR count failed: %s", hipGetErrorString(hipGetLastError()));
        dev_free(counts);
        if (rc == QSD_OK && nnz_out) *nnz_out = nnz;
        return rc;
    }
    int64_t nnz = 0;
    QSD_CHECK_HIP(hipMemcpyAsync(&nnz, d_indptr + h->N, 8, hipMemcpyDeviceToHost, st));
    QSD_CHECK_HIP(hipStreamSynchronize(st));
    const bool f32 = dtype == QSD_F32 || dtype == QSD_C64;
    int64_t *cols = nullptr;
    void *vals = nullptr;
    QSD_TRY(dev_alloc(&cols, nnz));
    int rc = f32 ? dev_alloc((float2 **)&vals, nnz) : dev_alloc((double2 **)&vals, nnz);
    if (rc == QSD_OK) {
        if (f32)
            fill_w<float>(h, d_indptr, cols, vals, st);
        else
            fill_w<double>(h, d_indptr, cols, vals, st);
        const unsigned grid = (unsigned)h->N;
        const bool cx = h->is_complex;
        if (index_type == QSD_INDEX_I32) {
            if (f32) {
                if (cx) k_csr_sort<float, int32_t, true><<<grid, kBlock, 0, st>>>(d_indptr, cols, (const float2 *)vals, (int32_t *)d_indices, (float *)d_data);
                else k_csr_sort<float, int32_t, false><<<grid, kBlock, 0, st>>>(d_indptr, cols, (const float2 *)vals, (int32_t *)d_indices, (float *)d_data);
            } else {
                if (cx) k_csr_sort<double, int32_t, true><<<grid, kBlock, 0, st>>>(d_indptr, cols, (const double2 *)vals, (int32_t *)d_indices, (double *)d_data);
                else k_csr_sort<double, int32_t, false><<<grid, kBlock, 0, st>>>(d_indptr, cols, (const double2 *)vals, (int32_t *)d_indices, (double *)d_data);
            }
        } else {
            if (f32) {
                if (cx) k_csr_sort<float, int64_t, true><<<grid, kBlock, 0, st>>>(d_indptr, cols, (const float2 *)vals, (int64_t *)d_indices, (float *)d_data);
                else k_csr_sort<float, int64_t, false><<<grid, kBlock, 0, st>>>(d_indptr, cols, (const float2 *)vals, (int64_t *)d_indices, (float *)d_data);
            } else {
                if (cx) k_csr_sort<double, int64_t, true><<<grid, kBlock, 0, st>>>(d_indptr, cols, (const double2 *)vals, (int64_t *)d_indices, (double *)d_data);
                else k_csr_sort<double, int64_t, false><<<grid, kBlock, 0, st>>>(d_indptr, cols, (const double2 *)vals, (int64_t *)d_indices, (double *)d_data);
            }
        }
        if (hipStreamSynchronize(st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "CSR fill failed: %s", hipGetErrorString(hipGetLastError()));
    }
    dev_free(cols);
    dev_free(vals);
    if (nnz_out) *nnz_out = nnz;
    return rc;
}

extern "C" int qsd_ham_work_counts(const qsd_ham *h, int64_t *probes, int64_t *hits, void *stream) {
    clear_error();
    if (!h) return fail(QSD_ERR_INVALID_ARG, "ham is NULL");
    AllocScope scope(&h->alloc, stream);
    hipStream_t st = (hipStream_t)stream;
    unsigned long long *acc = nullptr;
    QSD_TRY(dev_alloc(&acc, 2));
    unsigned long long hv[2] = {0, 0};
    int rc = QSD_OK;
    if (hipMemcpyAsync(acc, hv, 16, hipMemcpyHostToDevice, st) != hipSuccess) rc = fail(QSD_ERR_HIP, "copy failed");
    if (rc == QSD_OK) {
        const unsigned g = grid_for(h->N, kBlock);
        switch (h->Wp) {
            case 1: k_probe_count<1><<<g, kBlock, 0, st>>>(sview(h->s), view_of(h, false), acc); break;
            case 2: k_probe_count<2><<<g, kBlock, 0, st>>>(sview(h->s), view_of(h, false), acc); break;
            case 4: k_probe_count<4><<<g, kBlock, 0, st>>>(sview(h->s), view_of(h, false), acc); break;
            case 8: k_probe_count<8><<<g, kBlock, 0, st>>>(sview(h->s), view_of(h, false), acc); break;
            case 16: k_probe_count<16><<<g, kBlock, 0, st>>>(sview(h->s), view_of(h, false), acc); break;
        }
        if (hipMemcpyAsync(hv, acc, 16, hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "work count failed: %s", hipGetErrorString(hipGetLastError()));
    }
    dev_free(acc);
    if (rc != QSD_OK) return rc;
    if (probes) *probes = (int64_t)hv[0];
    if (hits) *hits = (int64_t)hv[1];
    return QSD_OK;
}

namespace {
// part[block] = min over the block's chunk of d[i] among values > floor (INFINITY if none)
__global__ __launch_bounds__(256) void k_min_above(const double *__restrict__ d, int64_t N, double floor,
                                                   double *__restrict__ part) {
    __shared__ double ws[4];
    double m = INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256)
        if (d[i] > floor) m = fmin(m, d[i]);
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) m = fmin(m, __shfl_xor(m, k, 64));
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmin(fmin(ws[0], ws[1]), fmin(ws[2], ws[3]));
}
}  // namespace

extern "C" int qsd_ham_diag_splitting(const qsd_ham *h, double *lowest, double *splitting, void *stream) {
    clear_error();
    if (!h) return fail(QSD_ERR_INVALID_ARG, "NULL handle");
    AllocScope scope(&h->alloc, stream);
    hipStream_t st = (hipStream_t)stream;
    constexpr int kParts = 1024;
    double *part = nullptr;
    QSD_TRY(dev_alloc(&part, kParts));
    std::vector<double> hp(kParts);
    double lo = INFINITY, next = INFINITY;
    int rc = QSD_OK;
    for (int pass = 0; pass < 2 && rc == QSD_OK; ++pass) {
        k_min_above<<<kParts, 256, 0, st>>>(h->diag, h->N, pass == 0 ? -INFINITY : lo, part);
        if (hipMemcpyAsync(hp.data(), part, kParts * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(QSD_ERR_HIP, "diagonal reduction failed");
            break;
        }
        double m = INFINITY;
        for (double v : hp) m = std::fmin(m, v);
        (pass == 0 ? lo : next) = m;
    }
    dev_free(part);
    if (rc != QSD_OK) return rc;
    if (lowest) *lowest = lo;
    if (splitting) *splitting = std::isinf(next) ? 0.0 : next - lo;
    return QSD_OK;
}

namespace qsd {
namespace {

// The per-row bits that the slot-order schedules split the SpMV by (built once per operator).
int ensure_rowbits(qsd_ham *h, hipStream_t st) {
    if (h->rowbits || h->N == 0) return QSD_OK;
    uint64_t *bits = nullptr;
    QSD_TRY(dev_alloc(&bits, (size_t)((h->N + 63) / 64)));
    const unsigned g = grid_for(h->N, kBlock);
    switch (h->Wp) {
        case 1: k_row_bits<1><<<g, kBlock, 0, st>>>(sview(h->s), view_of(h, false), bits); break;
        case 2: k_row_bits<2><<<g, kBlock, 0, st>>>(sview(h->s), view_of(h, false), bits); break;
        case 4: k_row_bits<4><<<g, kBlock, 0, st>>>(sview(h->s), view_of(h, false), bits); break;
        case 8: k_row_bits<8><<<g, kBlock, 0, st>>>(sview(h->s), view_of(h, false), bits); break;
        case 16: k_row_bits<16><<<g, kBlock, 0, st>>>(sview(h->s), view_of(h, false), bits); break;
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
        dev_free(bits);
        return fail(QSD_ERR_HIP, "row bits failed: %s", hipGetErrorString(hipGetLastError()));
    }
    h->rowbits = bits;
    return QSD_OK;
}

}  // namespace
}  // namespace qsd

extern "C" int qsd_ham_set_schedule(qsd_ham *h, uint32_t schedule) {
    clear_error();
    if (!h) return fail(QSD_ERR_INVALID_ARG, "NULL handle");
    if (schedule & ~kSchedBits) return fail(QSD_ERR_INVALID_ARG, "unknown schedule bits 0x%x", schedule);
    if ((schedule & QSD_SCHED_SLOT_ORDER) && !h->rowbits) {
        // no caller stream here: wait for all work on the device (the tables may still be
        // being written on another stream), then build on the default stream
        if (hipDeviceSynchronize() != hipSuccess) return fail(QSD_ERR_HIP, "device synchronize failed");
        AllocScope scope(&h->alloc, nullptr);
        QSD_TRY(ensure_rowbits(h, nullptr));
    }
    h->schedule = schedule;
    return QSD_OK;
}

extern "C" int qsd_ham_get_schedule(const qsd_ham *h, uint32_t *schedule) {
    clear_error();
    if (!h || !schedule) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    *schedule = h->schedule;
    return QSD_OK;
}

extern "C" int qsd_ham_autotune(qsd_ham *h, int32_t nvec, int32_t dtype, int32_t reps, uint32_t flags,
                                qsd_tune_result *result, void *stream) {
    clear_error();
    if (!h) return fail(QSD_ERR_INVALID_ARG, "NULL handle");
    if (nvec < 1 || nvec > 16) return fail(QSD_ERR_INVALID_ARG, "nvec must be in [1, 16]");
    if (reps < 1) return fail(QSD_ERR_INVALID_ARG, "reps must be >= 1");
    if (flags & ~(QSD_TUNE_SCHEDULE | QSD_TUNE_LOAD | QSD_TUNE_SPLIT)) return fail(QSD_ERR_INVALID_ARG, "unknown tuning flags");
    QSD_TRY(check_dtype(h, dtype));
    AllocScope scope(&h->alloc, stream);
    hipStream_t st = (hipStream_t)stream;
    qsd_subspace *sub = const_cast<qsd_subspace *>(h->s);
    const size_t esz = dtype == QSD_F64 ? 8 : dtype == QSD_F32 ? 4 : dtype == QSD_C128 ? 16 : 8;
    const size_t bytes = (size_t)h->N * nvec * esz;
    uint8_t *x = nullptr, *y = nullptr;
    QSD_TRY(dev_alloc(&x, bytes));
    int rc = dev_alloc(&y, bytes);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == QSD_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(QSD_ERR_HIP, "event create failed");
    if (rc == QSD_OK && hipMemsetAsync(x, 0, bytes, st) != hipSuccess) rc = fail(QSD_ERR_HIP, "memset failed");
    auto time_it = [&](float &ms_out) -> int {
        QSD_TRY(qsd_matvec(h, nvec, x, nvec, y, nvec, dtype, st));  // warm-up
        QSD_CHECK_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) QSD_TRY(qsd_matvec(h, nvec, x, nvec, y, nvec, dtype, st));
        QSD_CHECK_HIP(hipEventRecord(e1, st));
        QSD_CHECK_HIP(hipEventSynchronize(e1));
        QSD_CHECK_HIP(hipEventElapsedTime(&ms_out, e0, e1));
        ms_out /= reps;
        return QSD_OK;
    };
    if (rc == QSD_OK && (flags & QSD_TUNE_SCHEDULE)) rc = ensure_rowbits(h, st);
    const uint32_t sched0 = h->schedule;
    const int64_t C0 = sub->C;
    const int32_t split0 = sub->split;
    const double load0 = (double)sub->N / (double)sub->C;
    float ms_before = INFINITY, best_ms = INFINITY;
    if (rc == QSD_OK) rc = time_it(ms_before);
    uint32_t best_sched = sched0;
    double best_load = load0;
    int32_t best_split = split0;
    auto consider = [&](uint32_t sc, double l, float &ms) -> int {
        h->schedule = sc;
        QSD_TRY(time_it(ms));
        if (ms < best_ms) {
            best_ms = ms;
            best_sched = sc;
            best_load = l;
            best_split = sub->split;
        }
        return QSD_OK;
    };
    // every schedule on the current table, then the three fastest on every other table
    std::vector<std::pair<float, uint32_t>> ranked;
    if (flags & QSD_TUNE_SCHEDULE) {
        for (uint32_t sc = 0; sc <= kSchedAll && rc == QSD_OK; ++sc) {
            float ms = 0.0f;
            rc = consider(sc, load0, ms);
            ranked.push_back({ms, sc});
        }
        std::sort(ranked.begin(), ranked.end());
        if (ranked.size() > 3) ranked.resize(3);
    } else {
        ranked.push_back({0.0f, sched0});
    }
    // candidate tables: load x part-filter split (none, or at the middle qubit)
    std::vector<int32_t> splits{split0};
    if ((flags & QSD_TUNE_SPLIT) && h->s->n_qubits >= 2) splits.push_back(split0 ? 0 : h->s->n_qubits / 2);
    std::vector<std::pair<double, int32_t>> tables;
    // with a product map the SpMV does not read the table: its load changes nothing
    const bool sweep_load = (flags & QSD_TUNE_LOAD) && !(sub->prank && !(h->schedule & QSD_SCHED_HASH_LOOKUP));
    for (size_t k = 0; k < splits.size(); ++k) {
        if (sweep_load)
            for (double l : {0.03125, 0.0625, 0.125, 0.25, 0.5}) tables.push_back({l, splits[k]});
        else if (k > 0)
            tables.push_back({load0, splits[k]});
    }
    for (auto &tb : tables) {
        if (rc != QSD_OK) break;
        if ((rc = qsd_subspace_rehash(sub, tb.first, tb.second, stream)) != QSD_OK) break;
        if (sub->C == C0 && sub->split == split0 && (flags & QSD_TUNE_SCHEDULE)) {
            // the starting table, already timed under every schedule
            if (best_load == load0 && best_split == split0) best_load = tb.first;
            continue;
        }
        for (auto &p : ranked) {
            float ms = 0.0f;
            if ((rc = consider(p.second, tb.first, ms)) != QSD_OK) break;
        }
    }
    // keep the best table and schedule (or restore the starting ones after an error)
    if (rc == QSD_OK) {
        rc = qsd_subspace_rehash(sub, best_load, best_split, stream);
        h->schedule = best_sched;
    } else {
        h->schedule = sched0;
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    dev_free(x);
    dev_free(y);
    if (rc != QSD_OK) return rc;
    if (result) {
        result->schedule = best_sched;
        result->capacity = sub->C;
        result->max_load = best_load;
        result->split = sub->split;
        result->ms = best_ms;
        result->ms_before = ms_before;
    }
    return QSD_OK;
}
