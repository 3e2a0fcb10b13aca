// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "qsd.h"

namespace qsd {

// Error state (thread-local message) -------------------------------------------------
int fail(int code, const char *fmt, ...);
void clear_error();

#define QSD_CHECK_HIP(call)                                                                            \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return ::qsd::fail(QSD_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),    \
                               __FILE__, __LINE__);                                                    \
    } while (0)

#define QSD_TRY(expr)                                                                                  \
    do {                                                                                               \
        int rc_ = (expr);                                                                              \
        if (rc_ != QSD_OK) return rc_;                                                                 \
    } while (0)

constexpr int kMaxLadder = 4;   // ladder-integer ranges for groups of up to 4 ladder letters
constexpr int kMaxWords = 16;   // widest compiled key: 16 x 64 = 1024 qubits
constexpr int kBlock = 256;     // threads per workgroup for row kernels
constexpr uint32_t kSchedAll = QSD_SCHED_XCD_REMAP | QSD_SCHED_SLOT_ORDER | QSD_SCHED_LOCKSTEP | QSD_SCHED_FILTER_FIRST;
constexpr uint32_t kSchedBits = kSchedAll | QSD_SCHED_HASH_LOOKUP;  // every valid schedule bit

// Padded word count used by the kernels: 1, 2, 4, 8 or 16.
inline int padded_words(int n_qubits) {
    int W = (n_qubits + 63) / 64;
    int Wp = 1;
    while (Wp < W) Wp <<= 1;
    return Wp;
}

// GF(2)-linear hash of a bit-string: XOR of one fixed pseudo-random 64-bit word per set
// bit.  Linearity gives hash(row ^ mask) = hash(row) ^ hash(mask), so a probe for the
// column of any group costs one XOR once the row's hash is known.  The home slot is the low
// log2(C) bits, the tag the high 32.
//
uint64_t qubit_hash_value(int q);  // pseudo-random word of qubit q
void hash_words(int n_qubits, std::vector<uint64_t> &z);  // z[q] per qubit
void part_words(int n_qubits, int split, std::vector<uint32_t> &pz);  // packed part-index word per qubit
void hash_byte_tables(int Wp, const std::vector<uint64_t> &z, std::vector<uint64_t> &tab);  // [Wp*8][256]

// Device memory ----------------------------------------------------------------------
// Every device allocation goes through the allocator of the current scope: each entry point
// opens an AllocScope with the allocator of the handle it works for (or the one the caller
// passes) and its stream; outside any scope, or with a NULL allocator, hipMalloc / hipFree.
struct AllocScope {
    AllocScope(const qsd_allocator *a, void *stream);
    ~AllocScope();
    AllocScope(const AllocScope &) = delete;
    AllocScope &operator=(const AllocScope &) = delete;

  private:
    const qsd_allocator *prev_a;
    void *prev_s;
};
void *raw_alloc(size_t bytes);  // NULL on failure
void raw_free(void *p);
bool custom_allocator();         // the current scope has a caller's allocator

// The allocator a handle keeps (a copy of the caller's; all NULL = hipMalloc / hipFree).
inline qsd_allocator keep_allocator(const qsd_allocator *a) {
    qsd_allocator k{nullptr, nullptr, nullptr};
    if (a && a->alloc && a->free) k = *a;
    return k;
}

template <class T>
int dev_alloc(T **p, size_t count) {
    if (count == 0) count = 1;
    *p = (T *)raw_alloc(count * sizeof(T));
    if (!*p) return fail(QSD_ERR_OUT_OF_MEMORY, "device allocation of %zu bytes failed", count * sizeof(T));
    return QSD_OK;
}
template <class T>
void dev_free(T *&p) {
    raw_free((void *)p);
    p = nullptr;
}

// Hash of every off-diagonal group's flip mask under the subspace's hash words, and its packed
// part indices under the subspace's part words.
std::vector<uint64_t> group_hashes(const qsd_op *op, const std::vector<uint64_t> &z);
std::vector<uint32_t> group_parts(const qsd_op *op, const std::vector<uint32_t> &pz);

// Device-wide exclusive scan of int64 counts (in place allowed); n elements.
int exclusive_scan_i64(const int64_t *d_in, int64_t *d_out, int64_t n, hipStream_t stream);

}  // namespace qsd

// ------------------------------------------------------------------- handle contents

// The rows of a subspace in slot order (the order of their slots in the hash table), with their
// keys and hashes in that order; rebuilt with the table.
struct SlotRows {
    uint32_t *order = nullptr;  // [N] row index of each position
    uint64_t *keys = nullptr;   // [Wp][N]
    uint64_t *hkey = nullptr;   // [N]
    uint32_t *pkey = nullptr;   // [N] packed part indices (with part filters)
};
namespace qsd {
inline void free_rows(SlotRows &r) {
    dev_free(r.order);
    dev_free(r.keys);
    dev_free(r.hkey);
    dev_free(r.pkey);
}
}  // namespace qsd

struct qsd_subspace {
    qsd_allocator alloc{nullptr, nullptr, nullptr};  // device memory of this handle (all NULL: hipMalloc)
    void *stream = nullptr;                          // stream of the build (frees at destroy)
    int32_t n_qubits = 0;
    int32_t W = 0;   // words per string
    int32_t Wp = 0;  // padded words used by kernels
    int64_t N = 0;   // unique strings
    int64_t C = 0;   // hash slots (power of two)
    uint64_t *keys = nullptr;    // [Wp][N] word planes, ascending order
    uint64_t *hkey = nullptr;    // [N] linear hash of each key
    uint64_t *slots = nullptr;   // [C] (tag << 32) | index, empty = ~0
    uint32_t *bitmap = nullptr;  // [C / 32] slot occupancy
    uint64_t *ztab = nullptr;    // [Wp * 8][256] byte tabulation of the hash
    SlotRows rows;               // the rows in slot order
    bool exact = false;          // slots carry displacements (see device.h)
    std::vector<uint64_t> z;     // hash word of each qubit (host copy of what ztab tabulates)
    // Part filters (none when split = 0): the qubits below `split` form the low part, the others
    // the high part; pz[q] is qubit q's word of the packed part index (high << 16 | low), a
    // GF(2)-linear map (the identity on a part of at most 16 qubits, pseudo-random otherwise).
    int32_t split = 0;
    std::vector<uint32_t> pz;
    uint32_t *pfilt = nullptr;   // [kPartWords] low-part filter, then high-part filter
    uint32_t *pkey = nullptr;    // [N] packed part indices of the rows (canonical order)
    // Product map (parts of at most 16 qubits, and N = (low parts) x (high parts), so that the
    // subspace is the Cartesian product of its parts): word prefix counts of both filters.
    uint16_t *prank = nullptr;   // [kPartWords]
    uint32_t pna = 0;            // number of distinct low parts
    // operators bound to this subspace: their group hashes follow the hash words on a rehash
    mutable std::vector<qsd_ham *> bound;
};

// Whether slots of a table with C slots may use the exact layout: one-word keys, indices below
// 2^26, and the n qubit hash words, restricted to the bits that the home slot and the tag keep,
// linearly independent over GF(2) (then the map key -> (home slot, tag) is injective).
namespace qsd {
bool exact_tags_ok(const std::vector<uint64_t> &z, int W, int64_t N, int64_t C);
}

struct Letter {
    int32_t q;
    uint8_t code;
};

struct CompiledTerm {
    std::vector<Letter> word;  // ascending qubit
    std::complex<double> c;    // coefficient of the word
};

struct qsd_op {
    int32_t n_qubits = 0;
    int32_t Wp = 0;
    bool is_complex = false;
    std::vector<CompiledTerm> terms;      // group order; group 0 = diagonal
    std::vector<int64_t> group_ptr;       // G + 1
    std::vector<int32_t> group_ladder;    // G
    // Device-table images (host), built by the compiler -------------------------------
    // diagonal terms: care/want/sign words and c' = c * (-i)^{#Y}
    std::vector<uint64_t> diag_cws;       // [Td][3][Wp]
    std::vector<double> diag_coef;        // [Td][2]
    // off-diagonal groups
    std::vector<uint64_t> g_mask;         // [G-1][Wp] (their hashes depend on the subspace)
    std::vector<uint64_t> g_pos;          // [G-1] four 16-bit ladder positions
    std::vector<uint64_t> g_scan;         // [G-1] scan record: live table over 4 bits | 4 x 12-bit shifts
    std::vector<uint32_t> g_info;         // [G-1] k | ladder<<3 | care<<4 | live16<<16
    std::vector<uint32_t> g_term0;        // [G-1] first off-diagonal term
    std::vector<uint32_t> g_nterm;        // [G-1]
    std::vector<uint16_t> g_iptr;         // [G-1][kIptr] ladder ranges relative to g_term0
    std::vector<uint64_t> t_cws;          // [To][3][Wp]
    std::vector<double> t_coef;           // [To][2]
    // strings of at most 32 qubits: at the first term of each ladder range, the qubits of the
    // range's projector tail (its last terms, one per qubit in increasing order, each wanting
    // its one qubit beyond the flip mask set); 0 elsewhere
    std::vector<uint32_t> t_tail;         // [To]
    int64_t max_group_terms = 0;
};

constexpr int kIptr = 18;  // 2^4 + 1 pointers, padded to an even count

// Packed group descriptor bits.
constexpr uint32_t kInfoKMask = 7u;
constexpr uint32_t kInfoLadder = 1u << 3;
constexpr uint32_t kInfoCare = 1u << 4;

struct qsd_ham {
    qsd_allocator alloc{nullptr, nullptr, nullptr};
    void *stream = nullptr;
    const qsd_subspace *s = nullptr;
    const qsd_op *op = nullptr;
    int64_t N = 0;
    int64_t G = 0;   // off-diagonal groups
    int32_t Wp = 0;
    bool is_complex = false;
    // QSD_SCHED_* bits of the SpMV launch (results do not depend on it)
    uint32_t schedule = QSD_SCHED_XCD_REMAP | QSD_SCHED_FILTER_FIRST;
    double *diag = nullptr;       // [N] real part (FP64)
    double *diag_im = nullptr;    // [N] imaginary part (complex operators only)
    uint64_t *g_mask = nullptr;
    uint64_t *g_hash = nullptr;
    uint32_t *g_part = nullptr;   // [G] packed part indices (subspaces with part filters)
    uint64_t *g_pos = nullptr;
    uint64_t *g_scan = nullptr;
    uint32_t *g_info = nullptr;
    uint32_t *g_term0 = nullptr;
    uint32_t *g_nterm = nullptr;
    uint16_t *g_iptr = nullptr;
    uint64_t *t_cws = nullptr;
    uint32_t *t_cw32 = nullptr;   // [To][4] care, want, sign as 32-bit words, 0 (n_qubits <= 32)
    double *t_coef = nullptr;     // [To][2]
    float *t_coef32 = nullptr;    // [To][2]
    float *diag32 = nullptr;      // [N]
    float *diag32_im = nullptr;
    // [ceil(N / 64)] bit r = row r has an off-diagonal element; built for the slot-order schedules
    uint64_t *rowbits = nullptr;
};

struct qsd_csr {
    qsd_allocator alloc{nullptr, nullptr, nullptr};
    void *stream = nullptr;
    int64_t N = 0;
    int64_t nnz = 0;
    int32_t index_type = QSD_INDEX_I32;
    int32_t dtype = QSD_F64;
    bool cplx = false;
    int64_t *indptr = nullptr;  // [N + 1]
    void *indices = nullptr;    // [nnz] int32 or int64
    void *data = nullptr;       // [nnz] (x2 for complex) FP64 or FP32
    double *diag = nullptr;     // [N] real part of the diagonal (start vectors)
    int lpr = 1;                // SpMV lanes per row
};

namespace qsd {
// The operator an eigensolver applies: matrix-free (a bound Hamiltonian) or a stored CSR matrix.
struct SpmvOp {
    const qsd_ham *h = nullptr;
    const qsd_csr *c = nullptr;
    int64_t N() const { return c ? c->N : h->N; }
    bool is_complex() const { return c ? c->cplx : h->is_complex; }
    const double *diag() const { return c ? c->diag : h->diag; }
    const qsd_allocator *allocator() const { return c ? &c->alloc : &h->alloc; }
    bool takes(int32_t dtype) const { return !c || c->dtype == dtype; }
    int matvec(int nvec, const void *x, int64_t ldx, void *y, int64_t ldy, int32_t dtype, hipStream_t st) const {
        return c ? qsd_csr_matvec(c, nvec, x, ldx, y, ldy, dtype, st) : qsd_matvec(h, nvec, x, ldx, y, ldy, dtype, st);
    }
};
}  // namespace qsd
