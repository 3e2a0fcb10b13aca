/*
 * qsd.h - C-ABI of the MI355X (gfx950) subspace-Hamiltonian library.
 *
 * The library evaluates a Hamiltonian written over an extended operator alphabet on a subspace
 * of computational-basis bit-strings (Nation, Saki, Kang, "A generalized framework for quantum
 * subspace diagonalization", arXiv 2603.18731):
 *
 *   - bit-set subspaces of any width, hashed for lookup        (Methods, Subspace data structure)
 *   - operators over {Z, 0, 1, X, Y, -, +} and fermionic terms  (Methods, Hamiltonian representations)
 *   - grouping by off-diagonal structure and ladder integers    (Methods, Qubit / Fermionic Hamiltonians)
 *   - cached diagonal, matrix-free SpMV and two-pass CSR        (Methods, Matrix evaluation)
 *   - a ground-state Lanczos eigensolver built on the SpMV      (not in the paper, which hands the
 *                                                                operator to external eigensolvers)
 *
 * Conventions for every call:
 *   - The return value is a status code (QSD_OK = 0, negative on error).  On error a message
 *     is available from qsd_last_error() (per calling thread) and no output is valid.
 *   - Pointers documented "device" are HIP device (HBM) addresses on the current device;
 *     "host" pointers are ordinary CPU memory.  The library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is enqueued
 *     asynchronously on it unless a call is documented to synchronize.
 *   - Handles are created by *_build / *_compile / *_create and released by *_destroy.  A
 *     handle is immutable after creation; concurrent read-only use on several streams is
 *     safe.  Destroying a handle that is still referenced (a subspace or operator bound in a
 *     live qsd_ham) is the caller's error.
 *   - Bit-strings: qubit q is bit (q % 64) of 64-bit word (q / 64); W = ceil(n_qubits / 64)
 *     words per string (Supplemental Material, MSOB section: bit indexing starts from the
 *     right).  Bits at positions >= n_qubits must be zero.
 *   - Subspace index: strings are sorted ascending as unsigned integers (word W-1 most
 *     significant) and deduplicated; the index of a string is its rank (Methods, Lower /
 *     upper triangle evaluation).
 *   - Matrix convention: H_ij = <b_i|H|b_j>, y = H x.
 */
#ifndef QSD_H
#define QSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
#define QSD_OK 0
#define QSD_ERR_INVALID_ARG (-1)   /* malformed input; nothing was enqueued */
#define QSD_ERR_OUT_OF_MEMORY (-2) /* a device or host allocation failed */
#define QSD_ERR_HIP (-3)           /* a HIP runtime call failed */
#define QSD_ERR_CAPACITY (-4)      /* a size exceeds what the requested index type can hold */
#define QSD_ERR_NOT_HERMITIAN (-5) /* QSD_OP_CHECK_HERMITIAN failed */
#define QSD_ERR_NOT_CONVERGED (-6) /* Lanczos stopped at max_iter; outputs hold the best estimate */
#define QSD_ERR_DTYPE (-7)         /* dtype does not match the operator (real vs complex) */
#define QSD_ERR_UNSUPPORTED (-8)   /* a valid request outside what the library implements */

/* ----------------------------------------------------------------- value types */
#define QSD_F64 0  /* double */
#define QSD_F32 1  /* float elements and vectors, double accumulation */
#define QSD_C128 2 /* double complex, interleaved (re, im) */
#define QSD_C64 3  /* float complex, double accumulation */

#define QSD_INDEX_I32 0
#define QSD_INDEX_I64 1

/* -------------------------------------------------- extended alphabet (Methods, Qubit Hamiltonians) */
#define QSD_Z 0     /* Pauli Z */
#define QSD_P0 1    /* projector |0><0| */
#define QSD_P1 2    /* projector |1><1| */
#define QSD_X 3     /* Pauli X */
#define QSD_Y 4     /* Pauli Y */
#define QSD_LOWER 5 /* |0><1|; with QSD_OP_FERMIONIC: annihilator f */
#define QSD_RAISE 6 /* |1><0|; with QSD_OP_FERMIONIC: creator f^dagger */

/* --------------------------------------------------------------------- flags */
#define QSD_SUB_ASSUME_SORTED_UNIQUE 1u /* input is already ascending and duplicate-free */

#define QSD_OP_FERMIONIC 1u       /* terms are products of f / f^dagger (codes 5 / 6) */
#define QSD_OP_CHECK_HERMITIAN 2u /* fail with QSD_ERR_NOT_HERMITIAN unless H = H^dagger */
#define QSD_OP_FORCE_COMPLEX 4u   /* treat the matrix as complex even if every element is real */
#define QSD_OP_NO_LADDER_INT 8u   /* evaluate every group without ladder-integer ranges (ablation) */
#define QSD_OP_ORDER_BY_MASK 16u  /* order groups by flip mask only (default: weight, then mask) */
/* order groups by the halves of the qubits (below / from n_qubits / 2) they flip: low half only,
 * both, high half only; groups that flip both by the high half's flip, then weight, then the
 * low half's; the others by weight, then flip mask.  Groups that flip the high part of a string
 * alike then sit together, which lets a block of rows that share their high part (an alpha x
 * beta product subspace split at n_qubits / 2) reject them in bulk. */
#define QSD_OP_ORDER_BY_PARTS 32u

typedef struct qsd_subspace qsd_subspace;
typedef struct qsd_op qsd_op;
typedef struct qsd_ham qsd_ham;

/* ------------------------------------------------------------------ device memory
 * Every creating call (and every call that needs scratch) takes its device memory from a
 * caller-supplied allocator, so that a framework's caching allocator (PyTorch's, in the Python
 * binding) sees and accounts for every byte; NULL (or NULL function pointers) selects
 * hipMalloc / hipFree.
 *   alloc(ctx, bytes, stream)  returns `bytes` of device memory on the current device, usable
 *                              by work enqueued on `stream` (the stream of the library call),
 *                              or NULL when it cannot (the call then fails with
 *                              QSD_ERR_OUT_OF_MEMORY after releasing what it took).
 *   free(ctx, ptr, stream)     returns ptr; the library calls it once all of its work that
 *                              uses ptr has been enqueued on `stream` (stream-ordered release:
 *                              the allocator may hand the block to later work on that stream).
 * A handle keeps a copy of its allocator (ctx must outlive the handle) and releases its memory
 * through it when destroyed, on the stream it was created on; the caller must not destroy a
 * handle while work using it is pending on another stream.  Scratch of a call on a handle comes
 * from the handle's allocator unless the call takes an allocator of its own.  The library never
 * calls the allocator from another thread than the caller's. */
typedef struct {
    void *ctx;
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*free)(void *ctx, void *ptr, void *stream);
} qsd_allocator;

/* Message of the last failing call on this thread ("" if none).  Valid until the next call. */
const char *qsd_last_error(void);

/* Library version as an integer (major * 10000 + minor * 100 + patch). */
int qsd_version(void);

/* ============================================================ subspace (bit-set hash map)
 *
 * qsd_subspace_build - Methods, Subspace data structure.
 *   Copies, sorts and deduplicates n_in bit-strings and builds the lookup table: open
 *   addressing with linear probing over 2^k slots holding {32-bit tag, 32-bit index}, plus
 *   one occupancy bit per slot tested before any slot is read (the paper's bucket-occupancy
 *   bit-set).  k is the smallest power of two with N / 2^k <= max_load.
 *   d_bits    device, [n_in][W] uint64 row-major; read only during the call's stream work.
 *   n_in      number of input strings (>= 1).
 *   n_qubits  >= 1.  W = ceil(n_qubits / 64).
 *   flags     QSD_SUB_* bits.
 *   max_load  hash load factor in (0, 0.5]; 0 selects 0.125 (a low load lets most absent strings
 *             stop at an empty occupancy bit).
 *   alloc     device memory of the handle and of the build's scratch (NULL: hipMalloc).
 *   out       receives the new handle.
 *   A subspace of 2 to 32 qubits that is the Cartesian product of the distinct strings of its
 *   lower n_qubits / 2 qubits and those of its upper qubits (an alpha x beta product) is given
 *   part filters split there and the product map (qsd_subspace_hash_info); otherwise no part
 *   filters.  qsd_subspace_rehash changes either.
 *   Synchronizes `stream` (the unique count N is read back).  Errors: INVALID_ARG if n_in < 1,
 *   n_qubits < 1, a bit >= n_qubits is set, or max_load is out of range; CAPACITY if
 *   N >= 2^32 - 1; UNSUPPORTED if W exceeds the widest compiled key (see qsd_max_qubits).
 */
int qsd_subspace_build(const uint64_t *d_bits, int64_t n_in, int32_t n_qubits, uint32_t flags, double max_load,
                       const qsd_allocator *alloc, void *stream, qsd_subspace **out);

/* Largest n_qubits the library supports. */
int32_t qsd_max_qubits(void);

/* Sizes of a built subspace: N unique strings, n_qubits, W words per string, hash capacity
 * (slots).  Any output pointer may be NULL. */
int qsd_subspace_info(const qsd_subspace *s, int64_t *N, int32_t *n_qubits, int32_t *W, int64_t *capacity);

/* Rebuilds the hash table (slots, occupancy bitmap, slot order of the rows) for a new max_load in
 * (0, 0.5] (0 = the default 1/8), and the part filters for `split`; keys, canonical indices and
 * every lookup and SpMV result are unchanged.
 *   split  0: no part filters.  s in [1, n_qubits): the qubits below s form a string's low part,
 *          the others its high part, and two bitmaps record which low parts and which high parts
 *          occur in the subspace (parts of at most 16 qubits index them directly, longer parts
 *          through a 16-bit GF(2)-linear image).  A column b ^ M_g whose low or high part does
 *          not occur cannot be a member, so the row engine rejects it from the bitmaps (kept in
 *          LDS for keys of up to 128 qubits) without touching the hash table; a column that
 *          passes reads its home slot directly.  This is the membership test the occupancy
 *          bitmap gives (Methods, Subspace data structure), made cheap for subspaces built as
 *          Cartesian products of alpha and beta strings (Results): split at the first beta
 *          qubit, a column passes only if both its alpha and its beta string were sampled.
 * The subspace must not be in use on any stream meanwhile (operators bound to it through
 * qsd_ham_create are updated; serving requests hold the old table and must be removed first).
 * Synchronizes.  INVALID_ARG for max_load or split out of range. */
int qsd_subspace_rehash(qsd_subspace *s, double max_load, int32_t split, void *stream);

/* Split qubit of the part filters (0 = none), whether slots use the exact layout (one-word
 * keys whose (home slot, tag) pair is injective), and whether the subspace has a product map.
 * A product map exists when both parts have at most 16 qubits and the subspace is exactly the
 * Cartesian product of its distinct low parts and its distinct high parts (the alpha x beta
 * product subspaces of Results, fermionic examples): then a string (l, h) has the canonical
 * index rank(h) * |low parts| + rank(l), which the SpMV reads off the part filters instead of
 * probing the table.  Any output pointer may be NULL. */
int qsd_subspace_hash_info(const qsd_subspace *s, int32_t *split, int32_t *exact, int32_t *product);

/* New subspace of the strings whose byte in d_mask[N] (device) is nonzero, in the same order
 * (indices renumbered consecutively), with a table for max_load (0 = default).  INVALID_ARG when
 * the mask selects nothing.  Synchronizes. */
int qsd_subspace_select(const qsd_subspace *s, const uint8_t *d_mask, double max_load, void *stream,
                        qsd_subspace **out);

/* Copies the canonical (sorted, unique) strings to device memory d_out, [N][W] row-major. */
int qsd_subspace_keys(const qsd_subspace *s, uint64_t *d_out, void *stream);

/* Index lookup through the hash table: d_idx[i] = index of d_q[i] ([n][W] device) or -1.
 * Strings with bits >= n_qubits set are reported absent. */
int qsd_subspace_lookup(const qsd_subspace *s, const uint64_t *d_q, int64_t n, int64_t *d_idx, void *stream);

/* Probe-length statistics of the hash table (host outputs, synchronizes): mean and maximum
 * number of occupied slots inspected by a successful lookup of every stored string. */
int qsd_subspace_probe_stats(const qsd_subspace *s, double *mean_probe, int64_t *max_probe, void *stream);

int qsd_subspace_destroy(qsd_subspace *s);

/* ==================================================================== operator compile
 *
 * qsd_op_compile - Methods, Hamiltonian representations.  Host-only (no device work).
 *   Input is a flat list of terms c_t * word_t, word_t = product of single-qubit letters:
 *   term t has letters op_code[term_ptr[t] .. term_ptr[t+1]) acting on qubits op_idx[...],
 *   coefficient (coef_reim[2t], coef_reim[2t+1]).  An empty word is the identity.  Terms with
 *   a zero coefficient are ignored.
 *   Qubit mode: letters are QSD_Z..QSD_RAISE on distinct qubits (any order).
 *   QSD_OP_FERMIONIC: letters are QSD_LOWER (f) / QSD_RAISE (f^dagger) in product order; indices
 *   may repeat.  Each term is brought to ascending index order with the sign of every exchange
 *   of operators on different modes, repeated modes are merged with the 16 rules of
 *   Supplemental Table S1, and the extended Jordan-Wigner map (f_j -> |0><1|_j with Z on
 *   every lower qubit) produces a word over {Z, 0, 1, -, +}.
 *   Both modes then combine equal words (sum of coefficients; a word whose coefficients cancel
 *   is kept), split off the diagonal group (no off-diagonal letter), group off-diagonal words
 *   by their off-diagonal qubit set (ordered by set size, then by the set as an integer) and,
 *   inside a group whose off-diagonal letters are all ladders on at most 4 qubits, sort terms
 *   by ladder integer ('-' -> 0, '+' -> 1, k-th lowest qubit -> bit k) with 2^k + 1 range
 *   pointers.
 *   trim_tol  group trimming (Results, CH4-dimer runs): a group is the set of input terms with
 *             the same flip mask (X, Y, raise and lower letters of a qubit word; every ladder
 *             operator of a fermionic word flips its mode); the modulus of its matrix elements
 *             is bounded by the sum of |c| over its input terms, and groups whose bound is
 *             below trim_tol are dropped before compilation (diagonal terms never are).
 *             0 keeps everything; negative is INVALID_ARG.  The paper's relative tolerance is
 *             trim_tol = tol * qsd_ham_diag_splitting of the subspace.
 *   All arrays are host memory and are not retained.
 *   Errors: INVALID_ARG (index out of range, bad code, repeated qubit in qubit mode, NaN);
 *   NOT_HERMITIAN with QSD_OP_CHECK_HERMITIAN when some word's adjoint does not carry the
 *   conjugate coefficient (relative tolerance 1e-12).
 */
int qsd_op_compile(int32_t n_qubits, int64_t n_terms, const int64_t *term_ptr, const int32_t *op_idx,
                   const uint8_t *op_code, const double *coef_reim, uint32_t flags, double trim_tol, qsd_op **out);

/* Sizes of a compiled operator: T compiled terms, total letters, G groups (the diagonal
 * group counts as one), whether the matrix is complex, n_qubits.  Any pointer may be NULL. */
int qsd_op_info(const qsd_op *op, int64_t *T, int64_t *n_letters, int64_t *G, int32_t *is_complex,
                int32_t *n_qubits);

/* Exports the compiled terms (host buffers sized from qsd_op_info): term_ptr[T+1],
 * op_idx / op_code [n_letters] (ascending qubit per term, qubit-alphabet codes),
 * coef_reim[2T], group_ptr[G+1] (group 0 = diagonal terms, possibly empty), and
 * group_ladder[G] (1 if the group uses ladder-integer ranges).  Terms appear in group order,
 * each group sorted by ladder integer where applicable.  Any output pointer may be NULL. */
int qsd_op_export(const qsd_op *op, int64_t *term_ptr, int32_t *op_idx, uint8_t *op_code, double *coef_reim,
                  int64_t *group_ptr, int32_t *group_ladder);

int qsd_op_destroy(qsd_op *op);

/* ============================================================ subspace Hamiltonian
 *
 * qsd_ham_create - Methods, Matrix evaluation ("SubspaceHamiltonian").  Binds a subspace and
 *   an operator with the same n_qubits, uploads the group and term tables and computes the
 *   diagonal d_i = H_ii once (projector letters tested before any sign is formed).  The
 *   handle references `s` and `op`; they must outlive it.  flags: reserved, pass 0.
 *   alloc: device memory of the handle and the scratch of later calls on it (NULL: hipMalloc).
 *   Enqueued on `stream`.
 */
int qsd_ham_create(const qsd_subspace *s, const qsd_op *op, uint32_t flags, const qsd_allocator *alloc, void *stream,
                   qsd_ham **out);

/* Copies the cached diagonal (FP64 real part; imaginary parts of a Hermitian H are zero) to
 * device d_out[N]. */
int qsd_ham_diagonal(const qsd_ham *h, double *d_out, void *stream);

int qsd_ham_destroy(qsd_ham *h);

/* Sizes: N rows, G groups. */
int qsd_ham_info(const qsd_ham *h, int64_t *N, int64_t *G, int32_t *is_complex);

/* Work of one SpMV, counted by a separate pass (synchronizes): `probes` = (row, group) pairs
 * that the group filter leaves live (a non-empty ladder-integer range): the subspace lookups of
 * the method, whether the hash table, the part filters or the product map answers them;
 * `hits` = those whose column is in the subspace and whose range has a term passing the row's
 * projector bits (the off-diagonal stored entries).  Host outputs; either may be NULL. */
int qsd_ham_work_counts(const qsd_ham *h, int64_t *probes, int64_t *hits, void *stream);

/* Lowest diagonal element of H over the subspace and the smallest diagonal energy splitting,
 * read as the gap from it to the next larger distinct diagonal value (0 if all are equal): the
 * scale of group trimming (Results, CH4-dimer runs).  Host outputs (either may be NULL);
 * synchronizes. */
int qsd_ham_diag_splitting(const qsd_ham *h, double *lowest, double *splitting, void *stream);

/* SpMV schedule (launch shape only: every schedule gives bitwise the same results, since each
 * row is evaluated by one lane in the same group order whatever workgroup runs it).
 *   QSD_SCHED_XCD_REMAP   workgroups dispatched to one XCD take contiguous row tiles, so rows
 *                         whose columns and probes overlap share that XCD's L2.
 *   QSD_SCHED_SLOT_ORDER  a workgroup takes 256 consecutive rows of the slot order (the rows
 *                         listed by the position of their slot in the hash table, kept with the
 *                         table) instead of the canonical order.  The hash is linear, so the
 *                         columns b ^ M_g of rows whose slots are neighbours are neighbours too.
 *                         The launch then also writes y = d x, in canonical order, for the rows
 *                         without off-diagonal elements, and the slot-order rows write only the
 *                         rows that have some (per-row bits built once per operator, N / 8
 *                         bytes, by the first qsd_ham_set_schedule or qsd_ham_autotune call that
 *                         needs them; that call synchronizes).
 *   QSD_SCHED_LOCKSTEP    the 64 lanes of a wave probe the same group in the same instruction
 *                         (lanes whose row does not have it live sit idle) instead of each lane
 *                         walking its own live groups; with SLOT_ORDER the wave's occupancy-bit
 *                         loads for one group then fall in one or two cache lines.
 *   QSD_SCHED_FILTER_FIRST  a lane first reads the occupancy bits of all its live groups'
 *                         home slots (8 loads in flight), then the slots of the occupied ones
 *                         (4 in flight), instead of reading bit and slot group by group.
 *   QSD_SCHED_HASH_LOOKUP  columns are looked up in the hash table even when the subspace has a
 *                         product map (qsd_subspace_hash_info); without it they take their
 *                         index from the map and the table is not read.  Not swept by the
 *                         autotuner (the map needs no memory access).
 * A new operator starts with XCD_REMAP | FILTER_FIRST (faster than the plain schedule on every
 * workload measured; slot order pays off when most probes miss, which qsd_ham_autotune finds).
 * The batched entries (qsd_batch_*, qsd_matvec_batched) use each operator's schedule too.
 * qsd_ham_set_schedule sets the bits (INVALID_ARG for unknown bits). */
#define QSD_SCHED_XCD_REMAP 1u
#define QSD_SCHED_SLOT_ORDER 2u
#define QSD_SCHED_LOCKSTEP 4u
#define QSD_SCHED_FILTER_FIRST 8u
#define QSD_SCHED_HASH_LOOKUP 16u
int qsd_ham_set_schedule(qsd_ham *h, uint32_t schedule);
int qsd_ham_get_schedule(const qsd_ham *h, uint32_t *schedule);

/* Autotuner (not in the paper).  Times `reps` SpMVs (nvec vectors of `dtype`, internal buffers)
 * with HIP events for every candidate and keeps the fastest:
 *   QSD_TUNE_SCHEDULE  every schedule above (on the current table);
 *   QSD_TUNE_LOAD      hash-table loads 1/32, 1/16, 1/8, 1/4, 1/2 (with the three fastest
 *                      schedules when both flags are set; not swept when the subspace has a
 *                      product map, whose SpMV does not read the table): the table is rebuilt
 *                      (qsd_subspace_rehash), so the subspace must not be used meanwhile by
 *                      any other handle, batch or stream.  The best table depends on how the
 *                      occupancy bitmap and the slots fit the caches.
 *   QSD_TUNE_SPLIT     also the other part-filter choice (split at qubit n_qubits / 2 if the
 *                      subspace has none, none if it has one), at every load swept (or the
 *                      current load without QSD_TUNE_LOAD).
 * None changes any result bit.  `result` (host, may be NULL) receives the choice, the time
 * per SpMV before and after.  Synchronizes; allocates 2 N nvec elements while it runs. */
#define QSD_TUNE_SCHEDULE 1u
#define QSD_TUNE_LOAD 2u
#define QSD_TUNE_SPLIT 4u
typedef struct {
    uint32_t schedule; /* QSD_SCHED_* bits kept */
    int64_t capacity;  /* hash slots kept */
    double max_load;   /* load parameter of the kept table */
    int32_t split;     /* split qubit of the kept part filters (0 = none) */
    double ms;         /* SpMV time with the kept choice */
    double ms_before;  /* SpMV time before tuning */
} qsd_tune_result;
int qsd_ham_autotune(qsd_ham *h, int32_t nvec, int32_t dtype, int32_t reps, uint32_t flags, qsd_tune_result *result,
                     void *stream);

/* ==================================================================== matrix-free SpMV
 *
 * qsd_matvec - Methods, Matrix evaluation (matrix-free).  Y = H X for `nvec` vectors at once:
 *   every row evaluates each group once (ladder-integer range, column by XOR with the group
 *   mask, one hash probe, projector refinement, popcount-parity signs) and applies the element
 *   to all nvec vectors.
 *   Layout: interleaved, element (row j, vector v) at X[j * ldx + v] (nvec <= ldx < 2^31),
 *   likewise Y.
 *   dtype: QSD_F64 / QSD_F32 for a real matrix, QSD_C128 / QSD_C64 for a complex one
 *   (ld counts complex elements).  F32/C64 store elements and vectors in single precision and
 *   accumulate each row in double.
 *   1 <= nvec <= 16.  X and Y must not overlap.  Y is overwritten.
 */
int qsd_matvec(const qsd_ham *h, int32_t nvec, const void *d_x, int64_t ldx, void *d_y, int64_t ldy, int32_t dtype,
               void *stream);

/* Y_i = H_i X_i for n independent requests in one launch per key width (per chunk of four
 * complex vectors; requests on product subspaces, which take the product map, in a launch of
 * their own): the row tiles of all requests form one grid, so small subspaces share the GPU
 * instead of each under-filling it.  Per request: hams[i], device vectors xs[i] and ys[i]
 * with nvecs[i] (1..16) interleaved vectors (leading dimension nvecs[i]); dtype as for
 * qsd_matvec, the same for all requests and matching every operator (DTYPE otherwise).  Every
 * row is evaluated exactly as by qsd_matvec, so the results are bitwise those of n separate
 * calls.  The request table is uploaded to stream-ordered memory (hipMallocAsync) on `stream`;
 * the call does not synchronize.  Not in the paper (serving pattern). */
int qsd_matvec_batched(int32_t n, const qsd_ham *const *hams, const void *const *xs, void *const *ys,
                       const int32_t *nvecs, int32_t dtype, void *stream);

/* qsd_matvec_batched_noalloc - for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): qsd_matvec_batched with
 * the same arguments, kernels and results (bitwise), but its request and tile tables go to a
 * fixed device array of the library (under 1 MiB) instead of stream-ordered memory.  The call makes no
 * hipMalloc, hipFree, hipMallocAsync or allocator call.  Limits: at most
 * QSD_NOALLOC_MAX_REQUESTS request chunks (one per request and launch: a real request of up to 16
 * vectors is one chunk, a complex request one per four vectors) and QSD_NOALLOC_MAX_TILES row
 * tiles of 256 rows in total; beyond either it returns CAPACITY before touching the GPU.
 * Each GPU holds its own array until the process ends, and every call on that GPU shares it:
 * calls that overlap on one GPU (different streams or host threads without ordering between
 * them) race on the tables.  Calls in order on one stream are safe; the array keeps the last
 * call's tables, and each call rewrites all it reads before its kernels start. */
#define QSD_NOALLOC_MAX_REQUESTS 256
#define QSD_NOALLOC_MAX_TILES 65536
int qsd_matvec_batched_noalloc(int32_t n, const qsd_ham *const *hams, const void *const *xs, void *const *ys,
                               const int32_t *nvecs, int32_t dtype, void *stream);

/* ============================================================================= CSR
 *
 * qsd_csr_build - Methods, Matrix evaluation (two-pass CSR).
 *   Call 1 with d_indices == d_data == NULL: writes d_indptr[N+1] (int64, device), returns
 *   nnz in *nnz_out (synchronizes).  The caller allocates indices[nnz] and data[nnz].
 *   Call 2 with all pointers: fills column indices (ascending within each row; type
 *   QSD_INDEX_I32 or QSD_INDEX_I64) and values (dtype as for qsd_matvec).
 *   An entry (i, j) is stored iff j == i, or b_j is in the subspace and at least one term's
 *   element between b_i and b_j is nonzero (the stored value may cancel to 0.0).
 *   Errors: CAPACITY for QSD_INDEX_I32 with N >= 2^31.
 */
int qsd_csr_build(const qsd_ham *h, int64_t *d_indptr, void *d_indices, void *d_data, int32_t index_type,
                  int32_t dtype, int64_t *nnz_out, void *stream);

/* ========================================================================== Lanczos */
#define QSD_V0_UNIFORM 0  /* all ones, normalized */
#define QSD_V0_MIN_DIAG 1 /* unit spike at the smallest diagonal entry (lowest index on ties) */
#define QSD_V0_RANDOM 2   /* uniform [-1, 1) entries from a counter-based generator (seed) */
#define QSD_V0_USER 3     /* read from d_evec on entry */

typedef struct {
    int32_t max_iter;    /* Krylov dimension limit (default 300) */
    double tol;          /* stop when beta_k |s_k| <= tol |theta| (default 1e-10) */
    int32_t v0_mode;     /* QSD_V0_* */
    uint64_t seed;       /* QSD_V0_RANDOM */
    int32_t spmv_dtype;  /* QSD_F64 or QSD_F32 (real) / QSD_C128 or QSD_C64 (complex) */
    int32_t check_every; /* iterations between convergence checks (default 5) */
    int32_t want_vector; /* write the normalized Ritz vector to d_evec */
    int32_t use_graph;   /* capture one iteration in a HIP graph and replay it */
    const qsd_allocator *alloc; /* basis and work vectors (NULL: the operator's allocator) */
} qsd_lanczos_opts;

typedef struct {
    int32_t iterations;
    int32_t converged;
    double ritz_residual;     /* beta_k |s_k| at exit */
    double explicit_residual; /* ||H x - theta x|| / |theta| in FP64 (if want_vector) */
    double matvec_ms;         /* GPU time in SpMV (HIP events) */
    double total_ms;          /* wall time of the call */
} qsd_lanczos_info;

/* Fills opts with the defaults above. */
void qsd_lanczos_default_opts(qsd_lanczos_opts *opts);

/* Lowest eigenvalue of H (Hermitian) by Lanczos with full reorthogonalization (classical
 * Gram-Schmidt applied twice), FP64 basis and recurrence, tridiagonal eigenproblem by Sturm
 * bisection plus inverse iteration on the device.
 *   eval_out  host, receives theta.
 *   d_evec    device [N] (FP64, or complex FP64 for a complex H): Ritz vector if want_vector,
 *             start vector if v0_mode == QSD_V0_USER; may be NULL otherwise.
 *   A complex Hermitian H runs the same recurrence on interleaved complex vectors (projections
 *   conj(v)^T w, alpha the real part); spmv_dtype F64 / F32 then means C128 / C64 SpMV.
 *   info      host, may be NULL.
 * Synchronizes.  Returns NOT_CONVERGED (with outputs filled) if max_iter is reached.
 * The basis needs (max_iter + 1) * N * 8 bytes (x2 for complex) of device memory.
 */
int qsd_lanczos(const qsd_ham *h, const qsd_lanczos_opts *opts, double *eval_out, void *d_evec,
                qsd_lanczos_info *info, void *stream);

/* Block Lanczos (not in the paper): `block` (4, 8 or 16) vectors per step, so every hash probe
 * of the SpMM serves `block` vectors.  max_iter counts block steps: at most 80 for blocks of 4
 * and 8, 40 for blocks of 16 (the Ritz solve keeps T's band in one workgroup's LDS).  Block
 * classical Gram-Schmidt applied twice against the whole basis, Cholesky QR applied twice for
 * the next block, FP64 basis and recurrence;
 * spmv_dtype F32 stores SpMM elements and vectors in single precision with FP64 accumulation.
 * The lowest eigenvalue of the block tridiagonal T is found on the device by bisection with a
 * banded Cholesky positive-definiteness test, its eigenvector by inverse iteration; the
 * residual estimate is || B_k s_last ||.
 *   opts->max_iter   block steps, 1 .. 80 (capped at N / block - 1).
 *   opts->v0_mode    sets the first column of the start block (USER: d_evec); the other
 *                    columns are random (splitmix64 of seed, column, row).
 *   eval_out, d_evec, info, use_graph, check_every: as for qsd_lanczos (info->iterations counts
 *   block steps).
 * Synchronizes.  Returns NOT_CONVERGED (outputs filled) at the step limit or after a
 * rank-deficient residual block; INVALID_ARG if the subspace is smaller than 2 * block.
 * The basis needs (max_iter + 1) * N * block * 8 bytes of device memory.
 */
int qsd_block_lanczos(const qsd_ham *h, int32_t block, const qsd_lanczos_opts *opts, double *eval_out, void *d_evec,
                      qsd_lanczos_info *info, void *stream);

/* ============================================================ stored CSR operator
 *
 * qsd_csr_create - Methods, Matrix evaluation (CSR output) and Lower / upper triangle
 *   evaluation.  Builds the CSR matrix of `h` (same entries as qsd_csr_build: structural
 *   entries, columns ascending per row) and keeps it on the device for repeated SpMVs.
 *   flags 0: two passes over all rows (structure, then values).
 *   QSD_CSR_LOWER_MIRROR: each row evaluates only the groups whose column sorts below it (the
 *   row bit at the group's most significant off-diagonal bit is set), so every element is
 *   evaluated once; each entry is written into its row and, conjugated, into the column's row
 *   (atomic cursors), then rows are sorted.  Requires a Hermitian operator (the upper triangle
 *   is taken as the conjugate of the lower one).
 *   index_type QSD_INDEX_I32 / I64 (CAPACITY if N >= 2^31 with I32); dtype as for
 *   qsd_csr_build (F64 / F32 real, C128 / C64 complex; DTYPE if it does not match `h`).
 *   Synchronizes.  Device memory (from `alloc`, NULL: hipMalloc): (N + 1) * 8 + nnz * (index +
 *   value size), plus the build's scratch of nnz * (8 + 2 * value size) bytes while it runs.
 *   `h` may be destroyed after.
 * qsd_csr_info      N, nnz, device bytes held.
 * qsd_csr_export    copies indptr [N+1] (int64), indices [nnz], data [nnz] to device buffers
 *                   (any may be NULL); async on `stream`.
 * qsd_csr_matvec    Y = A X, same layout and dtype rules as qsd_matvec except that the vector
 *                   dtype must be the stored dtype (DTYPE otherwise).  LPR lanes per row with a
 *                   fixed reduction tree: bitwise reproducible.  Async.
 * qsd_csr_lanczos / qsd_csr_block_lanczos
 *                   qsd_lanczos / qsd_block_lanczos on the stored matrix (opts->spmv_dtype must
 *                   be the stored dtype).
 * qsd_csr_destroy   frees the matrix.
 */
#define QSD_CSR_LOWER_MIRROR 1u
typedef struct qsd_csr qsd_csr;
int qsd_csr_create(const qsd_ham *h, int32_t index_type, int32_t dtype, uint32_t flags, const qsd_allocator *alloc,
                   void *stream, qsd_csr **out);
int qsd_csr_info(const qsd_csr *c, int64_t *N, int64_t *nnz, int64_t *bytes);
int qsd_csr_export(const qsd_csr *c, int64_t *d_indptr, void *d_indices, void *d_data, void *stream);
int qsd_csr_matvec(const qsd_csr *c, int32_t nvec, const void *d_x, int64_t ldx, void *d_y, int64_t ldy, int32_t dtype,
                   void *stream);
int qsd_csr_lanczos(const qsd_csr *c, const qsd_lanczos_opts *opts, double *eval_out, void *d_evec,
                    qsd_lanczos_info *info, void *stream);
int qsd_csr_block_lanczos(const qsd_csr *c, int32_t block, const qsd_lanczos_opts *opts, double *eval_out,
                          void *d_evec, qsd_lanczos_info *info, void *stream);
int qsd_csr_destroy(qsd_csr *c);

/* ====================================================================== RAMPS
 *
 * qsd_ramps - Supplement, Recursive algorithm for a minimal perturbative subspace (Algorithm
 *   S1), restricted to the operator's subspace S_full (columns outside S_full are not
 *   followed), frontier-parallel on the device.  Every state of S_0 (host indices s0[n0] into
 *   S_full) starts a walk with prefactor 1/E; a frontier entry (j, pre) visits each off-diagonal
 *   element H_jk of its row with k in S_full and k not in S_0, forms
 *   amp = (pre * |H_jk|^2) / (E - H_kk) (in this order, no fused operations), and when
 *   |amp| > tau selects k and continues from it with prefactor amp / (E - H_kk).  A column
 *   reached along several paths is carried once per path.  Levels stop when the frontier is
 *   empty or after max_depth levels (then info->truncated = 1).
 *   d_selected  device [N] bytes, out: 1 for S_0 and every selected column, else 0.
 *   n_selected  host, out (may be NULL); info host, out (may be NULL).
 *   max_frontier  paths one level may hold; CAPACITY when a level needs more (outputs then
 *   undefined).  Real or complex H (|H_jk|^2).  Synchronizes once per level.
 *   Device memory: N bytes + 32 * max_frontier bytes.
 * Follow with qsd_subspace_select to build the trimmed subspace.
 */
typedef struct {
    int32_t levels;       /* levels run */
    int32_t truncated;    /* 1 if max_depth stopped a non-empty frontier */
    int64_t paths;        /* frontier entries created over all levels */
    int64_t max_frontier; /* largest level */
    int64_t selected;     /* strings in the output subspace */
} qsd_ramps_info;
int qsd_ramps(const qsd_ham *h, const int64_t *s0, int64_t n0, double E, double tau, int32_t max_depth,
              int64_t max_frontier, uint8_t *d_selected, int64_t *n_selected, qsd_ramps_info *info, void *stream);

/* ========================================================= batched Lanczos (serving)
 *
 * Many ground-state solves advance together: qsd_batch_step takes one Lanczos iteration (the
 * same algorithm as qsd_lanczos: FP64 basis, classical Gram-Schmidt applied twice) for every
 * active request with one SpMV launch over all requests' rows and a fixed number of BLAS
 * launches, so requests of different sizes share the GPU at iteration granularity (continuous
 * batching: requests are added and removed between steps).  A request's reductions are
 * partitioned by its own size only, so its iterates are bitwise identical alone and in any
 * mix.  Not in the paper (it hands its operator to external eigensolvers).
 *
 * qsd_batch_create     up to max_requests slots, at most max_iter iterations per request,
 *                      SpMV in spmv_dtype (QSD_F64, or QSD_F32 with FP64 accumulation); the
 *                      batch's own tables and library-allocated workspaces come from `alloc`
 *                      (NULL: hipMalloc).
 * qsd_batch_footprint  device bytes of one request's workspace for `h` (Krylov basis, work
 *                      vectors, partial sums, tridiagonal state).
 * qsd_batch_add        binds a real operator `h` (it must outlive the request) and starts
 *                      its Lanczos run from v0_mode (UNIFORM, MIN_DIAG or RANDOM(seed)); the
 *                      request converges when beta_k |s_k| <= tol |theta|.  `workspace` is
 *                      device memory of at least qsd_batch_footprint bytes, 256-byte aligned,
 *                      owned by the caller and kept valid until the slot is removed and the
 *                      work enqueued before has finished; NULL makes the library allocate it
 *                      (the batch's allocator) and free it at removal.  All requests of a batch must have
 *                      the same key width.  Errors: CAPACITY (no free slot), OUT_OF_MEMORY,
 *                      UNSUPPORTED (complex operator or other key width), INVALID_ARG (empty
 *                      subspace, short or misaligned workspace).  Synchronizes `stream`.
 * qsd_batch_add_csr    the same for a stored CSR operator (int32 columns, dtype = the batch's
 *                      SpMV dtype): its rows are evaluated from the matrix by the same lanes-per-row
 *                      reduction as qsd_csr_matvec, inside the same batched launch; requests of
 *                      both kinds and any key width mix freely.  The matrix must outlive the request.
 * qsd_batch_footprint_rows  workspace bytes for a request of N rows.
 * qsd_batch_step       `iterations` iterations for every active request (requests at their
 *                      limit idle).  Enqueued on `stream`.
 * qsd_batch_poll       solves every active request's tridiagonal problem and reports, per
 *                      slot (host arrays of max_requests entries, any may be NULL): status
 *                      0 free, 1 running, 2 converged, 3 iteration limit; energy (theta);
 *                      iterations taken; Ritz residual estimate.  Synchronizes.
 * qsd_batch_remove     frees a slot; a library-allocated workspace is released after the
 *                      device has finished the work enqueued on it.
 */
typedef struct qsd_batch qsd_batch;
int qsd_batch_create(int32_t max_requests, int32_t max_iter, int32_t spmv_dtype, const qsd_allocator *alloc,
                     qsd_batch **out);
int qsd_batch_footprint(const qsd_ham *h, int32_t max_iter, int32_t spmv_dtype, int64_t *bytes);
int qsd_batch_add(qsd_batch *b, const qsd_ham *h, int32_t v0_mode, uint64_t seed, double tol, void *workspace,
                  int64_t workspace_bytes, int32_t *slot_out, void *stream);
int qsd_batch_add_csr(qsd_batch *b, const qsd_csr *c, int32_t v0_mode, uint64_t seed, double tol, void *workspace,
                      int64_t workspace_bytes, int32_t *slot_out, void *stream);
int qsd_batch_footprint_rows(int64_t N, int32_t max_iter, int32_t spmv_dtype, int64_t *bytes);
int qsd_batch_step(qsd_batch *b, int32_t iterations, void *stream);
int qsd_batch_poll(qsd_batch *b, int32_t *status, double *energy, int32_t *iterations, double *ritz_residual,
                   void *stream);
int qsd_batch_remove(qsd_batch *b, int32_t slot);
int qsd_batch_destroy(qsd_batch *b);

/* ====================================================================== diagnostics */

#ifdef __cplusplus
}
#endif
#endif /* QSD_H */
