// Batched Lanczos for serving: many ground-state solves advance together, one iteration per
// step for every active request, with one SpMV launch and a fixed set of BLAS launches per
// iteration whatever the number of requests (continuous batching at iteration granularity).
//
// Requests are independent: every reduction of a request is partitioned by its own size only
// (2048-row tiles, summed in a fixed order), and its SpMV rows are evaluated exactly as by
// qsd_matvec, so a request's iterates are bitwise the same alone and in any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"
#include "matvec.h"
#include "tridiag.h"

namespace qsd {
namespace {

constexpr int kBT = 2048;  // rows per BLAS tile

struct ReqDev {
    SubView s;
    HamView h;
    const double *diag;
    const float *diag32;
    int64_t N;
    double *V;  // [m+1][N]
    double *x, *w;
    float *x32, *w32;
    double *part;  // [(m+1)][nbt]
    double *hv;    // [m+1]
    double *alpha, *beta;
    int *kdev;
    double *tri;  // [m+4]
    int m;
    int nbt;
    // stored CSR operator (int32 columns) instead of the row engine, when cptr is set
    const int64_t *cptr;
    const int32_t *cidx;
    const void *cval;
    int lpr;
    uint32_t sched;  // the operator's QSD_SCHED_* bits (row order and probe mode)
};

struct Tile {
    int slot;
    int idx;
};

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Row tiles of a request on a product subspace whose low-part count pna spans two or more tiles
// (and not in slot order): tile k of high part b takes rows b pna + 256 k .. (b + 1) pna, so its
// rows share their high part, as in qsd_matvec.  pm_tiles = how many (0: plain 256-row tiles).
__host__ __device__ inline int64_t pm_tiles(int64_t N, uint32_t pna, uint32_t sched) {
    if (pna < 2u * kBlock || (sched & QSD_SCHED_SLOT_ORDER)) return 0;
    return N / pna * ((pna + kBlock - 1) / kBlock);
}
__device__ __forceinline__ void pm_tile(uint32_t pna, uint32_t sched, int idx, int64_t &row0, int64_t &row_end) {
    if (pna < 2u * kBlock || (sched & QSD_SCHED_SLOT_ORDER)) return;
    const int64_t tpb = (pna + kBlock - 1) / kBlock, b = idx / tpb;
    row0 = b * (int64_t)pna + (idx - b * tpb) * kBlock;
    row_end = (b + 1) * (int64_t)pna;
}

// PF = 2: the tiles of matrix-free requests on product subspaces (product map); else PF = 1.
template <int Wp, class ET, int PF = 1>
__global__ __launch_bounds__(kBlock) void kb_matvec(const ReqDev *__restrict__ reqs, const Tile *__restrict__ tiles) {
    __shared__ ChunkLds<Wp> lds;
    const Tile t = tiles[blockIdx.x];
    const ReqDev &R = reqs[t.slot];
    if (*R.kdev >= R.m) return;  // at its iteration limit (uniform for the block)
    const bool f32 = std::is_same<ET, float>::value;
    const ET *dre = f32 ? (const ET *)R.diag32 : (const ET *)R.diag;
    const ET *x = f32 ? (const ET *)R.x32 : (const ET *)R.x;
    ET *y = f32 ? (ET *)R.w32 : (ET *)R.w;
    if (R.cptr) {
        // stored CSR: groups of lpr consecutive lanes take the tile's rows in turn; entries are
        // strided over a group's lanes and summed by the same shuffle tree as qsd_csr_matvec
        const int lpr = R.lpr;
        const int sub = threadIdx.x & (lpr - 1);
        const int64_t row0 = (int64_t)t.idx * kBlock, rend = min(R.N, row0 + kBlock);
        const ET *val = (const ET *)R.cval;
        for (int64_t r = row0 + threadIdx.x / lpr; r < row0 + kBlock; r += kBlock / lpr) {
            double acc = 0.0;
            if (r < rend) {
                const int64_t a = R.cptr[r], b = R.cptr[r + 1];
                // four entries (and their x gathers) in flight per lane, taken in order; past the
                // row's end the loads repeat its last entry and the term is skipped
                for (int64_t e = a + sub; e < b; e += 4 * lpr) {
                    double v[4], xv[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int64_t ek = min(e + (int64_t)k * lpr, b - 1);
                        v[k] = (double)val[ek];
                        xv[k] = (double)x[R.cidx[ek]];
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (e + (int64_t)k * lpr < b) acc += v[k] * xv[k];
                }
            }
            for (int d = lpr / 2; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
            if (sub == 0 && r < rend) y[r] = (ET)acc;
        }
        return;
    }
    // the operator's schedule, with the diagonal term formed in the row kernel (no separate pass)
    int64_t row0 = (int64_t)t.idx * kBlock, row_end = -1;
    if constexpr (PF == 2) pm_tile(R.s.pna, R.sched, t.idx, row0, row_end);
    matvec_block<Wp, 1, ET, false, PF>(R.s, R.h, dre, nullptr, x, 1, y, 1, 1, row0, lds,
                                       (R.sched & QSD_SCHED_SLOT_ORDER) != 0, (R.sched & QSD_SCHED_LOCKSTEP) != 0,
                                       (R.sched & QSD_SCHED_FILTER_FIRST) != 0, false, row_end);
}

// x32 = x (to_f32) or w = w32 (back), over 2048-row tiles
__global__ __launch_bounds__(256) void kb_convert(const ReqDev *__restrict__ reqs, const Tile *__restrict__ tiles,
                                                  int to_f32) {
    const Tile t = tiles[blockIdx.x];
    const ReqDev &R = reqs[t.slot];
    if (*R.kdev >= R.m) return;
    const int64_t a = (int64_t)t.idx * kBT, b = min(R.N, a + kBT);
    for (int64_t i = a + threadIdx.x; i < b; i += 256) {
        if (to_f32)
            R.x32[i] = (float)R.x[i];
        else
            R.w[i] = (double)R.w32[i];
    }
}

// part[j][tile] = sum over the tile's rows of V[j][i] w[i], j = 0..k; blockIdx.y selects
// kBJ basis vectors (w read once per row for all of them), block sums by a fixed tree.
constexpr int kBJ = 8;

__global__ __launch_bounds__(256) void kb_gemv_t(const ReqDev *__restrict__ reqs, const Tile *__restrict__ tiles) {
    __shared__ double red[kBJ][4];
    const Tile t = tiles[blockIdx.x];
    const ReqDev &R = reqs[t.slot];
    if (*R.kdev >= R.m) return;
    const int cnt = *R.kdev + 1;
    const int j0 = blockIdx.y * kBJ;
    if (j0 >= cnt) return;  // uniform for the block
    const int nj = min(kBJ, cnt - j0);
    const int64_t a = (int64_t)t.idx * kBT, b = min(R.N, a + kBT);
    double acc[kBJ];
#pragma unroll
    for (int q = 0; q < kBJ; ++q) acc[q] = 0.0;
    const double *v0 = R.V + (int64_t)j0 * R.N;
    for (int64_t i = a + threadIdx.x; i < b; i += 256) {
        const double wi = R.w[i];
#pragma unroll
        for (int q = 0; q < kBJ; ++q)
            if (q < nj) acc[q] += v0[(int64_t)q * R.N + i] * wi;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kBJ; ++q) {
        const double s = wsum(acc[q]);
        if (lane == 0) red[q][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < nj)
        R.part[(int64_t)(j0 + threadIdx.x) * R.nbt + t.idx] =
            (red[threadIdx.x][0] + red[threadIdx.x][1]) + (red[threadIdx.x][2] + red[threadIdx.x][3]);
}

// hv[j] = sum of part[j][*] in tile order; alpha[k] += hv[k].  One wave per j, four per block.
__global__ __launch_bounds__(256) void kb_reduce(const ReqDev *__restrict__ reqs, int nslots) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6), slot = blockIdx.y, lane = threadIdx.x & 63;
    if (slot >= nslots) return;
    const ReqDev &R = reqs[slot];
    if (R.N == 0) return;
    const int k = *R.kdev;
    if (k >= R.m || j > k) return;  // whole waves leave together
    double s = 0.0;
    for (int p = lane; p < R.nbt; p += 64) s += R.part[(int64_t)j * R.nbt + p];
    s = wsum(s);
    if (lane == 0) {
        R.hv[j] = s;
        if (j == k) R.alpha[k] += s;
    }
}

// w[i] -= sum_{j <= k} V[j][i] hv[j] over 256-row tiles
__global__ __launch_bounds__(kBlock) void kb_gemv_n_sub(const ReqDev *__restrict__ reqs, const Tile *__restrict__ tiles) {
    const Tile t = tiles[blockIdx.x];
    const ReqDev &R = reqs[t.slot];
    if (*R.kdev >= R.m) return;
    const int cnt = *R.kdev + 1;
    const int64_t i = (int64_t)t.idx * kBlock + threadIdx.x;
    if (i >= R.N) return;
    double acc = 0.0;
    for (int j = 0; j < cnt; ++j) acc += R.V[(int64_t)j * R.N + i] * R.hv[j];
    R.w[i] -= acc;
}

__global__ __launch_bounds__(256) void kb_sq_part(const ReqDev *__restrict__ reqs, const Tile *__restrict__ tiles) {
    __shared__ double ws[4];
    const Tile t = tiles[blockIdx.x];
    const ReqDev &R = reqs[t.slot];
    if (*R.kdev >= R.m) return;  // uniform for the block
    const int64_t a = (int64_t)t.idx * kBT, b = min(R.N, a + kBT);
    double s = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += 256) s += R.w[i] * R.w[i];
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) R.part[t.idx] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(64) void kb_beta(const ReqDev *__restrict__ reqs, int nslots) {
    const int slot = blockIdx.x;
    if (slot >= nslots) return;
    const ReqDev &R = reqs[slot];
    if (R.N == 0 || *R.kdev >= R.m) return;
    double s = 0.0;
    for (int p = threadIdx.x; p < R.nbt; p += 64) s += R.part[p];
    s = wsum(s);
    if (threadIdx.x == 0) R.beta[*R.kdev] = sqrt(s);
}

// x = V[k+1] = w / beta[k] (breakdown: zeros, first breakdown recorded in tri[2])
__global__ __launch_bounds__(kBlock) void kb_next(const ReqDev *__restrict__ reqs, const Tile *__restrict__ tiles) {
    const Tile t = tiles[blockIdx.x];
    const ReqDev &R = reqs[t.slot];
    const int k = *R.kdev;
    if (k >= R.m) return;
    const double b = R.beta[k];
    const double scale = fabs(R.alpha[k]) + (k > 0 ? R.beta[k - 1] : 0.0);
    const bool brk = R.tri[2] != 0.0 || !(b > 1e-12 * scale) || !(b > 1e-300);
    const double inv = brk ? 0.0 : 1.0 / b;
    const int64_t i = (int64_t)t.idx * kBlock + threadIdx.x;
    if (i < R.N) {
        const double v = R.w[i] * inv;
        R.x[i] = v;
        if (k + 1 <= R.m) R.V[(int64_t)(k + 1) * R.N + i] = v;
    }
}

// Breakdown bookkeeping and k += 1, one thread per slot (after kb_next has read k).
__global__ void kb_bump(const ReqDev *__restrict__ reqs, int nslots) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= nslots) return;
    const ReqDev &R = reqs[slot];
    if (R.N == 0) return;
    const int k = *R.kdev;
    if (k >= R.m) return;
    const double b = R.beta[k];
    const double scale = fabs(R.alpha[k]) + (k > 0 ? R.beta[k - 1] : 0.0);
    const bool brk = !(b > 1e-12 * scale) || !(b > 1e-300);
    if (brk && R.tri[2] == 0.0) {
        R.tri[2] = (double)(k + 1);
        R.beta[k] = 0.0;
    }
    if (k + 1 < R.m) *R.kdev = k + 1;
    else *R.kdev = R.m;  // saturates: no further iterations are taken
}

__global__ __launch_bounds__(kTriThreads) void kb_tridiag(const ReqDev *__restrict__ reqs, int nslots,
                                                         double *__restrict__ out /*[nslots][4]*/) {
    __shared__ TridiagLds L;
    const int slot = blockIdx.x;
    const ReqDev &R = reqs[slot];
    if (R.N == 0) return;
    const int done = R.tri[2] != 0.0 ? (int)R.tri[2] : *R.kdev;  // iterations with valid alpha
    if (done < 1) {
        if (threadIdx.x == 0) {
            out[4 * slot + 0] = 0.0;
            out[4 * slot + 1] = INFINITY;
            out[4 * slot + 2] = 0.0;
            out[4 * slot + 3] = 0.0;
        }
        return;
    }
    tridiag_lowest(R.alpha, R.beta, done, R.tri, L);
    if (threadIdx.x == 0) {
        out[4 * slot + 0] = R.tri[0];
        out[4 * slot + 1] = R.tri[2] != 0.0 ? 0.0 : R.tri[1];
        out[4 * slot + 2] = (double)done;
        out[4 * slot + 3] = R.tri[2];
    }
}

__global__ void kb_init(const ReqDev *__restrict__ reqs, int slot, int mode, uint64_t seed, int64_t spike) {
    const ReqDev &R = reqs[slot];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < R.N; i += (int64_t)gridDim.x * blockDim.x) {
        double v;
        if (mode == QSD_V0_UNIFORM) {
            v = 1.0;
        } else if (mode == QSD_V0_MIN_DIAG) {
            v = (i == spike) ? 1.0 : 0.0;
        } else {
            uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            v = (double)(z >> 11) * 0x1.0p-52 - 1.0;
        }
        R.x[i] = v;
    }
}

// x /= ||x||, V[0] = x, alpha = beta = 0, k = 0 (one block: setup only)
__global__ __launch_bounds__(256) void kb_start(const ReqDev *__restrict__ reqs, int slot) {
    __shared__ double ws[4];
    __shared__ double inv;
    const ReqDev &R = reqs[slot];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < R.N; i += 256) s += R.x[i] * R.x[i];
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) inv = 1.0 / sqrt(ws[0] + ws[1] + ws[2] + ws[3]);
    __syncthreads();
    for (int64_t i = threadIdx.x; i < R.N; i += 256) {
        R.x[i] *= inv;
        R.V[i] = R.x[i];
    }
    for (int j = threadIdx.x; j < R.m; j += 256) {
        R.alpha[j] = 0.0;
        R.beta[j] = 0.0;
    }
    if (threadIdx.x < 4) R.tri[threadIdx.x] = 0.0;
    if (threadIdx.x == 0) *R.kdev = 0;
}

__global__ __launch_bounds__(256) void kb_argmin(const double *__restrict__ d, int64_t N, int64_t *__restrict__ out) {
    __shared__ double bv[256];
    __shared__ int64_t bi[256];
    double v = INFINITY;
    int64_t idx = N;
    for (int64_t i = threadIdx.x; i < N; i += 256)
        if (d[i] < v) {
            v = d[i];
            idx = i;
        }
    bv[threadIdx.x] = v;
    bi[threadIdx.x] = idx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < 256; ++t)
            if (bv[t] < v || (bv[t] == v && bi[t] < idx)) {
                v = bv[t];
                idx = bi[t];
            }
        *out = idx;
    }
}


// Batched SpMV over independent operators: tile t of the launch is 256 rows of request
// tiles[t].slot; every row is evaluated exactly as by qsd_matvec.
struct MvReq {
    SubView s;
    HamView h;
    const void *dre, *dim;
    const void *x;
    void *y;
    int64_t ld;      // leading dimension of x and y (the request's vector count)
    int nv;          // vectors of this launch (at most the template width)
    uint32_t sched;  // the operator's QSD_SCHED_* bits (row order and probe mode)
};

// PF = 2: requests on product subspaces (product map, one-word keys); else PF = 1.
template <int Wp, int NV, class ET, bool CPLX, int PF = 1>
__global__ __launch_bounds__(kBlock) void kbm_matvec(const MvReq *__restrict__ reqs, const Tile *__restrict__ tiles) {
    __shared__ ChunkLds<Wp> lds;
    const Tile t = tiles[blockIdx.x];
    const MvReq &R = reqs[t.slot];
    int64_t row0 = (int64_t)t.idx * kBlock, row_end = -1;
    if constexpr (PF == 2) pm_tile(R.s.pna, R.sched, t.idx, row0, row_end);
    matvec_block<Wp, NV, ET, CPLX, PF>(R.s, R.h, (const ET *)R.dre, (const ET *)R.dim, (const ET *)R.x, R.ld, (ET *)R.y,
                                   R.ld, R.nv, row0, lds, (R.sched & QSD_SCHED_SLOT_ORDER) != 0,
                                   (R.sched & QSD_SCHED_LOCKSTEP) != 0, (R.sched & QSD_SCHED_FILTER_FIRST) != 0, false,
                                   row_end);
}

}  // namespace
}  // namespace qsd

using namespace qsd;

struct qsd_batch {
    qsd_allocator alloc{nullptr, nullptr, nullptr};  // tables and library-owned workspaces
    int max_slots = 0;
    int max_iter = 0;
    bool f32 = false;
    int Wp = 0;
    struct Slot {
        bool used = false;
        const qsd_ham *h = nullptr;
        ReqDev d{};
        void *mem = nullptr;      // the request's workspace
        bool owned = false;       // allocated by the library (else the caller's)
        void *stream = nullptr;   // stream of the request's add (an owned workspace is released on it)
        double tol = 1e-10;
        int steps = 0;
    };
    std::vector<Slot> slots;
    ReqDev *d_reqs = nullptr;
    Tile *d_mv = nullptr, *d_bl = nullptr;  // 256-row and 2048-row tiles
    int n_mv = 0, n_bl = 0;
    int n_mv_pm = 0;  // the first n_mv_pm row tiles belong to requests that take the product map
    size_t cap_mv = 0, cap_bl = 0;
    // the product-map SpMV's tiles (pm_tile: within the product's blocks of rows where a block
    // spans two or more tiles, else the 256-row tiles)
    Tile *d_pmt = nullptr;
    int n_pmt = 0;
    size_t cap_pmt = 0;
    double *d_out = nullptr;  // [max_slots][4]
    int64_t *d_spike = nullptr;
    bool dirty = true;
};

namespace {

void free_slot(const qsd_batch *b, qsd_batch::Slot &S) {
    if (S.owned) {
        AllocScope scope(&b->alloc, S.stream);
        dev_free(S.mem);
    }
    S = qsd_batch::Slot();
}

// Workspace layout of one request: every array starts on a 256-byte boundary.
struct Layout {
    int64_t V, x, w, x32, w32, part, hv, alpha, beta, kdev, tri, total;
};

Layout layout_of(int64_t N, int m, bool f32) {
    const int64_t nbt = (N + kBT - 1) / kBT;
    Layout L{};
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    L.V = take((int64_t)(m + 1) * N * 8);
    L.x = take(N * 8);
    L.w = take(N * 8);
    L.x32 = f32 ? take(N * 4) : -1;
    L.w32 = f32 ? take(N * 4) : -1;
    L.part = take((int64_t)(m + 1) * nbt * 8);
    L.hv = take((int64_t)(m + 1) * 8);
    L.alpha = take((int64_t)m * 8);
    L.beta = take((int64_t)m * 8);
    L.kdev = take(8);
    L.tri = take((int64_t)(m + 4) * 8);
    L.total = off;
    return L;
}

int sync_tables(qsd_batch *b, hipStream_t st) {
    if (!b->dirty) return QSD_OK;
    AllocScope scope(&b->alloc, st);
    std::vector<ReqDev> host(b->max_slots);
    std::vector<Tile> mv, mvo, bl, pmt;
    for (int i = 0; i < b->max_slots; ++i) {
        const auto &S = b->slots[i];
        if (!S.used) {
            host[i] = ReqDev{};
            host[i].N = 0;
            continue;
        }
        host[i] = S.d;
        // row tiles of matrix-free requests on product subspaces first (they take the product-map
        // kernel), then the others; no kernel depends on the order of the tiles
        const bool pm = b->Wp == 1 && !S.d.cptr && S.d.s.prank && !(S.d.sched & QSD_SCHED_HASH_LOOKUP);
        for (int64_t t = 0; t < (S.d.N + kBlock - 1) / kBlock; ++t) (pm ? mv : mvo).push_back({i, (int)t});
        if (pm) {
            const int64_t n = pm_tiles(S.d.N, S.d.s.pna, S.d.sched);
            for (int64_t t = 0; t < (n ? n : (S.d.N + kBlock - 1) / kBlock); ++t) pmt.push_back({i, (int)t});
        }
        for (int t = 0; t < S.d.nbt; ++t) bl.push_back({i, t});
    }
    const int n_pm = (int)mv.size();
    mv.insert(mv.end(), mvo.begin(), mvo.end());
    if (mv.size() > b->cap_mv) {
        dev_free(b->d_mv);
        b->cap_mv = mv.size() * 2;
        QSD_TRY(dev_alloc(&b->d_mv, b->cap_mv));
    }
    if (bl.size() > b->cap_bl) {
        dev_free(b->d_bl);
        b->cap_bl = bl.size() * 2;
        QSD_TRY(dev_alloc(&b->d_bl, b->cap_bl));
    }
    if (pmt.size() > b->cap_pmt) {
        dev_free(b->d_pmt);
        b->cap_pmt = pmt.size() * 2;
        QSD_TRY(dev_alloc(&b->d_pmt, b->cap_pmt));
    }
    QSD_CHECK_HIP(hipMemcpyAsync(b->d_reqs, host.data(), host.size() * sizeof(ReqDev), hipMemcpyHostToDevice, st));
    if (!mv.empty()) QSD_CHECK_HIP(hipMemcpyAsync(b->d_mv, mv.data(), mv.size() * sizeof(Tile), hipMemcpyHostToDevice, st));
    if (!bl.empty()) QSD_CHECK_HIP(hipMemcpyAsync(b->d_bl, bl.data(), bl.size() * sizeof(Tile), hipMemcpyHostToDevice, st));
    if (!pmt.empty())
        QSD_CHECK_HIP(hipMemcpyAsync(b->d_pmt, pmt.data(), pmt.size() * sizeof(Tile), hipMemcpyHostToDevice, st));
    // the host vectors are staged by the runtime before the calls return (pageable copies)
    QSD_CHECK_HIP(hipStreamSynchronize(st));
    b->n_mv = (int)mv.size();
    b->n_mv_pm = n_pm;
    b->n_pmt = (int)pmt.size();
    b->n_bl = (int)bl.size();
    b->dirty = false;
    return QSD_OK;
}

// The batched SpMV: product-map tiles in one launch (one-word keys), the others in another.
template <int Wp>
void launch_bmv(qsd_batch *b, hipStream_t st) {
    const int np = Wp == 1 ? b->n_mv_pm : 0, no = b->n_mv - np;
    if (np > 0) {
        if (b->f32)
            kb_matvec<1, float, 2><<<b->n_pmt, kBlock, 0, st>>>(b->d_reqs, b->d_pmt);
        else
            kb_matvec<1, double, 2><<<b->n_pmt, kBlock, 0, st>>>(b->d_reqs, b->d_pmt);
    }
    if (no > 0) {
        if (b->f32)
            kb_matvec<Wp, float><<<no, kBlock, 0, st>>>(b->d_reqs, b->d_mv + np);
        else
            kb_matvec<Wp, double><<<no, kBlock, 0, st>>>(b->d_reqs, b->d_mv + np);
    }
}

}  // namespace

extern "C" int qsd_batch_create(int32_t max_requests, int32_t max_iter, int32_t spmv_dtype, const qsd_allocator *alloc,
                                qsd_batch **out) {
    clear_error();
    if (!out) return fail(QSD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (max_requests < 1 || max_requests > 4096) return fail(QSD_ERR_INVALID_ARG, "max_requests must be in [1, 4096]");
    if (max_iter < 2 || max_iter > 1000) return fail(QSD_ERR_INVALID_ARG, "max_iter must be in [2, 1000]");
    if (spmv_dtype != QSD_F64 && spmv_dtype != QSD_F32) return fail(QSD_ERR_DTYPE, "spmv_dtype must be F64 or F32");
    auto *b = new (std::nothrow) qsd_batch();
    if (!b) return fail(QSD_ERR_OUT_OF_MEMORY, "host allocation failed");
    b->alloc = keep_allocator(alloc);
    AllocScope scope(&b->alloc, nullptr);
    b->max_slots = max_requests;
    b->max_iter = max_iter;
    b->f32 = spmv_dtype == QSD_F32;
    b->slots.resize(max_requests);
    int rc = dev_alloc(&b->d_reqs, max_requests);
    if (rc == QSD_OK) rc = dev_alloc(&b->d_out, 4 * (size_t)max_requests);
    if (rc == QSD_OK) rc = dev_alloc(&b->d_spike, 1);
    if (rc != QSD_OK) {
        dev_free(b->d_reqs);
        dev_free(b->d_out);
        dev_free(b->d_spike);
        delete b;
        return rc;
    }
    *out = b;
    return QSD_OK;
}

extern "C" int qsd_batch_footprint_rows(int64_t N, int32_t max_iter, int32_t spmv_dtype, int64_t *bytes) {
    clear_error();
    if (!bytes || N < 1) return fail(QSD_ERR_INVALID_ARG, "bad arguments");
    if (max_iter < 2 || max_iter > 1000) return fail(QSD_ERR_INVALID_ARG, "max_iter must be in [2, 1000]");
    *bytes = layout_of(N, (int)std::min<int64_t>(max_iter, N), spmv_dtype == QSD_F32).total;
    return QSD_OK;
}

extern "C" int qsd_batch_footprint(const qsd_ham *h, int32_t max_iter, int32_t spmv_dtype, int64_t *bytes) {
    clear_error();
    if (!h || !bytes) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    if (max_iter < 2 || max_iter > 1000) return fail(QSD_ERR_INVALID_ARG, "max_iter must be in [2, 1000]");
    *bytes = layout_of(h->N, (int)std::min<int64_t>(max_iter, h->N), spmv_dtype == QSD_F32).total;
    return QSD_OK;
}

namespace {

int add_impl(qsd_batch *b, const qsd_ham *h, const qsd_csr *c, int32_t v0_mode, uint64_t seed, double tol,
             void *workspace, int64_t workspace_bytes, int32_t *slot_out, void *stream) {
    if (!b || (!h && !c) || !slot_out) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    if (h ? h->is_complex : c->cplx) return fail(QSD_ERR_UNSUPPORTED, "batched Lanczos is real only");
    if (c && c->index_type != QSD_INDEX_I32) return fail(QSD_ERR_UNSUPPORTED, "serving needs int32 CSR columns");
    if (c && c->dtype != (b->f32 ? QSD_F32 : QSD_F64))
        return fail(QSD_ERR_DTYPE, "the stored matrix must have the batch's SpMV dtype");
    if (v0_mode != QSD_V0_UNIFORM && v0_mode != QSD_V0_MIN_DIAG && v0_mode != QSD_V0_RANDOM)
        return fail(QSD_ERR_INVALID_ARG, "v0_mode must be UNIFORM, MIN_DIAG or RANDOM");
    if (!(tol > 0)) return fail(QSD_ERR_INVALID_ARG, "tol must be > 0");
    const int64_t N = h ? h->N : c->N;
    if (N < 1) return fail(QSD_ERR_INVALID_ARG, "empty subspace");
    if (h) {
        bool any = false;
        for (auto &S : b->slots) any |= S.used && S.h;
        if (any && h->Wp != b->Wp)
            return fail(QSD_ERR_UNSUPPORTED, "all matrix-free requests of a batch must have the same key width");
    }
    int slot = -1;
    for (int i = 0; i < b->max_slots; ++i)
        if (!b->slots[i].used) {
            slot = i;
            break;
        }
    if (slot < 0) return fail(QSD_ERR_CAPACITY, "no free request slot");
    hipStream_t st = (hipStream_t)stream;
    auto &S = b->slots[slot];
    S = qsd_batch::Slot();
    ReqDev &d = S.d;
    d.N = N;
    d.m = (int)std::min<int64_t>(b->max_iter, N);
    d.nbt = (int)((N + kBT - 1) / kBT);
    if (h) {
        d.s = sub_view(h->s);
        d.h = ham_view(h, b->f32);
        d.diag = h->diag;
        d.diag32 = h->diag32;
        d.sched = h->schedule;
    } else {
        d.diag = c->diag;
        d.cptr = c->indptr;
        d.cidx = (const int32_t *)c->indices;
        d.cval = c->data;
        d.lpr = c->lpr;
    }
    const Layout L = layout_of(N, d.m, b->f32);
    int rc = QSD_OK;
    if (workspace) {
        if (((uintptr_t)workspace & 255) != 0) return fail(QSD_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
        if (workspace_bytes < L.total)
            return fail(QSD_ERR_INVALID_ARG, "workspace of %lld bytes is smaller than the %lld needed",
                        (long long)workspace_bytes, (long long)L.total);
        S.mem = workspace;
        S.owned = false;
    } else {
        AllocScope scope(&b->alloc, stream);
        uint8_t *p = nullptr;
        if ((rc = dev_alloc(&p, (size_t)L.total)) != QSD_OK) {
            S = qsd_batch::Slot();
            return rc;
        }
        S.mem = p;
        S.owned = true;
        S.stream = stream;
    }
    uint8_t *base = (uint8_t *)S.mem;
    d.V = (double *)(base + L.V);
    d.x = (double *)(base + L.x);
    d.w = (double *)(base + L.w);
    d.x32 = b->f32 ? (float *)(base + L.x32) : nullptr;
    d.w32 = b->f32 ? (float *)(base + L.w32) : nullptr;
    d.part = (double *)(base + L.part);
    d.hv = (double *)(base + L.hv);
    d.alpha = (double *)(base + L.alpha);
    d.beta = (double *)(base + L.beta);
    d.kdev = (int *)(base + L.kdev);
    d.tri = (double *)(base + L.tri);
    S.used = true;
    S.h = h;
    S.tol = tol;
    if (h) b->Wp = h->Wp;
    b->dirty = true;
    if ((rc = sync_tables(b, st)) != QSD_OK) {
        free_slot(b, S);
        b->dirty = true;
        return rc;
    }
    int64_t spike = 0;
    if (v0_mode == QSD_V0_MIN_DIAG) {
        kb_argmin<<<1, 256, 0, st>>>(d.diag, N, b->d_spike);
        if (hipMemcpyAsync(&spike, b->d_spike, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "argmin failed");
    }
    if (rc == QSD_OK) {
        kb_init<<<256, 256, 0, st>>>(b->d_reqs, slot, v0_mode, seed, spike);
        kb_start<<<1, 256, 0, st>>>(b->d_reqs, slot);
        if (hipGetLastError() != hipSuccess) rc = fail(QSD_ERR_HIP, "request start failed");
    }
    if (rc != QSD_OK) {
        free_slot(b, S);
        b->dirty = true;
        return rc;
    }
    *slot_out = slot;
    return QSD_OK;
}

}  // namespace

extern "C" int qsd_batch_add(qsd_batch *b, const qsd_ham *h, int32_t v0_mode, uint64_t seed, double tol,
                             void *workspace, int64_t workspace_bytes, int32_t *slot_out, void *stream) {
    clear_error();
    if (!h) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    return add_impl(b, h, nullptr, v0_mode, seed, tol, workspace, workspace_bytes, slot_out, stream);
}

extern "C" int qsd_batch_add_csr(qsd_batch *b, const qsd_csr *c, int32_t v0_mode, uint64_t seed, double tol,
                                 void *workspace, int64_t workspace_bytes, int32_t *slot_out, void *stream) {
    clear_error();
    if (!c) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    return add_impl(b, nullptr, c, v0_mode, seed, tol, workspace, workspace_bytes, slot_out, stream);
}

extern "C" int qsd_batch_step(qsd_batch *b, int32_t iterations, void *stream) {
    clear_error();
    if (!b || iterations < 0) return fail(QSD_ERR_INVALID_ARG, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    QSD_TRY(sync_tables(b, st));
    if (b->n_mv == 0) return QSD_OK;
    const int ns = b->max_slots;
    for (int it = 0; it < iterations; ++it) {
        if (b->f32) kb_convert<<<b->n_bl, 256, 0, st>>>(b->d_reqs, b->d_bl, 1);
        switch (b->Wp) {
            case 1: launch_bmv<1>(b, st); break;
            case 2: launch_bmv<2>(b, st); break;
            case 4: launch_bmv<4>(b, st); break;
            case 8: launch_bmv<8>(b, st); break;
            case 16: launch_bmv<16>(b, st); break;
            default: launch_bmv<1>(b, st); break;  // stored-CSR requests only
        }
        if (b->f32) kb_convert<<<b->n_bl, 256, 0, st>>>(b->d_reqs, b->d_bl, 0);
        for (int pass = 0; pass < 2; ++pass) {
            kb_gemv_t<<<dim3(b->n_bl, (b->max_iter + kBJ) / kBJ), 256, 0, st>>>(b->d_reqs, b->d_bl);
            kb_reduce<<<dim3((b->max_iter + 4) / 4, ns), 256, 0, st>>>(b->d_reqs, ns);
            kb_gemv_n_sub<<<b->n_mv, kBlock, 0, st>>>(b->d_reqs, b->d_mv);
        }
        kb_sq_part<<<b->n_bl, 256, 0, st>>>(b->d_reqs, b->d_bl);
        kb_beta<<<ns, 64, 0, st>>>(b->d_reqs, ns);
        kb_next<<<b->n_mv, kBlock, 0, st>>>(b->d_reqs, b->d_mv);
        kb_bump<<<(ns + 63) / 64, 64, 0, st>>>(b->d_reqs, ns);
    }
    for (auto &S : b->slots)
        if (S.used) S.steps += iterations;
    QSD_CHECK_HIP(hipGetLastError());
    return QSD_OK;
}

extern "C" int qsd_batch_poll(qsd_batch *b, int32_t *status, double *energy, int32_t *iterations,
                              double *ritz_residual, void *stream) {
    clear_error();
    if (!b) return fail(QSD_ERR_INVALID_ARG, "batch is NULL");
    hipStream_t st = (hipStream_t)stream;
    QSD_TRY(sync_tables(b, st));
    const int ns = b->max_slots;
    std::vector<double> out(4 * (size_t)ns, 0.0);
    if (b->n_mv > 0) {
        kb_tridiag<<<ns, kTriThreads, 0, st>>>(b->d_reqs, ns, b->d_out);
        QSD_CHECK_HIP(hipMemcpyAsync(out.data(), b->d_out, out.size() * 8, hipMemcpyDeviceToHost, st));
        QSD_CHECK_HIP(hipStreamSynchronize(st));
    }
    for (int i = 0; i < ns; ++i) {
        const auto &S = b->slots[i];
        int stv = 0;  // 0 = free slot
        if (S.used) {
            const double th = out[4 * i], rr = out[4 * i + 1];
            const int done = (int)out[4 * i + 2];
            const bool brk = out[4 * i + 3] != 0.0;
            if (brk || (done > 0 && rr <= S.tol * std::fabs(th)))
                stv = 2;  // converged
            else if (done >= S.d.m)
                stv = 3;  // iteration limit
            else
                stv = 1;  // running
            if (energy) energy[i] = th;
            if (iterations) iterations[i] = done;
            if (ritz_residual) ritz_residual[i] = rr;
        }
        if (status) status[i] = stv;
    }
    return QSD_OK;
}

extern "C" int qsd_batch_remove(qsd_batch *b, int32_t slot) {
    clear_error();
    if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(QSD_ERR_INVALID_ARG, "bad slot");
    // device work that reads the slot was enqueued before: an owned workspace is released
    // stream-ordered (or by hipFree, which waits for the device); a caller's workspace must
    // stay valid until that work has finished
    free_slot(b, b->slots[slot]);
    b->dirty = true;
    return QSD_OK;
}

extern "C" int qsd_batch_destroy(qsd_batch *b) {
    clear_error();
    if (!b) return QSD_OK;
    for (auto &S : b->slots)
        if (S.used) free_slot(b, S);
    AllocScope scope(&b->alloc, nullptr);
    dev_free(b->d_reqs);
    dev_free(b->d_mv);
    dev_free(b->d_bl);
    dev_free(b->d_pmt);
    dev_free(b->d_out);
    dev_free(b->d_spike);
    delete b;
    return QSD_OK;
}

namespace {

template <int Wp, class ET, bool CPLX, int PF = 1>
void launch_bmv_any(int nv_max, int tiles, const MvReq *reqs, const Tile *tl, hipStream_t st) {
    if (nv_max <= 1)
        kbm_matvec<Wp, 1, ET, CPLX, PF><<<tiles, kBlock, 0, st>>>(reqs, tl);
    else if (nv_max <= 4 || CPLX)
        kbm_matvec<Wp, 4, ET, CPLX, PF><<<tiles, kBlock, 0, st>>>(reqs, tl);
    else
        kbm_matvec<Wp, 16, ET, CPLX, PF><<<tiles, kBlock, 0, st>>>(reqs, tl);
}

template <class ET, bool CPLX>
void launch_bmv_w(int Wp, bool pm, int nv_max, int tiles, const MvReq *reqs, const Tile *tl, hipStream_t st) {
    switch (Wp) {
        case 1:
            if (pm)
                launch_bmv_any<1, ET, CPLX, 2>(nv_max, tiles, reqs, tl, st);
            else
                launch_bmv_any<1, ET, CPLX>(nv_max, tiles, reqs, tl, st);
            break;
        case 2: launch_bmv_any<2, ET, CPLX>(nv_max, tiles, reqs, tl, st); break;
        case 4: launch_bmv_any<4, ET, CPLX>(nv_max, tiles, reqs, tl, st); break;
        case 8: launch_bmv_any<8, ET, CPLX>(nv_max, tiles, reqs, tl, st); break;
        case 16: launch_bmv_any<16, ET, CPLX>(nv_max, tiles, reqs, tl, st); break;
    }
}

}  // namespace

namespace {

// The plan of a batched SpMV: request table, tile list (request, row tile) and one launch per
// (key width, vector chunk, product map or not); complex vectors go in chunks of four.
struct BatchedPlan {
    struct Launch {
        int Wp, nv_max;
        size_t t0, nt;
        bool pm;  // requests on product subspaces (one-word keys): the product-map kernel
    };
    std::vector<MvReq> reqs;
    std::vector<Tile> tiles;
    std::vector<Launch> launches;
};

int plan_batched(int32_t n, const qsd_ham *const *hams, const void *const *xs, void *const *ys, const int32_t *nvecs,
                 int32_t dtype, BatchedPlan &P) {
    if (n < 0 || (n > 0 && (!hams || !xs || !ys || !nvecs))) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    if (dtype < QSD_F64 || dtype > QSD_C64) return fail(QSD_ERR_INVALID_ARG, "unknown dtype %d", dtype);
    const bool cplx = dtype == QSD_C128 || dtype == QSD_C64;
    const bool f32 = dtype == QSD_F32 || dtype == QSD_C64;
    const size_t esz = dtype == QSD_F64 ? 8 : dtype == QSD_F32 ? 4 : dtype == QSD_C128 ? 16 : 8;
    for (int i = 0; i < n; ++i) {
        if (!hams[i] || !xs[i] || !ys[i]) return fail(QSD_ERR_INVALID_ARG, "NULL operator or vector in request %d", i);
        if (nvecs[i] < 1 || nvecs[i] > 16) return fail(QSD_ERR_INVALID_ARG, "nvecs[%d] must be in [1, 16]", i);
        if (hams[i]->is_complex != cplx)
            return fail(QSD_ERR_DTYPE, "dtype %d does not match the %s operator of request %d", dtype,
                        hams[i]->is_complex ? "complex" : "real", i);
    }
    const int chunk = cplx ? 4 : 16;
    for (int Wp : {1, 2, 4, 8, 16}) {
        for (int c0 = 0; c0 < 16; c0 += chunk) {
          for (int pm = (Wp == 1 ? 1 : 0); pm >= 0; --pm) {
            BatchedPlan::Launch L{Wp, 0, P.tiles.size(), 0, pm != 0};
            for (int i = 0; i < n; ++i) {
                const qsd_ham *h = hams[i];
                if (h->Wp != Wp || nvecs[i] <= c0 || h->N == 0) continue;
                const bool hpm = Wp == 1 && h->s->prank && !(h->schedule & QSD_SCHED_HASH_LOOKUP);
                if (hpm != (pm != 0)) continue;
                MvReq R{};
                R.s = sub_view(h->s);
                R.h = ham_view(h, f32);
                R.dre = f32 ? (const void *)h->diag32 : (const void *)h->diag;
                R.dim = cplx ? (f32 ? (const void *)h->diag32_im : (const void *)h->diag_im) : nullptr;
                R.x = (const char *)xs[i] + c0 * esz;
                R.y = (char *)ys[i] + c0 * esz;
                R.ld = nvecs[i];
                R.nv = std::min(chunk, nvecs[i] - c0);
                R.sched = h->schedule;
                L.nv_max = std::max(L.nv_max, R.nv);
                const int slot = (int)P.reqs.size();
                P.reqs.push_back(R);
                // product-map requests: tiles within the product's blocks of rows (see pm_tile)
                const int64_t nb = L.pm ? pm_tiles(h->N, h->s->pna, h->schedule) : 0;
                for (int64_t t = 0; t < (nb ? nb : (h->N + kBlock - 1) / kBlock); ++t) P.tiles.push_back({slot, (int)t});
            }
            L.nt = P.tiles.size() - L.t0;
            if (L.nt > 0) P.launches.push_back(L);
          }
        }
    }
    if (P.tiles.size() > (size_t)INT32_MAX) return fail(QSD_ERR_CAPACITY, "too many row tiles");
    return QSD_OK;
}

// Uploads the plan's tables to d_reqs / d_tiles and enqueues its launches on st.
int run_batched(const BatchedPlan &P, int32_t dtype, MvReq *d_reqs, Tile *d_tiles, hipStream_t st) {
    // pageable sources: the copies return once the host data is staged
    if (hipMemcpyAsync(d_reqs, P.reqs.data(), P.reqs.size() * sizeof(MvReq), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d_tiles, P.tiles.data(), P.tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(QSD_ERR_HIP, "table upload failed");
    for (const auto &L : P.launches) {
        const Tile *tl = d_tiles + L.t0;
        switch (dtype) {
            case QSD_F64: launch_bmv_w<double, false>(L.Wp, L.pm, L.nv_max, (int)L.nt, d_reqs, tl, st); break;
            case QSD_F32: launch_bmv_w<float, false>(L.Wp, L.pm, L.nv_max, (int)L.nt, d_reqs, tl, st); break;
            case QSD_C128: launch_bmv_w<double, true>(L.Wp, L.pm, L.nv_max, (int)L.nt, d_reqs, tl, st); break;
            case QSD_C64: launch_bmv_w<float, true>(L.Wp, L.pm, L.nv_max, (int)L.nt, d_reqs, tl, st); break;
        }
    }
    if (hipGetLastError() != hipSuccess) return fail(QSD_ERR_HIP, "batched matvec launch failed");
    return QSD_OK;
}

// Fixed device scratch of qsd_matvec_batched_noalloc: the request table, then the tile list.
// Every GPU the library runs on holds one until the process ends.  In host code the name is only
// a symbol: its device address comes from hipGetSymbolAddress, once per device.
constexpr int kScratchReqs = QSD_NOALLOC_MAX_REQUESTS;
constexpr size_t kScratchTiles = QSD_NOALLOC_MAX_TILES;
constexpr size_t kScratchTileOff = (kScratchReqs * sizeof(MvReq) + 255) / 256 * 256;
constexpr size_t kScratchBytes = kScratchTileOff + kScratchTiles * sizeof(Tile);
static_assert(kScratchBytes <= (size_t(1) << 20), "the fixed scratch stays under 1 MiB");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (resolved at the device's first call).
int scratch_address(void **out) {
    int dev = -1;
    QSD_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(QSD_ERR_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(QSD_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QSD_OK;
}

}  // namespace

extern "C" int qsd_matvec_batched(int32_t n, const qsd_ham *const *hams, const void *const *xs, void *const *ys,
                                  const int32_t *nvecs, int32_t dtype, void *stream) {
    clear_error();
    BatchedPlan P;
    QSD_TRY(plan_batched(n, hams, xs, ys, nvecs, dtype, P));
    if (P.launches.empty()) return QSD_OK;
    hipStream_t st = (hipStream_t)stream;
    // Stream-ordered tables: allocated, filled, used and released in order on `stream`, by the
    // first operator's allocator (stream-ordered by contract) or hipMallocAsync.
    AllocScope scope(&hams[0]->alloc, stream);
    const bool own_alloc = custom_allocator();
    MvReq *d_reqs = nullptr;
    Tile *d_tiles = nullptr;
    if (own_alloc) {
        QSD_TRY(dev_alloc(&d_reqs, P.reqs.size()));
        if (dev_alloc(&d_tiles, P.tiles.size()) != QSD_OK) {
            dev_free(d_reqs);
            return QSD_ERR_OUT_OF_MEMORY;
        }
    } else {
        QSD_CHECK_HIP(hipMallocAsync((void **)&d_reqs, P.reqs.size() * sizeof(MvReq), st));
        if (hipMallocAsync((void **)&d_tiles, P.tiles.size() * sizeof(Tile), st) != hipSuccess) {
            (void)hipFreeAsync(d_reqs, st);
            return fail(QSD_ERR_OUT_OF_MEMORY, "tile table allocation failed");
        }
    }
    const int rc = run_batched(P, dtype, d_reqs, d_tiles, st);
    if (own_alloc) {
        dev_free(d_tiles);
        dev_free(d_reqs);
    } else {
        (void)hipFreeAsync(d_tiles, st);
        (void)hipFreeAsync(d_reqs, st);
    }
    return rc;
}

extern "C" int qsd_matvec_batched_noalloc(int32_t n, const qsd_ham *const *hams, const void *const *xs,
                                          void *const *ys, const int32_t *nvecs, int32_t dtype, void *stream) {
    clear_error();
    BatchedPlan P;
    QSD_TRY(plan_batched(n, hams, xs, ys, nvecs, dtype, P));
    if (P.launches.empty()) return QSD_OK;
    if (P.reqs.size() > (size_t)kScratchReqs)
        return fail(QSD_ERR_CAPACITY, "%zu request chunks exceed the %d the fixed scratch holds", P.reqs.size(),
                    kScratchReqs);
    if (P.tiles.size() > kScratchTiles)
        return fail(QSD_ERR_CAPACITY, "%zu row tiles exceed the %zu the fixed scratch holds", P.tiles.size(),
                    (size_t)kScratchTiles);
    void *base = nullptr;
    QSD_TRY(scratch_address(&base));
    MvReq *d_reqs = (MvReq *)base;
    Tile *d_tiles = (Tile *)((unsigned char *)base + kScratchTileOff);
    // nothing in the scratch must start at zero: the call uploads its whole table first
    return run_batched(P, dtype, d_reqs, d_tiles, (hipStream_t)stream);
}
