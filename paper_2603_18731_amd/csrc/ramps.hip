// RAMPS restricted to the sampled subspace (Supplement, Recursive algorithm for a minimal
// perturbative subspace; Algorithm S1 with the S_full restriction), frontier-parallel.
//
// A frontier entry is (row index in S_full, prefactor).  One lane runs one entry through the
// row engine (group filter, column hash probe - which is the S_full membership test - and the
// term sums), so every off-diagonal element H_jk of the row with k in S_full is visited; for
// k outside S_0
//     amp = (pre * |H_jk|^2) / (E - H_kk)
// and |amp| > tau marks k selected and appends (k, amp / (E - H_kk)) to the next frontier
// (atomic cursor).  Levels run until the frontier is empty or max_depth.  The selected set does
// not depend on the order in which paths are processed, and every amplitude is formed with the
// same IEEE operations in the same order as written (no contraction), so the result is exact and
// reproducible.
#include <vector>

#include "common.h"
#include "matvec.h"

namespace qsd {
namespace {

template <int Wp>
__global__ __launch_bounds__(kBlock) void k_ramps_level(SubView s, HamView h, const double *__restrict__ diag,
                                                       const uint8_t *__restrict__ in_s0,
                                                       const int64_t *__restrict__ f_idx,
                                                       const double *__restrict__ f_pre, int64_t F, double E,
                                                       double tau, int64_t *__restrict__ n_idx,
                                                       double *__restrict__ n_pre,
                                                       unsigned long long *__restrict__ n_count, int64_t cap,
                                                       uint8_t *__restrict__ selected) {
    __shared__ ChunkLds<Wp> lds;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = t < F;
    const int64_t r = valid ? f_idx[t] : 0;
    const double pre = valid ? f_pre[t] : 0.0;
    uint64_t key[Wp];
#pragma unroll
    for (int w = 0; w < Wp; ++w) key[w] = s.keys[(int64_t)w * s.N + r];
    const uint64_t hrow = s.hkey[r];
    const uint32_t prow = s.pfilt ? s.pkey[r] : 0u;
    row_engine<Wp>(s, h, key, hrow, prow, valid, lds, sink<double>([&](int64_t k, double vre, double vim, int) {
        if (in_s0[k]) return;  // the model space is not followed
        double amp, next;
        {
#pragma clang fp contract(off)
            const double m2 = vre * vre + vim * vim;
            const double den = E - diag[k];
            amp = (pre * m2) / den;
            next = amp / den;
        }
        if (fabs(amp) > tau) {
            selected[k] = 1;
            const unsigned long long pos = atomicAdd(n_count, 1ull);
            if ((int64_t)pos < cap) {
                n_idx[pos] = k;
                n_pre[pos] = next;
            }
        }
    }), nullptr, false, true);
}

__global__ void k_mark(const int64_t *__restrict__ idx, int64_t n, uint8_t *__restrict__ a, uint8_t *__restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        a[idx[i]] = 1;
        b[idx[i]] = 1;
    }
}

__global__ void k_zero_u8(uint8_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_count_u8(const uint8_t *__restrict__ p, int64_t n, unsigned long long *__restrict__ out) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += p[i] ? 1ull : 0ull;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, c);
}

template <int Wp>
void launch_level(const qsd_ham *h, const uint8_t *in_s0, const int64_t *fi, const double *fp, int64_t F, double E,
                  double tau, int64_t *ni, double *np, unsigned long long *cnt, int64_t cap, uint8_t *sel,
                  hipStream_t st) {
    const unsigned grid = (unsigned)((F + kBlock - 1) / kBlock);
    k_ramps_level<Wp><<<grid, kBlock, 0, st>>>(sub_view(h->s), ham_view(h, false), h->diag, in_s0, fi, fp, F, E, tau,
                                              ni, np, cnt, cap, sel);
}

}  // namespace
}  // namespace qsd

using namespace qsd;

extern "C" int qsd_ramps(const qsd_ham *h, const int64_t *s0, int64_t n0, double E, double tau, int32_t max_depth,
                         int64_t max_frontier, uint8_t *d_selected, int64_t *n_selected, qsd_ramps_info *info,
                         void *stream) {
    clear_error();
    if (!h || !s0 || !d_selected) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    if (n0 < 1) return fail(QSD_ERR_INVALID_ARG, "the initial subspace is empty");
    if (!(tau >= 0.0)) return fail(QSD_ERR_INVALID_ARG, "tau must be >= 0");
    if (max_depth < 0) return fail(QSD_ERR_INVALID_ARG, "max_depth must be >= 0");
    if (max_frontier < n0) return fail(QSD_ERR_INVALID_ARG, "max_frontier must hold the initial subspace");
    if (!(E == E) || E == 0.0) return fail(QSD_ERR_INVALID_ARG, "E must be a nonzero number");
    for (int64_t i = 0; i < n0; ++i)
        if (s0[i] < 0 || s0[i] >= h->N) return fail(QSD_ERR_INVALID_ARG, "initial index %lld out of range", (long long)s0[i]);
    hipStream_t st = (hipStream_t)stream;
    AllocScope scope(&h->alloc, stream);
    const int64_t N = h->N;
    uint8_t *in_s0 = nullptr;
    int64_t *fi[2] = {nullptr, nullptr};
    double *fp[2] = {nullptr, nullptr};
    unsigned long long *cnt = nullptr;
    int rc = dev_alloc(&in_s0, N);
    if (rc == QSD_OK) rc = dev_alloc(&fi[0], max_frontier);
    if (rc == QSD_OK) rc = dev_alloc(&fi[1], max_frontier);
    if (rc == QSD_OK) rc = dev_alloc(&fp[0], max_frontier);
    if (rc == QSD_OK) rc = dev_alloc(&fp[1], max_frontier);
    if (rc == QSD_OK) rc = dev_alloc(&cnt, 1);
    qsd_ramps_info inf{};
    if (rc == QSD_OK) {
        std::vector<double> pre((size_t)n0, 1.0 / E);
        k_zero_u8<<<1024, 256, 0, st>>>(in_s0, N);
        k_zero_u8<<<1024, 256, 0, st>>>(d_selected, N);
        if (hipMemcpyAsync(fi[0], s0, n0 * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(fp[0], pre.data(), n0 * 8, hipMemcpyHostToDevice, st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "copy failed");
        if (rc == QSD_OK) k_mark<<<64, 256, 0, st>>>(fi[0], n0, in_s0, d_selected);
        // the pageable sources above must be consumed before `pre` goes out of scope
        if (rc == QSD_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(QSD_ERR_HIP, "setup failed");
    }
    int64_t F = n0;
    int cur = 0;
    while (rc == QSD_OK && F > 0 && inf.levels < max_depth) {
        unsigned long long zero = 0, next = 0;
        if (hipMemcpyAsync(cnt, &zero, 8, hipMemcpyHostToDevice, st) != hipSuccess) {
            rc = fail(QSD_ERR_HIP, "copy failed");
            break;
        }
        switch (h->Wp) {
            case 1: launch_level<1>(h, in_s0, fi[cur], fp[cur], F, E, tau, fi[1 - cur], fp[1 - cur], cnt, max_frontier, d_selected, st); break;
            case 2: launch_level<2>(h, in_s0, fi[cur], fp[cur], F, E, tau, fi[1 - cur], fp[1 - cur], cnt, max_frontier, d_selected, st); break;
            case 4: launch_level<4>(h, in_s0, fi[cur], fp[cur], F, E, tau, fi[1 - cur], fp[1 - cur], cnt, max_frontier, d_selected, st); break;
            case 8: launch_level<8>(h, in_s0, fi[cur], fp[cur], F, E, tau, fi[1 - cur], fp[1 - cur], cnt, max_frontier, d_selected, st); break;
            case 16: launch_level<16>(h, in_s0, fi[cur], fp[cur], F, E, tau, fi[1 - cur], fp[1 - cur], cnt, max_frontier, d_selected, st); break;
        }
        if (hipMemcpyAsync(&next, cnt, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(QSD_ERR_HIP, "RAMPS level failed: %s", hipGetErrorString(hipGetLastError()));
            break;
        }
        inf.levels += 1;
        inf.paths += (int64_t)next;
        if ((int64_t)next > inf.max_frontier) inf.max_frontier = (int64_t)next;
        if ((int64_t)next > max_frontier) {
            rc = fail(QSD_ERR_CAPACITY, "frontier of %llu paths at level %d exceeds max_frontier = %lld",
                      next, inf.levels, (long long)max_frontier);
            break;
        }
        F = (int64_t)next;
        cur = 1 - cur;
    }
    if (rc == QSD_OK) {
        unsigned long long zero = 0, total = 0;
        if (hipMemcpyAsync(cnt, &zero, 8, hipMemcpyHostToDevice, st) != hipSuccess) rc = fail(QSD_ERR_HIP, "copy failed");
        if (rc == QSD_OK) {
            k_count_u8<<<1024, 256, 0, st>>>(d_selected, N, cnt);
            if (hipMemcpyAsync(&total, cnt, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = fail(QSD_ERR_HIP, "count failed");
        }
        inf.selected = (int64_t)total;
        inf.truncated = F > 0 ? 1 : 0;
        if (n_selected) *n_selected = (int64_t)total;
        if (info) *info = inf;
    }
    dev_free(in_s0);
    dev_free(fi[0]);
    dev_free(fi[1]);
    dev_free(fp[0]);
    dev_free(fp[1]);
    dev_free(cnt);
    return rc;
}
