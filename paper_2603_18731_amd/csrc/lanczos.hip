// Ground-state Lanczos on the device (FP64 basis and recurrence, full reorthogonalization).
//
// The paper hands its SpMV operator to external eigensolvers; this solver keeps the whole
// iteration on the GPU.  Every buffer has a fixed address and the iteration number lives in
// device memory, so one iteration is a fixed kernel sequence that can be captured once in a
// HIP graph and replayed:
//   w = H x                       (SpMV, FP64 or FP32 elements with FP64 accumulation)
//   h = V^T w; w -= V h  (twice)  (classical Gram-Schmidt applied twice against v_0..v_k)
//   alpha_k = sum of the two h_k; beta_k = ||w||; v_{k+1} = x = w / beta_k
// The tridiagonal eigenproblem is solved on the device every few iterations (Sturm
// multisection for the lowest eigenvalue, inverse iteration for its vector); only theta and
// the Ritz residual estimate beta_k |s_k| are copied to the host.
#include <chrono>
#include <cmath>
#include <vector>

#include "common.h"
#include "tridiag.h"

namespace qsd {
namespace {

constexpr int kRed = 256;       // threads of reduction kernels
constexpr int kDotBlocks = 512; // partial-sum blocks (fixed => deterministic sums)

struct LzState {
    int64_t N = 0;           // rows
    int64_t NR = 0;          // doubles per vector: N (real) or 2N (complex, interleaved)
    bool cplx = false;
    int m = 0;               // max iterations
    double *V = nullptr;     // [m+1][N]
    double *x = nullptr;     // [N] current basis vector
    double *w = nullptr;     // [N]
    float *x32 = nullptr;    // [N]
    float *w32 = nullptr;    // [N]
    double *part = nullptr;  // [(m+1) * kDotBlocks]
    double *hv = nullptr;    // [m+1]
    double *alpha = nullptr; // [m]
    double *beta = nullptr;  // [m]
    int *kdev = nullptr;     // iteration number
    double *tri = nullptr;   // [m + 4]: theta, resid, breakdown flag, s[0..m)
    void free_all() {
        dev_free(V);
        dev_free(x);
        dev_free(w);
        dev_free(x32);
        dev_free(w32);
        dev_free(part);
        dev_free(hv);
        dev_free(alpha);
        dev_free(beta);
        dev_free(kdev);
        dev_free(tri);
    }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// partial[j][b] = sum over the rows of chunk b of V[j][i] * w[i], j = 0..k (k = *kdev).
// blockIdx.y selects kGemvJ basis vectors: each thread reads w[i] once and kGemvJ basis values,
// so the basis streams at full occupancy; block sums by a fixed tree (deterministic).
constexpr int kGemvJ = 8;

__global__ __launch_bounds__(kRed) void k_gemv_t(const double *__restrict__ V, const double *__restrict__ w, int64_t N,
                                                 const int *__restrict__ kdev, int extra, double *__restrict__ part) {
    __shared__ double red[kGemvJ][kRed / 64];
    const int cnt = *kdev + 1 + extra;
    const int j0 = blockIdx.y * kGemvJ;
    if (j0 >= cnt) return;
    const int nj = min(kGemvJ, cnt - j0);
    const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
    const int64_t a = (int64_t)blockIdx.x * chunk;
    const int64_t b = min(N, a + chunk);
    double acc[kGemvJ];
#pragma unroll
    for (int q = 0; q < kGemvJ; ++q) acc[q] = 0.0;
    const double *v0 = V + (int64_t)j0 * N;
    for (int64_t i = a + threadIdx.x; i < b; i += kRed) {
        const double wi = w[i];
#pragma unroll
        for (int q = 0; q < kGemvJ; ++q)
            if (q < nj) acc[q] += v0[(int64_t)q * N + i] * wi;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kGemvJ; ++q) {
        const double s = wave_sum(acc[q]);
        if (lane == 0) red[q][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < nj) {
        double t = 0.0;
        for (int q = 0; q < kRed / 64; ++q) t += red[threadIdx.x][q];
        part[(int64_t)(j0 + threadIdx.x) * gridDim.x + blockIdx.x] = t;
    }
}

// Complex (Hermitian) variant: part[j][b] and part[P + j][b] (P = plane stride) are the real
// and imaginary parts of sum over chunk b of conj(V[j][i]) w[i], vectors interleaved (re, im).
__global__ __launch_bounds__(kRed) void k_gemv_t_c(const double2 *__restrict__ V, const double2 *__restrict__ w,
                                                   int64_t N, const int *__restrict__ kdev, int64_t plane,
                                                   double *__restrict__ part) {
    __shared__ double red[2 * kGemvJ][kRed / 64];
    const int cnt = *kdev + 1;
    const int j0 = blockIdx.y * kGemvJ;
    if (j0 >= cnt) return;
    const int nj = min(kGemvJ, cnt - j0);
    const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
    const int64_t a = (int64_t)blockIdx.x * chunk;
    const int64_t b = min(N, a + chunk);
    double are[kGemvJ], aim[kGemvJ];
#pragma unroll
    for (int q = 0; q < kGemvJ; ++q) are[q] = aim[q] = 0.0;
    const double2 *v0 = V + (int64_t)j0 * N;
    for (int64_t i = a + threadIdx.x; i < b; i += kRed) {
        const double2 wi = w[i];
#pragma unroll
        for (int q = 0; q < kGemvJ; ++q)
            if (q < nj) {
                const double2 v = v0[(int64_t)q * N + i];
                are[q] += v.x * wi.x + v.y * wi.y;
                aim[q] += v.x * wi.y - v.y * wi.x;
            }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kGemvJ; ++q) {
        const double sr = wave_sum(are[q]), si = wave_sum(aim[q]);
        if (lane == 0) {
            red[2 * q][wave] = sr;
            red[2 * q + 1][wave] = si;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * nj) {
        double t = 0.0;
        for (int q = 0; q < kRed / 64; ++q) t += red[threadIdx.x][q];
        const int jj = threadIdx.x >> 1;
        part[(threadIdx.x & 1) * plane + (int64_t)(j0 + jj) * gridDim.x + blockIdx.x] = t;
    }
}

// w[i] -= sum_{j<=k} V[j][i] h[j] for complex vectors and coefficients (h interleaved)
__global__ __launch_bounds__(kRed) void k_gemv_n_sub_c(const double2 *__restrict__ V, const double *__restrict__ hv,
                                                       int64_t N, const int *__restrict__ kdev,
                                                       double2 *__restrict__ w) {
    __shared__ double sh[2 * 512];
    const int cnt = *kdev + 1;
    const int64_t i = (int64_t)blockIdx.x * kRed + threadIdx.x;
    double ar = 0.0, ai = 0.0;
    for (int j0 = 0; j0 < cnt; j0 += 512) {
        const int nj = min(512, cnt - j0);
        __syncthreads();
        for (int q = threadIdx.x; q < 2 * nj; q += kRed) sh[q] = hv[2 * j0 + q];
        __syncthreads();
        if (i < N)
            for (int q = 0; q < nj; ++q) {
                const double2 v = V[(int64_t)(j0 + q) * N + i];
                const double hr = sh[2 * q], hi = sh[2 * q + 1];
                ar += v.x * hr - v.y * hi;
                ai += v.x * hi + v.y * hr;
            }
    }
    if (i < N) {
        double2 t = w[i];
        t.x -= ar;
        t.y -= ai;
        w[i] = t;
    }
}

// hv[j] = sum_b part[j][b] (one block per j, fixed tree); optionally alpha[k] += hv[k].
// With planes = 2 (complex), blockIdx.y selects the real / imaginary plane at offset `plane`
// and hv holds interleaved pairs; alpha takes the real part.
__global__ __launch_bounds__(kRed) void k_reduce_parts(const double *__restrict__ part, int nparts,
                                                       const int *__restrict__ kdev, int extra, double *__restrict__ hv,
                                                       double *__restrict__ alpha, int planes = 1,
                                                       int64_t plane = 0) {
    __shared__ double ws[kRed / 64];
    const int cnt = *kdev + 1 + extra;
    const int j = blockIdx.x, im = blockIdx.y;
    if (j >= cnt) return;
    double s = 0.0;
    const double *pp = part + im * plane;
    for (int p = threadIdx.x; p < nparts; p += kRed) s += pp[(int64_t)j * nparts + p];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kRed / 64; ++q) t += ws[q];
        hv[planes * j + im] = t;
        if (alpha && im == 0 && j == *kdev) alpha[j] += t;
    }
}

// w[i] -= sum_{j<=k} V[j][i] hv[j]
__global__ __launch_bounds__(kRed) void k_gemv_n_sub(const double *__restrict__ V, const double *__restrict__ hv,
                                                     int64_t N, const int *__restrict__ kdev, double *__restrict__ w) {
    __shared__ double sh[1024];
    const int cnt = *kdev + 1;
    const int64_t i = (int64_t)blockIdx.x * kRed + threadIdx.x;
    double acc = 0.0;
    for (int j0 = 0; j0 < cnt; j0 += 1024) {
        const int nj = min(1024, cnt - j0);
        __syncthreads();
        for (int q = threadIdx.x; q < nj; q += kRed) sh[q] = hv[j0 + q];
        __syncthreads();
        if (i < N)
            for (int q = 0; q < nj; ++q) acc += V[(int64_t)(j0 + q) * N + i] * sh[q];
    }
    if (i < N) w[i] -= acc;
}

// y[i] = sum_{j<cnt} V[j][i] s[j]
__global__ __launch_bounds__(kRed) void k_gemv_n(const double *__restrict__ V, const double *__restrict__ s, int cnt,
                                                 int64_t N, double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * kRed + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (int j = 0; j < cnt; ++j) acc += V[(int64_t)j * N + i] * s[j];
    y[i] = acc;
}

__global__ __launch_bounds__(kRed) void k_sq_part(const double *__restrict__ w, int64_t N, double *__restrict__ part) {
    __shared__ double ws[kRed / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRed + threadIdx.x; i < N; i += (int64_t)gridDim.x * kRed) s += w[i] * w[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kRed / 64; ++q) t += ws[q];
        part[blockIdx.x] = t;
    }
}

// beta[k] = sqrt(sum part); flags breakdown in tri[2]
__global__ __launch_bounds__(kRed) void k_beta(const double *__restrict__ part, int nparts, const int *__restrict__ kdev,
                                               double *__restrict__ beta, double *__restrict__ tri) {
    __shared__ double ws[kRed / 64];
    double s = 0.0;
    for (int p = threadIdx.x; p < nparts; p += kRed) s += part[p];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kRed / 64; ++q) t += ws[q];
        beta[*kdev] = sqrt(t);
    }
}

// x = V[k+1] = w / beta[k]; k += 1 (the last block to finish bumps k)
// Breakdown (w vanished relative to the recurrence: an invariant subspace) records the
// number of valid iterations in tri[2] once; later iterations then carry zeros.
__global__ __launch_bounds__(kRed) void k_next(double *__restrict__ V, double *__restrict__ x,
                                               const double *__restrict__ w, int64_t N, const int *__restrict__ kdev,
                                               const double *__restrict__ alpha, double *__restrict__ beta, int m,
                                               double *__restrict__ tri) {
    const int k = *kdev;
    const double b = beta[k];
    const double scale = fabs(alpha[k]) + (k > 0 ? beta[k - 1] : 0.0);
    const bool brk = tri[2] != 0.0 || !(b > 1e-12 * scale) || !(b > 1e-300);
    const double inv = brk ? 0.0 : 1.0 / b;
    const int64_t i = (int64_t)blockIdx.x * kRed + threadIdx.x;
    if (i < N) {
        const double v = w[i] * inv;
        x[i] = v;
        if (k + 1 <= m) V[(int64_t)(k + 1) * N + i] = v;
    }
    __syncthreads();
    if (i == 0 && brk && tri[2] == 0.0) {
        tri[2] = (double)(k + 1);
        beta[k] = 0.0;
    }
}

__global__ void k_bump(int *kdev) { *kdev += 1; }

__global__ void k_f64_to_f32(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}
__global__ void k_f32_to_f64(const float *__restrict__ a, double *__restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (double)a[i];
}

// Lowest eigenpair of T_m for one Lanczos run (one block).
__global__ __launch_bounds__(kTriThreads) void k_tridiag(const double *__restrict__ alpha,
                                                        const double *__restrict__ beta, int m,
                                                        double *__restrict__ tri) {
    __shared__ TridiagLds L;
    tridiag_lowest(alpha, beta, m, tri, L);
}

// argmin of d (lowest index among ties); one block
__global__ __launch_bounds__(kRed) void k_argmin(const double *__restrict__ d, int64_t N, int64_t *__restrict__ out) {
    __shared__ double bv[kRed];
    __shared__ int64_t bi[kRed];
    double v = INFINITY;
    int64_t idx = N;
    for (int64_t i = threadIdx.x; i < N; i += kRed)
        if (d[i] < v) {
            v = d[i];
            idx = i;
        }
    bv[threadIdx.x] = v;
    bi[threadIdx.x] = idx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < kRed; ++t)
            if (bv[t] < v || (bv[t] == v && bi[t] < idx)) {
                v = bv[t];
                idx = bi[t];
            }
        *out = idx;
    }
}

__global__ void k_init_v0(double *__restrict__ x, int64_t N, int mode, uint64_t seed, const int64_t *__restrict__ spike,
                          int stride = 1) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double v;
        if (mode == QSD_V0_UNIFORM) {
            v = 1.0;
        } else if (mode == QSD_V0_MIN_DIAG) {
            v = (i == stride * *spike) ? 1.0 : 0.0;
        } else {
            // splitmix64 of (seed, i): uniform in [-1, 1)
            uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            v = (double)(z >> 11) * 0x1.0p-52 - 1.0;
        }
        x[i] = v;
    }
}

__global__ void k_scale(double *__restrict__ x, int64_t N, const double *__restrict__ part, int nparts) {
    // x /= sqrt(sum part) (sum recomputed per block in fixed order)
    __shared__ double inv;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int p = 0; p < nparts; ++p) t += part[p];
        inv = 1.0 / sqrt(t);
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        x[i] *= inv;
}

__global__ void k_copy_row(const double *__restrict__ x, double *__restrict__ V0, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        V0[i] = x[i];
}

// r = Hy - theta y -> partial sums of r^2 and of y^2
__global__ __launch_bounds__(kRed) void k_resid_part(const double *__restrict__ hy, const double *__restrict__ y,
                                                     double theta, int64_t N, double *__restrict__ part) {
    __shared__ double ws[kRed / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRed + threadIdx.x; i < N; i += (int64_t)gridDim.x * kRed) {
        const double r = hy[i] - theta * y[i];
        s += r * r;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kRed / 64; ++q) t += ws[q];
        part[blockIdx.x] = t;
    }
}

inline unsigned gridN(int64_t n) { return (unsigned)((n + kRed - 1) / kRed); }

int enqueue_iteration(const SpmvOp &op, LzState &S, bool f32, hipStream_t st) {
    const int64_t N = S.N, NR = S.NR;
    const int32_t dt64 = S.cplx ? QSD_C128 : QSD_F64, dt32 = S.cplx ? QSD_C64 : QSD_F32;
    if (f32) {
        k_f64_to_f32<<<1024, kRed, 0, st>>>(S.x, S.x32, NR);
        QSD_TRY(op.matvec(1, S.x32, 1, S.w32, 1, dt32, st));
        k_f32_to_f64<<<1024, kRed, 0, st>>>(S.w32, S.w, NR);
    } else {
        QSD_TRY(op.matvec(1, S.x, 1, S.w, 1, dt64, st));
    }
    const dim3 gt(kDotBlocks, (S.m + 1 + kGemvJ - 1) / kGemvJ);
    const int64_t plane = (int64_t)(S.m + 1) * kDotBlocks;
    for (int pass = 0; pass < 2; ++pass) {
        if (S.cplx) {
            k_gemv_t_c<<<gt, kRed, 0, st>>>((const double2 *)S.V, (const double2 *)S.w, N, S.kdev, plane, S.part);
            k_reduce_parts<<<dim3(S.m + 1, 2), kRed, 0, st>>>(S.part, kDotBlocks, S.kdev, 0, S.hv, S.alpha, 2, plane);
            k_gemv_n_sub_c<<<gridN(N), kRed, 0, st>>>((const double2 *)S.V, S.hv, N, S.kdev, (double2 *)S.w);
        } else {
            k_gemv_t<<<gt, kRed, 0, st>>>(S.V, S.w, N, S.kdev, 0, S.part);
            k_reduce_parts<<<S.m + 1, kRed, 0, st>>>(S.part, kDotBlocks, S.kdev, 0, S.hv, S.alpha);
            k_gemv_n_sub<<<gridN(N), kRed, 0, st>>>(S.V, S.hv, N, S.kdev, S.w);
        }
    }
    k_sq_part<<<kDotBlocks, kRed, 0, st>>>(S.w, NR, S.part);
    k_beta<<<1, kRed, 0, st>>>(S.part, kDotBlocks, S.kdev, S.beta, S.tri);
    k_next<<<gridN(NR), kRed, 0, st>>>(S.V, S.x, S.w, NR, S.kdev, S.alpha, S.beta, S.m, S.tri);
    k_bump<<<1, 1, 0, st>>>(S.kdev);
    QSD_CHECK_HIP(hipGetLastError());
    return QSD_OK;
}

__global__ void k_zero(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}
__global__ void k_zero_i(int *p) { *p = 0; }

}  // namespace
}  // namespace qsd

using namespace qsd;

extern "C" void qsd_lanczos_default_opts(qsd_lanczos_opts *o) {
    if (!o) return;
    o->max_iter = 300;
    o->tol = 1e-10;
    o->v0_mode = QSD_V0_UNIFORM;
    o->seed = 0;
    o->spmv_dtype = QSD_F64;
    o->check_every = 5;
    o->want_vector = 0;
    o->use_graph = 0;
    o->alloc = nullptr;
}

namespace {

int lanczos_impl(const SpmvOp &op, const qsd_lanczos_opts *opts, double *eval_out, void *d_evec,
                 qsd_lanczos_info *info, void *stream) {
    auto t_start = std::chrono::steady_clock::now();
    if (!eval_out) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    qsd_lanczos_opts o;
    qsd_lanczos_default_opts(&o);
    if (opts) o = *opts;
    const bool cplx = op.is_complex();
    if (o.max_iter < 1 || o.max_iter > 1000) return fail(QSD_ERR_INVALID_ARG, "max_iter must be in [1, 1000]");
    if (!(o.tol > 0)) return fail(QSD_ERR_INVALID_ARG, "tol must be > 0");
    if (o.spmv_dtype != QSD_F64 && o.spmv_dtype != QSD_F32) return fail(QSD_ERR_DTYPE, "spmv_dtype must be F64 or F32");
    const int32_t mv64 = cplx ? QSD_C128 : QSD_F64, mv32 = cplx ? QSD_C64 : QSD_F32;
    if (!op.takes(o.spmv_dtype == QSD_F32 ? mv32 : mv64))
        return fail(QSD_ERR_DTYPE, "spmv_dtype must be the stored matrix's dtype");
    if (o.v0_mode < QSD_V0_UNIFORM || o.v0_mode > QSD_V0_USER) return fail(QSD_ERR_INVALID_ARG, "bad v0_mode");
    if ((o.v0_mode == QSD_V0_USER || o.want_vector) && !d_evec)
        return fail(QSD_ERR_INVALID_ARG, "d_evec is required for QSD_V0_USER / want_vector");
    if (o.check_every < 1) o.check_every = 1;
    hipStream_t st = (hipStream_t)stream;
    // basis and work vectors from the caller's allocator or the operator's (the scope outlives S)
    AllocScope scope(o.alloc ? o.alloc : op.allocator(), stream);
    const int64_t N = op.N();
    const int64_t NR = cplx ? 2 * N : N;  // doubles per vector
    LzState S;
    S.N = N;
    S.NR = NR;
    S.cplx = cplx;
    S.m = (int)std::min<int64_t>(o.max_iter, N);
    const bool f32 = o.spmv_dtype == QSD_F32;
    int rc = QSD_OK;
    auto alloc_all = [&]() -> int {
        QSD_TRY(dev_alloc(&S.V, (size_t)(S.m + 1) * NR));
        QSD_TRY(dev_alloc(&S.x, NR));
        QSD_TRY(dev_alloc(&S.w, NR));
        if (f32) {
            QSD_TRY(dev_alloc(&S.x32, NR));
            QSD_TRY(dev_alloc(&S.w32, NR));
        }
        QSD_TRY(dev_alloc(&S.part, (size_t)(S.m + 1) * kDotBlocks * (cplx ? 2 : 1)));
        QSD_TRY(dev_alloc(&S.hv, (size_t)(S.m + 1) * (cplx ? 2 : 1)));
        QSD_TRY(dev_alloc(&S.alpha, S.m));
        QSD_TRY(dev_alloc(&S.beta, S.m));
        QSD_TRY(dev_alloc(&S.kdev, 1));
        QSD_TRY(dev_alloc(&S.tri, S.m + 4));
        return QSD_OK;
    };
    rc = alloc_all();
    if (rc != QSD_OK) {
        S.free_all();
        return rc;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    double theta = 0.0, ritz = INFINITY, expl = NAN;
    int iters = 0;
    bool converged = false;
    float mv_ms = 0.0f;
    do {
        // start vector
        if (o.v0_mode == QSD_V0_USER) {
            if (hipMemcpyAsync(S.x, d_evec, NR * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) {
                rc = fail(QSD_ERR_HIP, "copy failed");
                break;
            }
        } else {
            int64_t *spike = nullptr;
            if ((rc = dev_alloc(&spike, 1)) != QSD_OK) break;
            if (o.v0_mode == QSD_V0_MIN_DIAG) k_argmin<<<1, kRed, 0, st>>>(op.diag(), N, spike);
            k_init_v0<<<1024, kRed, 0, st>>>(S.x, NR, o.v0_mode, o.seed, spike, cplx ? 2 : 1);
            if (hipStreamSynchronize(st) != hipSuccess) rc = fail(QSD_ERR_HIP, "v0 failed");
            dev_free(spike);
            if (rc != QSD_OK) break;
        }
        k_sq_part<<<kDotBlocks, kRed, 0, st>>>(S.x, NR, S.part);
        k_scale<<<1024, kRed, 0, st>>>(S.x, NR, S.part, kDotBlocks);
        k_copy_row<<<1024, kRed, 0, st>>>(S.x, S.V, NR);
        k_zero<<<64, kRed, 0, st>>>(S.alpha, S.m);
        k_zero<<<64, kRed, 0, st>>>(S.beta, S.m);
        k_zero<<<1, 64, 0, st>>>(S.tri, 4);
        k_zero_i<<<1, 1, 0, st>>>(S.kdev);
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            rc = fail(QSD_ERR_HIP, "event create failed");
            break;
        }
        if (o.use_graph) {
            if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                rc = fail(QSD_ERR_HIP, "stream capture failed");
                break;
            }
            int erc = enqueue_iteration(op, S, f32, st);
            hipError_t ce = hipStreamEndCapture(st, &graph);
            if (erc != QSD_OK || ce != hipSuccess) {
                rc = erc != QSD_OK ? erc : fail(QSD_ERR_HIP, "end capture failed");
                break;
            }
            if (hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
                rc = fail(QSD_ERR_HIP, "graph instantiate failed");
                break;
            }
        }
        std::vector<double> tri(3);
        int done = 0;
        while (done < S.m) {
            const int nstep = std::min(o.check_every, S.m - done);
            for (int s = 0; s < nstep && rc == QSD_OK; ++s) {
                if (gexec) {
                    if (hipGraphLaunch(gexec, st) != hipSuccess) rc = fail(QSD_ERR_HIP, "graph launch failed");
                } else {
                    rc = enqueue_iteration(op, S, f32, st);
                }
            }
            if (rc != QSD_OK) break;
            done += nstep;
            k_tridiag<<<1, kRed, 0, st>>>(S.alpha, S.beta, done, S.tri);
            if (hipMemcpyAsync(tri.data(), S.tri, 3 * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                rc = fail(QSD_ERR_HIP, "Lanczos iteration failed: %s", hipGetErrorString(hipGetLastError()));
                break;
            }
            iters = done;
            if (tri[2] != 0.0) {
                // invariant subspace after tri[2] iterations: T of that size is exact
                iters = (int)tri[2];
                k_tridiag<<<1, kRed, 0, st>>>(S.alpha, S.beta, iters, S.tri);
                if (hipMemcpyAsync(tri.data(), S.tri, 2 * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess) {
                    rc = fail(QSD_ERR_HIP, "tridiagonal solve failed");
                    break;
                }
                theta = tri[0];
                ritz = 0.0;
                converged = true;
                break;
            }
            theta = tri[0];
            ritz = tri[1];
            if (ritz <= o.tol * std::fabs(theta)) {
                converged = true;
                break;
            }
        }
        if (rc != QSD_OK) break;
        // matvec timing: one extra timed SpMV (the Lanczos loop itself is not instrumented)
        hipEventRecord(e0, st);
        if (f32)
            rc = op.matvec(1, S.x32, 1, S.w32, 1, mv32, st);
        else
            rc = op.matvec(1, S.x, 1, S.w, 1, mv64, st);
        hipEventRecord(e1, st);
        if (rc != QSD_OK) break;
        hipEventSynchronize(e1);
        hipEventElapsedTime(&mv_ms, e0, e1);
        if (o.want_vector) {
            double *y = (double *)d_evec;
            k_gemv_n<<<gridN(NR), kRed, 0, st>>>(S.V, S.tri + 3, iters, NR, y);
            k_sq_part<<<kDotBlocks, kRed, 0, st>>>(y, NR, S.part);
            k_scale<<<1024, kRed, 0, st>>>(y, NR, S.part, kDotBlocks);
            if (op.takes(mv64)) {
                if ((rc = op.matvec(1, y, 1, S.w, 1, mv64, st)) != QSD_OK) break;
            } else {  // a stored FP32 matrix: the residual of the FP32 operator
                k_f64_to_f32<<<1024, kRed, 0, st>>>(y, S.x32, NR);
                if ((rc = op.matvec(1, S.x32, 1, S.w32, 1, mv32, st)) != QSD_OK) break;
                k_f32_to_f64<<<1024, kRed, 0, st>>>(S.w32, S.w, NR);
            }
            k_resid_part<<<kDotBlocks, kRed, 0, st>>>(S.w, y, theta, NR, S.part);
            std::vector<double> parts(kDotBlocks);
            if (hipMemcpyAsync(parts.data(), S.part, kDotBlocks * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                rc = fail(QSD_ERR_HIP, "residual failed");
                break;
            }
            double t = 0.0;
            for (double p : parts) t += p;
            expl = std::sqrt(t) / std::max(1e-300, std::fabs(theta));
        }
    } while (0);
    if (gexec) hipGraphExecDestroy(gexec);
    if (graph) hipGraphDestroy(graph);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    S.free_all();
    if (rc != QSD_OK) return rc;
    *eval_out = theta;
    if (info) {
        info->iterations = iters;
        info->converged = converged ? 1 : 0;
        info->ritz_residual = ritz;
        info->explicit_residual = expl;
        info->matvec_ms = mv_ms;
        info->total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    }
    if (!converged) return fail(QSD_ERR_NOT_CONVERGED, "Lanczos did not converge in %d iterations", iters);
    return QSD_OK;
}

}  // namespace

extern "C" int qsd_lanczos(const qsd_ham *h, const qsd_lanczos_opts *opts, double *eval_out, void *d_evec,
                           qsd_lanczos_info *info, void *stream) {
    clear_error();
    if (!h) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    SpmvOp op;
    op.h = h;
    return lanczos_impl(op, opts, eval_out, d_evec, info, stream);
}

extern "C" int qsd_csr_lanczos(const qsd_csr *c, const qsd_lanczos_opts *opts, double *eval_out, void *d_evec,
                               qsd_lanczos_info *info, void *stream) {
    clear_error();
    if (!c) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    SpmvOp op;
    op.c = c;
    return lanczos_impl(op, opts, eval_out, d_evec, info, stream);
}
