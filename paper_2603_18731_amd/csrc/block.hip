// Block Lanczos for the ground state: b vectors per step share every hash probe of the SpMM.
//
// Not in the paper (it hands its operator to external eigensolvers).  Per step k, with the
// orthonormal block X_k (N x b, rows interleaved as the SpMV expects) and the basis
// V = [X_0 .. X_k]:
//   W = H X_k                                       (SpMM, FP64 or FP32 elements)
//   C = V^T W; W -= V C   (twice)                   (block classical Gram-Schmidt, CGS2)
//   A_k = the X_k part of both C                    (diagonal block of T)
//   W = X_{k+1} B_k by Cholesky QR applied twice    (B_k upper triangular)
// T is block tridiagonal with bandwidth b; its lowest eigenvalue is found on the device by
// bisection with a banded Cholesky positive-definiteness test (T - sigma I is positive definite
// iff sigma is below every eigenvalue), its eigenvector s by inverse iteration, and the Ritz
// residual estimate is || B_k s_last || (s_last = the last b entries of s).
//
// As in the single-vector solver, every buffer has a fixed address and the step number lives
// in device memory, so one step is a fixed kernel sequence that can be captured in a HIP graph.
// All reductions use fixed partitions: results are bitwise reproducible.
#include <chrono>
#include <cmath>
#include <vector>

#include "common.h"

namespace qsd {
namespace {

constexpr int kThreads = 256;
constexpr int kGramTiles = 512;   // row tiles of the Gram reductions (a multiple of 4)
constexpr int kMaxSteps = 80;     // block steps for b = 4, 8; T is at most (kMaxSteps + 1) * b square
// Step limit per block size: the Ritz solve keeps T's band, (steps + 1) b rows of b + 1, in the
// LDS of one workgroup (gfx950 gives a workgroup up to 160 KB), so b = 16 takes at most 40 steps
// (a Krylov space of 640, 94 KB of band).
template <int B>
struct BlockLimits {
    static constexpr int steps = B <= 8 ? kMaxSteps : 40;
    static constexpr int ritz_rows = (steps + 1) * B;
    // coefficient blocks of C staged in LDS at a time by the update kernel (all of them for b <= 8)
    static constexpr int stage = B <= 8 ? kMaxSteps + 1 : 8;
};

struct BlzState {
    int64_t N = 0;
    int B = 0;
    int m = 0;                // block steps
    double *V = nullptr;      // [m+1][N][B]
    double *X = nullptr;      // [N][B] current block
    double *W = nullptr;      // [N][B]
    float *X32 = nullptr;
    float *W32 = nullptr;
    double *part = nullptr;   // [m+1][kGramTiles][B*B]
    double *C = nullptr;      // [m+1][B*B]
    double *A = nullptr;      // [B*B] diagonal block of the current step
    double *Rm = nullptr;     // [3][B*B]: R of pass 0, R of pass 1, inverse of the latest R
    double *Tb = nullptr;     // [(m+2)*B][B+1]: lower band of T, Tb[i][d] = T[i][i-d]
    double *flag = nullptr;   // [4]: [0] steps at an invariant subspace, [1] step with a rank-deficient block
    double *ritz = nullptr;   // [3 + (m+1)*B]: theta, residual estimate, -, s
    double *red = nullptr;    // [kGramTiles] scalar partial sums
    double *dead = nullptr;   // [(m+2)*B]: 1 for a deflated (zero) basis column
    int *kdev = nullptr;
    void free_all() {
        dev_free(V);
        dev_free(X);
        dev_free(W);
        dev_free(X32);
        dev_free(W32);
        dev_free(part);
        dev_free(C);
        dev_free(A);
        dev_free(Rm);
        dev_free(Tb);
        dev_free(flag);
        dev_free(ritz);
        dev_free(red);
        dev_free(dead);
        dev_free(kdev);
    }
};

// Basis blocks per launch row of the Gram kernel: J blocks keep J x B accumulators per lane,
// so J trades register pressure (occupancy) against re-reading W once per launch row.
template <int B>
constexpr int gram_blocks() {
    return 32 / B;
}

// part[j][tile] = sum over the tile's rows i of V_j[i][:]^T W[i][:] (B x B), j = 0 .. cnt-1,
// cnt = *kdev + 1 (or 1 without kdev).  gram_blocks<B>() basis blocks per launch row
// (blockIdx.y); lane p = tid % B owns column p of V_j and keeps a B x J accumulator tile.
template <int B>
__global__ __launch_bounds__(kThreads) void kbl_gram(const double *__restrict__ Vb, int64_t vstride,
                                                    const int *__restrict__ kdev, const double *__restrict__ W,
                                                    int64_t N, double *__restrict__ part) {
    constexpr int J = gram_blocks<B>();
    constexpr int RPB = kThreads / B;
    __shared__ double red[4][J][B][B];
    const int cnt = kdev ? *kdev + 1 : 1;
    const int j0 = blockIdx.y * J;
    if (j0 >= cnt) return;
    const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
    const int64_t a = (int64_t)blockIdx.x * chunk, e = min(N, a + chunk);
    const int p = threadIdx.x % B;
    double acc[J][B];
#pragma unroll
    for (int jj = 0; jj < J; ++jj)
#pragma unroll
        for (int q = 0; q < B; ++q) acc[jj][q] = 0.0;
    for (int64_t i = a + threadIdx.x / B; i < e; i += RPB) {
        double w[B];
#pragma unroll
        for (int q = 0; q < B; ++q) w[q] = W[i * B + q];
#pragma unroll
        for (int jj = 0; jj < J; ++jj) {
            if (j0 + jj < cnt) {
                const double v = Vb[(int64_t)(j0 + jj) * vstride + i * B + p];
#pragma unroll
                for (int q = 0; q < B; ++q) acc[jj][q] += v * w[q];
            }
        }
    }
    // lanes of one wave with the same p: offsets B, 2B, .. 32
#pragma unroll
    for (int jj = 0; jj < J; ++jj)
#pragma unroll
        for (int q = 0; q < B; ++q)
#pragma unroll
            for (int d = B; d < 64; d <<= 1) acc[jj][q] += __shfl_xor(acc[jj][q], d, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < B) {
#pragma unroll
        for (int jj = 0; jj < J; ++jj)
#pragma unroll
            for (int q = 0; q < B; ++q) red[wave][jj][lane][q] = acc[jj][q];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < J * B * B; t += kThreads) {
        const int jj = t / (B * B), pq = t % (B * B);
        if (j0 + jj < cnt) {
            const int pp = pq / B, qq = pq % B;
            part[((int64_t)(j0 + jj) * gridDim.x + blockIdx.x) * (B * B) + pq] =
                (red[0][jj][pp][qq] + red[1][jj][pp][qq]) + (red[2][jj][pp][qq] + red[3][jj][pp][qq]);
        }
    }
}

// C[j] = sum over tiles of part[j][tile] in tile order (four interleaved chains); the current
// block's coefficients are also added to A (the diagonal block of T) when A is given.
template <int B>
__global__ void kbl_reduce(const double *__restrict__ part, const int *__restrict__ kdev, double *__restrict__ C,
                           double *__restrict__ A) {
    const int cnt = kdev ? *kdev + 1 : 1;
    const int j = blockIdx.x, pq = threadIdx.x;
    if (j >= cnt || pq >= B * B) return;
    const double *pj = part + (int64_t)j * kGramTiles * (B * B) + pq;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int t = 0; t < kGramTiles; t += 4) {
        s0 += pj[(t + 0) * (B * B)];
        s1 += pj[(t + 1) * (B * B)];
        s2 += pj[(t + 2) * (B * B)];
        s3 += pj[(t + 3) * (B * B)];
    }
    const double s = (s0 + s1) + (s2 + s3);
    C[j * (B * B) + pq] = s;
    if (A && j == cnt - 1) A[pq] += s;
}

// W[i][q] -= sum_{j < cnt} sum_p V_j[i][p] C_j[p][q]; one thread per row (grid-stride), the row's
// B values of V_j read together, C staged in LDS (every lane reads the same entry: a broadcast).
template <int B>
__global__ __launch_bounds__(kThreads) void kbl_update(const double *__restrict__ Vb, int64_t vstride,
                                                      const int *__restrict__ kdev, const double *__restrict__ C,
                                                      double *__restrict__ W, int64_t N) {
    constexpr int JS = BlockLimits<B>::stage;  // blocks of C in LDS at a time
    __shared__ double Cs[JS * B * B];
    const int cnt = *kdev + 1;
    // the loop over row batches is uniform per workgroup, so every thread meets the barriers
    for (int64_t i0 = (int64_t)blockIdx.x * kThreads; i0 < N; i0 += (int64_t)gridDim.x * kThreads) {
        const int64_t i = i0 + threadIdx.x;
        const bool on = i < N;
        double acc[B];
#pragma unroll
        for (int q = 0; q < B; ++q) acc[q] = 0.0;
        for (int js = 0; js < cnt; js += JS) {
            const int jn = min(JS, cnt - js);
            __syncthreads();
            for (int t = threadIdx.x; t < jn * B * B; t += kThreads) Cs[t] = C[(int64_t)js * B * B + t];
            __syncthreads();
            if (!on) continue;
            for (int j = 0; j < jn; ++j) {
                double v[B];
#pragma unroll
                for (int p = 0; p < B; ++p) v[p] = Vb[(int64_t)(js + j) * vstride + i * B + p];
                const double *cj = Cs + j * B * B;
#pragma unroll
                for (int p = 0; p < B; ++p)
#pragma unroll
                    for (int q = 0; q < B; ++q) acc[q] += v[p] * cj[p * B + q];
            }
        }
        if (on) {
#pragma unroll
            for (int q = 0; q < B; ++q) W[i * B + q] -= acc[q];
        }
    }
}

// dst[i][q] = sum_{p <= q} src[i][p] Rinv[p][q]; also stored as basis block k + off when Vb is given.
template <int B>
__global__ __launch_bounds__(kThreads) void kbl_scale(const double *src, double *dst,  // may be the same buffer
                                                     const double *__restrict__ Rinv, int64_t N,
                                                     double *__restrict__ Vb, int64_t vstride,
                                                     const int *__restrict__ kdev, int off) {
    constexpr int RPB = kThreads / B;
    const int q = threadIdx.x % B;
    const int base = (threadIdx.x & 63) & ~(B - 1);
    double r[B];
#pragma unroll
    for (int p = 0; p < B; ++p) r[p] = Rinv[p * B + q];
    double *vdst = Vb ? Vb + (int64_t)((kdev ? *kdev : 0) + off) * vstride : nullptr;
    for (int64_t i = (int64_t)blockIdx.x * RPB + threadIdx.x / B; i < N; i += (int64_t)gridDim.x * RPB) {
        const double v = src[i * B + q];
        double acc = 0.0;
#pragma unroll
        for (int p = 0; p < B; ++p) {
            const double vp = __shfl(v, base + p, 64);
            if (p <= q) acc += vp * r[p];
        }
        dst[i * B + q] = acc;
        if (vdst) vdst[i * B + q] = acc;
    }
}

// Cholesky of the Gram matrix G (= C[0]) of a block: G = R^T R, R upper triangular.
//   mode 0 / 1: first / second pass on the start block;
//   mode 2 / 3: first / second pass at step k (mode 3 also writes A_k and B_k = R1 R0 into T).
// A column whose Schur pivot vanishes in absolute terms (squared norm <= 1e-24 ||A_k||_F^2, i.e.
// its residual direction is invariant to working accuracy) is deflated: its row of R and its
// column of R^-1 are zero, so that column of the next block is zero and stays zero; its indices
// in T are marked dead (decoupled, masked in the Ritz solve).  When every column vanishes the
// basis spans an invariant subspace: flag[0] = k + 1 (T is exact).  A pivot that is small only
// relative to the block (near dependence, beyond what Cholesky QR resolves: squared norm <= 1e-14
// of the block's largest) is deflated the same way at step k; the direction dropped is below 1e-7
// of the block's largest column, so the Ritz values stay Rayleigh quotients over an orthonormal
// basis and the run continues with the remaining columns.  In the start block it is an error:
// flag[1] = -1.
template <int B>
__global__ void kbl_chol(const double *__restrict__ G, int mode, const int *__restrict__ kdev, double *__restrict__ Rm,
                         double *__restrict__ A, double *__restrict__ Tb, double *__restrict__ dead,
                         double *__restrict__ flag) {
    if (threadIdx.x != 0) return;
    const int k = kdev ? *kdev : 0;
    double g[B][B], R[B][B], Ri[B][B];
    bool live[B];
    double gmax = 0.0;
    for (int p = 0; p < B; ++p)
        for (int q = 0; q < B; ++q) {
            g[p][q] = 0.5 * (G[p * B + q] + G[q * B + p]);
            R[p][q] = Ri[p][q] = 0.0;
        }
    for (int p = 0; p < B; ++p) gmax = fmax(gmax, g[p][p]);
    double ascale = 0.0;
    if (mode >= 2)
        for (int t = 0; t < B * B; ++t) ascale += A[t] * A[t];
    const double vanish = 1e-24 * ascale;  // zero for the start block
    bool near_dep = false;
    int nlive = 0;
    for (int p = 0; p < B; ++p) {
        double d = g[p][p];
        for (int r = 0; r < p; ++r) d -= R[r][p] * R[r][p];
        live[p] = false;
        if (!(d > vanish)) continue;          // vanished: deflated
        if (!(d > 1e-14 * gmax)) {            // near dependence
            near_dep = true;
            continue;
        }
        live[p] = true;
        ++nlive;
        const double rp = sqrt(d);
        R[p][p] = rp;
        for (int q = p + 1; q < B; ++q) {
            double s = g[p][q];
            for (int r = 0; r < p; ++r) s -= R[r][p] * R[r][q];
            R[p][q] = s / rp;
        }
    }
    // inverse of R restricted to the live indices (dead rows and columns stay zero)
    for (int q = 0; q < B; ++q) {
        if (!live[q]) continue;
        Ri[q][q] = 1.0 / R[q][q];
        for (int p = q - 1; p >= 0; --p) {
            if (!live[p]) continue;
            double s = 0.0;
            for (int r = p + 1; r <= q; ++r) s += R[p][r] * Ri[r][q];
            Ri[p][q] = -s / R[p][p];
        }
    }
    if (mode <= 1) {
        if (near_dep || nlive == 0) flag[1] = -1.0;
    } else if (flag[0] == 0.0 && flag[1] == 0.0 && nlive == 0 && !near_dep) {
        flag[0] = (double)(k + 1);
    }
    double *Rout = Rm + (mode & 1) * (B * B);
    for (int p = 0; p < B; ++p)
        for (int q = 0; q < B; ++q) {
            Rout[p * B + q] = R[p][q];
            Rm[2 * B * B + p * B + q] = Ri[p][q];
        }
    if (mode == 1)
        for (int p = 0; p < B; ++p) dead[p] = live[p] ? 0.0 : 1.0;
    if (mode == 3) {
        // B_k = R(pass 1) R(pass 0): rows (k+1)B + p, columns kB + q (q >= p) of T
        const double *R0 = Rm;
        for (int p = 0; p < B; ++p) {
            for (int q = p; q < B; ++q) {
                double s = 0.0;
                for (int r = p; r <= q; ++r) s += R[p][r] * R0[r * B + q];
                Tb[(int64_t)((k + 1) * B + p) * (B + 1) + (B + p - q)] = s;
            }
            dead[(k + 1) * B + p] = live[p] ? 0.0 : 1.0;
        }
        // A_k (symmetrized): rows kB + p, columns kB + q (q <= p); then cleared for the next step
        for (int p = 0; p < B; ++p)
            for (int q = 0; q <= p; ++q)
                Tb[(int64_t)(k * B + p) * (B + 1) + (p - q)] = 0.5 * (A[p * B + q] + A[q * B + p]);
        for (int t = 0; t < B * B; ++t) A[t] = 0.0;
    }
}

__global__ void kbl_bump(int *kdev) { *kdev += 1; }

// Start block: column 0 uniform, spike at the lowest diagonal element, random or the caller's
// vector; columns 1 .. B-1 random (splitmix64 of (seed, column, row), uniform in [-1, 1)).
template <int B>
__global__ void kbl_init(double *__restrict__ X, int64_t N, int mode, uint64_t seed, const int64_t *__restrict__ spike,
                         const double *__restrict__ user) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N * B; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / B;
        const int p = (int)(t % B);
        double v;
        if (p == 0 && mode == QSD_V0_UNIFORM) {
            v = 1.0;
        } else if (p == 0 && mode == QSD_V0_MIN_DIAG) {
            v = (i == *spike) ? 1.0 : 0.0;
        } else if (p == 0 && mode == QSD_V0_USER) {
            v = user[i];
        } else {
            uint64_t z = seed + (uint64_t)p * 0xD1B54A32D192ED03ull + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            v = (double)(z >> 11) * 0x1.0p-52 - 1.0;
        }
        X[t] = v;
    }
}

__global__ __launch_bounds__(kThreads) void kbl_argmin(const double *__restrict__ d, int64_t N, int64_t *__restrict__ out) {
    __shared__ double bv[kThreads];
    __shared__ int64_t bi[kThreads];
    double v = INFINITY;
    int64_t idx = 0;
    for (int64_t i = threadIdx.x; i < N; i += kThreads)
        if (d[i] < v) {
            v = d[i];
            idx = i;
        }
    bv[threadIdx.x] = v;
    bi[threadIdx.x] = idx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < kThreads; ++t)
            if (bv[t] < v || (bv[t] == v && bi[t] < idx)) {
                v = bv[t];
                idx = bi[t];
            }
        *out = idx;
    }
}

// Banded Cholesky of M (lower band, M[r][d] = M(r, r-d)) in place by one wave; returns false
// at the first non-positive pivot.  Pairs (a, b), 1 <= b <= a <= B, of the trailing update are
// spread over lanes.
template <int B>
__device__ bool band_chol(double *M, int n, int lane) {
    // pair number t -> (a, b): t = a (a - 1) / 2 + (b - 1); each pair updates its own element of
    // the band from column i only, so the pairs are independent (b = 16 has 136 of them, taken
    // 64 at a time)
    constexpr int kPairs = B * (B + 1) / 2;
    constexpr int kRounds = (kPairs + 63) / 64;
    int pa[kRounds], pb[kRounds];
#pragma unroll
    for (int k = 0; k < kRounds; ++k) {
        int t = lane + 64 * k, a = 1;
        while (a <= B && t >= a) {
            t -= a;
            ++a;
        }
        pa[k] = a;
        pb[k] = t + 1;  // valid when a <= B
    }
    for (int i = 0; i < n; ++i) {
        const double piv = M[i * (B + 1)];
        if (!(piv > 0.0)) return false;
        const double l = sqrt(piv);
        __syncthreads();
        if (lane >= 1 && lane <= B && i + lane < n) M[(i + lane) * (B + 1) + lane] /= l;
        if (lane == 0) M[i * (B + 1)] = l;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kRounds; ++k) {
            if (pa[k] <= B && i + pa[k] < n) {
                const int r = i + pa[k], c = i + pb[k];
                M[r * (B + 1) + (pa[k] - pb[k])] -= M[r * (B + 1) + pa[k]] * M[c * (B + 1) + pb[k]];
            }
        }
        __syncthreads();
    }
    return true;
}

// M = T - sigma I (lower band); a dead index gets the diagonal `big` (its row and column are
// zero), which moves its decoupled eigenvalue above the spectrum of the rest.
template <int B>
__device__ void band_load(double *M, const double *__restrict__ Tb, const double *__restrict__ dead, double big, int n,
                          double sigma, int lane) {
    for (int t = lane; t < n * (B + 1); t += 64) {
        const int r = t / (B + 1), d = t % (B + 1);
        double v = (r - d >= 0) ? Tb[t] : 0.0;
        if (d == 0) v = (dead[r] != 0.0 ? big : v) - sigma;
        M[t] = v;
    }
    __syncthreads();
}

// Lowest eigenvalue of the leading n x n part of T (n = nblocks * B) by bisection, its
// eigenvector by inverse iteration, and the residual estimate || B s_last ||.  One wave.
template <int B>
__global__ __launch_bounds__(64) void kbl_ritz(const double *__restrict__ Tb, const double *__restrict__ dead, int nblocks,
                                               double *__restrict__ out) {
    __shared__ double M[BlockLimits<B>::ritz_rows * (B + 1)];
    __shared__ double z[BlockLimits<B>::ritz_rows];
    __shared__ double sh[2];
    const int n = nblocks * B;
    const int lane = threadIdx.x;
    // Gershgorin lower bound and min diagonal (an upper bound on the lowest eigenvalue)
    double glo = INFINITY, dmin = INFINITY, tnorm = 0.0;
    for (int i = lane; i < n; i += 64) {
        if (dead[i] != 0.0) continue;
        double off = 0.0;
        for (int d = 1; d <= B; ++d) {
            if (i - d >= 0) off += fabs(Tb[i * (B + 1) + d]);
            if (i + d < n) off += fabs(Tb[(i + d) * (B + 1) + d]);
        }
        const double t = Tb[i * (B + 1)];
        glo = fmin(glo, t - off);
        dmin = fmin(dmin, t);
        tnorm = fmax(tnorm, fabs(t) + off);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        glo = fmin(glo, __shfl_xor(glo, d, 64));
        dmin = fmin(dmin, __shfl_xor(dmin, d, 64));
        tnorm = fmax(tnorm, __shfl_xor(tnorm, d, 64));
    }
    const double big = 2.0 * tnorm + 1.0;
    double lo = glo - 1e-12 * tnorm - 1e-300, hi = dmin;
    for (int it = 0; it < 200 && hi - lo > 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        band_load<B>(M, Tb, dead, big, n, mid, lane);
        if (band_chol<B>(M, n, lane))
            lo = mid;
        else
            hi = mid;
    }
    const double theta = 0.5 * (lo + hi);
    // inverse iteration with the factor of T - lo I (positive definite)
    band_load<B>(M, Tb, dead, big, n, lo, lane);
    const bool ok = band_chol<B>(M, n, lane);
    for (int i = lane; i < n; i += 64) z[i] = 1.0 + 0.01 * (double)((i * 37) % 11);
    __syncthreads();
    for (int rep = 0; rep < 3 && ok; ++rep) {
        // forward: L y = z
        for (int i = 0; i < n; ++i) {
            double s = (lane >= 1 && lane <= B && i - lane >= 0) ? M[i * (B + 1) + lane] * z[i - lane] : 0.0;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
            __syncthreads();
            if (lane == 0) z[i] = (z[i] - s) / M[i * (B + 1)];
            __syncthreads();
        }
        // backward: L^T x = y
        for (int i = n - 1; i >= 0; --i) {
            double s = (lane >= 1 && lane <= B && i + lane < n) ? M[(i + lane) * (B + 1) + lane] * z[i + lane] : 0.0;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
            __syncthreads();
            if (lane == 0) z[i] = (z[i] - s) / M[i * (B + 1)];
            __syncthreads();
        }
        double nn = 0.0;
        for (int i = lane; i < n; i += 64) nn += z[i] * z[i];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) nn += __shfl_xor(nn, d, 64);
        const double inv = 1.0 / sqrt(nn);
        __syncthreads();
        for (int i = lane; i < n; i += 64) z[i] *= inv;
        __syncthreads();
    }
    // residual estimate: B_k (rows n .. n+B-1, columns n-B .. n-1, upper triangular) times s_last
    double r2 = 0.0;
    if (lane < B) {
        const int p = lane;
        double s = 0.0;
        for (int q = p; q < B; ++q) s += Tb[(int64_t)(n + p) * (B + 1) + (B + p - q)] * z[n - B + q];
        r2 = s * s;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) r2 += __shfl_xor(r2, d, 64);
    if (lane == 0) {
        out[0] = theta;
        out[1] = ok ? sqrt(r2) : INFINITY;
        out[2] = hi - lo;
    }
    for (int i = lane; i < n; i += 64) out[3 + i] = z[i];
    (void)sh;
}

// y[i] = sum_{j < nblocks} sum_p V_j[i][p] s[jB + p]
template <int B>
__global__ __launch_bounds__(kThreads) void kbl_ritzvec(const double *__restrict__ Vb, int64_t vstride, int nblocks,
                                                       const double *__restrict__ s, double *__restrict__ y, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < nblocks; ++j)
#pragma unroll
            for (int p = 0; p < B; ++p) acc += Vb[(int64_t)j * vstride + i * B + p] * s[j * B + p];
        y[i] = acc;
    }
}

__global__ __launch_bounds__(kThreads) void kbl_sq(const double *__restrict__ a, const double *__restrict__ b, double c,
                                                  int64_t N, double *__restrict__ part) {
    // part[block] = sum over the block's chunk of (a - c b)^2  (b may be NULL)
    __shared__ double ws[kThreads / 64];
    const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
    const int64_t s0 = (int64_t)blockIdx.x * chunk, e = min(N, s0 + chunk);
    double s = 0.0;
    for (int64_t i = s0 + threadIdx.x; i < e; i += kThreads) {
        const double v = b ? a[i] - c * b[i] : a[i];
        s += v * v;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t += ws[w];
        part[blockIdx.x] = t;
    }
}

__global__ void kbl_scale_vec(double *__restrict__ y, int64_t N, const double *__restrict__ part, int nparts) {
    __shared__ double inv;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < nparts; ++k) t += part[k];
        inv = 1.0 / sqrt(t);
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        y[i] *= inv;
}

__global__ void kbl_to_f32(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}
__global__ void kbl_to_f64(const float *__restrict__ a, double *__restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (double)a[i];
}
__global__ void kbl_zero(double *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}
__global__ void kbl_zero_i(int *p) { *p = 0; }

inline unsigned rows_grid(int64_t N, int B) {
    const int64_t rpb = kThreads / B;
    return (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (N + rpb - 1) / rpb));
}

// Cholesky QR (twice) of the block in W: W <- W R0^-1, then dst <- W R1^-1 (and basis block
// k + off when Vb is given).  mode_base 0: start block, 2: step k (writes T).
template <int B>
void enqueue_cholqr2(BlzState &S, double *dst, double *Vb, int off, int mode_base, hipStream_t st) {
    const int64_t N = S.N;
    const int *kd = mode_base >= 2 ? S.kdev : nullptr;
    for (int pass = 0; pass < 2; ++pass) {
        kbl_gram<B><<<dim3(kGramTiles, 1), kThreads, 0, st>>>(S.W, 0, nullptr, S.W, N, S.part);
        kbl_reduce<B><<<1, B * B < 64 ? 64 : B * B, 0, st>>>(S.part, nullptr, S.C, nullptr);
        kbl_chol<B><<<1, 64, 0, st>>>(S.C, mode_base + pass, kd, S.Rm, S.A, S.Tb, S.dead, S.flag);
        if (pass == 0)
            kbl_scale<B><<<rows_grid(N, B), kThreads, 0, st>>>(S.W, S.W, S.Rm + 2 * B * B, N, nullptr, 0, nullptr, 0);
        else
            kbl_scale<B><<<rows_grid(N, B), kThreads, 0, st>>>(S.W, dst, S.Rm + 2 * B * B, N, Vb, N * B, kd, off);
    }
}

template <int B>
int enqueue_step(const SpmvOp &op, BlzState &S, bool f32, hipStream_t st) {
    const int64_t N = S.N;
    if (f32) {
        kbl_to_f32<<<1024, kThreads, 0, st>>>(S.X, S.X32, N * B);
        QSD_TRY(op.matvec(B, S.X32, B, S.W32, B, QSD_F32, st));
        kbl_to_f64<<<1024, kThreads, 0, st>>>(S.W32, S.W, N * B);
    } else {
        QSD_TRY(op.matvec(B, S.X, B, S.W, B, QSD_F64, st));
    }
    const unsigned jy = (unsigned)((S.m + 1 + gram_blocks<B>() - 1) / gram_blocks<B>());
    for (int pass = 0; pass < 2; ++pass) {
        kbl_gram<B><<<dim3(kGramTiles, jy), kThreads, 0, st>>>(S.V, N * B, S.kdev, S.W, N, S.part);
        kbl_reduce<B><<<S.m + 1, B * B < 64 ? 64 : B * B, 0, st>>>(S.part, S.kdev, S.C, S.A);
        kbl_update<B><<<rows_grid(N, B), kThreads, 0, st>>>(S.V, N * B, S.kdev, S.C, S.W, N);
    }
    enqueue_cholqr2<B>(S, S.X, S.V, 1, 2, st);
    kbl_bump<<<1, 1, 0, st>>>(S.kdev);
    QSD_CHECK_HIP(hipGetLastError());
    return QSD_OK;
}

template <int B>
int block_lanczos(const SpmvOp &op, const qsd_lanczos_opts &o, double *eval_out, void *d_evec, qsd_lanczos_info *info,
                  hipStream_t st) {
    auto t_start = std::chrono::steady_clock::now();
    const int64_t N = op.N();
    BlzState S;
    S.N = N;
    S.B = B;
    S.m = (int)std::min<int64_t>(o.max_iter, N / B - 1);
    if (S.m < 1) return fail(QSD_ERR_INVALID_ARG, "subspace of %lld strings is too small for blocks of %d",
                             (long long)N, B);
    const bool f32 = o.spmv_dtype == QSD_F32;
    int rc = QSD_OK;
    auto alloc_all = [&]() -> int {
        QSD_TRY(dev_alloc(&S.V, (size_t)(S.m + 1) * N * B));
        QSD_TRY(dev_alloc(&S.X, (size_t)N * B));
        QSD_TRY(dev_alloc(&S.W, (size_t)N * B));
        if (f32) {
            QSD_TRY(dev_alloc(&S.X32, (size_t)N * B));
            QSD_TRY(dev_alloc(&S.W32, (size_t)N * B));
        }
        QSD_TRY(dev_alloc(&S.part, (size_t)(S.m + 1) * kGramTiles * B * B));
        QSD_TRY(dev_alloc(&S.C, (size_t)(S.m + 1) * B * B));
        QSD_TRY(dev_alloc(&S.A, (size_t)B * B));
        QSD_TRY(dev_alloc(&S.Rm, (size_t)3 * B * B));
        QSD_TRY(dev_alloc(&S.Tb, (size_t)(S.m + 2) * B * (B + 1)));
        QSD_TRY(dev_alloc(&S.flag, 4));
        QSD_TRY(dev_alloc(&S.ritz, (size_t)3 + (S.m + 1) * B));
        QSD_TRY(dev_alloc(&S.red, kGramTiles));
        QSD_TRY(dev_alloc(&S.dead, (size_t)(S.m + 2) * B));
        QSD_TRY(dev_alloc(&S.kdev, 1));
        return QSD_OK;
    };
    if ((rc = alloc_all()) != QSD_OK) {
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
        kbl_zero<<<64, kThreads, 0, st>>>(S.Tb, (int64_t)(S.m + 2) * B * (B + 1));
        kbl_zero<<<1, 64, 0, st>>>(S.A, B * B);
        kbl_zero<<<1, 64, 0, st>>>(S.flag, 4);
        kbl_zero<<<4, 256, 0, st>>>(S.dead, (int64_t)(S.m + 2) * B);
        kbl_zero_i<<<1, 1, 0, st>>>(S.kdev);
        int64_t *spike = nullptr;
        if ((rc = dev_alloc(&spike, 1)) != QSD_OK) break;
        if (o.v0_mode == QSD_V0_MIN_DIAG) kbl_argmin<<<1, kThreads, 0, st>>>(op.diag(), N, spike);
        kbl_init<B><<<1024, kThreads, 0, st>>>(S.W, N, o.v0_mode, o.seed, spike, (const double *)d_evec);
        enqueue_cholqr2<B>(S, S.X, S.V, 0, 0, st);
        std::vector<double> fl(4);
        if (hipMemcpyAsync(fl.data(), S.flag, 32, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = fail(QSD_ERR_HIP, "start block failed: %s", hipGetErrorString(hipGetLastError()));
        dev_free(spike);
        if (rc != QSD_OK) break;
        if (fl[1] != 0.0) {
            rc = fail(QSD_ERR_INVALID_ARG, "the start block is rank-deficient");
            break;
        }
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            rc = fail(QSD_ERR_HIP, "event create failed");
            break;
        }
        if (o.use_graph) {
            if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                rc = fail(QSD_ERR_HIP, "stream capture failed");
                break;
            }
            int erc = enqueue_step<B>(op, S, f32, st);
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
        std::vector<double> rz(3);
        int done = 0;
        while (done < S.m) {
            const int nstep = std::min(o.check_every, S.m - done);
            for (int s = 0; s < nstep && rc == QSD_OK; ++s) {
                if (gexec) {
                    if (hipGraphLaunch(gexec, st) != hipSuccess) rc = fail(QSD_ERR_HIP, "graph launch failed");
                } else {
                    rc = enqueue_step<B>(op, S, f32, st);
                }
            }
            if (rc != QSD_OK) break;
            done += nstep;
            if (hipMemcpyAsync(fl.data(), S.flag, 32, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                rc = fail(QSD_ERR_HIP, "block Lanczos step failed: %s", hipGetErrorString(hipGetLastError()));
                break;
            }
            const int inv_at = (int)fl[0], def_at = (int)fl[1];
            const int nb = inv_at > 0 ? inv_at : def_at > 0 ? def_at : done;
            kbl_ritz<B><<<1, 64, 0, st>>>(S.Tb, S.dead, nb, S.ritz);
            if (hipMemcpyAsync(rz.data(), S.ritz, 3 * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                rc = fail(QSD_ERR_HIP, "Ritz solve failed: %s", hipGetErrorString(hipGetLastError()));
                break;
            }
            iters = nb;
            theta = rz[0];
            // an invariant subspace makes T exact; after a nearly dependent residual block the
            // stored B_k says nothing about the residual
            ritz = inv_at > 0 ? 0.0 : def_at > 0 ? INFINITY : rz[1];
            if (ritz <= o.tol * std::fabs(theta)) {
                converged = true;
                break;
            }
            if (inv_at > 0 || def_at > 0) break;  // cannot continue past a nearly dependent block
        }
        if (rc != QSD_OK) break;
        hipEventRecord(e0, st);
        if (f32)
            rc = op.matvec(B, S.X32, B, S.W32, B, QSD_F32, st);
        else
            rc = op.matvec(B, S.X, B, S.W, B, QSD_F64, st);
        hipEventRecord(e1, st);
        if (rc != QSD_OK) break;
        hipEventSynchronize(e1);
        hipEventElapsedTime(&mv_ms, e0, e1);
        if (o.want_vector) {
            double *y = (double *)d_evec;
            const unsigned g = (unsigned)std::min<int64_t>(4096, (N + kThreads - 1) / kThreads);
            kbl_ritzvec<B><<<g, kThreads, 0, st>>>(S.V, N * B, iters, S.ritz + 3, y, N);
            kbl_sq<<<kGramTiles, kThreads, 0, st>>>(y, nullptr, 0.0, N, S.red);
            kbl_scale_vec<<<g, kThreads, 0, st>>>(y, N, S.red, kGramTiles);
            if (op.takes(QSD_F64)) {
                if ((rc = op.matvec(1, y, 1, S.W, 1, QSD_F64, st)) != QSD_OK) break;
            } else {  // a stored FP32 matrix: the residual of the FP32 operator
                kbl_to_f32<<<1024, kThreads, 0, st>>>(y, S.X32, N);
                if ((rc = op.matvec(1, S.X32, 1, S.W32, 1, QSD_F32, st)) != QSD_OK) break;
                kbl_to_f64<<<1024, kThreads, 0, st>>>(S.W32, S.W, N);
            }
            kbl_sq<<<kGramTiles, kThreads, 0, st>>>(S.W, y, theta, N, S.red);
            std::vector<double> parts(kGramTiles);
            if (hipMemcpyAsync(parts.data(), S.red, kGramTiles * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
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
    if (!converged)
        return fail(QSD_ERR_NOT_CONVERGED, "block Lanczos did not converge in %d steps (Ritz residual %.3e)", iters,
                    ritz);
    return QSD_OK;
}

}  // namespace
}  // namespace qsd

using namespace qsd;

namespace {

int block_entry(const SpmvOp &op, int32_t block, const qsd_lanczos_opts *opts, double *eval_out, void *d_evec,
                qsd_lanczos_info *info, void *stream) {
    if (!eval_out) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    qsd_lanczos_opts o;
    qsd_lanczos_default_opts(&o);
    if (opts) o = *opts;
    if (op.is_complex()) return fail(QSD_ERR_UNSUPPORTED, "block Lanczos for complex operators is not implemented");
    if (block != 4 && block != 8 && block != 16) return fail(QSD_ERR_INVALID_ARG, "block must be 4, 8 or 16");
    const int max_steps = block == 16 ? BlockLimits<16>::steps : kMaxSteps;
    if (o.max_iter < 1 || o.max_iter > max_steps)
        return fail(QSD_ERR_INVALID_ARG, "max_iter (block steps) must be in [1, %d] for block %d", max_steps, block);
    if (!(o.tol > 0)) return fail(QSD_ERR_INVALID_ARG, "tol must be > 0");
    if (o.spmv_dtype != QSD_F64 && o.spmv_dtype != QSD_F32) return fail(QSD_ERR_DTYPE, "spmv_dtype must be F64 or F32");
    if (!op.takes(o.spmv_dtype)) return fail(QSD_ERR_DTYPE, "spmv_dtype must be the stored matrix's dtype");
    if (o.v0_mode < QSD_V0_UNIFORM || o.v0_mode > QSD_V0_USER) return fail(QSD_ERR_INVALID_ARG, "bad v0_mode");
    if ((o.v0_mode == QSD_V0_USER || o.want_vector) && !d_evec)
        return fail(QSD_ERR_INVALID_ARG, "d_evec is required for QSD_V0_USER / want_vector");
    if (o.check_every < 1) o.check_every = 1;
    hipStream_t st = (hipStream_t)stream;
    AllocScope scope(o.alloc ? o.alloc : op.allocator(), stream);
    return block == 16 ? block_lanczos<16>(op, o, eval_out, d_evec, info, st)
           : block == 8 ? block_lanczos<8>(op, o, eval_out, d_evec, info, st)
                        : block_lanczos<4>(op, o, eval_out, d_evec, info, st);
}

}  // namespace

extern "C" int qsd_block_lanczos(const qsd_ham *h, int32_t block, const qsd_lanczos_opts *opts, double *eval_out,
                                 void *d_evec, qsd_lanczos_info *info, void *stream) {
    clear_error();
    if (!h) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    SpmvOp op;
    op.h = h;
    return block_entry(op, block, opts, eval_out, d_evec, info, stream);
}

extern "C" int qsd_csr_block_lanczos(const qsd_csr *c, int32_t block, const qsd_lanczos_opts *opts, double *eval_out,
                                     void *d_evec, qsd_lanczos_info *info, void *stream) {
    clear_error();
    if (!c) return fail(QSD_ERR_INVALID_ARG, "NULL argument");
    SpmvOp op;
    op.c = c;
    return block_entry(op, block, opts, eval_out, d_evec, info, stream);
}
