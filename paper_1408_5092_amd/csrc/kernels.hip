// gfx950 kernels of the MPS-PT engine and the host side of device.hpp.
//
// * k_gemm_grouped: output-stationary grouped FP64 GEMM on MFMA
//   (v_mfma_f64_16x16x4f64).  A 256-thread workgroup owns one 32x32 tile of
//   one output block and sums every term of that block in list order, so a
//   block-sparse contraction is one launch and its result is deterministic.
// * k_axpy_grouped: linear combinations of dense blocks (MPO coefficients).
// * k_diag_grouped: Jacobi diagonal of the effective operator.
// * k_eig_jacobi: cyclic two-sided Jacobi eigensolver, one workgroup per
//   symmetric matrix, parallel rotations in round-robin order.
// * CG vector kernels with fixed-order two-pass reductions.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstdio>
#include <unordered_map>
#include <vector>

#include "../../include/mpspt.h"
#include "device.hpp"

namespace mpspt {
namespace dev {

namespace {
hipStream_t g_stream = nullptr;
int g_eig_lds_max = 0;
size_t g_lds_budget = 0;

void check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        int code = (e == hipErrorOutOfMemory) ? MPSPT_E_NOMEM : MPSPT_E_HIP;
        throw Error{code, std::string(what) + ": " + hipGetErrorString(e)};
    }
}

constexpr int TILE = 32;
constexpr int KC = 16;
constexpr int RED_THREADS = 256;

typedef double d4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------- GEMM
__global__ __launch_bounds__(256) void k_gemm_grouped(const GemmGroup* __restrict__ G, int ngroups,
                                                      const GemmTerm* __restrict__ T) {
    const int bid = blockIdx.x;
    int lo = 0, hi = ngroups - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (G[mid].tile0 <= bid) lo = mid;
        else hi = mid - 1;
    }
    const GemmGroup g = G[lo];
    const int tiles_n = (g.n + TILE - 1) / TILE;
    const int t = bid - g.tile0;
    const int row0 = (t / tiles_n) * TILE;
    const int col0 = (t % tiles_n) * TILE;

    __shared__ double As[KC][TILE + 1];  // op(A)[row0 + i][k0 + kk] at As[kk][i]
    __shared__ double Bs[KC][TILE + 1];  // op(B)[k0 + kk][col0 + j] at Bs[kk][j]
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 16, wn = (wave & 1) * 16;
    d4 acc = {0.0, 0.0, 0.0, 0.0};

    for (int ti = 0; ti < g.nterms; ++ti) {
        const GemmTerm tm = T[g.term0 + ti];
        for (int k0 = 0; k0 < tm.k; k0 += KC) {
            // A tile: 32 x 16 values, two per thread
            for (int e = tid; e < TILE * KC; e += 256) {
                int i, kk;
                if (tm.transA) { i = e % TILE; kk = e / TILE; }
                else { kk = e % KC; i = e / KC; }
                const int gi = row0 + i, gk = k0 + kk;
                double v = 0.0;
                if (gi < g.m && gk < tm.k)
                    v = tm.transA ? tm.A[(size_t)gk * tm.lda + gi] : tm.A[(size_t)gi * tm.lda + gk];
                As[kk][i] = v;
            }
            for (int e = tid; e < TILE * KC; e += 256) {
                int j, kk;
                if (tm.transB) { kk = e % KC; j = e / KC; }
                else { j = e % TILE; kk = e / TILE; }
                const int gj = col0 + j, gk = k0 + kk;
                double v = 0.0;
                if (gj < g.n && gk < tm.k)
                    v = tm.transB ? tm.B[(size_t)gj * tm.ldb + gk] : tm.B[(size_t)gk * tm.ldb + gj];
                Bs[kk][j] = v * tm.alpha;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < KC; kk += 4) {
                const double a = As[kk + (lane >> 4)][wm + (lane & 15)];
                const double b = Bs[kk + (lane >> 4)][wn + (lane & 15)];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
            __syncthreads();
        }
    }
    // accumulator register e of a lane holds D[lane / 16 + 4 e][lane % 16]
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int gi = row0 + wm + (lane >> 4) + 4 * e;
        const int gj = col0 + wn + (lane & 15);
        if (gi < g.m && gj < g.n) {
            double* c = g.C + (size_t)gi * g.ldc + gj;
            *c = g.accumulate ? *c + acc[e] : acc[e];
        }
    }
}

// ------------------------------------------------------------------- AXPY
__global__ __launch_bounds__(256) void k_axpy_grouped(const AxpyGroup* __restrict__ G,
                                                      const AxpyTerm* __restrict__ T) {
    const AxpyGroup g = G[blockIdx.x];
    const int total = g.m * g.n;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int i = e / g.n, j = e - i * g.n;
        double s = g.accumulate ? g.dst[(size_t)i * g.ldd + j] : 0.0;
        for (int t = 0; t < g.nterms; ++t) {
            const AxpyTerm tm = T[g.term0 + t];
            s += tm.alpha * (tm.trans ? tm.src[(size_t)j * tm.lds + i] : tm.src[(size_t)i * tm.lds + j]);
        }
        g.dst[(size_t)i * g.ldd + j] = s;
    }
}

// ------------------------------------------------------------------- DIAG
__global__ __launch_bounds__(256) void k_diag_grouped(const DiagGroup* __restrict__ G,
                                                      const DiagTerm* __restrict__ T) {
    const DiagGroup g = G[blockIdx.x];
    const int total = g.m * g.n;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int i = e / g.n, j = e - i * g.n;
        double s = g.shift;
        for (int t = 0; t < g.nterms; ++t) {
            const DiagTerm tm = T[g.term0 + t];
            s += tm.c * tm.L[(size_t)i * tm.ls] * tm.R[(size_t)j * tm.rs];
        }
        g.dst[(size_t)i * g.ldd + j] = s;
    }
}

// ------------------------------------------------------------------ EIGEN
__device__ double block_sum(double v, double* red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_eig_jacobi(const EigJob* __restrict__ jobs) {
    const EigJob J = jobs[blockIdx.x];
    const int n = J.n;
    double* A = J.A;
    double* V = J.V;
    const int tid = threadIdx.x;
    __shared__ double red[256];
    __shared__ double cs[256], sn[256];
    __shared__ int pp[256], qq[256];
    for (int e = tid; e < n * n; e += blockDim.x) V[e] = (e / n == e % n) ? 1.0 : 0.0;
    __syncthreads();
    const int m = n + (n & 1);
    const int npair = m / 2;
    for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < n * n; e += blockDim.x) {
            const double a = A[e];
            tot += a * a;
            if (e / n != e % n) off += a * a;
        }
        off = block_sum(off, red);
        tot = block_sum(tot, red);
        if (off <= 1e-30 * tot || tot == 0.0) break;
        for (int round = 0; round < m - 1; ++round) {
            for (int k = tid; k < npair; k += blockDim.x) {
                int p = (round + k) % (m - 1);
                int q = (k == 0) ? (m - 1) : (round - k + m - 1) % (m - 1);
                if (p > q) { int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = A[p * n + q];
                    if (apq != 0.0) {
                        const double app = A[p * n + p], aqq = A[q * n + q];
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                }
                pp[k] = p; qq[k] = q; cs[k] = c; sn[k] = s;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int e = tid; e < npair * n; e += blockDim.x) {
                const int k = e / n, j = e - k * n;
                const int p = pp[k], q = qq[k];
                if (q >= n || sn[k] == 0.0) continue;
                const double c = cs[k], s = sn[k];
                const double ap = A[p * n + j], aq = A[q * n + j];
                A[p * n + j] = c * ap - s * aq;
                A[q * n + j] = s * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (int e = tid; e < npair * n; e += blockDim.x) {
                const int k = e / n, i = e - k * n;
                const int p = pp[k], q = qq[k];
                if (q >= n || sn[k] == 0.0) continue;
                const double c = cs[k], s = sn[k];
                const double ap = A[i * n + p], aq = A[i * n + q];
                A[i * n + p] = c * ap - s * aq;
                A[i * n + q] = s * ap + c * aq;
                const double vp = V[i * n + p], vq = V[i * n + q];
                V[i * n + p] = c * vp - s * vq;
                V[i * n + q] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
    // eigenvalues descending (ties by index); eigenvectors into A
    for (int i = tid; i < n; i += blockDim.x) J.w[i] = A[i * n + i];
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
        const double di = J.w[i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double dj = J.w[j];
            rank += (dj > di) || (dj == di && j < i);
        }
        for (int r = 0; r < n; ++r) A[r * n + rank] = V[r * n + i];
    }
    __syncthreads();
    // sorted eigenvalues: write through V's diagonal slot then back
    for (int i = tid; i < n; i += blockDim.x) {
        const double di = J.w[i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double dj = J.w[j];
            rank += (dj > di) || (dj == di && j < i);
        }
        V[rank] = di;
    }
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) J.w[i] = V[i];
}

__device__ double block_sum_1024(double v, double* red16) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red16[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < 16; ++w) s += red16[w];
    __syncthreads();
    return s;
}

// Round-robin Jacobi on the packed upper triangle held in LDS.  The disjoint
// rotations of one round act on the matrix as J^T A J with J block diagonal in
// the pair basis, so every 2x2 block formed by two pairs (k1 <= k2) is
// updated independently: B' = G(k1) B G(k2)^T, with the diagonal blocks set
// by the closed Jacobi form (a_pq' = 0).  One barrier per round.  The
// transposed eigenvector matrix lives in LDS (VT_LDS) or in the job's V
// workspace.
__device__ __forceinline__ int tri_off(int i, int n) { return i * n - (i * (i - 1)) / 2; }
__device__ __forceinline__ int tri_idx(int i, int j, int n) {  // i <= j
    return tri_off(i, n) + (j - i);
}

template <bool VT_LDS>
__global__ __launch_bounds__(1024) void k_eig_jacobi_packed(const EigJob* __restrict__ jobs) {
    extern __shared__ double lds[];
    const EigJob J = jobs[blockIdx.x];
    const int n = J.n;
    const int tid = threadIdx.x;
    double* P = lds;                                           // n (n + 1) / 2
    double* Vt = VT_LDS ? lds + (n * (n + 1)) / 2 : J.V;       // n x n, row p = eigenvector p
    __shared__ double red16[16];
    __shared__ double cs[128], sn[128];
    __shared__ int pp[128], qq[128];
    for (int e = tid; e < n * n; e += 1024) {
        const int i = e / n, j = e - i * n;
        if (i <= j) P[tri_idx(i, j, n)] = J.A[e];
        Vt[e] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int m = n + (n & 1);
    const int npair = m / 2;
    for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < n * n; e += 1024) {
            const int i = e / n, j = e - i * n;
            if (i > j) continue;
            const double a = P[tri_idx(i, j, n)];
            tot += (i == j) ? a * a : 2.0 * a * a;
            if (i != j) off += 2.0 * a * a;
        }
        off = block_sum_1024(off, red16);
        tot = block_sum_1024(tot, red16);
        if (off <= 1e-30 * tot || tot == 0.0) break;
        for (int round = 0; round < m - 1; ++round) {
            if (tid < npair) {
                const int k = tid;
                int p = (round + k) % (m - 1);
                int q = (k == 0) ? (m - 1) : (round - k + m - 1) % (m - 1);
                if (p > q) { int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = P[tri_idx(p, q, n)];
                    if (apq != 0.0) {
                        const double app = P[tri_idx(p, p, n)], aqq = P[tri_idx(q, q, n)];
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                }
                pp[k] = p; qq[k] = q; cs[k] = c; sn[k] = s;
            }
            __syncthreads();
            // 2x2 blocks of pair-of-pairs, k1 <= k2
            for (int b = tid; b < npair * npair; b += 1024) {
                const int k1 = b / npair, k2 = b - k1 * npair;
                if (k1 > k2) continue;
                const double s1 = sn[k1], s2 = sn[k2];
                if (s1 == 0.0 && s2 == 0.0) continue;
                const int p1 = pp[k1], q1 = qq[k1], p2 = pp[k2], q2 = qq[k2];
                const double c1 = cs[k1], c2 = cs[k2];
                if (k1 == k2) {
                    if (q1 >= n) continue;
                    const double apq = P[tri_idx(p1, q1, n)];
                    const double t = s1 / c1;
                    P[tri_idx(p1, p1, n)] -= t * apq;
                    P[tri_idx(q1, q1, n)] += t * apq;
                    P[tri_idx(p1, q1, n)] = 0.0;
                    continue;
                }
                // rows {p1, q1} (q1 may be the dummy index n), columns {p2, q2}
                const bool r2 = q1 < n, c2ok = q2 < n;
                auto at = [&](int i, int j) -> double& {
                    return i <= j ? P[tri_idx(i, j, n)] : P[tri_idx(j, i, n)];
                };
                double b00 = at(p1, p2), b01 = c2ok ? at(p1, q2) : 0.0;
                double b10 = r2 ? at(q1, p2) : 0.0, b11 = (r2 && c2ok) ? at(q1, q2) : 0.0;
                // rows: G(k1) = [[c, -s], [s, c]]
                double u00 = c1 * b00 - s1 * b10, u01 = c1 * b01 - s1 * b11;
                double u10 = s1 * b00 + c1 * b10, u11 = s1 * b01 + c1 * b11;
                // columns
                double v00 = c2 * u00 - s2 * u01, v01 = s2 * u00 + c2 * u01;
                double v10 = c2 * u10 - s2 * u11, v11 = s2 * u10 + c2 * u11;
                at(p1, p2) = v00;
                if (c2ok) at(p1, q2) = v01;
                if (r2) at(q1, p2) = v10;
                if (r2 && c2ok) at(q1, q2) = v11;
            }
            // eigenvector rows p, q of Vt
            for (int e = tid; e < npair * n; e += 1024) {
                const int k = e / n, j = e - k * n;
                const int p = pp[k], q = qq[k];
                if (q >= n || sn[k] == 0.0) continue;
                const double c = cs[k], s = sn[k];
                const double vp = Vt[p * n + j], vq = Vt[q * n + j];
                Vt[p * n + j] = c * vp - s * vq;
                Vt[q * n + j] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < n; i += 1024) {
        const double di = P[tri_idx(i, i, n)];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double dj = P[tri_idx(j, j, n)];
            rank += (dj > di) || (dj == di && j < i);
        }
        J.w[rank] = di;
        for (int r = 0; r < n; ++r) J.A[r * n + rank] = Vt[i * n + r];
    }
}

// ---------------------------------------------------------------- vectors
__device__ void block_partial(double v, double* red, double* out) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) *out = red[0];
}

inline int n_blocks(size_t n) {
    size_t b = (n + RED_THREADS - 1) / RED_THREADS;
    if (b > (size_t)kPartials / 2) b = kPartials / 2;
    if (b < 1) b = 1;
    return (int)b;
}

// Thread t of block b covers elements b*RED_THREADS + t + k*(nb*RED_THREADS).
__global__ __launch_bounds__(RED_THREADS) void k_dot_partial(const double* a, const double* b, size_t n,
                                                             double* part) {
    __shared__ double red[RED_THREADS];
    double s = 0.0;
    for (size_t e = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * RED_THREADS)
        s += a[e] * b[e];
    block_partial(s, red, part + blockIdx.x);
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce(const double* part, int nb, int stride, double* scal,
                                                        int slot0, int slot1) {
    __shared__ double red[RED_THREADS];
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < nb; i += RED_THREADS) {
        s0 += part[i];
        if (slot1 >= 0) s1 += part[stride + i];
    }
    block_partial(s0, red, scal + slot0);
    __syncthreads();
    if (slot1 >= 0) block_partial(s1, red, scal + slot1);
}

__global__ __launch_bounds__(RED_THREADS) void k_cg_init(double* r, double* z, double* p, const double* b,
                                                         const double* q, const double* d, size_t n, double* part,
                                                         int stride) {
    __shared__ double red[RED_THREADS];
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (size_t e = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * RED_THREADS) {
        const double rv = -b[e] - q[e];
        const double zv = rv / d[e];
        r[e] = rv;
        z[e] = zv;
        p[e] = zv;
        rz += rv * zv;
        rr += rv * rv;
        bb += b[e] * b[e];
    }
    block_partial(rz, red, part + blockIdx.x);
    __syncthreads();
    block_partial(rr, red, part + stride + blockIdx.x);
    __syncthreads();
    block_partial(bb, red, part + 2 * stride + blockIdx.x);
}

__global__ __launch_bounds__(RED_THREADS) void k_shift_dot(double* q, const double* p, double shift, size_t n,
                                                           double* part) {
    __shared__ double red[RED_THREADS];
    double s = 0.0;
    for (size_t e = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * RED_THREADS) {
        const double qv = q[e] - shift * p[e];
        q[e] = qv;
        s += p[e] * qv;
    }
    block_partial(s, red, part + blockIdx.x);
}

__global__ __launch_bounds__(RED_THREADS) void k_cg_update(double* x, double* r, double* z, const double* p,
                                                           const double* q, const double* d, size_t n,
                                                           const double* scal, int rz_cur, double* part,
                                                           int stride) {
    __shared__ double red[RED_THREADS];
    const double alpha = scal[rz_cur] / scal[S_PQ];
    double rz = 0.0, rr = 0.0;
    for (size_t e = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * RED_THREADS) {
        x[e] += alpha * p[e];
        const double rv = r[e] - alpha * q[e];
        const double zv = rv / d[e];
        r[e] = rv;
        z[e] = zv;
        rz += rv * zv;
        rr += rv * rv;
    }
    block_partial(rz, red, part + blockIdx.x);
    __syncthreads();
    block_partial(rr, red, part + stride + blockIdx.x);
}

__global__ __launch_bounds__(RED_THREADS) void k_cg_direction(double* p, const double* z, size_t n,
                                                              const double* scal, int rz_cur, int rz_new) {
    const double beta = scal[rz_new] / scal[rz_cur];
    for (size_t e = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * RED_THREADS)
        p[e] = z[e] + beta * p[e];
}

__global__ __launch_bounds__(RED_THREADS) void k_axpby(double* y, const double* x, double a, double b, size_t n) {
    for (size_t e = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * RED_THREADS)
        y[e] = a * x[e] + b * y[e];
}

__global__ __launch_bounds__(RED_THREADS) void k_dav_precond(double* t, const double* r, const double* d,
                                                             double theta, size_t n) {
    for (size_t e = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * RED_THREADS) {
        double den = theta - d[e];
        if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
        t[e] = r[e] / den;
    }
}

}  // namespace

// ------------------------------------------------------------ host side
int device_count() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    return n;
}

void set_device(int device, void* stream) {
    int n = device_count();
    if (device < 0 || device >= n) throw Error{MPSPT_E_NODEV, "no HIP device " + std::to_string(device)};
    check(hipSetDevice(device), "hipSetDevice");
    hipDeviceProp_t prop;
    check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
        throw Error{MPSPT_E_NODEV, std::string("device is ") + prop.gcnArchName + ", the library is built for gfx950"};
    g_stream = static_cast<hipStream_t>(stream);
    // dynamic LDS available to the eigensolver next to ~4 KB of static shared memory;
    // the packed upper triangle (n (n + 1) / 2 doubles) must fit
    int lds = 0;
    check(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device), "hipDeviceGetAttribute");
    const long budget = (long)lds - 4096;
    g_lds_budget = budget > 0 ? (size_t)budget : 0;
    int nmax = 0;
    while ((long)(nmax + 1) * (nmax + 2) / 2 * 8 <= budget && nmax < 255) ++nmax;
    if (budget > 65536 - 4096) {
        check(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eig_jacobi_packed<true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)budget),
              "hipFuncSetAttribute");
        check(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_eig_jacobi_packed<false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)budget),
              "hipFuncSetAttribute");
    }
    g_eig_lds_max = nmax;
}

// Stream-ordered caching allocator.  All device work of the library is issued
// on one stream, so a block released here can be handed to the next request
// at once: any later use is ordered after every earlier use on that stream.
// Sizes are rounded to 1/8 steps between powers of two; nothing is returned
// to the runtime before trim().
namespace {
std::unordered_map<size_t, std::vector<void*>> g_free;
std::unordered_map<void*, size_t> g_size;

size_t size_class(size_t b) {
    if (b <= 256) return 256;
    size_t p = 1;
    while (p < b) p <<= 1;
    const size_t step = std::max<size_t>(p / 16, 256);
    return (b + step - 1) / step * step;
}
}  // namespace

void* alloc(size_t bytes) {
    if (bytes == 0) return nullptr;
    const size_t c = size_class(bytes);
    auto it = g_free.find(c);
    if (it != g_free.end() && !it->second.empty()) {
        void* p = it->second.back();
        it->second.pop_back();
        return p;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, c);
    if (e == hipErrorOutOfMemory) {  // give cached blocks back and retry once
        (void)hipGetLastError();
        trim();
        e = hipMalloc(&p, c);
    }
    check(e, "hipMalloc");
    g_size[p] = c;
    return p;
}
void release(void* p) {
    if (!p) return;
    auto it = g_size.find(p);
    if (it == g_size.end()) return;
    g_free[it->second].push_back(p);
}
void trim() {
    (void)hipStreamSynchronize(g_stream);
    for (auto& kv : g_free)
        for (void* p : kv.second) {
            (void)hipFree(p);
            g_size.erase(p);
        }
    g_free.clear();
}
void h2d(void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    // ordered on the stream; pageable sources are staged by the runtime before it returns
    check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, g_stream), "hipMemcpyAsync H2D");
}
void d2h(void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, g_stream), "hipMemcpyAsync D2H");
    check(hipStreamSynchronize(g_stream), "hipStreamSynchronize");
}
void d2d(void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, g_stream), "hipMemcpyAsync D2D");
}
void zero(void* p, size_t bytes) {
    if (!bytes) return;
    check(hipMemsetAsync(p, 0, bytes, g_stream), "hipMemsetAsync");
}
void sync() { check(hipStreamSynchronize(g_stream), "hipStreamSynchronize"); }
double now() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------ profiling
namespace {
struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double flops, bytes;
};
bool g_prof = false;
std::vector<ProfRec> g_pending;
std::vector<hipEvent_t> g_event_pool;
KernelStats g_stats[K_COUNT];

hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    check(hipEventCreate(&e), "hipEventCreate");
    return e;
}

void prof_flush() {
    if (g_pending.empty()) return;
    check(hipEventSynchronize(g_pending.back().b), "hipEventSynchronize");
    for (auto& r : g_pending) {
        float ms = 0;
        check(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
        KernelStats& s = g_stats[r.kind];
        s.seconds += ms * 1e-3;
        s.flops += r.flops;
        s.bytes += r.bytes;
        s.launches++;
        g_event_pool.push_back(r.a);
        g_event_pool.push_back(r.b);
    }
    g_pending.clear();
}

// Records events around one launch when profiling is on.
struct Prof {
    ProfRec r;
    bool on;
    Prof(int kind, double flops, double bytes) : on(g_prof) {
        if (!on) return;
        r = {kind, take_event(), take_event(), flops, bytes};
        check(hipEventRecord(r.a, g_stream), "hipEventRecord");
    }
    ~Prof() noexcept(false) {
        if (!on) return;
        check(hipEventRecord(r.b, g_stream), "hipEventRecord");
        g_pending.push_back(r);
        if (g_pending.size() >= 4096) prof_flush();
    }
};
}  // namespace

void profile_enable(bool on) {
    if (g_prof) prof_flush();
    g_prof = on;
    for (auto& s : g_stats) s = KernelStats();
}

KernelStats profile_stats(int kind) {
    prof_flush();
    if (kind < 0 || kind >= K_COUNT) return KernelStats();
    return g_stats[kind];
}

void gemm_grouped(const GemmGroup* groups, int ngroups, const GemmTerm* terms, int ntiles, double flops,
                  double bytes) {
    if (ntiles <= 0) return;
    Prof p(K_GEMM, flops, bytes);
    hipLaunchKernelGGL(k_gemm_grouped, dim3(ntiles), dim3(256), 0, g_stream, groups, ngroups, terms);
    check(hipGetLastError(), "k_gemm_grouped");
}
void axpy_grouped(const AxpyGroup* groups, int ngroups, const AxpyTerm* terms, double flops, double bytes) {
    if (ngroups <= 0) return;
    Prof p(K_AXPY, flops, bytes);
    hipLaunchKernelGGL(k_axpy_grouped, dim3(ngroups), dim3(256), 0, g_stream, groups, terms);
    check(hipGetLastError(), "k_axpy_grouped");
}
void diag_grouped(const DiagGroup* groups, int ngroups, const DiagTerm* terms) {
    if (ngroups <= 0) return;
    Prof p(K_DIAG, 0, 0);
    hipLaunchKernelGGL(k_diag_grouped, dim3(ngroups), dim3(256), 0, g_stream, groups, terms);
    check(hipGetLastError(), "k_diag_grouped");
}
void eig_batched(const EigJob* jobs, int njobs, int nmax) {
    if (njobs <= 0) return;
    Prof p(K_EIG, 0, 0);
    const size_t packed = (size_t)nmax * (nmax + 1) / 2 * sizeof(double);
    const size_t vt = (size_t)nmax * nmax * sizeof(double);
    if (packed + vt <= g_lds_budget) {
        hipLaunchKernelGGL(k_eig_jacobi_packed<true>, dim3(njobs), dim3(1024), packed + vt, g_stream, jobs);
        check(hipGetLastError(), "k_eig_jacobi_packed");
    } else if (packed <= g_lds_budget) {
        hipLaunchKernelGGL(k_eig_jacobi_packed<false>, dim3(njobs), dim3(1024), packed, g_stream, jobs);
        check(hipGetLastError(), "k_eig_jacobi_packed");
    } else {
        hipLaunchKernelGGL(k_eig_jacobi, dim3(njobs), dim3(256), 0, g_stream, jobs);
        check(hipGetLastError(), "k_eig_jacobi");
    }
}
int eig_class(int n) {
    const size_t packed = (size_t)n * (n + 1) / 2 * sizeof(double);
    const size_t vt = (size_t)n * n * sizeof(double);
    if (packed + vt <= g_lds_budget) return 0;
    if (packed <= g_lds_budget) return 1;
    return 2;
}

void dot(const double* a, const double* b, size_t n, double* scal, int slot, double* partials) {
    const int nb = n_blocks(n);
    hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(RED_THREADS), 0, g_stream, a, b, n, partials);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_THREADS), 0, g_stream, partials, nb, 0, scal, slot, -1);
    check(hipGetLastError(), "dot");
}
void cg_init(double* r, double* z, double* p, const double* b, const double* q, const double* d, size_t n,
             double* scal, double* partials) {
    const int nb = std::min(n_blocks(n), kPartials / 3);
    const int stride = kPartials / 3;
    hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(RED_THREADS), 0, g_stream, r, z, p, b, q, d, n, partials, stride);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_THREADS), 0, g_stream, partials, nb, stride, scal, (int)S_RZ0,
                       (int)S_RR);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_THREADS), 0, g_stream, partials + 2 * stride, nb, 0, scal,
                       (int)S_BB, -1);
    check(hipGetLastError(), "cg_init");
}
void cg_shift_dot(double* q, const double* p, double shift, size_t n, double* scal, double* partials) {
    const int nb = n_blocks(n);
    hipLaunchKernelGGL(k_shift_dot, dim3(nb), dim3(RED_THREADS), 0, g_stream, q, p, shift, n, partials);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_THREADS), 0, g_stream, partials, nb, 0, scal, (int)S_PQ, -1);
    check(hipGetLastError(), "cg_shift_dot");
}
void cg_update(double* x, double* r, double* z, const double* p, const double* q, const double* d, size_t n,
               double* scal, int rz_cur, int rz_new, double* partials) {
    const int nb = n_blocks(n);
    const int stride = kPartials / 2;
    hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(RED_THREADS), 0, g_stream, x, r, z, p, q, d, n, scal, rz_cur,
                       partials, stride);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(RED_THREADS), 0, g_stream, partials, nb, stride, scal, rz_new,
                       (int)S_RR);
    check(hipGetLastError(), "cg_update");
}
void cg_direction(double* p, const double* z, size_t n, const double* scal, int rz_cur, int rz_new) {
    const int nb = n_blocks(n);
    hipLaunchKernelGGL(k_cg_direction, dim3(nb), dim3(RED_THREADS), 0, g_stream, p, z, n, scal, rz_cur, rz_new);
    check(hipGetLastError(), "cg_direction");
}
void davidson_precond(double* t, const double* r, const double* d, double theta, size_t n) {
    if (!n) return;
    const int nb = n_blocks(n);
    hipLaunchKernelGGL(k_dav_precond, dim3(nb), dim3(RED_THREADS), 0, g_stream, t, r, d, theta, n);
    check(hipGetLastError(), "davidson_precond");
}
void axpby(double* y, const double* x, double a, double b, size_t n) {
    if (!n) return;
    const int nb = n_blocks(n);
    hipLaunchKernelGGL(k_axpby, dim3(nb), dim3(RED_THREADS), 0, g_stream, y, x, a, b, n);
    check(hipGetLastError(), "axpby");
}

}  // namespace dev
}  // namespace mpspt
