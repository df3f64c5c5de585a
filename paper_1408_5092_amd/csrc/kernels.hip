// gfx950 kernels of the MPS-PT engine and the host side of device.hpp.
//
// * k_gemm_grouped / k_gemm_grouped_split: output-stationary grouped GEMM on
//   MFMA over a work list of output blocks, each the sum of its terms in list
//   order, so a block-sparse contraction is one launch and its result is
//   deterministic (FP64; FP32 and BF16x3 instances for the reduced-precision
//   sigma).
// * k_axpy_grouped: linear combinations of dense blocks (MPO coefficients).
// * k_diag_grouped: Jacobi diagonal of the effective operator.
// * k_eig_tridiag: batched symmetric eigensolver (Householder tridiagonal
//   reduction, accumulated Q, implicit QL), one workgroup per matrix.
// * CG vector kernels with fixed-order two-pass reductions.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mpspt.h"
#include "device.hpp"

namespace mpspt {
namespace dev {

// shared with precond.hip
void check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        int code = (e == hipErrorOutOfMemory) ? MPSPT_E_NOMEM : MPSPT_E_HIP;
        throw Error{code, std::string(what) + ": " + hipGetErrorString(e)};
    }
}

namespace {
size_t g_lds_budget = 0;  // dynamic LDS granted to the eigensolver kernels (same on every gfx950)

constexpr int RED_THREADS = 256;

typedef double d4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------- GEMM
// Output-stationary grouped GEMM on MFMA.  A group is one output block; its
// 16 x 16 tiles are numbered consecutively and tile_group maps a tile to its
// group.  A tile sums every term of its group in list order, each term's k
// range cut into chunks of 16.  Two launch shapes over the same lists:
//   k_gemm_grouped:       one wave per tile (four tiles per workgroup), for
//                         lists whose tiles have short k chains;
//   k_gemm_grouped_split: one workgroup of W = 4, 8 or 16 waves per tile,
//                         the chunks dealt round-robin to the waves (chunk
//                         c to wave c % W) and the partial tiles added in
//                         wave order through LDS, for lists with long k
//                         chains.
// No LDS staging of operands: each lane loads its MFMA operands straight from
// global memory, two chunks in flight; rows, columns and k beyond the block
// read the block's last row, column or k index (so every load is issued
// without a branch) and are zeroed before the MFMA.  Results are
// deterministic for either shape.
// Element types: MODE 0 FP64 (v_mfma_f64_16x16x4f64), 1 FP32
// (v_mfma_f32_16x16x4f32), 2 BF16x3 on FP32 data (three
// v_mfma_f32_16x16x16bf16_1k products of head/tail-split operands).
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

template <int MODE>
struct GemmTypes {
    typedef float R;
    typedef f4 V;
    typedef BasesF B;
};
template <>
struct GemmTypes<0> {
    typedef double R;
    typedef d4 V;
    typedef Bases B;
};

// BF16 bits of x rounded to nearest even (finite x), and the BF16 bits of
// the remainder x - head.
__device__ inline void bf16_split(float x, short& head, short& tail) {
    uint32_t u = __float_as_uint(x);
    const uint32_t h = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    head = (short)(h >> 16);
    const float rest = x - __uint_as_float(h);
    uint32_t v = __float_as_uint(rest);
    v = v + 0x7FFFu + ((v >> 16) & 1u);
    tail = (short)(v >> 16);
}

// One wave's share of one tile: chunks c0, c0 + cs, c0 + 2 cs, ... of the
// group's chunk sequence.
template <int MODE>
__device__ inline typename GemmTypes<MODE>::V gemm_tile(const typename GemmTypes<MODE>::B& bs, const GemmGroup& g,
                                                        const GemmTerm* __restrict__ T, int row0, int col0,
                                                        int lane, int c0, int cs) {
    typedef typename GemmTypes<MODE>::R R;
    typedef typename GemmTypes<MODE>::V V;
    const int li = lane & 15, lk = lane >> 4;
    const int ar = row0 + li, bc = col0 + li;
    const bool aok = ar < g.m, bok = bc < g.n;
    // rows and columns past the block load its last row / column (in bounds)
    // and are zeroed at use, so the loads need no branches
    const int arc = aok ? ar : g.m - 1, bcc = bok ? bc : g.n - 1;
    V acc = {R(0), R(0), R(0), R(0)};
    int chunk0 = 0;  // chunks of the earlier terms
    for (int ti = 0; ti < g.nterms; ++ti) {
        const GemmTerm tm = T[g.term0 + ti];
        // element (row, kk) of op(A) at pa[kk * sa]; element (kk, col) of op(B) at pb[kk * sb]
        const R* A = bs.p[tm.sa] + tm.oa;
        const R* B = bs.p[tm.sb] + tm.ob;
        const R* pa = tm.transA ? A + arc : A + (size_t)arc * tm.lda;
        const size_t sa = tm.transA ? (size_t)tm.lda : 1;
        const R* pb = tm.transB ? B + (size_t)bcc * tm.ldb : B + bcc;
        const size_t sb = tm.transB ? 1 : (size_t)tm.ldb;
        const R alpha = (R)tm.alpha;
        const int k = tm.k;
        const int nch = (k + 15) >> 4;
        // first chunk of this term that is ours
        int c = cs == 1 ? 0 : (c0 - chunk0 % cs + cs) % cs;
        for (; c < nch; c += 2 * cs) {
            R a[8], b[8];
            // MODE 0/1: lane holds op(A)[row li][16 c + lk + 4 u], op(B)[16 c + lk + 4 u][col li]
            // MODE 2:   lane holds op(A)[row li][16 c + 4 lk + u], op(B)[16 c + 4 lk + u][col li]
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int kk = (c + h * cs) * 16 + (MODE == 2 ? 4 * lk + u : 4 * u + lk);
                    const bool in = kk < k;
                    const size_t kc = (size_t)(in ? kk : k - 1);
                    const R av = pa[kc * sa], bv = pb[kc * sb];
                    a[4 * h + u] = (aok && in) ? av : R(0);
                    b[4 * h + u] = (bok && in) ? alpha * bv : R(0);
                }
            if constexpr (MODE == 0) {
#pragma unroll
                for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
            } else if constexpr (MODE == 1) {
#pragma unroll
                for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], acc, 0, 0, 0);
            } else {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    s4 ah, at, bh, bt;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        short hh, tl;
                        bf16_split(a[4 * h + u], hh, tl);
                        ah[u] = hh;
                        at[u] = tl;
                        bf16_split(b[4 * h + u], hh, tl);
                        bh[u] = hh;
                        bt[u] = tl;
                    }
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(at, bh, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bt, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
                }
            }
        }
        chunk0 += nch;
    }
    return acc;
}

template <int MODE>
__device__ inline void gemm_store(const typename GemmTypes<MODE>::B& bs, const GemmGroup& g, int row0, int col0,
                                  int lane, const typename GemmTypes<MODE>::V& acc) {
    typedef typename GemmTypes<MODE>::R R;
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        // accumulator register e of a lane holds D[lane/16 + 4 e][lane%16] (f64 MFMA)
        // or D[4 (lane/16) + e][lane%16] (f32 and bf16 MFMA)
        const int gi = row0 + (MODE == 0 ? lk + 4 * e : 4 * lk + e), gj = col0 + li;
        if (gi < g.m && gj < g.n) {
            R* cp = bs.p[g.sc] + g.oc + (size_t)gi * g.ldc + gj;
            *cp = g.accumulate ? *cp + acc[e] : acc[e];
        }
    }
}

template <int MODE>
__device__ inline void gemm_wave_per_tile(const typename GemmTypes<MODE>::B& bs, const GemmGroup* __restrict__ G,
                                          const int* __restrict__ TG, const GemmTerm* __restrict__ T, int ntiles) {
    // the wave index is uniform across the wave: with it in a scalar register
    // the tile's group and term records come through scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + wave;
    if (tile >= ntiles) return;
    const GemmGroup g = G[TG[tile]];
    const int tiles_n = (g.n + GEMM_TILE - 1) / GEMM_TILE;
    const int t = tile - g.tile0;
    const int row0 = (t / tiles_n) * GEMM_TILE, col0 = (t % tiles_n) * GEMM_TILE;
    const auto acc = gemm_tile<MODE>(bs, g, T, row0, col0, lane, 0, 1);
    gemm_store<MODE>(bs, g, row0, col0, lane, acc);
}

template <int MODE, int W>
__device__ inline void gemm_split_tile(const typename GemmTypes<MODE>::B& bs, const GemmGroup* __restrict__ G,
                                       const int* __restrict__ TG, const GemmTerm* __restrict__ T,
                                       typename GemmTypes<MODE>::V (*part)[64]) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = blockIdx.x;
    const GemmGroup g = G[TG[tile]];
    const int tiles_n = (g.n + GEMM_TILE - 1) / GEMM_TILE;
    const int t = tile - g.tile0;
    const int row0 = (t / tiles_n) * GEMM_TILE, col0 = (t % tiles_n) * GEMM_TILE;
    auto acc = gemm_tile<MODE>(bs, g, T, row0, col0, lane, wave, W);
    if (wave > 0) part[wave - 1][lane] = acc;
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < W - 1; ++w) acc += part[w][lane];
    gemm_store<MODE>(bs, g, row0, col0, lane, acc);
}

__global__ __launch_bounds__(256) void k_gemm_grouped(Bases bs, const GemmGroup* __restrict__ G,
                                                      const int* __restrict__ TG, const GemmTerm* __restrict__ T,
                                                      int ntiles) {
    gemm_wave_per_tile<0>(bs, G, TG, T, ntiles);
}

template <int W>
__global__ __launch_bounds__(64 * W) void k_gemm_grouped_split(Bases bs, const GemmGroup* __restrict__ G,
                                                              const int* __restrict__ TG,
                                                              const GemmTerm* __restrict__ T) {
    __shared__ d4 part[W - 1][64];
    gemm_split_tile<0, W>(bs, G, TG, T, part);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_gemm_grouped_lo(BasesF bs, const GemmGroup* __restrict__ G,
                                                         const int* __restrict__ TG, const GemmTerm* __restrict__ T,
                                                         int ntiles) {
    gemm_wave_per_tile<MODE>(bs, G, TG, T, ntiles);
}

template <int MODE, int W>
__global__ __launch_bounds__(64 * W) void k_gemm_grouped_lo_split(BasesF bs, const GemmGroup* __restrict__ G,
                                                                 const int* __restrict__ TG,
                                                                 const GemmTerm* __restrict__ T) {
    __shared__ f4 part[W - 1][64];
    gemm_split_tile<MODE, W>(bs, G, TG, T, part);
}

// ------------------------------------------------------------------- AXPY
// One workgroup per output block.  The block's terms are staged in LDS, up
// to 256 at a time, as resolved source pointers (one coalesced read of the
// term records per chunk instead of a dependent scalar load of each record
// and its slot base per term).  A block with fewer elements than threads
// deals its terms round-robin to S = min(256 / elements, terms / 4) thread
// sets (term t to set t % S); each thread sums its terms in list order with
// eight loads in flight (a block with more elements keeps its running sums
// in the output between chunks), and the S partial sums of an element are
// added in set order through LDS, so the result is deterministic.
template <typename R>
struct AxpyTermL {
    const R* src;
    R alpha;
    int lds, trans;
};

template <typename R, typename BS>
__device__ inline void axpy_block(const BS& bs, const AxpyGroup& g, const AxpyTerm* __restrict__ T, R* red,
                                  AxpyTermL<R>* st) {
    R* dst = bs.p[g.sd] + g.od;
    const int total = g.m * g.n;
    if (total <= 0) return;
    const int S = total >= 256 ? 1 : max(1, min(256 / total, g.nterms / 4));
    auto stage = [&](int c0) {  // terms c0 .. c0 + 255 of the group into st
        const int cnt = min(256, g.nterms - c0);
        __syncthreads();        // the previous chunk's readers are done
        if ((int)threadIdx.x < cnt) {
            const AxpyTerm tm = T[g.term0 + c0 + threadIdx.x];
            st[threadIdx.x] = AxpyTermL<R>{bs.p[tm.ss] + tm.os, (R)tm.alpha, tm.lds, (int)tm.trans};
        }
        __syncthreads();
        return cnt;
    };
    auto val = [](const AxpyTermL<R>& tm, int i, int j) {
        return tm.alpha * (tm.trans ? tm.src[(size_t)j * tm.lds + i] : tm.src[(size_t)i * tm.lds + j]);
    };
    if (S == 1) {
        for (int c0 = 0; c0 == 0 || c0 < g.nterms; c0 += 256) {
            const int cnt = stage(c0);
            // element e = i n + j, advanced by the block size without dividing
            const int di = blockDim.x / g.n, dj = blockDim.x - di * g.n;
            int i = threadIdx.x / g.n, j = threadIdx.x - i * g.n;
            for (int e = threadIdx.x; e < total; e += blockDim.x) {
                R* d = dst + (size_t)i * g.ldd + j;
                R s = (c0 > 0 || g.accumulate) ? *d : R(0);
                int t = 0;
                for (; t + 8 <= cnt; t += 8) {
                    R v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = val(st[t + u], i, j);
#pragma unroll
                    for (int u = 0; u < 8; ++u) s += v[u];
                }
                for (; t < cnt; ++t) s += val(st[t], i, j);
                *d = s;
                i += di;
                j += dj;
                if (j >= g.n) {
                    j -= g.n;
                    ++i;
                }
            }
        }
        return;
    }
    const int e = threadIdx.x % total, set = threadIdx.x / total;
    const int i = e / g.n, j = e - i * g.n;
    R s = R(0);
    for (int c0 = 0; c0 < g.nterms; c0 += 256) {
        const int cnt = stage(c0);
        if (set < S) {
            // this set's terms in the chunk: global index c0 + t with (c0 + t) % S == set
            int t = (set - c0 % S + S) % S;
            for (; t + 7 * S < cnt; t += 8 * S) {
                R v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = val(st[t + u * S], i, j);
#pragma unroll
                for (int u = 0; u < 8; ++u) s += v[u];
            }
            for (; t < cnt; t += S) s += val(st[t], i, j);
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x < total) {
        R acc = g.accumulate ? dst[(size_t)i * g.ldd + j] : R(0);
        for (int q = 0; q < S; ++q) acc += red[q * total + e];
        dst[(size_t)i * g.ldd + j] = acc;
    }
}

__global__ __launch_bounds__(256) void k_axpy_grouped(Bases bs, const AxpyGroup* __restrict__ G,
                                                      const AxpyTerm* __restrict__ T) {
    __shared__ double red[256];
    __shared__ AxpyTermL<double> st[256];
    axpy_block<double>(bs, G[blockIdx.x], T, red, st);
}

// ------------------------------------------------- reduced-precision sigma
// The same work lists, run on FP32 copies of the operands (slot bases point
// at float arrays with the same element offsets); the GEMMs are the MODE 1/2
// instances above.
__global__ __launch_bounds__(256) void k_axpy_grouped_lo(BasesF bs, const AxpyGroup* __restrict__ G,
                                                         const AxpyTerm* __restrict__ T) {
    __shared__ float red[256];
    __shared__ AxpyTermL<float> st[256];
    axpy_block<float>(bs, G[blockIdx.x], T, red, st);
}

__global__ __launch_bounds__(256) void k_to_f32(float* __restrict__ dst, const double* __restrict__ src, size_t n) {
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) dst[e] = (float)src[e];
}

// ------------------------------------------------------------------- DIAG
__global__ __launch_bounds__(256) void k_diag_grouped(Bases bs, const DiagGroup* __restrict__ G,
                                                      const DiagTerm* __restrict__ T) {
    const DiagGroup g = G[blockIdx.x];
    double* dst = bs.p[g.sd] + g.od;
    const int total = g.m * g.n, di = blockDim.x / g.n, dj = blockDim.x - di * g.n;
    int i = threadIdx.x / g.n, j = threadIdx.x - i * g.n;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        double s = g.shift;
        for (int t = 0; t < g.nterms; ++t) {
            const DiagTerm tm = T[g.term0 + t];
            s += tm.c * bs.p[tm.sl][tm.ol + (size_t)i * tm.ls] * bs.p[tm.sr][tm.orr + (size_t)j * tm.rs];
        }
        dst[(size_t)i * g.ldd + j] = s;
        i += di;
        j += dj;
        if (j >= g.n) {
            j -= g.n;
            ++i;
        }
    }
}

// ------------------------------------------------------------------ EIGEN
// Symmetric eigensolver for density matrices, in two launches with the
// choice of the kept count on the host between them.  One 1024-thread
// workgroup per matrix.
//
// k_eig_reduce: Householder reduction to tridiagonal form (lower variant),
//   then every eigenvalue by multisection on Sturm counts: the eigenvalue of
//   ascending index j is owned by a group of L lanes (L = 1024 / n rounded
//   down to a power of two, at most 64) that evaluate L interior points of
//   its bracket at once, so each step shrinks the bracket (L + 1)-fold.
// k_eig_vectors: for the k largest eigenvalues, an orthonormal basis of
//   their invariant subspace: inverse iteration on the tridiagonal matrix
//   (one thread per vector, random start, three solves with partial
//   pivoting), sequential orthogonalisation inside clusters closer than
//   1000 ulps of the norm, two passes of Cholesky QR over all k vectors,
//   then the Householder reflectors applied backwards.
//
// Job buffers: A (n x n, row major) holds the symmetric input and, after
// k_eig_vectors, the basis in its first k columns; V (n x n) receives the
// reflectors (row r: tau at V[r][r], v at V[r][r+2..], v[r+1] = 1); w (n)
// the eigenvalues in descending order; t (eig_work(n) doubles) the
// tridiagonal matrix and scratch.
constexpr int EIG_MAXN = 512;
constexpr double EIG_EPS = 2.220446049250313e-16;

// Cross-lane moves through DPP (no LDS round trip), on both halves of a
// double; lanes that the control does not write (rows outside ROWS) get 0.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_f64(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over each aligned group of 8 lanes (all 8 active), the same bits in
// all of them: every step adds a lane's value to its partner's in either
// order, and a + b == b + a.  DPP controls: quad_perm [1,0,3,2] and
// [2,3,0,1], then row_half_mirror.
__device__ __forceinline__ double group8_sum(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    return v;
}

// Sum over a full wave, the same bits in every lane: 8-lane sums, row_mirror
// for the 16-lane rows, row_bcast:15 and row_bcast:31 to gather the rows in
// lane 63, which every lane then reads.
__device__ __forceinline__ double wave_sum(double v) {
    v = group8_sum(v);
    v += dpp_f64<0x140>(v);
    v += dpp_f64<0x142, 0xA>(v);
    v += dpp_f64<0x143, 0xC>(v);
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <bool LDSRES>
__global__ __launch_bounds__(1024) void k_eig_reduce(const EigJob* __restrict__ jobs) {
    extern __shared__ __align__(16) double dyn[];
    __shared__ double sv[EIG_MAXN], sp[EIG_MAXN], sd[EIG_MAXN], se[EIG_MAXN], stau[EIG_MAXN];
    __shared__ double s_lo, s_hi, s_tol, s_piv;
    const EigJob J = jobs[blockIdx.x];
    const int n = J.n;
    const int tid = threadIdx.x, lane = tid & 63;
    double* M = LDSRES ? dyn : J.A;
    const int ld = LDSRES ? n + 1 : n;
    double* V = J.V;
    if (LDSRES) {
        for (int e = tid; e < n * n; e += 1024) {
            const int i = e / n, j = e - i * n;
            M[i * ld + j] = J.A[e];
        }
    }
    __syncthreads();
    // ---- Householder: wave 0 forms the reflector (v in the column it
    // annihilates, which no later step reads; copied to V after the loop),
    // all threads form p = tau A22 v, then every wave computes K = tau p.v / 2
    // itself and applies A22 -= v w^T + w v^T with w = p - K v.
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        if (tid < 64) {
            double part = 0.0;
            for (int i = k + 2 + lane; i < n; i += 64) part += M[i * ld + k] * M[i * ld + k];
            part = wave_sum(part);
            const double alpha = M[(k + 1) * ld + k];
            double tau = 0.0, beta = alpha, scal = 0.0;
            if (part > 0.0) {
                beta = -copysign(sqrt(alpha * alpha + part), alpha);
                tau = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            for (int i = k + 1 + lane; i < n; i += 64) {
                const double vi = (i == k + 1) ? 1.0 : M[i * ld + k] * scal;
                sv[i] = vi;
                if (i >= k + 2) M[i * ld + k] = vi;
            }
            if (lane == 0) {
                sd[k] = M[k * ld + k];
                se[k] = beta;
                stau[k] = tau;
            }
        }
        __syncthreads();
        const double tau = stau[k];
        if (tau == 0.0) continue;
        for (int e = tid; e < m * 8; e += 1024) {
            const int i = k + 1 + (e >> 3), g = e & 7;
            double s = 0.0;
            for (int j = k + 1 + g; j < n; j += 8) s += M[i * ld + j] * sv[j];
            s = group8_sum(s);
            if (g == 0) sp[i] = tau * s;
        }
        __syncthreads();
        double part = 0.0;
        for (int i = k + 1 + lane; i < n; i += 64) part += sp[i] * sv[i];
        const double K = 0.5 * tau * wave_sum(part);
        for (int i = k + 1 + (tid >> 6); i < n; i += 16) {
            const double vi = sv[i], wi = sp[i] - K * vi;
            for (int j = k + 1 + lane; j < n; j += 64) {
                const double vj = sv[j];
                M[i * ld + j] -= vi * (sp[j] - K * vj) + wi * vj;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (n >= 2) {
            sd[n - 2] = M[(n - 2) * ld + (n - 2)];
            se[n - 2] = M[(n - 1) * ld + (n - 2)];
        }
        sd[n - 1] = M[(n - 1) * ld + (n - 1)];
        se[n - 1] = 0.0;
    }
    __syncthreads();
    for (int i = tid; i < n; i += 1024) {
        J.t[i] = sd[i];
        J.t[n + i] = se[i];
    }
    // the reflectors: row r of V holds tau_r at r and v_r below r + 1
    for (int e = tid; e < n * n; e += 1024) {
        const int r = e / n, i = e - r * n;
        if (r + 2 < n) {
            if (i >= r + 2)
                V[e] = M[i * ld + r];
            else if (i == r)
                V[e] = stau[r];
        }
    }
    // ---- Gershgorin bracket, pivot guard and tolerance (wave 0); sp <- e^2
    if (tid < 64) {
        double lo = 1e308, hi = -1e308, e2max = 0.0;
        for (int i = lane; i < n; i += 64) {
            const double ea = i > 0 ? fabs(se[i - 1]) : 0.0, eb = fabs(se[i]);
            lo = fmin(lo, sd[i] - ea - eb);
            hi = fmax(hi, sd[i] + ea + eb);
            e2max = fmax(e2max, se[i] * se[i]);
        }
        for (int off = 32; off > 0; off >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, off, 64));
            hi = fmax(hi, __shfl_xor(hi, off, 64));
            e2max = fmax(e2max, __shfl_xor(e2max, off, 64));
        }
        if (lane == 0) {
            const double tn = fmax(fabs(lo), fabs(hi));
            const double piv = 2.2250738585072014e-308 * fmax(1.0, e2max);
            const double fudge = 2.1 * tn * EIG_EPS * n + 4.2 * piv;
            s_lo = lo - fudge;
            s_hi = hi + fudge;
            s_tol = EIG_EPS * tn;
            s_piv = piv;
        }
    }
    for (int i = tid; i < n; i += 1024) sp[i] = se[i] * se[i];
    __syncthreads();
    // ---- multisection
    int L = 64;
    while (L > 1 && L * n > 1024) L >>= 1;
    const int u = tid % L, j = tid / L;
    const double piv = s_piv, tol = s_tol;
    double lo = s_lo, hi = s_hi;
    bool done = j >= n;
    for (int it = 0; it < 400; ++it) {
        if (!done && hi - lo <= fmax(tol, 2.0 * EIG_EPS * fmax(fabs(lo), fabs(hi)))) done = true;
        if (__ballot(!done) == 0) break;
        const double step = (hi - lo) / (L + 1);
        int cnt = 0;
        if (!done) {
            const double x = lo + (u + 1) * step;
            double q = sd[0] - x;
            if (fabs(q) <= piv) q = -piv;
            cnt = q < 0.0;
            // hardware reciprocal refined by one Newton step: each count
            // stays the exact count of a matrix within a few ulps of T; the
            // LDS reads of eight steps are issued ahead of their chain
            auto sturm = [&](double dv, double ev) {
                double r = __builtin_amdgcn_rcp(q);
                r = fma(r, fma(-q, r, 1.0), r);
                q = dv - x - ev * r;
                if (fabs(q) <= piv) q = -piv;
                cnt += q < 0.0;
            };
            int i = 1;
            for (; i + 8 <= n; i += 8) {
                double dv[8], ev[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    dv[t] = sd[i + t];
                    ev[t] = sp[i + t - 1];
                }
#pragma unroll
                for (int t = 0; t < 8; ++t) sturm(dv[t], ev[t]);
            }
            for (; i < n; ++i) sturm(sd[i], sp[i - 1]);
        }
        const unsigned long long bal = __ballot(!done && cnt > j);
        const int base = lane - u;
        const unsigned long long mask = L == 64 ? ~0ull : ((1ull << L) - 1);
        const unsigned long long gb = (bal >> base) & mask;
        const int us = gb ? __ffsll((long long)gb) - 1 : L;  // first point whose count exceeds j
        if (!done) {
            const double nlo = us == 0 ? lo : lo + us * step;
            const double nhi = us == L ? hi : lo + (us + 1) * step;
            lo = nlo;
            hi = nhi;
        }
    }
    if (j < n && u == 0) J.w[n - 1 - j] = 0.5 * (lo + hi);
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// 1 / b (b finite and nonzero) to about an ulp: the hardware reciprocal and
// two Newton steps, a shorter dependent chain than a correctly rounded
// division.
__device__ __forceinline__ double recip(double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(r, fma(-b, r, 1.0), r);
    r = fma(r, fma(-b, r, 1.0), r);
    return r;
}

// Solves (T - sigma I) y = y in place by Gaussian elimination with partial
// pivoting (pivots below `guard` in magnitude are raised to it); U's rows go to
// the thread's scratch columns.  Y(i) addresses the vector.
template <class YA>
__device__ void tri_solve(const double* sd, const double* se, int n, double sigma, double guard, YA Y,
                          double* U, int ustride) {
    double bi = sd[0] - sigma, ci = n > 1 ? se[0] : 0.0, yi = Y(0);
    for (int i = 0; i + 1 < n; ++i) {
        const double a1 = se[i], b1 = sd[i + 1] - sigma, c1 = i + 2 < n ? se[i + 1] : 0.0, y1 = Y(i + 1);
        double* Ui = U + (size_t)3 * i * ustride;
        if (fabs(bi) >= fabs(a1)) {
            if (fabs(bi) < guard) bi = bi < 0.0 ? -guard : guard;
            const double f = a1 * recip(bi);
            Ui[0] = bi;
            Ui[ustride] = ci;
            Ui[2 * ustride] = 0.0;
            Y(i) = yi;
            bi = b1 - f * ci;
            ci = c1;
            yi = y1 - f * yi;
        } else {
            const double f = bi * recip(a1);
            Ui[0] = a1;
            Ui[ustride] = b1;
            Ui[2 * ustride] = c1;
            Y(i) = y1;
            const double nb = ci - f * b1, nc = -f * c1, ny = yi - f * y1;
            bi = nb;
            ci = nc;
            yi = ny;
        }
    }
    if (fabs(bi) < guard) bi = bi < 0.0 ? -guard : guard;
    double y2 = 0.0, y1 = yi * recip(bi);
    Y(n - 1) = y1;
    // back substitution, the rows of U and y for four steps loaded up front
    int i = n - 2;
    for (; i >= 3; i -= 4) {
        double u0[4], u1[4], u2[4], yv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double* Ui = U + (size_t)3 * (i - q) * ustride;
            u0[q] = Ui[0];
            u1[q] = Ui[ustride];
            u2[q] = Ui[2 * ustride];
            yv[q] = Y(i - q);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double y0 = (yv[q] - u1[q] * y1 - u2[q] * y2) * recip(u0[q]);
            Y(i - q) = y0;
            y2 = y1;
            y1 = y0;
        }
    }
    for (; i >= 0; --i) {
        const double* Ui = U + (size_t)3 * i * ustride;
        const double y0 = (Y(i) - Ui[ustride] * y1 - Ui[2 * ustride] * y2) * recip(Ui[0]);
        Y(i) = y0;
        y2 = y1;
        y1 = y0;
    }
}

// LDS use of k_eig_vectors (doubles): the basis Y (n x (k+1)) and Gram matrix
// G (k x (k+1)) when LDS-resident, then per block of rb reflectors: the
// vectors (rb x n), V^T Y and T V^T Y (rb x (k+1) each), T and V^T V
// (rb x rb each) and the block's tau.
__host__ __device__ inline size_t eigv_lds_words(int n, int k, int rb, bool resident) {
    size_t w = (size_t)rb * n + 2 * (size_t)rb * (k + 1) + 2 * (size_t)rb * rb + rb;
    if (resident) w += (size_t)n * (k + 1) + (size_t)k * (k + 1);
    return w;
}

template <bool LDSRES>
__global__ __launch_bounds__(1024) void k_eig_vectors(const EigJob* __restrict__ jobs, int* __restrict__ status,
                                                      int rb, int u_lds) {
    extern __shared__ __align__(16) double dyn[];
    __shared__ double sd[EIG_MAXN], se[EIG_MAXN], sw[EIG_MAXN];
    __shared__ int s_fail;
    const EigJob J = jobs[blockIdx.x];
    const int n = J.n, k = J.k;
    if (k <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63;
    // Y (n x k) row major: in LDS with rows padded to k + 1, or the first k
    // columns of A; G (k x k, upper triangle used) in LDS or in t
    const int ldy = LDSRES ? k + 1 : n, ldg = LDSRES ? k + 1 : k;
    // 3 n k: rows of U of the inverse-iteration solves, in the LDS the later
    // phases use (after Y) when it fits
    double* U = u_lds ? dyn + (LDSRES ? (size_t)n * (k + 1) : 0) : J.t + 2 * n;
    double* Yb = LDSRES ? dyn : J.A;
    double* G = LDSRES ? dyn + (size_t)n * (k + 1) : J.t + 2 * n + (size_t)3 * n * k;
    double* blk = LDSRES ? G + (size_t)k * (k + 1) : dyn;
    double* Vb = blk;                        // rb x n
    double* Zb = Vb + (size_t)rb * n;        // rb x (k + 1)
    double* Wb = Zb + (size_t)rb * (k + 1);  // rb x (k + 1)
    double* Tb = Wb + (size_t)rb * (k + 1);  // rb x rb
    double* Cb = Tb + (size_t)rb * rb;       // rb x rb
    double* tb = Cb + (size_t)rb * rb;       // rb
    for (int i = tid; i < n; i += 1024) {
        sd[i] = J.t[i];
        se[i] = J.t[n + i];
    }
    for (int i = tid; i < k; i += 1024) sw[i] = J.w[i];
    if (tid == 0) s_fail = 0;
    __syncthreads();
    const double tnorm = fmax(fabs(J.w[0]), fabs(J.w[n - 1]));
    const double guard = tnorm > 0.0 ? EIG_EPS * tnorm : 2.2250738585072014e-308;
    const double tight = 1000.0 * EIG_EPS * tnorm;
    // ---- inverse iteration; a cluster of eigenvalues closer than `tight`
    // is done in order by its first thread, each vector kept orthogonal to
    // the cluster's earlier ones
    if (tid < k) {
        int j0 = tid;
        if (j0 == 0 || sw[j0 - 1] - sw[j0] > tight) {
            int j1 = j0;
            while (j1 + 1 < k && sw[j1] - sw[j1 + 1] <= tight) ++j1;
            for (int c = j0; c <= j1; ++c) {
                auto Yc = [&](int i) -> double& { return Yb[(size_t)i * ldy + c]; };
                for (int i = 0; i < n; ++i) {
                    const unsigned long long h = mix64(((unsigned long long)c << 32) ^ (unsigned long long)i);
                    Yc(i) = (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
                }
                for (int pass = 0; pass < 4; ++pass) {
                    for (int c2 = j0; c2 < c; ++c2) {  // against the cluster's earlier vectors
                        double dotv = 0.0;
                        for (int i = 0; i < n; ++i) dotv += Yb[(size_t)i * ldy + c2] * Yc(i);
                        for (int i = 0; i < n; ++i) Yc(i) -= dotv * Yb[(size_t)i * ldy + c2];
                    }
                    if (pass < 3) tri_solve(sd, se, n, sw[c], guard, Yc, U + c, k);
                    double nrm = 0.0;
                    for (int i = 0; i < n; ++i) nrm += Yc(i) * Yc(i);
                    const double sc = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
                    for (int i = 0; i < n; ++i) Yc(i) *= sc;
                }
            }
        }
    }
    __syncthreads();
    // ---- Cholesky QR: G = Y^T Y = R^T R, Y <- Y R^-1; a second pass when
    // the first Gram matrix was off the identity by more than 1e-6
    const int T4 = (k + 3) / 4, ntile = T4 * (T4 + 1) / 2;
    __shared__ int s_again;
    if (tid == 0) s_again = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1 && !s_again) break;
        for (int t = tid; t < ntile; t += 1024) {
            int ta = 0, rem = t;
            while (rem >= T4 - ta) { rem -= T4 - ta; ++ta; }
            const int tbi = ta + rem, a0 = ta * 4, b0 = tbi * 4;
            double acc[4][4] = {};
            for (int i = 0; i < n; ++i) {
                double ya[4], yb[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    ya[q] = a0 + q < k ? Yb[(size_t)i * ldy + a0 + q] : 0.0;
                    yb[q] = b0 + q < k ? Yb[(size_t)i * ldy + b0 + q] : 0.0;
                }
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[p][q] += ya[p] * yb[q];
            }
            bool off = false;
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int a = a0 + p, b = b0 + q;
                    if (a < k && b < k && a <= b) {
                        G[(size_t)a * ldg + b] = acc[p][q];
                        off |= fabs(acc[p][q] - (a == b ? 1.0 : 0.0)) > 1e-6;
                    }
                }
            if (off) s_again = 1;
        }
        __syncthreads();
        // upper Cholesky factor in place by wave 0 (the diagonal keeps 1 / R_cc)
        if (tid < 64) {
            for (int c = 0; c < k; ++c) {
                const double pv = G[(size_t)c * ldg + c];
                if (!(pv > 1e-24)) {
                    if (lane == 0) s_fail = 1;
                    break;
                }
                const double ri = 1.0 / sqrt(pv);
                for (int l = c + 1 + lane; l < k; l += 64) G[(size_t)c * ldg + l] *= ri;
                if (!LDSRES) __threadfence_block();
                // trailing update over the (m x m) square, upper part; the pair
                // index advances by 64 without dividing
                const int m = k - c - 1;
                if (m > 0) {
                    const int di = 64 / m, dj = 64 - di * m;
                    int i = lane / m, l = lane - i * m;
                    for (int e = lane; e < m * m; e += 64) {
                        if (l >= i)
                            G[(size_t)(c + 1 + i) * ldg + c + 1 + l] -=
                                G[(size_t)c * ldg + c + 1 + i] * G[(size_t)c * ldg + c + 1 + l];
                        i += di;
                        l += dj;
                        if (l >= m) {
                            l -= m;
                            ++i;
                        }
                    }
                }
                if (lane == 0) G[(size_t)c * ldg + c] = ri;
                if (!LDSRES) __threadfence_block();
            }
        }
        __syncthreads();
        if (s_fail) break;
        // rows of Y: x R = y by forward substitution
        for (int i = tid; i < n; i += 1024) {
            double* yr = Yb + (size_t)i * ldy;
            for (int l = 0; l < k; ++l) {
                double sacc = yr[l];
                for (int m2 = 0; m2 < l; ++m2) sacc -= yr[m2] * G[(size_t)m2 * ldg + l];
                yr[l] = sacc * G[(size_t)l * ldg + l];
            }
        }
        __syncthreads();
    }
    if (s_fail) {
        if (tid == 0) atomicAdd(status, 1);
        return;
    }
    // ---- back-transform Y <- H_0 H_1 ... H_{n-3} Y by blocks of rb reflectors,
    // last block first: H_lo ... H_hi = I - V T V^T (compact WY form)
    const double* V = J.V;
    for (int hi = n - 3; hi >= 0; hi -= rb) {
        const int lo = max(0, hi - rb + 1), nb = hi - lo + 1;
        for (int e = tid; e < nb * n; e += 1024) {
            const int j = e / n, i = e - j * n, r = lo + j;
            Vb[e] = i <= r ? 0.0 : (i == r + 1 ? 1.0 : V[(size_t)r * n + i]);
        }
        for (int j = tid; j < nb; j += 1024) tb[j] = V[(size_t)(lo + j) * n + lo + j];
        __syncthreads();
        for (int e = tid; e < nb * nb; e += 1024) {  // C = V^T V (strict upper part)
            const int a = e / nb, b = e - a * nb;
            if (a < b) {
                double sacc = 0.0;
                for (int i = lo + b + 1; i < n; ++i) sacc += Vb[(size_t)a * n + i] * Vb[(size_t)b * n + i];
                Cb[e] = sacc;
            }
        }
        for (int e = tid; e < nb * k * 4; e += 1024) {  // Z = V^T Y, four threads per entry
            const int q = e & 3, jl = e >> 2, j = jl / k, l = jl - j * k;
            double sacc = 0.0;
            for (int i = lo + j + 1 + q; i < n; i += 4) sacc += Vb[(size_t)j * n + i] * Yb[(size_t)i * ldy + l];
            sacc += __shfl_xor(sacc, 1, 4);
            sacc += __shfl_xor(sacc, 2, 4);
            if (q == 0) Zb[(size_t)j * (k + 1) + l] = sacc;
        }
        __syncthreads();
        if (tid < 64) {  // T, one column at a time; lane a owns row a
            for (int j = 0; j < nb; ++j) {
                if (lane < j) {
                    double sacc = 0.0;
                    for (int b = lane; b < j; ++b) sacc += Tb[lane * rb + b] * Cb[b * nb + j];
                    Tb[lane * rb + j] = -tb[j] * sacc;
                }
                if (lane == j) Tb[j * rb + j] = tb[j];
            }
        }
        __syncthreads();
        for (int e = tid; e < nb * k; e += 1024) {  // W = T Z
            const int a = e / k, l = e - a * k;
            double sacc = 0.0;
            for (int b = a; b < nb; ++b) sacc += Tb[a * rb + b] * Zb[(size_t)b * (k + 1) + l];
            Wb[(size_t)a * (k + 1) + l] = sacc;
        }
        __syncthreads();
        for (int i = lo + 1 + (tid >> 6); i < n; i += 16) {  // Y -= V W, rows by wave
            const int jmax = min(nb, i - lo);
            for (int l = lane; l < k; l += 64) {
                double sacc = 0.0;
                for (int j = 0; j < jmax; ++j) sacc += Vb[(size_t)j * n + i] * Wb[(size_t)j * (k + 1) + l];
                Yb[(size_t)i * ldy + l] -= sacc;
            }
        }
        __syncthreads();
    }
    if (LDSRES) {
        for (int e = tid; e < n * k; e += 1024) {
            const int i = e / k, l = e % k;
            J.A[(size_t)i * n + l] = Yb[(size_t)i * ldy + l];
        }
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
    if (b > (size_t)kPartials / 4) b = kPartials / 4;
    if (b < 1) b = 1;
    return (int)b;
}

// One-launch reduction of NV sums: every block writes its NV block sums to
// part[v * kPartials / 4 + block]; the last block to arrive (counted at
// part + kPartials) adds each row in block order, writes scal[slots[v]] and
// resets the counter.  The order of every addition is fixed.
// Returns true in the block that wrote the sums (the last to arrive).
template <int NV>
__device__ bool reduce_rows(const double (&v)[NV], double* part, double* scal, const int (&slots)[NV]) {
    __shared__ double red[RED_THREADS];
    __shared__ int last;
    constexpr int stride = kPartials / 4;
    for (int r = 0; r < NV; ++r) {
        block_partial(v[r], red, part + r * stride + blockIdx.x);
        __syncthreads();
    }
    int* counter = reinterpret_cast<int*>(part + kPartials);
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(counter, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    for (int r = 0; r < NV; ++r) {
        double sacc = 0.0;
        for (int i = threadIdx.x; i < (int)gridDim.x; i += RED_THREADS) sacc += part[r * stride + i];
        block_partial(sacc, red, scal + slots[r]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *counter = 0;
    return true;
}

// Thread t of block b covers elements b*RED_THREADS + t + k*(nb*RED_THREADS).
__global__ __launch_bounds__(RED_THREADS) void k_dot(const double* a, const double* b, size_t n, double* part,
                                                     double* scal, int slot) {
    double s = 0.0;
    for (size_t e = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * RED_THREADS)
        s += a[e] * b[e];
    reduce_rows<1>({s}, part, scal, {slot});
}

__global__ __launch_bounds__(RED_THREADS) void k_cg_init(double* r, double* z, double* p, const double* b,
                                                         const double* q, const double* d, size_t n, double* part,
                                                         double* scal) {
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
    reduce_rows<3>({rz, rr, bb}, part, scal, {(int)S_RZ0, (int)S_RR, (int)S_BB});
}

__global__ __launch_bounds__(RED_THREADS) void k_shift_dot(double* q, const double* p, double shift, size_t n,
                                                           double* part, double* scal) {
    double s = 0.0;
    for (size_t e = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * RED_THREADS) {
        const double qv = q[e] - shift * p[e];
        q[e] = qv;
        s += p[e] * qv;
    }
    reduce_rows<1>({s}, part, scal, {(int)S_PQ});
}

// alpha = rz / pq (0 when pq is 0: a search direction that vanished)
__global__ __launch_bounds__(RED_THREADS) void k_cg_update(double* x, double* r, double* z, const double* p,
                                                           const double* q, const double* d, size_t n,
                                                           double* scal, int rz_cur, int rz_new, double* part,
                                                           double* host_out) {
    const double pq = scal[S_PQ];
    const double alpha = pq != 0.0 ? scal[rz_cur] / pq : 0.0;
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
    const bool last = reduce_rows<2>({rz, rr}, part, scal, {rz_new, (int)S_RR});
    // the scalars also go to the caller's pinned host buffer (its thread 0
    // wrote the new sums itself), flushed to system scope
    if (last && host_out != nullptr && threadIdx.x == 0) {
        for (int sl = 0; sl < S_N; ++sl) host_out[sl] = scal[sl];
        __threadfence_system();
    }
}

__global__ __launch_bounds__(RED_THREADS) void k_cg_direction(double* p, const double* z, size_t n,
                                                              const double* scal, int rz_cur, int rz_new) {
    const double den = scal[rz_cur];
    const double beta = den != 0.0 ? scal[rz_new] / den : 0.0;
    for (size_t e = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * RED_THREADS)
        p[e] = z[e] + beta * p[e];
}

// reduced-precision sigma: the direction also goes out as FP32 ...
__global__ __launch_bounds__(RED_THREADS) void k_cg_direction_lo(double* p, float* pf, const double* z, size_t n,
                                                                 const double* scal, int rz_cur, int rz_new) {
    const double den = scal[rz_cur];
    const double beta = den != 0.0 ? scal[rz_new] / den : 0.0;
    for (size_t e = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * RED_THREADS) {
        const double v = z[e] + beta * p[e];
        p[e] = v;
        pf[e] = (float)v;
    }
}

// ... and its FP32 product comes back as q = qf - shift p with p.q in FP64
__global__ __launch_bounds__(RED_THREADS) void k_shift_dot_lo(double* q, const float* qf, const double* p,
                                                              double shift, size_t n, double* part, double* scal) {
    double s = 0.0;
    for (size_t e = (size_t)blockIdx.x * RED_THREADS + threadIdx.x; e < n; e += (size_t)gridDim.x * RED_THREADS) {
        const double qv = (double)qf[e] - shift * p[e];
        q[e] = qv;
        s += p[e] * qv;
    }
    reduce_rows<1>({s}, part, scal, {(int)S_PQ});
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

struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double flops, bytes;
};

struct Stream {
    int device = 0;
    hipStream_t stream = nullptr;
    Tuning tune;
    // caching pool
    std::unordered_map<size_t, std::vector<void*>> free_blocks;
    std::unordered_map<void*, size_t> block_size;
    // profiling: every prof_every-th launch of each kind is recorded
    bool prof = false;
    int prof_every = 1;
    std::vector<ProfRec> pending;
    std::vector<hipEvent_t> event_pool;
    KernelStats stats[K_COUNT];
};

namespace {
thread_local Stream* t_cur = nullptr;
thread_local int t_device = -1;
std::mutex g_setup_mutex;
std::vector<bool> g_setup_done;

Stream& cur() {
    if (!t_cur) throw Error{MPSPT_E_STATE, "no library context bound to this thread"};
    return *t_cur;
}
hipStream_t cur_stream() { return cur().stream; }

// Once per device: LDS left for the eigensolver next to at most ~25 KB of
// static shared memory, granted to the kernels that take it dynamically.
void setup_device(int device) {
    std::lock_guard<std::mutex> lock(g_setup_mutex);
    if ((int)g_setup_done.size() <= device) g_setup_done.resize(device + 1, false);
    if (g_setup_done[device]) return;
    hipDeviceProp_t prop;
    check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
        throw Error{MPSPT_E_NODEV, std::string("device is ") + prop.gcnArchName + ", the library is built for gfx950"};
    int lds = 0;
    check(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device), "hipDeviceGetAttribute");
    const long budget = ((long)lds - 6 * EIG_MAXN * 8 - 1024) / 16 * 16;
    if (budget < 4096) throw Error{MPSPT_E_NODEV, "not enough LDS for the eigensolver"};
    if (g_lds_budget != 0 && g_lds_budget != (size_t)budget)
        throw Error{MPSPT_E_NODEV, "devices with different LDS sizes"};
    g_lds_budget = (size_t)budget;
    const void* ks[] = {reinterpret_cast<const void*>(&k_eig_reduce<true>),
                        reinterpret_cast<const void*>(&k_eig_vectors<true>),
                        reinterpret_cast<const void*>(&k_eig_vectors<false>)};
    for (const void* f : ks)
        check(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)budget), "hipFuncSetAttribute");
    g_setup_done[device] = true;
}
}  // namespace

Tuning& tuning() { return cur().tune; }

Stream* stream_create(int device, void* hip_stream) {
    int n = 0;
    const hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess)
        throw Error{MPSPT_E_NODEV, std::string("hipGetDeviceCount: ") + hipGetErrorString(e)};
    if (device < 0 || device >= n)
        throw Error{MPSPT_E_NODEV, "no HIP device " + std::to_string(device) + " (" + std::to_string(n) + " visible)"};
    check(hipSetDevice(device), "hipSetDevice");
    t_device = device;
    setup_device(device);
    Stream* s = new Stream();
    s->device = device;
    s->stream = static_cast<hipStream_t>(hip_stream);
    return s;
}

void bind(Stream* s) {
    t_cur = s;
    if (s && t_device != s->device) {
        check(hipSetDevice(s->device), "hipSetDevice");
        t_device = s->device;
    }
}

void stream_destroy(Stream* s) {
    if (!s) return;
    Stream* prev = t_cur;
    bind(s);
    (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->free_blocks)
        for (void* p : kv.second) (void)hipFree(p);
    for (auto& r : s->pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t ev : s->event_pool) (void)hipEventDestroy(ev);
    // blocks still handed out (none once the engine is gone) stay with the runtime
    delete s;
    t_cur = prev == s ? nullptr : prev;
}

// Stream-ordered caching allocator.  All device work of the library is issued
// on one stream, so a block released here can be handed to the next request
// at once: any later use is ordered after every earlier use on that stream.
// Sizes are rounded to 1/8 steps between powers of two; nothing is returned
// to the runtime before trim().
namespace {
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
    Stream& st = cur();
    const size_t c = size_class(bytes);
    auto it = st.free_blocks.find(c);
    if (it != st.free_blocks.end() && !it->second.empty()) {
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
    st.block_size[p] = c;
    return p;
}
void release(void* p) {
    if (!p) return;
    Stream& st = cur();
    auto it = st.block_size.find(p);
    if (it == st.block_size.end()) return;
    st.free_blocks[it->second].push_back(p);
}
void trim() {
    Stream& st = cur();
    (void)hipStreamSynchronize(st.stream);
    for (auto& kv : st.free_blocks)
        for (void* p : kv.second) {
            (void)hipFree(p);
            st.block_size.erase(p);
        }
    st.free_blocks.clear();
}
void h2d(void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    // ordered on the stream; pageable sources are staged by the runtime before it returns
    check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, cur_stream()), "hipMemcpyAsync H2D");
}
void d2h(void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, cur_stream()), "hipMemcpyAsync D2H");
    check(hipStreamSynchronize(cur_stream()), "hipStreamSynchronize");
}
void d2d(void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, cur_stream()), "hipMemcpyAsync D2D");
}
void zero(void* p, size_t bytes) {
    if (!bytes) return;
    check(hipMemsetAsync(p, 0, bytes, cur_stream()), "hipMemsetAsync");
}
void sync() { check(hipStreamSynchronize(cur_stream()), "hipStreamSynchronize"); }
hipStream_t stream() { return cur_stream(); }
void* host_alloc(size_t bytes) {
    void* p = nullptr;
    check(hipHostMalloc(&p, bytes, hipHostMallocDefault), "hipHostMalloc");
    return p;
}
void host_free(void* p) {
    if (p) (void)hipHostFree(p);
}
void d2h_async(void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, cur_stream()), "hipMemcpyAsync D2H");
}
void* event_create() {
    hipEvent_t e;
    check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    return e;
}
void event_destroy(void* e) {
    if (e) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
}
void event_record(void* e) { check(hipEventRecord(static_cast<hipEvent_t>(e), cur_stream()), "hipEventRecord"); }
void event_wait(void* e) { check(hipEventSynchronize(static_cast<hipEvent_t>(e)), "hipEventSynchronize"); }
double now() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------ profiling
namespace {

// Whether launch number c of a kind is recorded: a hash of (kind, c), so the
// one-in-every choice does not lock onto the period of a solver's launch
// pattern (a fixed stride would time the same stage of every iteration).
inline bool sampled(int kind, long long c, int every) {
    if (every <= 1) return true;
    uint64_t z = (uint64_t)c + 0x9E3779B97F4A7C15ull * (uint64_t)(kind + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z % (uint64_t)every == 0;
}

hipEvent_t take_event() {
    auto& pool = cur().event_pool;
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    check(hipEventCreate(&e), "hipEventCreate");
    return e;
}

void prof_flush() {
    Stream& st = cur();
    if (st.pending.empty()) return;
    check(hipEventSynchronize(st.pending.back().b), "hipEventSynchronize");
    for (auto& r : st.pending) {
        float ms = 0;
        check(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
        KernelStats& s = st.stats[r.kind];
        s.seconds += ms * 1e-3;
        s.flops += r.flops;
        s.bytes += r.bytes;
        s.launches++;
        st.event_pool.push_back(r.a);
        st.event_pool.push_back(r.b);
    }
    st.pending.clear();
}

// Launches on the library stream.  While recording, the launch goes through
// hipExtLaunchKernelGGL with a pair of events that take the dispatch's own
// start and end times, so the recorded durations are kernel execution only.
template <typename F, typename... Args>
void launch(int kind, double flops, double bytes, F kernel, dim3 grid, dim3 block, size_t shm, Args... args) {
    Stream& st = cur();
    if (st.prof && sampled(kind, st.stats[kind].launches_all++, st.prof_every)) {
        ProfRec r{kind, take_event(), take_event(), flops, bytes};
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)shm, st.stream, r.a, r.b, 0, args...);
        st.pending.push_back(r);
        if (st.pending.size() >= 4096) prof_flush();
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, st.stream, args...);
    }
}
}  // namespace

// Empty kernel launched whenever recording starts or stops, so that an
// external kernel trace can find the recorded window.
__global__ void k_profile_mark(int on) {}

void profile_enable(int every) {
    Stream& st = cur();
    if (st.prof) prof_flush();
    const bool on = every > 0;
    st.prof = on;
    st.prof_every = on ? every : 1;
    for (auto& s : st.stats) s = KernelStats();
    hipLaunchKernelGGL(k_profile_mark, dim3(1), dim3(64), 0, cur_stream(), on ? 1 : 0);
    check(hipGetLastError(), "k_profile_mark");
}

KernelStats profile_stats(int kind) {
    prof_flush();
    if (kind < 0 || kind >= K_COUNT) return KernelStats();
    return cur().stats[kind];
}

void gemm_grouped(const Bases& b, const GemmGroup* groups, const int* tile_group, const GemmTerm* terms, int ntiles,
                  int waves, double flops, double bytes) {
    if (ntiles <= 0) return;
    if (waves != 0 && waves != 4 && waves != 8 && waves != 16)
        throw Error{MPSPT_E_ARG, "grouped GEMM: waves per tile must be 0, 4, 8 or 16"};
    if (waves) {
        const int w = waves;
        if (w == 16)
            launch(K_GEMM, flops, bytes, k_gemm_grouped_split<16>, dim3(ntiles), dim3(1024), 0, b, groups, tile_group,
                   terms);
        else if (w == 8)
            launch(K_GEMM, flops, bytes, k_gemm_grouped_split<8>, dim3(ntiles), dim3(512), 0, b, groups, tile_group,
                   terms);
        else
            launch(K_GEMM, flops, bytes, k_gemm_grouped_split<4>, dim3(ntiles), dim3(256), 0, b, groups, tile_group,
                   terms);
    } else
        launch(K_GEMM, flops, bytes, k_gemm_grouped, dim3((ntiles + 3) / 4), dim3(256), 0, b, groups, tile_group,
               terms, ntiles);
    check(hipGetLastError(), "k_gemm_grouped");
}
void axpy_grouped(const Bases& b, const AxpyGroup* groups, int ngroups, const AxpyTerm* terms, double flops,
                  double bytes) {
    if (ngroups <= 0) return;
    launch(K_AXPY, flops, bytes, k_axpy_grouped, dim3(ngroups), dim3(256), 0, b, groups, terms);
    check(hipGetLastError(), "k_axpy_grouped");
}
void diag_grouped(const Bases& b, const DiagGroup* groups, int ngroups, const DiagTerm* terms) {
    if (ngroups <= 0) return;
    launch(K_DIAG, 0, 0, k_diag_grouped, dim3(ngroups), dim3(256), 0, b, groups, terms);
    check(hipGetLastError(), "k_diag_grouped");
}
void eig_reduce(const EigJob* jobs, int njobs, int nmax) {
    if (njobs <= 0) return;
    if (nmax > EIG_MAXN) throw Error{MPSPT_E_ARG, "eigensolver limited to n <= 512"};
    if (eig_reduce_class(nmax) == 0) {
        const size_t shm = (size_t)nmax * (nmax + 1) * sizeof(double);
        launch(K_EIG, 0, 0, k_eig_reduce<true>, dim3(njobs), dim3(1024), shm, jobs);
    } else {
        launch(K_EIG, 0, 0, k_eig_reduce<false>, dim3(njobs), dim3(1024), 0, jobs);
    }
    check(hipGetLastError(), "k_eig_reduce");
}
void eig_vectors(const EigJob* jobs, int njobs, int nmax, int kmax, int* status) {
    if (njobs <= 0) return;
    if (nmax > EIG_MAXN || kmax > nmax) throw Error{MPSPT_E_ARG, "eigensolver limited to k <= n <= 512"};
    const size_t words = g_lds_budget / sizeof(double);
    const size_t uw = (size_t)3 * nmax * kmax;  // solve rows, aliasing the later phases' LDS
    if (eig_vectors_class(nmax, kmax) == 0) {
        const size_t base = (size_t)nmax * (kmax + 1);
        const size_t need = eigv_lds_words(nmax, kmax, 16, true);
        const int u_lds = base + uw <= words ? 1 : 0;
        const size_t shm = std::max(need, u_lds ? base + uw : 0) * sizeof(double);
        launch(K_EIGV, 0, 0, k_eig_vectors<true>, dim3(njobs), dim3(1024), shm, jobs, status, 16, u_lds);
    } else {
        int rb = 16;
        while (rb > 1 && eigv_lds_words(nmax, kmax, rb, false) > words) --rb;
        const size_t need = eigv_lds_words(nmax, kmax, rb, false);
        const int u_lds = uw <= words ? 1 : 0;
        const size_t shm = std::max(need, u_lds ? uw : 0) * sizeof(double);
        launch(K_EIGV, 0, 0, k_eig_vectors<false>, dim3(njobs), dim3(1024), shm, jobs, status, rb, u_lds);
    }
    check(hipGetLastError(), "k_eig_vectors");
}
int eig_reduce_class(int n) { return (size_t)n * (n + 1) * sizeof(double) <= g_lds_budget ? 0 : 1; }
int eig_vectors_class(int n, int k) { return eigv_lds_words(n, k, 16, true) * sizeof(double) <= g_lds_budget ? 0 : 1; }
size_t eig_work(int n) { return 2 * (size_t)n + 4 * (size_t)n * n; }

void dot(const double* a, const double* b, size_t n, double* scal, int slot, double* partials) {
    const int nb = n_blocks(n);
    launch(K_VEC, 2.0 * n, 16.0 * n, k_dot, dim3(nb), dim3(RED_THREADS), 0, a, b, n, partials, scal, slot);
    check(hipGetLastError(), "dot");
}
void cg_init(double* r, double* z, double* p, const double* b, const double* q, const double* d, size_t n,
             double* scal, double* partials) {
    const int nb = n_blocks(n);
    launch(K_VEC, 6.0 * n, 48.0 * n, k_cg_init, dim3(nb), dim3(RED_THREADS), 0, r, z, p, b, q, d, n, partials, scal);
    check(hipGetLastError(), "cg_init");
}
void cg_shift_dot(double* q, const double* p, double shift, size_t n, double* scal, double* partials) {
    const int nb = n_blocks(n);
    launch(K_VEC, 4.0 * n, 24.0 * n, k_shift_dot, dim3(nb), dim3(RED_THREADS), 0, q, p, shift, n, partials, scal);
    check(hipGetLastError(), "cg_shift_dot");
}
void cg_update(double* x, double* r, double* z, const double* p, const double* q, const double* d, size_t n,
               double* scal, int rz_cur, int rz_new, double* partials, double* host_out) {
    const int nb = n_blocks(n);
    launch(K_VEC, 9.0 * n, 64.0 * n, k_cg_update, dim3(nb), dim3(RED_THREADS), 0, x, r, z, p, q, d, n, scal, rz_cur,
           rz_new, partials, host_out);
    check(hipGetLastError(), "cg_update");
}
void cg_direction(double* p, const double* z, size_t n, const double* scal, int rz_cur, int rz_new) {
    const int nb = n_blocks(n);
    launch(K_VEC, 2.0 * n, 24.0 * n, k_cg_direction, dim3(nb), dim3(RED_THREADS), 0, p, z, n, scal, rz_cur, rz_new);
    check(hipGetLastError(), "cg_direction");
}
void cg_direction_lo(double* p, float* pf, const double* z, size_t n, const double* scal, int rz_cur, int rz_new) {
    const int nb = n_blocks(n);
    launch(K_VEC, 2.0 * n, 28.0 * n, k_cg_direction_lo, dim3(nb), dim3(RED_THREADS), 0, p, pf, z, n, scal, rz_cur,
           rz_new);
    check(hipGetLastError(), "cg_direction_lo");
}
void cg_shift_dot_lo(double* q, const float* qf, const double* p, double shift, size_t n, double* scal,
                     double* partials) {
    const int nb = n_blocks(n);
    launch(K_VEC, 4.0 * n, 20.0 * n, k_shift_dot_lo, dim3(nb), dim3(RED_THREADS), 0, q, qf, p, shift, n, partials,
           scal);
    check(hipGetLastError(), "cg_shift_dot_lo");
}
void to_f32(float* dst, const double* src, size_t n) {
    if (n == 0) return;
    const int nb = (int)std::min<size_t>((n + 255) / 256, 2048);
    launch(K_VEC, 0.0, 12.0 * n, k_to_f32, dim3(nb), dim3(256), 0, dst, src, n);
    check(hipGetLastError(), "to_f32");
}
template <int MODE>
static void gemm_lo_launch(const BasesF& b, const GemmGroup* groups, const int* tile_group, const GemmTerm* terms,
                           int ntiles, int waves, double flops, double bytes) {
    if (waves == 16)
        launch(K_GEMM_LO, flops, bytes, k_gemm_grouped_lo_split<MODE, 16>, dim3(ntiles), dim3(1024), 0, b, groups,
               tile_group, terms);
    else if (waves == 8)
        launch(K_GEMM_LO, flops, bytes, k_gemm_grouped_lo_split<MODE, 8>, dim3(ntiles), dim3(512), 0, b, groups,
               tile_group, terms);
    else if (waves == 4)
        launch(K_GEMM_LO, flops, bytes, k_gemm_grouped_lo_split<MODE, 4>, dim3(ntiles), dim3(256), 0, b, groups,
               tile_group, terms);
    else
        launch(K_GEMM_LO, flops, bytes, k_gemm_grouped_lo<MODE>, dim3((ntiles + 3) / 4), dim3(256), 0, b, groups,
               tile_group, terms, ntiles);
}
void gemm_grouped_lo(const BasesF& b, int mode, const GemmGroup* groups, const int* tile_group, const GemmTerm* terms,
                     int ntiles, int waves, double flops, double bytes) {
    if (ntiles <= 0) return;
    if (mode != 1 && mode != 2) throw Error{MPSPT_E_ARG, "reduced-precision GEMM mode must be 1 (FP32) or 2 (BF16x3)"};
    if (waves != 0 && waves != 4 && waves != 8 && waves != 16)
        throw Error{MPSPT_E_ARG, "grouped GEMM: waves per tile must be 0, 4, 8 or 16"};
    if (mode == 1)
        gemm_lo_launch<1>(b, groups, tile_group, terms, ntiles, waves, flops, bytes);
    else
        gemm_lo_launch<2>(b, groups, tile_group, terms, ntiles, waves, flops, bytes);
    check(hipGetLastError(), "k_gemm_grouped_lo");
}
void axpy_grouped_lo(const BasesF& b, const AxpyGroup* groups, int ngroups, const AxpyTerm* terms, double flops,
                     double bytes) {
    if (ngroups <= 0) return;
    launch(K_AXPY_LO, flops, bytes, k_axpy_grouped_lo, dim3(ngroups), dim3(256), 0, b, groups, terms);
    check(hipGetLastError(), "k_axpy_grouped_lo");
}
void davidson_precond(double* t, const double* r, const double* d, double theta, size_t n) {
    if (!n) return;
    const int nb = n_blocks(n);
    launch(K_VEC, 3.0 * n, 24.0 * n, k_dav_precond, dim3(nb), dim3(RED_THREADS), 0, t, r, d, theta, n);
    check(hipGetLastError(), "davidson_precond");
}
void axpby(double* y, const double* x, double a, double b, size_t n) {
    if (!n) return;
    const int nb = n_blocks(n);
    launch(K_VEC, 3.0 * n, 24.0 * n, k_axpby, dim3(nb), dim3(RED_THREADS), 0, y, x, a, b, n);
    check(hipGetLastError(), "axpby");
}

}  // namespace dev
}  // namespace mpspt
