// Learned block-scaled Jacobi preconditioner for the local CG solves.
//
// Every block B of the two-site tensor gets the preconditioner s_B D_B^-1
// instead of D_B^-1, with s_B > 0 predicted by an 8-64-64-1 network (tanh
// hidden layers, softplus output) from statistics of the block's diagonal
// and right-hand side.  A positive block scaling keeps the preconditioner
// symmetric positive definite, so CG converges to the same solution.  The
// statistics are those of the diagonal and of the initial residual r0 of the
// warm-started CG; training targets fit the initial error by the Jacobi step
// of r0 block by block.
//
// * k_block_stats: per block, sums of log d, (log d)^2, r^2, z.e and z.z
//   (z = r / d, the Jacobi step of a residual r; e an error estimate) and the
//   extremes of log d.
// * k_precond_scales: features from those statistics, the network's
//   forward pass (parameters in LDS), one thread per block.
// * k_scale_blocks: d <- d / s_B on every element of block B.
// * k_mlp_train: loss, backpropagation and optionally one Adam step over a
//   batch of (features, target) samples in one 256-thread workgroup; every
//   sum runs over the samples in index order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/mpspt.h"
#include "device.hpp"

namespace mpspt {
namespace dev {
void check(hipError_t e, const char* what);
hipStream_t stream();

namespace {
constexpr int NF = kMlpIn, NH = kMlpHidden;
// offsets of the flat parameter vector
constexpr int OW1 = 0, OB1 = NH * NF, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH, OB3 = OW3 + NH;
static_assert(OB3 + 1 == kMlpParams, "parameter layout");
constexpr int ST = 8;  // statistics per block

__device__ inline double wave_sum_d(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// 256 threads per block of the two-site tensor
__global__ __launch_bounds__(256) void k_block_stats(const BlockRef* __restrict__ blocks, const double* d,
                                                     const double* r, const double* e, double* stats) {
    __shared__ double red[4][6];
    __shared__ double mn[4], mx[4];
    const BlockRef B = blocks[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double s_ld = 0, s_ld2 = 0, s_b2 = 0, s_zx = 0, s_zz = 0, lo = 1e300, hi = -1e300;
    const int total = B.m * B.n;
    for (int el = tid; el < total; el += 256) {
        const int i = el / B.n, j = el - i * B.n;
        const size_t o = (size_t)B.off + (size_t)i * B.ld + j;
        const double dv = d[o], rv = r[o], l = log(dv), z = rv / dv;
        s_ld += l;
        s_ld2 += l * l;
        s_b2 += rv * rv;
        s_zz += z * z;
        if (e) s_zx += z * e[o];
        lo = fmin(lo, l);
        hi = fmax(hi, l);
    }
    double v[6] = {s_ld, s_ld2, s_b2, s_zx, s_zz, 0.0};
    for (int k = 0; k < 5; ++k) v[k] = wave_sum_d(v[k]);
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if (lane == 0) {
        for (int k = 0; k < 5; ++k) red[wave][k] = v[k];
        mn[wave] = lo;
        mx[wave] = hi;
    }
    __syncthreads();
    if (tid == 0) {
        double* s = stats + (size_t)blockIdx.x * ST;
        for (int k = 0; k < 5; ++k) s[k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
        s[5] = fmin(fmin(mn[0], mn[1]), fmin(mn[2], mn[3]));
        s[6] = fmax(fmax(mx[0], mx[1]), fmax(mx[2], mx[3]));
        s[7] = (double)total;
    }
}

__device__ inline float softplusf(float o) { return fmaxf(o, 0.0f) + log1pf(expf(-fabsf(o))); }

// one thread per block; every workgroup recomputes the total |b|^2 in the same order
__global__ __launch_bounds__(256) void k_precond_scales(const double* __restrict__ stats,
                                                        const BlockRef* __restrict__ blocks, int nb, float site_frac,
                                                        const float* __restrict__ params, float* feat,
                                                        float* scale) {
    __shared__ float P[kMlpParams];
    __shared__ double red[256];
    for (int k = threadIdx.x; k < kMlpParams; k += 256) P[k] = params[k];
    double part = 0.0;
    for (int k = threadIdx.x; k < nb; k += 256) part += stats[(size_t)k * ST + 2];
    red[threadIdx.x] = part;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double ball = fmax(sqrt(red[0]), 1e-300);
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= nb) return;
    const double* s = stats + (size_t)k * ST;
    const double cnt = s[7], mu = s[0] / cnt;
    const double var = fmax(s[1] / cnt - mu * mu, 0.0);
    float f[NF];
    f[0] = (float)mu;
    f[1] = (float)sqrt(var);
    f[2] = (float)(s[5] - mu);
    f[3] = (float)(s[6] - mu);
    f[4] = logf((float)blocks[k].m);
    f[5] = logf((float)blocks[k].n);
    f[6] = (float)log(fmax(sqrt(s[2]), 1e-300) / ball);
    f[7] = site_frac;
    if (feat)
        for (int q = 0; q < NF; ++q) feat[(size_t)k * NF + q] = f[q];
    float h1[NH];
    for (int j = 0; j < NH; ++j) {
        float a = P[OB1 + j];
        for (int q = 0; q < NF; ++q) a += P[OW1 + j * NF + q] * f[q];
        h1[j] = tanhf(a);
    }
    float o = P[OB3];
    for (int j = 0; j < NH; ++j) {
        float a = P[OB2 + j];
        for (int q = 0; q < NH; ++q) a += P[OW2 + j * NH + q] * h1[q];
        o += P[OW3 + j] * tanhf(a);
    }
    scale[k] = softplusf(o);
}

__global__ __launch_bounds__(256) void k_scale_blocks(const BlockRef* __restrict__ blocks,
                                                      const float* __restrict__ scale, double* d) {
    const BlockRef B = blocks[blockIdx.x];
    const double inv = 1.0 / (double)scale[blockIdx.x];
    const int total = B.m * B.n;
    for (int e = threadIdx.x; e < total; e += 256) {
        const int i = e / B.n, j = e - i * B.n;
        d[(size_t)B.off + (size_t)i * B.ld + j] *= inv;
    }
}

// Scratch per sample: h1[NH], h2[NH], da1[NH], da2[NH], dL/do.
constexpr int SCR = 4 * NH + 1;

__global__ __launch_bounds__(256) void k_mlp_train(const float* __restrict__ X, const float* __restrict__ t, int n,
                                                    float* params, float* m, float* v, float* grad, float* loss,
                                                    int step, float lr, int update, float* scr) {
    __shared__ float P[kMlpParams];
    __shared__ float red[256];
    const int tid = threadIdx.x;
    for (int k = tid; k < kMlpParams; k += 256) P[k] = params[k];
    __syncthreads();
    // ---- forward and backpropagation per sample
    float lpart = 0.0f;
    for (int sm = tid; sm < n; sm += 256) {
        float* S = scr + (size_t)sm * SCR;
        const float* xs = X + (size_t)sm * NF;
        float h1[NH];
        for (int j = 0; j < NH; ++j) {
            float a = P[OB1 + j];
            for (int q = 0; q < NF; ++q) a += P[OW1 + j * NF + q] * xs[q];
            h1[j] = tanhf(a);
            S[j] = h1[j];
        }
        float o = P[OB3];
        for (int j = 0; j < NH; ++j) {
            float a = P[OB2 + j];
            for (int q = 0; q < NH; ++q) a += P[OW2 + j * NH + q] * h1[q];
            const float h2 = tanhf(a);
            S[NH + j] = h2;
            o += P[OW3 + j] * h2;
        }
        const float sp = softplusf(o);
        const float r = logf(sp) - logf(t[sm]);
        lpart += r * r;
        const float sig = 1.0f / (1.0f + expf(-o));
        const float dout = (2.0f / (float)n) * r * sig / sp;
        S[4 * NH] = dout;
        float da1[NH];
        for (int q = 0; q < NH; ++q) da1[q] = 0.0f;
        for (int j = 0; j < NH; ++j) {
            const float h2 = S[NH + j];
            const float da2 = dout * P[OW3 + j] * (1.0f - h2 * h2);
            S[3 * NH + j] = da2;
            for (int q = 0; q < NH; ++q) da1[q] += P[OW2 + j * NH + q] * da2;
        }
        for (int q = 0; q < NH; ++q) S[2 * NH + q] = da1[q] * (1.0f - h1[q] * h1[q]);
    }
    red[tid] = lpart;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) *loss = red[0] / (float)n;
    // ---- parameter gradients: sums over the samples in order
    for (int k = tid; k < kMlpParams; k += 256) {
        float g = 0.0f;
        if (k < OB1) {  // W1[j][q]
            const int j = k / NF, q = k - j * NF;
            for (int sm = 0; sm < n; ++sm) g += scr[(size_t)sm * SCR + 2 * NH + j] * X[(size_t)sm * NF + q];
        } else if (k < OW2) {  // b1[j]
            const int j = k - OB1;
            for (int sm = 0; sm < n; ++sm) g += scr[(size_t)sm * SCR + 2 * NH + j];
        } else if (k < OB2) {  // W2[j][q]
            const int j = (k - OW2) / NH, q = (k - OW2) - j * NH;
            for (int sm = 0; sm < n; ++sm) g += scr[(size_t)sm * SCR + 3 * NH + j] * scr[(size_t)sm * SCR + q];
        } else if (k < OW3) {  // b2[j]
            const int j = k - OB2;
            for (int sm = 0; sm < n; ++sm) g += scr[(size_t)sm * SCR + 3 * NH + j];
        } else if (k < OB3) {  // w3[j]
            const int j = k - OW3;
            for (int sm = 0; sm < n; ++sm) g += scr[(size_t)sm * SCR + 4 * NH] * scr[(size_t)sm * SCR + NH + j];
        } else {  // b3
            for (int sm = 0; sm < n; ++sm) g += scr[(size_t)sm * SCR + 4 * NH];
        }
        if (grad) grad[k] = g;
        if (update) {
            const float b1c = 1.0f - powf(0.9f, (float)step), b2c = 1.0f - powf(0.999f, (float)step);
            const float mk = 0.9f * m[k] + 0.1f * g, vk = 0.999f * v[k] + 0.001f * g * g;
            m[k] = mk;
            v[k] = vk;
            params[k] = P[k] - lr * (mk / b1c) / (sqrtf(vk / b2c) + 1e-8f);
        }
    }
}
}  // namespace

void block_stats(const BlockRef* blocks, int nb, const double* d, const double* r, const double* e, double* stats) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_block_stats, dim3(nb), dim3(256), 0, stream(), blocks, d, r, e, stats);
    check(hipGetLastError(), "k_block_stats");
}
void precond_scales(const double* stats, const BlockRef* blocks, int nb, float site_frac, const float* params,
                    float* feat, float* scale) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_precond_scales, dim3((nb + 255) / 256), dim3(256), 0, stream(), stats, blocks, nb,
                       site_frac, params, feat, scale);
    check(hipGetLastError(), "k_precond_scales");
}
void scale_blocks(const BlockRef* blocks, int nb, const float* scale, double* d) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_scale_blocks, dim3(nb), dim3(256), 0, stream(), blocks, scale, d);
    check(hipGetLastError(), "k_scale_blocks");
}
void mlp_train(const float* X, const float* t, int n, float* params, float* m, float* v, float* grad, float* loss,
               int step, float lr, bool update, float* scratch) {
    if (n <= 0) throw Error{MPSPT_E_ARG, "training batch is empty"};
    hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(256), 0, stream(), X, t, n, params, m, v, grad, loss, step, lr,
                       update ? 1 : 0, scratch);
    check(hipGetLastError(), "k_mlp_train");
}
size_t mlp_scratch_floats(int n) { return (size_t)n * SCR; }

}  // namespace dev
}  // namespace mpspt
