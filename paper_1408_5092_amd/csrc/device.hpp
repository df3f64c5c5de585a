// Device-side primitives of the MPS-PT engine (implemented in kernels.hip).
//
// The host engine expresses every contraction as a work list of small dense
// block operations and hands it to one of these grouped kernels.  Work lists
// are output-stationary: each group owns one output block and sums all of
// its terms in a fixed order, so results are deterministic and no atomics
// are involved.
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>

namespace mpspt {
namespace dev {

// Work lists address device memory as (slot, offset): the launch passes the
// base pointer of each slot, so a list built once stays valid when the
// buffers it reads and writes move.  Slot kAbsSlot has base 0 (the offset is
// the address itself).
constexpr int kSlots = 8;
constexpr int kAbsSlot = kSlots - 1;
struct Bases {
    double* p[kSlots];
};
// The same slots over FP32 copies (reduced-precision sigma; no absolute slot).
struct BasesF {
    float* p[kSlots];
};

// C (m x n, leading dimension ldc) [+]= sum_t alpha_t op(A_t) op(B_t), computed in
// GEMM_TILE x GEMM_TILE output tiles
constexpr int GEMM_TILE = 16;
struct GemmTerm {
    int64_t oa, ob;
    double alpha;
    int32_t lda, ldb, k;
    int8_t sa, sb;
    int8_t transA, transB;  // op(A) = A^T when set (A stored k x m)
};
struct GemmGroup {
    int64_t oc;
    int32_t ldc, m, n;
    int32_t term0, nterms;
    int32_t tile0;  // first tile index of this group in the launch
    int8_t sc;
    int8_t accumulate;  // 0: overwrite C, 1: add to C
};

// dst (m x n) [+]= sum_t alpha_t op(src_t)
struct AxpyTerm {
    int64_t os;
    double alpha;
    int32_t lds;
    int8_t ss, trans;
};
struct AxpyGroup {
    int64_t od;
    int32_t ldd, m, n;
    int32_t term0, nterms;
    int8_t sd, accumulate;
};

// dst (m x n) = shift + sum_t c_t L_t[i * ls] R_t[j * rs]
struct DiagTerm {
    int64_t ol, orr;
    double c;
    int32_t ls, rs;
    int8_t sl, sr;
};
struct DiagGroup {
    int64_t od;
    double shift;
    int32_t ldd, m, n;
    int32_t term0, nterms;
    int8_t sd;
};

// Symmetric eigenproblem of a density-matrix sector.  eig_reduce: A (n x n,
// row major, symmetric) is reduced to tridiagonal form (reflectors in V, n x n;
// tridiagonal in t) and w receives all eigenvalues, descending.  eig_vectors:
// the first k columns of A receive an orthonormal basis of the invariant
// subspace of the k largest eigenvalues.  t holds eig_work(n) doubles.
struct EigJob {
    double* A;
    double* V;
    double* w;
    double* t;
    int32_t n, k;
};

struct Error {
    int code;  // mpspt_status value
    std::string msg;
};

// Device state of one library context: its device, its HIP stream, a caching
// pool ordered on that stream and its profiling records.  Every call below
// acts on the state bound to the calling thread, so contexts on different
// threads (and streams) run side by side; one state serves one thread at a time.
struct Stream;
Stream* stream_create(int device, void* hip_stream);  // throws Error
void stream_destroy(Stream* s);                        // waits for the stream, frees its pool
void bind(Stream* s);                                  // make s current on this thread
// Launch-shape parameters of the grouped GEMM work lists, per context:
// wide_chunks: a list whose longest tile k chain has this many chunks of 16
// runs one workgroup of split_waves (4, 8 or 16) waves per tile with the
// chunks spread over them (else one wave per tile); kseg_min / kseg_div: a
// group whose summed k exceeds max(kseg_min, list work / kseg_div) is split
// into segments reduced in order.
struct Tuning {
    int wide_chunks = 8, kseg_min = 512, kseg_div = 8192, split_waves = 4;
};
Tuning& tuning();                                      // of the context bound to this thread
int device_count();
void* alloc(size_t bytes);                  // throws Error (MPSPT_E_NOMEM); stream-ordered pool
void release(void* p);                      // back to the pool; safe while earlier launches run
void trim();                                // return cached blocks to the runtime
void h2d(void* dst, const void* src, size_t bytes);
void d2h(void* dst, const void* src, size_t bytes);  // synchronous
void d2d(void* dst, const void* src, size_t bytes);
void zero(void* p, size_t bytes);
void sync();
// Ordered device-to-host copy into pinned host memory that does not wait;
// event_record/event_wait mark and await its completion.
void* host_alloc(size_t bytes);  // pinned
void host_free(void* p);
void d2h_async(void* dst, const void* src, size_t bytes);
void* event_create();
void event_destroy(void* e);
void event_record(void* e);
void event_wait(void* e);
double now();  // host seconds

// flops / bytes: algorithmic work of the launch, used only by the profiler
// tile_group[t]: the group of tile t.  waves = 4, 8 or 16: one workgroup of
// that many waves per tile with the tile's k chunks spread over them (long k
// chains); 0: one wave per tile.
void gemm_grouped(const Bases& b, const GemmGroup* groups, const int* tile_group, const GemmTerm* terms, int ntiles,
                  int waves, double flops = 0, double bytes = 0);
void axpy_grouped(const Bases& b, const AxpyGroup* groups, int ngroups, const AxpyTerm* terms, double flops = 0,
                  double bytes = 0);

// Per-kernel timing with HIP events recorded on the library's stream.
enum KernelKind { K_GEMM = 0, K_AXPY = 1, K_EIG = 2, K_DIAG = 3, K_EIGV = 4, K_VEC = 5, K_GEMM_LO = 6, K_AXPY_LO = 7,
                  K_COUNT = 8 };
// seconds / flops / bytes / launches cover the recorded (sampled) launches;
// launches_all counts every launch of the kind while recording was on.
struct KernelStats {
    double seconds = 0, flops = 0, bytes = 0;
    long long launches = 0, launches_all = 0;
};
// every >= 1: record each launch with probability 1/every (a hash of the kind
// and the launch count decides; 1: all); 0: off.
// Resets the counters.
void profile_enable(int every);
KernelStats profile_stats(int kind);   // waits for outstanding launches
void diag_grouped(const Bases& b, const DiagGroup* groups, int ngroups, const DiagTerm* terms);
// nmax / kmax: largest n / k among the jobs.  Variant 0 of each kernel keeps
// the matrix (eig_reduce) or the basis (eig_vectors) in LDS, variant 1 in
// global memory; batch jobs of one class together.  eig_vectors adds one to
// *status (device int) per job whose basis could not be orthonormalised.
void eig_reduce(const EigJob* jobs, int njobs, int nmax);
void eig_vectors(const EigJob* jobs, int njobs, int nmax, int kmax, int* status);
int eig_reduce_class(int n);
int eig_vectors_class(int n, int k);
size_t eig_work(int n);

// Vector kernels over length-n double vectors.  `scal` is a small device
// array of scalars; `partials` is the reduction workspace of kPartialsWords
// doubles whose last words (a counter) must be zero before first use and are
// left zero by every call.  All reductions are fixed-order, one launch each.
enum Scalar { S_PQ = 0, S_RZ0 = 1, S_RZ1 = 2, S_RR = 3, S_BB = 4, S_DOT = 5, S_N = 8 };
void dot(const double* a, const double* b, size_t n, double* scal, int slot, double* partials);
// r = -b - q ; z = r / d ; p = z ; scal[RZ0] = r.z ; scal[RR] = r.r ; scal[BB] = b.b
void cg_init(double* r, double* z, double* p, const double* b, const double* q, const double* d,
             size_t n, double* scal, double* partials);
// q -= shift * p ; scal[PQ] = p.q
void cg_shift_dot(double* q, const double* p, double shift, size_t n, double* scal, double* partials);
// alpha = rz_cur / pq (0 if pq = 0) ; x += alpha p ; r -= alpha q ; z = r / d ;
// scal[rz_new] = r.z ; scal[RR] = r.r ; host_out (pinned, from host_alloc;
// may be null) receives scal[0 .. S_N) once the sums are in, readable after
// an event recorded behind the launch has completed
void cg_update(double* x, double* r, double* z, const double* p, const double* q, const double* d,
               size_t n, double* scal, int rz_cur, int rz_new, double* partials, double* host_out = nullptr);
// p = z + (rz_new / rz_cur) p (beta = 0 if rz_cur = 0)
void cg_direction(double* p, const double* z, size_t n, const double* scal, int rz_cur, int rz_new);
// y = a x + b y
void axpby(double* y, const double* x, double a, double b, size_t n);
// Reduced-precision sigma (mode 1: FP32 MFMA, 2: BF16x3 split products with
// FP32 accumulation) over the same work lists, on FP32 operand copies.
void gemm_grouped_lo(const BasesF& b, int mode, const GemmGroup* groups, const int* tile_group, const GemmTerm* terms,
                     int ntiles, int waves, double flops = 0, double bytes = 0);
void axpy_grouped_lo(const BasesF& b, const AxpyGroup* groups, int ngroups, const AxpyTerm* terms, double flops = 0,
                     double bytes = 0);
void to_f32(float* dst, const double* src, size_t n);
// p = z + beta p as in cg_direction, also written to pf in FP32
void cg_direction_lo(double* p, float* pf, const double* z, size_t n, const double* scal, int rz_cur, int rz_new);
// q = qf - shift * p (qf: FP32 product) ; scal[PQ] = p.q
void cg_shift_dot_lo(double* q, const float* qf, const double* p, double shift, size_t n, double* scal,
                     double* partials);
// t = r / (theta - d), with |theta - d| floored at 1e-8 (Davidson correction)
void davidson_precond(double* t, const double* r, const double* d, double theta, size_t n);

// Learned preconditioner (precond.hip).  A block of a two-site vector:
// offset (doubles), leading dimension, rows, columns.
struct BlockRef {
    int64_t off;
    int32_t ld, m, n;
};
constexpr int kMlpIn = 8, kMlpHidden = 64;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + 2 * kMlpHidden + 1;
constexpr int kBlockStats = 8;  // per block: sum log d, sum (log d)^2, |r|^2, z.e, z.z, min / max log d, count
// stats[nb][kBlockStats] of d, r and (if e is not null) e, with z = r / d
void block_stats(const BlockRef* blocks, int nb, const double* d, const double* r, const double* e, double* stats);
// features feat[nb][kMlpIn] (if not null) and network scales scale[nb]
void precond_scales(const double* stats, const BlockRef* blocks, int nb, float site_frac, const float* params,
                    float* feat, float* scale);
// d <- d / scale on every element of each block
void scale_blocks(const BlockRef* blocks, int nb, const float* scale, double* d);
// Loss (and gradient into grad, if not null) of the network over n samples,
// then one Adam step when update is set (step counts from 1).
void mlp_train(const float* X, const float* t, int n, float* params, float* m, float* v, float* grad, float* loss,
               int step, float lr, bool update, float* scratch);
size_t mlp_scratch_floats(int n);

constexpr int kPartials = 512;        // block sums: four rows of kPartials / 4
constexpr int kPartialsWords = 520;   // with the arrival counter after them

}  // namespace dev
}  // namespace mpspt
