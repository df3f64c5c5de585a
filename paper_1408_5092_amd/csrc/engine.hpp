// Host side of the MPS-PT sweep: block-sparse tensors, work-list builders and
// the two-site sweep driver.  All arithmetic on tensor data runs in the
// grouped device kernels of device.hpp.
#pragma once
#include <map>
#include <memory>
#include <set>
#include <string>
#include <cstring>
#include <vector>

#include "device.hpp"
#include "mpo.hpp"

namespace mpspt {

// ---------------------------------------------------------------- storage
class DevBuf {
  public:
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept { swap(o); }
    DevBuf& operator=(DevBuf&& o) noexcept { swap(o); return *this; }
    ~DevBuf() { reset(); }
    void reset();
    void alloc(size_t count);   // exactly count doubles; contents undefined
    void ensure(size_t count);  // at least count doubles; contents undefined when it grows
    double* p = nullptr;
    size_t n = 0;

  private:
    void swap(DevBuf& o) { std::swap(p, o.p); std::swap(n, o.n); }
};

template <class T>
class DevArr {
  public:
    DevArr() = default;
    DevArr(const DevArr&) = delete;
    DevArr& operator=(const DevArr&) = delete;
    ~DevArr() {
        if (p) dev::release(p);  // stream-ordered pool
    }
    void upload(const std::vector<T>& v) {
        ensure(v.size());
        if (!v.empty()) dev::h2d(p, v.data(), v.size() * sizeof(T));
    }
    void ensure(size_t n) {  // capacity for n elements (contents not kept)
        if (n > cap) {
            if (p) dev::release(p);
            cap = n + n / 2 + 16;
            p = static_cast<T*>(dev::alloc(cap * sizeof(T)));
        }
    }
    T* p = nullptr;
    size_t cap = 0;
};

// Host arrays staged back to back (each on a 256-byte boundary) so that a
// work list reaches the device in one copy.
class Packer {
  public:
    // places v at the next 256-byte boundary; v must stay unchanged until upload()
    template <class T>
    size_t add(const std::vector<T>& v) {
        const size_t off = (size_ + 255) & ~size_t(255);
        if (!v.empty()) sec_.push_back({off, v.data(), v.size() * sizeof(T)});
        size_ = off + v.size() * sizeof(T);
        return off;
    }
    size_t size() const { return size_; }
    // copies the sections into buf (grown to size() bytes): small lists as
    // one host image in one copy, large ones section by section straight from
    // their vectors (the runtime stages pageable memory itself, so an image
    // would only add a pass over the bytes)
    void upload(DevArr<char>& buf) const;

  private:
    struct Sec {
        size_t off;
        const void* p;
        size_t n;
    };
    std::vector<Sec> sec_;
    size_t size_ = 0;
};

struct Bond {
    std::vector<QN> q;
    std::vector<int> d;
    int find(QN x) const;
    int total() const;
    bool operator==(const Bond& o) const { return q == o.q && d == o.d; }
};

// MPS site tensor: blocks (left sector il, local state s) -> right sector jr,
// stored as one row panel per left sector with its blocks side by side.
struct Site {
    Bond L, R;
    struct Blk { int il, s, jr, rows, cols, col; };
    std::vector<Blk> blk;
    std::vector<int> idx;      // il * 4 + s -> block or -1
    std::vector<int> pw;       // panel width per left sector
    std::vector<size_t> po;    // panel offset per left sector
    std::vector<std::vector<int>> by_jr;
    size_t size = 0;
    DevBuf data;
    double* at(int b) const { return data.p + po[blk[b].il] + blk[b].col; }
    int ld(int b) const { return pw[blk[b].il]; }
};
Site make_site(const Bond& L, const Bond& R);

// Two-site tensor of a window: blocks (il, s1, s2) -> jr, one row panel per il.
struct Two {
    Bond L, R;
    struct Blk { int il, s1, s2, jr, rows, cols, col; };
    std::vector<Blk> blk;
    std::vector<int> idx;      // (il * 4 + s1) * 4 + s2 -> block or -1
    std::vector<int> pw;
    std::vector<size_t> po;
    size_t size = 0;
    size_t off(int b) const { return po[blk[b].il] + blk[b].col; }
    int ld(int b) const { return pw[blk[b].il]; }
};
Two make_two(const Bond& L, const Bond& R, const std::set<QN>* mid_ok);

// Environment: per MPO channel w a block-sparse bra x ket matrix whose
// blocks (ib, ik) satisfy q_bra = q_ket + dq(w).
struct Env {
    int nch = 0;
    Bond bra, ket;
    struct Blk { int w, ib, ik, rows, cols; size_t off; };
    std::vector<Blk> blk;
    std::vector<int> idx;      // w * nbra + ib -> block or -1
    std::vector<std::vector<int>> by_w;
    std::vector<std::vector<int>> by_ib;  // blocks per bra sector, ascending channel
    std::vector<QN> dq;        // per channel
    size_t size = 0;
    DevBuf data;
    int find(int w, int ib) const { return idx[(size_t)w * bra.q.size() + ib]; }
    void index();
    void copy_layout(const Env& o);  // everything but the data
};

// Two-site operator of a window: sum over the middle channel of W_i (x) W_{i+1}.
struct TwoOp {
    struct E { int w, s1, s2; double v; };
    int nin = 0, nout = 0;
    std::vector<std::vector<E>> by_out;  // (w' * 16 + s1' * 4 + s2') -> terms
};
TwoOp make_twoop(const MPO& m, int i);

// Slots of a work list: the device buffers it addresses, each as a base
// pointer and an extent in doubles.  Pointers handed to group()/term() are
// stored relative to the slot that contains them (the absolute slot when
// none does); rebinding a slot moves every reference to it.
class SlotMap {
  public:
    void bind(int slot, const double* base, size_t count) {
        base_[slot] = base;
        cnt_[slot] = count;
    }
    void ref(const double* p, int8_t& slot, int64_t& off) const;
    dev::Bases bases() const;

  private:
    const double* base_[dev::kSlots] = {};
    size_t cnt_[dev::kSlots] = {};
    mutable int last_ = 0;  // slot of the previous match, tried first
};

// Work list of grouped block axpys, reusable across launches.
class AxpyBatch {
  public:
    void clear() { g_.clear(); t_.clear(); flops_ = 0; bytes_ = 0; abs_ = false; }
    void bind(int slot, const double* base, size_t count) { slots_.bind(slot, base, count); }
    void group(double* dst, int ldd, int m, int n, bool acc);
    void term(const double* src, int lds, bool trans, double alpha);
    // slot-relative forms
    void group_ref(int8_t slot, int64_t off, int ldd, int m, int n, bool acc);
    void term_ref(int8_t slot, int64_t off, int lds, bool trans, double alpha);
    void reserve(size_t groups, size_t terms) { g_.reserve(groups); t_.reserve(terms); }
    void upload();
    // upload() in two halves, for a list that travels inside another's copy:
    // stage the groups and terms, then point at their device copy
    void pack(Packer& pk);
    void attach(const char* dev_base);
    void run() const { run(slots_.bases()); }
    void run(const dev::Bases& b) const;
    void run_lo(const dev::BasesF& b) const;  // FP32 copies of the slots
    bool empty() const { return g_.empty(); }
    double flops() const { return flops_; }  // counted by pack()
    double bytes() const { return bytes_; }

  private:
    SlotMap slots_;
    std::vector<dev::AxpyGroup> g_;
    std::vector<dev::AxpyTerm> t_;
    DevArr<char> buf_;  // groups and terms, one copy
    size_t og_ = 0, ot_ = 0;
    const dev::AxpyGroup* dg_ = nullptr;
    const dev::AxpyTerm* dt_ = nullptr;
    double flops_ = 0, bytes_ = 0;
    bool abs_ = false;  // some reference lies outside the bound slots
};

// Work list of grouped GEMMs, reusable across launches.  Slot kPartSlot is
// the batch's own split-k scratch.
class GemmBatch {
  public:
    static constexpr int kPartSlot = dev::kAbsSlot - 1;
    void clear() { g_.clear(); t_.clear(); tiles_ = 0; flops_ = 0; bytes_ = 0; red_.clear(); split_ = false; abs_ = false; }
    void bind(int slot, const double* base, size_t count) { slots_.bind(slot, base, count); }
    void group(double* C, int ldc, int m, int n, bool acc);
    void term(const double* A, int lda, bool tA, const double* B, int ldb, bool tB, int k, double alpha);
    void upload();
    void run() const;
    // mode 1: FP32, 2: BF16x3, on FP32 copies of the slots (the split-k
    // scratch is reused as FP32)
    void run_lo(const dev::BasesF& b, int mode) const;
    bool empty() const { return g_.empty(); }
    double flops() const { return flops_; }
    double bytes() const { return bytes_; }  // operand blocks read once, output blocks written once
    size_t nterms() const { return t_.size(); }

  private:
    SlotMap slots_;
    std::vector<dev::GemmGroup> g_;
    std::vector<dev::GemmTerm> t_;
    DevArr<char> buf_;  // groups, terms, tile -> group map and the split-k sums' lists, one copy
    const dev::GemmGroup* dg_ = nullptr;
    const dev::GemmTerm* dt_ = nullptr;
    const int* dtg_ = nullptr;
    int waves_ = 0;  // launch shape: waves per tile's workgroup (long k chains), 0: one wave per tile
    int tiles_ = 0;
    double flops_ = 0, bytes_ = 0;
    void upload_lists();
    AxpyBatch red_;  // sums split-k partials into the outputs
    DevBuf part_;
    bool split_ = false;
    bool abs_ = false;
};

// y = sum L (x) O (x) R applied to x (three grouped launches).  Slots:
// 0 left environment, 1 right environment, 2 x, 3 y, 4 U, 5 V.
struct EffOp {
    GemmBatch st1;
    AxpyBatch st2;
    GemmBatch st3;
    DevBuf U, V;
    double flops = 0, bytes = 0;
    void bind(int slot, const double* base, size_t count) {
        st1.bind(slot, base, count);
        st2.bind(slot, base, count);
        st3.bind(slot, base, count);
    }
    void run() const { st1.run(); st2.run(); st3.run(); }
    // Reduced precision: slots 0..3 as FP32 copies, U and V reused as FP32.
    void run_lo(dev::BasesF b, int mode) const {
        b.p[4] = reinterpret_cast<float*>(U.p);
        b.p[5] = reinterpret_cast<float*>(V.p);
        st1.run_lo(b, mode);
        st2.run_lo(b);
        st3.run_lo(b, mode);
    }
};

// Layout signature of the inputs a work list was built from; a cached list
// is reused while the signature is unchanged.
struct Sig {
    std::vector<int64_t> v;
    void add(int64_t x) { v.push_back(x); }
    bool operator==(const Sig& o) const { return v == o.v; }
    bool operator!=(const Sig& o) const { return v != o.v; }
};

struct StepRecord {
    double e2, discarded, t;
    int cg_iters;
};

struct SweepParams {
    int M1 = 16, n_sweeps = 0, max_sweeps = 10, cg_max_iter = 500, compute_e3 = 1;
    int precond = 0;  // 0 Jacobi, 1 learned block scaling
    // sigma inside CG: 0 FP64, 1 FP32, 2 BF16x3; with 1 or 2 the solve is
    // refined on FP64 residuals, each inner CG cutting its residual by inner_rel_tol
    int precision = 0;
    double e_tol = 1e-9, cg_rel_tol = 1e-10, inner_rel_tol = 0;
};

struct SweepResult {
    double e0 = 0, e2 = 0, e3 = 0, max_disc = 0, flops = 0, bytes = 0, t_total = 0;
    int n_sweeps = 0, n_steps = 0, flags = 0;
    long long cg_iters = 0, sigma_calls = 0;
    std::vector<double> e2_sweep;
    // host wall time per phase: two-site operators, work-list builds, local
    // solves (including waits on the device), truncation, environment updates,
    // next guess
    double t_phase[6] = {0, 0, 0, 0, 0, 0};
    long long plan_builds = 0, plan_hits = 0;  // work lists built / replayed from the plan caches
    long long sigma_lo_calls = 0, refinements = 0;  // reduced-precision applications, FP64 residual restarts
};

class Engine {
  public:
    Engine() = default;
    Engine(const Engine&) = delete;
    Engine& operator=(const Engine&) = delete;
    ~Engine();
    // inputs
    void set_integrals(int k_a, int k_v, std::vector<double> h, std::vector<double> eri);
    void set_partition(std::vector<double> eps);
    void set_psi0(int n_elec, int two_sz, const std::vector<Bond>& bonds, const std::vector<std::vector<double>>& sites);
    // Allowed electron counts per virtual site (bit c set: c electrons allowed); all 7 by default.
    void restrict_virtual(const std::vector<int>& masks);
    void set_psi1(const std::vector<Bond>& bonds, const std::vector<std::vector<double>>& sites);
    SweepResult sweep(const SweepParams& p);
    // Two-site DMRG for the lowest state of H_act in (n_elec, two_sz) on the
    // active sites, from a guess MPS; the result is loaded as Psi0.
    double ground_state(int n_elec, int two_sz, const std::vector<Bond>& bonds,
                        const std::vector<std::vector<double>>& sites, int M0, int n_sweeps, double e_tol);

    const std::vector<StepRecord>& trace() const { return trace_; }
    const Bond& bond(int which, int b) const;
    int n_sites() const { return n_; }
    int k_a() const { return k_a_; }
    int k_v() const { return k_v_; }
    void site_dense(int which, int i, std::vector<double>& out, int& Dl, int& Dr) const;

    bool have_ints = false, have_part = false, have_psi0 = false, have_psi1 = false;

    // learned preconditioner: parameters, training, harvested samples
    void precond_set(const float* p, int n);
    void precond_get(float* p, int n) const;
    float mlp_step(const float* X, const float* t, int n, float lr, bool update, float* grad);
    void set_harvest(bool on);
    const std::vector<float>& harvest_X() const { return hx_; }
    const std::vector<float>& harvest_t() const { return ht_; }

  private:
    // problem
    int k_a_ = 0, k_v_ = 0, n_ = 0, N_ = 0, tsz_ = 0;
    std::vector<double> h_, eri_, eps_;
    MPO mpo_h0_, mpo_v_, mpo_e3_;  // H0, V on Psi0, V within the Psi1 space (E3)
    double E0_ = 0;
    // states
    std::vector<Site> P0_;      // extended Psi0
    std::vector<Two> P0x_lay_;  // two-site layouts of Psi0 per window
    std::vector<DevBuf> P0x_;
    std::vector<Site> A_;       // Psi1
    std::vector<std::set<QN>> adm_;
    std::vector<int> virt_occ_;  // per virtual site, bit c: c electrons allowed
    void compute_adm();
    // environments
    std::vector<Env> LH_, RH_, LV_, RV_;
    // work buffers
    DevBuf T_, rho_, eigV_, eigw_, eigT_, eigS_, partials_, scal_;
    DevBuf x_, b_, d_, r_, z_, p_, q_, xg_;
    Two xlay_, last_lay_;
    double cg_tol2_ = 1e-20;
    int cg_max_ = 500;
    int precision_ = 0;
    double inner_tol2_ = 0;
    DevBuf lf_, rf_, pf_, qf_;  // FP32 copies: environments of the window, direction, product
    std::vector<StepRecord> trace_;
    SweepResult res_;
    std::vector<std::vector<double>> psi1_guess_;
    std::vector<Bond> psi1_bonds_;
    double t0_ = 0;
    bool gs_ = false;            // ground-state sweep (Davidson) instead of the linear solve
    double dav_tol_ = 1e-9;
    DevBuf dav_V_, dav_AV_;
    std::vector<StepRecord> gs_trace_;

    void build_mpos();
    // cached work lists per window (layout signature + device lists)
    struct EffPlan {
        Sig sig;
        EffOp op;
    };
    struct EnvPlan {
        Sig sig;
        Env lay;
        GemmBatch ga, gb;
        size_t tsz = 0;
    };
    struct DiagPlan {
        Sig sig;
        DevArr<dev::DiagGroup> dg;
        DevArr<dev::DiagTerm> dt;
        int ng = 0;
    };
    std::vector<std::unique_ptr<EffPlan>> eff_plans_[2];  // sigma, right-hand side
    std::vector<std::unique_ptr<EnvPlan>> env_plans_[4];  // LH, LV, RH, RV updates
    std::vector<std::unique_ptr<DiagPlan>> diag_plans_;
    void clear_plans();
    void ensure_partials();
    // learned preconditioner state (floats stored in double buffers)
    DevBuf mlp_, mlp_m_, mlp_v_, mlp_scr_, mlp_io_, pstats_, pfeat_, pscale_, pr0_, px0_;
    DevArr<dev::BlockRef> pblocks_;
    int mlp_step_ = 0, precond_ = 0;
    bool mlp_set_ = false, harvest_ = false;
    std::vector<float> hx_, ht_;
    int precond_blocks(const Two& lay);  // uploads the block list, returns its length
    void precond_apply(int i, int nb);
    void harvest_window(int i, int nb);
    double* hsc_ = nullptr;  // pinned host copies of the CG scalars, two slots
    // The eigensolver's failure flag is read back without waiting: a pinned
    // copy and an event, checked before the flag is reused and at the end of
    // the sweeps, so the host builds the next tensors while the kernel runs.
    int* eig_status_h_ = nullptr;
    void* eig_ev_ = nullptr;
    bool eig_pending_ = false;
    void check_eig_status();
    void drop_eig_status();
    void* ev_[2] = {nullptr, nullptr};
    EffOp& effop(int r, int i, const Env& L, const Env& R, const TwoOp& O, const Two& ket, const double* xket,
                 const Two& bra, double* ybra);
    void bind_env(GemmBatch& g, const Env& in, const Site& Abra, const Site& Aket, size_t tsz, const Env& out);
    bool env_cached(Env& out, const Env& in, const Site& Abra, const Site& Aket, const MPO& m, int i,
                    std::unique_ptr<EnvPlan>* plan, Sig& sig);
    // two-site operators per window, built once per MPO (which = 0: H0, 1: V)
    std::vector<std::unique_ptr<TwoOp>> twoop_cache_[2];
    const TwoOp& twoop(int which, int i);
    Env trivial_env(const Bond& bra, const Bond& ket) const;
    void env_left(Env& out, const Env& L, const Site& Abra, const Site& Aket, const MPO& m, int i,
                  std::unique_ptr<EnvPlan>* plan = nullptr);
    void env_right(Env& out, const Env& R, const Site& Abra, const Site& Aket, const MPO& m, int i,
                   std::unique_ptr<EnvPlan>* plan = nullptr);
    void build_effop(EffOp& op, const Env& L, const Env& R, const TwoOp& O, const Two& ket,
                     const double* xket, const Two& bra, double* ybra);
    void build_diag(int i, const Env& L, const Env& R, const TwoOp& O, const Two& lay, double* d, double shift);
    void contract_sites(const Site& A, const Site& B, const Two& lay, double* out);
    // zero: x vanishes (the local right-hand side was zero); no eigensolve
    double truncate(int i, bool forward, const Two& lay, const double* x, int M, Site& C, bool zero = false);
    bool x_zero_ = false;  // the last local solve returned x = 0
    void next_guess(int i, bool forward, Site& C);
    int solve(int i, double& e2);
    int davidson(int i, double& e);
    void start(const std::vector<Bond>& bonds, const std::vector<std::vector<double>>& sites, int M);
    double run_sweeps(int M, int n_sweeps, int max_sweeps, double e_tol);
    void upd_left(int i);
    void upd_right(int i);
    double e3_final(int window);
    void load_site(Site& s, const std::vector<double>& dense);
};

}  // namespace mpspt
