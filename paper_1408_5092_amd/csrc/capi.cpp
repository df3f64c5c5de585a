// extern "C" boundary of the library (declared in include/mpspt.h).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mpspt.h"
#include "engine.hpp"

struct mpspt_ctx {
    mpspt::dev::Stream* dev = nullptr;  // outlives eng: the engine's blocks go back to its pool
    mpspt::Engine eng;
    std::string err;
    int device = 0;
};

namespace {
using mpspt::Bond;
using mpspt::QN;

thread_local std::string g_err;

template <class F>
mpspt_status guard(mpspt_ctx* ctx, F&& f) {
    try {
        if (ctx) mpspt::dev::bind(ctx->dev);
        f();
        return MPSPT_OK;
    } catch (const mpspt::dev::Error& e) {
        (ctx ? ctx->err : g_err) = e.msg;
        return static_cast<mpspt_status>(e.code);
    } catch (const std::bad_alloc&) {
        (ctx ? ctx->err : g_err) = "host allocation failed";
        return MPSPT_E_NOMEM;
    } catch (const std::exception& e) {
        (ctx ? ctx->err : g_err) = e.what();
        return MPSPT_E_ARG;
    }
}

mpspt::dev::Error argerr(const std::string& m) { return mpspt::dev::Error{MPSPT_E_ARG, m}; }

void check_finite(const double* p, size_t n, const char* what) {
    if (!p) throw argerr(std::string(what) + " is null");
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) throw argerr(std::string(what) + " has a non-finite entry");
}

std::vector<double> eri_from_cholesky(int k, int nc, const double* B) {
    const size_t kk = (size_t)k * k;
    std::vector<double> eri(kk * kk, 0.0);
    for (int L = 0; L < nc; ++L) {
        const double* b = B + (size_t)L * kk;
        for (size_t pq = 0; pq < kk; ++pq) {
            const double v = b[pq];
            if (v == 0.0) continue;
            double* row = eri.data() + pq * kk;
            for (size_t rs = 0; rs < kk; ++rs) row[rs] += v * b[rs];
        }
    }
    return eri;
}

void check_ints(int k_a, int k_v, const double* h) {
    if (k_a < 1 || k_v < 1 || k_a + k_v > 128) throw argerr("need k_a >= 1, k_v >= 1, k_a + k_v <= 128");
    const int k = k_a + k_v;
    check_finite(h, (size_t)k * k, "h");
    for (int p = 0; p < k; ++p)
        for (int q = 0; q < p; ++q)
            if (std::fabs(h[p * k + q] - h[q * k + p]) > 1e-12 * (1 + std::fabs(h[p * k + q])))
                throw argerr("h is not symmetric");
}

std::vector<Bond> read_bonds(int nb, const int32_t* dims, const int32_t* qn) {
    if (!dims || !qn) throw argerr("bond arrays are null");
    std::vector<Bond> out(nb);
    size_t pos = 0;
    for (int b = 0; b < nb; ++b) {
        if (dims[b] < 1) throw argerr("bond dimension < 1");
        Bond& B = out[b];
        for (int i = 0; i < dims[b]; ++i, ++pos) {
            QN q{qn[2 * pos], qn[2 * pos + 1]};
            if (B.q.empty() || B.q.back() != q) {
                if (!B.q.empty() && !(B.q.back() < q))
                    throw mpspt::dev::Error{MPSPT_E_QN, "bond labels must be grouped in ascending (N, 2Sz) order"};
                B.q.push_back(q);
                B.d.push_back(0);
            }
            B.d.back()++;
        }
    }
    return out;
}

std::vector<std::vector<double>> read_sites(const std::vector<Bond>& b, const double* const* site) {
    if (!site) throw argerr("site pointer array is null");
    std::vector<std::vector<double>> out;
    for (size_t i = 0; i + 1 < b.size(); ++i) {
        size_t n = (size_t)b[i].total() * 4 * b[i + 1].total();
        check_finite(site[i], n, "site tensor");
        out.emplace_back(site[i], site[i] + n);
    }
    return out;
}
}  // namespace

extern "C" {

mpspt_status mpspt_create(int hip_device, void* hip_stream, mpspt_ctx** out) {
    if (!out) return MPSPT_E_ARG;
    *out = nullptr;
    return guard(nullptr, [&] {
        mpspt::dev::Stream* s = mpspt::dev::stream_create(hip_device, hip_stream);
        mpspt::dev::bind(s);
        mpspt_ctx* c = nullptr;
        try {
            c = new mpspt_ctx();
        } catch (...) {
            mpspt::dev::stream_destroy(s);
            throw;
        }
        c->dev = s;
        c->device = hip_device;
        *out = c;
    });
}

void mpspt_destroy(mpspt_ctx* ctx) {
    if (!ctx) return;
    try {
        mpspt::dev::bind(ctx->dev);
        mpspt::dev::Stream* s = ctx->dev;
        delete ctx;                       // the engine's device blocks go back to the pool
        mpspt::dev::stream_destroy(s);    // and the pool to the runtime
    } catch (...) {
    }
}

const char* mpspt_last_error(const mpspt_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

mpspt_status mpspt_load_integrals(mpspt_ctx* ctx, int32_t k_a, int32_t k_v, const double* h, int32_t n_chol,
                                  const double* B) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        check_ints(k_a, k_v, h);
        const int k = k_a + k_v;
        if (n_chol < 1) throw argerr("n_chol < 1");
        check_finite(B, (size_t)n_chol * k * k, "B");
        std::vector<double> hv(h, h + (size_t)k * k);
        ctx->eng.set_integrals(k_a, k_v, std::move(hv), eri_from_cholesky(k, n_chol, B));
    });
}

mpspt_status mpspt_load_integrals_eri(mpspt_ctx* ctx, int32_t k_a, int32_t k_v, const double* h, const double* eri) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        check_ints(k_a, k_v, h);
        const size_t k = k_a + k_v;
        check_finite(eri, k * k * k * k, "eri");
        std::vector<double> hv(h, h + k * k);
        ctx->eng.set_integrals(k_a, k_v, std::move(hv), std::vector<double>(eri, eri + k * k * k * k));
    });
}

mpspt_status mpspt_load_h0_partition(mpspt_ctx* ctx, int32_t kind, const double* eps_virt) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        if (kind != 0) throw argerr("only the Dyall partition (kind 0) is implemented");
        if (!ctx->eng.have_ints) throw mpspt::dev::Error{MPSPT_E_STATE, "load integrals first"};
        const int kv = ctx->eng.k_v();
        check_finite(eps_virt, kv, "eps_virt");
        ctx->eng.set_partition(std::vector<double>(eps_virt, eps_virt + kv));
    });
}

mpspt_status mpspt_load_psi0(mpspt_ctx* ctx, int32_t n_elec, int32_t two_sz, const int32_t* bond_dims,
                             const int32_t* bond_qn, const double* const* site) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        if (!ctx->eng.have_part) throw mpspt::dev::Error{MPSPT_E_STATE, "load integrals and the H0 partition first"};
        int ka = ctx->eng.k_a();
        auto b = read_bonds(ka + 1, bond_dims, bond_qn);
        ctx->eng.set_psi0(n_elec, two_sz, b, read_sites(b, site));
    });
}

mpspt_status mpspt_ground_state(mpspt_ctx* ctx, int32_t n_elec, int32_t two_sz, const int32_t* bond_dims,
                                const int32_t* bond_qn, const double* const* site, int32_t M0, int32_t n_sweeps,
                                double e_tol, double* e_out) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        if (!ctx->eng.have_part) throw mpspt::dev::Error{MPSPT_E_STATE, "load integrals and the H0 partition first"};
        if (n_sweeps < 0 || n_sweeps > 64) throw argerr("n_sweeps must be in [0, 64]");
        int ka = ctx->eng.k_a();
        auto b = read_bonds(ka + 1, bond_dims, bond_qn);
        double e = ctx->eng.ground_state(n_elec, two_sz, b, read_sites(b, site), M0, n_sweeps,
                                         e_tol > 0 ? e_tol : 1e-10);
        if (e_out) *e_out = e;
    });
}

mpspt_status mpspt_restrict_virtual(mpspt_ctx* ctx, const int32_t* masks) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        if (!ctx->eng.have_ints) throw mpspt::dev::Error{MPSPT_E_STATE, "load integrals first"};
        const int kv = ctx->eng.k_v();
        std::vector<int> m(kv, 7);
        if (masks) m.assign(masks, masks + kv);
        ctx->eng.restrict_virtual(m);
    });
}

mpspt_status mpspt_load_psi1_guess(mpspt_ctx* ctx, const int32_t* bond_dims, const int32_t* bond_qn,
                                   const double* const* site) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        if (!ctx->eng.have_psi0) throw mpspt::dev::Error{MPSPT_E_STATE, "load Psi0 first"};
        int n = ctx->eng.n_sites();
        auto b = read_bonds(n + 1, bond_dims, bond_qn);
        ctx->eng.set_psi1(b, read_sites(b, site));
    });
}

mpspt_status mpspt_sweep(mpspt_ctx* ctx, const mpspt_sweep_params* params, mpspt_result* out) {
    if (!ctx || !params || !out) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        mpspt::SweepParams p;
        p.M1 = params->M1;
        p.n_sweeps = params->n_sweeps;
        p.max_sweeps = params->max_sweeps > 0 ? std::min(params->max_sweeps, 64) : 10;
        p.e_tol = params->e_tol > 0 ? params->e_tol : 1e-9;
        p.cg_rel_tol = params->cg_rel_tol > 0 ? params->cg_rel_tol : 1e-10;
        p.cg_max_iter = params->cg_max_iter > 0 ? params->cg_max_iter : 500;
        p.compute_e3 = params->compute_e3;
        p.precond = params->precond;
        p.precision = params->precision;
        p.inner_rel_tol = params->inner_rel_tol;
        if (p.n_sweeps > 64 || p.n_sweeps < 0) throw argerr("n_sweeps must be in [0, 64]");
        mpspt::SweepResult r = ctx->eng.sweep(p);
        std::memset(out, 0, sizeof(*out));
        out->e0 = r.e0;
        out->e2 = r.e2;
        out->e3 = r.e3;
        out->n_sweeps_done = r.n_sweeps;
        out->n_steps = r.n_steps;
        for (size_t i = 0; i < r.e2_sweep.size() && i < 64; ++i) out->e2_sweep[i] = r.e2_sweep[i];
        out->max_discarded = r.max_disc;
        out->cg_iters = r.cg_iters;
        out->sigma_calls = r.sigma_calls;
        out->sigma_flops = r.flops;
        out->sigma_bytes = r.bytes;
        out->t_total_s = r.t_total;
        out->flags = r.flags;
        for (int k = 0; k < 6; ++k) out->t_phase[k] = r.t_phase[k];
        out->plan_builds = r.plan_builds;
        out->plan_hits = r.plan_hits;
        out->sigma_lo_calls = r.sigma_lo_calls;
        out->refinements = r.refinements;
    });
}

mpspt_status mpspt_set_tuning(mpspt_ctx* ctx, int32_t wide_chunks, int32_t kseg_min, int32_t kseg_div,
                              int32_t split_waves) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        if (wide_chunks < 1 || kseg_min < 16 || kseg_div < 1) throw argerr("tuning values out of range");
        if (split_waves != 4 && split_waves != 8 && split_waves != 16) throw argerr("split_waves must be 4, 8 or 16");
        mpspt::dev::Tuning& t = mpspt::dev::tuning();
        t.wide_chunks = wide_chunks;
        t.kseg_min = kseg_min;
        t.kseg_div = kseg_div;
        t.split_waves = split_waves;
    });
}

mpspt_status mpspt_get_tuning(mpspt_ctx* ctx, int32_t* wide_chunks, int32_t* kseg_min, int32_t* kseg_div,
                              int32_t* split_waves) {
    if (!ctx || !wide_chunks || !kseg_min || !kseg_div || !split_waves) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        const mpspt::dev::Tuning& t = mpspt::dev::tuning();
        *wide_chunks = t.wide_chunks;
        *kseg_min = t.kseg_min;
        *kseg_div = t.kseg_div;
        *split_waves = t.split_waves;
    });
}

mpspt_status mpspt_profile(mpspt_ctx* ctx, int32_t enable) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        if (enable < 0) throw argerr("enable must be >= 0");
        mpspt::dev::profile_enable(enable);
    });
}

mpspt_status mpspt_precond_set(mpspt_ctx* ctx, const float* params, int32_t n) {
    if (!ctx || !params) return MPSPT_E_ARG;
    return guard(ctx, [&] { ctx->eng.precond_set(params, n); });
}

mpspt_status mpspt_precond_get(mpspt_ctx* ctx, float* params, int32_t n) {
    if (!ctx || !params) return MPSPT_E_ARG;
    return guard(ctx, [&] { ctx->eng.precond_get(params, n); });
}

mpspt_status mpspt_mlp_grad(mpspt_ctx* ctx, const float* X, const float* t, int32_t n, float* grad, float* loss) {
    if (!ctx || !X || !t || !loss) return MPSPT_E_ARG;
    return guard(ctx, [&] { *loss = ctx->eng.mlp_step(X, t, n, 0.0f, false, grad); });
}

mpspt_status mpspt_mlp_train_step(mpspt_ctx* ctx, const float* X, const float* t, int32_t n, float lr,
                                  float* loss) {
    if (!ctx || !X || !t) return MPSPT_E_ARG;
    if (!(lr > 0.0f)) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        const float l = ctx->eng.mlp_step(X, t, n, lr, true, nullptr);
        if (loss) *loss = l;
    });
}

mpspt_status mpspt_harvest(mpspt_ctx* ctx, int32_t enable) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(ctx, [&] { ctx->eng.set_harvest(enable != 0); });
}

mpspt_status mpspt_harvest_get(mpspt_ctx* ctx, int64_t cap, float* X, float* t, int64_t* n_out) {
    if (!ctx || !n_out) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        const auto& hx = ctx->eng.harvest_X();
        const auto& ht = ctx->eng.harvest_t();
        *n_out = (int64_t)ht.size();
        if (cap <= 0) return;
        if (!X || !t || cap < (int64_t)ht.size()) throw argerr("output smaller than the harvested sample count");
        std::copy(hx.begin(), hx.end(), X);
        std::copy(ht.begin(), ht.end(), t);
    });
}

mpspt_status mpspt_kernel_stats(mpspt_ctx* ctx, int32_t kind, double* seconds, int64_t* launches, double* flops,
                                double* bytes, int64_t* launches_all) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        if (kind < 0 || kind >= mpspt::dev::K_COUNT) throw argerr("unknown kernel kind");
        mpspt::dev::KernelStats s = mpspt::dev::profile_stats(kind);
        if (seconds) *seconds = s.seconds;
        if (launches) *launches = s.launches;
        if (flops) *flops = s.flops;
        if (bytes) *bytes = s.bytes;
        if (launches_all) *launches_all = s.launches_all;
    });
}

mpspt_status mpspt_get_trace(const mpspt_ctx* ctx, int32_t cap, double* e2, int32_t* cg_iters, double* discarded,
                             double* t_s, int32_t* n_out) {
    if (!ctx) return MPSPT_E_ARG;
    const auto& t = ctx->eng.trace();
    if (n_out) *n_out = (int32_t)t.size();
    for (int32_t i = 0; i < cap && i < (int32_t)t.size(); ++i) {
        if (e2) e2[i] = t[i].e2;
        if (cg_iters) cg_iters[i] = t[i].cg_iters;
        if (discarded) discarded[i] = t[i].discarded;
        if (t_s) t_s[i] = t[i].t;
    }
    return MPSPT_OK;
}

mpspt_status mpspt_get_bond(const mpspt_ctx* ctx, int32_t which, int32_t bond, int32_t cap, int32_t* qn_dims,
                            int32_t* n_out) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(const_cast<mpspt_ctx*>(ctx), [&] {
        const Bond& b = ctx->eng.bond(which, bond);
        if (n_out) *n_out = (int32_t)b.q.size();
        for (int32_t i = 0; i < cap && i < (int32_t)b.q.size(); ++i) {
            qn_dims[3 * i] = b.q[i].n;
            qn_dims[3 * i + 1] = b.q[i].s;
            qn_dims[3 * i + 2] = b.d[i];
        }
    });
}

mpspt_status mpspt_get_site(mpspt_ctx* ctx, int32_t which, int32_t site, size_t cap, double* dense, int32_t* dims) {
    if (!ctx) return MPSPT_E_ARG;
    return guard(ctx, [&] {
        std::vector<double> v;
        int Dl = 0, Dr = 0;
        ctx->eng.site_dense(which, site, v, Dl, Dr);
        if (dims) { dims[0] = Dl; dims[1] = Dr; }
        if (dense) {
            if (cap < v.size()) throw argerr("output buffer too small");
            std::memcpy(dense, v.data(), v.size() * sizeof(double));
        }
    });
}

mpspt_status mpspt_mpo_dims(int32_t k_a, int32_t k_v, const double* h, const double* eri, const double* eps_virt,
                            int32_t which, int32_t* dims, int32_t cap) {
    return guard(nullptr, [&] {
        check_ints(k_a, k_v, h);
        const size_t k = k_a + k_v;
        check_finite(eri, k * k * k * k, "eri");
        check_finite(eps_virt, k_v, "eps_virt");
        if (which < 0 || which > 3) throw argerr("which must be 0, 1, 2 or 3");
        mpspt::OpKind kind = which == 0   ? mpspt::OpKind::H0
                             : which == 1 ? mpspt::OpKind::VPsi0
                             : which == 2 ? mpspt::OpKind::VFull
                                          : mpspt::OpKind::VPsi1;
        mpspt::MPO m = mpspt::build_mpo(kind, k_a, k_v, std::vector<double>(h, h + k * k),
                                        std::vector<double>(eri, eri + k * k * k * k),
                                        std::vector<double>(eps_virt, eps_virt + k_v));
        for (int32_t i = 0; i < cap && i < (int32_t)m.dims.size(); ++i) dims[i] = m.dims[i];
    });
}

mpspt_status mpspt_mpo_dense(int32_t k_a, int32_t k_v, const double* h, const double* eri, const double* eps_virt,
                             int32_t which, double* out, size_t cap) {
    return guard(nullptr, [&] {
        check_ints(k_a, k_v, h);
        const int n = k_a + k_v;
        if (n > 6) throw argerr("dense MPO contraction is limited to 6 sites");
        const size_t k = n;
        check_finite(eri, k * k * k * k, "eri");
        check_finite(eps_virt, k_v, "eps_virt");
        if (which < 0 || which > 3) throw argerr("which must be 0, 1, 2 or 3");
        size_t dim = 1;
        for (int i = 0; i < n; ++i) dim *= 4;
        if (!out || cap < dim * dim) throw argerr("output buffer too small");
        mpspt::OpKind kind = which == 0   ? mpspt::OpKind::H0
                             : which == 1 ? mpspt::OpKind::VPsi0
                             : which == 2 ? mpspt::OpKind::VFull
                                          : mpspt::OpKind::VPsi1;
        mpspt::MPO m = mpspt::build_mpo(kind, k_a, k_v, std::vector<double>(h, h + k * k),
                                        std::vector<double>(eri, eri + k * k * k * k),
                                        std::vector<double>(eps_virt, eps_virt + k_v));
        // T[c] = left part of channel c as a dense (4^b x 4^b) matrix
        std::vector<std::vector<double>> T(1, std::vector<double>(1, 1.0));
        size_t d = 1;
        for (int i = 0; i < n; ++i) {
            std::vector<std::vector<double>> N(m.dims[i + 1]);
            const size_t d2 = d * 4;
            for (const auto& e : m.W[i]) {
                const auto& A = T[e.cin];
                if (A.empty()) continue;
                auto& C = N[e.cout];
                if (C.empty()) C.assign(d2 * d2, 0.0);
                for (size_t a = 0; a < d; ++a)
                    for (size_t b = 0; b < d; ++b) {
                        const double v = A[a * d + b];
                        if (v == 0.0) continue;
                        for (int s = 0; s < 4; ++s)
                            for (int t = 0; t < 4; ++t) C[(a * 4 + s) * d2 + b * 4 + t] += v * e.m[s * 4 + t];
                    }
            }
            T.swap(N);
            d = d2;
        }
        std::memset(out, 0, dim * dim * sizeof(double));
        if (!T.empty() && !T[0].empty()) std::memcpy(out, T[0].data(), dim * dim * sizeof(double));
    });
}

}  // extern "C"
