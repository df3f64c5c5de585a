// Two-site MPS-PT sweep (host driver).
//
// Window (i, i+1) of Psi1 is optimised with the rest fixed: the partial
// derivative of the Hylleraas functional with respect to the two-site tensor
// x vanishes when (H0_eff - E0) x = -b with b = <local basis|V|Psi0>; this is
// solved by Jacobi-preconditioned CG, its functional value x.(A x) + 2 x.b is
// the running E2, and x is split by the reduced density matrix of the half
// being renormalised, keeping the M1 most significant states.  Environments
// of <Psi1|H0|Psi1> and of the mixed <Psi1|V|Psi0> are carried along.
#include "engine.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <unordered_map>

#include "../../include/mpspt.h"

namespace mpspt {

namespace {
dev::Error err(int code, const std::string& m) { return dev::Error{code, m}; }
constexpr int kTile = dev::GEMM_TILE;

// Output blocks of an environment update keyed by (channel, bra sector) and
// visited in ascending key order.
template <class Tm>
class OutTable {
  public:
    OutTable(int nch, int nbra) : nbra_(nbra), ik_((size_t)nch * nbra, -1), terms_((size_t)nch * nbra) {}
    void add(int w, int ib, int ik, const Tm& t) {
        const size_t s = (size_t)w * nbra_ + ib;
        if (ik_[s] < 0) {
            ik_[s] = ik;
            used_.push_back(s);
        } else if (ik_[s] != ik) {
            throw err(MPSPT_E_QN, "inconsistent channel quantum numbers");
        }
        terms_[s].push_back(t);
    }
    template <class F>
    void each(F&& f) {
        std::sort(used_.begin(), used_.end());
        for (size_t s : used_) f((int)(s / nbra_), (int)(s % nbra_), ik_[s], terms_[s]);
    }

  private:
    size_t nbra_;
    std::vector<int> ik_;
    std::vector<std::vector<Tm>> terms_;
    std::vector<size_t> used_;
};
}  // namespace

// ------------------------------------------------------------- storage
void DevBuf::reset() {
    if (p) dev::release(p);  // stream-ordered pool: no wait needed
    p = nullptr;
    n = 0;
}
void DevBuf::alloc(size_t c) {
    reset();
    if (c) p = static_cast<double*>(dev::alloc(c * sizeof(double)));
    n = c;
}
void DevBuf::ensure(size_t c) {
    if (c > n) alloc(c + c / 4 + 64);
}

int Bond::find(QN x) const {
    auto it = std::lower_bound(q.begin(), q.end(), x);
    if (it == q.end() || *it != x) return -1;
    return (int)(it - q.begin());
}
int Bond::total() const {
    int t = 0;
    for (int v : d) t += v;
    return t;
}

Site make_site(const Bond& L, const Bond& R) {
    Site s;
    s.L = L;
    s.R = R;
    const int nl = (int)L.q.size();
    s.idx.assign((size_t)nl * 4, -1);
    s.pw.assign(nl, 0);
    s.po.assign(nl, 0);
    s.by_jr.assign(R.q.size(), {});
    size_t off = 0;
    for (int il = 0; il < nl; ++il) {
        s.po[il] = off;
        int col = 0;
        for (int st = 0; st < 4; ++st) {
            int jr = R.find(L.q[il] + site_dq(st));
            if (jr < 0) continue;
            s.idx[il * 4 + st] = (int)s.blk.size();
            s.by_jr[jr].push_back((int)s.blk.size());
            s.blk.push_back({il, st, jr, L.d[il], R.d[jr], col});
            col += R.d[jr];
        }
        s.pw[il] = col;
        off += (size_t)L.d[il] * col;
    }
    s.size = off;
    s.data.alloc(off);
    return s;
}

Two make_two(const Bond& L, const Bond& R, const std::set<QN>* mid_ok) {
    Two t;
    t.L = L;
    t.R = R;
    const int nl = (int)L.q.size();
    t.idx.assign((size_t)nl * 16, -1);
    t.pw.assign(nl, 0);
    t.po.assign(nl, 0);
    size_t off = 0;
    for (int il = 0; il < nl; ++il) {
        t.po[il] = off;
        int col = 0;
        for (int s1 = 0; s1 < 4; ++s1) {
            QN mid = L.q[il] + site_dq(s1);
            if (mid_ok && !mid_ok->count(mid)) continue;
            for (int s2 = 0; s2 < 4; ++s2) {
                int jr = R.find(mid + site_dq(s2));
                if (jr < 0) continue;
                t.idx[(il * 4 + s1) * 4 + s2] = (int)t.blk.size();
                t.blk.push_back({il, s1, s2, jr, L.d[il], R.d[jr], col});
                col += R.d[jr];
            }
        }
        t.pw[il] = col;
        off += (size_t)L.d[il] * col;
    }
    t.size = off;
    return t;
}

void Env::index() {
    idx.assign((size_t)nch * bra.q.size(), -1);
    by_w.assign(nch, {});
    by_ib.assign(bra.q.size(), {});
    for (size_t b = 0; b < blk.size(); ++b) {
        idx[(size_t)blk[b].w * bra.q.size() + blk[b].ib] = (int)b;
        by_w[blk[b].w].push_back((int)b);
    }
    for (int w = 0; w < nch; ++w)
        for (size_t ib = 0; ib < bra.q.size(); ++ib) {
            int b = idx[(size_t)w * bra.q.size() + ib];
            if (b >= 0) by_ib[ib].push_back(b);
        }
}

void Env::copy_layout(const Env& o) {
    nch = o.nch;
    bra = o.bra;
    ket = o.ket;
    blk = o.blk;
    idx = o.idx;
    by_w = o.by_w;
    by_ib = o.by_ib;
    dq = o.dq;
    size = o.size;
}

namespace {
// every field separately: equal signatures mean equal layouts
void sig_bond(Sig& g, const Bond& b) {
    g.add((int64_t)b.q.size());
    for (size_t k = 0; k < b.q.size(); ++k) {
        g.add(b.q[k].n);
        g.add(b.q[k].s);
        g.add(b.d[k]);
    }
}
void sig_env(Sig& g, const Env& e) {
    g.add(e.nch);
    sig_bond(g, e.bra);
    sig_bond(g, e.ket);
    g.add((int64_t)e.blk.size());
    for (const auto& b : e.blk) {
        g.add(b.w);
        g.add(b.ib);
        g.add(b.ik);
        g.add((int64_t)b.off);
    }
}
void sig_site(Sig& g, const Site& a) {
    sig_bond(g, a.L);
    sig_bond(g, a.R);
    g.add((int64_t)a.blk.size());
    for (const auto& b : a.blk) {
        g.add(b.il);
        g.add(b.s);
        g.add(b.jr);
        g.add(b.col);
    }
    for (size_t k = 0; k < a.po.size(); ++k) {
        g.add((int64_t)a.po[k]);
        g.add(a.pw[k]);
    }
}
void sig_two(Sig& g, const Two& a) {
    sig_bond(g, a.L);
    sig_bond(g, a.R);
    g.add((int64_t)a.blk.size());
    for (const auto& b : a.blk) {
        g.add(b.il);
        g.add(b.s1);
        g.add(b.s2);
        g.add(b.jr);
        g.add(b.col);
    }
    for (size_t k = 0; k < a.po.size(); ++k) {
        g.add((int64_t)a.po[k]);
        g.add(a.pw[k]);
    }
}
}  // namespace

TwoOp make_twoop(const MPO& m, int i) {
    TwoOp O;
    O.nin = m.dims[i];
    O.nout = m.dims[i + 2];
    const auto& W1 = m.W[i];
    const auto& W2 = m.W[i + 1];
    // W2 entries grouped by output channel, each group in (middle channel, entry) order
    std::vector<std::vector<int>> by_out(O.nout);
    for (size_t e = 0; e < W2.size(); ++e) by_out[W2[e].cout].push_back((int)e);
    std::vector<std::vector<int>> in_mid(m.dims[i + 1]);
    for (size_t e = 0; e < W1.size(); ++e) in_mid[W1[e].cout].push_back((int)e);
    // dense accumulator over (s1' s2', w, s1 s2) for one output channel w'
    const size_t row = (size_t)O.nin * 16;
    std::vector<double> acc(16 * row, 0.0);
    std::vector<char> hit(16 * row, 0);
    std::vector<size_t> touched;
    std::vector<size_t> by_sp[16];
    O.by_out.assign((size_t)O.nout * 16, {});
    for (int wo = 0; wo < O.nout; ++wo) {
        auto& list = by_out[wo];
        std::stable_sort(list.begin(), list.end(), [&](int a, int b) { return W2[a].cin < W2[b].cin; });
        touched.clear();
        for (int b : list) {
            const MPOEntry& e2 = W2[b];
            for (int a : in_mid[e2.cin]) {
                const MPOEntry& e1 = W1[a];
                for (int s1p = 0; s1p < 4; ++s1p)
                    for (int s1 = 0; s1 < 4; ++s1) {
                        const double v1 = e1.m[s1p * 4 + s1];
                        if (v1 == 0.0) continue;
                        for (int s2p = 0; s2p < 4; ++s2p)
                            for (int s2 = 0; s2 < 4; ++s2) {
                                const double v2 = e2.m[s2p * 4 + s2];
                                if (v2 == 0.0) continue;
                                const size_t k = (size_t)(s1p * 4 + s2p) * row + (size_t)e1.cin * 16 + s1 * 4 + s2;
                                if (!hit[k]) {
                                    hit[k] = 1;
                                    touched.push_back(k);
                                }
                                acc[k] += v1 * v2;
                            }
                    }
            }
        }
        // ascending k: by output local state sp (k / row), then within it
        for (auto& bk : by_sp) bk.clear();
        for (size_t k : touched) by_sp[k / row].push_back(k);
        for (int sp = 0; sp < 16; ++sp) {
            std::sort(by_sp[sp].begin(), by_sp[sp].end());
            for (size_t k : by_sp[sp]) {
                const int rest = (int)(k - (size_t)sp * row);
                if (acc[k] != 0.0)
                    O.by_out[(size_t)wo * 16 + sp].push_back({rest / 16, (rest % 16) / 4, rest % 4, acc[k]});
                acc[k] = 0.0;
                hit[k] = 0;
            }
        }
    }
    return O;
}

// ---------------------------------------------------------- work lists
void Packer::upload(DevArr<char>& buf) const {
    constexpr size_t kImageMax = 256 << 10;
    buf.ensure(size_);
    if (size_ <= kImageMax) {
        std::vector<char> h(size_);
        for (const Sec& c : sec_) std::memcpy(h.data() + c.off, c.p, c.n);
        buf.upload(h);
        return;
    }
    for (const Sec& c : sec_) dev::h2d(buf.p + c.off, c.p, c.n);
}

void SlotMap::ref(const double* p, int8_t& slot, int64_t& off) const {
    // consecutive references usually fall in the same buffer; slots do not overlap
    if (base_[last_] && p >= base_[last_] && p < base_[last_] + cnt_[last_]) {
        slot = (int8_t)last_;
        off = p - base_[last_];
        return;
    }
    for (int k = 0; k < dev::kAbsSlot; ++k)
        if (base_[k] && p >= base_[k] && p < base_[k] + cnt_[k]) {
            last_ = k;
            slot = (int8_t)k;
            off = p - base_[k];
            return;
        }
    slot = (int8_t)dev::kAbsSlot;
    off = (int64_t)(reinterpret_cast<uintptr_t>(p) / sizeof(double));
}
dev::Bases SlotMap::bases() const {
    dev::Bases b;
    for (int k = 0; k < dev::kSlots; ++k) b.p[k] = const_cast<double*>(base_[k]);
    b.p[dev::kAbsSlot] = nullptr;
    return b;
}

void GemmBatch::group(double* C, int ldc, int m, int n, bool acc) {
    dev::GemmGroup g{};
    g.term0 = (int)t_.size();
    if (m <= 0 || n <= 0) {
        g.tile0 = -1;  // placeholder, dropped
        g_.push_back(g);
        return;
    }
    slots_.ref(C, g.sc, g.oc);
    if (g.sc == dev::kAbsSlot) abs_ = true;
    g.ldc = ldc;
    g.m = m;
    g.n = n;
    g.accumulate = acc ? 1 : 0;
    g.tile0 = tiles_;
    tiles_ += ((m + kTile - 1) / kTile) * ((n + kTile - 1) / kTile);
    g_.push_back(g);
    bytes_ += 8.0 * m * n * (acc ? 2 : 1);
}
void GemmBatch::term(const double* A, int lda, bool tA, const double* B, int ldb, bool tB, int k, double alpha) {
    dev::GemmGroup& g = g_.back();
    if (g.tile0 < 0 || k <= 0 || alpha == 0.0) return;
    dev::GemmTerm t{};
    slots_.ref(A, t.sa, t.oa);
    slots_.ref(B, t.sb, t.ob);
    if (t.sa == dev::kAbsSlot || t.sb == dev::kAbsSlot) abs_ = true;
    t.alpha = alpha;
    t.lda = lda;
    t.ldb = ldb;
    t.k = k;
    t.transA = tA ? 1 : 0;
    t.transB = tB ? 1 : 0;
    t_.push_back(t);
    ++g.nterms;
    flops_ += 2.0 * g.m * g.n * k;
    bytes_ += 8.0 * ((double)g.m * k + (double)k * g.n);
}
// Groups whose summed k is long compared with the launch's work are split
// into segments (at term boundaries, or inside a long term) that write
// partial products to the batch's scratch; a grouped axpy then adds the
// segments into C in order, so the result stays deterministic.
void GemmBatch::upload() {
    if (split_) {  // already laid out
        upload_lists();
        return;
    }
    split_ = true;
    std::vector<dev::GemmGroup> live;
    std::vector<long> ksum;
    live.reserve(g_.size());
    double work = 0;
    for (auto& g : g_) {
        if (g.tile0 < 0) continue;
        long K = 0;
        for (int t = 0; t < g.nterms; ++t) K += t_[g.term0 + t].k;
        const int tl = ((g.m + kTile - 1) / kTile) * ((g.n + kTile - 1) / kTile);
        work += (double)tl * K;
        live.push_back(g);
        ksum.push_back(K);
    }
    const dev::Tuning& tu = dev::tuning();
    const long kseg = std::max<long>(tu.kseg_min, (long)(work / (double)tu.kseg_div));
    size_t psz = 0;
    std::vector<int> nseg(live.size(), 1);
    for (size_t gi = 0; gi < live.size(); ++gi)
        if (ksum[gi] > kseg) {
            nseg[gi] = (int)((ksum[gi] + kseg - 1) / kseg);
            psz += (size_t)nseg[gi] * live[gi].m * live[gi].n;
        }
    part_.ensure(std::max<size_t>(psz, 1));
    red_.clear();
    if (psz == 0 && live.size() == g_.size()) {
        // nothing to split or drop: the lists are already laid out (groups
        // in order, terms contiguous per group, tiles numbered in order)
        upload_lists();
        return;
    }
    std::vector<dev::GemmGroup> gs;
    std::vector<dev::GemmTerm> ts;
    gs.reserve(live.size());
    ts.reserve(t_.size());
    int tiles = 0;
    int64_t poff = 0;
    for (size_t gi = 0; gi < live.size(); ++gi) {
        const auto& g = live[gi];
        const int tl = ((g.m + kTile - 1) / kTile) * ((g.n + kTile - 1) / kTile);
        if (nseg[gi] == 1) {
            dev::GemmGroup c = g;
            c.term0 = (int)ts.size();
            c.tile0 = tiles;
            tiles += tl;
            ts.insert(ts.end(), t_.begin() + g.term0, t_.begin() + g.term0 + g.nterms);
            gs.push_back(c);
            continue;
        }
        const long per = (ksum[gi] + nseg[gi] - 1) / nseg[gi];
        red_.group_ref(g.sc, g.oc, g.ldc, g.m, g.n, g.accumulate != 0);
        auto fresh = [&]() {
            dev::GemmGroup c{};
            c.sc = (int8_t)kPartSlot;
            c.oc = poff;
            c.ldc = g.n;
            c.m = g.m;
            c.n = g.n;
            c.term0 = (int)ts.size();
            c.tile0 = tiles;
            return c;
        };
        dev::GemmGroup cur = fresh();
        long used = 0;
        auto close = [&]() {
            if (cur.nterms == 0) return;
            gs.push_back(cur);
            tiles += tl;
            red_.term_ref((int8_t)kPartSlot, cur.oc, g.n, false, 1.0);
            poff += (int64_t)g.m * g.n;
            cur = fresh();
            used = 0;
        };
        for (int t = 0; t < g.nterms; ++t) {
            const dev::GemmTerm tm = t_[g.term0 + t];
            int k0 = 0;
            while (k0 < tm.k) {
                const int take = (int)std::min<long>(tm.k - k0, per - used);
                dev::GemmTerm sub = tm;
                sub.oa = tm.oa + (int64_t)k0 * (tm.transA ? tm.lda : 1);
                sub.ob = tm.ob + (int64_t)k0 * (tm.transB ? 1 : tm.ldb);
                sub.k = take;
                ts.push_back(sub);
                ++cur.nterms;
                used += take;
                k0 += take;
                if (used >= per) close();
            }
        }
        close();
    }
    g_.swap(gs);
    t_.swap(ts);
    tiles_ = tiles;
    upload_lists();
}
void GemmBatch::upload_lists() {
    std::vector<int> tg((size_t)std::max(tiles_, 0));
    long maxc = 0;
    for (size_t gi = 0; gi < g_.size(); ++gi) {
        const auto& g = g_[gi];
        const int tl = ((g.m + kTile - 1) / kTile) * ((g.n + kTile - 1) / kTile);
        for (int t = 0; t < tl; ++t) tg[(size_t)g.tile0 + t] = (int)gi;
        long kc = 0;
        for (int t = 0; t < g.nterms; ++t) kc += (t_[g.term0 + t].k + 15) / 16;
        maxc = std::max(maxc, kc);
    }
    // launch shape: one workgroup per tile, k spread over its waves, once some
    // tile of the list has a long enough k chain
    waves_ = maxc >= dev::tuning().wide_chunks ? dev::tuning().split_waves : 0;
    Packer pk;
    const size_t og = pk.add(g_), ot = pk.add(t_), otg = pk.add(tg);
    red_.pack(pk);
    pk.upload(buf_);
    dg_ = reinterpret_cast<const dev::GemmGroup*>(buf_.p + og);
    dt_ = reinterpret_cast<const dev::GemmTerm*>(buf_.p + ot);
    dtg_ = reinterpret_cast<const int*>(buf_.p + otg);
    red_.attach(buf_.p);
}
void GemmBatch::run() const {
    dev::Bases b = slots_.bases();
    b.p[kPartSlot] = part_.p;
    if (tiles_ > 0) dev::gemm_grouped(b, dg_, dtg_, dt_, tiles_, waves_, flops_, bytes_);
    red_.run(b);
}
void GemmBatch::run_lo(const dev::BasesF& b, int mode) const {
    if (abs_) throw err(MPSPT_E_STATE, "reduced-precision work list refers outside its bound buffers");
    dev::BasesF c = b;
    c.p[kPartSlot] = reinterpret_cast<float*>(part_.p);
    if (tiles_ > 0) dev::gemm_grouped_lo(c, mode, dg_, dtg_, dt_, tiles_, waves_, flops_, bytes_ / 2);
    red_.run_lo(c);
}

void AxpyBatch::group(double* dst, int ldd, int m, int n, bool acc) {
    int8_t sl;
    int64_t off;
    slots_.ref(dst, sl, off);
    group_ref(sl, off, ldd, m, n, acc);
}
void AxpyBatch::group_ref(int8_t slot, int64_t off, int ldd, int m, int n, bool acc) {
    if (slot == dev::kAbsSlot) abs_ = true;
    dev::AxpyGroup g{};
    g.sd = slot;
    g.od = off;
    g.ldd = ldd;
    g.m = m;
    g.n = n;
    g.term0 = (int)t_.size();
    g.accumulate = acc ? 1 : 0;
    g_.push_back(g);
}
void AxpyBatch::term(const double* src, int lds, bool trans, double alpha) {
    int8_t sl;
    int64_t off;
    slots_.ref(src, sl, off);
    term_ref(sl, off, lds, trans, alpha);
}
void AxpyBatch::term_ref(int8_t slot, int64_t off, int lds, bool trans, double alpha) {
    if (slot == dev::kAbsSlot) abs_ = true;
    dev::AxpyGroup& g = g_.back();
    dev::AxpyTerm t{};
    t.ss = slot;
    t.os = off;
    t.lds = lds;
    t.trans = trans ? 1 : 0;
    t.alpha = alpha;
    t_.push_back(t);
    ++g.nterms;
}
void AxpyBatch::pack(Packer& pk) {
    // empty groups are dropped here; the counts of the launch (each term
    // reads its block once, each group writes its block, reading it too
    // when it accumulates) are taken over the rest, once per list
    std::vector<dev::AxpyGroup> keep;
    keep.reserve(g_.size());
    flops_ = bytes_ = 0;
    for (auto& g : g_)
        if (g.m > 0 && g.n > 0) {
            const double mn = (double)g.m * g.n;
            flops_ += 2.0 * mn * g.nterms;
            bytes_ += 8.0 * mn * (g.nterms + (g.accumulate ? 2 : 1));
            keep.push_back(g);
        }
    g_.swap(keep);
    og_ = pk.add(g_);
    ot_ = pk.add(t_);
}
void AxpyBatch::attach(const char* dev_base) {
    dg_ = reinterpret_cast<const dev::AxpyGroup*>(dev_base + og_);
    dt_ = reinterpret_cast<const dev::AxpyTerm*>(dev_base + ot_);
}
void AxpyBatch::upload() {
    Packer pk;
    pack(pk);
    pk.upload(buf_);
    attach(buf_.p);
}
void AxpyBatch::run(const dev::Bases& b) const {
    if (!g_.empty()) dev::axpy_grouped(b, dg_, (int)g_.size(), dt_, flops_, bytes_);
}
void AxpyBatch::run_lo(const dev::BasesF& b) const {
    if (abs_) throw err(MPSPT_E_STATE, "reduced-precision work list refers outside its bound buffers");
    if (!g_.empty()) dev::axpy_grouped_lo(b, dg_, (int)g_.size(), dt_, flops_, bytes_ / 2);
}

// ------------------------------------------------------------- inputs
void Engine::set_integrals(int k_a, int k_v, std::vector<double> h, std::vector<double> eri) {
    k_a_ = k_a;
    k_v_ = k_v;
    n_ = k_a + k_v;
    h_ = std::move(h);
    eri_ = std::move(eri);
    virt_occ_.assign(k_v, 7);
    have_ints = true;
    have_part = have_psi0 = have_psi1 = false;
}

void Engine::set_partition(std::vector<double> eps) {
    if (!have_ints) throw err(MPSPT_E_STATE, "load integrals before the H0 partition");
    eps_ = std::move(eps);
    build_mpos();
    have_part = true;
    have_psi0 = have_psi1 = false;
}

// ------------------------------------------------- learned preconditioner
void Engine::precond_set(const float* p, int n) {
    if (n != dev::kMlpParams) throw err(MPSPT_E_ARG, "the network has " + std::to_string(dev::kMlpParams) + " parameters");
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(p[k])) throw err(MPSPT_E_ARG, "non-finite network parameter");
    const size_t words = (dev::kMlpParams + 1) / 2;
    for (DevBuf* b : {&mlp_, &mlp_m_, &mlp_v_}) b->ensure(words);
    dev::h2d(mlp_.p, p, n * sizeof(float));
    dev::zero(mlp_m_.p, words * sizeof(double));
    dev::zero(mlp_v_.p, words * sizeof(double));
    dev::sync();
    mlp_step_ = 0;
    mlp_set_ = true;
}

void Engine::precond_get(float* p, int n) const {
    if (!mlp_set_) throw err(MPSPT_E_STATE, "no preconditioner network loaded");
    if (n < dev::kMlpParams) throw err(MPSPT_E_ARG, "output too small for the network parameters");
    dev::d2h(p, mlp_.p, dev::kMlpParams * sizeof(float));
}

float Engine::mlp_step(const float* X, const float* t, int n, float lr, bool update, float* grad) {
    if (!mlp_set_) throw err(MPSPT_E_STATE, "no preconditioner network loaded");
    if (n <= 0) throw err(MPSPT_E_ARG, "training batch is empty");
    for (int k = 0; k < n; ++k)
        if (!(t[k] > 0.0f) || !std::isfinite(t[k])) throw err(MPSPT_E_ARG, "targets must be positive and finite");
    for (size_t k = 0; k < (size_t)n * dev::kMlpIn; ++k)
        if (!std::isfinite(X[k])) throw err(MPSPT_E_ARG, "non-finite feature");
    // io: X (n * in), t (n), grad (params), loss (1)
    const size_t fl = (size_t)n * dev::kMlpIn + n + dev::kMlpParams + 2;
    mlp_io_.ensure((fl + 1) / 2);
    float* io = reinterpret_cast<float*>(mlp_io_.p);
    float *dX = io, *dt = io + (size_t)n * dev::kMlpIn, *dg = dt + n, *dl = dg + dev::kMlpParams;
    dev::h2d(dX, X, (size_t)n * dev::kMlpIn * sizeof(float));
    dev::h2d(dt, t, (size_t)n * sizeof(float));
    mlp_scr_.ensure((dev::mlp_scratch_floats(n) + 1) / 2);
    if (update) ++mlp_step_;
    dev::mlp_train(dX, dt, n, reinterpret_cast<float*>(mlp_.p), reinterpret_cast<float*>(mlp_m_.p),
                   reinterpret_cast<float*>(mlp_v_.p), grad ? dg : nullptr, dl, mlp_step_, lr, update,
                   reinterpret_cast<float*>(mlp_scr_.p));
    float loss = 0.0f;
    dev::d2h(&loss, dl, sizeof(float));
    if (grad) dev::d2h(grad, dg, dev::kMlpParams * sizeof(float));
    return loss;
}

void Engine::set_harvest(bool on) {
    harvest_ = on;
    hx_.clear();
    ht_.clear();
}

int Engine::precond_blocks(const Two& lay) {
    std::vector<dev::BlockRef> br;
    br.reserve(lay.blk.size());
    for (size_t bb = 0; bb < lay.blk.size(); ++bb) {
        const auto& Y = lay.blk[bb];
        if (Y.rows > 0 && Y.cols > 0) br.push_back({(int64_t)lay.off((int)bb), lay.ld((int)bb), Y.rows, Y.cols});
    }
    pblocks_.upload(br);
    const int nb = (int)br.size();
    pstats_.ensure(std::max<size_t>((size_t)nb * dev::kBlockStats, 1));
    pfeat_.ensure(std::max<size_t>(((size_t)nb * dev::kMlpIn + 1) / 2, 1));
    pscale_.ensure(std::max<size_t>(((size_t)nb + 1) / 2, 1));
    return nb;
}

// d <- d / s_B with s_B from the network (the block-scaled Jacobi preconditioner)
void Engine::precond_apply(int i, int nb) {
    const float frac = n_ > 2 ? (float)i / (float)(n_ - 2) : 0.0f;
    dev::block_stats(pblocks_.p, nb, d_.p, r_.p, nullptr, pstats_.p);
    dev::precond_scales(pstats_.p, pblocks_.p, nb, frac, reinterpret_cast<const float*>(mlp_.p), nullptr,
                        reinterpret_cast<float*>(pscale_.p));
    dev::scale_blocks(pblocks_.p, nb, reinterpret_cast<const float*>(pscale_.p), d_.p);
}

// Features and targets of the window's blocks from the converged solution:
// t_B = <e0_B, z_B> / <z_B, z_B> with z = r0 / d (the Jacobi step of the
// initial residual) and e0 = x - x0 (the initial error), kept when positive
// (clipped to [0.05, 20]).
void Engine::harvest_window(int i, int nb) {
    if (nb <= 0) return;
    const float frac = n_ > 2 ? (float)i / (float)(n_ - 2) : 0.0f;
    const size_t words = (dev::kMlpParams + 1) / 2;
    if (!mlp_set_) {  // features do not depend on the parameters; give the kernel zeros
        mlp_.ensure(words);
        dev::zero(mlp_.p, words * sizeof(double));
    }
    const size_t n = xlay_.size;
    dev::axpby(px0_.p, x_.p, 1.0, -1.0, n);  // e0 = x - x0
    dev::block_stats(pblocks_.p, nb, d_.p, pr0_.p, px0_.p, pstats_.p);
    dev::precond_scales(pstats_.p, pblocks_.p, nb, frac, reinterpret_cast<const float*>(mlp_.p),
                        reinterpret_cast<float*>(pfeat_.p), reinterpret_cast<float*>(pscale_.p));
    std::vector<double> st((size_t)nb * dev::kBlockStats);
    std::vector<float> ft((size_t)nb * dev::kMlpIn);
    dev::d2h(st.data(), pstats_.p, st.size() * sizeof(double));
    dev::d2h(ft.data(), pfeat_.p, ft.size() * sizeof(float));
    for (int k = 0; k < nb; ++k) {
        const double zx = st[(size_t)k * dev::kBlockStats + 3], zz = st[(size_t)k * dev::kBlockStats + 4];
        if (!(zz > 0.0)) continue;
        const double t = zx / zz;
        if (!(t > 0.0)) continue;
        hx_.insert(hx_.end(), ft.begin() + (size_t)k * dev::kMlpIn, ft.begin() + (size_t)(k + 1) * dev::kMlpIn);
        ht_.push_back((float)std::min(20.0, std::max(0.05, t)));
    }
}

void Engine::ensure_partials() {
    if (partials_.n >= (size_t)dev::kPartialsWords) return;
    partials_.ensure(dev::kPartialsWords);
    dev::zero(partials_.p, dev::kPartialsWords * sizeof(double));
}

Engine::~Engine() {
    // copies into the pinned buffers below may still be in flight (a sweep
    // that stopped on an error leaves them): drain the stream first
    try {
        dev::sync();
    } catch (...) {
    }
    dev::host_free(hsc_);
    for (void* e : ev_) dev::event_destroy(e);
    dev::host_free(eig_status_h_);
    dev::event_destroy(eig_ev_);
}

void Engine::drop_eig_status() {  // a flag left by an earlier call that stopped on an error
    if (!eig_pending_) return;
    dev::event_wait(eig_ev_);
    eig_pending_ = false;
}

void Engine::check_eig_status() {
    if (!eig_pending_) return;
    dev::event_wait(eig_ev_);
    eig_pending_ = false;
    if (*eig_status_h_) throw err(MPSPT_E_STATE, "eigensolver could not orthonormalise a kept basis");
}

void Engine::clear_plans() {
    for (auto& v : eff_plans_) v.clear();
    for (auto& v : env_plans_) v.clear();
    diag_plans_.clear();
}

void Engine::build_mpos() {
    clear_plans();
    mpo_h0_ = build_mpo(OpKind::H0, k_a_, k_v_, h_, eri_, eps_);
    mpo_v_ = build_mpo(OpKind::VPsi0, k_a_, k_v_, h_, eri_, eps_);
    mpo_e3_ = MPO();  // built on first use (E3 only)
    twoop_cache_[0].clear();
    clear_plans();
    twoop_cache_[1].clear();
}

const TwoOp& Engine::twoop(int which, int i) {
    auto& cache = twoop_cache_[which];
    if ((int)cache.size() < n_ - 1) cache.resize(n_ - 1);
    if (!cache[i]) cache[i] = std::make_unique<TwoOp>(make_twoop(which == 0 ? mpo_h0_ : mpo_v_, i));
    return *cache[i];
}

void Engine::load_site(Site& s, const std::vector<double>& dense) {
    const int Dl = s.L.total(), Dr = s.R.total();
    if (dense.size() != (size_t)Dl * 4 * Dr) throw err(MPSPT_E_ARG, "site tensor size does not match bond dimensions");
    std::vector<int> ol(s.L.q.size() + 1, 0), orr(s.R.q.size() + 1, 0);
    for (size_t a = 0; a < s.L.q.size(); ++a) ol[a + 1] = ol[a] + s.L.d[a];
    for (size_t a = 0; a < s.R.q.size(); ++a) orr[a + 1] = orr[a] + s.R.d[a];
    std::vector<char> covered(dense.size(), 0);
    std::vector<double> host(s.size, 0.0);
    for (size_t b = 0; b < s.blk.size(); ++b) {
        const auto& B = s.blk[b];
        size_t base = s.po[B.il] + B.col;
        for (int r = 0; r < B.rows; ++r)
            for (int c = 0; c < B.cols; ++c) {
                size_t di = ((size_t)(ol[B.il] + r) * 4 + B.s) * Dr + orr[B.jr] + c;
                host[base + (size_t)r * s.pw[B.il] + c] = dense[di];
                covered[di] = 1;
            }
    }
    for (size_t i = 0; i < dense.size(); ++i) {
        if (!std::isfinite(dense[i])) throw err(MPSPT_E_ARG, "non-finite entry in a site tensor");
        if (!covered[i] && dense[i] != 0.0) throw err(MPSPT_E_QN, "site tensor entry outside the blocks its labels allow");
    }
    if (s.size) dev::h2d(s.data.p, host.data(), s.size * sizeof(double));
    dev::sync();  // the staging vector is released on return
}

Env Engine::trivial_env(const Bond& bra, const Bond& ket) const {
    Env e;
    e.nch = 1;
    e.bra = bra;
    e.ket = ket;
    e.blk.push_back({0, 0, 0, 1, 1, 0});
    e.size = 1;
    e.dq = {QN{0, 0}};
    e.index();
    e.data.alloc(1);
    double one = 1.0;
    dev::h2d(e.data.p, &one, sizeof(double));
    dev::sync();
    return e;
}

static MPO identity_mpo(int n) {
    MPO m;
    m.n = n;
    m.dims.assign(n + 1, 1);
    m.dq.assign(n + 1, std::vector<QN>{QN{0, 0}});
    m.W.resize(n);
    for (int i = 0; i < n; ++i) {
        MPOEntry e{0, 0, {0}};
        for (int s = 0; s < 4; ++s) e.m[s * 4 + s] = 1.0;
        m.W[i].push_back(e);
    }
    return m;
}

void Engine::set_psi0(int n_elec, int two_sz, const std::vector<Bond>& bonds,
                      const std::vector<std::vector<double>>& sites) {
    if (!have_part) throw err(MPSPT_E_STATE, "load integrals and the H0 partition before Psi0");
    if ((int)bonds.size() != k_a_ + 1 || (int)sites.size() != k_a_) throw err(MPSPT_E_ARG, "Psi0 needs k_a sites");
    clear_plans();
    if (bonds[0].q.size() != 1 || bonds[0].q[0] != QN{0, 0} || bonds[0].d[0] != 1)
        throw err(MPSPT_E_QN, "first bond of Psi0 must be the single label (0, 0)");
    if (bonds[k_a_].q.size() != 1 || bonds[k_a_].q[0] != QN{n_elec, two_sz} || bonds[k_a_].d[0] != 1)
        throw err(MPSPT_E_QN, "last bond of Psi0 must be the single label (n_elec, two_sz)");
    N_ = n_elec;
    tsz_ = two_sz;
    std::vector<Bond> b = bonds;
    for (int i = k_a_ + 1; i <= n_; ++i) b.push_back(bonds[k_a_]);
    P0_.clear();
    for (int i = 0; i < n_; ++i) {
        P0_.push_back(make_site(b[i], b[i + 1]));
        if (i < k_a_) {
            load_site(P0_[i], sites[i]);
        } else {
            std::vector<double> v(4, 0.0);
            v[0] = 1.0;
            load_site(P0_[i], v);
        }
    }
    // normalise and E0 = <Psi0|H0|Psi0>
    MPO idm = identity_mpo(n_);
    Env ov = trivial_env(b[0], b[0]), eh = trivial_env(b[0], b[0]);
    for (int i = 0; i < n_; ++i) {
        Env o2, e2;
        env_left(o2, ov, P0_[i], P0_[i], idm, i);
        env_left(e2, eh, P0_[i], P0_[i], mpo_h0_, i);
        ov = std::move(o2);
        eh = std::move(e2);
    }
    double norm = 0, eh0 = 0;
    if (ov.blk.size() != 1 || eh.blk.size() != 1) throw err(MPSPT_E_QN, "Psi0 has no weight in its target sector");
    dev::d2h(&norm, ov.data.p, sizeof(double));
    dev::d2h(&eh0, eh.data.p, sizeof(double));
    if (!(norm > 0.0)) throw err(MPSPT_E_ARG, "Psi0 has zero norm");
    E0_ = eh0 / norm;
    dev::axpby(P0_[0].data.p, P0_[0].data.p, 0.0, 1.0 / std::sqrt(norm), P0_[0].size);
    P0x_lay_.clear();
    P0x_.clear();
    for (int i = 0; i + 1 < n_; ++i) {
        P0x_lay_.push_back(make_two(b[i], b[i + 2], nullptr));
        P0x_.emplace_back();
        P0x_.back().alloc(std::max<size_t>(P0x_lay_.back().size, 1));
        contract_sites(P0_[i], P0_[i + 1], P0x_lay_.back(), P0x_.back().p);
    }
    compute_adm();
    have_psi0 = true;
    have_psi1 = false;
}

void Engine::restrict_virtual(const std::vector<int>& masks) {
    if (!have_ints) throw err(MPSPT_E_STATE, "load integrals before restricting the virtual sites");
    if ((int)masks.size() != k_v_) throw err(MPSPT_E_ARG, "one occupancy mask per virtual site");
    for (int m : masks)
        if (m < 1 || m > 7) throw err(MPSPT_E_ARG, "occupancy masks must lie in [1, 7]");
    std::vector<int> prev = virt_occ_;
    virt_occ_ = masks;
    if (have_psi0) {
        try {
            compute_adm();
        } catch (...) {
            virt_occ_ = prev;
            compute_adm();
            throw;
        }
        clear_plans();
        have_psi1 = false;
    }
}

// Admissible (N, 2Sz) at every bond of Psi1: one or two virtual electrons, and
// on each virtual site an electron count its mask allows.
void Engine::compute_adm() {
    auto site_ok = [&](int i, int s) { return i < k_a_ || ((virt_occ_[i - k_a_] >> site_dq(s).n) & 1); };
    std::vector<std::set<std::tuple<int, int, int>>> left(n_ + 1), right(n_ + 1);
    left[0].insert({0, 0, 0});
    for (int i = 0; i < n_; ++i)
        for (auto& t : left[i])
            for (int s = 0; s < 4; ++s) {
                if (!site_ok(i, s)) continue;
                QN d = site_dq(s);
                left[i + 1].insert({std::get<0>(t) + d.n, std::get<1>(t) + d.s, std::get<2>(t) + (i >= k_a_ ? d.n : 0)});
            }
    right[n_].insert({0, 0, 0});
    for (int i = n_ - 1; i >= 0; --i)
        for (auto& t : right[i + 1])
            for (int s = 0; s < 4; ++s) {
                if (!site_ok(i, s)) continue;
                QN d = site_dq(s);
                right[i].insert({std::get<0>(t) + d.n, std::get<1>(t) + d.s, std::get<2>(t) + (i >= k_a_ ? d.n : 0)});
            }
    std::vector<std::set<QN>> adm(n_ + 1);
    for (int bb = 0; bb <= n_; ++bb)
        for (auto& l : left[bb])
            for (int nvr = 0; nvr <= 2; ++nvr) {
                int nv = std::get<2>(l) + nvr;
                if (nv < 1 || nv > 2) continue;
                if (right[bb].count({N_ - std::get<0>(l), tsz_ - std::get<1>(l), nvr}))
                    adm[bb].insert(QN{std::get<0>(l), std::get<1>(l)});
            }
    // The sweep restricts only bond labels.  Every label to the right of the
    // active block fixes the electron count still to come, so a site's count is
    // the difference of its two labels; refuse masks that some pair of
    // admissible neighbouring labels would violate.
    for (int i = k_a_; i < n_; ++i)
        for (const QN& l : adm[i])
            for (int s = 0; s < 4; ++s)
                if (adm[i + 1].count(l + site_dq(s)) && !site_ok(i, s))
                    throw err(MPSPT_E_ARG, "virtual occupancy masks cannot be expressed through bond sectors");
    adm_ = std::move(adm);
}

void Engine::set_psi1(const std::vector<Bond>& bonds, const std::vector<std::vector<double>>& sites) {
    if (!have_psi0) throw err(MPSPT_E_STATE, "load Psi0 before the Psi1 guess");
    if ((int)bonds.size() != n_ + 1 || (int)sites.size() != n_) throw err(MPSPT_E_ARG, "Psi1 needs k_a + k_v sites");
    if (bonds[0].q.size() != 1 || bonds[0].q[0] != QN{0, 0} || bonds[0].d[0] != 1)
        throw err(MPSPT_E_QN, "first bond of Psi1 must be the single label (0, 0)");
    if (bonds[n_].q.size() != 1 || bonds[n_].q[0] != QN{N_, tsz_} || bonds[n_].d[0] != 1)
        throw err(MPSPT_E_QN, "last bond of Psi1 must be the single label (n_elec, two_sz)");
    for (int b = 0; b <= n_; ++b)
        for (auto& q : bonds[b].q)
            if (!adm_[b].count(q)) throw err(MPSPT_E_QN, "Psi1 bond sector outside the one/two virtual electron space");
    // validate now (block structure), keep host copies for each sweep call
    for (int i = 0; i < n_; ++i) {
        Site s = make_site(bonds[i], bonds[i + 1]);
        load_site(s, sites[i]);
    }
    psi1_bonds_ = bonds;
    psi1_guess_ = sites;
    have_psi1 = true;
}

// ------------------------------------------------------ contractions
void Engine::contract_sites(const Site& A, const Site& B, const Two& lay, double* out) {
    GemmBatch g;
    for (size_t b = 0; b < lay.blk.size(); ++b) {
        const auto& X = lay.blk[b];
        g.group(out + lay.off((int)b), lay.ld((int)b), X.rows, X.cols, false);
        int a = A.idx[X.il * 4 + X.s1];
        if (a < 0) continue;
        int jm = A.blk[a].jr;
        int bb = B.idx[jm * 4 + X.s2];
        if (bb < 0 || B.blk[bb].jr != X.jr) continue;
        g.term(A.at(a), A.ld(a), false, B.at(bb), B.ld(bb), false, A.blk[a].cols, 1.0);
    }
    g.upload();
    g.run();
}

void Engine::bind_env(GemmBatch& g, const Env& in, const Site& Abra, const Site& Aket, size_t tsz, const Env& out) {
    g.bind(0, in.data.p, in.size);
    g.bind(1, Abra.data.p, Abra.size);
    g.bind(2, Aket.data.p, Aket.size);
    g.bind(3, T_.p, tsz);
    g.bind(4, out.data.p, out.size);
}

// Replays a cached environment update when its input layouts are unchanged.
bool Engine::env_cached(Env& out, const Env& in, const Site& Abra, const Site& Aket, const MPO& m, int i,
                        std::unique_ptr<EnvPlan>* plan, Sig& sig) {
    if (!plan) return false;
    sig.add((int64_t)(uintptr_t)&m);
    sig.add(i);
    sig_env(sig, in);
    sig_site(sig, Abra);
    sig_site(sig, Aket);
    if (!*plan || (*plan)->sig != sig) return false;
    EnvPlan& P = **plan;
    out.copy_layout(P.lay);
    out.data.ensure(std::max<size_t>(out.size, 1));
    T_.ensure(std::max<size_t>(P.tsz, 1));
    bind_env(P.ga, in, Abra, Aket, P.tsz, out);
    bind_env(P.gb, in, Abra, Aket, P.tsz, out);
    P.ga.run();
    P.gb.run();
    ++res_.plan_hits;
    return true;
}

void Engine::env_left(Env& out, const Env& L, const Site& Abra, const Site& Aket, const MPO& m, int i,
                      std::unique_ptr<EnvPlan>* plan) {
    Sig sig;
    if (env_cached(out, L, Abra, Aket, m, i, plan, sig)) return;
    DevBuf keep = std::move(out.data);
    out = Env();
    out.data = std::move(keep);
    out.nch = m.dims[i + 1];
    out.bra = Abra.R;
    out.ket = Aket.R;
    auto fresh = std::make_unique<EnvPlan>();
    GemmBatch& ga = fresh->ga;
    GemmBatch& gb = fresh->gb;
    // stage a: T[lb] = L block . row panel of Aket
    std::vector<size_t> toff(L.blk.size(), (size_t)-1);
    size_t tsz = 0;
    for (size_t lb = 0; lb < L.blk.size(); ++lb) {
        int ik = L.blk[lb].ik;
        if (Aket.pw[ik] == 0) continue;
        toff[lb] = tsz;
        tsz += (size_t)L.blk[lb].rows * Aket.pw[ik];
    }
    T_.ensure(std::max<size_t>(tsz, 1));
    bind_env(ga, L, Abra, Aket, tsz, out);
    for (size_t lb = 0; lb < L.blk.size(); ++lb) {
        if (toff[lb] == (size_t)-1) continue;
        const auto& B = L.blk[lb];
        ga.group(T_.p + toff[lb], Aket.pw[B.ik], B.rows, Aket.pw[B.ik], false);
        ga.term(L.data.p + B.off, B.cols, false, Aket.data.p + Aket.po[B.ik], Aket.pw[B.ik], false, B.cols, 1.0);
    }
    // stage b: contributions per output block (channel, bra sector)
    struct Tm { const double* A; int lda; const double* B; int ldb; int k; double a; };
    OutTable<Tm> outs(out.nch, (int)out.bra.q.size());
    for (const MPOEntry& e : m.W[i]) {
        for (int s = 0; s < 4; ++s)
            for (int t = 0; t < 4; ++t) {
                double v = e.m[s * 4 + t];
                if (v == 0.0) continue;
                for (int lb : L.by_w[e.cin]) {
                    if (toff[lb] == (size_t)-1) continue;
                    const auto& B = L.blk[lb];
                    int ab = Abra.idx[B.ib * 4 + s];
                    int ak = Aket.idx[B.ik * 4 + t];
                    if (ab < 0 || ak < 0) continue;
                    outs.add(e.cout, Abra.blk[ab].jr, Aket.blk[ak].jr,
                             {Abra.at(ab), Abra.ld(ab), T_.p + toff[lb] + Aket.blk[ak].col, Aket.pw[B.ik], B.rows, v});
                }
            }
    }
    size_t off = 0;
    outs.each([&](int w, int ib, int ik, const std::vector<Tm>&) {
        out.blk.push_back({w, ib, ik, out.bra.d[ib], out.ket.d[ik], off});
        off += (size_t)out.bra.d[ib] * out.ket.d[ik];
    });
    out.size = off;
    out.dq = m.dq[i + 1];
    out.index();
    out.data.ensure(std::max<size_t>(off, 1));
    bind_env(gb, L, Abra, Aket, tsz, out);
    size_t bi = 0;
    outs.each([&](int, int, int, const std::vector<Tm>& terms) {
        const auto& B = out.blk[bi++];
        gb.group(out.data.p + B.off, B.cols, B.rows, B.cols, false);
        for (const Tm& t : terms) gb.term(t.A, t.lda, true, t.B, t.ldb, false, t.k, t.a);
    });
    ga.upload();
    gb.upload();
    ga.run();
    gb.run();
    if (plan) {
        fresh->sig = std::move(sig);
        fresh->lay.copy_layout(out);
        fresh->tsz = tsz;
        *plan = std::move(fresh);
        ++res_.plan_builds;
    }
}

void Engine::env_right(Env& out, const Env& R, const Site& Abra, const Site& Aket, const MPO& m, int i,
                       std::unique_ptr<EnvPlan>* plan) {
    Sig sig;
    if (env_cached(out, R, Abra, Aket, m, i, plan, sig)) return;
    DevBuf keep = std::move(out.data);
    out = Env();
    out.data = std::move(keep);
    out.nch = m.dims[i];
    out.bra = Abra.L;
    out.ket = Aket.L;
    auto fresh = std::make_unique<EnvPlan>();
    GemmBatch& ga = fresh->ga;
    GemmBatch& gb = fresh->gb;
    struct Tm { const double* A; int lda; size_t toff; int ldb; int k; double a; };
    // T(rb, t) = R block rb . (Aket block with right sector ib_ket(rb) and local state t)^T;
    // for a fixed R block and local state that Aket block is unique
    std::vector<size_t> toff(R.blk.size() * 4, (size_t)-1);
    struct Ta { int rb, ak; size_t off; };
    std::vector<Ta> tlist;
    size_t tsz = 0;
    OutTable<Tm> outs(out.nch, (int)out.bra.q.size());
    for (const MPOEntry& e : m.W[i]) {
        for (int s = 0; s < 4; ++s)
            for (int t = 0; t < 4; ++t) {
                double v = e.m[s * 4 + t];
                if (v == 0.0) continue;
                for (int rb : R.by_w[e.cout]) {
                    const auto& B = R.blk[rb];
                    for (int ab : Abra.by_jr[B.ib]) {
                        if (Abra.blk[ab].s != s) continue;
                        for (int ak : Aket.by_jr[B.ik]) {
                            if (Aket.blk[ak].s != t) continue;
                            size_t& to = toff[(size_t)rb * 4 + t];
                            if (to == (size_t)-1) {
                                to = tsz;
                                tlist.push_back({rb, ak, to});
                                tsz += (size_t)B.rows * Aket.blk[ak].rows;
                            }
                            outs.add(e.cin, Abra.blk[ab].il, Aket.blk[ak].il,
                                     {Abra.at(ab), Abra.ld(ab), to, Aket.blk[ak].rows, B.rows, v});
                        }
                    }
                }
            }
    }
    T_.ensure(std::max<size_t>(tsz, 1));
    bind_env(ga, R, Abra, Aket, tsz, out);
    for (const Ta& t : tlist) {
        const auto& B = R.blk[t.rb];
        const auto& K = Aket.blk[t.ak];
        ga.group(T_.p + t.off, K.rows, B.rows, K.rows, false);
        ga.term(R.data.p + B.off, B.cols, false, Aket.at(t.ak), Aket.ld(t.ak), true, B.cols, 1.0);
    }
    size_t off = 0;
    outs.each([&](int w, int ib, int ik, const std::vector<Tm>&) {
        out.blk.push_back({w, ib, ik, out.bra.d[ib], out.ket.d[ik], off});
        off += (size_t)out.bra.d[ib] * out.ket.d[ik];
    });
    out.size = off;
    out.dq = m.dq[i];
    out.index();
    out.data.ensure(std::max<size_t>(off, 1));
    bind_env(gb, R, Abra, Aket, tsz, out);
    size_t bi = 0;
    outs.each([&](int, int, int, const std::vector<Tm>& terms) {
        const auto& B = out.blk[bi++];
        gb.group(out.data.p + B.off, B.cols, B.rows, B.cols, false);
        for (const Tm& t : terms) gb.term(t.A, t.lda, false, T_.p + t.toff, t.ldb, false, t.k, t.a);
    });
    ga.upload();
    gb.upload();
    ga.run();
    gb.run();
    if (plan) {
        fresh->sig = std::move(sig);
        fresh->lay.copy_layout(out);
        fresh->tsz = tsz;
        *plan = std::move(fresh);
        ++res_.plan_builds;
    }
}

void Engine::build_effop(EffOp& op, const Env& L, const Env& R, const TwoOp& O, const Two& ket,
                         const double* xket, const Two& bra, double* ybra) {
    op.st1.clear();
    op.st2.clear();
    op.st3.clear();
    op.flops = op.bytes = 0;
    op.bind(0, L.data.p, L.size);
    op.bind(1, R.data.p, R.size);
    op.bind(2, xket, ket.size);
    op.bind(3, ybra, bra.size);
    // stage 1 layout: U[lb] = L block . ket row panel
    std::vector<size_t> uoff(L.blk.size(), (size_t)-1);
    size_t usz = 0;
    std::vector<char> lused(L.blk.size(), 0), rused(R.blk.size(), 0);
    for (size_t lb = 0; lb < L.blk.size(); ++lb) {
        int ik = L.blk[lb].ik;
        if (ket.pw[ik] == 0) continue;
        uoff[lb] = usz;
        usz += (size_t)L.blk[lb].rows * ket.pw[ik];
    }
    // stage 2: V blocks per (bra block, w'), emitted straight into the
    // middle-stage list as they are found (slot-relative references: U is
    // slot 4, V slot 5; a block's group is opened at its first term)
    struct VB { int bb, rb; size_t off; int rows, cols; };
    std::vector<VB> vbs;
    size_t vsz = 0;
    {
        size_t ng = 0, nt = 0;  // upper bounds, for one allocation of each list
        for (size_t bb = 0; bb < bra.blk.size(); ++bb) {
            const auto& Y = bra.blk[bb];
            for (int rb : R.by_ib[Y.jr]) {
                ++ng;
                nt += O.by_out[(size_t)R.blk[rb].w * 16 + Y.s1 * 4 + Y.s2].size();
            }
        }
        op.st2.reserve(ng, nt);
        vbs.reserve(ng);
    }
    for (size_t bb = 0; bb < bra.blk.size(); ++bb) {
        const auto& Y = bra.blk[bb];
        for (int rb : R.by_ib[Y.jr]) {
            const int wp = R.blk[rb].w;
            const auto& terms = O.by_out[(size_t)wp * 16 + Y.s1 * 4 + Y.s2];
            if (terms.empty()) continue;
            const int jrk = R.blk[rb].ik;
            const int cols = R.blk[rb].cols;
            bool open = false;
            for (const auto& t : terms) {
                // the L block of channel w at this bra sector fixes the ket sector
                const int lb = L.find(t.w, Y.il);
                if (lb < 0 || uoff[lb] == (size_t)-1) continue;
                const int ik = L.blk[lb].ik;
                const int xb = ket.idx[(ik * 4 + t.s1) * 4 + t.s2];
                if (xb < 0 || ket.blk[xb].jr != jrk) continue;
                if (!open) {
                    op.st2.group_ref(5, (int64_t)vsz, cols, Y.rows, cols, false);
                    open = true;
                }
                op.st2.term_ref(4, (int64_t)(uoff[lb] + ket.blk[xb].col), ket.pw[ik], false, t.v);
                lused[lb] = 1;
            }
            if (!open) continue;
            vbs.push_back({(int)bb, rb, vsz, Y.rows, cols});
            vsz += (size_t)Y.rows * cols;
            rused[rb] = 1;
        }
    }
    op.U.ensure(std::max<size_t>(usz, 1));
    op.V.ensure(std::max<size_t>(vsz, 1));
    op.bind(4, op.U.p, usz);
    op.bind(5, op.V.p, vsz);
    for (size_t lb = 0; lb < L.blk.size(); ++lb) {
        if (uoff[lb] == (size_t)-1 || !lused[lb]) continue;
        const auto& B = L.blk[lb];
        op.st1.group(op.U.p + uoff[lb], ket.pw[B.ik], B.rows, ket.pw[B.ik], false);
        op.st1.term(L.data.p + B.off, B.cols, false, xket + ket.po[B.ik], ket.pw[B.ik], false, B.cols, 1.0);
        op.bytes += 8.0 * B.rows * B.cols;
    }
    size_t vi = 0;
    for (size_t bb = 0; bb < bra.blk.size(); ++bb) {
        const auto& Y = bra.blk[bb];
        op.st3.group(ybra + bra.off((int)bb), bra.ld((int)bb), Y.rows, Y.cols, false);
        while (vi < vbs.size() && vbs[vi].bb == (int)bb) {
            const VB& v = vbs[vi++];
            const auto& RB = R.blk[v.rb];
            op.st3.term(op.V.p + v.off, v.cols, false, R.data.p + RB.off, RB.cols, true, v.cols, 1.0);
        }
    }
    for (size_t rb = 0; rb < R.blk.size(); ++rb)
        if (rused[rb]) op.bytes += 8.0 * R.blk[rb].rows * R.blk[rb].cols;
    op.bytes += 8.0 * (ket.size + bra.size);
    op.st1.upload();
    op.st2.upload();
    op.st3.upload();
    op.flops = op.st1.flops() + op.st2.flops() + op.st3.flops();
}

// The effective operator of window i in role r (0: H0 - E0 on the two-site
// space, 1: the right-hand side from Psi0), rebuilt only when its layouts
// changed since the last sweep.
EffOp& Engine::effop(int r, int i, const Env& L, const Env& R, const TwoOp& O, const Two& ket, const double* xket,
                     const Two& bra, double* ybra) {
    auto& plans = eff_plans_[r];
    if ((int)plans.size() <= i) plans.resize(i + 1);
    Sig sig;
    sig.add((int64_t)(uintptr_t)&O);
    sig_env(sig, L);
    sig_env(sig, R);
    sig_two(sig, ket);
    sig_two(sig, bra);
    auto& pl = plans[i];
    if (!pl || pl->sig != sig) {
        pl = std::make_unique<EffPlan>();
        build_effop(pl->op, L, R, O, ket, xket, bra, ybra);
        pl->sig = std::move(sig);
        ++res_.plan_builds;
    } else {
        EffOp& op = pl->op;
        op.bind(0, L.data.p, L.size);
        op.bind(1, R.data.p, R.size);
        op.bind(2, xket, ket.size);
        op.bind(3, ybra, bra.size);
        op.bind(4, op.U.p, op.U.n);
        op.bind(5, op.V.p, op.V.n);
        ++res_.plan_hits;
    }
    return pl->op;
}

void Engine::build_diag(int i, const Env& L, const Env& R, const TwoOp& O, const Two& lay, double* d, double shift) {
    if ((int)diag_plans_.size() <= i) diag_plans_.resize(i + 1);
    Sig sig;
    sig.add((int64_t)(uintptr_t)&O);
    int64_t sbits;
    std::memcpy(&sbits, &shift, sizeof(sbits));
    sig.add(sbits);
    sig_env(sig, L);
    sig_env(sig, R);
    sig_two(sig, lay);
    auto& pl = diag_plans_[i];
    if (!pl || pl->sig != sig) {
        pl = std::make_unique<DiagPlan>();
        SlotMap sm;
        sm.bind(0, L.data.p, L.size);
        sm.bind(1, R.data.p, R.size);
        sm.bind(2, d, lay.size);
        std::vector<dev::DiagGroup> gs;
        std::vector<dev::DiagTerm> ts;
        for (size_t bb = 0; bb < lay.blk.size(); ++bb) {
            const auto& Y = lay.blk[bb];
            dev::DiagGroup g{};
            sm.ref(d + lay.off((int)bb), g.sd, g.od);
            g.shift = shift;
            g.ldd = lay.ld((int)bb);
            g.m = Y.rows;
            g.n = Y.cols;
            g.term0 = (int)ts.size();
            for (int rb : R.by_ib[Y.jr]) {
                const int wp = R.blk[rb].w;
                if (R.blk[rb].ik != Y.jr) continue;
                for (const auto& t : O.by_out[(size_t)wp * 16 + Y.s1 * 4 + Y.s2]) {
                    if (t.s1 != Y.s1 || t.s2 != Y.s2) continue;
                    int lb = L.find(t.w, Y.il);
                    if (lb < 0 || L.blk[lb].ik != Y.il) continue;
                    dev::DiagTerm dt{};
                    sm.ref(L.data.p + L.blk[lb].off, dt.sl, dt.ol);
                    sm.ref(R.data.p + R.blk[rb].off, dt.sr, dt.orr);
                    dt.ls = L.blk[lb].cols + 1;
                    dt.rs = R.blk[rb].cols + 1;
                    dt.c = t.v;
                    ts.push_back(dt);
                    ++g.nterms;
                }
            }
            if (Y.rows > 0 && Y.cols > 0) gs.push_back(g);
        }
        pl->ng = (int)gs.size();
        pl->dg.upload(gs);
        pl->dt.upload(ts);
        pl->sig = std::move(sig);
        ++res_.plan_builds;
    } else {
        ++res_.plan_hits;
    }
    SlotMap sm;
    sm.bind(0, L.data.p, L.size);
    sm.bind(1, R.data.p, R.size);
    sm.bind(2, d, lay.size);
    if (pl->ng > 0) dev::diag_grouped(sm.bases(), pl->dg.p, pl->ng, pl->dt.p);
}

// ----------------------------------------------------------- truncation
namespace {
struct Sel {
    std::vector<int> kept;  // per group
    double disc = 0;
};
// Keep the M largest eigenvalues over all sectors (ties by sector, then
// index); drop eigenvalues <= 1e-14 of the trace; never cut between two
// eigenvalues within a relative 1e-4 of each other (spin multiplets stay
// whole) unless that would keep nothing.
Sel select_states(const std::vector<std::vector<double>>& w, int M) {
    struct E { double l; int g, j; };
    std::vector<E> all;
    double tr = 0;
    for (size_t g = 0; g < w.size(); ++g)
        for (size_t j = 0; j < w[g].size(); ++j) {
            all.push_back({w[g][j], (int)g, (int)j});
            tr += w[g][j];
        }
    std::stable_sort(all.begin(), all.end(), [](const E& a, const E& b) {
        if (a.l != b.l) return a.l > b.l;
        if (a.g != b.g) return a.g < b.g;
        return a.j < b.j;
    });
    // a vanishing density matrix (zero local solution) keeps min(M, dim)
    // states in (sector, index) order: every basis is equally significant
    int nsig = tr > 0 ? 0 : (int)all.size();
    if (tr > 0)
        for (auto& e : all) nsig += e.l > 1e-14 * tr;
    int K0 = std::min(M, nsig), K = K0;
    while (K > 0 && K < (int)all.size() && all[K - 1].l <= (1.0 + 1e-4) * all[K].l) --K;
    if (K == 0) K = K0;
    Sel s;
    s.kept.assign(w.size(), 0);
    double kept = 0;
    for (int i = 0; i < K; ++i) {
        s.kept[all[i].g]++;
        kept += all[i].l;
    }
    s.disc = tr > 0 ? 1.0 - kept / tr : 0.0;
    return s;
}
}  // namespace

double Engine::truncate(int i, bool forward, const Two& lay, const double* x, int M, Site& C, bool zero) {
    // groups of rows (forward: (il, s1)) or columns (backward: (s2, jr)) by middle sector
    struct Part { int a, b, off, dim; };  // forward: a=il b=s1 ; backward: a=s2 b=jr
    std::map<QN, std::vector<Part>> groups;
    if (forward) {
        for (int il = 0; il < (int)lay.L.q.size(); ++il)
            for (int s1 = 0; s1 < 4; ++s1) {
                bool any = false;
                for (int s2 = 0; s2 < 4; ++s2) any |= lay.idx[(il * 4 + s1) * 4 + s2] >= 0;
                if (any) groups[lay.L.q[il] + site_dq(s1)].push_back({il, s1, 0, lay.L.d[il]});
            }
    } else {
        std::set<std::pair<int, int>> cols;
        for (const auto& Y : lay.blk) cols.insert({Y.s2, Y.jr});
        for (auto& c : cols) groups[lay.R.q[c.second] - site_dq(c.first)].push_back({c.first, c.second, 0, lay.R.d[c.second]});
    }
    std::vector<QN> gq;
    std::vector<int> gdim;
    std::vector<size_t> goff;
    size_t rsz = 0;
    for (auto& kv : groups) {
        int d = 0;
        for (auto& p : kv.second) { p.off = d; d += p.dim; }
        gq.push_back(kv.first);
        gdim.push_back(d);
        goff.push_back(rsz);
        rsz += (size_t)d * d;
    }
    const int ng = (int)gq.size();
    for (int d : gdim)
        if (d > 512) throw err(MPSPT_E_ARG, "density-matrix sector larger than 512 (eigensolver limit)");
    rho_.ensure(std::max<size_t>(rsz, 1));
    eigV_.ensure(std::max<size_t>(rsz, 1));
    size_t wsz = 0;
    std::vector<size_t> woff(ng);
    for (int g = 0; g < ng; ++g) { woff[g] = wsz; wsz += gdim[g]; }
    eigw_.ensure(std::max<size_t>(wsz, 1));
    Sel sel;
    if (zero) {
        // x = 0: the density matrices vanish; keep identity bases (any
        // orthonormal basis spans an equally insignificant kept space)
        std::vector<std::vector<double>> w(ng);
        for (int q = 0; q < ng; ++q) w[q].assign(gdim[q], 0.0);
        sel = select_states(w, M);
        std::vector<double> eye(std::max<size_t>(rsz, 1), 0.0);
        for (int q = 0; q < ng; ++q)
            for (int r = 0; r < gdim[q]; ++r) eye[goff[q] + (size_t)r * gdim[q] + r] = 1.0;
        dev::h2d(rho_.p, eye.data(), rsz * sizeof(double));
    } else {
    // reduced density matrices
    GemmBatch gr;
    int g = 0;
    for (auto& kv : groups) {
        const auto& parts = kv.second;
        const int d = gdim[g];
        for (const auto& pa : parts)
            for (const auto& pb : parts) {
                gr.group(rho_.p + goff[g] + (size_t)pa.off * d + pb.off, d, pa.dim, pb.dim, false);
                if (forward) {
                    for (int s2 = 0; s2 < 4; ++s2) {
                        int xa = lay.idx[(pa.a * 4 + pa.b) * 4 + s2];
                        int xb = lay.idx[(pb.a * 4 + pb.b) * 4 + s2];
                        if (xa < 0 || xb < 0) continue;
                        gr.term(x + lay.off(xa), lay.ld(xa), false, x + lay.off(xb), lay.ld(xb), true,
                                lay.blk[xa].cols, 1.0);
                    }
                } else {
                    for (int il = 0; il < (int)lay.L.q.size(); ++il)
                        for (int s1 = 0; s1 < 4; ++s1) {
                            int xa = lay.idx[(il * 4 + s1) * 4 + pa.a];
                            int xb = lay.idx[(il * 4 + s1) * 4 + pb.a];
                            if (xa < 0 || xb < 0 || lay.blk[xa].jr != pa.b || lay.blk[xb].jr != pb.b) continue;
                            gr.term(x + lay.off(xa), lay.ld(xa), true, x + lay.off(xb), lay.ld(xb), false,
                                    lay.L.d[il], 1.0);
                        }
                }
            }
        ++g;
    }
    gr.upload();
    gr.run();
    // tridiagonal reduction and all eigenvalues: one launch per kernel variant
    // (by whether the matrix fits in LDS)
    size_t tsz = 0;
    std::vector<size_t> toff(ng);
    for (int q = 0; q < ng; ++q) {
        toff[q] = tsz;
        tsz += dev::eig_work(gdim[q]);
    }
    eigT_.ensure(std::max<size_t>(tsz, 1));
    std::vector<dev::EigJob> all(ng);
    for (int q = 0; q < ng; ++q)
        all[q] = {rho_.p + goff[q], eigV_.p + goff[q], eigw_.p + woff[q], eigT_.p + toff[q], gdim[q], 0};
    {
        std::vector<dev::EigJob> jobs[2];
        int nmax[2] = {0, 0};
        for (int q = 0; q < ng; ++q) {
            if (gdim[q] <= 0) continue;
            const int c = dev::eig_reduce_class(gdim[q]);
            jobs[c].push_back(all[q]);
            nmax[c] = std::max(nmax[c], gdim[q]);
        }
        DevArr<dev::EigJob> dj[2];
        for (int c = 0; c < 2; ++c) {
            dj[c].upload(jobs[c]);
            if (!jobs[c].empty()) dev::eig_reduce(dj[c].p, (int)jobs[c].size(), nmax[c]);
        }
    }
    std::vector<double> wall(std::max<size_t>(wsz, 1));
    dev::d2h(wall.data(), eigw_.p, wsz * sizeof(double));
    std::vector<std::vector<double>> w(ng);
    for (int q = 0; q < ng; ++q) w[q].assign(wall.begin() + woff[q], wall.begin() + woff[q] + gdim[q]);
    sel = select_states(w, M);
    // orthonormal bases of the kept subspaces (first kept[q] columns of each
    // density matrix's buffer)
    {
        std::vector<dev::EigJob> jobs[2];
        int nmax[2] = {0, 0}, kmax[2] = {0, 0};
        for (int q = 0; q < ng; ++q) {
            if (sel.kept[q] <= 0) continue;
            dev::EigJob j = all[q];
            j.k = sel.kept[q];
            const int c = dev::eig_vectors_class(j.n, j.k);
            jobs[c].push_back(j);
            nmax[c] = std::max(nmax[c], j.n);
            kmax[c] = std::max(kmax[c], j.k);
        }
        eigS_.ensure(1);
        int* status = reinterpret_cast<int*>(eigS_.p);
        check_eig_status();  // the previous window's flag, before it is reset
        dev::zero(status, sizeof(int));
        DevArr<dev::EigJob> dj[2];
        for (int c = 0; c < 2; ++c) {
            dj[c].upload(jobs[c]);
            if (!jobs[c].empty()) dev::eig_vectors(dj[c].p, (int)jobs[c].size(), nmax[c], kmax[c], status);
        }
        if (!eig_status_h_) {
            eig_status_h_ = static_cast<int*>(dev::host_alloc(sizeof(int)));
            eig_ev_ = dev::event_create();
        }
        dev::d2h_async(eig_status_h_, status, sizeof(int));
        dev::event_record(eig_ev_);
        eig_pending_ = true;
    }
    }  // !zero
    Bond nb;
    std::vector<int> gid;  // new sector -> group
    for (int q = 0; q < ng; ++q)
        if (sel.kept[q] > 0) {
            nb.q.push_back(gq[q]);
            nb.d.push_back(sel.kept[q]);
            gid.push_back(q);
        }
    if (nb.q.empty()) throw err(MPSPT_E_STATE, "truncation kept no states (zero two-site tensor)");
    std::vector<std::vector<Part>*> gparts;
    for (auto& kv : groups) gparts.push_back(&kv.second);
    const double* EV = rho_.p;  // kept bases replace the density matrices
    if (forward) {
        Site An = make_site(lay.L, nb);
        AxpyBatch cp;
        for (size_t b = 0; b < An.blk.size(); ++b) {
            const auto& B = An.blk[b];
            int q = gid[B.jr];
            cp.group(An.at((int)b), An.ld((int)b), B.rows, B.cols, false);
            for (const auto& p : *gparts[q])
                if (p.a == B.il && p.b == B.s) cp.term(EV + goff[q] + (size_t)p.off * gdim[q], gdim[q], false, 1.0);
        }
        C = make_site(nb, lay.R);
        GemmBatch gc;
        for (size_t b = 0; b < C.blk.size(); ++b) {
            const auto& B = C.blk[b];
            int q = gid[B.il];
            gc.group(C.at((int)b), C.ld((int)b), B.rows, B.cols, false);
            for (const auto& p : *gparts[q]) {
                int xb = lay.idx[(p.a * 4 + p.b) * 4 + B.s];
                if (xb < 0) continue;
                gc.term(EV + goff[q] + (size_t)p.off * gdim[q], gdim[q], true, x + lay.off(xb), lay.ld(xb), false,
                        p.dim, 1.0);
            }
        }
        cp.upload();
        gc.upload();
        // zero blocks with no terms are written by the kernels (overwrite mode)
        cp.run();
        gc.run();
        A_[i] = std::move(An);
    } else {
        Site An = make_site(nb, lay.R);
        AxpyBatch cp;
        for (size_t b = 0; b < An.blk.size(); ++b) {
            const auto& B = An.blk[b];
            int q = gid[B.il];
            cp.group(An.at((int)b), An.ld((int)b), B.rows, B.cols, false);
            for (const auto& p : *gparts[q])
                if (p.a == B.s && p.b == B.jr) cp.term(EV + goff[q] + (size_t)p.off * gdim[q], gdim[q], true, 1.0);
        }
        C = make_site(lay.L, nb);
        GemmBatch gc;
        for (size_t b = 0; b < C.blk.size(); ++b) {
            const auto& B = C.blk[b];
            int q = gid[B.jr];
            gc.group(C.at((int)b), C.ld((int)b), B.rows, B.cols, false);
            for (const auto& p : *gparts[q]) {
                int xb = lay.idx[(B.il * 4 + B.s) * 4 + p.a];
                if (xb < 0 || lay.blk[xb].jr != p.b) continue;
                gc.term(x + lay.off(xb), lay.ld(xb), false, EV + goff[q] + (size_t)p.off * gdim[q], gdim[q], false,
                        p.dim, 1.0);
            }
        }
        cp.upload();
        gc.upload();
        cp.run();
        gc.run();
        A_[i + 1] = std::move(An);
    }
    return sel.disc;
}

void Engine::upd_left(int i) {
    if ((int)env_plans_[0].size() < n_) for (auto& v : env_plans_) v.resize(n_);
    env_left(LH_[i + 1], LH_[i], A_[i], A_[i], mpo_h0_, i, &env_plans_[0][i]);
    if (!gs_) env_left(LV_[i + 1], LV_[i], A_[i], P0_[i], mpo_v_, i, &env_plans_[1][i]);
}

void Engine::upd_right(int i) {
    if ((int)env_plans_[0].size() < n_) for (auto& v : env_plans_) v.resize(n_);
    env_right(RH_[i], RH_[i + 1], A_[i], A_[i], mpo_h0_, i, &env_plans_[2][i]);
    if (!gs_) env_right(RV_[i], RV_[i + 1], A_[i], P0_[i], mpo_v_, i, &env_plans_[3][i]);
}

// ---------------------------------------------------------- local solve
int Engine::solve(int i, double& e2) {
    const Two& lay = xlay_;
    const size_t n = lay.size;
    for (DevBuf* b : {&x_, &b_, &d_, &r_, &z_, &p_, &q_}) b->ensure(std::max<size_t>(n, 1));
    ensure_partials();
    scal_.ensure(dev::S_N);
    double t = dev::now();
    const TwoOp& O = twoop(0, i);
    const TwoOp& Ov = twoop(1, i);
    res_.t_phase[0] += dev::now() - t;
    t = dev::now();
    effop(1, i, LV_[i], RV_[i + 2], Ov, P0x_lay_[i], P0x_[i].p, lay, b_.p).run();
    build_diag(i, LH_[i], RH_[i + 2], O, lay, d_.p, -E0_);
    const EffOp& sig = effop(0, i, LH_[i], RH_[i + 2], O, lay, p_.p, lay, q_.p);
    const int nb = (precond_ == 1 || harvest_) ? precond_blocks(lay) : 0;
    res_.t_phase[1] += dev::now() - t;
    t = dev::now();
    struct PhaseTimer {
        double t0;
        double& acc;
        ~PhaseTimer() { acc += dev::now() - t0; }
    } cg_timer{t, res_.t_phase[2]};
    auto apply = [&]() {
        sig.run();
        dev::cg_shift_dot(q_.p, p_.p, E0_, n, scal_.p, partials_.p);
        res_.sigma_calls++;
        res_.flops += sig.flops;
        res_.bytes += sig.bytes;
    };
    // Reduced precision: the CG iterations apply the operator on FP32 copies
    // of the environments and the direction; every restart recomputes the
    // residual -b - A x in FP64 (iterative refinement), so the converged x
    // meets the same FP64 residual test as the plain solve.
    const bool lo = precision_ != 0;
    dev::BasesF fb{};
    if (lo) {
        const Env& L = LH_[i];
        const Env& R = RH_[i + 2];
        auto words = [](size_t floats) { return std::max<size_t>((floats + 1) / 2, 1); };
        lf_.ensure(words(L.size));
        rf_.ensure(words(R.size));
        pf_.ensure(words(n));
        qf_.ensure(words(n));
        fb.p[0] = reinterpret_cast<float*>(lf_.p);
        fb.p[1] = reinterpret_cast<float*>(rf_.p);
        fb.p[2] = reinterpret_cast<float*>(pf_.p);
        fb.p[3] = reinterpret_cast<float*>(qf_.p);
        dev::to_f32(fb.p[0], L.data.p, L.size);
        dev::to_f32(fb.p[1], R.data.p, R.size);
    }
    auto apply_inner = [&]() {
        if (!lo) return apply();
        sig.run_lo(fb, precision_);
        dev::cg_shift_dot_lo(q_.p, fb.p[3], p_.p, E0_, n, scal_.p, partials_.p);
        res_.sigma_calls++;
        res_.sigma_lo_calls++;
        res_.flops += sig.flops;
        res_.bytes += sig.bytes / 2;
    };
    double sc[dev::S_N];
    // start from the best multiple of the guess: x0 <- a x0, a = -x0.b / x0.A x0
    dev::d2d(x_.p, xg_.p, n * sizeof(double));
    dev::d2d(p_.p, x_.p, n * sizeof(double));
    apply();
    dev::dot(x_.p, b_.p, n, scal_.p, dev::S_DOT, partials_.p);
    dev::d2h(sc, scal_.p, sizeof(sc));
    if (sc[dev::S_PQ] > 0.0) {
        const double a = -sc[dev::S_DOT] / sc[dev::S_PQ];
        dev::axpby(x_.p, x_.p, 0.0, a, n);
        dev::axpby(q_.p, q_.p, 0.0, a, n);
    }
    int it = 0;
    bool solved = false;
    x_zero_ = false;
    // CG on A x = -b; convergence is confirmed on the true residual -b - A x
    // and CG restarts from x when the updated residual has drifted.
    const int max_restarts = lo ? 12 : 4;
    for (int restart = 0;; ++restart) {
        dev::cg_init(r_.p, z_.p, p_.p, b_.p, q_.p, d_.p, n, scal_.p, partials_.p);
        if (restart == 0 && precond_ == 1) {
            // block scales from the initial residual, then the scaled start
            precond_apply(i, nb);
            dev::cg_init(r_.p, z_.p, p_.p, b_.p, q_.p, d_.p, n, scal_.p, partials_.p);
        }
        if (restart == 0 && harvest_) {  // initial residual and state, for the targets
            pr0_.ensure(std::max<size_t>(n, 1));
            px0_.ensure(std::max<size_t>(n, 1));
            dev::d2d(pr0_.p, r_.p, n * sizeof(double));
            dev::d2d(px0_.p, x_.p, n * sizeof(double));
        }
        dev::d2h(sc, scal_.p, sizeof(sc));
        const double bb = sc[dev::S_BB];
        double rr = sc[dev::S_RR];
        if (bb == 0.0) {
            dev::zero(x_.p, n * sizeof(double));
            dev::zero(q_.p, n * sizeof(double));
            x_zero_ = true;
            solved = true;
            break;
        }
        if (rr <= cg_tol2_ * bb) {
            solved = true;
            break;
        }
        if (it >= cg_max_ || restart == max_restarts) break;  // not converged: flagged below
        if (restart > 0) res_.refinements++;
        // an inner (reduced-precision) round stops once it has cut its own
        // starting residual by inner_rel_tol, or at the final tolerance
        const double stop2 = std::max(cg_tol2_ * bb, inner_tol2_ * rr);
        if (lo) dev::to_f32(fb.p[2], p_.p, n);
        // Iteration k's scalars go to pinned slot k % 2 (the update kernel
        // writes them there itself); the host examines
        // iteration k - 1 while iteration k runs, so the device never waits
        // for the host.  When k - 1 has converged, x carries the one extra
        // iteration k.
        if (!hsc_) {
            hsc_ = static_cast<double*>(dev::host_alloc(2 * dev::S_N * sizeof(double)));
            for (void*& e : ev_) e = dev::event_create();
        }
        int cur = dev::S_RZ0, nxt = dev::S_RZ1;
        int seen = it;  // iterations before `seen` have been examined
        bool conv = false;
        while (!conv) {
            if (it < cg_max_) {
                apply_inner();
                dev::cg_update(x_.p, r_.p, z_.p, p_.p, q_.p, d_.p, n, scal_.p, cur, nxt, partials_.p,
                               hsc_ + (it & 1) * dev::S_N);
                dev::event_record(ev_[it & 1]);
                if (lo) dev::cg_direction_lo(p_.p, fb.p[2], z_.p, n, scal_.p, cur, nxt);
                else dev::cg_direction(p_.p, z_.p, n, scal_.p, cur, nxt);
                std::swap(cur, nxt);
                ++it;
            } else if (seen == it) {
                break;  // iteration cap
            }
            // examine the oldest unexamined iteration, unless it is the one just issued
            while (seen < it && (seen < it - 1 || it >= cg_max_)) {
                dev::event_wait(ev_[seen & 1]);
                const double* h = hsc_ + (seen & 1) * dev::S_N;
                ++seen;
                if (!(h[dev::S_PQ] > 0.0))
                    throw err(MPSPT_E_INDEFINITE, "CG met p.Ap <= 0: H0 - E0 is not positive definite on the local space");
                rr = h[dev::S_RR];
                if (rr <= stop2) {
                    conv = true;
                    break;
                }
            }
        }
        dev::d2d(p_.p, x_.p, n * sizeof(double));
        apply();  // q = A x, scal[PQ] = x.A x
    }
    if (!solved) res_.flags |= 1;  // iteration cap, or restarts exhausted above the tolerance
    // Hylleraas value of x: x.(A x) + 2 x.b  (q = A x from the last application)
    dev::d2d(p_.p, x_.p, n * sizeof(double));
    dev::cg_shift_dot(q_.p, p_.p, 0.0, n, scal_.p, partials_.p);
    dev::dot(x_.p, b_.p, n, scal_.p, dev::S_DOT, partials_.p);
    dev::d2h(sc, scal_.p, sizeof(sc));
    e2 = sc[dev::S_PQ] + 2.0 * sc[dev::S_DOT];
    if (harvest_) harvest_window(i, nb);
    return it;
}

void Engine::next_guess(int i, bool forward, Site& C) {
    Two lay;
    if (forward) {
        if (i < n_ - 2) {
            lay = make_two(C.L, A_[i + 2].R, &adm_[i + 2]);
            xg_.ensure(std::max<size_t>(lay.size, 1));
            contract_sites(C, A_[i + 2], lay, xg_.p);
        } else {
            lay = make_two(A_[i].L, C.R, &adm_[i + 1]);
            xg_.ensure(std::max<size_t>(lay.size, 1));
            contract_sites(A_[i], C, lay, xg_.p);
            A_[i + 1] = std::move(C);
        }
    } else {
        if (i > 0) {
            lay = make_two(A_[i - 1].L, C.R, &adm_[i]);
            xg_.ensure(std::max<size_t>(lay.size, 1));
            contract_sites(A_[i - 1], C, lay, xg_.p);
        } else {
            lay = make_two(C.L, A_[1].R, &adm_[1]);
            xg_.ensure(std::max<size_t>(lay.size, 1));
            contract_sites(C, A_[1], lay, xg_.p);
            A_[0] = std::move(C);
        }
    }
    xlay_ = std::move(lay);
}

double Engine::e3_final(int window) {
    if (mpo_e3_.n == 0) mpo_e3_ = build_mpo(OpKind::VPsi1, k_a_, k_v_, h_, eri_, eps_);
    const MPO& mf = mpo_e3_;
    Env R = trivial_env(A_[n_ - 1].R, A_[n_ - 1].R);
    for (int j = n_ - 1; j >= window + 2; --j) {
        Env R2;
        env_right(R2, R, A_[j], A_[j], mf, j);
        R = std::move(R2);
    }
    Env L = trivial_env(A_[0].L, A_[0].L);
    if (window != 0) throw err(MPSPT_E_STATE, "E3 is evaluated at the first window");
    TwoOp O = make_twoop(mf, window);
    EffOp op;
    build_effop(op, L, R, O, last_lay_, x_.p, last_lay_, q_.p);
    op.run();
    dev::dot(x_.p, q_.p, last_lay_.size, scal_.p, dev::S_DOT, partials_.p);
    double sc[dev::S_N];
    dev::d2h(sc, scal_.p, sizeof(sc));
    return sc[dev::S_DOT];
}

void Engine::start(const std::vector<Bond>& bonds, const std::vector<std::vector<double>>& sites, int M) {
    A_.clear();
    for (int i = 0; i < n_; ++i) {
        A_.push_back(make_site(bonds[i], bonds[i + 1]));
        load_site(A_[i], sites[i]);
    }
    for (auto* v : {&LH_, &RH_, &LV_, &RV_}) {
        v->clear();
        v->resize(n_ + 1);
    }
    LH_[0] = trivial_env(A_[0].L, A_[0].L);
    RH_[n_] = trivial_env(A_[n_ - 1].R, A_[n_ - 1].R);
    if (!gs_) {
        LV_[0] = trivial_env(A_[0].L, P0_[0].L);
        RV_[n_] = trivial_env(A_[n_ - 1].R, P0_[n_ - 1].R);
    }
    // right-canonical start: backward pass without solves
    for (int i = n_ - 2; i >= 0; --i) {
        Two lay = make_two(A_[i].L, A_[i + 1].R, &adm_[i + 1]);
        x_.ensure(std::max<size_t>(lay.size, 1));
        contract_sites(A_[i], A_[i + 1], lay, x_.p);
        Site C;
        truncate(i, false, lay, x_.p, M, C);
        A_[i] = std::move(C);
        upd_right(i + 1);
    }
    xlay_ = make_two(A_[0].L, A_[1].R, &adm_[1]);
    xg_.ensure(std::max<size_t>(xlay_.size, 1));
    contract_sites(A_[0], A_[1], xlay_, xg_.p);
}

double Engine::run_sweeps(int M, int n_sweeps, int max_sweeps, double e_tol) {
    double e2 = 0;
    for (int sw = 0; sw < 64; ++sw) {
        double maxd = 0;
        for (int dir = 0; dir < 2; ++dir) {
            const bool fwd = dir == 0;
            for (int k = 0; k < n_ - 1; ++k) {
                const int i = fwd ? k : n_ - 2 - k;
                int it = gs_ ? davidson(i, e2) : solve(i, e2);
                res_.cg_iters += it;
                last_lay_ = xlay_;
                Site C;
                double t = dev::now();
                double disc = truncate(i, fwd, xlay_, x_.p, M, C, !gs_ && x_zero_);
                res_.t_phase[3] += dev::now() - t;
                t = dev::now();
                if (fwd) upd_left(i);
                else upd_right(i + 1);
                res_.t_phase[4] += dev::now() - t;
                t = dev::now();
                next_guess(i, fwd, C);
                dev::sync();
                res_.t_phase[5] += dev::now() - t;
                trace_.push_back({e2, disc, dev::now() - t0_, it});
                maxd = std::max(maxd, disc);
                res_.n_steps++;
            }
        }
        res_.e2_sweep.push_back(e2);
        res_.n_sweeps = sw + 1;
        res_.max_disc = maxd;
        if (n_sweeps > 0) {
            if (res_.n_sweeps >= n_sweeps) break;
        } else {
            size_t ns = res_.e2_sweep.size();
            if (ns > 1 && std::fabs(res_.e2_sweep[ns - 1] - res_.e2_sweep[ns - 2]) < e_tol) break;
            if (res_.n_sweeps >= max_sweeps) break;
        }
    }
    check_eig_status();
    return e2;
}

SweepResult Engine::sweep(const SweepParams& p) {
    if (!have_psi1) throw err(MPSPT_E_STATE, "load integrals, the H0 partition, Psi0 and a Psi1 guess first");
    if (p.M1 < 1) throw err(MPSPT_E_ARG, "M1 must be positive");
    drop_eig_status();
    res_ = SweepResult();
    res_.e0 = E0_;
    trace_.clear();
    cg_tol2_ = p.cg_rel_tol * p.cg_rel_tol;
    cg_max_ = p.cg_max_iter;
    if (p.precond != 0 && p.precond != 1) throw err(MPSPT_E_ARG, "precond must be 0 (Jacobi) or 1 (learned)");
    if (p.precond == 1 && !mlp_set_) throw err(MPSPT_E_STATE, "load the preconditioner network first");
    if (p.precond == 1 && harvest_) throw err(MPSPT_E_ARG, "harvesting needs the Jacobi preconditioner");
    precond_ = p.precond;
    if (p.precision < 0 || p.precision > 2) throw err(MPSPT_E_ARG, "precision must be 0 (FP64), 1 (FP32) or 2 (BF16x3)");
    if (!(p.inner_rel_tol >= 0.0 && p.inner_rel_tol < 1.0)) throw err(MPSPT_E_ARG, "inner_rel_tol must lie in [0, 1)");
    precision_ = p.precision;
    {
        // default inner reduction: a little above what the product's rounding allows
        const double inner = p.inner_rel_tol > 0 ? p.inner_rel_tol : (precision_ == 1 ? 1e-5 : 1e-3);
        inner_tol2_ = precision_ ? inner * inner : 0.0;
    }
    clear_plans();  // plans are reused across the sweeps of one call only
    dev::sync();
    t0_ = dev::now();
    start(psi1_bonds_, psi1_guess_, p.M1);
    res_.e2 = run_sweeps(p.M1, p.n_sweeps, p.max_sweeps, p.e_tol);
    dev::sync();
    res_.t_total = dev::now() - t0_;
    if (p.compute_e3) res_.e3 = e3_final(0);
    return res_;
}

double Engine::ground_state(int n_elec, int two_sz, const std::vector<Bond>& bonds,
                            const std::vector<std::vector<double>>& sites, int M0, int n_sweeps, double e_tol) {
    drop_eig_status();
    if (!have_part) throw err(MPSPT_E_STATE, "load integrals and the H0 partition before the ground-state sweep");
    if ((int)bonds.size() != k_a_ + 1 || (int)sites.size() != k_a_) throw err(MPSPT_E_ARG, "guess needs k_a sites");
    if (k_a_ < 2) throw err(MPSPT_E_ARG, "the ground-state sweep needs at least two active orbitals");
    if (M0 < 1) throw err(MPSPT_E_ARG, "M0 must be positive");
    // admissible sectors of the active space alone
    std::vector<std::set<std::pair<int, int>>> left(k_a_ + 1), right(k_a_ + 1);
    left[0].insert({0, 0});
    right[k_a_].insert({0, 0});
    for (int i = 0; i < k_a_; ++i)
        for (auto& t : left[i])
            for (int s = 0; s < 4; ++s) left[i + 1].insert({t.first + site_dq(s).n, t.second + site_dq(s).s});
    for (int i = k_a_ - 1; i >= 0; --i)
        for (auto& t : right[i + 1])
            for (int s = 0; s < 4; ++s) right[i].insert({t.first + site_dq(s).n, t.second + site_dq(s).s});
    std::vector<std::set<QN>> adm(k_a_ + 1);
    for (int b = 0; b <= k_a_; ++b)
        for (auto& l : left[b])
            if (right[b].count({n_elec - l.first, two_sz - l.second})) adm[b].insert(QN{l.first, l.second});
    for (int b = 0; b <= k_a_; ++b)
        for (auto& q : bonds[b].q)
            if (!adm[b].count(q)) throw err(MPSPT_E_QN, "guess bond sector cannot reach the target (N, 2Sz)");
    // run the sweep on the active sites with H_act, then load the result as Psi0
    const int n_save = n_;
    MPO h0_save = std::move(mpo_h0_);
    std::vector<std::set<QN>> adm_save = std::move(adm_);
    gs_ = true;
    n_ = k_a_;
    mpo_h0_ = build_mpo(OpKind::HAct, k_a_, k_v_, h_, eri_, eps_);
    twoop_cache_[0].clear();
    clear_plans();
    adm_ = adm;
    res_ = SweepResult();
    trace_.clear();
    double e = 0;
    std::vector<Bond> out_b;
    std::vector<std::vector<double>> out_s;
    try {
        dev::sync();
        t0_ = dev::now();
        start(bonds, sites, M0);
        e = run_sweeps(M0, n_sweeps, 64, e_tol);
        for (int i = 0; i < n_; ++i) out_b.push_back(A_[i].L);
        out_b.push_back(A_[n_ - 1].R);
        for (int i = 0; i < n_; ++i) {
            std::vector<double> v;
            int Dl, Dr;
            site_dense(0, i, v, Dl, Dr);
            out_s.push_back(std::move(v));
        }
    } catch (...) {
        gs_ = false;
        n_ = n_save;
        mpo_h0_ = std::move(h0_save);
        twoop_cache_[0].clear();
        clear_plans();
    clear_plans();
        adm_ = std::move(adm_save);
        A_.clear();
        throw;
    }
    gs_ = false;
    n_ = n_save;
    mpo_h0_ = std::move(h0_save);
    twoop_cache_[0].clear();
    clear_plans();
    adm_ = std::move(adm_save);
    A_.clear();
    gs_trace_ = trace_;
    set_psi0(n_elec, two_sz, out_b, out_s);
    return e;
}

// Lowest eigenpair of H_eff at window i by Davidson with the Jacobi
// preconditioner; the normalised eigenvector is left in x_.
int Engine::davidson(int i, double& e) {
    const Two& lay = xlay_;
    const size_t n = lay.size;
    constexpr int kMax = 16;
    for (DevBuf* b : {&x_, &d_, &r_, &z_, &p_, &q_}) b->ensure(std::max<size_t>(n, 1));
    dav_V_.ensure(std::max<size_t>(n, 1) * kMax);
    dav_AV_.ensure(std::max<size_t>(n, 1) * kMax);
    ensure_partials();
    scal_.ensure(dev::S_N);
    const TwoOp& O = twoop(0, i);
    build_diag(i, LH_[i], RH_[i + 2], O, lay, d_.p, 0.0);
    const EffOp& sig = effop(0, i, LH_[i], RH_[i + 2], O, lay, p_.p, lay, q_.p);
    double sc[dev::S_N];
    auto dotp = [&](const double* a, const double* b) {
        dev::dot(a, b, n, scal_.p, dev::S_DOT, partials_.p);
        dev::d2h(sc, scal_.p, sizeof(sc));
        return sc[dev::S_DOT];
    };
    auto Vk = [&](int k) { return dav_V_.p + (size_t)k * n; };
    auto AVk = [&](int k) { return dav_AV_.p + (size_t)k * n; };
    auto applyA = [&](const double* v, double* out) {
        dev::d2d(p_.p, v, n * sizeof(double));
        sig.run();
        dev::d2d(out, q_.p, n * sizeof(double));
        res_.sigma_calls++;
        res_.flops += sig.flops;
        res_.bytes += sig.bytes;
    };
    // start from the guess
    dev::d2d(Vk(0), xg_.p, n * sizeof(double));
    double nrm = std::sqrt(dotp(Vk(0), Vk(0)));
    if (!(nrm > 0)) throw err(MPSPT_E_STATE, "zero guess in the ground-state sweep");
    dev::axpby(Vk(0), Vk(0), 0.0, 1.0 / nrm, n);
    applyA(Vk(0), AVk(0));
    std::vector<double> Hs(kMax * kMax, 0.0);
    Hs[0] = dotp(Vk(0), AVk(0));
    int m = 1, it = 0;
    double theta = Hs[0];
    std::vector<double> cvec(1, 1.0);
    for (; it < cg_max_; ++it) {
        // Ritz pair of the projected matrix (host, m <= 16)
        std::vector<double> a(m * m), v(m * m, 0.0);
        for (int r = 0; r < m; ++r)
            for (int c = 0; c < m; ++c) a[r * m + c] = 0.5 * (Hs[r * kMax + c] + Hs[c * kMax + r]);
        for (int r = 0; r < m; ++r) v[r * m + r] = 1.0;
        for (int swp = 0; swp < 100; ++swp) {
            double off = 0;
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < m; ++c)
                    if (r != c) off += a[r * m + c] * a[r * m + c];
            if (off < 1e-30) break;
            for (int pp = 0; pp < m; ++pp)
                for (int qq = pp + 1; qq < m; ++qq) {
                    double apq = a[pp * m + qq];
                    if (apq == 0) continue;
                    double tau = (a[qq * m + qq] - a[pp * m + pp]) / (2 * apq);
                    double t = (tau >= 0 ? 1 : -1) / (std::fabs(tau) + std::sqrt(1 + tau * tau));
                    double c = 1 / std::sqrt(1 + t * t), s = t * c;
                    for (int j = 0; j < m; ++j) {
                        double x1 = a[pp * m + j], x2 = a[qq * m + j];
                        a[pp * m + j] = c * x1 - s * x2;
                        a[qq * m + j] = s * x1 + c * x2;
                    }
                    for (int j = 0; j < m; ++j) {
                        double x1 = a[j * m + pp], x2 = a[j * m + qq];
                        a[j * m + pp] = c * x1 - s * x2;
                        a[j * m + qq] = s * x1 + c * x2;
                        double v1 = v[j * m + pp], v2 = v[j * m + qq];
                        v[j * m + pp] = c * v1 - s * v2;
                        v[j * m + qq] = s * v1 + c * v2;
                    }
                }
        }
        int lo = 0;
        for (int r = 1; r < m; ++r)
            if (a[r * m + r] < a[lo * m + lo]) lo = r;
        theta = a[lo * m + lo];
        cvec.assign(m, 0.0);
        for (int r = 0; r < m; ++r) cvec[r] = v[r * m + lo];
        // x = V c, Ax = AV c, residual r = Ax - theta x
        dev::zero(x_.p, n * sizeof(double));
        dev::zero(z_.p, n * sizeof(double));
        for (int r = 0; r < m; ++r) {
            dev::axpby(x_.p, Vk(r), cvec[r], 1.0, n);
            dev::axpby(z_.p, AVk(r), cvec[r], 1.0, n);
        }
        dev::d2d(r_.p, z_.p, n * sizeof(double));
        dev::axpby(r_.p, x_.p, -theta, 1.0, n);
        double rn = std::sqrt(dotp(r_.p, r_.p));
        if (rn < dav_tol_) break;
        if (m == kMax) {  // restart from the current Ritz vector
            dev::d2d(Vk(0), x_.p, n * sizeof(double));
            dev::d2d(AVk(0), z_.p, n * sizeof(double));
            Hs.assign(kMax * kMax, 0.0);
            Hs[0] = theta;
            m = 1;
        }
        // correction t = r / (theta - D), orthogonalised twice against V
        dev::davidson_precond(Vk(m), r_.p, d_.p, theta, n);
        for (int pass = 0; pass < 2; ++pass)
            for (int r = 0; r < m; ++r) {
                double ov = dotp(Vk(r), Vk(m));
                dev::axpby(Vk(m), Vk(r), -ov, 1.0, n);
            }
        double tn = std::sqrt(dotp(Vk(m), Vk(m)));
        if (!(tn > 1e-14)) break;
        dev::axpby(Vk(m), Vk(m), 0.0, 1.0 / tn, n);
        applyA(Vk(m), AVk(m));
        for (int r = 0; r <= m; ++r) {
            Hs[r * kMax + m] = dotp(Vk(r), AVk(m));
            Hs[m * kMax + r] = Hs[r * kMax + m];
        }
        ++m;
    }
    double xn = std::sqrt(dotp(x_.p, x_.p));
    dev::axpby(x_.p, x_.p, 0.0, 1.0 / xn, n);
    e = theta;
    return it;
}

const Bond& Engine::bond(int which, int b) const {
    if (b < 0 || b > n_) throw err(MPSPT_E_ARG, "bond index out of range");
    if (which == 0) {
        if (A_.empty()) throw err(MPSPT_E_STATE, "no Psi1 yet");
        return b < n_ ? A_[b].L : A_[n_ - 1].R;
    }
    if (P0_.empty()) throw err(MPSPT_E_STATE, "no Psi0 yet");
    return b < n_ ? P0_[b].L : P0_[n_ - 1].R;
}

void Engine::site_dense(int which, int i, std::vector<double>& out, int& Dl, int& Dr) const {
    const std::vector<Site>& v = which == 0 ? A_ : P0_;
    if (i < 0 || i >= (int)v.size()) throw err(MPSPT_E_ARG, "site index out of range");
    const Site& s = v[i];
    Dl = s.L.total();
    Dr = s.R.total();
    std::vector<double> host(s.size);
    if (s.size) dev::d2h(host.data(), s.data.p, s.size * sizeof(double));
    out.assign((size_t)Dl * 4 * Dr, 0.0);
    std::vector<int> ol(s.L.q.size() + 1, 0), orr(s.R.q.size() + 1, 0);
    for (size_t a = 0; a < s.L.q.size(); ++a) ol[a + 1] = ol[a] + s.L.d[a];
    for (size_t a = 0; a < s.R.q.size(); ++a) orr[a + 1] = orr[a] + s.R.d[a];
    for (const auto& B : s.blk)
        for (int r = 0; r < B.rows; ++r)
            for (int c = 0; c < B.cols; ++c)
                out[((size_t)(ol[B.il] + r) * 4 + B.s) * Dr + orr[B.jr] + c] =
                    host[s.po[B.il] + B.col + (size_t)r * s.pw[B.il] + c];
}

}  // namespace mpspt
