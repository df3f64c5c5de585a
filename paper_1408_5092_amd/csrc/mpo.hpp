// Matrix product operators of the Dyall H0 and of the perturbation V
// (Eq. mpo), assembled term by term from the integrals.
#pragma once
#include <cstdint>
#include <vector>

namespace mpspt {

struct QN {
    int n = 0, s = 0;  // particle number, 2 Sz
    bool operator==(const QN& o) const { return n == o.n && s == o.s; }
    bool operator!=(const QN& o) const { return !(*this == o); }
    bool operator<(const QN& o) const { return n != o.n ? n < o.n : s < o.s; }
    QN operator+(const QN& o) const { return {n + o.n, s + o.s}; }
    QN operator-(const QN& o) const { return {n - o.n, s - o.s}; }
};

// (dN, d2Sz) of the local states |0>, |up>, |dn>, |up dn>.
inline QN site_dq(int s) {
    static const QN d[4] = {{0, 0}, {1, 1}, {1, -1}, {2, 0}};
    return d[s];
}

struct MPOEntry {
    int cin, cout;   // channel at the left / right bond of the site
    double m[16];    // <s|op|t> at m[4 s + t]
};

struct MPO {
    int n = 0;                              // sites
    std::vector<int> dims;                  // channels per bond, n + 1 values
    std::vector<std::vector<QN>> dq;        // per bond: change the left part applies to the left block
    std::vector<std::vector<MPOEntry>> W;   // per site
};

// H0: Dyall H0; VPsi0: the terms of V = H - H0 that act on Psi0 (annihilators
// active); VFull: all of V; VPsi1: the terms of V that connect states with one
// or two virtual electrons (the number of virtual electrons changes by at most
// one), enough for <Psi1|V|Psi1>; HAct: H on the active sites alone.
enum class OpKind { H0, VPsi0, VFull, HAct, VPsi1 };

// Integrals of the whole orbital space (k = k_a + k_v): h[k*k], eri[k^4].
// HAct builds the active-space Hamiltonian on k_a sites only.
MPO build_mpo(OpKind kind, int k_a, int k_v, const std::vector<double>& h,
              const std::vector<double>& eri, const std::vector<double>& eps_virt);

}  // namespace mpspt
