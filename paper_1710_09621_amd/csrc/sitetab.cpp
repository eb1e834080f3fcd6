// Host construction of the site-local s-operator tables used by the fused hop epilogues.
//
// Per 4D site and per chirality half (P+ couples slice s to s-1 through L_+(m+), P- couples
// s to s+1 through L_-(m-) = L_+(m-)^T), the operators are products of
//   diagonal scalings, the shift (1 +/- L) and the inverse of a cyclic bidiagonal matrix
//   d_s x_s + e_s (S x)_s,   (S x)_s = x_{s+sig} or tau * x_{s+sig mod Ns} at the ring wrap.
// The inverse is evaluated on the device as a ring scan: with c_s = -(e_s/d_s) tw_s,
//   x_s = g_s/d_s + c_s x_{s+sig}  =>  x_s = (1 - prod c)^{-1} sum_j (prod_{i<j} c_{s+i sig}) g_{s+j sig}/d_{s+j sig},
// accumulated in log2(Ns) doubling steps with the tables q[k][s] = prod_{i<2^k} c_{s+i sig}.
//
//   A_T^{-1} = omega^{1/2} (1 + L) A^{-1} omega^{1/2},   A = (4 - m0) omega (1 + L) + (1 - L)
//   M        = omega^{-1/2} (1 - L) (1 + L)^{-1} omega^{-1/2}
//   A, omega (1 + L) and their transposes (shift only: the scan tables stay zero), for
//   D_odwf = A - (1/2) H omega (1 + L) and D_odwf^dag = A^dag - (1/2) (1 + L)^dag omega H^dag
// (A_T = 4 - m0 + M is the x-diagonal block of D_T in Eq.(DTm1m2); A is the same block of the
// optimal-DWF operator, A_T = omega^{-1/2} A (1 + L)^{-1} omega^{-1/2}), and their transposes.
#include <cmath>
#include <cstring>

#include "eofa_int.h"

namespace eofa {

namespace {

struct Ring {
    int Ns, sig;
    double tau;
    bool wrap(int s) const { return s + sig < 0 || s + sig >= Ns; }
    double tw(int s) const { return wrap(s) ? tau : 1.0; }
    int nb(int s) const { return ((s + sig) % Ns + Ns) % Ns; }
};

// q tables and kappa = 1/(1 - prod c) for x_s = h_s + c_s x_{s+sig}
double fill_scan(ChirTab& t, const Ring& r, const double* c) {
    int K = 0;
    while ((1 << K) < r.Ns) K++;
    for (int k = 0; k < 6; k++)
        for (int s = 0; s < MAXNS; s++) t.q[k][s] = 0.0;
    for (int k = 0; k < K; k++)
        for (int s = 0; s < r.Ns; s++) {
            double p = 1.0;
            for (int i = 0; i < (1 << k); i++) p *= c[(((s + i * r.sig) % r.Ns) + r.Ns) % r.Ns];
            t.q[k][s] = p;
        }
    double C = 1.0;
    for (int s = 0; s < r.Ns; s++) C *= c[s];
    return 1.0 / (1.0 - C);
}

void build_half(ChirTab& t, SiteKind kind, int Ns, double m0, const double* om, double m, int sigL) {
    std::memset(&t, 0, sizeof(t));
    const bool dag = (kind == SK_AINV_DAG || kind == SK_M_DAG || kind == SK_A_DAG || kind == SK_OM1L_DAG);
    Ring r{Ns, dag ? -sigL : sigL, -m};
    double c[MAXNS], kappa;
    switch (kind) {
    case SK_AINV: {
        for (int s = 0; s < Ns; s++) {
            double a = (4.0 - m0) * om[s] + 1.0, b = (4.0 - m0) * om[s] - 1.0;
            c[s] = -(b / a) * r.tw(s);
            t.pre[s] = std::sqrt(om[s]) / a;
            t.shf[s] = r.tw(s);
            t.mid[s] = 1.0;
        }
        kappa = fill_scan(t, r, c);
        for (int s = 0; s < Ns; s++) t.post[s] = std::sqrt(om[s]) * kappa;
        break;
    }
    case SK_AINV_DAG: {
        for (int s = 0; s < Ns; s++) {
            double a = (4.0 - m0) * om[s] + 1.0;
            double bn = (4.0 - m0) * om[r.nb(s)] - 1.0;
            c[s] = -(bn / a) * r.tw(s);
            t.pre[s] = std::sqrt(om[s]);
            t.shf[s] = r.tw(s);
            t.mid[s] = 1.0 / a;
        }
        kappa = fill_scan(t, r, c);
        for (int s = 0; s < Ns; s++) t.post[s] = std::sqrt(om[s]) * kappa;
        break;
    }
    case SK_A:        // A = (4 - m0) omega (1 + L) + (1 - L): y_s = a_s x_s + b_s tw x_{s+sig}, no solve
    case SK_A_DAG: {  // A^dag: y_s = a_s x_s + b_{s+sig} tw x_{s+sig}
        for (int s = 0; s < Ns; s++) {
            const double a = (4.0 - m0) * om[s] + 1.0;
            const double b = (4.0 - m0) * om[dag ? r.nb(s) : s] - 1.0;
            t.pre[s] = 1.0;
            t.mid[s] = 1.0;
            t.shf[s] = b * r.tw(s) / a;
            t.post[s] = a;
        }
        break;
    }
    case SK_OM1L:        // omega (1 + L): y_s = omega_s (x_s + tw x_{s+sig})
    case SK_OM1L_DAG: {  // (1 + L)^dag omega: y_s = omega_s x_s + tw omega_{s+sig} x_{s+sig}
        for (int s = 0; s < Ns; s++) {
            t.pre[s] = dag ? om[s] : 1.0;
            t.mid[s] = 1.0;
            t.shf[s] = r.tw(s);
            t.post[s] = dag ? 1.0 : om[s];
        }
        break;
    }
    case SK_M:
    case SK_M_DAG: {
        for (int s = 0; s < Ns; s++) {
            c[s] = -r.tw(s);
            t.pre[s] = 1.0 / std::sqrt(om[s]);
            t.shf[s] = -r.tw(s);
            t.mid[s] = 1.0;
        }
        kappa = fill_scan(t, r, c);
        for (int s = 0; s < Ns; s++) t.post[s] = kappa / std::sqrt(om[s]);
        break;
    }
    case SK_NKIND:  // not a table kind: the tables stay zero
        break;
    }
}

}  // namespace

void build_site_op(SiteOp& op, SiteKind kind, int Ns, double m0, const double* omega, double mp, double mm) {
    build_half(op.h[0], kind, Ns, m0, omega, mp, -1);  // P+ : L_+ couples s to s-1
    build_half(op.h[1], kind, Ns, m0, omega, mm, +1);  // P- : L_- couples s to s+1
}

}  // namespace eofa
