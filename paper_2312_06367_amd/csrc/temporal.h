// Temporal basis pairs (h_0, q_0) of order p and the coefficients that turn
// x-weighted shell moments into the raw lag matrices (Sec. IV-A; the Remark
// of Sec. IV-B: q_i' = (h_i - h_{i+1})/dt).
//
// h_0 of order p: on [(m-1) dt, m dt), m = 0..p, the Lagrange polynomial
// through the nodes (m-p) dt .. m dt that is 1 at t = 0 (p = 1: the hat
// function).  q_0 = integral of (h_0(s) - h_0(s - dt))/dt, on m = 0..p+1.
// A source at distance R in shell j (x = R/dt - j) tested at t = k dt sees
// the retarded time in interval m = k - j at u = t/dt = m - x, so
//   A_k  = -(1/dt) sum_m sum_{a<p}   dh[m][a] V^(a)_{k-m}
//   Sq_k = sum_m sum_{a<p+2}         q[m][a]  S^(a)_{k-m}
//   C_k  = G/2 [k = 0] + sum_m sum_{a<=p} mf(k, m, a) N^(a)_{k-m}
// with dh the x-coefficients of dh_0/du, q those of q_0 and mf those of
// h_0 + (R/dt) dh_0/du (the MFIE kernel h(tau)/R^3 + h'(tau)/R^2).
#pragma once

#include <vector>

namespace qhp {

struct TemporalBasis {
    int p = 1;
    std::vector<std::vector<double>> h;   // h_0 pieces in u, m = 0..p
    std::vector<std::vector<double>> dh;  // dh_0/du in x, m = 0..p (p coefficients)
    std::vector<std::vector<double>> q;   // q_0 in x, m = 0..p+1 (p + 2 coefficients)
    explicit TemporalBasis(int order);
    // x-coefficient a of h_0 + (R/dt) dh_0/du on interval m for lag k
    double mf(int k, int m, int a) const;
};

}  // namespace qhp
