// Temporal basis pairs of order p (see temporal.h).
#include "temporal.h"

#include <cmath>

namespace qhp {

namespace {

using Poly = std::vector<double>;  // ascending powers

Poly mul(const Poly &a, const Poly &b)
{
    Poly r(a.size() + b.size() - 1, 0.0);
    for (size_t i = 0; i < a.size(); ++i)
        for (size_t j = 0; j < b.size(); ++j) r[i + j] += a[i] * b[j];
    return r;
}

Poly add(const Poly &a, const Poly &b, double sb = 1.0)
{
    Poly r(std::max(a.size(), b.size()), 0.0);
    for (size_t i = 0; i < a.size(); ++i) r[i] += a[i];
    for (size_t i = 0; i < b.size(); ++i) r[i] += sb * b[i];
    return r;
}

double eval(const Poly &a, double u)
{
    double v = 0.0;
    for (size_t i = a.size(); i-- > 0;) v = v * u + a[i];
    return v;
}

// c(alpha + beta v) as a polynomial in v
Poly compose_linear(const Poly &c, double alpha, double beta)
{
    Poly r{0.0}, pw{1.0};
    for (double ci : c) {
        r = add(r, pw, ci);
        pw = mul(pw, Poly{alpha, beta});
    }
    return r;
}

Poly derivative(const Poly &a)
{
    if (a.size() <= 1) return Poly{0.0};
    Poly r(a.size() - 1);
    for (size_t i = 1; i < a.size(); ++i) r[i - 1] = i * a[i];
    return r;
}

Poly antiderivative(const Poly &a)
{
    Poly r(a.size() + 1, 0.0);
    for (size_t i = 0; i < a.size(); ++i) r[i + 1] = a[i] / (double)(i + 1);
    return r;
}

Poly sized(Poly a, size_t n)
{
    a.resize(n, 0.0);
    return a;
}

}  // namespace

TemporalBasis::TemporalBasis(int order) : p(order)
{
    // h_0 pieces in u: Lagrange through nodes m-p..m, 1 at 0
    for (int m = 0; m <= p; ++m) {
        Poly c{1.0};
        for (int n = m - p; n <= m; ++n)
            if (n != 0) c = mul(c, Poly{-(double)n / (0.0 - n), 1.0 / (0.0 - n)});
        h.push_back(c);
    }
    for (int m = 0; m <= p; ++m) dh.push_back(sized(compose_linear(derivative(h[m]), m, -1.0), p));
    // q_0 pieces in u: integral from u = -1 of h_0(v) - h_0(v - 1), continuous
    double left = 0.0;
    for (int m = 0; m <= p + 1; ++m) {
        Poly g = m <= p ? h[m] : Poly{0.0};
        if (m >= 1) g = add(g, compose_linear(h[m - 1], -1.0, 1.0), -1.0);  // h_0(u - 1) on piece m
        Poly G = antiderivative(g);
        G[0] += left - eval(G, m - 1.0);
        left = eval(G, (double)m);
        q.push_back(sized(compose_linear(G, m, -1.0), p + 2));
    }
}

double TemporalBasis::mf(int k, int m, int a) const
{
    if (m < 0 || m > p || a < 0 || a > p) return 0.0;
    // h_0(m - x) + (k - m + x) dh_0/du(m - x) in x
    const Poly hx = compose_linear(h[m], m, -1.0);
    const Poly dx = compose_linear(derivative(h[m]), m, -1.0);
    const Poly c = add(hx, mul(Poly{(double)(k - m), 1.0}, dx));
    return a < (int)c.size() ? c[a] : 0.0;
}

}  // namespace qhp
