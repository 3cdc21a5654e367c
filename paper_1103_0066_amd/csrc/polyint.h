// Exact integration of polynomials over the reference simplex, host only:
// rationals, barycentric monomials, the scalar Lagrange bases of degree 1 and
// 2, reference derivatives, and int_ref lambda^alpha = alpha! / (|alpha| + dim)!.
// Used where reference tensors are built a priori (Sec. 3.1): the form front
// end at plan creation and the table generator at build time.
#pragma once

#include <array>
#include <cstdint>
#include <map>
#include <numeric>
#include <vector>

namespace fei {
namespace poly {

// Rational with int64 parts (the values here stay far below the int64 range:
// denominators divide (4 + 3)! times small integers).
struct Rat {
    int64_t p = 0, q = 1;
    Rat() = default;
    Rat(int64_t a, int64_t b = 1) : p(a), q(b) { norm(); }
    void norm()
    {
        if (q < 0) { p = -p; q = -q; }
        const int64_t g = std::gcd(p < 0 ? -p : p, q);
        if (g > 1) { p /= g; q /= g; }
    }
    Rat operator+(const Rat &o) const { return Rat(p * o.q + o.p * q, q * o.q); }
    Rat operator*(const Rat &o) const { return Rat(p * o.p, q * o.q); }
    double value() const { return double(p) / double(q); }
};

using Mono = std::array<int, 4>;            // exponents of lambda_0 .. lambda_3
using Poly = std::map<Mono, Rat>;

inline void add_term(Poly &P, const Mono &m, const Rat &c)
{
    if (c.p == 0) return;
    auto it = P.find(m);
    if (it == P.end()) P.emplace(m, c);
    else {
        it->second = it->second + c;
        if (it->second.p == 0) P.erase(it);
    }
}

// Scalar Lagrange basis of degree 1 or 2 as barycentric polynomials: vertices
// a (P1: lambda_a; P2: 2 lambda_a^2 - lambda_a), then P2 edges (a, b), a < b,
// in the order (0,1), (0,2), .., (0,dim), (1,2), ..: 4 lambda_a lambda_b.
inline std::vector<Poly> lagrange_basis(int dim, int degree)
{
    const int nv = dim + 1;
    std::vector<Poly> B;
    for (int a = 0; a < nv; ++a) {
        Poly P;
        Mono m1{}; m1[a] = 1;
        if (degree == 1) {
            add_term(P, m1, Rat(1));
        } else {
            Mono m2{}; m2[a] = 2;
            add_term(P, m2, Rat(2));
            add_term(P, m1, Rat(-1));
        }
        B.push_back(P);
    }
    if (degree == 2)
        for (int a = 0; a < nv; ++a)
            for (int b = a + 1; b < nv; ++b) {
                Poly P;
                Mono m{}; m[a] = 1; m[b] = 1;
                add_term(P, m, Rat(4));
                B.push_back(P);
            }
    return B;
}

// d/dxi_mu of a barycentric polynomial: lambda_0 = 1 - sum xi, lambda_{mu+1} =
// xi_mu, so d/dxi_mu = d/dlambda_{mu+1} - d/dlambda_0.
inline Poly dxi(const Poly &P, int mu)
{
    Poly D;
    for (const auto &t : P) {
        for (int k : {mu + 1, 0}) {
            if (t.first[k] == 0) continue;
            Mono m = t.first;
            const int e = m[k]--;
            add_term(D, m, t.second * Rat(k == 0 ? -e : e));
        }
    }
    return D;
}

inline Poly mul(const Poly &A, const Poly &B)
{
    Poly P;
    for (const auto &a : A)
        for (const auto &b : B) {
            Mono m;
            for (int k = 0; k < 4; ++k) m[k] = a.first[k] + b.first[k];
            add_term(P, m, a.second * b.second);
        }
    return P;
}

inline int64_t factorial(int k)
{
    int64_t f = 1;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

// int over the unit reference simplex of dimension dim.
inline Rat integrate_ref(const Poly &P, int dim)
{
    Rat s(0);
    for (const auto &t : P) {
        int64_t num = 1;
        int tot = 0;
        for (int k = 0; k <= dim; ++k) {
            num *= factorial(t.first[k]);
            tot += t.first[k];
        }
        s = s + t.second * Rat(num, factorial(tot + dim));
    }
    return s;
}


}  // namespace poly
}  // namespace fei
