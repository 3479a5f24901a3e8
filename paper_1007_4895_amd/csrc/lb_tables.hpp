// lb_tables.hpp -- compile-time velocity-set tables.
//
// The n-point Gauss-Hermite rule (Sec. 2.1): abscissae are the roots of the
// probabilists' Hermite polynomial He_n (weight exp(-x^2/2)), weights follow
// Eq. (weight), w = n! / [n He_{n-1}(x)]^2.  The roots are located on a
// coarse scan and refined by Newton's method (He_n' = n He_{n-1}), then
// symmetrised (He_n has parity (-1)^n).  The 2D sets are tensor products:
// population a = p + n*q has velocity (x_p, x_q) and weight w_p w_q.
//
// Everything here is constexpr, so the kernels see the abscissae, weights
// and He_k(x_p)/k! as immediates and the upwind direction of every
// population is resolved at compile time.
#pragma once

namespace lbt {

constexpr double hermite(int k, double x) {
    if (k == 0) return 1.0;
    double hm = 1.0, h = x;
    for (int i = 1; i < k; ++i) {
        double hp = x * h - double(i) * hm;
        hm = h;
        h = hp;
    }
    return h;
}

constexpr double factorial(int k) {
    double r = 1.0;
    for (int i = 2; i <= k; ++i) r *= double(i);
    return r;
}

constexpr double cabs(double x) { return x < 0 ? -x : x; }

template <int N>
struct Rule {
    double x[N];
    double w[N];
};

template <int N>
constexpr Rule<N> make_rule() {
    Rule<N> r{};
    double R = 1.0;
    while (R * R < 4.0 * N + 2.0) R += 0.25;   // all roots lie in |x| < sqrt(4N+2)
    int found = 0;
    const int scan = 2048;
    double a = -R, fa = hermite(N, a);
    for (int s = 1; s <= scan && found < N; ++s) {
        double b = -R + 2.0 * R * double(s) / double(scan);
        double fb = hermite(N, b);
        if (fa == 0.0) {
            r.x[found++] = a;
        } else if (fa * fb < 0.0) {
            double x = 0.5 * (a + b);
            for (int it = 0; it < 100; ++it) {
                double d = double(N) * hermite(N - 1, x);
                double step = hermite(N, x) / d;
                double xn = x - step;
                if (xn == x) break;
                x = xn;
            }
            r.x[found++] = x;
        }
        a = b;
        fa = fb;
    }
    for (int p = 0; p < N / 2; ++p) r.x[p] = -r.x[N - 1 - p];
    if (N % 2 == 1) r.x[N / 2] = 0.0;
    for (int p = 0; p < N; ++p) {
        double d = double(N) * hermite(N - 1, r.x[p]);
        r.w[p] = factorial(N) / (d * d);
    }
    return r;
}

template <int N>
struct Tab {
    static constexpr Rule<N> rule = make_rule<N>();
    // He_k(x_p) / k!  for k = 0..N  (index [k][p])
    struct HK {
        double v[N + 1][N];
    };
    static constexpr HK make_hk() {
        HK h{};
        for (int k = 0; k <= N; ++k)
            for (int p = 0; p < N; ++p) h.v[k][p] = hermite(k, rule.x[p]) / factorial(k);
        return h;
    }
    static constexpr HK hk = make_hk();
    // He_k(x_p) for k = 0..N
    static constexpr HK make_h() {
        HK h{};
        for (int k = 0; k <= N; ++k)
            for (int p = 0; p < N; ++p) h.v[k][p] = hermite(k, rule.x[p]);
        return h;
    }
    static constexpr HK he = make_h();
    static constexpr double xmax() { return rule.x[N - 1]; }
};

// A velocity set with its equilibrium order (the force uses the same order).
// TH: thermal lattice -- every node's temperature comes from its energy
// moment and enters the equilibrium's Hermite coefficients; otherwise T = 1.
template <int N_, int EQ_, bool TH_ = false>
struct VSet {
    static constexpr int N = N_;
    static constexpr int Q = N_ * N_;
    static constexpr int EQ = EQ_;
    static constexpr bool TH = TH_;
    using T = Tab<N_>;
};

// Placeholder for "no partner set" (uniform runs).
struct NoSet {
    static constexpr int N = 0;
    static constexpr int Q = 0;
    static constexpr int EQ = 0;
    static constexpr bool TH = false;
};

}  // namespace lbt
