/*
 * tables_ct.h -- the 1D tables of the sum factorisation evaluated at
 * compile time, so that the kernels see every coefficient as an immediate
 * (no table lives in registers across the cell loop).
 *
 * Same definitions as the host tables of setup_host.cpp: Lagrange basis on
 * the k+1 Gauss-Lobatto-Legendre points of [0,1], evaluated at the k+1
 * Gauss-Legendre points (S), and the collocation derivative of the Lagrange
 * basis on the Gauss points (D); both rules by Newton iteration on the
 * Legendre recurrence (textbook).  Computed in double here, so entries may
 * differ from the long-double host tables in the last bit.
 */
#pragma once

namespace mfcg {
namespace ct {

constexpr double PI = 3.14159265358979323846264338327950288;

constexpr double cabs(double x) { return x < 0 ? -x : x; }

/* cos by its Taylor series after reduction to [0, pi/2] */
constexpr double ccos(double x)
{
    x = cabs(x);
    while (x > 2 * PI) x -= 2 * PI;
    if (x > PI) x = 2 * PI - x;
    double sign = 1.0;
    if (x > PI / 2) {
        x = PI - x;
        sign = -1.0;
    }
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 30; ++k) {
        term *= -x * x / ((2 * k - 1) * (2 * k));
        sum += term;
    }
    return sign * sum;
}

/* P_n(t) and P_n'(t) */
constexpr void legendre(int n, double t, double &p, double &dp)
{
    double a = 1.0, b = t;
    if (n == 0) {
        p = 1.0;
        dp = 0.0;
        return;
    }
    for (int m = 2; m <= n; ++m) {
        const double c = ((2 * m - 1) * t * b - (m - 1) * a) / m;
        a = b;
        b = c;
    }
    p = b;
    dp = n * (a - t * b) / (1.0 - t * t);
}

template <int NP>
struct Tab {
    double S[NP * NP];
    double D[NP * NP];
    double xq[NP];
    double wq[NP]; /* Gauss weights on [0,1] (Gauss tables only) */
    double gll[NP];
};

/* GLLQ = false: quadrature on the NP Gauss points; true: on the NP GLL
 * points themselves (collocation: S is the identity, D the nodal
 * differentiation matrix). */
template <int NP, bool GLLQ = false>
constexpr Tab<NP> make_tab()
{
    Tab<NP> t{};
    constexpr int n = NP, k = NP - 1;
    /* Gauss points on [0,1], ascending */
    for (int i = 0; i < n && !GLLQ; ++i) {
        double x = -ccos(PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p = 0, dp = 0;
            legendre(n, x, p, dp);
            const double dx = p / dp;
            x -= dx;
            if (cabs(dx) < 1e-17) break;
        }
        t.xq[i] = 0.5 * (1.0 + x);
        double p = 0, dp = 0;
        legendre(n, x, p, dp);
        t.wq[i] = 1.0 / ((1.0 - x * x) * dp * dp); /* 2 / ((1 - x^2) P_n'(x)^2), halved for [0,1] */
    }
    /* GLL points on [0,1] */
    t.gll[0] = 0.0;
    t.gll[k] = 1.0;
    for (int i = 1; i < k; ++i) {
        double x = -ccos(PI * i / k);
        for (int it = 0; it < 100; ++it) {
            double p = 0, dp = 0;
            legendre(k, x, p, dp);
            const double ddp = (2.0 * x * dp - k * (k + 1.0) * p) / (1.0 - x * x);
            const double dx = dp / ddp;
            x -= dx;
            if (cabs(dx) < 1e-17) break;
        }
        t.gll[i] = 0.5 * (1.0 + x);
    }
    if (GLLQ)
        for (int i = 0; i < n; ++i) t.xq[i] = t.gll[i];
    /* S[q][i] = phi_i(xq_q) */
    for (int q = 0; q < n; ++q)
        for (int i = 0; i < n; ++i) {
            double v = 1.0;
            for (int j = 0; j < n; ++j)
                if (j != i) v *= (t.xq[q] - t.gll[j]) / (t.gll[i] - t.gll[j]);
            t.S[q * n + i] = v;
        }
    /* D[q][m] = l_m'(xq_q) on the Gauss points (barycentric form) */
    double w[NP] = {};
    for (int i = 0; i < n; ++i) {
        w[i] = 1.0;
        for (int j = 0; j < n; ++j)
            if (j != i) w[i] /= (t.xq[i] - t.xq[j]);
    }
    for (int q = 0; q < n; ++q) {
        double diag = 0.0;
        for (int m = 0; m < n; ++m) {
            if (m == q) continue;
            t.D[q * n + m] = (w[m] / w[q]) / (t.xq[q] - t.xq[m]);
            diag -= t.D[q * n + m];
        }
        t.D[q * n + q] = diag;
    }
    return t;
}

/* NQ = NP + 1 Gauss points with the NP-node GLL basis (the (k+2)-point
 * rules of the benchmark problems): S is NQ x NP, D is NQ x NQ (the
 * collocation derivative on the Gauss points), both row-major. */
template <int NP, int NQ>
struct Tab2 {
    double S[NQ * NP];
    double D[NQ * NQ];
    double xq[NQ];
    double wq[NQ]; /* Gauss weights on [0,1] */
    double gll[NP];
};

template <int NP, int NQ>
constexpr Tab2<NP, NQ> make_tab2()
{
    Tab2<NP, NQ> t{};
    constexpr int k = NP - 1;
    for (int i = 0; i < NQ; ++i) {
        double x = -ccos(PI * (i + 0.75) / (NQ + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p = 0, dp = 0;
            legendre(NQ, x, p, dp);
            const double dx = p / dp;
            x -= dx;
            if (cabs(dx) < 1e-17) break;
        }
        t.xq[i] = 0.5 * (1.0 + x);
        double p = 0, dp = 0;
        legendre(NQ, x, p, dp);
        t.wq[i] = 1.0 / ((1.0 - x * x) * dp * dp);
    }
    t.gll[0] = 0.0;
    t.gll[k] = 1.0;
    for (int i = 1; i < k; ++i) {
        double x = -ccos(PI * i / k);
        for (int it = 0; it < 100; ++it) {
            double p = 0, dp = 0;
            legendre(k, x, p, dp);
            const double ddp = (2.0 * x * dp - k * (k + 1.0) * p) / (1.0 - x * x);
            const double dx = dp / ddp;
            x -= dx;
            if (cabs(dx) < 1e-17) break;
        }
        t.gll[i] = 0.5 * (1.0 + x);
    }
    for (int q = 0; q < NQ; ++q)
        for (int i = 0; i < NP; ++i) {
            double v = 1.0;
            for (int j = 0; j < NP; ++j)
                if (j != i) v *= (t.xq[q] - t.gll[j]) / (t.gll[i] - t.gll[j]);
            t.S[q * NP + i] = v;
        }
    double w[NQ] = {};
    for (int i = 0; i < NQ; ++i) {
        w[i] = 1.0;
        for (int j = 0; j < NQ; ++j)
            if (j != i) w[i] /= (t.xq[i] - t.xq[j]);
    }
    for (int q = 0; q < NQ; ++q) {
        double diag = 0.0;
        for (int m = 0; m < NQ; ++m) {
            if (m == q) continue;
            t.D[q * NQ + m] = (w[m] / w[q]) / (t.xq[q] - t.xq[m]);
            diag -= t.D[q * NQ + m];
        }
        t.D[q * NQ + q] = diag;
    }
    return t;
}

template <int NP>
struct Tables1D {
    static constexpr Tab<NP> t = make_tab<NP>();
};

}  // namespace ct
}  // namespace mfcg
