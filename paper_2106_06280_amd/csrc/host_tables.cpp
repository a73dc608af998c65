// Host construction of the orthonormal triangle basis (Section 2, eq.
// triangleBasis) and of the Gauss rules, from the three-term recurrence of
// the Jacobi polynomials and Newton iterations for their roots (long double).
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "internal.h"

namespace cswdg {

namespace {

// P_n^{(a,b)}(x) (standard normalisation) and its derivative
void jacobi_pd(int n, long double a, long double b, long double x, long double& p,
               long double& dp) {
    long double p0 = 1.0L, p1 = 0.5L * ((a + b + 2.0L) * x + (a - b));
    if (n == 0) {
        p = 1.0L;
        dp = 0.0L;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        long double kk = k;
        long double c0 = 2.0L * kk * (kk + a + b) * (2.0L * kk + a + b - 2.0L);
        long double c1 = (2.0L * kk + a + b - 1.0L) *
                         ((2.0L * kk + a + b) * (2.0L * kk + a + b - 2.0L) * x + a * a - b * b);
        long double c2 = 2.0L * (kk + a - 1.0L) * (kk + b - 1.0L) * (2.0L * kk + a + b);
        long double p2 = (c1 * p1 - c2 * p0) / c0;
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    // d/dx P_n^{(a,b)} = (n+a+b+1)/2 P_{n-1}^{(a+1,b+1)}
    long double q, dq;
    jacobi_pd(n - 1, a + 1.0L, b + 1.0L, x, q, dq);
    dp = 0.5L * (n + a + b + 1.0L) * q;
}

long double jacobi_norm_factor(int n, long double alpha) {
    // 1/sqrt(2^{alpha+1}/(2n+alpha+1)) for beta = 0
    return 1.0L / std::sqrt(std::pow(2.0L, alpha + 1.0L) / (2.0L * n + alpha + 1.0L));
}

void normalised_jacobi(int n, double alpha, double x, double& v, double& dv) {
    long double p, dp;
    jacobi_pd(n, alpha, 0.0L, x, p, dp);
    long double f = jacobi_norm_factor(n, alpha);
    v = (double)(p * f);
    dv = (double)(dp * f);
}

}  // namespace

Rule1D gauss_jacobi(int n, double alpha) {
    Rule1D r;
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        // Chebyshev-like start, refined by Newton with deflation of found roots
        long double x = -std::cos(pi * (i + 0.75L) / (n + 0.5L));
        for (int it = 0; it < 100; ++it) {
            long double p, dp;
            jacobi_pd(n, alpha, 0.0L, x, p, dp);
            long double s = 0.0L;
            for (long double y : r.x) s += 1.0L / (x - y);
            long double dx = p / (dp - s * p);
            x -= dx;
            if (std::fabs(dx) < 1e-19L) break;
        }
        r.x.push_back(x);
    }
    // weights for weight (1-x)^alpha (1+x)^0:
    // w_i = 2^{alpha+1} Gamma(n+alpha+1) Gamma(n+1) / (Gamma(n+alpha+1) n!) / ((1-x^2) P'(x)^2)
    for (int i = 0; i < n; ++i) {
        long double p, dp;
        jacobi_pd(n, alpha, 0.0L, r.x[i], p, dp);
        long double x = r.x[i];
        r.w.push_back(std::pow(2.0L, alpha + 1.0L) / ((1.0L - x * x) * dp * dp));
    }
    // sort ascending
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (r.x[j] < r.x[i]) {
                std::swap(r.x[i], r.x[j]);
                std::swap(r.w[i], r.w[j]);
            }
    for (int i = 0; i + 1 < n; ++i)
        if (!(r.x[i] < r.x[i + 1])) throw std::runtime_error("gauss_jacobi: roots not distinct");
    return r;
}

Rule2D triangle_rule(int n) {
    Rule1D a = gauss_jacobi(n, 0.0), b = gauss_jacobi(n, 1.0);
    Rule2D t;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            long double r = 0.5L * (1.0L + a.x[i]) * (1.0L - b.x[j]) - 1.0L;
            t.r.push_back((double)r);
            t.s.push_back((double)b.x[j]);
            t.w.push_back((double)(0.5L * a.w[i] * b.w[j]));
        }
    return t;
}

int n_modes(int N) { return (N + 1) * (N + 2) / 2; }

void basis_eval(int N, double r, double s, double* psi, double* dr, double* ds) {
    double b = s;
    double om = 1.0 - b;
    double a = (std::fabs(om) > 1e-14) ? 2.0 * (1.0 + r) / om - 1.0 : -1.0;
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j + i <= N; ++j) {
            int m = j + (N + 1) * i + 1 - (i * (i - 1)) / 2;  // 1-based index
            int n = m - 1;
            double A, dA, B, dB;
            normalised_jacobi(i, 0.0, a, A, dA);
            normalised_jacobi(j, 2.0 * i + 1.0, b, B, dB);
            const double sq2 = 1.41421356237309504880;
            psi[n] = sq2 * A * B * std::pow(om, i);
            if (dr) {
                if (i == 0) {
                    dr[n] = 0.0;
                    ds[n] = sq2 * A * dB;
                } else {
                    // a = 2(1+r)/(1-s) - 1: da/dr = 2/(1-s), da/ds = (1+a)/(1-s)
                    dr[n] = sq2 * dA * B * 2.0 * std::pow(om, i - 1);
                    ds[n] = sq2 * (dA * (1.0 + a) * B * std::pow(om, i - 1) +
                                   A * (dB * std::pow(om, i) - i * B * std::pow(om, i - 1)));
                }
            }
        }
}

void basis_monomial_form(int N, std::vector<double>& C) {
    // fit psi_n on the equispaced lattice r = -1 + 2i/N, s = -1 + 2j/N
    // (unisolvent for degree N) in long double Gaussian elimination
    int np = n_modes(N);
    std::vector<long double> Vm(np * np), Y(np * np);
    int row = 0;
    std::vector<double> psi(np);
    for (int i = 0; i <= N; ++i)
        for (int j = 0; i + j <= N; ++j) {
            double r = -1.0 + 2.0 * i / N, s = -1.0 + 2.0 * j / N;
            int k = 0;
            for (int d = 0; d <= N; ++d)
                for (int bb = 0; bb <= d; ++bb) {
                    int aa = d - bb;
                    Vm[row * np + k++] = std::pow((long double)r, aa) * std::pow((long double)s, bb);
                }
            basis_eval(N, r, s, psi.data());
            for (int n = 0; n < np; ++n) Y[row * np + n] = psi[n];
            ++row;
        }
    // solve Vm * X = Y (X[k][n])
    for (int c = 0; c < np; ++c) {
        int piv = c;
        for (int r2 = c + 1; r2 < np; ++r2)
            if (std::fabs(Vm[r2 * np + c]) > std::fabs(Vm[piv * np + c])) piv = r2;
        for (int k = 0; k < np; ++k) {
            std::swap(Vm[c * np + k], Vm[piv * np + k]);
            std::swap(Y[c * np + k], Y[piv * np + k]);
        }
        for (int r2 = 0; r2 < np; ++r2) {
            if (r2 == c) continue;
            long double f = Vm[r2 * np + c] / Vm[c * np + c];
            for (int k = 0; k < np; ++k) {
                Vm[r2 * np + k] -= f * Vm[c * np + k];
                Y[r2 * np + k] -= f * Y[c * np + k];
            }
        }
    }
    C.assign(np * np, 0.0);
    for (int k = 0; k < np; ++k)
        for (int n = 0; n < np; ++n) C[n * np + k] = (double)(Y[k * np + n] / Vm[k * np + k]);
}

template <int N>
void fill_tables(Tab<N>& t) {
    using D = Dims<N>;
    std::memset(&t, 0, sizeof(t));
    Rule2D vr = triangle_rule(D::NV1);
    double psi[D::NP], dr[D::NP], ds[D::NP];
    for (int q = 0; q < D::NQ; ++q) {
        basis_eval(N, vr.r[q], vr.s[q], psi, dr, ds);
        for (int n = 0; n < D::NP; ++n) {
            t.V[q][n] = psi[n];
            t.wDr[q][n] = vr.w[q] * dr[n];
            t.wDs[q][n] = vr.w[q] * ds[n];
        }
    }
    Rule1D e = gauss_jacobi(D::NE, 0.0);
    // symmetrise so that point g of one side is point NE-1-g of the other
    for (int g = 0; g < D::NE; ++g) {
        double x = (double)(0.5L * (e.x[g] - e.x[D::NE - 1 - g]));
        double w = (double)(0.5L * (e.w[g] + e.w[D::NE - 1 - g]));
        t.we[g] = w;
        t.es[g] = 0.5 * (1.0 + x);
        for (int f = 0; f < 3; ++f) {
            double r, s;
            if (f == 0) {
                r = x;
                s = -1.0;
            } else if (f == 1) {
                r = -x;
                s = x;
            } else {
                r = -1.0;
                s = -x;
            }
            basis_eval(N, r, s, psi);
            for (int n = 0; n < D::NP; ++n) {
                t.PF[f][g][n] = psi[n];
                t.wPF[f][g][n] = w * psi[n];
            }
        }
    }
    for (int n = 0; n < D::NP; ++n) t.wmean[n] = (n == 0) ? kPsi0 : 0.0;
    // face midpoints: (0, -1), (0, 0), (-1, 0)
    const double mr[3] = {0.0, 0.0, -1.0}, ms[3] = {-1.0, 0.0, 0.0};
    for (int f = 0; f < 3; ++f) {
        basis_eval(N, mr[f], ms[f], psi);
        for (int n = 0; n < D::NP; ++n) t.PMID[f][n] = psi[n];
    }
}

template void fill_tables<1>(Tab<1>&);
template void fill_tables<2>(Tab<2>&);
template void fill_tables<3>(Tab<3>&);

}  // namespace cswdg
