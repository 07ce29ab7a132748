// Host-side FP64 builders of the 1D ingredients (run once per model).
#include "ppq_model.hpp"

#include <cmath>

namespace ppq {

std::vector<double> sine_dvr_points(int n, double lo, double hi)
{
    std::vector<double> q(n);
    double dx = (hi - lo) / (n + 1);
    for (int i = 0; i < n; ++i) q[i] = lo + (i + 1) * dx;
    return q;
}

std::vector<double> sine_dvr_kinetic(int n, double lo, double hi, double mass)
{
    const double L = hi - lo;
    std::vector<double> U((size_t)n * n), e(n), T((size_t)n * n, 0.0);
    const double nrm = std::sqrt(2.0 / (n + 1));
    for (int i = 1; i <= n; ++i)
        for (int k = 1; k <= n; ++k) U[(size_t)(i - 1) * n + (k - 1)] = nrm * std::sin(M_PI * i * k / (n + 1));
    for (int k = 1; k <= n; ++k) {
        double p = k * M_PI / L;
        e[k - 1] = p * p / (2.0 * mass);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += U[(size_t)i * n + k] * e[k] * U[(size_t)j * n + k];
            T[(size_t)i * n + j] = s;
        }
    // exact symmetry
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double s = 0.5 * (T[(size_t)i * n + j] + T[(size_t)j * n + i]);
            T[(size_t)i * n + j] = s;
            T[(size_t)j * n + i] = s;
        }
    return T;
}

std::vector<cd> pvb_projection(const std::vector<double> &q, double dxg, double lo, double hi, int ns, int nl)
{
    const int n = (int)q.size();
    const double cell = (hi - lo) / ns;
    const double dp = 2.0 * M_PI / cell;
    const double a = dp / (2.0 * cell);
    const double pref = std::sqrt(dxg) * std::pow(2.0 * a / M_PI, 0.25);
    std::vector<cd> G((size_t)n * n);
    for (int s = 0; s < ns; ++s) {
        double xs = lo + (s + 0.5) * cell;
        for (int l = 0; l < nl; ++l) {
            double pl = (l - 0.5 * (nl - 1)) * dp;
            for (int j = 0; j < n; ++j) {
                double d = q[j] - xs;
                G[(size_t)j * n + (s * nl + l)] = pref * std::exp(cd(-a * d * d, pl * d));
            }
        }
    }
    return G;
}

// Real symmetric eigen-decomposition by cyclic Jacobi rotations (a is
// consumed): w receives the eigenvalues, v the eigenvectors as columns.
static void jacobi_eigen(std::vector<double> a, int n, std::vector<double> &w, std::vector<double> &v)
{
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double x = a[(size_t)i * n + j];
                if (i == j) diag += x * x;
                else off += x * x;
            }
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - sn * akq;
                    a[(size_t)k * n + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - sn * aqk;
                    a[(size_t)q * n + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = c * vkp - sn * vkq;
                    v[(size_t)k * n + q] = sn * vkp + c * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
}

// Projected Weylets (Sec. II.D): the momentum-symmetrized Gaussians of
// Eq. sG_def on a doubly dense lattice (cell dx, dp = pi / dx, momenta
// p_l = (l + 1/2) dp > 0, alpha = dp / (2 dx)), projected on the grid points
// q with quadrature weight dxg (Eq. psG_def) as Phi, then orthogonalised: W = Phi S^{-1/2},
// S = Phi^T Phi.  Returned as a complex n x n matrix (real values).
std::vector<cd> weylet_projection(const std::vector<double> &q, double dxg, double lo, double hi, int nx, int np)
{
    const int n = (int)q.size();
    const double cell = (hi - lo) / nx;
    const double dp = M_PI / cell;
    const double a = dp / (2.0 * cell);
    const double pref = std::sqrt(dxg) * std::pow(8.0 * a / M_PI, 0.25);
    const double shift = std::sqrt(M_PI / (8.0 * a));
    std::vector<double> phi((size_t)n * n);
    for (int s = 0; s < nx; ++s) {
        const double xs = lo + (s + 0.5) * cell;
        for (int l = 0; l < np; ++l) {
            const double pl = (l + 0.5) * dp;
            for (int j = 0; j < n; ++j) {
                const double d = q[j] - xs;
                phi[(size_t)j * n + (s * np + l)] = pref * std::exp(-a * d * d) * std::sin(pl * (d - shift));
            }
        }
    }
    std::vector<double> S((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int r = 0; r < n; ++r) acc += phi[(size_t)r * n + i] * phi[(size_t)r * n + j];
            S[(size_t)i * n + j] = acc;
        }
    std::vector<double> w, v;
    jacobi_eigen(S, n, w, v);
    double wmax = 0.0;
    for (double x : w) wmax = std::max(wmax, x);
    std::vector<double> sih((size_t)n * n, 0.0);  // S^{-1/2} = V diag(w^-1/2) V^T
    for (int k = 0; k < n; ++k) {
        if (!(w[k] > 1e-14 * wmax)) throw std::runtime_error("linearly dependent Weylet lattice");
        const double f = 1.0 / std::sqrt(w[k]);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) sih[(size_t)i * n + j] += v[(size_t)i * n + k] * f * v[(size_t)j * n + k];
    }
    std::vector<cd> W((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int r = 0; r < n; ++r) acc += phi[(size_t)i * n + r] * sih[(size_t)r * n + j];
            W[(size_t)i * n + j] = acc;
        }
    return W;
}

// Kinetic energy -1/(2 mass) d^2/dx^2 on the periodic Fourier grid of n
// (odd) points over the period hi - lo, from its spectral definition:
// T_ij = (1/n) sum_m k_m^2 / (2 mass) cos(k_m (x_i - x_j)), k_m = 2 pi m / L,
// |m| <= (n-1)/2.
std::vector<double> fgh_kinetic(int n, double lo, double hi, double mass)
{
    const double L = hi - lo;
    const int M = (n - 1) / 2;
    std::vector<double> T((size_t)n * n);
    for (int d = 0; d < n; ++d) {
        double acc = 0.0;
        for (int m = 1; m <= M; ++m) {
            const double km = 2.0 * M_PI * m / L;
            acc += 2.0 * km * km / (2.0 * mass) * std::cos(2.0 * M_PI * m * d / n);
        }
        for (int i = 0; i < n; ++i) T[(size_t)i * n + (i + d) % n] = acc / n;
    }
    // the entries depend on (i - j) mod n only and are even in it: exactly symmetric
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) T[(size_t)j * n + i] = T[(size_t)i * n + j];
    return T;
}

bool invert(std::vector<cd> &a, int n)
{
    std::vector<cd> inv((size_t)n * n, cd(0.0, 0.0));
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        double best = std::abs(a[(size_t)c * n + c]);
        for (int r = c + 1; r < n; ++r) {
            double v = std::abs(a[(size_t)r * n + c]);
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        if (best == 0.0) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(a[(size_t)c * n + k], a[(size_t)piv * n + k]);
                std::swap(inv[(size_t)c * n + k], inv[(size_t)piv * n + k]);
            }
        cd d = 1.0 / a[(size_t)c * n + c];
        for (int k = 0; k < n; ++k) {
            a[(size_t)c * n + k] *= d;
            inv[(size_t)c * n + k] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            cd f = a[(size_t)r * n + c];
            if (f == cd(0.0, 0.0)) continue;
            for (int k = 0; k < n; ++k) {
                a[(size_t)r * n + k] -= f * a[(size_t)c * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
            }
        }
    }
    a.swap(inv);
    return true;
}

std::vector<cd> matmul(const std::vector<cd> &a, const std::vector<cd> &b, int n)
{
    std::vector<cd> c((size_t)n * n, cd(0.0, 0.0));
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            cd aik = a[(size_t)i * n + k];
            for (int j = 0; j < n; ++j) c[(size_t)i * n + j] += aik * b[(size_t)k * n + j];
        }
    return c;
}

std::vector<cd> adjoint(const std::vector<cd> &a, int n)
{
    std::vector<cd> t((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) t[(size_t)j * n + i] = std::conj(a[(size_t)i * n + j]);
    return t;
}

}  // namespace ppq
