// Host-side FP64 builders of the 1D ingredients (run once per model).
#pragma once
#include <complex>
#include <vector>

namespace ppq {

using cd = std::complex<double>;

// Sine-DVR on the box (lo, hi) with n interior points (particle-in-a-box DVR):
// grid points q_i = lo + i*dx, i = 1..n, dx = (hi-lo)/(n+1).
std::vector<double> sine_dvr_points(int n, double lo, double hi);
// Kinetic matrix -1/(2 mass) d^2/dq^2 in the sine DVR, assembled from its
// spectral form T = U diag(e) U^T, U_in = sqrt(2/(n+1)) sin(pi i n'/(n+1)),
// e_n' = (n' pi / L)^2 / (2 mass).  Row-major n x n.
std::vector<double> sine_dvr_kinetic(int n, double lo, double hi, double mass);

// Projected von Neumann lattice on a sine-DVR grid (n_s * n_l == n):
// G[j][s*n_l + l] = sqrt(dx) (2a/pi)^{1/4} exp(-a (q_j - x_s)^2 + i p_l (q_j - x_s)).
std::vector<cd> pvb_projection(const std::vector<double> &q, double dxg, double lo, double hi, int ns, int nl);
// kinetic energy on the periodic Fourier grid (odd n), row-major n x n
std::vector<double> fgh_kinetic(int n, double lo, double hi, double mass);
// projected Weylets (orthogonal, real): W = Phi S^{-1/2} on an nx x np doubly dense lattice
std::vector<cd> weylet_projection(const std::vector<double> &q, double dxg, double lo, double hi, int nx, int np);

// In-place inverse of a dense complex matrix (Gauss-Jordan, partial pivoting).
// Returns false if singular.
bool invert(std::vector<cd> &a, int n);

// c = a * b for row-major n x n complex matrices.
std::vector<cd> matmul(const std::vector<cd> &a, const std::vector<cd> &b, int n);
std::vector<cd> adjoint(const std::vector<cd> &a, int n);

}  // namespace ppq
