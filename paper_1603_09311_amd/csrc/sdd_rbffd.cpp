// Sub-domain solver of stochastic domain decomposition (Sec. 3.2): RBF-FD on
// a rectangular sub-domain whose boundary values are given (interface values
// from the walks, outer values from the Dirichlet data).  Host stage.
//
// Each interior node gets two 9-node stencils (itself and its 8 grid
// neighbours, the 3x3 block around it) whose weights make d2/dy2 and d2/dz2
// exact on the multiquadric phi(r) = sqrt(1 + (eps r)^2) centred at each
// stencil node; the TE equation  Laplace E = i alpha E  then gives one sparse
// row per interior node, solved by a band LU with partial pivoting.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#include "sdd.h"

using cplx = std::complex<double>;

// Error reporting shared with the rest of the library.
sdd_status sdd_rbffd_fail(sdd_status st, const char *msg);

namespace {

// Dense solve of the symmetric 9x9 RBF system for two right-hand sides
// (Gaussian elimination with partial pivoting) in the host's extended
// precision: near-flat multiquadrics (eps h ~ 0.02) make the system
// ill-conditioned (condition numbers near 1e13), and the 64-bit significand
// keeps the weights to about 1e-6 there.  Returns false if singular.
using real = long double;

bool solve9(real A[9][9], real b[2][9]) {
  for (int c = 0; c < 9; ++c) {
    int p = c;
    for (int r = c + 1; r < 9; ++r)
      if (fabsl(A[r][c]) > fabsl(A[p][c])) p = r;
    if (A[p][c] == 0.0) return false;
    if (p != c) {
      for (int k = 0; k < 9; ++k) std::swap(A[p][k], A[c][k]);
      for (int s = 0; s < 2; ++s) std::swap(b[s][p], b[s][c]);
    }
    for (int r = c + 1; r < 9; ++r) {
      const real f = A[r][c] / A[c][c];
      if (f == 0.0) continue;
      for (int k = c; k < 9; ++k) A[r][k] -= f * A[c][k];
      for (int s = 0; s < 2; ++s) b[s][r] -= f * b[s][c];
    }
  }
  for (int s = 0; s < 2; ++s)
    for (int r = 8; r >= 0; --r) {
      real v = b[s][r];
      for (int k = r + 1; k < 9; ++k) v -= A[r][k] * b[s][k];
      b[s][r] = v / A[r][r];
    }
  return true;
}

// Band matrix with kl sub- and ku super-diagonals, stored for LU with partial
// pivoting (room for kl extra super-diagonals of fill), column-major bands:
// element (i, j) at ab[(kl + ku + i - j) + j * ldab].
struct Band {
  int n, kl, ku, ldab;
  std::vector<cplx> ab;
  Band(int n_, int kl_, int ku_) : n(n_), kl(kl_), ku(ku_), ldab(2 * kl_ + ku_ + 1), ab((size_t)ldab * n_) {}
  cplx &at(int i, int j) { return ab[(size_t)(kl + ku + i - j) + (size_t)j * ldab]; }
};

// In-place LU with partial pivoting and solve (the LAPACK band algorithm
// written out); returns false on a zero pivot.
bool band_solve(Band &B, std::vector<cplx> &x) {
  const int n = B.n, kl = B.kl, ku = B.ku;
  std::vector<int> piv(n);
  int ju = 0;   // last column touched by the fill so far
  for (int j = 0; j < n; ++j) {
    const int km = std::min(kl, n - 1 - j);
    int p = j;
    double best = std::abs(B.at(j, j));
    for (int i = j + 1; i <= j + km; ++i)
      if (std::abs(B.at(i, j)) > best) { best = std::abs(B.at(i, j)); p = i; }
    piv[j] = p;
    if (best == 0.0) return false;
    ju = std::max(ju, std::min(j + ku + (p - j), n - 1));
    if (p != j)
      for (int k = j; k <= ju; ++k) std::swap(B.at(p, k), B.at(j, k));
    const cplx d = B.at(j, j);
    for (int i = j + 1; i <= j + km; ++i) B.at(i, j) /= d;
    for (int k = j + 1; k <= ju; ++k) {
      const cplx u = B.at(j, k);
      if (u == cplx(0.0, 0.0)) continue;
      for (int i = j + 1; i <= j + km; ++i) B.at(i, k) -= B.at(i, j) * u;
    }
  }
  // forward: L y = P b
  for (int j = 0; j < n; ++j) {
    if (piv[j] != j) std::swap(x[j], x[piv[j]]);
    const int km = std::min(kl, n - 1 - j);
    for (int i = j + 1; i <= j + km; ++i) x[i] -= B.at(i, j) * x[j];
  }
  // backward: U x = y (U has up to kl + ku super-diagonals)
  for (int j = n - 1; j >= 0; --j) {
    x[j] /= B.at(j, j);
    const int lo = std::max(0, j - kl - ku);
    for (int i = lo; i < j; ++i) x[i] -= B.at(i, j) * x[j];
  }
  return true;
}

inline real mq(real eps2, real r2) { return sqrtl(1.0L + eps2 * r2); }
// d2/dy2 of sqrt(1 + eps^2 (dy^2 + dz^2)) with respect to the evaluation point
inline real mq_yy(real eps2, real dy, real dz) {
  const real q = 1.0L + eps2 * (dy * dy + dz * dz);
  return eps2 / sqrtl(q) - eps2 * eps2 * dy * dy / (q * sqrtl(q));
}

}  // namespace

extern "C" sdd_status sdd_rbffd_weights(uint32_t ny, uint32_t nz, const double *y, const double *z, double eps,
                                        double *w_yy, double *w_zz) {
  if (!y || !z || !w_yy || !w_zz) return sdd_rbffd_fail(SDD_E_INVALID, "NULL argument");
  if (ny < 3 || nz < 3) return sdd_rbffd_fail(SDD_E_INVALID, "the grid needs at least 3 x 3 nodes");
  if (!(eps != 0.0) || !std::isfinite(eps)) return sdd_rbffd_fail(SDD_E_INVALID, "eps must be finite and nonzero");
  for (uint32_t i = 1; i < ny; ++i)
    if (!(y[i] > y[i - 1]) || !std::isfinite(y[i])) return sdd_rbffd_fail(SDD_E_INVALID, "y must increase");
  for (uint32_t j = 1; j < nz; ++j)
    if (!(z[j] > z[j - 1]) || !std::isfinite(z[j])) return sdd_rbffd_fail(SDD_E_INVALID, "z must increase");
  for (uint32_t j = 1; j + 1 < nz; ++j)
    for (uint32_t i = 1; i + 1 < ny; ++i) {
      // eps > 0: one shape parameter everywhere; eps < 0: |eps| / h at each
      // node, h the largest grid spacing next to it (eps h fixed)
      real e = (real)eps;
      if (eps < 0.0) {
        const double h = std::max(std::max(y[i + 1] - y[i], y[i] - y[i - 1]), std::max(z[j + 1] - z[j], z[j] - z[j - 1]));
        e = (real)(-eps) / (real)h;
      }
      const real e2 = e * e;
      real py[9], pz[9];
      int k = 0;
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di, ++k) {
          py[k] = y[i + di];
          pz[k] = z[j + dj];
        }
      real A[9][9], b[2][9];
      for (int r = 0; r < 9; ++r) {
        for (int c = 0; c < 9; ++c) {
          const real dy = py[r] - py[c], dz = pz[r] - pz[c];
          A[r][c] = mq(e2, dy * dy + dz * dz);
        }
        // the operator applied to phi(|x - x_r|) at the centre x_0 = node 4
        const real dy = (real)y[i] - py[r], dz = (real)z[j] - pz[r];
        b[0][r] = mq_yy(e2, dy, dz);
        b[1][r] = mq_yy(e2, dz, dy);
      }
      if (!solve9(A, b)) return sdd_rbffd_fail(SDD_E_INVALID, "singular RBF system");
      const size_t row = ((size_t)(j - 1) * (ny - 2) + (i - 1)) * 9;
      for (int r = 0; r < 9; ++r) {
        w_yy[row + r] = (double)b[0][r];
        w_zz[row + r] = (double)b[1][r];
      }
    }
  return SDD_OK;
}

extern "C" sdd_status sdd_rbffd_solve(uint32_t ny, uint32_t nz, const double *y, const double *z, double alpha,
                                      double eps, double *field) {
  if (!field) return sdd_rbffd_fail(SDD_E_INVALID, "NULL argument");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return sdd_rbffd_fail(SDD_E_INVALID, "alpha must be finite, >= 0");
  if (ny < 3 || nz < 3) return sdd_rbffd_fail(SDD_E_INVALID, "the grid needs at least 3 x 3 nodes");
  const size_t nint = (size_t)(ny - 2) * (nz - 2);
  if (nint > (1u << 24)) return sdd_rbffd_fail(SDD_E_INVALID, "at most 2^24 interior nodes");
  for (size_t k = 0; k < (size_t)ny * nz * 2; ++k) {
    const uint32_t i = (uint32_t)((k / 2) % ny), j = (uint32_t)((k / 2) / ny);
    const bool boundary = i == 0 || j == 0 || i == ny - 1 || j == nz - 1;
    if (boundary && !std::isfinite(field[k])) return sdd_rbffd_fail(SDD_E_INVALID, "boundary values must be finite");
  }
  std::vector<double> wy(nint * 9), wz(nint * 9);
  sdd_status st = sdd_rbffd_weights(ny, nz, y, z, eps, wy.data(), wz.data());
  if (st != SDD_OK) return st;
  // unknowns ordered y fastest: (i, j) -> (j - 1) (ny - 2) + (i - 1)
  const int m = (int)(ny - 2);
  const int bw = m + 1;
  Band B((int)nint, bw, bw);
  std::vector<cplx> rhs(nint, cplx(0.0, 0.0));
  auto val = [&](uint32_t i, uint32_t j) { return cplx(field[2 * ((size_t)j * ny + i)], field[2 * ((size_t)j * ny + i) + 1]); };
  for (uint32_t j = 1; j + 1 < nz; ++j)
    for (uint32_t i = 1; i + 1 < ny; ++i) {
      const int row = (int)((j - 1) * m + (i - 1));
      const size_t w0 = (size_t)row * 9;
      int k = 0;
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di, ++k) {
          const uint32_t ii = i + di, jj = j + dj;
          cplx w(wy[w0 + k] + wz[w0 + k], 0.0);
          if (di == 0 && dj == 0) w -= cplx(0.0, alpha);   // Laplace E - i alpha E = 0
          const bool boundary = ii == 0 || jj == 0 || ii == ny - 1 || jj == nz - 1;
          if (boundary) {
            rhs[row] -= w * val(ii, jj);
          } else {
            const int col = (int)((jj - 1) * m + (ii - 1));
            B.at(row, col) += w;
          }
        }
    }
  if (!band_solve(B, rhs)) return sdd_rbffd_fail(SDD_E_INVALID, "singular RBF-FD system");
  for (uint32_t j = 1; j + 1 < nz; ++j)
    for (uint32_t i = 1; i + 1 < ny; ++i) {
      const cplx v = rhs[(j - 1) * m + (i - 1)];
      field[2 * ((size_t)j * ny + i)] = v.real();
      field[2 * ((size_t)j * ny + i) + 1] = v.imag();
    }
  return SDD_OK;
}
