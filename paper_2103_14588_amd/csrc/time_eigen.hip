// time_eigen.hip -- eigen-decomposition of the Galerkin time pencil (host).
//
// Along time the reduced operator has the 1D factors (rows and columns
// tau = 1..n_t; the t = 0 node was moved to the right-hand side, Sec. 2.1):
//   mass       M[t][t] = 2h/3 (h/3 in the last row), M[t][t+-1] = h/6
//   derivative D[t][t+-1] = +-1/2, D[n_t-1][n_t-1] = 1/2, else 0
// (test function times the time derivative of the trial function).  The
// operator is A = D (x) X0 + M (x) X1 with spatial parts X0, X1, so with the
// generalised eigen-decomposition D W = M W diag(lambda),
//   A^{-1} = (W (x) I) (diag(lambda) (x) X0 + I (x) X1)^{-1} (Q (x) I),
//   Q = W^{-1} M^{-1},
// which splits one spacetime solve into n_t independent spatial solves.
//
// Method: the eigenvalues are the roots of det(D - lambda M), evaluated with
// the three-term recurrence of tridiagonal determinants in ratio form (no
// overflow) together with its derivative, and found simultaneously with the
// Aberth-Ehrlich iteration (Gauss-Seidel sweeps).  Right and left
// eigenvectors follow from the same recurrence run as a two-term
// propagation of (D - lambda M) w = 0 and w^T (D - lambda M) = 0; with
// delta_k = u_k^T M w_k the rows of Q are u_k^T / delta_k.  The result is
// checked before use: every right-eigenpair residual and W Q M x = x on a
// fixed test vector.
#include <cmath>
#include <complex>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "common.hpp"
#include "time_eigen.hpp"

namespace dst {

using cd = std::complex<double>;

namespace {

struct Pencil {
  int n;
  std::vector<double> dA, mA;  // diagonal
  std::vector<double> dB, mB;  // (k, k-1), index k >= 1
  std::vector<double> dC, mC;  // (k-1, k), index k >= 1
};

Pencil make_pencil(int n, double h) {
  Pencil P;
  P.n = n;
  P.dA.assign(n, 0.0);
  P.mA.assign(n, 2.0 * h / 3.0);
  P.dB.assign(n, -0.5);
  P.mB.assign(n, h / 6.0);
  P.dC.assign(n, 0.5);
  P.mC.assign(n, h / 6.0);
  P.dA[n - 1] = 0.5;
  P.mA[n - 1] = h / 3.0;
  P.dB[0] = P.mB[0] = P.dC[0] = P.mC[0] = 0.0;
  return P;
}

// Newton correction p(z) / p'(z) of p(z) = det(D - z M).
cd newton_step(const Pencil &P, cd z) {
  cd r_prev(1.0, 0.0), rp_prev(0.0, 0.0), s(0.0, 0.0);
  for (int k = 0; k < P.n; k++) {
    const cd ak = P.dA[k] - z * P.mA[k];
    const double akp = -P.mA[k];
    cd r, rp;
    if (k == 0) {
      r = ak;
      rp = akp;
    } else {
      const cd bk = P.dB[k] - z * P.mB[k], ck = P.dC[k] - z * P.mC[k];
      const cd bc = bk * ck;
      const cd bcp = -P.mB[k] * ck - bk * P.mC[k];
      r = ak - bc / r_prev;
      rp = akp - bcp / r_prev + bc * rp_prev / (r_prev * r_prev);
    }
    if (r == cd(0.0, 0.0)) return cd(0.0, 0.0);  // z is a root of a leading minor: no move
    s += rp / r;
    r_prev = r;
    rp_prev = rp;
  }
  return cd(1.0, 0.0) / s;
}

}  // namespace

static int time_eigen_core(int n, double h, std::vector<cd> &lam, std::vector<cd> &W, std::vector<cd> &Q) {
  DST_CHECK(n >= 1 && n <= kTimeEigenMax, "time eigen-decomposition needs 1 <= n_t <= %d", kTimeEigenMax);
  DST_CHECK(h > 0.0 && std::isfinite(h), "time step must be positive");
  const Pencil P = make_pencil(n, h);
  lam.assign(n, cd(0, 0));
  W.assign((size_t)n * n, cd(0, 0));
  Q.assign((size_t)n * n, cd(0, 0));
  // starting points along the segment the spectrum clusters on (the symbol
  // of the interior rows is 3 i sin(th) / (h (2 + cos th)), |.| <= sqrt(3)/h),
  // shifted into the right half-plane and slightly off the symmetry axis
  const double T = n * h;
  for (int k = 0; k < n; k++)
    lam[k] = cd(1.0 / T, std::sqrt(3.0) / h * std::cos(M_PI * (k + 0.5) / n) + 0.01 / T * std::sin(k + 1.0));
  std::vector<char> done(n, 0);
  int sweeps = 0;
  for (; sweeps < 300; sweeps++) {
    bool all = true;
    for (int i = 0; i < n; i++) {
      if (done[i]) continue;
      const cd N = newton_step(P, lam[i]);
      cd S(0, 0);
      for (int j = 0; j < n; j++)
        if (j != i) S += cd(1.0, 0.0) / (lam[i] - lam[j]);
      const cd den = cd(1.0, 0.0) - N * S;
      const cd dz = (std::abs(den) > 1e-300) ? N / den : N;
      if (!std::isfinite(dz.real()) || !std::isfinite(dz.imag())) {
        done[i] = 1;
        continue;
      }
      lam[i] -= dz;
      // cubic convergence: a step this small leaves an error far below rounding
      if (std::abs(dz) <= 1e-11 * std::abs(lam[i])) done[i] = 1;
      else all = false;
    }
    if (all) break;
  }
  // eigenvectors: w_0 = 1, row k of (D - lambda M) w = 0 gives w_{k+1};
  // u_0 = 1, column k of u^T (D - lambda M) = 0 gives u_{k+1}
  std::vector<cd> w(n), u(n), Mw(n);
  for (int j = 0; j < n; j++) {
    const cd l = lam[j];
    w[0] = u[0] = cd(1.0, 0.0);
    for (int k = 0; k + 1 < n; k++) {
      const cd ak = P.dA[k] - l * P.mA[k];
      cd sw = ak * w[k], su = ak * u[k];
      if (k > 0) {
        sw += (P.dB[k] - l * P.mB[k]) * w[k - 1];  // A[k][k-1]
        su += (P.dC[k] - l * P.mC[k]) * u[k - 1];  // A[k-1][k]
      }
      w[k + 1] = -sw / (P.dC[k + 1] - l * P.mC[k + 1]);  // A[k][k+1]
      u[k + 1] = -su / (P.dB[k + 1] - l * P.mB[k + 1]);  // A[k+1][k]
    }
    double wm = 0.0, um = 0.0;
    for (int k = 0; k < n; k++) {
      wm = std::max(wm, std::abs(w[k]));
      um = std::max(um, std::abs(u[k]));
    }
    for (int k = 0; k < n; k++) {
      w[k] /= wm;
      u[k] /= um;
    }
    // delta = u^T M w
    cd delta(0, 0);
    for (int k = 0; k < n; k++) {
      cd mw = P.mA[k] * w[k];
      if (k > 0) mw += P.mB[k] * w[k - 1];
      if (k + 1 < n) mw += P.mC[k + 1] * w[k + 1];
      Mw[k] = mw;
      delta += u[k] * mw;
    }
    // right residual |(D - lambda M) w| relative to (|D| + |lambda| |M|) |w|
    double res = 0.0;
    for (int k = 0; k < n; k++) {
      cd dw = P.dA[k] * w[k];
      if (k > 0) dw += P.dB[k] * w[k - 1];
      if (k + 1 < n) dw += P.dC[k + 1] * w[k + 1];
      res = std::max(res, std::abs(dw - l * Mw[k]));
    }
    const double scale = 1.0 + std::abs(l) * h;
    DST_CHECK(std::isfinite(res) && res <= 1e-6 * scale && std::abs(delta) > 0.0,
              "time eigen-decomposition failed (n_t = %d, pair %d, residual %.3g)", n, j, res / scale);
    for (int k = 0; k < n; k++) {
      W[(size_t)k * n + j] = w[k];
      Q[(size_t)j * n + k] = u[k] / delta;
    }
  }
  // W Q M x = x on a fixed vector
  std::vector<cd> x(n), y(n), z(n);
  for (int k = 0; k < n; k++) x[k] = cd(std::cos(0.7 * k + 0.3), std::sin(1.3 * k));
  for (int k = 0; k < n; k++) {
    cd mx = P.mA[k] * x[k];
    if (k > 0) mx += P.mB[k] * x[k - 1];
    if (k + 1 < n) mx += P.mC[k + 1] * x[k + 1];
    y[k] = mx;
  }
  double err = 0.0, nx = 0.0;
  for (int j = 0; j < n; j++) {
    cd s(0, 0);
    for (int k = 0; k < n; k++) s += Q[(size_t)j * n + k] * y[k];
    z[j] = s;
  }
  for (int k = 0; k < n; k++) {
    cd s(0, 0);
    for (int j = 0; j < n; j++) s += W[(size_t)k * n + j] * z[j];
    err = std::max(err, std::abs(s - x[k]));
    nx = std::max(nx, std::abs(x[k]));
  }
  DST_CHECK(std::isfinite(err) && err <= 1e-8 * nx,
            "time eigen-decomposition inaccurate (n_t = %d, reconstruction error %.3g)", n, err / nx);
  return 0;
}

// Process-wide cache: the decomposition depends on (n_t, h_t) only, and every
// operator of a batch or of a sequence of solves on one mesh shares it.
namespace {
struct EigenEntry {
  std::vector<cd> lam, W, Q;
};
std::mutex g_eig_mu;
std::map<std::pair<int, double>, EigenEntry> g_eig;
size_t g_eig_bytes = 0;
constexpr size_t kEigenCacheBytes = size_t(256) << 20;
size_t entry_bytes(int n) { return (2 * (size_t)n * n + n) * sizeof(cd); }
}  // namespace

int time_eigen(int n, double h, std::vector<cd> &lam, std::vector<cd> &W, std::vector<cd> &Q) {
  const std::pair<int, double> key(n, h);
  {
    std::lock_guard<std::mutex> lk(g_eig_mu);
    auto it = g_eig.find(key);
    if (it != g_eig.end()) {
      lam = it->second.lam;
      W = it->second.W;
      Q = it->second.Q;
      return 0;
    }
  }
  if (int rc = time_eigen_core(n, h, lam, W, Q)) return rc;
  std::lock_guard<std::mutex> lk(g_eig_mu);
  if (g_eig.count(key) || entry_bytes(n) > kEigenCacheBytes) return 0;
  while (!g_eig.empty() && g_eig_bytes + entry_bytes(n) > kEigenCacheBytes) {
    g_eig_bytes -= entry_bytes(g_eig.begin()->first.first);
    g_eig.erase(g_eig.begin());
  }
  g_eig[key] = EigenEntry{lam, W, Q};
  g_eig_bytes += entry_bytes(n);
  return 0;
}

}  // namespace dst

extern "C" int dirac_st_time_eigen(int32_t nt, double ht, double *lam, double *W, double *Q) {
  dst::clear_error();
  DST_CHECK(lam && W && Q, "output arrays must be set");
  std::vector<dst::cd> l, w, q;
  if (int rc = dst::time_eigen(nt, ht, l, w, q)) return rc;
  for (int k = 0; k < nt; k++) {
    lam[2 * k] = l[k].real();
    lam[2 * k + 1] = l[k].imag();
  }
  for (size_t e = 0; e < (size_t)nt * nt; e++) {
    W[2 * e] = w[e].real();
    W[2 * e + 1] = w[e].imag();
    Q[2 * e] = q[e].real();
    Q[2 * e + 1] = q[e].imag();
  }
  return 0;
}
