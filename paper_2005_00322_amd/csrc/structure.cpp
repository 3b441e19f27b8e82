// Toeplitz-plus-Hankel form of the collapsed per-axis operators (host, FP64).
//
// Every operator of §3 is a forward trig transform, a diagonal and an inverse trig transform.  A product
// of a cosine or sine of (r + a)θ by one of (c + b)θ is a sum of two trig functions of (r - c)θ and
// (r + c)θ, so summing over the modes gives, away from the walls,
//     A[r][c] = f(r - c) + g(r + c)
// (the derivative of the periodic extension of §3.2 evaluated at the output points: the direct image of
// the input node gives the Toeplitz part and its mirror image about a wall the Hankel part).  Only the
// first and last row and column deviate, by one factor each: a wall node counted once instead of twice
// in the extension (factor 1/2), or a Dirichlet node kept at zero (factor 0).  So
//     A = diag(wr) (F + H) diag(wc)
// with wr and wc equal to one except at their two ends.  The split-bf16 contraction uses this to form
// the operator slices on the chip from the 2 (R + C) values of f and g instead of reading R x C entries.
//
// The decomposition is found from the matrix itself (no case analysis): g from the differences along
// diagonals of the interior block, f from its entries, the end weights by least squares on the
// boundary lines, the few diagonals that only reach a boundary line or corner from those entries; then
// every entry is checked against the reconstruction.  f and g are fixed only up to one constant per
// parity class of r + c (f + a, g - a leaves A unchanged); the constants are chosen to minimise the sum
// of squares of f and g so that forming f + g in FP32 cancels as little as possible.
#include <cmath>
#include <vector>

#include "common.h"

namespace pstd {

bool toeplitz_hankel(const double* A, int R, int C, double tol, std::vector<double>* f_out,
                     std::vector<double>* g_out, double w[4], double* resid_out) {
  if (R < 6 || C < 6) return false;
  const int nd = R + C - 1;   // f(d), d in [1 - C, R - 1], stored at d + C - 1;  g(s), s in [0, R + C - 2]
  std::vector<double> f(nd, 0.0), g(nd, 0.0);
  std::vector<char> fk(nd, 0), gk(nd, 0);
  auto at = [&](int r, int c) { return A[static_cast<size_t>(r) * C + c]; };
  auto F = [&](int d) -> double& { return f[d + C - 1]; };
  auto Fk = [&](int d) -> char& { return fk[d + C - 1]; };
  double amax = 0.0;
  for (size_t i = 0; i < static_cast<size_t>(R) * C; ++i) amax = std::fmax(amax, std::fabs(A[i]));
  if (!(amax > 0.0) || !std::isfinite(amax)) return false;

  // interior block rows 1..R-2, columns 1..C-2: g(s + 2) - g(s) = A[r+1][c+1] - A[r][c] with r + c = s
  g[2] = g[3] = 0.0;
  gk[2] = gk[3] = 1;
  for (int s = 4; s <= R + C - 4; ++s) {
    int r = std::max(1, s - 2 - (C - 3));
    int c = s - 2 - r;
    if (r > R - 3 || c < 1) return false;
    g[s] = g[s - 2] + at(r + 1, c + 1) - at(r, c);
    gk[s] = 1;
  }
  for (int d = 3 - C; d <= R - 3; ++d) {
    const int r = std::max(1, d + 1), c = r - d;
    if (c < 1 || c > C - 2 || r > R - 2) return false;
    F(d) = at(r, c) - g[r + c];
    Fk(d) = 1;
  }
  // end weights from the boundary-line entries whose two diagonals are known
  struct Line { bool row; int idx; };
  const Line lines[4] = {{true, 0}, {true, R - 1}, {false, 0}, {false, C - 1}};
  for (int l = 0; l < 4; ++l) {
    double num = 0.0, den = 0.0, lmax = 0.0;
    const int len = lines[l].row ? C : R;
    for (int t = 1; t < len - 1; ++t) {
      const int r = lines[l].row ? lines[l].idx : t, c = lines[l].row ? t : lines[l].idx;
      lmax = std::fmax(lmax, std::fabs(at(r, c)));
      const int d = r - c, s = r + c;
      if (!Fk(d) || !gk[s]) continue;
      const double p = F(d) + g[s];
      num += at(r, c) * p;
      den += p * p;
    }
    if (lmax <= 1e-12 * amax) {
      w[l] = 0.0;                       // a zero line (to the tables' rounding) is held at exactly zero
    } else {
      if (!(den > 0.0)) return false;
      double v = num / den;
      const double half = std::round(2.0 * v) / 2.0;
      if (std::fabs(v - half) < 1e-10) v = half;
      w[l] = v;
    }
  }
  // diagonals that reach only boundary lines: take each from a line with a nonzero weight
  auto settle = [&](int r, int c, double wt) {
    if (wt == 0.0) return;
    const int d = r - c, s = r + c;
    if (Fk(d) && !gk[s]) {
      g[s] = at(r, c) / wt - F(d);
      gk[s] = 1;
    } else if (!Fk(d) && gk[s]) {
      F(d) = at(r, c) / wt - g[s];
      Fk(d) = 1;
    }
  };
  for (int pass = 0; pass < 2; ++pass) {
    for (int t = 1; t < C - 1; ++t) {
      settle(0, t, w[0]);
      settle(R - 1, t, w[1]);
    }
    for (int t = 1; t < R - 1; ++t) {
      settle(t, 0, w[2]);
      settle(t, C - 1, w[3]);
    }
    settle(0, 0, w[0] * w[2]);
    settle(0, C - 1, w[0] * w[3]);
    settle(R - 1, 0, w[1] * w[2]);
    settle(R - 1, C - 1, w[1] * w[3]);
  }
  // gauge: one constant per parity class, least squares on f and g together
  for (int par = 0; par < 2; ++par) {
    double sum = 0.0;
    int cnt = 0;
    for (int d = 1 - C; d <= R - 1; ++d)
      if (((d % 2) + 2) % 2 == par) {
        sum -= F(d);
        ++cnt;
      }
    for (int s = 0; s <= R + C - 2; ++s)
      if (s % 2 == par) {
        sum += g[s];
        ++cnt;
      }
    const double a = sum / cnt;
    for (int d = 1 - C; d <= R - 1; ++d)
      if (((d % 2) + 2) % 2 == par) F(d) += a;
    for (int s = 0; s <= R + C - 2; ++s)
      if (s % 2 == par) g[s] -= a;
  }
  // check every entry
  double resid = 0.0;
  for (int r = 0; r < R; ++r) {
    const double wr = r == 0 ? w[0] : (r == R - 1 ? w[1] : 1.0);
    for (int c = 0; c < C; ++c) {
      const double wc = c == 0 ? w[2] : (c == C - 1 ? w[3] : 1.0);
      const double p = wr * wc * (F(r - c) + g[r + c]);
      resid = std::fmax(resid, std::fabs(p - at(r, c)));
    }
  }
  if (resid_out) *resid_out = resid / amax;
  if (!(resid <= tol * amax)) return false;
  *f_out = f;
  *g_out = g;
  return true;
}

}  // namespace pstd
