// FP64 host construction of the per-axis PSTD operators.
//
// For one axis with n pressure nodes (walls on nodes 0 and n-1, implied period M = 2(n-1)) and the
// boundary pair of Table transform_choices, the velocity step of Eq. (dtt_pstd_solution_a) applies
//     G = T2^{-1} R12 diag(a1 k) T1            (p nodes -> staggered points)
// and the pressure step of Eq. (dtt_pstd_solution_b) applies
//     D = T1^{-1} R21 diag(a2 k) T2            (staggered points -> p nodes),
// where T1/T2 are the FFTW-convention DCT/DST of §3.2, T^{-1} = T_pair / M per Eq.
// (inverse_transforms), k_n are the wavenumbers of Table DTT_wavenumber_groups and R12/R21 move the
// k-space entries between the two transforms' wavenumber ranges (dropping or zero-filling the DC and
// Nyquist entries, appendix tables "Differentiation with staggered grids").  The product is formed once
// per (n, case) in double precision; the GPU then applies the collapsed matrices as one contraction
// per axis, which is the same linear map as the three-stage recipe.
#include <cmath>
#include <map>
#include <mutex>
#include <thread>

#include "common.h"

namespace pstd {
namespace {

enum Kind { COS = 0, SIN = 1 };

struct Transform {
  Kind kind;
  int type;
};

// FFTW REDFT/RODFT definitions (unnormalised): entry (k, j) of the length-L forward transform.
double dtt_entry(Transform t, int L, int k, int j) {
  const double pi = M_PI;
  if (t.kind == COS) {
    switch (t.type) {
      case 1:  // REDFT00
        if (j == 0) return 1.0;
        if (j == L - 1) return (k % 2) ? -1.0 : 1.0;
        return 2.0 * std::cos(pi * j * k / (L - 1));
      case 2:  // REDFT10
        return 2.0 * std::cos(pi * (j + 0.5) * k / L);
      case 3:  // REDFT01
        if (j == 0) return 1.0;
        return 2.0 * std::cos(pi * j * (k + 0.5) / L);
      default:  // REDFT11
        return 2.0 * std::cos(pi * (j + 0.5) * (k + 0.5) / L);
    }
  }
  switch (t.type) {
    case 1:  // RODFT00
      return 2.0 * std::sin(pi * (j + 1.0) * (k + 1.0) / (L + 1));
    case 2:  // RODFT10
      return 2.0 * std::sin(pi * (j + 0.5) * (k + 1.0) / L);
    case 3:  // RODFT01
      if (j == L - 1) return (k % 2) ? -1.0 : 1.0;
      return 2.0 * std::sin(pi * (j + 1.0) * (k + 0.5) / L);
    default:  // RODFT11
      return 2.0 * std::sin(pi * (j + 0.5) * (k + 0.5) / L);
  }
}

// Logical period of a length-L sample (Table DTT_wavenumber_groups).
int dtt_period(Transform t, int L) {
  if (t.type == 1) return t.kind == COS ? 2 * (L - 1) : 2 * (L + 1);
  return 2 * L;
}

// Eq. (inverse_transforms) for types 1..4: the inverse of T_j is T_pair / M.
Transform inverse_partner(Transform t) {
  if (t.type == 2) return {t.kind, 3};
  if (t.type == 3) return {t.kind, 2};
  return t;
}

// Wavenumber index n of output entry m (Table DTT_wavenumber_groups): DST-I/II start at n = 1.
int wave_index(Transform t, int m) { return (t.kind == SIN && t.type <= 2) ? m + 1 : m; }
bool antiperiodic(Transform t) { return t.type >= 3; }

struct CaseInfo {
  Transform T1, T2;
  double a1, a2;
};

// Table transform_choices.
CaseInfo case_info(AxisCase c) {
  switch (c) {
    case CASE_NN: return {{COS, 1}, {SIN, 2}, -1.0, +1.0};
    case CASE_ND: return {{COS, 3}, {SIN, 4}, -1.0, +1.0};
    case CASE_DN: return {{SIN, 3}, {COS, 4}, +1.0, -1.0};
    default:      return {{SIN, 1}, {COS, 2}, +1.0, -1.0};
  }
}

std::vector<double> dense(Transform t, int L) {
  std::vector<double> T(static_cast<size_t>(L) * L);
  for (int k = 0; k < L; ++k)
    for (int j = 0; j < L; ++j) T[static_cast<size_t>(k) * L + j] = dtt_entry(t, L, k, j);
  return T;
}

// out (Lo x Li) = Inv (Lo x Lo, = partner(Tout)/M) * S (Lo x Li), rows split across threads.
void matmul(const std::vector<double>& A, const std::vector<double>& B, std::vector<double>& C, int Mr,
            int Kc, int Nc) {
  C.assign(static_cast<size_t>(Mr) * Nc, 0.0);
  auto work = [&](int r0, int r1) {
    for (int i = r0; i < r1; ++i) {
      double* c = &C[static_cast<size_t>(i) * Nc];
      for (int k = 0; k < Kc; ++k) {
        const double a = A[static_cast<size_t>(i) * Kc + k];
        if (a == 0.0) continue;
        const double* b = &B[static_cast<size_t>(k) * Nc];
        for (int j = 0; j < Nc; ++j) c[j] += a * b[j];
      }
    }
  };
  const int64_t flops = static_cast<int64_t>(Mr) * Kc * Nc;
  unsigned nt = flops > (1 << 22) ? std::max(1u, std::min(16u, std::thread::hardware_concurrency())) : 1u;
  if (nt == 1) {
    work(0, Mr);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) {
    int r0 = static_cast<int>(static_cast<int64_t>(Mr) * t / nt);
    int r1 = static_cast<int>(static_cast<int64_t>(Mr) * (t + 1) / nt);
    th.emplace_back(work, r0, r1);
  }
  for (auto& x : th) x.join();
}

// Build  Out = Tout^{-1} * Reindex(diag(sign*k) * Tin)  as an (Lout x Lin) matrix (without the k factor
// when with_k is false: a change of sampling grid only).
std::vector<double> collapsed(Transform Tin, int Lin, Transform Tout, int Lout, double sign, int M,
                              bool with_k = true) {
  std::vector<double> Fin = dense(Tin, Lin);
  // k-space matrix with the rows re-indexed from Tin's wavenumber range onto Tout's.
  std::vector<double> S(static_cast<size_t>(Lout) * Lin, 0.0);
  const double shift = antiperiodic(Tin) ? 0.5 : 0.0;
  for (int mo = 0; mo < Lout; ++mo) {
    const int nw = wave_index(Tout, mo);
    int mi = -1;
    for (int m = 0; m < Lin; ++m)
      if (wave_index(Tin, m) == nw) { mi = m; break; }
    if (mi < 0) continue;  // wavenumber absent from the forward range: zero entry
    const double k = with_k ? 2.0 * M_PI * (nw + shift) / M : 1.0;  // dx = 1
    for (int j = 0; j < Lin; ++j) S[static_cast<size_t>(mo) * Lin + j] = sign * k * Fin[static_cast<size_t>(mi) * Lin + j];
  }
  std::vector<double> Inv = dense(inverse_partner(Tout), Lout);
  for (double& v : Inv) v /= M;
  std::vector<double> Out;
  matmul(Inv, S, Out, Lout, Lout, Lin);
  return Out;
}

std::mutex g_cache_mu;
std::map<std::pair<int, int>, AxisTables> g_cache;

}  // namespace

// A periodic axis, Eq. (fourier_pstd_solution): both operators are circulant.  With k_m = 2 pi m / n
// over the signed indices of §2 (m = -n/2 .. n/2 - 1 for even n), entry (j, l) of G is
// (1/n) sum_m Re(i k_m e^{i k_m (j - l + 1/2)}) = -(1/n) sum_m k_m sin(k_m (j - l + 1/2)), and of D the same
// with j - l - 1/2 (the Nyquist term is real, so the sums are exact).
static AxisTables periodic_tables(int n) {
  std::vector<double> g(n), d(n);
  const int m_lo = -(n / 2), m_hi = (n - 1) / 2;
  for (int r = 0; r < n; ++r) {
    double sg = 0.0, sd = 0.0;
    for (int m = m_lo; m <= m_hi; ++m) {
      const double k = 2.0 * M_PI * m / n;
      sg -= k * std::sin(k * (r + 0.5));
      sd -= k * std::sin(k * (r - 0.5));
    }
    g[r] = sg / n;
    d[r] = sd / n;
  }
  AxisTables t;
  t.n = n;
  t.c = CASE_PP;
  t.G.assign(static_cast<size_t>(n) * n, 0.0);
  t.D.assign(static_cast<size_t>(n) * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int l = 0; l < n; ++l) {
      const int r = ((j - l) % n + n) % n;
      t.G[static_cast<size_t>(j) * n + l] = g[r];
      t.D[static_cast<size_t>(j) * n + l] = d[r];
    }
  t.kmax = 2.0 * M_PI * (n / 2) / n;
  return t;
}

// A wall on node 0 and a wall half a step beyond node n-1 (groups III/IV of Table
// DTT_wavenumber_groups, types V-VIII, implied period M = 2n - 1).  The forward DTT of each sequence is
// the matrix of its sampled modes, cos(k x) or sin(k x) with k = 2 pi (m + s) / M (s = 0 when both walls
// are of one kind, 1/2 otherwise); the symmetric extension over one period makes the modes orthogonal
// under the weights w = 1/2 on a sample lying on a wall, 1 elsewhere, with squared norm M/4 (M/2 for
// k = 0 and k = pi), so the inverse is the transposed, weighted mode matrix divided by the norms.  Then
//   G = Psi diag(s1 k) Phi^{-1},  D = Phi diag(s2 k) Psi^{-1}
// with Phi the p modes on the nodes and Psi the u modes on the staggered points.
struct HalfWallModes {
  bool left_n, right_n;
  double shift;
  int p_lo, u_count;                 // first p sample, number of u samples
  int m1_lo, m1_hi, m2_lo, m2_hi;    // mode index ranges of p and u
};

HalfWallModes half_wall_modes(int n, AxisCase c) {
  HalfWallModes h{};
  h.left_n = (c == CASE_NNH || c == CASE_NDH);
  h.right_n = (c == CASE_NNH || c == CASE_DNH);
  h.shift = (h.left_n == h.right_n) ? 0.0 : 0.5;
  h.p_lo = h.left_n ? 0 : 1;
  h.u_count = h.right_n ? n - 1 : n;
  if (h.left_n && h.right_n) { h.m1_lo = 0; h.m1_hi = n - 1; h.m2_lo = 1; h.m2_hi = n - 1; }
  else if (h.left_n)         { h.m1_lo = 0; h.m1_hi = n - 1; h.m2_lo = 0; h.m2_hi = n - 1; }
  else if (h.right_n)        { h.m1_lo = 0; h.m1_hi = n - 2; h.m2_lo = 0; h.m2_hi = n - 2; }
  else                       { h.m1_lo = 1; h.m1_hi = n - 1; h.m2_lo = 0; h.m2_hi = n - 1; }
  return h;
}

static AxisTables half_wall_tables(int n, AxisCase c) {
  const HalfWallModes h = half_wall_modes(n, c);
  const double M = 2.0 * n - 1.0;
  auto kof = [&](int m) { return 2.0 * M_PI * (m + h.shift) / M; };
  auto norm = [&](int m) { return (2.0 * (m + h.shift) == 0.0 || 2.0 * (m + h.shift) == M) ? M / 2.0 : M / 4.0; };
  auto pmode = [&](int m, double x) { return h.left_n ? std::cos(kof(m) * x) : std::sin(kof(m) * x); };
  auto umode = [&](int m, double x) { return h.left_n ? std::sin(kof(m) * x) : std::cos(kof(m) * x); };
  const double s1 = h.left_n ? -1.0 : 1.0, s2 = -s1;
  // modes shared by p and u (a mode with k = 0 has no derivative)
  const int lo = std::max(h.m1_lo, h.m2_lo), hi = std::min(h.m1_hi, h.m2_hi), nm = hi - lo + 1;
  // G = A (n x nm) * B (nm x n): A = u modes on all n staggered points times s1 k / norm, B = weighted p modes
  std::vector<double> A(static_cast<size_t>(n) * nm), B(static_cast<size_t>(nm) * n, 0.0);
  std::vector<double> Cm(static_cast<size_t>(n) * nm), Em(static_cast<size_t>(nm) * n, 0.0);
  for (int q = 0; q < nm; ++q) {
    const int m = lo + q;
    const double k = kof(m), nr = norm(m);
    for (int r = 0; r < n; ++r) {
      A[static_cast<size_t>(r) * nm + q] = umode(m, r + 0.5) * s1 * k / nr;
      Cm[static_cast<size_t>(r) * nm + q] = pmode(m, r) * s2 * k / nr;
    }
    for (int j = h.p_lo; j < n; ++j)
      B[static_cast<size_t>(q) * n + j] = (j == 0 ? 0.5 : 1.0) * pmode(m, j);
    for (int j = 0; j < h.u_count; ++j)
      Em[static_cast<size_t>(q) * n + j] = (j == n - 1 ? 0.5 : 1.0) * umode(m, j + 0.5);
  }
  AxisTables t;
  t.n = n;
  t.c = c;
  matmul(A, B, t.G, n, nm, n);
  matmul(Cm, Em, t.D, n, nm, n);
  t.kmax = kof(h.m1_hi);
  return t;
}

double axis_kmax(int n, AxisCase c) {
  if (c == CASE_PP) return 2.0 * M_PI * (n / 2) / n;
  if (c >= CASE_NNH) {
    const HalfWallModes h = half_wall_modes(n, c);
    return 2.0 * M_PI * (h.m1_hi + h.shift) / (2.0 * n - 1.0);
  }
  const CaseInfo ci = case_info(c);
  const bool left_d = (c == CASE_DN || c == CASE_DD);
  const bool right_d = (c == CASE_ND || c == CASE_DD);
  const int Lp = (right_d ? n - 2 : n - 1) - (left_d ? 1 : 0) + 1;
  const double shift = antiperiodic(ci.T1) ? 0.5 : 0.0;
  return 2.0 * M_PI * (wave_index(ci.T1, Lp - 1) + shift) / (2.0 * (n - 1));
}

// Collocated differentiation (§3.3) and half-step interpolation (§3.4).  Differentiating swaps a
// sequence's symmetry (symmetric <-> antisymmetric), shifting by half a step swaps whole-sample and
// half-sample ends; either way the inverse transform is the one of the resulting symmetry.  On the nodes
// the sequence of the symmetry opposite to p's is transformed by the other kind of T1 (same type); its
// sample includes the node of a Dirichlet wall and excludes the node of a Neumann wall.  On the staggered
// points the opposite symmetry to u's is transformed by the other kind of T2.
std::vector<double> resample_table(int n, AxisCase c, int kind, int* rows, int* cols) {
  const CaseInfo ci = case_info(c);
  const bool left_d = (c == CASE_DN || c == CASE_DD);
  const bool right_d = (c == CASE_ND || c == CASE_DD);
  const int p_lo = left_d ? 1 : 0, Lp = (right_d ? n - 2 : n - 1) - p_lo + 1;
  const int q_lo = left_d ? 0 : 1, Lq = (right_d ? n - 1 : n - 2) - q_lo + 1;
  const int m = n - 1, M = 2 * (n - 1);
  const Transform Q1{ci.T1.kind == COS ? SIN : COS, ci.T1.type};
  const Transform Q2{ci.T2.kind == COS ? SIN : COS, ci.T2.type};
  std::vector<double> out;
  if (kind == 2) {  // d/dx on the nodes: n x n
    *rows = n;
    *cols = n;
    const std::vector<double> s = collapsed(ci.T1, Lp, Q1, Lq, ci.a1, M);
    out.assign(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i < Lq; ++i)
      for (int j = 0; j < Lp; ++j) out[static_cast<size_t>(q_lo + i) * n + p_lo + j] = s[static_cast<size_t>(i) * Lp + j];
  } else if (kind == 3) {  // d/dx on the staggered points: m x m
    *rows = m;
    *cols = m;
    out = collapsed(ci.T2, m, Q2, m, ci.a2, M);
  } else if (kind == 4) {  // nodes -> staggered points: m x n
    *rows = m;
    *cols = n;
    const std::vector<double> s = collapsed(ci.T1, Lp, Q2, m, 1.0, M, false);
    out.assign(static_cast<size_t>(m) * n, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < Lp; ++j) out[static_cast<size_t>(i) * n + p_lo + j] = s[static_cast<size_t>(i) * Lp + j];
  } else {  // staggered points -> nodes: n x m
    *rows = n;
    *cols = m;
    const std::vector<double> s = collapsed(ci.T2, m, Q1, Lq, 1.0, M, false);
    out.assign(static_cast<size_t>(n) * m, 0.0);
    for (int i = 0; i < Lq; ++i)
      for (int j = 0; j < m; ++j) out[static_cast<size_t>(q_lo + i) * m + j] = s[static_cast<size_t>(i) * m + j];
  }
  return out;
}

const AxisTables& axis_tables(int n, AxisCase c) {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  auto key = std::make_pair(n, static_cast<int>(c));
  auto it = g_cache.find(key);
  if (it != g_cache.end()) return it->second;
  if (c == CASE_PP) return g_cache.emplace(key, periodic_tables(n)).first->second;
  if (c >= CASE_NNH) return g_cache.emplace(key, half_wall_tables(n, c)).first->second;

  const CaseInfo ci = case_info(c);
  const bool left_d = (c == CASE_DN || c == CASE_DD);
  const bool right_d = (c == CASE_ND || c == CASE_DD);
  const int p_lo = left_d ? 1 : 0;
  const int p_hi = right_d ? n - 2 : n - 1;
  const int Lp = p_hi - p_lo + 1;
  const int Lu = n - 1;
  const int M = 2 * (n - 1);

  AxisTables t;
  t.n = n;
  t.c = c;
  // velocity operator: p sample (Lp) -> u (Lu)
  std::vector<double> g = collapsed(ci.T1, Lp, ci.T2, Lu, ci.a1, M);
  // pressure operator: u (Lu) -> p sample (Lp)
  std::vector<double> d = collapsed(ci.T2, Lu, ci.T1, Lp, ci.a2, M);
  t.G.assign(static_cast<size_t>(Lu) * n, 0.0);
  t.D.assign(static_cast<size_t>(n) * Lu, 0.0);
  for (int i = 0; i < Lu; ++i)
    for (int j = 0; j < Lp; ++j) t.G[static_cast<size_t>(i) * n + (p_lo + j)] = g[static_cast<size_t>(i) * Lp + j];
  for (int i = 0; i < Lp; ++i)
    for (int j = 0; j < Lu; ++j) t.D[static_cast<size_t>(p_lo + i) * Lu + j] = d[static_cast<size_t>(i) * Lu + j];
  // largest wavenumber of the pressure basis
  const double shift = antiperiodic(ci.T1) ? 0.5 : 0.0;
  t.kmax = 2.0 * M_PI * (wave_index(ci.T1, Lp - 1) + shift) / M;
  return g_cache.emplace(key, std::move(t)).first->second;
}

}  // namespace pstd
