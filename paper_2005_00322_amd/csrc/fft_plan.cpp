// Host tables of the FFT path (kernels_fft.hip): the radix plan, the two-level table of roots of unity
// (formed in FP64, rounded once to the state dtype) and the magnitude factors of the spectral multipliers.
#include <cmath>
#include <complex>

#include "common.h"

namespace pstd {

bool fft_factor(int L, int* npass, int* radix) {
  if (L < 16 || L % 16 != 0) return false;
  int m = L, a = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++a;
  }
  int np = 0;
  int r[16];
  for (int i = 0; i < a / 4; ++i) r[np++] = 16;
  if (a % 4) r[np++] = 1 << (a % 4);
  while (m % 3 == 0 && np < 16) {
    r[np++] = 3;
    m /= 3;
  }
  while (m % 5 == 0 && np < 16) {
    r[np++] = 5;
    m /= 5;
  }
  if (m != 1 || np > 8) return false;
  *npass = np;
  for (int i = 0; i < np; ++i) radix[i] = r[i];
  return true;
}

bool fft_axis_possible(int n, int prec) {
  int np, r[8];
  const int L = 2 * (n - 1);
  return fft_factor(L, &np, r) && L <= fft_capacity(prec == PSTD_FP64);
}

namespace {

template <typename T>
int upload_complex(const std::vector<std::complex<double>>& h, void** out) {
  std::vector<T> v(2 * h.size());
  for (size_t i = 0; i < h.size(); ++i) {
    v[2 * i] = static_cast<T>(h[i].real());
    v[2 * i + 1] = static_cast<T>(h[i].imag());
  }
  if (hipMalloc(out, v.size() * sizeof(T)) != hipSuccess) return fail(PSTD_E_OOM, "hipMalloc of an FFT table failed");
  PSTD_HIP(hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return PSTD_OK;
}

}  // namespace

int fft_axis_setup(pstd_plan_s* P, int a, double sG, double sD) {
  FftAxis& f = P->fft[a];
  const int n = static_cast<int>(P->n[a]);
  if (!fft_axis_possible(n, P->prec) || P->bc[2 * a] == PSTD_PERIODIC || half_wall(P->bc[2 * a + 1]))
    return PSTD_OK;  // dense path only
  const int N = n - 1, L = 2 * N;
  f.N = N;
  f.L = L;
  fft_factor(L, &f.npass, f.radix);
  f.sL = P->bc[2 * a] == PSTD_DIRICHLET ? -1 : 1;
  f.sR = P->bc[2 * a + 1] == PSTD_DIRICHLET ? -1 : 1;
  // roots of unity w^t, w = e^{-2 pi i / 4L}: w^l for l < 64, then w^{64 h} for h < 4L / 64
  const double pi = M_PI;
  const int L4 = 4 * L;
  std::vector<std::complex<double>> tab(64 + L4 / 64);
  for (int l = 0; l < 64; ++l) tab[l] = std::polar(1.0, -2.0 * pi * l / L4);
  for (int h = 0; h < L4 / 64; ++h) tab[64 + h] = std::polar(1.0, -2.0 * pi * (64.0 * h) / L4);
  // |H_k| = |kappa_k| c / L with kappa_k = pi m_k / N: the kernel multiplies m_k by pi c / (N L)
  f.kfac[0] = pi * sG / (static_cast<double>(N) * L);
  f.kfac[1] = pi * sD / (static_cast<double>(N) * L);
  const bool dbl = P->prec == PSTD_FP64;
  const int st = dbl ? upload_complex<double>(tab, &f.tab) : upload_complex<float>(tab, &f.tab);
  if (st != PSTD_OK) return st;
  f.ok = true;
  return PSTD_OK;
}

void fft_axis_free(FftAxis* f) {
  if (f->tab) (void)hipFree(f->tab);
  *f = FftAxis();
}
}  // namespace pstd
