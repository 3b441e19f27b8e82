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
  const bool per = P->bc[2 * a] == PSTD_PERIODIC;
  if (half_wall(P->bc[2 * a + 1])) return PSTD_OK;   // dense path only
  if (per) {
    // a periodic axis is its own period: L = n, the Fourier modes of Eq. (fourier_pstd_solution); only the
    // power-of-two kernel (float state) takes it
    if (P->prec == PSTD_FP64 || fft_pow2_lines(n) == 0) return PSTD_OK;
  } else if (!fft_axis_possible(n, P->prec)) {
    return PSTD_OK;
  }
  const int L = per ? n : 2 * (n - 1), N = L / 2;
  f.N = N;
  f.L = L;
  f.periodic = per;
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
  int st = dbl ? upload_complex<double>(tab, &f.tab) : upload_complex<float>(tab, &f.tab);
  if (st != PSTD_OK) return st;
  if (P->prec != PSTD_FP64 && fft_pow2_lines(L) > 0) {
    // fft_pow2_kernel: radix-16 passes, then one pass of the remaining factor 2, 4 or 8.  Per pass after
    // the first, w, w^2, w^4, w^8 for w = e^{-2 pi i (j mod Ns) / (Ns R)}; per thread t < L/16 of a
    // transform, e^{i pi (2t + a) / (2L)} (a = 1 for mixed walls: the multiplier's phase, whose other
    // factors the kernel forms) and e^{-i pi t / L} (the mixed-wall pre-twiddle's)
    int lg = 0;
    while ((1 << lg) < L) ++lg;
    const int np = (lg + 3) / 4, rl = 1 << (lg - 4 * (np - 1)), q = L / 16;
    std::vector<std::complex<double>> tw;
    for (int p = 1, ns = 16; p < np; ++p, ns *= 16) {
      const int R = p < np - 1 ? 16 : rl;
      for (int jm = 0; jm < ns; ++jm)
        for (int e = 1; e <= 8; e *= 2) tw.push_back(std::polar(1.0, -2.0 * pi * jm * e / (static_cast<double>(ns) * R)));
    }
    st = upload_complex<float>(tw, &f.tw);
    const int anti = f.sL * f.sR < 0 ? 1 : 0;
    std::vector<std::complex<double>> hb(q), pre(q);
    for (int t = 0; t < q; ++t) {
      hb[t] = std::polar(1.0, pi * (2.0 * t + anti) / (2.0 * L));
      pre[t] = std::polar(1.0, -pi * t / L);
    }
    if (st == PSTD_OK) st = upload_complex<float>(hb, &f.hb);
    if (st == PSTD_OK && anti) st = upload_complex<float>(pre, &f.pre);
    if (st != PSTD_OK) return st;
  }
  f.ok = true;
  return PSTD_OK;
}

void fft_axis_free(FftAxis* f) {
  if (f->tab) (void)hipFree(f->tab);
  if (f->tw) (void)hipFree(f->tw);
  if (f->hb) (void)hipFree(f->hb);
  if (f->pre) (void)hipFree(f->pre);
  *f = FftAxis();
}
}  // namespace pstd
