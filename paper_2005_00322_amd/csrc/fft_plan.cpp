// Host tables of the FFT path (kernels_fft.hip): radix plan, twiddles, the mixed-wall pre-twiddle and
// the spectral multipliers of G and D, all formed in FP64 and rounded once to the state dtype.
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
  if (!fft_axis_possible(n, P->prec)) return PSTD_OK;  // dense path only
  const int N = n - 1, L = 2 * N;
  f.N = N;
  f.L = L;
  fft_factor(L, &f.npass, f.radix);
  f.sL = P->bc[2 * a] == PSTD_DIRICHLET ? -1 : 1;
  f.sR = P->bc[2 * a + 1] == PSTD_DIRICHLET ? -1 : 1;
  const bool anti = f.sL * f.sR < 0;
  const double pi = M_PI;
  std::vector<std::complex<double>> tw(L), om(L), hg(L), hd(L);
  for (int t = 0; t < L; ++t) tw[t] = std::polar(1.0, -2.0 * pi * t / L);
  for (int j = 0; j < L; ++j) om[j] = std::polar(1.0, -pi * j / L);
  const std::complex<double> I(0.0, 1.0);
  for (int k = 0; k < L; ++k) {
    double kap;
    if (anti) kap = pi * ((k < N ? k : k - L) + 0.5) / N;
    else kap = pi * (k <= N ? k : k - L) / N;
    if (!anti && k == N) {
      // Nyquist: the derivative of the cosine interpolant, real
      hg[k] = -pi * sG / L;
      hd[k] = pi * sD / L;
    } else {
      hg[k] = I * kap * std::polar(1.0, 0.5 * kap) * (sG / L);
      hd[k] = I * kap * std::polar(1.0, -0.5 * kap) * (sD / L);
    }
  }
  const bool dbl = P->prec == PSTD_FP64;
  int st = dbl ? upload_complex<double>(tw, &f.tw) : upload_complex<float>(tw, &f.tw);
  if (st == PSTD_OK && anti) st = dbl ? upload_complex<double>(om, &f.om) : upload_complex<float>(om, &f.om);
  if (st == PSTD_OK) st = dbl ? upload_complex<double>(hg, &f.H[0]) : upload_complex<float>(hg, &f.H[0]);
  if (st == PSTD_OK) st = dbl ? upload_complex<double>(hd, &f.H[1]) : upload_complex<float>(hd, &f.H[1]);
  if (st != PSTD_OK) return st;
  f.ok = true;
  return PSTD_OK;
}

void fft_axis_free(FftAxis* f) {
  if (f->tw) (void)hipFree(f->tw);
  if (f->om) (void)hipFree(f->om);
  for (void* h : f->H)
    if (h) (void)hipFree(h);
  *f = FftAxis();
}

}  // namespace pstd
