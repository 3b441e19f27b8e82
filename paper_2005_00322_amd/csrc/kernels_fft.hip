// FFT path of one axis operator (axes whose extended period 2(n-1) factors into 2, 3 and 5).
//
// The collapsed operators G = T2^{-1} diag(a1) R T1 and D = T1^{-1} diag(a2) R T2 of Table
// transform_choices are staggered spectral derivatives of the field's symmetric extension (each DTT of
// §3.2 is the DFT of a sequence extended evenly or oddly about the walls, Table DTT_wavenumber_groups).
// Along one line, with N = n - 1 and L = 2N:
//   extend   the n node values (G) or the N half-node values (D) to e_j, j = 0 .. L-1, even or odd
//            about each wall as that wall's boundary condition makes the field symmetric;
//   period   L when both walls are alike (NN, DD).  Otherwise (ND, DN) the extension changes sign after
//            L, its wavenumbers are pi (k + 1/2) / N, and the pre-twiddle e^{-i pi j / L} on the input
//            (its conjugate on the output) turns the transform into a plain length-L DFT;
//   multiply the DFT by H_k = i kappa_k exp(i kappa_k s)/L with s = +1/2 (G: nodes -> half nodes) or
//            s = -1/2 (D: half nodes -> nodes).  The Nyquist entry of the periodic case is the real
//            -+pi: the derivative of the cosine interpolant, the entry the DTT tables keep;
//   invert   and keep the n - 1 (G) or n (D) samples of the line.
// H also carries -dt/(rho0 dx) (G) or -dt rho0 c0^2/dx (D), folded in FP64 on the host.
//
// Two real lines share one complex transform (real and imaginary parts); H_{-k} = conj(H_k), so the two
// results come back separated in the real and imaginary parts.  The inverse reuses the forward transform
// through conjugation: IFFT(X) L = conj(FFT(conj(X))).
//
// A block holds F transforms of length L in LDS (F L <= 16384 complex floats or 8192 complex doubles,
// 139 KB with one pad entry per 16) and runs mixed-radix Stockham passes in place: each thread reads its
// butterflies' inputs into registers, the block synchronises, then each thread writes its outputs.  The
// first forward pass reads through the extension rule; the last forward pass applies H.  Each block has
// F L / 16 threads, so a radix-R pass gives every thread 16 / R butterflies.  The field goes from HBM to
// LDS once and the output is read, updated (formed in FP64, rounded once) and written once.
#include <type_traits>

#include "common.h"

namespace pstd {
namespace {

template <typename T>
struct Cx;
template <>
struct Cx<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Cx<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

template <typename V>
using elem_t = std::remove_cv_t<std::remove_reference_t<decltype(V{}.x)>>;

template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V>
__device__ __forceinline__ V conj(V a) {
  return V{a.x, -a.y};
}
// a * (-i)
template <typename V>
__device__ __forceinline__ V mul_mi(V a) {
  return V{a.y, -a.x};
}

// cos and sin of 2 pi k / 16, k = 0..7
constexpr double kC16[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                            0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613};
constexpr double kS16[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                            1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173};

// a * e^{-2 pi i IDX / 16}
template <typename V, int IDX>
__device__ __forceinline__ V w16(V a) {
  if constexpr (IDX == 0) {
    return a;
  } else if constexpr (IDX == 4) {
    return mul_mi(a);
  } else {
    typedef elem_t<V> T;
    const T c = static_cast<T>(kC16[IDX]), s = static_cast<T>(kS16[IDX]);
    return V{a.x * c + a.y * s, a.y * c - a.x * s};
  }
}

// Length-R DFT (forward, natural order) of v in registers, R a power of two up to 16: radix-2
// decimation in time with constant twiddles.
template <typename V, int R, int K = 0>
__device__ __forceinline__ void combine2(V* v, const V* e, const V* o) {
  if constexpr (K < R / 2) {
    const V t = w16<V, K*(16 / R)>(o[K]);
    v[K] = e[K] + t;
    v[K + R / 2] = e[K] - t;
    combine2<V, R, K + 1>(v, e, o);
  }
}
template <typename V, int R>
__device__ __forceinline__ void dft_pow2(V* v) {
  if constexpr (R > 1) {
    V e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    dft_pow2<V, R / 2>(e);
    dft_pow2<V, R / 2>(o);
    combine2<V, R>(v, e, o);
  }
}

template <typename V, int R>
__device__ __forceinline__ void dft(V* v) {
  typedef elem_t<V> T;
  if constexpr (R == 3) {
    const T s1 = static_cast<T>(0.86602540378443864676);  // sin(2 pi / 3)
    const V t1 = v[1] + v[2];
    const V t2 = v[0] - static_cast<T>(0.5) * t1;
    const V t3 = s1 * (v[1] - v[2]);
    v[0] = v[0] + t1;
    v[1] = t2 + mul_mi(t3);
    v[2] = t2 - mul_mi(t3);
  } else if constexpr (R == 5) {
    const T c1 = static_cast<T>(0.30901699437494742410), c2 = static_cast<T>(-0.80901699437494742410);
    const T s1 = static_cast<T>(0.95105651629515357212), s2 = static_cast<T>(0.58778525229247312917);
    const V b1 = v[1] + v[4], b2 = v[2] + v[3];
    const V d1 = v[1] - v[4], d2 = v[2] - v[3];
    const V a0 = v[0];
    const V r1 = a0 + c1 * b1 + c2 * b2, r2 = a0 + c2 * b1 + c1 * b2;
    const V i1 = s1 * d1 + s2 * d2, i2 = s2 * d1 - s1 * d2;
    v[0] = a0 + b1 + b2;
    v[1] = r1 + mul_mi(i1);
    v[4] = r1 - mul_mi(i1);
    v[2] = r2 + mul_mi(i2);
    v[3] = r2 - mul_mi(i2);
  } else {
    dft_pow2<V, R>(v);
  }
}

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// Load entry i of a table at a wave-uniform base with a 32-bit offset (one address register per load).
template <typename V>
__device__ __forceinline__ V ldt(const void* base, int i) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + static_cast<uint32_t>(i) * sizeof(V));
}

// v[r] *= w^r for r = 1 .. R-1 with w^r = tw[t r]: powers of two are loaded, the others are products of
// at most three loaded powers (a few ulp), which keeps live registers low.
template <typename V, int R, int P = 1>
__device__ __forceinline__ void twiddle(V* v, const void* tw, int t, V* w) {
  if constexpr (P < R) {
    if constexpr ((P & (P - 1)) == 0) {
      w[P] = ldt<V>(tw, t * P);
    } else {
      constexpr int hb = 1 << (31 - __builtin_clz(P));
      w[P] = cmul(w[hb], w[P - hb]);
    }
    v[P] = cmul(v[P], w[P]);
    twiddle<V, R, P + 1>(v, tw, t, w);
  }
}

// Value j (0 <= j < L) of the extended, pre-twiddled input sequence of transform f.  The raw samples of
// the line pair sit at entries 0 .. nin-1 of the transform's LDS slot.
template <typename T>
__device__ __forceinline__ typename Cx<T>::type ext_read(const FftArgs& a, const typename Cx<T>::type* z, int f,
                                                         int j) {
  typedef typename Cx<T>::type V;
  const int N = a.N;
  int src = j;
  T sgn = 1;
  if (a.dir == 0) {
    if (j > N) {
      src = 2 * N - j;
      sgn = static_cast<T>(a.sR);
    }
    // a Dirichlet wall node is not an unknown: it enters as 0
    if ((src == 0 && a.sL < 0) || (src == N && a.sR < 0)) sgn = 0;
  } else if (j >= N) {
    src = 2 * N - 1 - j;
    sgn = static_cast<T>(-a.sR);
  }
  const V x = z[pad(f * a.L + src)];
  V r = sgn == 0 ? V{0, 0} : sgn * x;
  if (a.anti) r = cmul(r, ldt<V>(a.om, j));
  return r;
}

// One in-place Stockham pass of radix R over the F transforms of the block.  first: read through the
// extension rule (first forward pass); last: store conj(H_k X_k) (last forward pass).
template <typename T, int R>
__device__ __forceinline__ void stockham_pass(const FftArgs& a, typename Cx<T>::type* z, int Ns, bool first,
                                              bool last) {
  typedef typename Cx<T>::type V;
  constexpr int NB = (16 + R - 1) / R;
  const int L = a.L;
  const int per = L / R;
  const int total = a.F * per;
  const int nt = blockDim.x;
  V v[NB][R];
  int fo[NB], jo[NB];
  // An opaque copy of the thread index: keeps the compiler from hoisting this pass's index arithmetic out
  // of the pass loop, where it would stay live (in registers or spilled) through every other pass.
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int g = tid + b * nt;
    fo[b] = -1;
    if (g < total) {
      const int f = g / per;
      const int j = g - f * per;
      fo[b] = f;
      jo[b] = j;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (first) v[b][r] = ext_read<T>(a, z, f, j + r * per);
        else v[b][r] = z[pad(f * L + j + r * per)];
      }
      if (Ns > 1) {
        V w[R];
        twiddle<V, R>(v[b], a.tw, (j % Ns) * (L / (Ns * R)), w);
      }
      dft<V, R>(v[b]);
    }
  }
  lds_barrier();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (fo[b] >= 0) {
      const int j = jo[b];
      const int k0 = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = k0 + r * Ns;
        V x = v[b][r];
        if (last) x = conj(cmul(ldt<V>(a.H, k), x));
        z[pad(fo[b] * L + k)] = x;
      }
    }
  }
  lds_barrier();
}

template <typename T>
__device__ __forceinline__ void run_pass(const FftArgs& a, typename Cx<T>::type* z, int R, int Ns, bool first,
                                         bool last) {
  switch (R) {
    case 16: stockham_pass<T, 16>(a, z, Ns, first, last); break;
    case 8: stockham_pass<T, 8>(a, z, Ns, first, last); break;
    case 4: stockham_pass<T, 4>(a, z, Ns, first, last); break;
    case 2: stockham_pass<T, 2>(a, z, Ns, first, last); break;
    case 3: stockham_pass<T, 3>(a, z, Ns, first, last); break;
    default: stockham_pass<T, 5>(a, z, Ns, first, last); break;
  }
}

template <typename T>
constexpr int max_threads() {
  return sizeof(T) == 4 ? 1024 : 512;
}

template <typename T>
__global__ __launch_bounds__(max_threads<T>()) void fft_axis_kernel(FftArgs a) {
  typedef typename Cx<T>::type V;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  V* z = reinterpret_cast<V*>(smem);
  // consecutive line groups run back to back on one XCD (blocks are dealt to the 8 XCDs in turn)
  int64_t grp = blockIdx.x;
  if (a.xcd_spread) grp = static_cast<int64_t>(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
  if (grp >= a.groups) return;
  const int W = 2 * a.F;
  const int nt = blockDim.x;
  const int tid = threadIdx.x;
  const int L = a.L;
  int64_t b = 0, l0;
  int nl;
  if (a.contig) {
    l0 = grp * W;
    nl = static_cast<int>(min<int64_t>(W, a.ncols - l0));
  } else {
    b = grp / a.gpb;
    l0 = (grp - b * a.gpb) * W;
    nl = static_cast<int>(min<int64_t>(W, a.ncols - l0));
  }
  const T* X = static_cast<const T*>(a.X) + b * a.x_bstride;
  T* Y = static_cast<T*>(a.Y) + b * a.y_bstride;
  const T* S = a.scale ? static_cast<const T*>(a.scale) + b * a.y_bstride : nullptr;

  // ---- load: line c of the group -> part (c & 1) of transform c / 2, entries 0 .. nin-1
  {
    const int nin = a.nin;
    const int cnt = W * nin;
    T* zs = reinterpret_cast<T*>(z);
    for (int e0 = 0; e0 < cnt; e0 += 8 * nt) {
      T v[8];
      int c[8], k[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + tid + u * nt;
        if (a.contig) {
          c[u] = e / nin;
          k[u] = e - c[u] * nin;
        } else {
          c[u] = e % W;
          k[u] = e / W;
        }
        const bool ok = e < cnt && c[u] < nl;
        const int64_t off = a.contig ? (l0 + c[u]) * nin + k[u] : static_cast<int64_t>(k[u]) * a.ncols + l0 + c[u];
        v[u] = ok ? X[off] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + tid + u * nt;
        if (e < cnt) zs[2 * pad((c[u] >> 1) * L + k[u]) + (c[u] & 1)] = v[u];
      }
    }
  }
  lds_barrier();

  // ---- forward transform with the extension on input and H on output, then the inverse
  // passes 0 .. npass-1: forward transform; npass .. 2 npass-1: the inverse (forward of the conjugate)
  int Ns = 1;
  for (int q = 0; q < 2 * a.npass; ++q) {
    const int p = q < a.npass ? q : q - a.npass;
    if (p == 0) Ns = 1;
    const int R = a.radix[p];
    run_pass<T>(a, z, R, Ns, q == 0, q == a.npass - 1);
    Ns *= R;
  }

  // ---- epilogue: Y = beta Y + alpha scale out, formed in FP64
  {
    const int nout = a.nout;
    const int cnt = W * nout;
    for (int e0 = 0; e0 < cnt; e0 += 4 * nt) {
      T yv[4], sv[4], ov[4];
      int64_t off[4];
      bool ok[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + tid + u * nt;
        int c, m;
        if (a.contig) {
          c = e / nout;
          m = e - c * nout;
        } else {
          c = e % W;
          m = e / W;
        }
        ok[u] = e < cnt && c < nl;
        off[u] = a.contig ? (l0 + c) * nout + m : static_cast<int64_t>(m) * a.ncols + l0 + c;
        yv[u] = ok[u] && a.beta != 0.0 ? Y[off[u]] : T(0);
        sv[u] = ok[u] && S ? S[off[u]] : T(1);
        ov[u] = 0;
        if (e < cnt) {
          V w = conj(z[pad((c >> 1) * L + m)]);
          if (a.anti) w = cmul(w, conj(ldt<V>(a.om, m)));
          ov[u] = (c & 1) ? w.y : w.x;
          // pressure at a Dirichlet wall node stays 0
          if (a.dir == 1 && ((m == 0 && a.sL < 0) || (m == a.N && a.sR < 0))) ov[u] = 0;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (ok[u])
          Y[off[u]] = static_cast<T>(a.beta * static_cast<double>(yv[u]) +
                                     a.alpha * static_cast<double>(sv[u]) * static_cast<double>(ov[u]));
    }
  }
}

template <typename T>
hipError_t launch_typed(const FftArgs& a, hipStream_t s) {
  static bool configured = false;
  const int cap = fft_capacity(sizeof(T) == 8);
  const size_t lds = static_cast<size_t>(cap + cap / 16) * 2 * sizeof(T);
  if (!configured) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fft_axis_kernel<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    configured = true;
  }
  const int threads = a.F * a.L / 16;
  const size_t shm = static_cast<size_t>(a.F * a.L + (a.F * a.L) / 16) * 2 * sizeof(T);
  int64_t blocks = a.groups;
  if (a.xcd_spread) blocks = round_up(blocks, 8);
  hipLaunchKernelGGL(fft_axis_kernel<T>, dim3(static_cast<unsigned>(blocks)), dim3(threads), shm, s, a);
  return hipGetLastError();
}

}  // namespace

int fft_capacity(bool dbl) { return dbl ? 8192 : 16384; }

hipError_t launch_fft_axis(bool dbl, const FftArgs& a, hipStream_t s) {
  return dbl ? launch_typed<double>(a, s) : launch_typed<float>(a, s);
}

}  // namespace pstd
