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
// H also carries -dt/(rho0 dx) (G) or -dt rho0 c0^2/dx (D).
//
// Two real lines share one complex transform (real and imaginary parts); H_{-k} = conj(H_k), so the two
// results come back separated in the real and imaginary parts.  The inverse reuses the forward transform
// through conjugation: IFFT(X) L = conj(FFT(conj(X))).
//
// Every root of unity the kernel needs (Stockham twiddles, the pre/post-twiddle, the phase of H) is a
// power of w = e^{-2 pi i / 4L}, taken from a two-level table in LDS: w^t = Th[t / 64] Tl[t % 64] (both
// rounded once from FP64 on the host; one complex product).  The block reads the field and the table
// from HBM at the start and the old output values during the last inverse pass, so its only exposed
// global latency is the first one.
//
// A block holds F transforms of length L in LDS (bank-swizzled; 64 KB or less except for single
// transforms above that) and runs mixed-radix Stockham passes in place: each thread reads its
// butterflies' inputs into registers, the block synchronises, then each thread writes its outputs.  Three
// sweeps over LDS apply the extension and pre-twiddle, conj(H X), and the conjugation and post-twiddle.
// Each block has F L / 16 threads, so a radix-R pass gives every thread 16 / R butterflies.  The field
// goes from HBM to LDS once and the output is read, updated (formed in FP64, rounded once) and written
// once.
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

// LDS position of entry j of a transform: bits 4..8 are XORed into bits 0..4, a permutation of every
// aligned group of 32 entries.  Stride-16 and stride-256 Stockham writes then spread over all banks
// without padding.  Each transform occupies a slot of Ls = round_up(L, 32) entries.
__device__ __forceinline__ int sw(int j) { return j ^ ((j >> 4) & 31); }

// q = g / d for 0 <= g < 2^24 through a float reciprocal (one correction step).
__device__ __forceinline__ int fdiv(int g, int d, float inv) {
  int q = static_cast<int>(static_cast<float>(g) * inv);
  const int r = g - q * d;
  q += (r >= d) - (r < 0);
  return q;
}

// w^t, w = e^{-2 pi i / 4L}, 0 <= t < 4L, from the LDS table: entries 0..63 hold w^l, entries 64.. hold
// w^{64 h}.
template <typename V>
__device__ __forceinline__ V root(const V* tab, int t) {
  return cmul(tab[64 + (t >> 6)], tab[t & 63]);
}

// v[r] *= W_L^{t r} = w^{4 t r} for r = 1 .. R-1: powers of two from the table, the others as products of
// at most three of them.
template <typename V, int R, int P = 1>
__device__ __forceinline__ void twiddle(V* v, const V* tab, int t, V* w) {
  if constexpr (P < R) {
    if constexpr ((P & (P - 1)) == 0) {
      w[P] = root(tab, 4 * t * P);
    } else {
      constexpr int hb = 1 << (31 - __builtin_clz(P));
      w[P] = cmul(w[hb], w[P - hb]);
    }
    v[P] = cmul(v[P], w[P]);
    twiddle<V, R, P + 1>(v, tab, t, w);
  }
}

// Entry j (0 <= j < L) of the extended input sequence is sgn * raw[src] (before the pre-twiddle); the
// raw samples of a line pair sit at entries 0 .. nin-1 of the transform's slot.  Selects only.
__device__ __forceinline__ void ext_source(const FftArgs& a, int j, int& src, float& sgn) {
  const int N = a.N;
  if (a.dir == 0) {
    const bool mirror = j > N;
    src = mirror ? 2 * N - j : j;
    sgn = mirror ? static_cast<float>(a.sR) : 1.0f;
    // a Dirichlet wall node is not an unknown: it enters as 0
    sgn = ((src == 0 && a.sL < 0) || (src == N && a.sR < 0)) ? 0.0f : sgn;
  } else {
    const bool mirror = j >= N;
    src = mirror ? 2 * N - 1 - j : j;
    sgn = mirror ? static_cast<float>(-a.sR) : 1.0f;
  }
}

// Each thread owns transform f of the block and the 16 entries lt + u L/16 (u < 16) of its slot; a
// radix-R pass gives it the butterflies lt + b L/16, b < ceil(16/R) (guarded only when R does not
// divide 16).
struct Lane {
  int f;       // transform of the block
  int lt;      // 0 .. L/16 - 1
  int q;       // L / 16
  int base;    // f * Ls
};

// One in-place Stockham pass of radix R: reads of every butterfly input, a block barrier, then writes.
template <typename T, int R>
__device__ __forceinline__ void stockham_pass(const FftArgs& a, typename Cx<T>::type* z,
                                              const typename Cx<T>::type* tab, const Lane& ln, int Ns) {
  typedef typename Cx<T>::type V;
  constexpr int NB = (16 + R - 1) / R;
  constexpr bool EXACT = 16 % R == 0;
  const int L = a.L;
  const int per = L / R;
  const float inv_ns = 1.0f / static_cast<float>(Ns);
  const int tstep = L / (Ns * R);
  // an opaque copy of the slot index keeps the compiler from hoisting this pass's index arithmetic out
  // of the pass loop, where it would stay live through every other pass
  int lt = ln.lt;
  asm volatile("" : "+v"(lt));
  V v[NB][R];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lt + b * ln.q;
    if (EXACT || j < per) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = z[ln.base + sw(j + r * per)];
      if (Ns > 1) {
        V w[R];
        twiddle<V, R>(v[b], tab, (j - fdiv(j, Ns, inv_ns) * Ns) * tstep, w);
      }
      dft<V, R>(v[b]);
    }
  }
  lds_barrier();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lt + b * ln.q;
    if (EXACT || j < per) {
      const int jq = fdiv(j, Ns, inv_ns);
      const int k0 = jq * Ns * R + (j - jq * Ns);
#pragma unroll
      for (int r = 0; r < R; ++r) z[ln.base + sw(k0 + r * Ns)] = v[b][r];
    }
  }
  lds_barrier();
}

template <typename T>
__device__ __forceinline__ void run_pass(const FftArgs& a, typename Cx<T>::type* z, const typename Cx<T>::type* tab,
                                         const Lane& ln, int R, int Ns) {
  switch (R) {
    case 16: stockham_pass<T, 16>(a, z, tab, ln, Ns); break;
    case 8: stockham_pass<T, 8>(a, z, tab, ln, Ns); break;
    case 4: stockham_pass<T, 4>(a, z, tab, ln, Ns); break;
    case 2: stockham_pass<T, 2>(a, z, tab, ln, Ns); break;
    case 3: stockham_pass<T, 3>(a, z, tab, ln, Ns); break;
    default: stockham_pass<T, 5>(a, z, tab, ln, Ns); break;
  }
}

// In-place sweep over the thread's 16 entries j = lt + u L/16: every thread reads E of them (with their
// table values) before any thread writes.  With E = 16 one batch covers the block, so g may read any
// entry of the slot.
template <int E, typename V, typename Fn>
__device__ __forceinline__ void sweep(V* z, const Lane& ln, Fn g) {
  int lt = ln.lt;
  asm volatile("" : "+v"(lt));
#pragma unroll
  for (int u0 = 0; u0 < 16; u0 += E) {
    V v[E];
#pragma unroll
    for (int u = 0; u < E; ++u) v[u] = g.read(z, ln.base, lt + (u0 + u) * ln.q);
    lds_barrier();
#pragma unroll
    for (int u = 0; u < E; ++u) z[ln.base + sw(lt + (u0 + u) * ln.q)] = v[u];
    lds_barrier();
  }
}

// Extension of the raw samples to the full period, times the pre-twiddle e^{-i pi j / L} = w^{2j} for
// mixed walls.
template <typename V>
struct ExtendOp {
  const FftArgs& a;
  const V* tab;
  __device__ V read(const V* z, int base, int j) const {
    int src;
    float sgn;
    ext_source(a, j, src, sgn);
    V x = z[base + sw(src)];
    x = V{x.x * sgn, x.y * sgn};
    if (a.anti) x = cmul(x, root(tab, 2 * j));
    return x;
  }
};

// conj(H_k X_k).  H_k = i kappa_k (c/L) e^{i s kappa_k / 2} with kappa_k = pi m_k / N, m_k = k (+1/2 for
// mixed walls) folded to the signed frequency; the phase is w^{-2 s m_k} and kfac = pi c / (N L).
template <typename V>
struct MultiplyOp {
  const FftArgs& a;
  const V* tab;
  __device__ V read(const V* z, int base, int k) const {
    typedef elem_t<V> T;
    const int L = a.L;
    const bool neg = a.anti ? k >= a.N : k > a.N;
    const int m2 = 2 * k + a.anti - (neg ? 2 * L : 0);   // 2 m_k
    const int L4 = 4 * L;
    int t = a.dir == 0 ? -m2 : m2;                        // w^{-2 s m_k}: s = +1 for G, -1 for D
    t += t < 0 ? L4 : 0;
    const V ph = root(tab, t);
    const T mag = static_cast<T>(0.5) * static_cast<T>(m2) * static_cast<T>(a.kfac);
    const V h = V{-mag * ph.y, mag * ph.x};                 // i mag ph
    return conj(cmul(h, z[base + sw(k)]));
  }
};

// Result of the inverse: conjugate back, times the post-twiddle e^{i pi j / L} = w^{4L - 2j} for mixed
// walls.
template <typename V>
struct FinishOp {
  const FftArgs& a;
  const V* tab;
  __device__ V read(const V* z, int base, int j) const {
    const V x = conj(z[base + sw(j)]);
    if (!a.anti) return x;
    return cmul(x, root(tab, j == 0 ? 0 : 4 * a.L - 2 * j));
  }
};

constexpr size_t kSmallLds = 65536;

template <typename T>
constexpr int max_threads() {
  return sizeof(T) == 4 ? 1024 : 512;
}

// BIG: one transform above 64 KB (L > 8192 floats, > 4096 doubles).  Such launches opt in to the larger
// LDS through a function attribute of their own instance; every other launch stays within the 64 KB a
// block may take without it, so the attribute never inflates their per-block allocation.
template <typename T, bool BIG>
__global__ __launch_bounds__(max_threads<T>(), sizeof(T) == 4 ? 5 : 2) void fft_axis_kernel(FftArgs a) {
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
  const int Ls = (L + 31) & ~31;
  int64_t b = 0, l0;
  if (a.contig) {
    l0 = grp * W;
  } else {
    b = grp / a.gpb;
    l0 = (grp - b * a.gpb) * W;
  }
  const int nl = static_cast<int>(min<int64_t>(W, a.ncols - l0));
  const T* X = static_cast<const T*>(a.X) + b * a.x_bstride;
  T* Y = static_cast<T*>(a.Y) + b * a.y_bstride;
  const T* S = a.scale ? static_cast<const T*>(a.scale) + b * a.y_bstride : nullptr;
  const int nin = a.nin, nout = a.nout;
  const float inv_nin = 1.0f / static_cast<float>(nin), inv_nout = 1.0f / static_cast<float>(nout);
  Lane ln;
  ln.q = L / 16;
  ln.f = fdiv(tid, ln.q, 1.0f / static_cast<float>(ln.q));
  ln.lt = tid - ln.f * ln.q;
  ln.base = ln.f * Ls;
  V* tab = z + a.F * Ls;
  const int ntab = 64 + L / 16;
  const V* gtab = static_cast<const V*>(a.tab);

  // element e of the group's input (output) lines: line c, position k along the axis; offsets stay below
  // 2^31 elements (plans hold at most 2^31 points)
  auto in_pos = [&](int e, int& c, int& k) {
    if (a.contig) {
      c = fdiv(e, nin, inv_nin);
      k = e - c * nin;
    } else {
      c = e % W;
      k = e / W;
    }
  };
  auto out_pos = [&](int e, int& c, int& m) {
    if (a.contig) {
      c = fdiv(e, nout, inv_nout);
      m = e - c * nout;
    } else {
      c = e % W;
      m = e / W;
    }
  };
  auto in_off = [&](int c, int k) -> uint32_t {
    return a.contig ? static_cast<uint32_t>((l0 + c) * nin + k) : static_cast<uint32_t>(k * a.ncols + l0 + c);
  };
  auto out_off = [&](int c, int m) -> uint32_t {
    return a.contig ? static_cast<uint32_t>((l0 + c) * nout + m) : static_cast<uint32_t>(m * a.ncols + l0 + c);
  };

  // Every thread takes up to EB input elements of the group per batch (2F lines of at most N + 1 values
  // over F L / 16 threads: at most 16 + 16/N, so 17 covers every N >= 16; longer is looped) and EO
  // output elements per batch.
  constexpr int EB = 17, EO = 8;
  const int cnt_in = W * nin, cnt_out = W * nout;
  const bool read_y = a.beta != 0.0;

  // ---- load: line c of the group -> part (c & 1) of transform c / 2, entries 0 .. nin-1; the root table
  {
    T* zs = reinterpret_cast<T*>(z);
    for (int e0 = 0; e0 < cnt_in; e0 += EB * nt) {
      T v[EB];
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        const int e = e0 + tid + u * nt;
        int c, k;
        in_pos(e, c, k);
        v[u] = (e < cnt_in && c < nl) ? X[in_off(c, k)] : T(0);
      }
      if (e0 == 0)
        for (int i = tid; i < ntab; i += nt) tab[i] = gtab[i];
      int tid3 = threadIdx.x;   // positions recomputed, not kept live across the loads
      asm volatile("" : "+v"(tid3));
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        const int e = e0 + tid3 + u * nt;
        int c, k;
        in_pos(e, c, k);
        if (e < cnt_in) zs[2 * ((c >> 1) * Ls + sw(k)) + (c & 1)] = v[u];
      }
    }
  }
  lds_barrier();

  // ---- extend, forward transform, multiply by H, inverse (the forward transform of the conjugate)
  sweep<16>(z, ln, ExtendOp<V>{a, tab});   // reads other entries of the slot: one batch
  int Ns = 1;
  for (int p = 0; p < a.npass; ++p) {
    run_pass<T>(a, z, tab, ln, a.radix[p], Ns);
    Ns *= a.radix[p];
  }
  sweep<8>(z, ln, MultiplyOp<V>{a, tab});
  Ns = 1;
  for (int p = 0; p + 1 < a.npass; ++p) {
    run_pass<T>(a, z, tab, ln, a.radix[p], Ns);
    Ns *= a.radix[p];
  }
  // the old output values of the first batch are read while the last pass runs; output positions are
  // recomputed from an opaque thread index rather than kept live through the transforms
  int tid2 = threadIdx.x;
  asm volatile("" : "+v"(tid2));
  T yv[EO];
#pragma unroll
  for (int u = 0; u < EO; ++u) {
    const int e = tid2 + u * nt;
    int c, m;
    out_pos(e, c, m);
    yv[u] = (read_y && e < cnt_out && c < nl) ? Y[out_off(c, m)] : T(0);
  }
  run_pass<T>(a, z, tab, ln, a.radix[a.npass - 1], Ns);
  sweep<8>(z, ln, FinishOp<V>{a, tab});

  // ---- epilogue: Y = beta Y + alpha scale out, formed in FP64
  for (int e0 = 0; e0 < cnt_out; e0 += EO * nt) {
    T sv[EO];
#pragma unroll
    for (int u = 0; u < EO; ++u) {
      const int e = e0 + tid2 + u * nt;
      int c, m;
      out_pos(e, c, m);
      const bool ok = e < cnt_out && c < nl;
      sv[u] = (S && ok) ? S[out_off(c, m)] : T(1);
      if (e0 != 0) yv[u] = (read_y && ok) ? Y[out_off(c, m)] : T(0);
    }
#pragma unroll
    for (int u = 0; u < EO; ++u) {
      const int e = e0 + tid2 + u * nt;
      int c, m;
      out_pos(e, c, m);
      if (e < cnt_out && c < nl) {
        const V w = z[(c >> 1) * Ls + sw(m)];
        T ov = (c & 1) ? w.y : w.x;
        // pressure at a Dirichlet wall node stays 0
        if (a.dir == 1 && ((m == 0 && a.sL < 0) || (m == a.N && a.sR < 0))) ov = 0;
        Y[out_off(c, m)] = static_cast<T>(a.beta * static_cast<double>(yv[u]) +
                                          a.alpha * static_cast<double>(sv[u]) * static_cast<double>(ov));
      }
    }
  }
}

// LDS bytes of a launch: F slots of round_up(L, 32) entries and the root table.
template <typename T>
size_t lds_bytes(const FftArgs& a) {
  return static_cast<size_t>(a.F * round_up(a.L, 32) + 64 + a.L / 16) * 2 * sizeof(T);
}

template <typename T>
hipError_t launch_typed(const FftArgs& a, hipStream_t s) {
  const int threads = a.F * a.L / 16;
  const size_t shm = lds_bytes<T>(a);
  int64_t blocks = a.groups;
  if (a.xcd_spread) blocks = round_up(blocks, 8);
  if (shm <= kSmallLds) {
    hipLaunchKernelGGL((fft_axis_kernel<T, false>), dim3(static_cast<unsigned>(blocks)), dim3(threads), shm, s, a);
    return hipGetLastError();
  }
  static bool configured = false;
  if (!configured) {
    const int cap = fft_capacity(sizeof(T) == 8);
    const size_t lds = static_cast<size_t>(cap + 64 + cap / 16) * 2 * sizeof(T);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fft_axis_kernel<T, true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    configured = true;
  }
  hipLaunchKernelGGL((fft_axis_kernel<T, true>), dim3(static_cast<unsigned>(blocks)), dim3(threads), shm, s, a);
  return hipGetLastError();
}

// ---- FP32 transforms of a power-of-two length L = 2^LG, 256 <= L <= 8192 ----------------------------
// The same operator as fft_axis_kernel with the length, the pass plan and the LDS layout fixed at compile
// time, so that index arithmetic is shifts and most LDS accesses of a pass are one of a few base
// registers plus an immediate offset:
//   layout   entry e of a transform at sw(e) (the bank swizzle above), F = 4096 / L transforms per block:
//            32 KB of LDS per block up to L = 4096, so five blocks fit a CU;
//   passes   radix 16, then one radix 2, 4 or 8 pass for the remaining factor; thread t of a transform
//            holds entries t + s L/16 (s < 16) at the start of the first pass and at the end of the last;
//   tables   formed in FP64 on the host and rounded once: per pass after the first, w, w^2, w^4, w^8 for
//            w = W_{Ns R}^{j mod Ns} (the other powers as products of at most four of them); per thread
//            t < L/16, e^{i pi (2t + a)/(2L)} (a = 1 for mixed walls) for the spectral multiplier and
//            e^{-i pi t/L} for the mixed-wall pre-twiddle.  The entries t + s L/16 add a factor
//            e^{+-i pi s/16} (constants) to these;
//   fusion   the extension (and pre-twiddle) is applied as the first pass reads the raw samples; the last
//            forward pass leaves each thread exactly the entries its first inverse pass needs, so
//            conj(H X) and that inverse pass follow in registers; the conjugation (and post-twiddle) is
//            applied as the last inverse pass writes;
//   memory   every thread issues all its loads of the input lines at once, and of the old output values
//            at once, without branches; on unit-stride axes with walls the old output values are loaded
//            with the input (their loads overlap; all but the last one to four per thread, which would
//            spill), on strided and periodic ones in the epilogue (registers);
//   launches one per axis, or the velocity terms of every axis of a step in one launch (below): the
//            blocks of the slower strided axes first, then the unit-stride ones fill the CUs as those end.
template <int LG>
struct Pow2 {
  static constexpr int L = 1 << LG, N = L / 2, Q = L / 16;
  static constexpr int F = L <= 4096 ? 4096 / L : 1;   // transforms per block
  static constexpr int NT = F * Q;                      // threads per block
  static constexpr int NP = (LG + 3) / 4;               // passes
  static constexpr int RL = 1 << (LG - 4 * (NP - 1));   // radix of the last pass
  static constexpr int EPT = 17;                        // input / output elements per thread (2F lines)
  static constexpr int EPT_PER = 32;                    // the same on a periodic axis (L values per line)
  static constexpr int radix(int p) { return p < NP - 1 ? 16 : RL; }
  static constexpr int ns(int p) { return 1 << (4 * p); }
  // offset of pass p's twiddles in the table (passes 1 .. NP-1, four entries per j mod Ns)
  static constexpr int toff(int p) { return p <= 1 ? 0 : toff(p - 1) + 4 * ns(p - 1); }
};

typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

// cos and sin of pi r / 16, r = 0..15
constexpr float kC32[16] = {1.0f, 0.98078528040323044913f, 0.92387953251128675613f, 0.83146961230254523708f,
                            0.70710678118654752440f, 0.55557023301960222474f, 0.38268343236508977173f,
                            0.19509032201612826785f, 0.0f, -0.19509032201612826785f, -0.38268343236508977173f,
                            -0.55557023301960222474f, -0.70710678118654752440f, -0.83146961230254523708f,
                            -0.92387953251128675613f, -0.98078528040323044913f};
constexpr float kS32[16] = {0.0f, 0.19509032201612826785f, 0.38268343236508977173f, 0.55557023301960222474f,
                            0.70710678118654752440f, 0.83146961230254523708f, 0.92387953251128675613f,
                            0.98078528040323044913f, 1.0f, 0.98078528040323044913f, 0.92387953251128675613f,
                            0.83146961230254523708f, 0.70710678118654752440f, 0.55557023301960222474f,
                            0.38268343236508977173f, 0.19509032201612826785f};

// slot + sw(e + OFF) from A = slot + sw(e) (slot a multiple of 256) when e < OFF's lowest set bit and OFF
// is a multiple of 32: OFF's bits 4..8 enter the XOR, its low five bits are zero (otherwise computed in
// full; called with OFF a constant after unrolling)
__device__ __forceinline__ int sw_add(int A, int e, int OFF) {
  return OFF % 32 == 0 ? (A ^ ((OFF >> 4) & 31)) + OFF : A - sw(e) + sw(e + OFF);
}

// An opaque copy of a per-thread index: addresses derived from it are recomputed where they are used
// instead of being kept live (or spilled) from one pass to another that uses the same ones.
__device__ __forceinline__ int fresh(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// w, w^2, w^4, w^8 of pass P for butterfly j
template <int LG, int P>
__device__ __forceinline__ void tw_load(const f2v* __restrict__ tw, int j, f4v (&t)[2]) {
  typedef Pow2<LG> C;
  const f4v* p = reinterpret_cast<const f4v*>(tw + C::toff(P) + 4 * (j & (C::ns(P) - 1)));
  t[0] = p[0];
  t[1] = p[1];
}

// v[r] *= w^r, r = 1 .. R-1, from t = (w, w^2, w^4, w^8)
template <int R>
__device__ __forceinline__ void tw_apply(f2v* v, const f4v (&t)[2]) {
  f2v w[16];
  w[1] = f2v{t[0].x, t[0].y};
  w[2] = f2v{t[0].z, t[0].w};
  w[4] = f2v{t[1].x, t[1].y};
  w[8] = f2v{t[1].z, t[1].w};
#pragma unroll
  for (int p = 3; p < R; ++p) {
    if ((p & (p - 1)) == 0) continue;
    const int hb = 1 << (31 - __builtin_clz(p));
    w[p] = cmul(w[hb], w[p - hb]);
  }
#pragma unroll
  for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
}

// Stockham pass P (P >= 1) of the plan: read, twiddle, DFT; the outputs stay in v for the caller.
template <int LG, int P>
__device__ __forceinline__ void pow2_pass_in(const f2v* __restrict__ z, const f2v* __restrict__ tw, int jt, int A,
                                             f2v (&v)[16]) {
  typedef Pow2<LG> C;
  constexpr int R = C::radix(P), NB = 16 / R, PER = C::L / R;
  jt = fresh(jt);
  A = fresh(A);
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = z[sw_add(A, jt, (i / R) * C::Q + (i % R) * PER)];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    f4v t[2];
    tw_load<LG, P>(tw, jt + b * C::Q, t);
    tw_apply<R>(v + b * R, t);
    dft<f2v, R>(v + b * R);
  }
}

// write of 16 outputs of an Ns = 1 radix-16 pass: entry 16 jt + r
__device__ __forceinline__ void pow2_write_ns1(f2v* z, int slot, int jt, const f2v (&v)[16]) {
  jt = fresh(jt);
  slot = fresh(slot);
  // sw(16 jt + r) = (16 jt with bit 4 cleared) + 16 ((jt ^ jt >> 4) & 1) + (r ^ (jt & 15))
  const int base = slot + (16 * jt & ~31) + 16 * ((jt ^ (jt >> 4)) & 1);
  const int x = jt & 15;
#pragma unroll
  for (int r = 0; r < 16; ++r) z[base + (x ^ r)] = v[r];
}

// Stockham write of pass P's outputs (an inner pass: radix 16, Ns >= 16)
template <int LG, int P>
__device__ __forceinline__ void pow2_pass_out(f2v* __restrict__ z, int slot, int jt, const f2v (&v)[16]) {
  typedef Pow2<LG> C;
  constexpr int R = C::radix(P), NS = C::ns(P);
  static_assert(R == 16 && NS >= 16, "inner passes are radix 16");
  jt = fresh(jt);
  slot = fresh(slot);
  if constexpr (NS == 16) {
    // entry k0 + 16 r, k0 = 256 (jt >> 4) + (jt & 15): bits 0..3 are (jt & 15) ^ r, bit 4 is
    // (r ^ jt >> 4) & 1, bits 5.. are 256 (jt >> 4) + 32 (r >> 1)
    const int hi = slot + 256 * (jt >> 4);
    const int b0 = hi + 16 * ((jt >> 4) & 1), b1 = hi + 16 * (((jt >> 4) & 1) ^ 1);
    const int x = jt & 15;
#pragma unroll
    for (int r = 0; r < 16; ++r) z[((r & 1) ? b1 : b0) + (x ^ r) + 32 * (r >> 1)] = v[r];
  } else {
    const int k0 = ((jt / NS) * NS * R) + (jt & (NS - 1));
    const int K = slot + sw(k0);
#pragma unroll
    for (int i = 0; i < 16; ++i) z[(K ^ (((i * NS) >> 4) & 31)) + i * NS] = v[i];
  }
}

template <int LG, int P>
__device__ __forceinline__ void pow2_inner(f2v* z, const f2v* tw, int slot, int jt, int A) {
  if constexpr (P < Pow2<LG>::NP - 1) {
    f2v v[16];
    pow2_pass_in<LG, P>(z, tw, jt, A, v);
    lds_barrier();
    pow2_pass_out<LG, P>(z, slot, jt, v);
    lds_barrier();
    pow2_inner<LG, P + 1>(z, tw, slot, jt, A);
  }
}

// outputs of the last pass (radix RL, NB = 16 / RL butterflies per thread) in the order of the entries
// jt + s L/16: s = b + r NB
template <int LG>
__device__ __forceinline__ void pow2_gather(const f2v (&v)[16], f2v (&u)[16]) {
  constexpr int R = Pow2<LG>::RL, NB = 16 / R;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < R; ++r) u[b + r * NB] = v[b * R + r];
}

// One block of a launch over the line groups of one axis: block `blk` of `nblk` (nblk a multiple of 8
// when the groups are spread per XCD).
template <int LG, bool CONTIG, bool PER>
__device__ __forceinline__ void fft_pow2_block(const FftArgs& a, unsigned blk, unsigned nblk) {
  typedef Pow2<LG> C;
  constexpr int L = C::L, N = C::N, Q = C::Q, W = 2 * C::F, EPT = PER ? C::EPT_PER : C::EPT;
  // the old output values load with the input where they fit the registers (unit stride, walls)
  constexpr bool YPRE = CONTIG && !PER;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  f2v* z = reinterpret_cast<f2v*>(smem);
  const f2v* tw = static_cast<const f2v*>(a.tw);
  int64_t grp = blk;
  if (a.xcd_spread) grp = static_cast<int64_t>(blk % 8) * (nblk / 8) + blk / 8;
  if (grp >= a.groups) return;
  const int tid = threadIdx.x;
  int64_t b = 0, l0;
  if (CONTIG) {
    l0 = grp * W;
  } else {
    b = grp / a.gpb;
    l0 = (grp - b * a.gpb) * W;
  }
  const int nl = static_cast<int>(min<int64_t>(W, a.ncols - l0));
  const int nin = a.nin, nout = a.nout;
  // the group's first line; offsets from there stay below 2^31 elements (plans hold at most 2^31 points)
  const int64_t xo = b * a.x_bstride + (CONTIG ? l0 * nin : l0);
  const int64_t yo = b * a.y_bstride + (CONTIG ? l0 * nout : l0);
  const float* X = static_cast<const float*>(a.X) + xo;
  float* Y = static_cast<float*>(a.Y) + yo;
  const int ld = static_cast<int>(a.ncols);   // strided: elements between consecutive positions of a line
  const float inv_nin = __builtin_amdgcn_rcpf(static_cast<float>(nin));
  const float inv_nout = __builtin_amdgcn_rcpf(static_cast<float>(nout));
  // element e of the group's lines of n values: line c, position k along it.  On a unit-stride axis the
  // lines are consecutive rows, so e is also the element's offset from the group's first one.
  struct Pos {
    int c, k;
    __device__ Pos(int e, int n, float inv) {
      if (CONTIG) {
        c = fdiv(e, n, inv);
        k = e - c * n;
      } else {
        c = e & (W - 1);
        k = e / W;
      }
    }
    // the position of element e + NT (n >= N: at most NT / N + 1 wraps to the next line)
    __device__ void next(int n) {
      if (CONTIG) {
        k += C::NT;
#pragma unroll
        for (int i = 0; i < (C::NT + N - 1) / N; ++i) {
          const bool w = k >= n;
          k -= w ? n : 0;
          c += w ? 1 : 0;
        }
      } else {
        k += C::NT / W;
      }
    }
  };
  auto in_off = [&](int c, int k) { return CONTIG ? c * nin + k : k * ld + c; };
  auto out_off = [&](int c, int m) { return CONTIG ? c * nout + m : m * ld + c; };

  // ---- loads: the input lines and the old output values (W lines of at most N + 1 values, 17 per thread;
  // L values and 32 per thread on a periodic axis)
  const bool read_y = a.beta != 0.0;
  // every thread issues all its loads (an element past the lines reads the group's first element and
  // is dropped), so no load waits behind a branch
  float xv[EPT];
  const int cin = nl * nin, cout = nl * nout;
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = tid + u * C::NT;
    int off;
    bool ok;
    if (CONTIG) {
      off = e;
      ok = e < cin;
    } else {
      const Pos p(e, nin, inv_nin);
      off = in_off(p.c, p.k);
      ok = p.c < nl && p.k < nin;
    }
    const float t = X[ok ? off : 0];
    xv[u] = ok ? t : 0.0f;
  }
  // (the first YP of each thread's values; the rest, among them the last, which only a few threads of a
  // group hold, load in the epilogue: fewer registers through the transforms, where they would spill)
  constexpr int YP = LG >= 12 ? EPT - 1 : EPT - 4;
  float yv[EPT];
  if (YPRE) {
    const int t0 = fresh(tid);
#pragma unroll
    for (int u = 0; u < YP; ++u) {
      const int e = t0 + u * C::NT;
      yv[u] = read_y ? Y[e < cout ? e : 0] : 0.0f;
    }
  }
  {
    // positions recomputed, not kept live across the loads
    float* zs = reinterpret_cast<float*>(z);
    Pos p(fresh(tid), nin, inv_nin);
#pragma unroll
    for (int u = 0; u < EPT; ++u, p.next(nin))
      if (p.c < W && p.k < nin) zs[2 * ((p.c >> 1) * L + sw(p.k)) + (p.c & 1)] = xv[u];
  }
  lds_barrier();

  const int f = tid / Q, jt = tid & (Q - 1);
  const int slot = f * L;
  const int A = slot + sw(jt);   // slot + sw(jt): the layout of transform f
  // the pre-twiddle's per-thread factor (loaded again where it is used last, and the multiplier's just
  // before it is used: neither is kept in registers through the passes)
  const f2v pb = a.anti ? static_cast<const f2v*>(a.pre)[jt] : f2v{1.f, 0.f};
  f2v v[16];
  // ---- first forward pass: extension (mirror about the right wall, sign sR for G, -sR for D; Dirichlet
  // wall nodes enter as 0), pre-twiddle for mixed walls, radix 16 without twiddles
  {
    if (PER) {
      // a periodic line is its own period
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = z[sw_add(A, jt, i * Q)];
    } else {
      const float sg = a.dir == 0 ? static_cast<float>(a.sR) : static_cast<float>(-a.sR);
      const int mo = a.dir == 0 ? -jt : -1 - jt;   // mirrored entry: (16 - r) Q + mo
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = i < 8 ? z[sw_add(A, jt, i * Q)] : z[slot + sw((16 - i) * Q + mo)];
#pragma unroll
      for (int r = 8; r < 16; ++r) v[r] = f2v{v[r].x * sg, v[r].y * sg};
      if (a.dir == 0 && jt == 0) {
        if (a.sL < 0) v[0] = f2v{0.f, 0.f};
        if (a.sR < 0) v[8] = f2v{0.f, 0.f};
      }
    }
    if (a.anti) {
      // e^{-i pi (jt + r Q) / L} = e^{-i pi jt / L} e^{-i pi r / 16}
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = cmul(v[r], cmul(pb, f2v{kC32[r], -kS32[r]}));
    }
    dft<f2v, 16>(v);
    lds_barrier();
    pow2_write_ns1(z, slot, jt, v);
    lds_barrier();
  }
  pow2_inner<LG, 1>(z, tw, slot, jt, A);
  // ---- last forward pass, conj(H X), first inverse pass (radix 16 without twiddles)
  {
    pow2_pass_in<LG, C::NP - 1>(z, tw, jt, A, v);
    f2v u[16];
    pow2_gather<LG>(v, u);
    // H_k = i g_k e^{i sigma pi (t + s L/8) / (2L)} at k = jt + s L/16, t = 2 jt + a (a = 1 for mixed
    // walls), sigma = +1 (G) or -1 (D): the signed frequency 2 m_k = t + s L/8 folded by -2L (which flips
    // the phase's sign) from s = 8 on, g_k = |2 m_k| kfac / 2
    const float sgm = a.dir == 0 ? 1.0f : -1.0f;
    const f2v hb = static_cast<const f2v*>(a.h)[fresh(jt)];
    const f2v B = f2v{hb.x, sgm * hb.y};
    // kfac / 2 as a pair of floats: each g_k is rounded once, not every mode scaled by one rounded factor
    const double khd = 0.5 * a.kfac;
    const float kh = static_cast<float>(khd), kl = static_cast<float>(khd - static_cast<double>(kh));
    const float t = static_cast<float>(2 * jt + a.anti);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const f2v d = cmul(B, f2v{kC32[s], sgm * kS32[s]});
      const float n2 = s < 8 ? static_cast<float>(s * (L / 8)) + t : static_cast<float>((16 - s) * (L / 8)) - t;
      const float g = __builtin_fmaf(kh, n2, kl * n2);
      const f2v p = cmul(d, u[s]);
      u[s] = f2v{-g * p.y, -g * p.x};   // conj(i g p)
    }
    dft<f2v, 16>(u);
    lds_barrier();
    pow2_write_ns1(z, slot, jt, u);
    lds_barrier();
  }
  pow2_inner<LG, 1>(z, tw, slot, jt, A);
  // ---- last inverse pass, conjugation and post-twiddle
  {
    pow2_pass_in<LG, C::NP - 1>(z, tw, jt, A, v);
    f2v u[16];
    pow2_gather<LG>(v, u);
    if (a.anti) {
      const f2v pb2 = static_cast<const f2v*>(a.pre)[fresh(jt)];
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const f2v t = cmul(pb2, f2v{kC32[s], -kS32[s]});   // e^{-i pi j / L}; the post-twiddle is its conjugate
        u[s] = f2v{u[s].x * t.x - u[s].y * t.y, -(u[s].x * t.y + u[s].y * t.x)};   // conj(u) conj(t)
      }
    } else {
#pragma unroll
      for (int s = 0; s < 16; ++s) u[s].y = -u[s].y;
    }
    lds_barrier();
    const int A2 = fresh(A), jt2 = fresh(jt);
#pragma unroll
    for (int i = 0; i < 16; ++i) z[sw_add(A2, jt2, i * Q)] = u[i];
    lds_barrier();
  }

  // ---- epilogue: Y = beta Y + alpha scale out, formed in FP64
  const float* S = a.scale ? static_cast<const float*>(a.scale) + yo : nullptr;
  // positions recomputed from an opaque thread index: the compiler would otherwise keep the load phase's
  // offsets live through the transforms
  const int tid3 = fresh(tid);
  if (YPRE) {
#pragma unroll
    for (int u = YP; u < EPT; ++u) {
      const int e = tid3 + u * C::NT;
      yv[u] = read_y ? Y[e < cout ? e : 0] : 0.0f;
    }
  } else {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const Pos p(tid3 + u * C::NT, nout, inv_nout);
      const bool ok = p.c < nl && p.k < nout;
      yv[u] = read_y ? Y[ok ? out_off(p.c, p.k) : 0] : 0.0f;
    }
  }
#pragma unroll
  for (int u = 0; u < EPT; ++u) asm volatile("" : "+v"(yv[u]));   // widened to FP64 here, not at the load
  const int tid4 = fresh(tid3);
  Pos p(tid4, nout, inv_nout);
#pragma unroll
  for (int u = 0; u < EPT; ++u, p.next(nout)) {
    const int e = tid4 + u * C::NT;
    const int c = p.c, m = p.k;
    if (c < nl && m < nout) {
      const int off = CONTIG ? e : out_off(c, m);
      const float sv = S ? S[off] : 1.0f;
      const f2v v2 = z[(c >> 1) * L + sw(m)];
      float ov = (c & 1) ? v2.y : v2.x;
      // pressure at a Dirichlet wall node stays 0
      if (!PER && a.dir == 1 && ((m == 0 && a.sL < 0) || (m == N && a.sR < 0))) ov = 0.0f;
      Y[off] = static_cast<float>(a.beta * static_cast<double>(yv[u]) +
                                  a.alpha * static_cast<double>(sv) * static_cast<double>(ov));
    }
  }
}

// (second bound: waves per SIMD the registers are planned for, five 4-wave blocks per CU up to L = 4096)
template <int LG, bool CONTIG, bool PER>
__global__ __launch_bounds__(Pow2<LG>::NT, LG <= 12 ? 5 : 2) void fft_pow2_kernel(FftArgs a) {
  fft_pow2_block<LG, CONTIG, PER>(a, blockIdx.x, gridDim.x);
}

// Several axes of one half step in one launch (transforms of one length, all periodic or none): the
// blocks of axis i follow those of axes 0 .. i-1, each axis's range padded as in a launch of its own
// (to a multiple of eight blocks where its line groups spread over the XCDs, so that they spread the
// same way).  Blocks of different axes then share the CUs, and the scheduler places the later ones where
// the earlier ones finish.
struct FftMulti {
  FftArgs a[3];
  unsigned end[3];   // one past the last block of axis i
  int count;
};

template <int LG, bool PER>
__global__ __launch_bounds__(Pow2<LG>::NT, LG <= 12 ? 5 : 2) void fft_pow2_multi_kernel(FftMulti m) {
  unsigned blk = blockIdx.x, lo = 0;
  int i = 0;
  while (i + 1 < m.count && blk >= m.end[i]) lo = m.end[i++];
  const FftArgs& a = m.a[i];
  if (a.contig) fft_pow2_block<LG, true, PER>(a, blk - lo, m.end[i] - lo);
  else fft_pow2_block<LG, false, PER>(a, blk - lo, m.end[i] - lo);
}

int64_t pow2_blocks(const FftArgs& a) { return a.xcd_spread ? round_up(a.groups, 8) : a.groups; }

template <int LG>
hipError_t launch_pow2(const FftArgs& a, hipStream_t s) {
  typedef Pow2<LG> C;
  const size_t shm = static_cast<size_t>(C::F) * C::L * sizeof(f2v);
  const dim3 g(static_cast<unsigned>(pow2_blocks(a))), t(C::NT);
  if (a.periodic) {
    if (a.contig) hipLaunchKernelGGL((fft_pow2_kernel<LG, true, true>), g, t, shm, s, a);
    else hipLaunchKernelGGL((fft_pow2_kernel<LG, false, true>), g, t, shm, s, a);
  } else {
    if (a.contig) hipLaunchKernelGGL((fft_pow2_kernel<LG, true, false>), g, t, shm, s, a);
    else hipLaunchKernelGGL((fft_pow2_kernel<LG, false, false>), g, t, shm, s, a);
  }
  return hipGetLastError();
}

template <int LG>
hipError_t launch_pow2_multi(const FftMulti& m, hipStream_t s) {
  typedef Pow2<LG> C;
  const size_t shm = static_cast<size_t>(C::F) * C::L * sizeof(f2v);
  const dim3 g(static_cast<unsigned>(m.end[m.count - 1])), t(C::NT);
  if (m.a[0].periodic) hipLaunchKernelGGL((fft_pow2_multi_kernel<LG, true>), g, t, shm, s, m);
  else hipLaunchKernelGGL((fft_pow2_multi_kernel<LG, false>), g, t, shm, s, m);
  return hipGetLastError();
}

}  // namespace

int fft_capacity(bool dbl) { return dbl ? 8192 : 16384; }

int fft_max_per_block(bool dbl, int L) {
  const int64_t esz = dbl ? 16 : 8;
  const int64_t room = static_cast<int64_t>(kSmallLds) / esz - 64 - L / 16;   // entries left for the slots
  const int64_t f = room / round_up(L, 32);
  return f < 1 ? 1 : static_cast<int>(f);
}

hipError_t launch_fft_axis(bool dbl, const FftArgs& a, hipStream_t s) {
  return dbl ? launch_typed<double>(a, s) : launch_typed<float>(a, s);
}

int fft_pow2_lines(int L) {
  if (L < 256 || L > 8192 || (L & (L - 1)) != 0) return 0;
  return L <= 4096 ? 2 * (4096 / L) : 2;
}

hipError_t launch_fft_pow2(const FftArgs& a, hipStream_t s) {
  switch (a.L) {
    case 256: return launch_pow2<8>(a, s);
    case 512: return launch_pow2<9>(a, s);
    case 1024: return launch_pow2<10>(a, s);
    case 2048: return launch_pow2<11>(a, s);
    case 4096: return launch_pow2<12>(a, s);
    case 8192: return launch_pow2<13>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fft_pow2_multi(const FftArgs* a, int count, hipStream_t s) {
  if (count < 1 || count > 3) return hipErrorInvalidValue;
  FftMulti m{};
  m.count = count;
  int64_t end = 0;
  for (int i = 0; i < count; ++i) {
    if (a[i].L != a[0].L || a[i].periodic != a[0].periodic) return hipErrorInvalidValue;
    m.a[i] = a[i];
    end += pow2_blocks(a[i]);
    if (end > 0x7fffffff) return hipErrorInvalidValue;
    m.end[i] = static_cast<unsigned>(end);
  }
  switch (a[0].L) {
    case 256: return launch_pow2_multi<8>(m, s);
    case 512: return launch_pow2_multi<9>(m, s);
    case 1024: return launch_pow2_multi<10>(m, s);
    case 2048: return launch_pow2_multi<11>(m, s);
    case 4096: return launch_pow2_multi<12>(m, s);
    case 8192: return launch_pow2_multi<13>(m, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pstd
