// Dense per-axis contraction on MFMA with the leapfrog update fused into the epilogue (FP32 / FP64).
//
// One call applies an axis operator A (M x K, constants folded in) along one axis of a field X and
// updates the field Y on the other grid in place:  Y = beta * Y + alpha * scale .* (A X).
// This is one half of Eq. (dtt_pstd_solution) for one axis: the forward transform, k-space multiply
// with the sine<->cosine switch and inverse transform collapsed into one matrix, then the
// finite-difference time update.
//
// Two layouts:
//   strided     the contracted axis is not the last one.  X is viewed as [batch][K][C] and Y as
//               [batch][M][C] (C = product of the trailing extents, unit stride):
//               Y[b][m][c] += sum_k A[m][k] X[b][k][c]              (a GEMM  A * X_b)
//   contiguous  the contracted axis is the last one.  X is [R][K], Y is [R][M]:
//               Y[r][m] += sum_k X[r][k] A[m][k]                    (a GEMM  X * A^T)
// Both are computed as C^T-free MFMA tiles: the operator always feeds the MFMA "A" port (rows m) and
// the field the "B" port (columns c or r), so both layouts share the inner loop.
//
// FP32 accuracy: a long FP32 accumulation of the cancelling terms of a spectral derivative loses more than
// the FP32 rounding of the operator and the state together (about 1e-5 against 2e-6 relative L2 after
// 2000 steps of a 256 x 256 box).  The FP32 kernel therefore sums each BK-deep K slice on the MFMA in
// FP32 and adds the slice sums into FP64 registers; the FP64 kernel accumulates in FP64 throughout.
//
// MFMA v_mfma_{f32,f64}_16x16x4: lane l holds A[l%16][l/16] and B[l/16][l%16].  Accumulator register
// r of lane l holds C[4*(l/16)+r][l%16] for f32 but C[4*r+l/16][l%16] for f64 (measured on gfx950).
#include "common.h"

namespace pstd {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<float> {
  using acc_t = f32x4;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mma<double> {
  using acc_t = f64x4;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename T>
struct KArgs {
  const T* A;
  int lda, M, K;
  const T* X;
  T* Y;
  int64_t ncols, x_bstride, y_bstride;
  double alpha, beta;
  const T* scale;
};

// BM x BN output tile per block, BK-deep K slices staged in LDS; WM x WN waves of 64 lanes.
template <typename T, bool CONTIG, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void contract_kernel(KArgs<T> a) {
  constexpr int NT = 64 * WM * WN;
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  static_assert(TM >= 1 && TN >= 1 && BK % 4 == 0, "tile shape");
  using acc_t = typename Mma<T>::acc_t;

  __shared__ T As[BM][BK + 1];
  __shared__ T Xs[CONTIG ? BN : BK][CONTIG ? BK + 1 : BN + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int m0 = blockIdx.y * BM;
  const int64_t n0 = static_cast<int64_t>(blockIdx.x) * BN;
  const int64_t b = blockIdx.z;
  const T* X = a.X + b * a.x_bstride;

  constexpr bool kFlush = sizeof(T) == 4;   // FP32: flush slice sums into FP64 registers
  acc_t acc[TM][TN];
  double accd[kFlush ? TM : 1][kFlush ? TN : 1][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  if (kFlush) {
#pragma unroll
    for (int i = 0; i < (kFlush ? TM : 1); ++i)
#pragma unroll
      for (int j = 0; j < (kFlush ? TN : 1); ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) accd[i][j][r] = 0.0;
  }

  for (int k0 = 0; k0 < a.K; k0 += BK) {
    lds_barrier();
    // operator and field slices: every load of the slice is issued before the first LDS store.
    // The operator is zero padded on the host (no bounds checks); the field is zero-filled outside
    // [0,K) x [0,ncols).
    constexpr int AIT = BM * BK / NT, XIT = BN * BK / NT;
    static_assert(AIT * NT == BM * BK && XIT * NT == BN * BK, "tile must split evenly over the block");
    T av_[AIT], xv_[XIT];
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      const int e = tid + it * NT;
      av_[it] = a.A[static_cast<int64_t>(m0 + e / BK) * a.lda + k0 + e % BK];
    }
#pragma unroll
    for (int it = 0; it < XIT; ++it) {
      const int e = tid + it * NT;
      if (CONTIG) {
        const int64_t gr = n0 + e / BK;
        const int gk = k0 + e % BK;
        xv_[it] = (gr < a.ncols && gk < a.K) ? X[gr * a.K + gk] : T(0);
      } else {
        const int64_t gc = n0 + e % BN;
        const int gk = k0 + e / BN;
        xv_[it] = (gc < a.ncols && gk < a.K) ? X[static_cast<int64_t>(gk) * a.ncols + gc] : T(0);
      }
    }
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      const int e = tid + it * NT;
      As[e / BK][e % BK] = av_[it];
    }
#pragma unroll
    for (int it = 0; it < XIT; ++it) {
      const int e = tid + it * NT;
      if (CONTIG) Xs[e / BK][e % BK] = xv_[it];
      else Xs[e / BN][e % BN] = xv_[it];
    }
    lds_barrier();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) av[i] = As[wm * WTM + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = wn * WTN + j * 16 + (lane & 15);
        bv[j] = CONTIG ? Xs[col][kk + (lane >> 4)] : Xs[kk + (lane >> 4)][col];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = Mma<T>::mma(av[i], bv[j], acc[i][j]);
    }
    if (kFlush) {
#pragma unroll
      for (int i = 0; i < (kFlush ? TM : 1); ++i)
#pragma unroll
        for (int j = 0; j < (kFlush ? TN : 1); ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) accd[i][j][r] += static_cast<double>(acc[i][j][r]);
          acc[i][j] = acc_t{0, 0, 0, 0};
        }
    }
  }

  // fused update epilogue: every load of Y (and of the map) first, then every store
  T* Y = a.Y + b * a.y_bstride;
  const T* S = a.scale ? a.scale + b * a.y_bstride : nullptr;
  auto out_index = [&](int i, int j, int r) -> int64_t {
    const int64_t col = n0 + wn * WTN + j * 16 + (lane & 15);
    const int m = m0 + wm * WTM + i * 16 + (sizeof(T) == 8 ? 4 * r + (lane >> 4) : 4 * (lane >> 4) + r);
    if (m >= a.M || col >= a.ncols) return -1;
    return CONTIG ? col * a.M + m : static_cast<int64_t>(m) * a.ncols + col;
  };
  T yv[TM][TN][4], sv[TM][TN][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t idx = out_index(i, j, r);
        yv[i][j][r] = (idx >= 0 && a.beta != 0.0) ? Y[idx] : T(0);
        sv[i][j][r] = (idx >= 0 && S) ? S[idx] : T(1);
      }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t idx = out_index(i, j, r);
        if (idx < 0) continue;
        // the product, the map factor and the update are formed in FP64 and rounded once
        const double prod = kFlush ? accd[kFlush ? i : 0][kFlush ? j : 0][r] : static_cast<double>(acc[i][j][r]);
        const double v = a.alpha * prod * static_cast<double>(sv[i][j][r]);
        Y[idx] = static_cast<T>(a.beta * static_cast<double>(yv[i][j][r]) + v);
      }
}

template <typename T, int BM, int BN, int BK, int WM, int WN>
hipError_t launch_t(const ContractArgs& c, bool contiguous, hipStream_t s) {
  KArgs<T> a;
  a.A = static_cast<const T*>(c.A);
  a.lda = c.lda;
  a.M = c.M;
  a.K = c.K;
  a.X = static_cast<const T*>(c.X);
  a.Y = static_cast<T*>(c.Y);
  a.ncols = c.ncols;
  a.x_bstride = c.x_bstride;
  a.y_bstride = c.y_bstride;
  a.alpha = c.alpha_d;
  a.beta = c.beta_d;
  a.scale = static_cast<const T*>(c.scale);
  const int64_t nb = (c.ncols + BN - 1) / BN;
  const int64_t mb = (c.M + BM - 1) / BM;
  if (nb > 0x7fffffff || mb > 65535 || c.batch > 65535 || c.batch < 1) return hipErrorInvalidConfiguration;
  static_assert(kRowPad % BM == 0 && kColPad % BK == 0, "operator padding must cover whole tiles");
  dim3 grid(static_cast<unsigned>(nb), static_cast<unsigned>(mb), static_cast<unsigned>(c.batch));
  if (contiguous)
    hipLaunchKernelGGL((contract_kernel<T, true, BM, BN, BK, WM, WN>), grid, dim3(64 * WM * WN), 0, s, a);
  else
    hipLaunchKernelGGL((contract_kernel<T, false, BM, BN, BK, WM, WN>), grid, dim3(64 * WM * WN), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_contract_fp32(const ContractArgs& c, bool contiguous, hipStream_t s) {
  return launch_t<float, 64, 64, 16, 2, 2>(c, contiguous, s);
}

hipError_t launch_contract_fp64(const ContractArgs& c, bool contiguous, hipStream_t s) {
  return launch_t<double, 64, 64, 8, 2, 2>(c, contiguous, s);
}

}  // namespace pstd
