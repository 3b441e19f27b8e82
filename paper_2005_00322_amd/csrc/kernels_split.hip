// Split-bfloat16 per-axis contraction on MFMA with the fused leapfrog update (FP32 state).
//
// Same operation as kernels_contract.hip, Y = beta*Y + alpha*scale.*(A X) along one axis, but the
// product is formed as  A_hi X_hi + A_hi X_lo + A_lo X_hi  with bfloat16 operands and FP32
// accumulation: A = A_hi + A_lo is split from FP64 on the host, X = X_hi + X_lo is split from FP32 while
// a K-slice is staged into LDS.  The dropped A_lo X_lo term is below 2^-16 of the product.
//
// MFMA v_mfma_f32_32x32x16_bf16: lane l supplies P[l%32][8*(l/32) .. +7] and Q[l%32][8*(l/32) .. +7]
// (both operands read as rows of a [row][k] LDS tile, 16 bytes per lane) and receives
// C[8*(r/4) + 4*(l/32) + r%4][l%32] in accumulator register r.  Output columns follow the lane index,
// so the operand whose rows are unit-stride in Y goes to the Q port:
//   strided layout   (Y[b][m][c]): P = operator rows m, Q = field columns c
//   contiguous layout (Y[r][m]):   P = field rows r,   Q = operator rows m
// Blocks sharing one field tile are placed on the same XCD back to back so the field tile is fetched
// from HBM once and re-read from that XCD's L2.
#include "common.h"

namespace pstd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct SArgs {
  const uint16_t* Ahi;
  const uint16_t* Alo;
  int lda, M, K;
  const float* X;
  float* Y;
  int64_t ncols, batch, x_bstride, y_bstride;
  int op_tiles;        // tiles along the operator rows
  int64_t fld_tiles;   // tiles along the field (columns or rows) times batch
  float alpha, beta;
  const float* scale;
};

constexpr int BK = 32;          // K slice staged per iteration (two MFMA K-steps)
constexpr int LDK = BK + 8;     // LDS row stride in bf16 elements (80 bytes: conflict-free 16-byte reads)

__device__ __forceinline__ void split2(float x, __bf16& hi, __bf16& lo) {
  hi = static_cast<__bf16>(x);
  lo = static_cast<__bf16>(x - static_cast<float>(hi));
}

template <bool CONTIG, int BP, int BQ, int WP, int WQ>
__global__ __launch_bounds__(64 * WP * WQ) void split_kernel(SArgs a) {
  constexpr int NT = 64 * WP * WQ;
  constexpr int WTP = BP / WP, WTQ = BQ / WQ;
  constexpr int TP = WTP / 32, TQ = WTQ / 32;
  static_assert(TP >= 1 && TQ >= 1, "wave tile must be a multiple of 32x32");
  // operator tile rows and field tile extent in this layout
  constexpr int BOP = CONTIG ? BQ : BP;   // operator rows per block
  constexpr int BFL = CONTIG ? BP : BQ;   // field columns (strided) or rows (contiguous) per block
  constexpr int OPCH = BOP * (BK / 8);    // 16-byte chunks of one operator part per slice
  constexpr int OPC_PER_T = (OPCH + NT - 1) / NT;
  constexpr int FLG = BFL * (BK / 8);     // (field line, 8-k group) pairs per slice
  constexpr int FLG_PER_T = (FLG + NT - 1) / NT;

  __shared__ __attribute__((aligned(16))) __bf16 Ph[BP * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Pl[BP * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Qh[BQ * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Ql[BQ * LDK];
  __bf16* Oh = CONTIG ? Qh : Ph;   // operator tile
  __bf16* Ol = CONTIG ? Ql : Pl;
  __bf16* Fh = CONTIG ? Ph : Qh;   // field tile
  __bf16* Fl = CONTIG ? Pl : Ql;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wp = wave % WP, wq = wave / WP;

  // tile coordinates: XCD-grouped when the field tile count allows it
  const int64_t t = blockIdx.x;
  int op_t;
  int64_t fl_t;
  if ((a.fld_tiles & 7) == 0) {
    const int64_t xcd = t & 7, slot = t >> 3;
    op_t = static_cast<int>(slot % a.op_tiles);
    fl_t = (slot / a.op_tiles) * 8 + xcd;
  } else {
    op_t = static_cast<int>(t % a.op_tiles);
    fl_t = t / a.op_tiles;
  }
  int64_t b, f0;
  if (CONTIG) {
    b = 0;
    f0 = fl_t * BFL;
  } else {
    const int64_t per = (a.ncols + BFL - 1) / BFL;
    b = fl_t / per;
    f0 = (fl_t % per) * BFL;
  }
  const int o0 = op_t * BOP;
  const float* X = a.X + b * a.x_bstride;

  // register staging of one slice
  uint4 rOh[OPC_PER_T], rOl[OPC_PER_T];
  float rF[FLG_PER_T][8];

  auto load_slice = [&](int k0) {
#pragma unroll
    for (int i = 0; i < OPC_PER_T; ++i) {
      const int e = tid + i * NT;
      if (e < OPCH) {
        const int r = e / (BK / 8), ch = e % (BK / 8);
        const size_t off = static_cast<size_t>(o0 + r) * a.lda + k0 + ch * 8;
        rOh[i] = *reinterpret_cast<const uint4*>(a.Ahi + off);
        rOl[i] = *reinterpret_cast<const uint4*>(a.Alo + off);
      }
    }
#pragma unroll
    for (int i = 0; i < FLG_PER_T; ++i) {
      const int e = tid + i * NT;
      if (CONTIG) {
        // field rows r, 8 consecutive k: lanes e%4 cover one 32-k row segment
        const int r = e / (BK / 8), g = e % (BK / 8);
        const int64_t gr = f0 + r;
        const int kb = k0 + g * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          rF[i][j] = (e < FLG && gr < a.ncols && kb + j < a.K) ? X[gr * a.K + kb + j] : 0.f;
      } else {
        // field column c, 8 consecutive k: lanes take consecutive columns (coalesced rows of X)
        const int c = e % BFL, g = e / BFL;
        const int64_t gc = f0 + c;
        const int kb = k0 + g * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          rF[i][j] = (e < FLG && gc < a.ncols && kb + j < a.K) ? X[static_cast<int64_t>(kb + j) * a.ncols + gc] : 0.f;
      }
    }
  };

  auto store_slice = [&]() {
#pragma unroll
    for (int i = 0; i < OPC_PER_T; ++i) {
      const int e = tid + i * NT;
      if (e < OPCH) {
        const int r = e / (BK / 8), ch = e % (BK / 8);
        *reinterpret_cast<uint4*>(Oh + r * LDK + ch * 8) = rOh[i];
        *reinterpret_cast<uint4*>(Ol + r * LDK + ch * 8) = rOl[i];
      }
    }
#pragma unroll
    for (int i = 0; i < FLG_PER_T; ++i) {
      const int e = tid + i * NT;
      if (e < FLG) {
        int line, g;
        if (CONTIG) {
          line = e / (BK / 8);
          g = e % (BK / 8);
        } else {
          line = e % BFL;
          g = e / BFL;
        }
        bf16x8 h, l;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __bf16 hj, lj;
          split2(rF[i][j], hj, lj);
          h[j] = hj;
          l[j] = lj;
        }
        *reinterpret_cast<bf16x8*>(Fh + line * LDK + g * 8) = h;
        *reinterpret_cast<bf16x8*>(Fl + line * LDK + g * 8) = l;
      }
    }
  };

  f32x16 acc[TP][TQ];
#pragma unroll
  for (int i = 0; i < TP; ++i)
#pragma unroll
    for (int j = 0; j < TQ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  load_slice(0);
  for (int k0 = 0; k0 < a.K; k0 += BK) {
    __syncthreads();
    store_slice();
    __syncthreads();
    if (k0 + BK < a.K) load_slice(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      bf16x8 ph[TP], pl[TP], qh[TQ], ql[TQ];
      const int koff = kk + 8 * (lane >> 5);
#pragma unroll
      for (int i = 0; i < TP; ++i) {
        const int row = wp * WTP + i * 32 + (lane & 31);
        ph[i] = *reinterpret_cast<const bf16x8*>(Ph + row * LDK + koff);
        pl[i] = *reinterpret_cast<const bf16x8*>(Pl + row * LDK + koff);
      }
#pragma unroll
      for (int j = 0; j < TQ; ++j) {
        const int row = wq * WTQ + j * 32 + (lane & 31);
        qh[j] = *reinterpret_cast<const bf16x8*>(Qh + row * LDK + koff);
        ql[j] = *reinterpret_cast<const bf16x8*>(Ql + row * LDK + koff);
      }
#pragma unroll
      for (int i = 0; i < TP; ++i)
#pragma unroll
        for (int j = 0; j < TQ; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pl[i], qh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph[i], ql[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph[i], qh[j], acc[i][j], 0, 0, 0);
        }
    }
  }

  // fused update epilogue; lanes 0..31 write 32 consecutive floats of one output line
  float* Y = a.Y + b * a.y_bstride;
  const float* S = a.scale ? a.scale + b * a.y_bstride : nullptr;
#pragma unroll
  for (int i = 0; i < TP; ++i)
#pragma unroll
    for (int j = 0; j < TQ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int prow = wp * WTP + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int qcol = wq * WTQ + j * 32 + (lane & 31);
        int64_t idx;
        bool ok;
        if (CONTIG) {
          const int64_t rr = f0 + prow;
          const int m = o0 + qcol;
          ok = rr < a.ncols && m < a.M;
          idx = rr * a.M + m;
        } else {
          const int m = o0 + prow;
          const int64_t c = f0 + qcol;
          ok = m < a.M && c < a.ncols;
          idx = static_cast<int64_t>(m) * a.ncols + c;
        }
        if (ok) {
          float v = a.alpha * acc[i][j][r];
          if (S) v *= S[idx];
          Y[idx] = (a.beta == 0.f) ? v : a.beta * Y[idx] + v;
        }
      }
}

template <bool CONTIG, int BP, int BQ, int WP, int WQ>
hipError_t launch_s(const ContractArgs& c, hipStream_t s) {
  constexpr int BOP = CONTIG ? BQ : BP;
  constexpr int BFL = CONTIG ? BP : BQ;
  static_assert(BOP <= kRowPad && kRowPad % BOP == 0 && kColPad % BK == 0, "padding");
  SArgs a;
  a.Ahi = static_cast<const uint16_t*>(c.A);
  a.Alo = static_cast<const uint16_t*>(c.A_lo);
  a.lda = c.lda;
  a.M = c.M;
  a.K = c.K;
  a.X = static_cast<const float*>(c.X);
  a.Y = static_cast<float*>(c.Y);
  a.ncols = c.ncols;
  a.batch = c.batch;
  a.x_bstride = c.x_bstride;
  a.y_bstride = c.y_bstride;
  a.alpha = c.alpha;
  a.beta = c.beta;
  a.scale = static_cast<const float*>(c.scale);
  a.op_tiles = (c.M + BOP - 1) / BOP;
  a.fld_tiles = ((c.ncols + BFL - 1) / BFL) * (CONTIG ? 1 : c.batch);
  const int64_t blocks = a.fld_tiles * a.op_tiles;
  if (blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((split_kernel<CONTIG, BP, BQ, WP, WQ>), dim3(static_cast<unsigned>(blocks)), dim3(64 * WP * WQ),
                     0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_contract_split(const ContractArgs& c, bool contiguous, hipStream_t s) {
  if (contiguous) return launch_s<true, 128, 128, 2, 2>(c, s);
  return launch_s<false, 128, 128, 2, 2>(c, s);
}

}  // namespace pstd
