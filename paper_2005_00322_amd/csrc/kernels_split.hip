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
//   strided layout   (Y[b][m][c]): P = operator rows m, Q = field columns (b, c)
//   contiguous layout (Y[r][m]):   P = field rows r,   Q = operator rows m
//
// Tiles: 192 operator rows x 256 field lines per block of eight waves (one block per CU: 160 KB of LDS).
// What bounds these launches is the traffic from L2 into the CUs (every block fetches its operator and
// field slices from L2; the field comes from HBM once), so the tile is as large as the accumulators
// allow: per K-slice a block fetches 192 + 256 rows for 192 x 256 outputs, 43% less traffic per output
// than 128 x 128 tiles.  A field tile may span several outer blocks of a strided layout (its lines are
// the flattened (b, c) pairs), so every axis has batch x extent / 256 field tiles.
//
// Pipeline: two LDS buffers and two register sets.  While the MFMAs consume K-slice s from one LDS
// buffer, the global loads of slices s+1 and s+2 are in flight in the two register sets; after the
// MFMAs slice s+1 is split into bf16 hi/lo and written to the other buffer, the loads of slice s+3 are
// issued into the freed register set, and one barrier per slice separates the two buffers.  The
// epilogue issues every load of Y before its first store.  The two operator tiles of a field tile are
// placed on the same XCD back to back, so the field tile comes from HBM once and from that XCD's L2
// for the second.
//
// One block fits a CU, so a launch runs in rounds of one tile per CU, and a last round that holds only
// part of a round's tiles would cost as much as a full one.  When that remainder is at most half a round,
// its field tiles are split into tiles of half the lines (the waves whose lines all lie past them skip
// their MFMAs), which fill the last round across every CU at about two thirds of a full tile's time.
//
// Operators formed on the chip (TH): every operator here is diag(wr) (F + H) diag(wc), F Toeplitz and
// H Hankel (structure.cpp), so an operator slice is built in LDS from two short vectors, Fr[i] =
// f(383 - i) and G[i] = g(i), staged in LDS once per block: entry (r, k) = Fr[k - r + 383] + G[r + k]
// in FP32, split into bf16 hi and lo like the field.  Only the field and the output then travel from
// L2, so the tile takes all the operator rows (up to 384) and 128 field lines: every field element is
// fetched once, and per output the traffic into the CU falls to the field slice and the update.  The
// end weights act on the data instead: wc on the first and last field element of each line as it is
// staged, wr on the first and last output row in the epilogue.  Operator slices sit in LDS without
// padding, their 16-byte chunks XOR-swizzled by row ((row / 4) mod 4) so that the MFMA operand reads
// stay free of bank conflicts.
#include <algorithm>

#include "common.h"

namespace pstd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct SArgs {
  const uint16_t* Ahi;
  uint32_t lo_off;         // byte offset of the lo part from the hi part
  int lda, M, K;
  int mrows;               // allocated (padded) operator rows
  const float* X;
  float* Y;
  int64_t ncols, x_bstride, y_bstride;
  int64_t lines;           // field lines: batch * ncols (strided) or rows (contiguous)
  const float* th;         // TH: [Fr | G], th_len values each
  int th_len;
  float thw[4];            // TH: weights of the first / last output row, first / last input element
  int rw_general;          // TH: rows to scale in the epilogue (a weight other than 0 and 1, or beta != 1)
  uint32_t oob;            // kOOB
  int op_tiles;            // tiles along the operator rows
  int64_t fld_tiles;       // full-width (BF) tiles along the field lines
  int64_t narrow_tiles;    // half-width tiles after them, covering the remaining lines
  float alpha, beta;
  const float* scale;
};

constexpr int BK = 32;            // K slice per pipeline stage (two MFMA K-steps)
constexpr int LDK = BK + 8;       // LDS row stride in bf16 of padded tiles (80 bytes: conflict-free reads)
constexpr int NT = 512;           // eight waves
// operator rows and field lines per tile: stored operators 192 x 256, operators formed on the chip 384 x 128
template <bool TH> constexpr int tile_ops() { return TH ? kThRowsMax : 192; }
template <bool TH> constexpr int tile_lines() { return TH ? 128 : 256; }
constexpr int OP_CH = 192 * (BK / 8) * 2 / NT;  // stored operators: 16-byte chunks (hi and lo) per thread (3)
constexpr int TH_CH = kThRowsMax * (BK / 8) / NT;   // formed operators: rows per thread and slice (3)

typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t kOOB = 0x80000000u;   // byte offset past every buffer used here (all < 2 GiB)

// Raw buffer resource over `bytes` bytes: a load at an offset >= bytes returns 0 without a memory access
// and a store there is dropped, which replaces bounds checks by out-of-range offsets.
__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes), 0x00020000);
}
__device__ __forceinline__ float ld_f32(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void st_f32(rsrc_t r, float v, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ u32x4 ld_b128(rsrc_t r, uint32_t voff) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
}

__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& h, bf16x8& l) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const __bf16 hj = static_cast<__bf16>(x[j]);
    h[j] = hj;
    l[j] = static_cast<__bf16>(x[j] - static_cast<float>(hj));
  }
}

// FMODE: 0 = strided layout, one 4-byte load per field element, 8 consecutive k per thread;
// 1 = contiguous layout, one 4-byte load per element with the lanes along k (two rows of 32 consecutive
// floats per wave instruction, coalesced at any row length and alignment), neighbouring lanes pairing
// their values with a DPP swap so that each lane stores one packed bf16 pair (even lanes the hi parts,
// odd lanes the lo parts); 2 = contiguous layout, two 16-byte loads per 8 floats (X 16-byte aligned and
// K % 4 == 0).
template <bool CONTIG, int FMODE, bool TH>
__global__ __launch_bounds__(NT, 1) void split_kernel(SArgs a) {
  constexpr bool VEC = FMODE == 2;
  constexpr bool LANEK = CONTIG && FMODE == 1;
  constexpr int BO = tile_ops<TH>(), BF = tile_lines<TH>();
  constexpr int FL_G = BF * (BK / 8) / NT;          // 8-float field groups per thread (2, or 1 for TH)
  // ports: P rows and Q rows of the tile, the wave grid over them and each wave's 32 x 32 MFMA tiles
  constexpr int BP = CONTIG ? BF : BO, BQ = CONTIG ? BO : BF;
  constexpr int WP = (CONTIG != TH) ? 4 : 2, WQ = 8 / WP;
  constexpr int TP = BP / WP, TQ = BQ / WQ;          // 64 x 96 (contiguous) or 96 x 64 (strided)
  constexpr int IP = TP / 32, JQ = TQ / 32;
  // the operator's port: rows of BK (swizzled) when formed on the chip, else padded rows like the field
  constexpr bool P_SW = TH && !CONTIG, Q_SW = TH && CONTIG;
  constexpr int P_LD = P_SW ? BK : LDK, Q_LD = Q_SW ? BK : LDK;
  constexpr int P_ELEMS = BP * P_LD, Q_ELEMS = BQ * Q_LD;
  constexpr int BUF_ELEMS = 2 * (P_ELEMS + Q_ELEMS);
  // [buffer][P hi | P lo | Q hi | Q lo]
  __shared__ __attribute__((aligned(16))) __bf16 lds[2 * BUF_ELEMS];
  __shared__ __attribute__((aligned(16))) float sfg[TH ? 2 * kThLen : 4];   // TH: Fr then G
  constexpr int PH = 0, PL = P_ELEMS, QH = 2 * P_ELEMS, QL = 2 * P_ELEMS + Q_ELEMS;
  constexpr int OPH = CONTIG ? QH : PH, OPL = CONTIG ? QL : PL;
  constexpr int FLH = CONTIG ? PH : QH, FLL = CONTIG ? PL : QL;
  // element offset of 16-byte chunk `chunk` of row `row` in a port
  auto p_at = [](int row, int chunk) { return row * P_LD + (P_SW ? (chunk ^ ((row >> 2) & 3)) : chunk) * 8; };
  auto q_at = [](int row, int chunk) { return row * Q_LD + (Q_SW ? (chunk ^ ((row >> 2) & 3)) : chunk) * 8; };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // TH: the field-line port index is the slower one, so that a half-width tile's live waves sit one per SIMD
  const int wp = (CONTIG && TH) ? wave / WQ : wave % WP, wq = (CONTIG && TH) ? wave % WQ : wave / WP;

  // tile coordinates: full-width tiles first, then the half-width ones; the op_tiles tiles of a field
  // tile run on one XCD when the count allows it
  const int64_t full_blocks = a.fld_tiles * a.op_tiles;
  const bool narrow = static_cast<int64_t>(blockIdx.x) >= full_blocks;
  const int64_t t = narrow ? blockIdx.x - full_blocks : blockIdx.x;
  const int64_t nfl = narrow ? a.narrow_tiles : a.fld_tiles;
  int op_t;
  int64_t fl_t;
  if ((nfl & 7) == 0) {
    const int64_t xcd = t & 7, slot = t >> 3;
    op_t = static_cast<int>(slot % a.op_tiles);
    fl_t = (slot / a.op_tiles) * 8 + xcd;
  } else {
    op_t = static_cast<int>(t % a.op_tiles);
    fl_t = t / a.op_tiles;
  }
  const int width = narrow ? BF / 2 : BF;
  const int64_t f0 = narrow ? a.fld_tiles * BF + fl_t * (BF / 2) : fl_t * BF;
  const int64_t lend = min(a.lines, f0 + width);   // lines of this tile: [f0, lend)
  // waves whose field lines all lie past the tile's width have no MFMA work
  const bool wave_live = (CONTIG ? wp * TP : wq * TQ) < width;
  const int o0 = op_t * BO;
  // buffer resources over the whole input and output (both below 2 GiB)
  const uint32_t x_bytes = static_cast<uint32_t>(4 * (CONTIG ? a.lines * a.K : (a.lines / a.ncols) * a.x_bstride));
  const uint32_t y_bytes = static_cast<uint32_t>(4 * (CONTIG ? a.lines * a.M : (a.lines / a.ncols) * a.y_bstride));
  const rsrc_t rX = make_rsrc(a.X, x_bytes);
  const rsrc_t rY = make_rsrc(a.Y, y_bytes);
  const rsrc_t rS = make_rsrc(a.scale ? a.scale : a.Y, a.scale ? y_bytes : 0u);
  const rsrc_t rA = make_rsrc(a.Ahi, TH ? 0u : 2u * a.lo_off);   // hi part then lo part

  // stored operators: this thread's operator chunks (hi and lo parts in one index space); rows past the
  // allocation read the last allocated row (its outputs lie past M and are not stored)
  int op_dst[OP_CH];
  uint32_t op_voff[OP_CH];
  if (!TH) {
#pragma unroll
    for (int i = 0; i < OP_CH; ++i) {
      const int c = tid + i * NT;
      const int part = c / (BO * (BK / 8));
      const int rem = c % (BO * (BK / 8));
      const int row = rem / (BK / 8), chk = rem % (BK / 8);
      op_dst[i] = (part ? OPL : OPH) + row * LDK + chk * 8;
      const int grow = min(o0 + row, a.mrows - 1);
      op_voff[i] = (part ? a.lo_off : 0u) + 2u * static_cast<uint32_t>(grow * a.lda + chk * 8);
    }
  }
  // formed operators: per slice this thread forms rows 3g .. 3g+2 (g = tid / 4) at the 8 k of chunk
  // tid % 4, which take 10 consecutive values of Fr (from th_fb + k0) and 10 of G (from th_gb + k0)
  int th_dst[TH_CH], th_fb = 0, th_gb = 0;
  if (TH) {
    const int g3 = 3 * (tid >> 2), q = tid & 3;
#pragma unroll
    for (int j = 0; j < TH_CH; ++j) th_dst[j] = CONTIG ? q_at(g3 + j, q) : p_at(g3 + j, q);
    th_fb = 8 * q - g3 + (BO - 1) - (TH_CH - 1);
    th_gb = g3 + 8 * q;
    for (int i = tid; i < 2 * a.th_len; i += NT) sfg[i] = a.th[i];
  }
  const float* sF = sfg;
  const float* sG = sfg + (TH ? a.th_len : 0);
  // this thread's field groups: line and first k of 8
  int fl_line[FL_G], fl_grp[FL_G];
  uint32_t fl_voff[FL_G];
  bool fl_ok[FL_G];
#pragma unroll
  for (int i = 0; i < FL_G; ++i) {
    const int e = tid + i * NT;
    fl_line[i] = CONTIG ? e / (BK / 8) : e % BF;
    fl_grp[i] = CONTIG ? e % (BK / 8) : e / BF;
    const int64_t line = f0 + fl_line[i];
    fl_ok[i] = line < lend;
    if (CONTIG) {
      fl_voff[i] = static_cast<uint32_t>(4 * (line * a.K + fl_grp[i] * 8));
    } else {
      // strided: line (b, c) holds X[b][k][c] at b x_bstride + k ncols + c
      const int64_t b = line / a.ncols, c = line - b * a.ncols;
      fl_voff[i] = static_cast<uint32_t>(4 * (b * a.x_bstride + static_cast<int64_t>(fl_grp[i]) * 8 * a.ncols + c));
    }
  }
  const uint32_t kstride = CONTIG ? 4u : static_cast<uint32_t>(4 * a.ncols);   // bytes per unit of k
  // FMODE 1: element q (0 .. 15) of a slice is row (tid / 32) + 16 q, k = k0 + tid % 32
  const int lk = tid & 31, lrow = tid >> 5;
  const uint32_t lk_base = static_cast<uint32_t>(4 * ((f0 + lrow) * a.K + lk));
  const uint32_t lk_qstride = static_cast<uint32_t>(4 * 16 * a.K);

  u32x4 rO[2][TH ? 1 : OP_CH];
  float rF[2][FL_G][8];
  const int nslices = (a.K + BK - 1) / BK;
  const int kend = nslices * BK;        // loads of slices past the last one read nothing

#define PSTD_LOAD_SLICE(R, K0)                                                                        \
  {                                                                                                   \
    const int k0_ = (K0);                                                                             \
    const bool kin_ = k0_ < kend;                                                                     \
    if (!TH) _Pragma("unroll") for (int i = 0; i < OP_CH; ++i)                                        \
      rO[R][i] = ld_b128(rA, kin_ ? op_voff[i] + 2u * k0_ : kOOB);                                    \
    _Pragma("unroll") for (int i = 0; i < FL_G; ++i) {                                                \
      const int kb = k0_ + fl_grp[i] * 8;                                                             \
      if (VEC) {                                                                                      \
        /* each 16-byte half is all valid or all past the row (K % 4 == 0) */                         \
        const bool h0 = fl_ok[i] && kb + 4 <= a.K, h1 = fl_ok[i] && kb + 8 <= a.K;                    \
        const f32x4 v0 = __builtin_bit_cast(f32x4, ld_b128(rX, h0 ? fl_voff[i] + 4u * k0_ : kOOB));   \
        const f32x4 v1 = __builtin_bit_cast(f32x4, ld_b128(rX, h1 ? fl_voff[i] + 16u + 4u * k0_ : kOOB)); \
        _Pragma("unroll") for (int j = 0; j < 4; ++j) {                                               \
          rF[R][i][j] = v0[j];                                                                        \
          rF[R][i][4 + j] = v1[j];                                                                    \
        }                                                                                             \
      } else if (LANEK) {                                                                             \
        _Pragma("unroll") for (int j = 0; j < 8; ++j) {                                               \
          const int q_ = 8 * i + j;                                                                   \
          const bool ok_ = f0 + lrow + 16 * q_ < lend && k0_ + lk < a.K;                              \
          rF[R][i][j] = ld_f32(rX, ok_ ? lk_base + q_ * lk_qstride : kOOB, 4u * k0_);                  \
        }                                                                                             \
      } else {                                                                                        \
        _Pragma("unroll") for (int j = 0; j < 8; ++j)                                                 \
          rF[R][i][j] = ld_f32(rX, (fl_ok[i] && kb + j < a.K) ? fl_voff[i] + j * kstride : kOOB,      \
                               static_cast<uint32_t>(k0_) * kstride);                                 \
      }                                                                                               \
    }                                                                                                 \
  }

#define PSTD_STORE_SLICE(R, BUF, K0)                                                                  \
  {                                                                                                   \
    __bf16* L = lds + (BUF) * BUF_ELEMS;                                                              \
    const int sk0_ = (K0);                                                                            \
    if (!TH) {                                                                                        \
      _Pragma("unroll") for (int i = 0; i < OP_CH; ++i) *reinterpret_cast<u32x4*>(L + op_dst[i]) = rO[R][i]; \
    } else {                                                                                          \
      /* slices past the last (never multiplied) rebuild the last one, which keeps the reads in range */ \
      const int bk0_ = min(sk0_, kend - BK);                                                          \
      /* entry (r, k) = Fr[k - r + 383] + G[r + k], split into hi and lo; row 3g + j, k = k0 + 8q + t */ \
      /* takes Fr[th_fb + k0 + t - j + 2] and G[th_gb + k0 + j + t] */                                \
      float fw_[TH_CH + 7], gw_[TH_CH + 7];                                                           \
      _Pragma("unroll") for (int u = 0; u < TH_CH + 7; ++u) {                                         \
        fw_[u] = sF[th_fb + bk0_ + u];                                                                \
        gw_[u] = sG[th_gb + bk0_ + u];                                                                \
      }                                                                                               \
      _Pragma("unroll") for (int j = 0; j < TH_CH; ++j) {                                             \
        float v_[8];                                                                                  \
        _Pragma("unroll") for (int t = 0; t < 8; ++t) v_[t] = fw_[t - j + TH_CH - 1] + gw_[j + t];    \
        bf16x8 h_, l_;                                                                                \
        split8(v_, h_, l_);                                                                           \
        *reinterpret_cast<bf16x8*>(L + OPH + th_dst[j]) = h_;                                         \
        *reinterpret_cast<bf16x8*>(L + OPL + th_dst[j]) = l_;                                         \
      }                                                                                               \
    }                                                                                                 \
    if (TH && (sk0_ == 0 || sk0_ + BK >= a.K)) {                                                      \
      /* end weights of the input: the first and last element of every line */                        \
      _Pragma("unroll") for (int i = 0; i < FL_G; ++i) _Pragma("unroll") for (int j = 0; j < 8; ++j) { \
        const int ke_ = sk0_ + (LANEK ? lk : fl_grp[i] * 8 + j);                                      \
        rF[R][i][j] *= ke_ == 0 ? a.thw[2] : (ke_ == a.K - 1 ? a.thw[3] : 1.f);                       \
      }                                                                                               \
    }                                                                                                 \
    if (LANEK) {                                                                                      \
      /* lanes 2m and 2m+1 hold k = 2m, 2m+1 of one row: after the swap both hold the pair; the even */ \
      /* lane stores its hi parts, the odd lane its lo parts, each as one dword */                    \
      const bool odd_ = (lk & 1) != 0;                                                                \
      __bf16* dst_ = L + (odd_ ? FLL : FLH) + (lk & ~1);                                              \
      _Pragma("unroll") for (int i = 0; i < FL_G; ++i) _Pragma("unroll") for (int j = 0; j < 8; ++j) { \
        const float x_ = rF[R][i][j];                                                                 \
        const float y_ = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x_), 0xB1, 0xF, 0xF, false)); \
        const float e_ = odd_ ? y_ : x_, o_ = odd_ ? x_ : y_;                                         \
        const __bf16 he_ = static_cast<__bf16>(e_), ho_ = static_cast<__bf16>(o_);                    \
        const __bf16 pe_ = odd_ ? static_cast<__bf16>(e_ - static_cast<float>(he_)) : he_;            \
        const __bf16 po_ = odd_ ? static_cast<__bf16>(o_ - static_cast<float>(ho_)) : ho_;            \
        const uint32_t w_ = static_cast<uint32_t>(__builtin_bit_cast(uint16_t, pe_)) |                \
                            (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, po_)) << 16);         \
        *reinterpret_cast<uint32_t*>(dst_ + (lrow + 16 * (8 * i + j)) * LDK) = w_;                    \
      }                                                                                               \
    } else {                                                                                          \
      _Pragma("unroll") for (int i = 0; i < FL_G; ++i) {                                              \
        bf16x8 h, l;                                                                                  \
        split8(rF[R][i], h, l);                                                                       \
        const int o = fl_line[i] * LDK + fl_grp[i] * 8;                                               \
        *reinterpret_cast<bf16x8*>(L + FLH + o) = h;                                                  \
        *reinterpret_cast<bf16x8*>(L + FLL + o) = l;                                                  \
      }                                                                                               \
    }                                                                                                 \
  }

  f32x16 acc[IP][JQ];
#pragma unroll
  for (int i = 0; i < IP; ++i)
#pragma unroll
    for (int j = 0; j < JQ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int prow = wp * TP + (lane & 31);
  const int qrow = wq * TQ + (lane & 31);

#define PSTD_COMPUTE(BUF)                                                                             \
  {                                                                                                   \
    const __bf16* L = lds + (BUF) * BUF_ELEMS;                                                        \
    _Pragma("unroll") for (int kk = 0; kk < BK; kk += 16) {                                           \
      const int kch = (kk >> 3) + (lane >> 5);   /* 16-byte chunk of this lane's 8 k */                \
      bf16x8 ph[IP], pl[IP], qh[JQ], ql[JQ];                                                          \
      _Pragma("unroll") for (int i = 0; i < IP; ++i) {                                                \
        ph[i] = *reinterpret_cast<const bf16x8*>(L + PH + p_at(prow + 32 * i, kch));                  \
        pl[i] = *reinterpret_cast<const bf16x8*>(L + PL + p_at(prow + 32 * i, kch));                  \
      }                                                                                               \
      _Pragma("unroll") for (int j = 0; j < JQ; ++j) {                                                \
        qh[j] = *reinterpret_cast<const bf16x8*>(L + QH + q_at(qrow + 32 * j, kch));                  \
        ql[j] = *reinterpret_cast<const bf16x8*>(L + QL + q_at(qrow + 32 * j, kch));                  \
      }                                                                                               \
      _Pragma("unroll") for (int i = 0; i < IP; ++i) _Pragma("unroll") for (int j = 0; j < JQ; ++j) { \
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pl[i], qh[j], acc[i][j], 0, 0, 0);        \
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph[i], ql[j], acc[i][j], 0, 0, 0);        \
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph[i], qh[j], acc[i][j], 0, 0, 0);        \
      }                                                                                               \
    }                                                                                                 \
  }

  // slice s lives in LDS buffer s&1 and (before that) in register set s&1.  Prefetches past the last
  // slice use out-of-range offsets (no memory access), which keeps the loop body straight-line so that
  // each wait covers only the loads it needs.
  if (TH) lds_barrier();   // the staged vectors are read by every thread's first slice
  PSTD_LOAD_SLICE(0, 0);
  PSTD_LOAD_SLICE(1, BK);
  PSTD_STORE_SLICE(0, 0, 0);
  PSTD_LOAD_SLICE(0, 2 * BK);
  lds_barrier();
  // Output geometry of the epilogue.  Register r
  // of block (i, j) lies rr(r) = 8 (r / 4) + r % 4 P rows past the block's first row for this lane, so
  // its offset is the lane's block offset plus rr(r) times the (uniform) byte distance of consecutive P
  // rows, which the buffer instructions take as their scalar offset.  An invalid element (past the
  // field's lines or the operator's rows) gets an out-of-range offset: its load returns 0 and its store
  // is dropped.  With beta = 1, rows whose end weight is zero are invalid rows (their update is zero).
  const int lrow4 = 4 * (lane >> 5), lcol = lane & 31;
  const int m_lo = (TH && a.beta == 1.f && a.thw[0] == 0.f) ? 1 : 0;
  const int m_hi = (TH && a.beta == 1.f && a.thw[1] == 0.f) ? a.M - 1 : a.M;
  const uint32_t rstep = static_cast<uint32_t>(4 * (CONTIG ? static_cast<int64_t>(a.M) : a.ncols));
  auto rr = [](int r) { return 8 * (r >> 2) + (r & 3); };
  // block (i, j): this lane's offset of register 0 (kOOB where the lane's column is out) and its valid
  // rr range plo <= rr < phi (phi >= plo); i and j may be runtime values
  auto block_geom = [&](int i, int j, uint32_t& vb, int& plo, int& phi) {
    const int p0 = wp * TP + i * 32 + lrow4;
    const int qc = wq * TQ + j * 32 + lcol;
    bool qok;
    int64_t off;
    if (CONTIG) {               // P = field lines: line f0 + p0 + rr < lend; Q = operator rows m
      plo = 0;
      phi = static_cast<int>(max<int64_t>(min<int64_t>(lend - (f0 + p0), 64), 0));
      const int m = o0 + qc;
      qok = m >= m_lo && m < m_hi;
      off = (f0 + p0) * a.M + m;
    } else {                    // P = operator rows: m_lo <= o0 + p0 + rr < m_hi; Q = field lines
      plo = m_lo - (o0 + p0);
      phi = max(m_hi - (o0 + p0), plo);
      const int64_t line = f0 + qc;
      const int64_t b = line / a.ncols, c = line - b * a.ncols;
      qok = line < lend;
      off = b * a.y_bstride + c + static_cast<int64_t>(o0 + p0) * a.ncols;
    }
    vb = qok ? static_cast<uint32_t>(4 * off) : kOOB;
  };
  // one unsigned compare per element: plo <= rr < phi
  auto sel = [&](uint32_t vb, int plo, int phi, int r, uint32_t oob) -> uint32_t {
    return static_cast<uint32_t>(rr(r) - plo) < static_cast<uint32_t>(phi - plo) ? vb : oob;
  };

  // Only the MFMA work is conditional: the stores and (clamped) loads run in every step, so each load
  // stays where it is issued instead of being moved next to its store behind a branch.
  for (int s = 0; s < nslices; s += 2) {
    // even slice s: LDS buffer 0; slice s+1 waits in register set 1, slice s+2 in set 0
    if (wave_live) PSTD_COMPUTE(0);
    PSTD_STORE_SLICE(1, 1, (s + 1) * BK);
    PSTD_LOAD_SLICE(1, (s + 3) * BK);
    lds_barrier();
    // odd slice s+1 (none past the last): LDS buffer 1; slice s+2 waits in set 0, slice s+3 in set 1
    if (wave_live && s + 1 < nslices) PSTD_COMPUTE(1);
    PSTD_STORE_SLICE(0, 0, (s + 2) * BK);
    PSTD_LOAD_SLICE(0, (s + 4) * BK);
    lds_barrier();
  }
#undef PSTD_COMPUTE
#undef PSTD_LOAD_SLICE
#undef PSTD_STORE_SLICE

  if (!wave_live) return;   // no barrier follows
  // fused update epilogue; lanes 0..31 write 32 consecutive floats of one output line.  Every load of
  // Y is issued before the first store: one memory round trip.
  uint32_t vb[IP][JQ];
  int plo[IP], phi[IP];      // the valid range depends on the block row only
#pragma unroll
  for (int i = 0; i < IP; ++i)
#pragma unroll
    for (int j = 0; j < JQ; ++j) block_geom(i, j, vb[i][j], plo[i], phi[i]);
  auto yoff = [&](int i, int j, int r, uint32_t oob) -> uint32_t { return sel(vb[i][j], plo[i], phi[i], r, oob); };
  if (TH && a.rw_general) {
    // end weights other than 0 and 1 (operators of half-step walls): scale the first and last row
#pragma unroll
    for (int i = 0; i < IP; ++i)
#pragma unroll
      for (int j = 0; j < JQ; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = CONTIG ? o0 + wq * TQ + j * 32 + lcol : o0 + wp * TP + i * 32 + lrow4 + rr(r);
          acc[i][j][r] *= m == 0 ? a.thw[0] : (m == a.M - 1 ? a.thw[1] : 1.f);
        }
  }
  if (a.scale) {
#pragma unroll
    for (int i = 0; i < IP; ++i)
#pragma unroll
      for (int j = 0; j < JQ; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] *= ld_f32(rS, yoff(i, j, r, kOOB), rstep * rr(r));
  }
  // the stores select their out-of-range offset from a kernel argument (the same value), so that the
  // compiler forms each store offset anew instead of keeping 96 load offsets live across the loads
  if (a.beta != 0.f) {
    float yv[IP][JQ][16];
#pragma unroll
    for (int i = 0; i < IP; ++i)
#pragma unroll
      for (int j = 0; j < JQ; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) yv[i][j][r] = ld_f32(rY, yoff(i, j, r, kOOB), rstep * rr(r));
#pragma unroll
    for (int i = 0; i < IP; ++i)
#pragma unroll
      for (int j = 0; j < JQ; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          st_f32(rY, a.beta * yv[i][j][r] + a.alpha * acc[i][j][r], yoff(i, j, r, a.oob), rstep * rr(r));
  } else {
#pragma unroll
    for (int i = 0; i < IP; ++i)
#pragma unroll
      for (int j = 0; j < JQ; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) st_f32(rY, a.alpha * acc[i][j][r], yoff(i, j, r, a.oob), rstep * rr(r));
  }
}

// compute units of the current device (one block of this kernel per CU), looked up once per device
int64_t cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] <= 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    cached[dev] = n;
  }
  return cached[dev];
}

template <bool CONTIG>
hipError_t launch_s(const ContractArgs& c, hipStream_t s) {
  static_assert(kColPad % BK == 0, "operator columns must be padded to whole K slices");
  // operators formed on the chip: all rows in one tile, vectors within the staged length
  const bool th = c.th && c.M <= kThRowsMax && c.K <= kThColsMax && c.th_len >= kThRowsMax + c.K + 8 &&
                  c.th_len <= kThLen;
  const int BO = th ? tile_ops<true>() : tile_ops<false>();
  const int BF = th ? tile_lines<true>() : tile_lines<false>();
  SArgs a;
  a.th = c.th;
  a.th_len = c.th_len;
  for (int i = 0; i < 4; ++i) a.thw[i] = c.thw[i];
  // with beta = 1 a row of weight zero is left as it is (its update is zero); otherwise it is scaled
  a.rw_general = c.beta == 1.f ? !((c.thw[0] == 0.f || c.thw[0] == 1.f) && (c.thw[1] == 0.f || c.thw[1] == 1.f))
                               : (c.thw[0] != 1.f || c.thw[1] != 1.f);
  a.oob = kOOB;
  a.Ahi = static_cast<const uint16_t*>(c.A);
  a.lda = c.lda;
  a.M = c.M;
  a.K = c.K;
  a.mrows = static_cast<int>(round_up(c.M, kRowPad));   // the allocation of upload_operator
  a.X = static_cast<const float*>(c.X);
  a.Y = static_cast<float*>(c.Y);
  a.ncols = c.ncols;
  a.x_bstride = c.x_bstride;
  a.y_bstride = c.y_bstride;
  a.lines = CONTIG ? c.ncols : c.ncols * c.batch;
  a.alpha = c.alpha;
  a.beta = c.beta;
  a.scale = static_cast<const float*>(c.scale);
  a.op_tiles = (c.M + BO - 1) / BO;
  a.fld_tiles = (a.lines + BF - 1) / BF;
  a.narrow_tiles = 0;
  // a last round at most half full: its field tiles become twice as many half-width tiles
  const int64_t cus = cu_count();
  const int64_t rem = (a.fld_tiles * a.op_tiles) % cus;
  if (rem != 0) {
    const int64_t conv = (rem + a.op_tiles - 1) / a.op_tiles;          // field tiles to split
    if (conv <= a.fld_tiles && 2 * conv * a.op_tiles <= cus) {
      a.fld_tiles -= conv;
      a.narrow_tiles = (a.lines - a.fld_tiles * BF + BF / 2 - 1) / (BF / 2);
    }
  }
  const int64_t blocks = (a.fld_tiles + a.narrow_tiles) * a.op_tiles;
  if (blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  // buffer offsets are 32-bit: the whole input and output must stay below 2 GiB (checked at plan creation)
  const int64_t xb = 4 * (CONTIG ? a.lines * c.K : c.batch * c.x_bstride);
  const int64_t yb = 4 * (CONTIG ? a.lines * c.M : c.batch * c.y_bstride);
  const int64_t ob = reinterpret_cast<const char*>(c.A_lo) - reinterpret_cast<const char*>(c.A);
  if (xb >= (int64_t(1) << 31) || yb >= (int64_t(1) << 31) || ob <= 0 || 2 * ob >= (int64_t(1) << 31))
    return hipErrorInvalidValue;
  if (!CONTIG && (c.x_bstride != static_cast<int64_t>(c.K) * c.ncols || c.y_bstride != static_cast<int64_t>(c.M) * c.ncols))
    return hipErrorInvalidValue;
  a.lo_off = static_cast<uint32_t>(ob);
  const dim3 grid(static_cast<unsigned>(blocks));
  // contiguous rows that start 16-byte aligned take two 16-byte loads per 8 floats
  const bool vec = CONTIG && c.K % 4 == 0 && (reinterpret_cast<uintptr_t>(c.X) & 15) == 0;
  if (th) {
    if (vec)
      hipLaunchKernelGGL((split_kernel<CONTIG, 2, true>), grid, dim3(NT), 0, s, a);
    else if (CONTIG)
      hipLaunchKernelGGL((split_kernel<CONTIG, 1, true>), grid, dim3(NT), 0, s, a);
    else
      hipLaunchKernelGGL((split_kernel<CONTIG, 0, true>), grid, dim3(NT), 0, s, a);
  } else if (vec) {
    hipLaunchKernelGGL((split_kernel<CONTIG, 2, false>), grid, dim3(NT), 0, s, a);
  } else if (CONTIG) {   // other contiguous rows: lanes along k
    hipLaunchKernelGGL((split_kernel<CONTIG, 1, false>), grid, dim3(NT), 0, s, a);
  } else {
    hipLaunchKernelGGL((split_kernel<CONTIG, 0, false>), grid, dim3(NT), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_contract_split(const ContractArgs& c, bool contiguous, hipStream_t s) {
  return contiguous ? launch_s<true>(c, s) : launch_s<false>(c, s);
}

}  // namespace pstd
