// Kernels of the DCT-basis neural-operator surrogate: one strided batched GEMM on the bf16 matrix
// cores (FP32 accumulation) with fused epilogues, and the small elementwise/reduction kernels around it.
//
// Every contraction of the network (the truncated DCT along each axis, the per-mode channel mixing, the
// inverse DCT, the pointwise channel mixing, the lift and projection, and all their backward products)
// is  C[z] = alpha A[z] B[z] (+ beta C[z]) (+ bias[m]) (+ D[z]) (-> GELU)  with arbitrary element
// strides, so one kernel serves all of them without transposes in HBM.  Operands are FP32 in HBM and
// rounded to bf16 while they are staged into LDS; with `split` each operand is also kept as a bf16
// remainder and the product is formed as hi*hi + hi*lo + lo*hi (close to FP32 accuracy; used by the
// parity tests).
//
// MFMA v_mfma_f32_32x32x16_bf16: lane l supplies A[l%32][8*(l/32) .. +7] and B^T[l%32][8*(l/32) .. +7]
// (both staged as [row][k] in LDS) and receives C[8*(r/4) + 4*(l/32) + r%4][l%32] in register r.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.h"

namespace pstd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t kOOB = 0x80000000u;   // buffer offset past every range: the load returns zero

// A buffer descriptor that is the same for the whole wave, built from base and size passed through
// readfirstlane so it lives in scalar registers (no per-lane loop over descriptors around each access).
__device__ __forceinline__ rsrc_t wave_rsrc(const void* p, uint32_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a >> 32));
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>((static_cast<uint64_t>(hi) << 32) | lo), 0,
                                           static_cast<int>(__builtin_amdgcn_readfirstlane(bytes)), 0x00020000);
}

// One activation element through a buffer descriptor: a float, or a bf16 widened to float; an offset
// of kOOB reads zero, so no load needs a branch around it.
template <typename T>
__device__ __forceinline__ float ld_elem(rsrc_t r, uint32_t byte_off) {
  if (sizeof(T) == 4) return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
  return static_cast<float>(__builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(r, byte_off, 0, 0)));
}

constexpr int BK = 32;
constexpr int LDK = BK + 8;     // LDS row stride in bf16 (80 bytes: conflict-free 16-byte reads)
constexpr int NT = 256;         // 4 waves

// GELU x Phi(x) with the normal CDF from Hastings' rational approximation of erfc (Abramowitz & Stegun
// 7.1.26, |error| <= 1.5e-7): branch-free, a reciprocal, five FMAs and one exponential.  Phi(x) =
// erfc(-x/sqrt2)/2, with erfc(z) = t P(t) exp(-z^2), t = 1/(1 + p z) for z >= 0.  Worst absolute error of
// the GELU value in FP32 over [-10, 10]: 4.2e-7.  The backward pass keeps the exact derivative.
__device__ __forceinline__ float gelu_f(float x) {
  const float z = fabsf(x) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, z, 1.0f));
  float poly = fmaf(1.061405429f, t, -1.453152027f);
  poly = fmaf(poly, t, 1.421413741f);
  poly = fmaf(poly, t, -0.284496736f);
  poly = fmaf(poly, t, 0.254829592f);
  const float y = t * poly * __expf(-z * z);     // erfc(z)
  return x * (x >= 0.f ? fmaf(-0.5f, y, 1.0f) : 0.5f * y);
}
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// Element e (0 .. ROWS*BK-1) of an operand tile: row r (m for A, n for B) and column k.  Lanes run along
// k when the operand is contiguous in k, along the rows otherwise, so the loads coalesce either way.
template <int ROWS>
__device__ __forceinline__ void tile_pos(int e, bool kcontig, int& r, int& k) {
  if (kcontig) {
    k = e & (BK - 1);
    r = e >> 5;
  } else {
    r = e % ROWS;
    k = e / ROWS;
  }
}

// Tile of WMW x WNW waves, each computing FM x FN blocks of 32 x 32 outputs:
// BM = 32 WMW FM rows, BN = 32 WNW FN columns.
template <int WMW, int WNW, int FM, int FN>
__global__ __launch_bounds__(NT) void nop_gemm_kernel(NopGemm g) {
  constexpr int BM = 32 * WMW * FM, BN = 32 * WNW * FN;
  constexpr int PA = BM * BK / NT, PB = BN * BK / NT;   // operand elements staged per thread
  __shared__ __attribute__((aligned(16))) __bf16 lds[2 * (BM + BN) * LDK];   // A hi, A lo, B hi, B lo
  __bf16* Ah = lds;
  __bf16* Al = lds + BM * LDK;
  __bf16* Bh = lds + 2 * BM * LDK;
  __bf16* Bl = Bh + BN * LDK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WMW, wn = wave / WMW;
  const int tiles_m = (g.M + BM - 1) / BM;
  const int m0 = (blockIdx.x % tiles_m) * BM, n0 = (blockIdx.x / tiles_m) * BN;
  const int z = blockIdx.y;
  const int z1 = z / g.nb2, z2 = z - z1 * g.nb2;
  const float* A = g.A + z1 * g.bA1 + z2 * g.bA2;
  const float* B = g.B + z1 * g.bB1 + z2 * g.bB2;
  const bool akc = g.sAk == 1, bkc = g.sBk == 1;
  const bool split = g.split != 0;
  // element offsets within one batch entry fit in 32 bits (the host checks every operand's extent)
  const uint32_t sAm = static_cast<uint32_t>(g.sAm), sAk = static_cast<uint32_t>(g.sAk);
  const uint32_t sBk = static_cast<uint32_t>(g.sBk), sBn = static_cast<uint32_t>(g.sBn);

  float ra[PA], rb[PB];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      int r, k;
      tile_pos<BM>(tid + i * NT, akc, r, k);
      const int m = m0 + r, kk = k0 + k;
      ra[i] = (m < g.M && kk < g.K) ? A[static_cast<uint32_t>(m) * sAm + static_cast<uint32_t>(kk) * sAk] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      int r, k;
      tile_pos<BN>(tid + i * NT, bkc, r, k);
      const int n = n0 + r, kb = k0 + k;
      rb[i] = (n < g.N && kb < g.K) ? B[static_cast<uint32_t>(kb) * sBk + static_cast<uint32_t>(n) * sBn] : 0.f;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < PA; ++i) {
      int r, k;
      tile_pos<BM>(tid + i * NT, akc, r, k);
      const __bf16 h = static_cast<__bf16>(ra[i]);
      Ah[r * LDK + k] = h;
      if (split) Al[r * LDK + k] = static_cast<__bf16>(ra[i] - static_cast<float>(h));
    }
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      int r, k;
      tile_pos<BN>(tid + i * NT, bkc, r, k);
      const __bf16 h = static_cast<__bf16>(rb[i]);
      Bh[r * LDK + k] = h;
      if (split) Bl[r * LDK + k] = static_cast<__bf16>(rb[i] - static_cast<float>(h));
    }
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  const int nsl = (g.K + BK - 1) / BK;
  load(0);
  store();
  lds_barrier();
  const int koff = 8 * (lane >> 5);
  for (int s = 0; s < nsl; ++s) {
    if (s + 1 < nsl) load((s + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      bf16x8 ah[FM], bh[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        ah[i] = *reinterpret_cast<const bf16x8*>(&Ah[((wm * FM + i) * 32 + (lane & 31)) * LDK + kk + koff]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bh[j] = *reinterpret_cast<const bf16x8*>(&Bh[((wn * FN + j) * 32 + (lane & 31)) * LDK + kk + koff]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      if (split) {
        bf16x8 al[FM], bl[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
          al[i] = *reinterpret_cast<const bf16x8*>(&Al[((wm * FM + i) * 32 + (lane & 31)) * LDK + kk + koff]);
#pragma unroll
        for (int j = 0; j < FN; ++j)
          bl[j] = *reinterpret_cast<const bf16x8*>(&Bl[((wn * FN + j) * 32 + (lane & 31)) * LDK + kk + koff]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          }
      }
    }
    lds_barrier();
    if (s + 1 < nsl) {
      store();
      lds_barrier();
    }
  }

  // epilogue
  float* C = g.C + z1 * g.bC1 + z2 * g.bC2;
  const float* Dp = g.add ? g.add + z1 * g.bD1 + z2 * g.bD2 : nullptr;
  float* Pp = g.pre ? g.pre + z1 * g.bC1 + z2 * g.bC2 : nullptr;
  const float* Gp = g.dgelu ? g.dgelu + z1 * g.bC1 + z2 * g.bC2 : nullptr;
  const uint32_t sCm = static_cast<uint32_t>(g.sCm), sCn = static_cast<uint32_t>(g.sCn);
  const uint32_t sDm = static_cast<uint32_t>(g.sDm), sDn = static_cast<uint32_t>(g.sDn);
  // All reads of a 32 x 32 block (old C, the added tensor, the GELU argument, the bias) are issued before
  // its first store: the stores may alias nothing the loads touch, but the compiler cannot know that,
  // and interleaving would serialise every element on a memory round trip.
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + (wn * FN + j) * 32 + (lane & 31);
      float ext[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + (wm * FM + i) * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const bool ok = m < g.M && n < g.N;
        const uint32_t co = static_cast<uint32_t>(m) * sCm + static_cast<uint32_t>(n) * sCn;
        float e = 0.f;
        if (ok) {
          if (g.beta != 0.f) e += g.beta * C[co];
          if (g.bias_m) e += g.bias_m[m];
          if (Dp) e += Dp[static_cast<uint32_t>(m) * sDm + static_cast<uint32_t>(n) * sDn];
        }
        ext[r] = e;
      }
      float gg[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + (wm * FM + i) * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const uint32_t co = static_cast<uint32_t>(m) * sCm + static_cast<uint32_t>(n) * sCn;
        gg[r] = (Gp && m < g.M && n < g.N) ? Gp[co] : 0.f;
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + (wm * FM + i) * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (m < g.M && n < g.N) {
          const uint32_t co = static_cast<uint32_t>(m) * sCm + static_cast<uint32_t>(n) * sCn;
          float v = g.alpha * acc[i][j][r] + ext[r];
          if (Gp) v *= gelu_grad_f(gg[r]);
          if (g.act) {
            if (Pp) Pp[co] = v;
            v = gelu_f(v);
          }
          C[co] = v;
        }
      }
    }
}

// Natural spectral layout [b][c][kh][kw] <-> block layout [blk][q][b][c] (blk = (kh/2)(Mm/2) + kw/2,
// q = 2 (kh%2) + kw%2): the modes that share one mixing matrix become one contiguous GEMM operand.
// One block moves the C x 64 slab of modes m0 .. m0+63 (m = kh Mm + kw) of one sample through LDS: the
// natural side is read or written as 64 consecutive modes per channel, the block side as C consecutive
// channels per mode.  C <= 32.
__global__ __launch_bounds__(256) void nop_mode_transpose_kernel(const float* __restrict__ in, float* __restrict__ out,
                                                                 int B, int C, int Mm, int to_block) {
  __shared__ float tile[32][65];
  const int M2 = Mm * Mm;
  const int m0 = blockIdx.x * 64;
  const int64_t b = blockIdx.y;
  const int t = threadIdx.x;
  // natural side: lane -> mode, wave -> channel
  const int nm = m0 + (t & 63);
  // block side: lane -> channel, half-wave -> mode
  const int bc = t & 31;
  int64_t boff[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int m = m0 + (t >> 5) + 8 * u;
    const int kh = m / Mm, kw = m - kh * Mm;
    const int blk = (kh >> 1) * (Mm >> 1) + (kw >> 1), q = 2 * (kh & 1) + (kw & 1);
    boff[u] = m < M2 ? ((static_cast<int64_t>(blk) * 4 + q) * B + b) * C + bc : -1;
  }
  if (to_block) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = (t >> 6) + 4 * u;
      if (c < C && nm < M2) tile[c][t & 63] = in[(b * C + c) * M2 + nm];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (bc < C && boff[u] >= 0) out[boff[u]] = tile[bc][(t >> 5) + 8 * u];
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (bc < C && boff[u] >= 0) tile[bc][(t >> 5) + 8 * u] = in[boff[u]];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = (t >> 6) + 4 * u;
      if (c < C && nm < M2) out[(b * C + c) * M2 + nm] = tile[c][t & 63];
    }
  }
}

// Input features [b][4][H][W]: p0, (c0 - 1500)/100, x = i/(H-1), y = j/(W-1).
__global__ void nop_features_kernel(const float* p0, const float* c0, float* f, int B, int H, int W) {
  const int64_t P = static_cast<int64_t>(H) * W;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B * P) return;
  const int64_t b = i / P, p = i - b * P;
  const int h = static_cast<int>(p / W), w = static_cast<int>(p % W);
  float* fb = f + b * 4 * P;
  fb[p] = p0[i];
  fb[P + p] = (c0[i] - 1500.0f) / 100.0f;
  fb[2 * P + p] = H > 1 ? static_cast<float>(h) / static_cast<float>(H - 1) : 0.f;
  fb[3 * P + p] = W > 1 ? static_cast<float>(w) / static_cast<float>(W - 1) : 0.f;
}

// d = g * GELU'(pre), elementwise.
__global__ void nop_gelu_bwd_kernel(const float* gin, const float* pre, float* d, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) d[i] = gin[i] * gelu_grad_f(pre[i]);
}

// out[j] = sum over blocks b < nb and positions p < P of x[(b rows + j) P + p]: one block per j.
// Layout of x: [nb][rows][P]; sums in double, written as float (deterministic).
__global__ void nop_rowsum_kernel(const float* x, float* out, int nb, int rows, int64_t P) {
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) {
    const float* r = x + (static_cast<int64_t>(b) * rows + j) * P;
    for (int64_t p = threadIdx.x; p < P; p += blockDim.x) s += r[p];
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = static_cast<float>(red[0]);
}

// out[j] = sum_z part[z n + j], j < n (the split-K partial products).
__global__ void nop_partial_sum_kernel(const float* part, float* out, int nz, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int zz = 0; zz < nz; ++zz) s += part[static_cast<int64_t>(zz) * n + j];
  out[j] = static_cast<float>(s);
}

// Per sample b: num_b = |out - t|^2, den_b = |t|^2 (one block per sample, double sums).
__global__ void nop_loss_terms_kernel(const float* out, const float* tgt, double* terms, int64_t P) {
  const int b = blockIdx.x;
  const float* o = out + b * P;
  const float* t = tgt + b * P;
  double sn = 0.0, sd = 0.0;
  for (int64_t p = threadIdx.x; p < P; p += blockDim.x) {
    const double d = static_cast<double>(o[p]) - t[p];
    sn += d * d;
    sd += static_cast<double>(t[p]) * t[p];
  }
  __shared__ double rn[256], rd[256];
  rn[threadIdx.x] = sn;
  rd[threadIdx.x] = sd;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) {
      rn[threadIdx.x] += rn[threadIdx.x + w];
      rd[threadIdx.x] += rd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    terms[2 * b] = rn[0];
    terms[2 * b + 1] = rd[0];
  }
}

// dout = 2 (out - t) / (den_b B).
__global__ void nop_loss_grad_kernel(const float* out, const float* tgt, const double* terms, float* dout, int B,
                                     int64_t P) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B * P) return;
  const int64_t b = i / P;
  dout[i] = static_cast<float>(2.0 * (static_cast<double>(out[i]) - tgt[i]) / (terms[2 * b + 1] * B));
}

// Adam (Kingma & Ba, Algorithm 1) with bias correction; c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void nop_adam_kernel(float* th, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                                float eps, float c1, float c2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Per-sample input statistics for the surrogate's gate: c0 min, c0 max, max |p0|, and the share of
// sum p0^2 within `margin` nodes of a wall.  One block per sample; double sums.
__global__ void nop_input_stats_kernel(const float* p0, const float* c0, double* stats, int H, int W, int margin) {
  const int b = blockIdx.x;
  const int64_t P = static_cast<int64_t>(H) * W;
  const float* p = p0 + b * P;
  const float* c = c0 + b * P;
  double cmin = 1e300, cmax = -1e300, pmax = 0.0, e_all = 0.0, e_wall = 0.0;
  for (int64_t i = threadIdx.x; i < P; i += blockDim.x) {
    const int h = static_cast<int>(i / W), w = static_cast<int>(i % W);
    const double cv = c[i], pv = p[i];
    cmin = fmin(cmin, cv);
    cmax = fmax(cmax, cv);
    pmax = fmax(pmax, fabs(pv));
    e_all += pv * pv;
    if (h < margin || h >= H - margin || w < margin || w >= W - margin) e_wall += pv * pv;
  }
  __shared__ double r[5][256];
  r[0][threadIdx.x] = cmin;
  r[1][threadIdx.x] = cmax;
  r[2][threadIdx.x] = pmax;
  r[3][threadIdx.x] = e_all;
  r[4][threadIdx.x] = e_wall;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) {
      r[0][threadIdx.x] = fmin(r[0][threadIdx.x], r[0][threadIdx.x + w]);
      r[1][threadIdx.x] = fmax(r[1][threadIdx.x], r[1][threadIdx.x + w]);
      r[2][threadIdx.x] = fmax(r[2][threadIdx.x], r[2][threadIdx.x + w]);
      r[3][threadIdx.x] += r[3][threadIdx.x + w];
      r[4][threadIdx.x] += r[4][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[4 * b] = r[0][0];
    stats[4 * b + 1] = r[1][0];
    stats[4 * b + 2] = r[2][0];
    stats[4 * b + 3] = r[3][0] > 0 ? r[4][0] / r[3][0] : 0.0;
  }
}

// Eight consecutive k of one operand row as bf16, and (split) the bf16 remainder.
__device__ __forceinline__ void to_bf16x8(const float (&x)[8], bf16x8& hi, bf16x8& lo, bool split) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = static_cast<__bf16>(x[e]);
    hi[e] = h;
    lo[e] = split ? static_cast<__bf16>(x[e] - static_cast<float>(h)) : static_cast<__bf16>(0.f);
  }
}

// acc += P . Q over one K-step of 16 on the bf16 matrix cores; with split as hi*hi + hi*lo + lo*hi.
__device__ __forceinline__ void mma_bf16(const float (&p)[8], const float (&q)[8], f32x16& acc, bool split) {
  bf16x8 ph, pl, qh, ql;
  to_bf16x8(p, ph, pl, split);
  to_bf16x8(q, qh, ql, split);
  if (split) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pl, qh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph, ql, acc, 0, 0, 0);
  }
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ph, qh, acc, 0, 0, 0);
}

// dst[r * ldd + k] = element (r, k) of an R x K matrix, read row-major (src[r * K + k]) or, with trans,
// from its K x R transpose (src[k * R + r]); 256 threads, eight loads per thread in flight before their
// LDS stores.  The row/column split uses a float reciprocal: (i + 1/2) / cols is at least 1/(2 cols)
// away from an integer and its relative error is below 2^-23, exact for R K < 2^22.
template <typename TS>
__device__ __forceinline__ void stage_matrix(float* dst, int ldd, const TS* __restrict__ src, int R, int K,
                                             bool trans) {
  const int n = R * K;
  const int cols = trans ? R : K;
  const float inv = 1.0f / static_cast<float>(cols);
  const rsrc_t rs = wave_rsrc(src, static_cast<uint32_t>(n * sizeof(TS)));
  // indices past the end are clamped to the last element, whose value they store again: no branch, so
  // the loads stay ahead of the stores
  for (int base = 0; base < n; base += 8 * 256) {
    float v[8];
    int idx[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      idx[u] = min(base + static_cast<int>(threadIdx.x) + 256 * u, n - 1);
      v[u] = ld_elem<TS>(rs, static_cast<uint32_t>(idx[u] * sizeof(TS)));
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = idx[u];
      const int q = static_cast<int>((static_cast<float>(i) + 0.5f) * inv);
      const int rem = i - q * cols;
      dst[(trans ? rem : q) * ldd + (trans ? q : rem)] = v[u];
    }
  }
}

// Pointwise channel mixing on the bf16 matrix cores (FP32 accumulation): Y[b][o][p] = sum_i A[o][i]
// X[b][i][p] (+ bias[o]) (+ D[b][o][p]) (+ sum_k T[b][h][o][k] Cw[k][w] at p = (h, w)), then optionally
// pre = value and Y = GELU(value), for O <= 32 output channels.  A block covers up to 128 consecutive
// positions of one grid row, a wave 32 of them; each wave computes all O outputs of its positions with
// v_mfma_f32_32x32x16_bf16: lane l supplies A[l%32][k0 + 8(l/32) .. +7] and X[k0 + 8(l/32) .. +7][l%32]
// and receives Y[8(r/4) + 4(l/32) + r%4][l%32] in register r.  X is read straight from HBM, coalesced
// along the positions; A (O x I row-major, or I x O with tA), the bias and the block's row of T
// ([b][h][o][Mm]) are staged in LDS by coalesced loads, since a lane-per-row read of them would touch one
// cache line per lane.  With T the second term is the last stage of the inverse DCT, T being the first
// stage (along H) for the row: its K extent (the retained modes along W) continues the same
// accumulation.  split: every product as hi*hi + hi*lo + lo*hi (near FP32).
// TX, TY, TT: storage types of X, Y and T (float, or __bf16 for inference activations, which every
// consumer rounds to bf16 before its product anyway).
template <typename TX, typename TY, typename TT>
__global__ __launch_bounds__(256) void nop_mix_kernel(const float* __restrict__ A, const TX* __restrict__ X,
                                                      TY* __restrict__ Y, const float* __restrict__ bias,
                                                      const float* __restrict__ D, float* __restrict__ pre,
                                                      const TT* __restrict__ T, const float* __restrict__ Cw, int O,
                                                      int I, int H, int W, int Mm, int act, int tA, int split) {
  extern __shared__ float sm[];
  const int lda = I + 1, ldt = Mm + 1;
  float* sA = sm;                          // [32][I + 1]: A as [o][k]
  float* sT = sA + 32 * lda;               // [32][Mm + 1]: T row as [o][k]
  float* sb = sT + (T ? 32 * ldt : 0);     // [32]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t b = blockIdx.y;
  const int64_t P = static_cast<int64_t>(H) * W;
  const int groups = (W + 127) >> 7;       // 128-position groups per row
  const int h = blockIdx.x / groups;
  const int w = (blockIdx.x - h * groups) * 128 + wave * 32 + (lane & 31);
  const int kh = 8 * (lane >> 5), o = lane & 31;
  const bool nok = w < W;
  const int64_t n = nok ? static_cast<int64_t>(h) * W + w : 0;
  constexpr uint32_t XS = sizeof(TX);
  const rsrc_t rX = wave_rsrc(X + b * I * P, static_cast<uint32_t>(I * P) * XS);
  const rsrc_t rC = wave_rsrc(Cw, T ? static_cast<uint32_t>(Mm * W * 4) : 0u);
  auto xoff = [&](int k) { return (nok && k < I) ? XS * static_cast<uint32_t>(k * P + n) : kOOB; };
  // the first 32 k of X in flight while the block stages its operands
  float xv[2][8];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int e = 0; e < 8; ++e) xv[c][e] = ld_elem<TX>(rX, xoff(16 * c + kh + e));
  stage_matrix(sA, lda, A, O, I, tA != 0);
  if (T) stage_matrix(sT, ldt, T + (b * H + h) * static_cast<int64_t>(O) * Mm, O, Mm, false);
  if (tid < 32) sb[tid] = (bias && tid < O) ? bias[tid] : 0.f;
  __syncthreads();
  const bool sp = split != 0;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  // the first two K-steps from the prefetched registers, the rest loaded in the loop (k0 wave-uniform)
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (16 * c >= I) break;
    float af[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 16 * c + kh + e;
      af[e] = (o < O && k < I) ? sA[o * lda + k] : 0.f;
    }
    mma_bf16(af, xv[c], acc, sp);
  }
  for (int k0 = 32; k0 < I; k0 += 16) {
    float xf[8], af[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + kh + e;
      xf[e] = ld_elem<TX>(rX, xoff(k));
      af[e] = (o < O && k < I) ? sA[o * lda + k] : 0.f;
    }
    mma_bf16(af, xf, acc, sp);
  }
  if (T) {
    for (int k0 = 0; k0 < Mm; k0 += 16) {
      float cf[8], tf[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + kh + e;
        cf[e] = ld_elem<float>(rC, (nok && k < Mm) ? 4u * static_cast<uint32_t>(k * W + w) : kOOB);
        tf[e] = (o < O && k < Mm) ? sT[o * ldt + k] : 0.f;
      }
      mma_bf16(tf, cf, acc, sp);
    }
  }
  float e[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int oo = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    e[r] = (oo < O && nok) ? ((D ? D[(b * O + oo) * P + n] : 0.f) + sb[oo]) : 0.f;
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int oo = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (oo < O && nok) {
      const int64_t off = (b * O + oo) * P + n;
      float v = acc[r] + e[r];
      if (act) {
        if (pre) pre[off] = v;
        v = gelu_f(v);
      }
      Y[off] = static_cast<TY>(v);
    }
  }
}

// Register-resident form of the same product for O <= 32, I <= 32 and at most KT K-steps of modes (no D
// term): each block walks `rpb` consecutive rows r = b H + h of up to 128 positions.  A, the bias and the
// Cw columns of the block's positions are loaded once and kept in registers; bf16 T rows arrive as
// 16-byte vectors when TVEC (Mm % 8 == 0).  Three register sets form a ring: the X and T operands of
// rows r + 1 and r + 2 are in flight while row r is multiplied and stored.
// The MFMA sequence (X K-steps, then T K-steps, each hi/lo-split when split) is the one of
// nop_mix_kernel, so both forms give the same bits.
typedef unsigned u32x4r __attribute__((ext_vector_type(4)));
template <typename TX, typename TY, typename TT, int KT, bool TVEC, bool SPLIT, bool KFULL>
__global__ __launch_bounds__(256) void nop_mixrows_kernel(const float* __restrict__ A, const TX* __restrict__ X,
                                                          TY* __restrict__ Y, const float* __restrict__ bias,
                                                          float* __restrict__ pre, const TT* __restrict__ T,
                                                          const float* __restrict__ Cw, int O, int I, int H, int W,
                                                          int Mm, int B, int rpb, int act, int tA) {
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int groups = (W + 127) >> 7;
  const int blk = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x));
  const int g = blk % groups;
  const int rows = B * H;
  const int r0 = (blk / groups) * rpb, r1 = min(r0 + rpb, rows);
  const int w = g * 128 + wave * 32 + (lane & 31);
  const int kh = 8 * (lane >> 5), o = lane & 31;
  const bool nok = w < W;
  const int P = H * W;
  constexpr bool sp = SPLIT;
  constexpr uint32_t XS = sizeof(TX), YS = sizeof(TY), TS = sizeof(TT);
  const rsrc_t rX = wave_rsrc(X, static_cast<uint32_t>(B * I * P) * XS);
  const rsrc_t rY = wave_rsrc(Y, static_cast<uint32_t>(B * O * P) * YS);
  const rsrc_t rPre = wave_rsrc(pre ? static_cast<void*>(pre) : static_cast<void*>(Y), pre ? static_cast<uint32_t>(B * O * P) * 4u : 0u);
  const rsrc_t rT = wave_rsrc(T ? static_cast<const void*>(T) : static_cast<const void*>(X),
                              T ? static_cast<uint32_t>(rows * O * Mm) * TS : 0u);

  // operands that stay for all rows: A (P port of the X steps), Cw (Q port of the T steps), bias; all
  // their loads are issued together (out-of-range lanes read zero through the descriptors)
  const rsrc_t rA = wave_rsrc(A, static_cast<uint32_t>(O * I) * 4u);
  const rsrc_t rC = wave_rsrc(Cw, T ? static_cast<uint32_t>(Mm * W) * 4u : 0u);
  float af[2][8];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 16 * c + kh + e;
      const uint32_t off = (4u * static_cast<uint32_t>(tA ? k * O + o : o * I + k)) | ((o < O && k < I) ? 0u : kOOB);
      af[c][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rA, off, 0, 0));
    }
  float cf[KT > 0 ? KT : 1][8];
#pragma unroll
  for (int t = 0; t < KT; ++t)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int m = 16 * t + kh + e;
      const uint32_t off = (4u * static_cast<uint32_t>(m * W + w)) | ((nok && m < Mm) ? 0u : kOOB);
      cf[t][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rC, off, 0, 0));
    }
  bf16x8 ah[2], al[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) to_bf16x8(af[c], ah[c], al[c], sp);
  bf16x8 ch[KT > 0 ? KT : 1], cl[KT > 0 ? KT : 1];
#pragma unroll
  for (int t = 0; t < KT; ++t) to_bf16x8(cf[t], ch[t], cl[t], sp);
  __shared__ __attribute__((aligned(16))) float sb[32];
  if (tid < 32) sb[tid] = (bias && tid < O) ? bias[tid] : 0.f;
  __syncthreads();
  const int nxs = I > 16 ? 2 : 1;                         // X K-steps
  const int nts = T ? (Mm + 15) / 16 : 0;                 // T K-steps (<= KT)

  // three register sets of row operands.  Offsets are split into a per-lane part, which an out-of-range
  // lane ORs with kOOB (a select between constants: no branch around the load), and a row-uniform part
  // passed as the scalar offset.
  // bf16 X elements go straight into packed bf16 operands (16-bit loads into register halves)
  constexpr bool XH = sizeof(TX) == 2;
  float xr[3][2][XH ? 1 : 8];
  bf16x8 xb[3][2];
  u32x4r tr[3][KT > 0 ? KT : 1];
  float te[3][KT > 0 ? KT : 1][TVEC ? 1 : 8];
  static_assert(!TVEC || TS == 2, "16-byte T rows are read for bf16 storage only");
  const uint32_t xlane = XS * static_cast<uint32_t>(kh * P + w);
  const uint32_t xlane_ok = xlane | (nok ? 0u : kOOB);
  const uint32_t tlane = TS * static_cast<uint32_t>(o * Mm + kh);
  auto load_row = [&](int set, int r) {
    const int b = r / H, h = r - b * H;
    const uint32_t xrow = XS * static_cast<uint32_t>(b * I * P + h * W);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 16 * c + kh + e;
        // with all 32 inputs present the per-lane offset is one register and the channel goes into the
        // scalar offset; otherwise each element carries its own range mask
        const uint32_t kst = XS * static_cast<uint32_t>((16 * c + e) * P);
        const uint32_t off = KFULL ? xlane_ok : (xlane + kst) | ((nok && k < I) ? 0u : kOOB);
        const uint32_t so = KFULL ? xrow + kst : xrow;
        if (XH)
          xb[set][c][e] = __builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(rX, off, so, 0));
        else
          xr[set][c][XH ? 0 : e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rX, off, so, 0));
      }
    const uint32_t trow = TS * static_cast<uint32_t>(r * O * Mm);
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const int m0 = 16 * t + kh;
      if (TVEC) {
        const uint32_t off = (tlane + TS * 16u * t) | ((o < O && m0 < Mm) ? 0u : kOOB);
        tr[set][t] = __builtin_bit_cast(u32x4r, __builtin_amdgcn_raw_buffer_load_b128(rT, off, trow, 0));
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t off = (tlane + TS * static_cast<uint32_t>(16 * t + e)) | ((o < O && m0 + e < Mm) ? 0u : kOOB);
          if (TS == 4)
            te[set][t][TVEC ? 0 : e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rT, off, trow, 0));
          else
            te[set][t][TVEC ? 0 : e] = static_cast<float>(
                __builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(rT, off, trow, 0)));
        }
      }
    }
  };
  auto row = [&](int set, int r, bool valid) {
    const int b = r / H, h = r - b * H;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (c >= nxs) break;
      bf16x8 xh, xl;
      if (XH) {   // bf16 storage: hi is the stored value, lo is zero
        xh = xb[set][c];
#pragma unroll
        for (int e = 0; e < 8; ++e) xl[e] = static_cast<__bf16>(0.f);
      } else {
        float xf[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) xf[e] = xr[set][c][XH ? 0 : e];
        to_bf16x8(xf, xh, xl, sp);
      }
      if (sp) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[c], xh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[c], xl, acc, 0, 0, 0);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[c], xh, acc, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      if (t >= nts) break;
      bf16x8 th, tl;
      if (TVEC) {   // bf16 storage: the loaded words are the hi operand, the lo part is zero
        th = __builtin_bit_cast(bf16x8, tr[set][t]);
#pragma unroll
        for (int e = 0; e < 8; ++e) tl[e] = static_cast<__bf16>(0.f);
      } else {
        float tf[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) tf[e] = te[set][t][TVEC ? 0 : e];
        to_bf16x8(tf, th, tl, sp);
      }
      if (sp) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(tl, ch[t], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(th, cl[t], acc, 0, 0, 0);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(th, ch[t], acc, 0, 0, 0);
    }
    const uint32_t yrow = static_cast<uint32_t>(b * O * P + h * W);     // elements, row-uniform
    // one branch per row picks the epilogue form; each form is straight-line over the 16 outputs
    auto epilogue = [&](auto gelu, auto keep_pre) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int oo = 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        const uint32_t bad = (valid && nok && oo < O) ? 0u : kOOB;
        const uint32_t e = static_cast<uint32_t>(oo * P + w);
        float v = acc[i] + sb[oo];
        if (decltype(keep_pre)::value)
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rPre, (4u * e) | bad, 4u * yrow, 0);
        if (decltype(gelu)::value) v = gelu_f(v);
        if (YS == 4)
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rY, (4u * e) | bad, 4u * yrow, 0);
        else
          __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, static_cast<__bf16>(v)), rY,
                                                (2u * e) | bad, 2u * yrow, 0);
      }
    };
    if (!act) epilogue(std::false_type{}, std::false_type{});
    else if (!pre) epilogue(std::true_type{}, std::false_type{});
    else epilogue(std::true_type{}, std::true_type{});
  };
  if (r0 >= r1) return;
  // rows past the block's last are clamped to it (loaded again, computed, not stored): every load and
  // store is issued unconditionally, so each wait covers exactly the loads it needs
  load_row(0, r0);
  load_row(1, min(r0 + 1, r1 - 1));
  for (int r = r0; r < r1; r += 3) {
    load_row(2, min(r + 2, r1 - 1));
    row(0, r, true);
    load_row(0, min(r + 3, r1 - 1));
    row(1, min(r + 1, r1 - 1), r + 1 < r1);
    load_row(1, min(r + 4, r1 - 1));
    row(2, min(r + 2, r1 - 1), r + 2 < r1);
  }
}

// Fused projection on the bf16 matrix cores (FP32 accumulation): out[b][p] = sum_j Q2[j] GELU(sum_c
// Q1[j][c] v[b][c][p] + q1b[j]) + q2b (C <= 32 channels), 32 hidden rows per pass; each lane sums its
// rows, the two halves of the wave are added with a lane exchange.  Q1, q1b and Q2 are staged in LDS once
// per block.  With keep (qpre non-null), qpre and q ([b][Hp][P]) are stored.
template <typename TV>
__global__ __launch_bounds__(256) void nop_project_kernel(const float* __restrict__ Q1, const float* __restrict__ q1b,
                                                          const float* __restrict__ Q2, const float* __restrict__ q2b,
                                                          const TV* __restrict__ v, float* __restrict__ out,
                                                          float* __restrict__ qpre, float* __restrict__ q, int C,
                                                          int Hp, int64_t P, int split) {
  extern __shared__ float sm[];
  const int ldq = C + 1;
  float* sQ1 = sm;                  // [Hp][C + 1]
  float* sb = sQ1 + Hp * ldq;       // [Hp]
  float* s2 = sb + Hp;              // [Hp]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t b = blockIdx.y;
  const int64_t n = static_cast<int64_t>(blockIdx.x) * 128 + wave * 32 + (lane & 31);
  const int kh = 8 * (lane >> 5), o = lane & 31;
  const bool nok = n < P;
  const rsrc_t rv = wave_rsrc(v + b * C * P, static_cast<uint32_t>(C * P * sizeof(TV)));
  float xv[2][8];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 16 * c + kh + e;
      xv[c][e] = ld_elem<TV>(rv, (nok && k < C) ? static_cast<uint32_t>((k * P + n) * sizeof(TV)) : kOOB);
    }
  stage_matrix(sQ1, ldq, Q1, Hp, C, false);
  for (int i = tid; i < Hp; i += 256) {
    sb[i] = q1b[i];
    s2[i] = Q2[i];
  }
  __syncthreads();
  const bool sp = split != 0;
  bf16x8 xh[2], xl[2];
  to_bf16x8(xv[0], xh[0], xl[0], sp);
  to_bf16x8(xv[1], xh[1], xl[1], sp);
  float part = 0.f;
  for (int t0 = 0; t0 < Hp; t0 += 32) {
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (16 * c >= C) break;
      float af[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 16 * c + kh + e;
        af[e] = (t0 + o < Hp && k < C) ? sQ1[(t0 + o) * ldq + k] : 0.f;
      }
      bf16x8 ah, al;
      to_bf16x8(af, ah, al, sp);
      if (sp) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, xh[c], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xl[c], acc, 0, 0, 0);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xh[c], acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int jj = t0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (jj < Hp) {
        const float hv = acc[r] + sb[jj];
        const float g = gelu_f(hv);
        if (qpre && nok) {
          const int64_t off = (b * Hp + jj) * P + n;
          qpre[off] = hv;
          q[off] = g;
        }
        part = fmaf(s2[jj], g, part);
      }
    }
  }
  part += __shfl_xor(part, 32);
  if (lane < 32 && nok) out[b * P + n] = part + q2b[0];
}

// Chunk-walking form of the projection for Hp <= 128 and C <= 32: each block walks `rpb` chunks of 128
// consecutive positions of one plane.  Q1 is converted once to bf16 MFMA operands in LDS, q1b and Q2 sit
// in LDS, and the v operands of the next two chunks are in flight while a chunk is multiplied; the
// hidden tiles of a chunk run one after the other, so one tile's accumulators are live at a time.  The
// MFMA sequence, the epilogue arithmetic and the order of the Q2 dot product are those of
// nop_project_kernel, so both forms give the same bits for finite activations.  KFULL: C == 32 (no channel masks); KEEP: the
// pre-activations and activations are stored for the backward pass.
template <typename TV, bool SPLIT, bool KFULL, bool KEEP>
__global__ __launch_bounds__(256) void nop_projrows_kernel(const float* __restrict__ Q1, const float* __restrict__ q1b,
                                                           const float* __restrict__ Q2, const float* __restrict__ q2b,
                                                           const TV* __restrict__ v, float* __restrict__ out,
                                                           float* __restrict__ qpre, float* __restrict__ q, int C,
                                                           int Hp, int P, int B, int rpb) {
  constexpr int MAXT = 4;                          // hidden tiles of 32
  __shared__ float sb[32 * MAXT], s2[32 * MAXT];
  __shared__ bf16x8 sah[2 * MAXT][64], sal[SPLIT ? 2 * MAXT : 1][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nc = (P + 127) >> 7;                  // chunks per plane
  const int blk = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x));
  const int q0 = blk * rpb, q1 = min(q0 + rpb, B * nc);
  const int kh = 8 * (lane >> 5), o = lane & 31;
  const int wl = wave * 32 + (lane & 31);
  const int nth = (Hp + 31) >> 5;
  constexpr bool sp = SPLIT;
  constexpr uint32_t VS = sizeof(TV);
  constexpr bool VH = VS == 2;
  for (int i = tid; i < 32 * MAXT; i += 256) {
    sb[i] = i < Hp ? q1b[i] : 0.f;
    s2[i] = i < Hp ? Q2[i] : 0.f;
  }
  // Q1 rows 32 th + o as the P operand of tile th, in operand order (entry (th, c) of lane l at
  // [2 th + c][l]); each wave converts every fourth entry
  const rsrc_t rQ = wave_rsrc(Q1, static_cast<uint32_t>(Hp * C) * 4u);
  for (int pe = wave; pe < 2 * nth; pe += 4) {
    const int th = pe >> 1, c = pe & 1;
    float af[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int j = 32 * th + o, k = 16 * c + kh + e;
      const uint32_t off = (4u * static_cast<uint32_t>(j * C + k)) | ((j < Hp && k < C) ? 0u : kOOB);
      af[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rQ, off, 0, 0));
    }
    bf16x8 h, l;
    to_bf16x8(af, h, l, sp);
    sah[pe][lane] = h;
    if (SPLIT) sal[SPLIT ? pe : 0][lane] = l;
  }
  const float b2 = q2b[0];
  __syncthreads();
  const int nxs = C > 16 ? 2 : 1;
  const rsrc_t rV = wave_rsrc(v, static_cast<uint32_t>(B * C * P) * VS);
  const rsrc_t rQp = wave_rsrc(KEEP ? static_cast<void*>(qpre) : static_cast<void*>(out),
                               KEEP ? static_cast<uint32_t>(B * Hp * P) * 4u : 0u);
  const rsrc_t rQg = wave_rsrc(KEEP ? static_cast<void*>(q) : static_cast<void*>(out),
                               KEEP ? static_cast<uint32_t>(B * Hp * P) * 4u : 0u);
  const rsrc_t rO = wave_rsrc(out, static_cast<uint32_t>(B * P) * 4u);

  float xr[3][2][VH ? 1 : 8];
  bf16x8 xb[3][2];
  auto load_chunk = [&](int set, int qi) {
    const int b = qi / nc, n = (qi - b * nc) * 128 + wl;
    const uint32_t vrow = VS * static_cast<uint32_t>(b * C * P);
    // with all 32 channels present the per-lane offset is one register and the channel goes into the
    // scalar offset; otherwise each element carries its own range mask
    const uint32_t vlane = (VS * static_cast<uint32_t>(kh * P + n)) | (n < P ? 0u : kOOB);
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 16 * c + kh + e;
        const uint32_t off = KFULL ? vlane : (VS * static_cast<uint32_t>(k * P + n)) | ((n < P && k < C) ? 0u : kOOB);
        const uint32_t so = KFULL ? vrow + VS * static_cast<uint32_t>((16 * c + e) * P) : vrow;
        if (VH)
          xb[set][c][e] = __builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(rV, off, so, 0));
        else
          xr[set][c][VH ? 0 : e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rV, off, so, 0));
      }
  };
  auto chunk = [&](int set, int qi, bool valid) {
    const int b = qi / nc, n = (qi - b * nc) * 128 + wl;
    const bool nok = valid && n < P;
    bf16x8 xh[2], xl[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (VH) {
        xh[c] = xb[set][c];
#pragma unroll
        for (int e = 0; e < 8; ++e) xl[c][e] = static_cast<__bf16>(0.f);
      } else {
        float xf[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) xf[e] = xr[set][c][VH ? 0 : e];
        to_bf16x8(xf, xh[c], xl[c], sp);
      }
    }
    const uint32_t qrow = static_cast<uint32_t>(b * Hp * P);
    float part = 0.f;
#pragma unroll 1
    for (int th = 0; th < nth; ++th) {
      f32x16 acc;
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = 0.f;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (c >= nxs) break;
        const bf16x8 ah = sah[2 * th + c][lane];
        if (sp) {
          const bf16x8 al = sal[SPLIT ? 2 * th + c : 0][lane];
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, xh[c], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xl[c], acc, 0, 0, 0);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xh[c], acc, 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int jj = 32 * th + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        const float hv = acc[i] + sb[jj];
        const float g = gelu_f(hv);
        if (KEEP) {
          const uint32_t off = (4u * static_cast<uint32_t>(jj * P + n)) | ((nok && jj < Hp) ? 0u : kOOB);
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, hv), rQp, off, 4u * qrow, 0);
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, g), rQg, off, 4u * qrow, 0);
        }
        // rows past Hp have zero Q1 rows, bias and Q2 entries: they add 0 * GELU(0) = 0
        part = fmaf(s2[jj], g, part);
      }
    }
    part += __shfl_xor(part, 32);
    const uint32_t ooff = (4u * static_cast<uint32_t>(b * P + n)) | ((lane < 32 && nok) ? 0u : kOOB);
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, part + b2), rO, ooff, 0, 0);
  };
  if (q0 >= q1) return;
  load_chunk(0, q0);
  load_chunk(1, min(q0 + 1, q1 - 1));
  for (int qi = q0; qi < q1; qi += 3) {
    load_chunk(2, min(qi + 2, q1 - 1));
    chunk(0, qi, true);
    load_chunk(0, min(qi + 3, q1 - 1));
    chunk(1, min(qi + 1, q1 - 1), qi + 1 < q1);
    load_chunk(1, min(qi + 4, q1 - 1));
    chunk(2, min(qi + 2, q1 - 1), qi + 2 < q1);
  }
}

// Truncated 2D DCT of every (b, c) plane, entirely in registers: A[pl][kh][kw] = sum_h sum_w Ch[kh][h]
// V[pl][h][w] Cw[kw][w] (natural layout [b][c][kh][kw]), one plane per wave, on the bf16 matrix cores
// (FP32 accumulation; split: hi/lo parts).  v_mfma_f32_16x16x16_bf16: lane l = 16 g + j supplies
// P[j][4g .. 4g+3] and Q[j][4g .. 4g+3] and receives C[4g + r][j] in register r.
//   pass 1, per block of 16 rows h:  C1[h][kw] = sum_w V[h][w] Cw[kw][w]   (P: 4 consecutive w of one
//            row of V, a 16-byte load; Q: a row of Cw)
//   pass 2:  A[kh][kw] += sum_h Ch[kh][h] C1[h][kw] over the same 16 rows   (P: a row of Ch; Q: C1 as it
//            sits in the registers, since lane (g, j) holds rows 4g .. 4g+3 of column j)
// so the intermediate never leaves the wave.  The DCT tables are staged in LDS as bf16 (and remainders),
// zero padded to multiples of 16.  NT = ceil(Mm / 16) tiles per mode axis; W <= 128.
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a), __builtin_bit_cast(s16x4, b), c, 0, 0,
                                                   0);
}
__device__ __forceinline__ void to_bf16x4(const float (&x)[4], bf16x4& hi, bf16x4& lo, bool split) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const __bf16 h = static_cast<__bf16>(x[e]);
    hi[e] = h;
    lo[e] = split ? static_cast<__bf16>(x[e] - static_cast<float>(h)) : static_cast<__bf16>(0.f);
  }
}
// acc += P Q^T over one K-step of 16 (hi*hi, and with split hi*lo + lo*hi)
__device__ __forceinline__ f32x4 mma16(bf16x4 ph, bf16x4 pl, bf16x4 qh, bf16x4 ql, f32x4 acc, bool split) {
  if (split) {
    acc = mfma16(pl, qh, acc);
    acc = mfma16(ph, ql, acc);
  }
  return mfma16(ph, qh, acc);
}


// LDS <- n16 16-byte chunks from global memory, eight loads per thread in flight before their stores.
typedef unsigned u32x4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void stage_bytes(void* dst, const void* __restrict__ src, int n16) {
  const u32x4v* s4 = static_cast<const u32x4v*>(src);
  u32x4v* d4 = static_cast<u32x4v*>(dst);
  for (int base = 0; base < n16; base += 8 * 256) {
    u32x4v v[8];
    int idx[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {   // clamped: lanes past the end copy the last chunk again
      idx[u] = min(base + static_cast<int>(threadIdx.x) + 256 * u, n16 - 1);
      v[u] = s4[idx[u]];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) d4[idx[u]] = v[u];
  }
}

// LDS images of the DCT tables for the per-plane kernels, built once per surrogate, in exactly the
// layout those kernels read (bf16, and the bf16 remainders with split; zero padded to multiples of 16):
//   dct2 image:    Cw [M16][W16 + 4] hi, (lo), then Ch [M16][H16 + 4] hi, (lo)
//   idct_h image:  Ch^T [H16][M16 + 4] hi, (lo)
__global__ void nop_tables_kernel(const float* __restrict__ Ch, const float* __restrict__ Cw, __bf16* dimg,
                                  __bf16* iimg, int H, int W, int Mm, int M16, int split) {
  const int H16 = (H + 15) & ~15, W16 = (W + 15) & ~15;
  const int ldw = W16 + 4, ldh = H16 + 4, ldc = M16 + 4;
  const int parts = split ? 2 : 1;
  const int64_t nd = static_cast<int64_t>(parts) * M16 * (ldw + ldh), ni = static_cast<int64_t>(parts) * H16 * ldc;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nd + ni;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    float x = 0.f;
    bool lo = false;
    if (i < nd) {
      const int64_t cwn = static_cast<int64_t>(parts) * M16 * ldw;
      if (i < cwn) {
        const int64_t e = i % (static_cast<int64_t>(M16) * ldw);
        lo = i >= static_cast<int64_t>(M16) * ldw;
        const int r = static_cast<int>(e / ldw), c = static_cast<int>(e % ldw);
        x = (r < Mm && c < W) ? Cw[r * W + c] : 0.f;
      } else {
        const int64_t e0 = i - cwn, e = e0 % (static_cast<int64_t>(M16) * ldh);
        lo = e0 >= static_cast<int64_t>(M16) * ldh;
        const int r = static_cast<int>(e / ldh), c = static_cast<int>(e % ldh);
        x = (r < Mm && c < H) ? Ch[r * H + c] : 0.f;
      }
    } else {
      const int64_t e0 = i - nd, e = e0 % (static_cast<int64_t>(H16) * ldc);
      lo = e0 >= static_cast<int64_t>(H16) * ldc;
      const int r = static_cast<int>(e / ldc), c = static_cast<int>(e % ldc);
      x = (r < H && c < Mm) ? Ch[c * H + r] : 0.f;
    }
    const __bf16 h = static_cast<__bf16>(x);
    const __bf16 v = lo ? static_cast<__bf16>(x - static_cast<float>(h)) : h;
    if (i < nd) dimg[i] = v;
    else iimg[i - nd] = v;
  }
}

template <int NT, bool VEC, typename TV>
__global__ __launch_bounds__(256) void nop_dct2_kernel(const TV* __restrict__ V, float* __restrict__ A,
                                                       const __bf16* __restrict__ img, int planes, int H, int W, int Mm,
                                                       int split) {
  constexpr int M16 = 16 * NT;
  extern __shared__ __attribute__((aligned(16))) __bf16 tb[];
  const int H16 = (H + 15) & ~15, W16 = (W + 15) & ~15;
  const int ldw = W16 + 4, ldh = H16 + 4;       // bf16 row strides (8-byte aligned rows)
  const bool sp = split != 0;
  __bf16* cwh = tb;                              // [M16][ldw]
  __bf16* cwl = cwh + M16 * ldw;
  __bf16* chh = cwl + (sp ? M16 * ldw : 0);      // [M16][ldh]
  __bf16* chl = chh + M16 * ldh;
  const int tid = threadIdx.x;
  stage_bytes(tb, img, static_cast<int>((sp ? 2 : 1) * M16 * (ldw + ldh) * sizeof(__bf16) / 16));
  __syncthreads();
  const int lane = tid & 63, g = lane >> 4, j = lane & 15;
  // the wave index through readfirstlane: the plane and its buffer descriptor stay in scalar registers
  const int64_t pl = static_cast<int64_t>(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(tid >> 6);
  if (pl >= planes) return;
  // loads through a buffer resource over the plane: an out-of-range offset reads zero, so no load is
  // predicated and the next block's loads stay in flight during this block's MFMAs
  constexpr uint32_t ES = sizeof(TV);
  const rsrc_t rv = wave_rsrc(V + pl * H * W, static_cast<uint32_t>(H * W) * ES);
  const int KS = W16 >> 4, MT = H16 >> 4;
  f32x4 acc[NT][NT];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  auto load_rows = [&](float (&v)[8][4], int mt) {
    const int h = 16 * mt + j;
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int w0 = 16 * ks + 4 * g;
      if (VEC) {   // W % 4 == 0: a 4-element group is all inside the row or all past it
        const uint32_t off = (h < H && w0 < W) ? ES * static_cast<uint32_t>(h * W + w0) : kOOB;
        if (ES == 4) {
          const f32x4 x = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rv, off, 0, 0));
#pragma unroll
          for (int e = 0; e < 4; ++e) v[ks][e] = x[e];
        } else {
          const bf16x4 x = __builtin_bit_cast(bf16x4, __builtin_amdgcn_raw_buffer_load_b64(rv, off, 0, 0));
#pragma unroll
          for (int e = 0; e < 4; ++e) v[ks][e] = static_cast<float>(x[e]);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t off = (h < H && w0 + e < W) ? ES * static_cast<uint32_t>(h * W + w0 + e) : kOOB;
          if (ES == 4)
            v[ks][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rv, off, 0, 0));
          else
            v[ks][e] = static_cast<float>(__builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(rv, off, 0, 0)));
        }
      }
    }
  };
  auto block = [&](const float (&v)[8][4], int mt) {
    f32x4 c1[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) c1[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      if (ks < KS) {
        bf16x4 vh, vl;
        to_bf16x4(v[ks], vh, vl, sp);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int o = (16 * nt + j) * ldw + 16 * ks + 4 * g;
          const bf16x4 qh = *reinterpret_cast<const bf16x4*>(cwh + o);
          const bf16x4 ql = sp ? *reinterpret_cast<const bf16x4*>(cwl + o) : qh;
          c1[nt] = mma16(vh, vl, qh, ql, c1[nt], sp);
        }
      }
    }
    bf16x4 yh[NT], yl[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const float y[4] = {c1[nt][0], c1[nt][1], c1[nt][2], c1[nt][3]};
      to_bf16x4(y, yh[nt], yl[nt], sp);
    }
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const int o = (16 * a + j) * ldh + 16 * mt + 4 * g;
      const bf16x4 ph = *reinterpret_cast<const bf16x4*>(chh + o);
      const bf16x4 pq = sp ? *reinterpret_cast<const bf16x4*>(chl + o) : ph;
#pragma unroll
      for (int c = 0; c < NT; ++c) acc[a][c] = mma16(ph, pq, yh[c], yl[c], acc[a][c], sp);
    }
  };
  float va[8][4], vb[8][4];
  load_rows(va, 0);
  for (int mt = 0; mt < MT; mt += 2) {
    if (mt + 1 < MT) load_rows(vb, mt + 1);
    block(va, mt);
    if (mt + 1 >= MT) break;
    if (mt + 2 < MT) load_rows(va, mt + 2);
    block(vb, mt + 1);
  }
  float* ap = A + pl * Mm * Mm;
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int kh = 16 * a + 4 * g + r, kw = 16 * c + j;
        if (kh < Mm && kw < Mm) ap[kh * Mm + kw] = acc[a][c][r];
      }
}

// Streaming form of the same transform (W % 4 == 0): each wave takes planes pl0, pl0 + stride, ... and
// walks their 16-row blocks as one sequence, so the loads of the next two row blocks are in flight while
// a block is multiplied, across plane boundaries too.  bf16 planes enter the MFMAs as loaded.  Same
// products in the same order as nop_dct2_kernel, so both forms give the same bits.
template <int NT, typename TV>
__global__ __launch_bounds__(256) void nop_dct2w_kernel(const TV* __restrict__ V, float* __restrict__ A,
                                                        const __bf16* __restrict__ img, int planes, int H, int W,
                                                        int Mm, int split) {
  constexpr int M16 = 16 * NT;
  constexpr bool RAW = sizeof(TV) == 2;      // bf16 planes: the loaded words are the hi operand
  extern __shared__ __attribute__((aligned(16))) __bf16 tb[];
  const int H16 = (H + 15) & ~15, W16 = (W + 15) & ~15;
  const int ldw = W16 + 4, ldh = H16 + 4;
  const bool sp = split != 0;
  __bf16* cwh = tb;
  __bf16* cwl = cwh + M16 * ldw;
  __bf16* chh = cwl + (sp ? M16 * ldw : 0);
  __bf16* chl = chh + M16 * ldh;
  const int tid = threadIdx.x;
  stage_bytes(tb, img, static_cast<int>((sp ? 2 : 1) * M16 * (ldw + ldh) * sizeof(__bf16) / 16));
  __syncthreads();
  const int lane = tid & 63, g = lane >> 4, j = lane & 15;
  const int wv = static_cast<int>(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(tid >> 6);
  const int stride = static_cast<int>(gridDim.x) * 4;
  if (wv >= planes) return;
  const int np = (planes - 1 - wv) / stride + 1;   // planes of this wave
  const int KS = W16 >> 4, MT = H16 >> 4;
  const int n = np * MT;                           // row blocks of this wave
  constexpr uint32_t ES = sizeof(TV);
  f32x4 acc[NT][NT];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  // three register sets: raw bf16 quads (RAW) or FP32 quads
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  u32x2 rb[3][8];
  f32x4 rf[3][RAW ? 1 : 8];
  auto load_blk = [&](int set, int it) {
    const int q = it / MT, mt = it - q * MT;
    const int pl = wv + q * stride;
    const rsrc_t rv = wave_rsrc(V + static_cast<int64_t>(pl) * H * W, static_cast<uint32_t>(H * W) * ES);
    const int h = 16 * mt + j;
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int w0 = 16 * ks + 4 * g;
      const uint32_t off = (ES * static_cast<uint32_t>(h * W + w0)) | ((h < H && w0 < W) ? 0u : kOOB);
      if (RAW)
        rb[set][ks] = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rv, off, 0, 0));
      else
        rf[set][RAW ? 0 : ks] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rv, off, 0, 0));
    }
  };
  auto process = [&](int set, int it, bool valid) {
    if (!valid) return;
    const int q = it / MT, mt = it - q * MT;
    f32x4 c1[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) c1[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      if (ks < KS) {
        bf16x4 vh, vl;
        if (RAW) {
          vh = __builtin_bit_cast(bf16x4, rb[set][ks]);
#pragma unroll
          for (int e = 0; e < 4; ++e) vl[e] = static_cast<__bf16>(0.f);
        } else {
          const float x[4] = {rf[set][RAW ? 0 : ks][0], rf[set][RAW ? 0 : ks][1], rf[set][RAW ? 0 : ks][2],
                              rf[set][RAW ? 0 : ks][3]};
          to_bf16x4(x, vh, vl, sp);
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int o = (16 * nt + j) * ldw + 16 * ks + 4 * g;
          const bf16x4 qh = *reinterpret_cast<const bf16x4*>(cwh + o);
          const bf16x4 ql = sp ? *reinterpret_cast<const bf16x4*>(cwl + o) : qh;
          c1[nt] = mma16(vh, vl, qh, ql, c1[nt], sp);
        }
      }
    }
    bf16x4 yh[NT], yl[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const float y[4] = {c1[nt][0], c1[nt][1], c1[nt][2], c1[nt][3]};
      to_bf16x4(y, yh[nt], yl[nt], sp);
    }
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const int o = (16 * a + j) * ldh + 16 * mt + 4 * g;
      const bf16x4 ph = *reinterpret_cast<const bf16x4*>(chh + o);
      const bf16x4 pq = sp ? *reinterpret_cast<const bf16x4*>(chl + o) : ph;
#pragma unroll
      for (int c = 0; c < NT; ++c) acc[a][c] = mma16(ph, pq, yh[c], yl[c], acc[a][c], sp);
    }
    if (mt == MT - 1) {   // the plane is complete
      float* ap = A + static_cast<int64_t>(wv + q * stride) * Mm * Mm;
#pragma unroll
      for (int a = 0; a < NT; ++a)
#pragma unroll
        for (int c = 0; c < NT; ++c) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int kh = 16 * a + 4 * g + r, kw = 16 * c + j;
            if (kh < Mm && kw < Mm) ap[kh * Mm + kw] = acc[a][c][r];
          }
          acc[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
  };
  // items past the wave's last are clamped to it (loaded again, not processed): the loads are
  // unconditional, so each wait covers exactly the loads it needs
  load_blk(0, 0);
  load_blk(1, min(1, n - 1));
  for (int it = 0; it < n; it += 3) {
    load_blk(2, min(it + 2, n - 1));
    process(0, it, true);
    load_blk(0, min(it + 3, n - 1));
    process(1, min(it + 1, n - 1), it + 1 < n);
    load_blk(1, min(it + 4, n - 1));
    process(2, min(it + 2, n - 1), it + 2 < n);
  }
}

// First stage of the inverse DCT for every (b, c) plane: T[b][h][c][kw] = sum_kh Ch[kh][h] Z[b][c][kh][kw]
// (Z in natural layout, T laid out for the channel-mixing kernel), one plane per wave on MFMA 16x16x16
// bf16: P = Ch^T rows from LDS (bf16, remainders with split), Q = the plane's Mm x Mm coefficients,
// loaded once into registers and reused for every 16 rows of h.  NT = ceil(Mm / 16).
template <int NT, typename TT>
__global__ __launch_bounds__(256) void nop_idct_h_kernel(const float* __restrict__ Z, TT* __restrict__ T,
                                                         const __bf16* __restrict__ img, int B, int C, int H, int Mm,
                                                         int split) {
  constexpr int M16 = 16 * NT;
  constexpr int ldc = M16 + 4;                   // bf16 row stride of Ch^T
  extern __shared__ __attribute__((aligned(16))) __bf16 tb[];
  const int H16 = (H + 15) & ~15;
  const bool sp = split != 0;
  __bf16* cth = tb;                              // [H16][ldc]: Ch^T
  __bf16* ctl = cth + H16 * ldc;
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, j = lane & 15;
  stage_bytes(tb, img, static_cast<int>((sp ? 2 : 1) * H16 * ldc * sizeof(__bf16) / 16));
  __syncthreads();
  const int64_t pl = static_cast<int64_t>(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(tid >> 6);
  if (pl >= static_cast<int64_t>(B) * C) return;
  const int64_t b = pl / C;
  const int c = static_cast<int>(pl - b * C);
  const rsrc_t rz = wave_rsrc(Z + pl * Mm * Mm, static_cast<uint32_t>(Mm * Mm * 4));
  // Q operands: lane (g, j) of K-step ks and column tile nt holds Z[16 ks + 4 g + e][16 nt + j]
  bf16x4 qh[NT][NT], ql[NT][NT];
#pragma unroll
  for (int ks = 0; ks < NT; ++ks)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      float z[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int kh = 16 * ks + 4 * g + e, kw = 16 * nt + j;
        const uint32_t off = (kh < Mm && kw < Mm) ? 4u * static_cast<uint32_t>(kh * Mm + kw) : kOOB;
        z[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rz, off, 0, 0));
      }
      to_bf16x4(z, qh[ks][nt], ql[ks][nt], sp);
    }
  const int64_t rowstride = static_cast<int64_t>(C) * Mm;      // T: one h row holds every channel
  TT* tp = T + b * H * rowstride + static_cast<int64_t>(c) * Mm;
  for (int mt = 0; mt < (H16 >> 4); ++mt) {
    f32x4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < NT; ++ks) {
      const int o = (16 * mt + j) * ldc + 16 * ks + 4 * g;
      const bf16x4 ph = *reinterpret_cast<const bf16x4*>(cth + o);
      const bf16x4 pq = sp ? *reinterpret_cast<const bf16x4*>(ctl + o) : ph;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[nt] = mma16(ph, pq, qh[ks][nt], ql[ks][nt], acc[nt], sp);
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int h = 16 * mt + 4 * g + r, kw = 16 * nt + j;
        if (h < H && kw < Mm) tp[h * rowstride + kw] = static_cast<TT>(acc[nt][r]);
      }
  }
}

unsigned blocks_for(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

}  // namespace

// Tile shape by operand shape: few output rows (channel mixing, K = 32) take 32 x 256 tiles so each
// block streams a long run of positions; the rest 64 x 64.
hipError_t launch_nop_gemm(const NopGemm& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.nb1 * g.nb2 <= 0) return hipSuccess;
  const dim3 grid_z(1, g.nb1 * g.nb2);
  auto tiles = [&](int bm, int bn) { return ((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn); };
  if (g.M <= 32 && g.N >= 256) {
    hipLaunchKernelGGL((nop_gemm_kernel<1, 4, 1, 2>), dim3(tiles(32, 256), g.nb1 * g.nb2), dim3(NT), 0, s, g);
  } else {
    hipLaunchKernelGGL((nop_gemm_kernel<2, 2, 1, 1>), dim3(tiles(64, 64), g.nb1 * g.nb2), dim3(NT), 0, s, g);
  }
  (void)grid_z;
  return hipGetLastError();
}

namespace {

template <typename TX, typename TY, typename TT, int KT, bool TVEC>
void launch_mixrows_t(const float* A, bool transA, const void* X, void* Y, const float* bias, float* pre, const void* T,
                      const float* Cw, int Mm, int O, int I, int H, int W, int B, bool act, bool split, hipStream_t s) {
  const int64_t rows = static_cast<int64_t>(B) * H, groups = (W + 127) / 128;
  // about 1024 blocks of 4 waves, each walking its rows with loads two rows ahead
  const int rpb = static_cast<int>(std::max<int64_t>(1, (rows * groups + 1023) / 1024));
  const unsigned nblk = static_cast<unsigned>(((rows + rpb - 1) / rpb) * groups);
  const TX* x = static_cast<const TX*>(X);
  const TT* t = static_cast<const TT*>(T);
  TY* y = static_cast<TY*>(Y);
  const int a = act ? 1 : 0, ta = transA ? 1 : 0;
  // bf16 activations come with plain products only; the lift (FP32 features into bf16) has four inputs
  constexpr bool half_act = sizeof(TX) == 2, lift = sizeof(TX) == 4 && sizeof(TY) == 2;
  if constexpr (!half_act) {
    if (split) {
      if constexpr (!lift) {
        if (I == 32) {
          hipLaunchKernelGGL((nop_mixrows_kernel<TX, TY, TT, KT, TVEC, true, true>), dim3(nblk), dim3(256), 0, s, A, x,
                             y, bias, pre, t, Cw, O, I, H, W, Mm, B, rpb, a, ta);
          return;
        }
      }
      hipLaunchKernelGGL((nop_mixrows_kernel<TX, TY, TT, KT, TVEC, true, false>), dim3(nblk), dim3(256), 0, s, A, x, y,
                         bias, pre, t, Cw, O, I, H, W, Mm, B, rpb, a, ta);
      return;
    }
  }
  if constexpr (!lift) {
    if (I == 32) {
      hipLaunchKernelGGL((nop_mixrows_kernel<TX, TY, TT, KT, TVEC, false, true>), dim3(nblk), dim3(256), 0, s, A, x, y,
                         bias, pre, t, Cw, O, I, H, W, Mm, B, rpb, a, ta);
      return;
    }
  }
  hipLaunchKernelGGL((nop_mixrows_kernel<TX, TY, TT, KT, TVEC, false, false>), dim3(nblk), dim3(256), 0, s, A, x, y,
                     bias, pre, t, Cw, O, I, H, W, Mm, B, rpb, a, ta);
}

template <typename TX, typename TY, typename TT>
void launch_mixrows(const float* A, bool transA, const void* X, void* Y, const float* bias, float* pre, const void* T,
                    const float* Cw, int Mm, int O, int I, int H, int W, int B, bool act, bool split, hipStream_t s) {
  const int kt = T ? (Mm + 15) / 16 : 0;
  const bool vec = T && Mm % 8 == 0 && sizeof(TT) == 2;
#define PSTD_MIXROWS(KTV)                                                                                        \
  if constexpr (sizeof(TT) == 2) {                                                                               \
    if (vec) launch_mixrows_t<TX, TY, TT, KTV, true>(A, transA, X, Y, bias, pre, T, Cw, Mm, O, I, H, W, B, act, split, s); \
    else launch_mixrows_t<TX, TY, TT, KTV, false>(A, transA, X, Y, bias, pre, T, Cw, Mm, O, I, H, W, B, act, split, s); \
  } else {                                                                                                       \
    launch_mixrows_t<TX, TY, TT, KTV, false>(A, transA, X, Y, bias, pre, T, Cw, Mm, O, I, H, W, B, act, split, s); \
  }
  switch (kt) {
    case 0: launch_mixrows_t<TX, TY, TT, 0, false>(A, transA, X, Y, bias, pre, T, Cw, Mm, O, I, H, W, B, act, split, s); break;
    case 1: PSTD_MIXROWS(1) break;
    case 2: PSTD_MIXROWS(2) break;
    case 3: PSTD_MIXROWS(3) break;
    default: PSTD_MIXROWS(4) break;
  }
#undef PSTD_MIXROWS
}

}  // namespace

hipError_t launch_nop_mix(const float* A, bool transA, const void* X, void* Y, const float* bias, const float* D,
                          float* pre, const void* T, const float* Cw, int Mm, int O, int I, int H, int W, int B, bool act,
                          bool split, int act_types, hipStream_t s) {
  if (O > 32 || H < 1 || W < 1 || I < 1 || B < 1) return hipErrorInvalidValue;
  {
    // the register-resident row form: no D term, at most 32 inputs and 64 modes, 32-bit offsets
    const int64_t P = static_cast<int64_t>(H) * W;
    const int64_t xs = act_types == 2 ? 2 : 4, ts = act_types == 2 ? 2 : 4;
    const bool fits = static_cast<int64_t>(B) * I * P * xs < (int64_t(1) << 31) &&
                      static_cast<int64_t>(B) * O * P * 4 < (int64_t(1) << 31) &&
                      (!T || static_cast<int64_t>(B) * H * O * Mm * ts < (int64_t(1) << 31));
    if (!D && I <= 32 && (!T || (Mm >= 1 && Mm <= 64)) && fits) {
      typedef __bf16 bf;
      switch (act_types) {
        case 0: launch_mixrows<float, float, float>(A, transA, X, Y, bias, pre, T, Cw, Mm, O, I, H, W, B, act, split, s); break;
        case 1: launch_mixrows<float, bf, float>(A, transA, X, Y, bias, pre, T, Cw, Mm, O, I, H, W, B, act, split, s); break;
        default: launch_mixrows<bf, bf, bf>(A, transA, X, Y, bias, pre, T, Cw, Mm, O, I, H, W, B, act, split, s); break;
      }
      return hipGetLastError();
    }
  }
  const size_t lds = sizeof(float) * (32 * (I + 1) + (T ? 32 * (Mm + 1) : 0) + 32);
  if (lds > 65536) return hipErrorInvalidValue;
  const int64_t blocks = static_cast<int64_t>(H) * ((W + 127) / 128);
  const dim3 grid(static_cast<unsigned>(blocks), B), blk(256);
  const int a = act ? 1 : 0, t = transA ? 1 : 0, sp = split ? 1 : 0;
  typedef __bf16 bf;
  switch (act_types) {
    case 0:   // FP32 X, Y, T
      hipLaunchKernelGGL((nop_mix_kernel<float, float, float>), grid, blk, lds, s, A, static_cast<const float*>(X),
                         static_cast<float*>(Y), bias, D, pre, static_cast<const float*>(T), Cw, O, I, H, W, Mm, a, t, sp);
      break;
    case 1:   // FP32 X (the features), bf16 Y
      hipLaunchKernelGGL((nop_mix_kernel<float, bf, float>), grid, blk, lds, s, A, static_cast<const float*>(X),
                         static_cast<bf*>(Y), bias, D, pre, static_cast<const float*>(T), Cw, O, I, H, W, Mm, a, t, sp);
      break;
    default:  // bf16 X, Y, T
      hipLaunchKernelGGL((nop_mix_kernel<bf, bf, bf>), grid, blk, lds, s, A, static_cast<const bf*>(X), static_cast<bf*>(Y),
                         bias, D, pre, static_cast<const bf*>(T), Cw, O, I, H, W, Mm, a, t, sp);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_nop_project(const float* Q1, const float* q1b, const float* Q2, const float* q2b, const void* v,
                              float* out, float* qpre, float* q, int C, int Hp, int64_t P, int B, bool split, bool half,
                              hipStream_t s) {
  const size_t lds = sizeof(float) * (static_cast<size_t>(Hp) * (C + 1) + 2 * Hp);
  if (C > 32 || lds > 65536) return hipErrorInvalidValue;
  const int64_t vs = half ? 2 : 4;
  const bool fits = static_cast<int64_t>(B) * C * P * vs < (int64_t(1) << 31) &&
                    static_cast<int64_t>(B) * P * 4 < (int64_t(1) << 31) &&
                    (!qpre || static_cast<int64_t>(B) * Hp * P * 4 < (int64_t(1) << 31));
  const bool keep = qpre != nullptr;
  if (Hp >= 1 && Hp <= 128 && C >= 1 && fits && keep == (q != nullptr) && !(half && (split || keep))) {
    // the chunk-walking form: about 1024 blocks of 4 waves
    const int64_t chunks = static_cast<int64_t>(B) * ((P + 127) / 128);
    const int rpb = static_cast<int>(std::max<int64_t>(1, (chunks + 1023) / 1024));
    const dim3 grid(static_cast<unsigned>((chunks + rpb - 1) / rpb)), blk(256);
    const int Pi = static_cast<int>(P);
#define PSTD_PROJ_K(TVV, SPV, KPV)                                                                                \
  if (C == 32) hipLaunchKernelGGL((nop_projrows_kernel<TVV, SPV, true, KPV>), grid, blk, 0, s, Q1, q1b, Q2, q2b,    \
                                  static_cast<const TVV*>(v), out, qpre, q, C, Hp, Pi, B, rpb);                   \
  else hipLaunchKernelGGL((nop_projrows_kernel<TVV, SPV, false, KPV>), grid, blk, 0, s, Q1, q1b, Q2, q2b,          \
                          static_cast<const TVV*>(v), out, qpre, q, C, Hp, Pi, B, rpb);
    if (half) {        // the inference form: bf16 activations
      PSTD_PROJ_K(__bf16, false, false)
    } else if (split) {
      if (keep) { PSTD_PROJ_K(float, true, true) } else { PSTD_PROJ_K(float, true, false) }
    } else {
      if (keep) { PSTD_PROJ_K(float, false, true) } else { PSTD_PROJ_K(float, false, false) }
    }
#undef PSTD_PROJ_K
    return hipGetLastError();
  }
  if (half)
    hipLaunchKernelGGL(nop_project_kernel<__bf16>, dim3(blocks_for(P, 128), B), dim3(256), lds, s, Q1, q1b, Q2, q2b,
                       static_cast<const __bf16*>(v), out, qpre, q, C, Hp, P, split ? 1 : 0);
  else
    hipLaunchKernelGGL(nop_project_kernel<float>, dim3(blocks_for(P, 128), B), dim3(256), lds, s, Q1, q1b, Q2, q2b,
                       static_cast<const float*>(v), out, qpre, q, C, Hp, P, split ? 1 : 0);
  return hipGetLastError();
}

void nop_table_bytes(int H, int W, int Mm, bool split, size_t* dct2_bytes, size_t* idct_bytes) {
  const int M16 = (Mm + 15) & ~15, H16 = (H + 15) & ~15, W16 = (W + 15) & ~15;
  const size_t parts = split ? 2 : 1;
  *dct2_bytes = parts * M16 * ((W16 + 4) + (H16 + 4)) * sizeof(__bf16);
  *idct_bytes = parts * H16 * (M16 + 4) * sizeof(__bf16);
}

hipError_t launch_nop_tables(const float* Ch, const float* Cw, void* dct2_img, void* idct_img, int H, int W, int Mm,
                             bool split, hipStream_t s) {
  const int M16 = (Mm + 15) & ~15;
  hipLaunchKernelGGL(nop_tables_kernel, dim3(256), dim3(256), 0, s, Ch, Cw, static_cast<__bf16*>(dct2_img),
                     static_cast<__bf16*>(idct_img), H, W, Mm, M16, split ? 1 : 0);
  return hipGetLastError();
}

bool nop_dct2_supported(int H, int W, int Mm) { return W <= 128 && Mm <= 64 && H >= 1 && W >= 1 && Mm >= 1; }

hipError_t launch_nop_dct2(const void* V, float* A, const void* img, int planes, int H, int W, int Mm, bool split,
                           bool half, hipStream_t s) {
  if (!nop_dct2_supported(H, W, Mm) || planes < 1) return hipErrorInvalidValue;
  if ((W & 3) == 0 && (reinterpret_cast<uintptr_t>(V) & (half ? 7 : 15)) != 0) return hipErrorInvalidValue;
  const int NT = (Mm + 15) / 16;
  const int H16 = (H + 15) & ~15, W16 = (W + 15) & ~15;
  const size_t lds = sizeof(__bf16) * (split ? 2 : 1) * 16 * NT * ((W16 + 4) + (H16 + 4));
  if (lds > 65536 || static_cast<int64_t>(H) * W * 4 >= (int64_t(1) << 31)) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>((planes + 3) / 4)), blk(256);
  const int sp = split ? 1 : 0;
  const bool vec = (W & 3) == 0;
  const __bf16* tab = static_cast<const __bf16*>(img);
  const float* Vf = static_cast<const float*>(V);
  const __bf16* Vh = static_cast<const __bf16*>(V);
  // streaming form for rows of whole 4-element groups: about 512 blocks (two per CU), every wave walking
  // its planes' row blocks with loads two blocks ahead
  const dim3 sgrid(static_cast<unsigned>(std::min<int64_t>((planes + 3) / 4, 512)));
#define PSTD_DCT2(NTV)                                                                                          \
  if (half && vec) hipLaunchKernelGGL((nop_dct2w_kernel<NTV, __bf16>), sgrid, blk, lds, s, Vh, A, tab, planes, H, W, Mm, sp); \
  else if (half) hipLaunchKernelGGL((nop_dct2_kernel<NTV, false, __bf16>), grid, blk, lds, s, Vh, A, tab, planes, H, W, Mm, sp); \
  else if (vec) hipLaunchKernelGGL((nop_dct2w_kernel<NTV, float>), sgrid, blk, lds, s, Vf, A, tab, planes, H, W, Mm, sp); \
  else hipLaunchKernelGGL((nop_dct2_kernel<NTV, false, float>), grid, blk, lds, s, Vf, A, tab, planes, H, W, Mm, sp);
  switch (NT) {
    case 1: PSTD_DCT2(1) break;
    case 2: PSTD_DCT2(2) break;
    case 3: PSTD_DCT2(3) break;
    default: PSTD_DCT2(4) break;
  }
#undef PSTD_DCT2
  return hipGetLastError();
}

hipError_t launch_nop_idct_h(const float* Z, void* T, const void* img, int B, int C, int H, int Mm, bool split,
                             bool half, hipStream_t s) {
  if (Mm < 1 || Mm > 64 || H < 1 || B < 1 || C < 1) return hipErrorInvalidValue;
  const int NT = (Mm + 15) / 16;
  const int H16 = (H + 15) & ~15;
  const size_t lds = sizeof(__bf16) * (split ? 2 : 1) * H16 * (16 * NT + 4);
  if (lds > 65536) return hipErrorInvalidValue;
  const int64_t planes = static_cast<int64_t>(B) * C;
  const dim3 grid(static_cast<unsigned>((planes + 3) / 4)), blk(256);
  const int sp = split ? 1 : 0;
  const __bf16* tab = static_cast<const __bf16*>(img);
  float* Tf = static_cast<float*>(T);
  __bf16* Th = static_cast<__bf16*>(T);
#define PSTD_IDCT(NTV)                                                                                          \
  if (half) hipLaunchKernelGGL((nop_idct_h_kernel<NTV, __bf16>), grid, blk, lds, s, Z, Th, tab, B, C, H, Mm, sp);    \
  else hipLaunchKernelGGL((nop_idct_h_kernel<NTV, float>), grid, blk, lds, s, Z, Tf, tab, B, C, H, Mm, sp);
  switch (NT) {
    case 1: PSTD_IDCT(1) break;
    case 2: PSTD_IDCT(2) break;
    case 3: PSTD_IDCT(3) break;
    default: PSTD_IDCT(4) break;
  }
#undef PSTD_IDCT
  return hipGetLastError();
}

hipError_t launch_nop_mode_transpose(const float* in, float* out, int B, int C, int Mm, bool to_block, hipStream_t s) {
  if (C > 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(nop_mode_transpose_kernel, dim3(blocks_for(static_cast<int64_t>(Mm) * Mm, 64), B), dim3(256), 0,
                     s, in, out, B, C, Mm, to_block ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_nop_features(const float* p0, const float* c0, float* f, int B, int H, int W, hipStream_t s) {
  hipLaunchKernelGGL(nop_features_kernel, dim3(blocks_for(static_cast<int64_t>(B) * H * W, 256)), dim3(256), 0, s, p0,
                     c0, f, B, H, W);
  return hipGetLastError();
}

hipError_t launch_nop_gelu_bwd(const float* gin, const float* pre, float* d, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(nop_gelu_bwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, gin, pre, d, n);
  return hipGetLastError();
}

hipError_t launch_nop_rowsum(const float* x, float* out, int nb, int rows, int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(nop_rowsum_kernel, dim3(rows), dim3(256), 0, s, x, out, nb, rows, P);
  return hipGetLastError();
}

hipError_t launch_nop_partial_sum(const float* part, float* out, int nz, int n, hipStream_t s) {
  hipLaunchKernelGGL(nop_partial_sum_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, part, out, nz, n);
  return hipGetLastError();
}

hipError_t launch_nop_loss(const float* out, const float* tgt, double* terms, float* dout, int B, int64_t P,
                           hipStream_t s) {
  hipLaunchKernelGGL(nop_loss_terms_kernel, dim3(B), dim3(256), 0, s, out, tgt, terms, P);
  if (dout)
    hipLaunchKernelGGL(nop_loss_grad_kernel, dim3(blocks_for(static_cast<int64_t>(B) * P, 256)), dim3(256), 0, s, out,
                       tgt, terms, dout, B, P);
  return hipGetLastError();
}

hipError_t launch_nop_input_stats(const float* p0, const float* c0, double* stats, int B, int H, int W, int margin,
                                  hipStream_t s) {
  hipLaunchKernelGGL(nop_input_stats_kernel, dim3(B), dim3(256), 0, s, p0, c0, stats, H, W, margin);
  return hipGetLastError();
}

hipError_t launch_nop_adam(float* th, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(nop_adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, th, g, m, v, n, lr, b1, b2, eps, c1,
                     c2);
  return hipGetLastError();
}

}  // namespace pstd
