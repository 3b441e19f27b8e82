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
#include <cmath>

#include "common.h"

namespace pstd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int LDK = BK + 8;     // LDS row stride in bf16 (80 bytes: conflict-free 16-byte reads)
constexpr int NT = 256;         // 4 waves, 2 x 2, each 32 x 32
constexpr int PER = BM * BK / NT;   // elements of each operand tile per thread (8)

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// Element e (0 .. BM*BK-1) of an operand tile: row r (m for A, n for B) and column k.  Lanes run along
// k when the operand is contiguous in k, along the rows otherwise, so the loads coalesce either way.
__device__ __forceinline__ void tile_pos(int e, bool kcontig, int& r, int& k) {
  if (kcontig) {
    k = e & (BK - 1);
    r = e >> 5;
  } else {
    r = e & (BM - 1);
    k = e >> 6;
  }
}

__global__ __launch_bounds__(NT) void nop_gemm_kernel(NopGemm g) {
  __shared__ __attribute__((aligned(16))) __bf16 lds[4][BM * LDK];   // A hi, A lo, B hi, B lo ([row][k])
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int tiles_m = (g.M + BM - 1) / BM;
  const int m0 = (blockIdx.x % tiles_m) * BM, n0 = (blockIdx.x / tiles_m) * BN;
  const int z = blockIdx.y;
  const int z1 = z / g.nb2, z2 = z - z1 * g.nb2;
  const float* A = g.A + z1 * g.bA1 + z2 * g.bA2;
  const float* B = g.B + z1 * g.bB1 + z2 * g.bB2;
  const bool akc = g.sAk == 1, bkc = g.sBk == 1;
  const bool split = g.split != 0;

  float ra[PER], rb[PER];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      int r, k;
      tile_pos(tid + i * NT, akc, r, k);
      const int m = m0 + r, kk = k0 + k;
      ra[i] = (m < g.M && kk < g.K) ? A[m * g.sAm + kk * g.sAk] : 0.f;
      tile_pos(tid + i * NT, bkc, r, k);
      const int n = n0 + r;
      const int kb = k0 + k;
      rb[i] = (n < g.N && kb < g.K) ? B[kb * g.sBk + n * g.sBn] : 0.f;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      int r, k;
      tile_pos(tid + i * NT, akc, r, k);
      const __bf16 h = static_cast<__bf16>(ra[i]);
      lds[0][r * LDK + k] = h;
      if (split) lds[1][r * LDK + k] = static_cast<__bf16>(ra[i] - static_cast<float>(h));
      tile_pos(tid + i * NT, bkc, r, k);
      const __bf16 hb = static_cast<__bf16>(rb[i]);
      lds[2][r * LDK + k] = hb;
      if (split) lds[3][r * LDK + k] = static_cast<__bf16>(rb[i] - static_cast<float>(hb));
    }
  };

  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  const int nsl = (g.K + BK - 1) / BK;
  load(0);
  store();
  lds_barrier();
  const int arow = wm * 32 + (lane & 31), brow = wn * 32 + (lane & 31);
  const int koff = 8 * (lane >> 5);
  for (int s = 0; s < nsl; ++s) {
    if (s + 1 < nsl) load((s + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&lds[0][arow * LDK + kk + koff]);
      const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&lds[2][brow * LDK + kk + koff]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
      if (split) {
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(&lds[1][arow * LDK + kk + koff]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&lds[3][brow * LDK + kk + koff]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
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
  const int n = n0 + wn * 32 + (lane & 31);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (m < g.M && n < g.N) {
      const int64_t co = m * g.sCm + n * g.sCn;
      float v = g.alpha * acc[r];
      if (g.beta != 0.f) v += g.beta * C[co];
      if (g.bias_m) v += g.bias_m[m];
      if (Dp) v += Dp[m * g.sDm + n * g.sDn];
      if (Gp) v *= gelu_grad_f(Gp[co]);
      if (g.act) {
        if (Pp) Pp[co] = v;
        v = gelu_f(v);
      }
      C[co] = v;
    }
  }
}

// Natural spectral layout [b][c][kh][kw] <-> block layout [blk][q][b][c] (blk = (kh/2)(Mm/2) + kw/2,
// q = 2 (kh%2) + kw%2): the modes that share one mixing matrix become one contiguous GEMM operand.
__global__ void nop_mode_transpose_kernel(const float* in, float* out, int B, int C, int Mm, int to_block) {
  const int64_t total = static_cast<int64_t>(B) * C * Mm * Mm;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  // i enumerates the natural layout
  const int kw = static_cast<int>(i % Mm);
  const int kh = static_cast<int>((i / Mm) % Mm);
  const int64_t bc = i / (static_cast<int64_t>(Mm) * Mm);
  const int c = static_cast<int>(bc % C);
  const int b = static_cast<int>(bc / C);
  const int blk = (kh >> 1) * (Mm >> 1) + (kw >> 1);
  const int q = 2 * (kh & 1) + (kw & 1);
  const int64_t j = ((static_cast<int64_t>(blk) * 4 + q) * B + b) * C + c;
  if (to_block) out[j] = in[i];
  else out[i] = in[j];
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

unsigned blocks_for(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

}  // namespace

hipError_t launch_nop_gemm(const NopGemm& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.nb1 * g.nb2 <= 0) return hipSuccess;
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  hipLaunchKernelGGL(nop_gemm_kernel, dim3(tiles, g.nb1 * g.nb2), dim3(NT), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_nop_mode_transpose(const float* in, float* out, int B, int C, int Mm, bool to_block, hipStream_t s) {
  const int64_t n = static_cast<int64_t>(B) * C * Mm * Mm;
  hipLaunchKernelGGL(nop_mode_transpose_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, B, C, Mm,
                     to_block ? 1 : 0);
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
