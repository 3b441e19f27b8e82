// Two fused phase kernels per step for 2D FP32 plans with at most 512 nodes per axis.
//
// Eq. (dtt_pstd_solution) in its 2D form (§4.3) splits into a velocity phase and a pressure phase:
//   velocity  u_x += G~x p   and   u_y += p G~y^T           (one launch, every u_x and u_y tile)
//   pressure  p += c2 .* (D~x u_x + u_y D~y^T)               (one launch; each p tile takes both axes'
//                                                             terms, so p is read and written once)
// A small box is bound by latency, so each block computes one 32 x 32 output tile from full-K operand
// slices staged into LDS in one pass (no K loop of dependent loads).  The kernel boundary between the
// phases is the grid-wide dependency of the scheme; graph replay keeps the launch gaps short.
// Each wave computes one 16 x 16 quarter with four independent MFMA accumulator chains whose sums
// are flushed into FP64 registers every 16 k; the update is formed in FP64 and rounded once.
//
// MFMA v_mfma_f32_16x16x4: lane l supplies P[l%16][l/16] and Q[l%16][l/16] (both staged as [row][k])
// and receives C[4*(l/16)+r][l%16] in register r.  The operand whose rows run along the output's
// unit-stride axis goes to the Q port, so lanes 0..15 write 16 consecutive floats.
#include "common.h"

namespace pstd {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TILE = 32;        // output tile edge
constexpr int KMAX = 512;       // largest contracted extent handled
constexpr int LDT = KMAX + 1;   // LDS row stride (floats), odd: conflict-free reads down a column
constexpr int NT = 256;         // 4 waves

struct Phase2DArgs {
  const float* Gx; int ldgx;    // (nx-1) x nx, zero padded to row stride ldgx
  const float* Gy; int ldgy;    // (ny-1) x ny
  const float* Dx; int lddx;    // nx x (nx-1)
  const float* Dy; int lddy;    // ny x (ny-1)
  float* p;                     // nx x ny
  float* ux;                    // (nx-1) x ny
  float* uy;                    // nx x (ny-1)
  const float* c2;              // nx x ny or null
  int nx, ny;
};

// Rows [r0, r0+TILE) x k [0, Kpad) of a row-major matrix (row stride ld) into LDS as [row][k]: wave w
// takes rows w, w+4, ...; lanes stride along k.  Reads only rows < `rows` and k < K; the rest is zero.
// Loads are issued in batches of four rows before their LDS stores, so a batch costs one round trip.
__device__ __forceinline__ void stage_rows(float* dst, const float* __restrict__ src, int64_t ld, int r0, int rows,
                                           int K, int Kpad) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int RPW = TILE / (NT / 64);   // rows per wave
  constexpr int KCH = KMAX / 64;          // k chunks per row
#pragma unroll
  for (int g = 0; g < RPW; g += 4) {
    float v[4][KCH];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wave + (NT / 64) * (g + i);
      const bool rv = r0 + r < rows;
      const float* s = src + static_cast<int64_t>(rv ? r0 + r : 0) * ld;
#pragma unroll
      for (int j = 0; j < KCH; ++j) {
        const int k = lane + 64 * j;
        v[i][j] = (rv && k < K) ? s[k] : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wave + (NT / 64) * (g + i);
#pragma unroll
      for (int j = 0; j < KCH; ++j) {
        const int k = lane + 64 * j;
        if (k < Kpad) dst[r * LDT + k] = v[i][j];
      }
    }
  }
}

// Columns [c0, c0+TILE) x k [0, Kpad) of a row-major matrix X[k][c] (row stride ld) transposed into LDS
// as [c][k]: each wave instruction reads two 32-float row segments.  Reads only c < `cols`, k < K.
// Loads are issued 16 at a time before their LDS stores.
__device__ __forceinline__ void stage_cols(float* dst, const float* __restrict__ src, int64_t ld, int c0, int cols,
                                           int K, int Kpad) {
  const int c = threadIdx.x & 31;
  const int kb = threadIdx.x >> 5;
  const bool cv = c0 + c < cols;
  constexpr int KS = NT / 32;             // k stride between a thread's elements
  for (int k0 = 0; k0 < Kpad; k0 += 16 * KS) {
    float v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = k0 + kb + KS * u;
      v[u] = (cv && k < K) ? src[static_cast<int64_t>(k) * ld + c0 + c] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int k = k0 + kb + KS * u;
      if (k < Kpad) dst[c * LDT + k] = v[u];
    }
  }
}

// accd (this wave's 16 x 16 quarter) += P[rows][0..K) . Q[cols][0..K)^T; K a multiple of 16, zero padded.
__device__ __forceinline__ void mma_tile(const float* P, const float* Q, int K, double (&accd)[4]) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int kl = lane >> 4;
  const float* Pp = P + ((wave & 1) * 16 + (lane & 15)) * LDT + kl;
  const float* Qp = Q + ((wave >> 1) * 16 + (lane & 15)) * LDT + kl;
  for (int k0 = 0; k0 < K; k0 += 16) {
    f32x4 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0}, c2 = {0, 0, 0, 0}, c3 = {0, 0, 0, 0};
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Pp[k0], Qp[k0], c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Pp[k0 + 4], Qp[k0 + 4], c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(Pp[k0 + 8], Qp[k0 + 8], c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(Pp[k0 + 12], Qp[k0 + 12], c3, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      accd[r] += (static_cast<double>(c0[r]) + static_cast<double>(c1[r])) +
                 (static_cast<double>(c2[r]) + static_cast<double>(c3[r]));
  }
}

// Tile-local output coordinates of this lane's register r.
__device__ __forceinline__ int tile_row(int r) { return ((threadIdx.x >> 6) & 1) * 16 + 4 * ((threadIdx.x & 63) >> 4) + r; }
__device__ __forceinline__ int tile_col() { return (threadIdx.x >> 7) * 16 + (threadIdx.x & 15); }

__device__ __forceinline__ int pad16(int k) { return (k + 15) & ~15; }

__global__ __launch_bounds__(NT) void velocity2d_kernel(Phase2DArgs a) {
  extern __shared__ float lds[];
  float* P = lds;
  float* Q = lds + TILE * LDT;
  const int nx = a.nx, ny = a.ny;
  const int tux_n = (ny + TILE - 1) / TILE;
  const int n_ux = ((nx - 1 + TILE - 1) / TILE) * tux_n;
  const int t = blockIdx.x;
  double accd[4] = {0, 0, 0, 0};
  int i0, j0, rows, cols;
  int64_t ldy;
  float* Y;
  if (t < n_ux) {
    // u_x[i][j] += sum_k Gx[i][k] p[k][j]: P = Gx rows i, Q = p columns j
    i0 = (t / tux_n) * TILE;
    j0 = (t % tux_n) * TILE;
    stage_rows(P, a.Gx, a.ldgx, i0, nx - 1, nx, pad16(nx));
    stage_cols(Q, a.p, ny, j0, ny, nx, pad16(nx));
    lds_barrier();
    mma_tile(P, Q, pad16(nx), accd);
    Y = a.ux;
    ldy = ny;
    rows = nx - 1;
    cols = ny;
  } else {
    // u_y[i][j] += sum_k p[i][k] Gy[j][k]: P = p rows i, Q = Gy rows j
    const int tuy_n = (ny - 1 + TILE - 1) / TILE;
    const int tt = t - n_ux;
    i0 = (tt / tuy_n) * TILE;
    j0 = (tt % tuy_n) * TILE;
    stage_rows(P, a.p, ny, i0, nx, ny, pad16(ny));
    stage_rows(Q, a.Gy, a.ldgy, j0, ny - 1, ny, pad16(ny));
    lds_barrier();
    mma_tile(P, Q, pad16(ny), accd);
    Y = a.uy;
    ldy = ny - 1;
    rows = nx;
    cols = ny - 1;
  }
  // read all four outputs, then write them (one round trip)
  const int j = j0 + tile_col();
  float yv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + tile_row(r);
    yv[r] = (i < rows && j < cols) ? Y[static_cast<int64_t>(i) * ldy + j] : 0.f;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + tile_row(r);
    if (i < rows && j < cols)
      Y[static_cast<int64_t>(i) * ldy + j] = static_cast<float>(static_cast<double>(yv[r]) + accd[r]);
  }
}

__global__ __launch_bounds__(NT) void pressure2d_kernel(Phase2DArgs a) {
  extern __shared__ float lds[];
  float* P = lds;
  float* Q = lds + TILE * LDT;
  const int nx = a.nx, ny = a.ny;
  const int tp_n = (ny + TILE - 1) / TILE;
  const int i0 = (blockIdx.x / tp_n) * TILE, j0 = (blockIdx.x % tp_n) * TILE;
  double accd[4] = {0, 0, 0, 0};
  // p[i][j] += sum_k Dx[i][k] u_x[k][j]
  stage_rows(P, a.Dx, a.lddx, i0, nx, nx - 1, pad16(nx - 1));
  stage_cols(Q, a.ux, ny, j0, ny, nx - 1, pad16(nx - 1));
  lds_barrier();
  mma_tile(P, Q, pad16(nx - 1), accd);
  lds_barrier();
  // + sum_k u_y[i][k] Dy[j][k]
  stage_rows(P, a.uy, ny - 1, i0, nx, ny - 1, pad16(ny - 1));
  stage_rows(Q, a.Dy, a.lddy, j0, ny, ny - 1, pad16(ny - 1));
  lds_barrier();
  mma_tile(P, Q, pad16(ny - 1), accd);
  // read all four outputs (and map factors), then write them (one round trip)
  const int j = j0 + tile_col();
  float pv[4], cv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + tile_row(r);
    const bool ok = i < nx && j < ny;
    const int64_t idx = static_cast<int64_t>(i) * ny + j;
    pv[r] = ok ? a.p[idx] : 0.f;
    cv[r] = (ok && a.c2) ? a.c2[idx] : 1.f;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + tile_row(r);
    if (i < nx && j < ny)
      a.p[static_cast<int64_t>(i) * ny + j] =
          static_cast<float>(static_cast<double>(pv[r]) + accd[r] * static_cast<double>(cv[r]));
  }
}

constexpr size_t kLds = sizeof(float) * 2 * TILE * LDT;

hipError_t configure(const void* fn) {
  static int configured[2] = {-1, -1};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const int slot = fn == reinterpret_cast<const void*>(velocity2d_kernel) ? 0 : 1;
  if (configured[slot] == dev) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLds));
  if (e == hipSuccess) configured[slot] = dev;
  return e;
}

}  // namespace

bool phase2d_supported(int nx, int ny) { return nx >= 3 && ny >= 3 && nx <= KMAX && ny <= KMAX; }

hipError_t launch_phase2d_one(int which, const DevOperator& Gx, const DevOperator& Gy, const DevOperator& Dx,
                              const DevOperator& Dy, float* p, float* ux, float* uy, const float* c2, int nx, int ny,
                              hipStream_t s) {
  if (!phase2d_supported(nx, ny)) return hipErrorInvalidValue;
  hipError_t e = configure(reinterpret_cast<const void*>(velocity2d_kernel));
  if (e == hipSuccess) e = configure(reinterpret_cast<const void*>(pressure2d_kernel));
  if (e != hipSuccess) return e;
  Phase2DArgs a{static_cast<const float*>(Gx.data), Gx.Kp, static_cast<const float*>(Gy.data), Gy.Kp,
                static_cast<const float*>(Dx.data), Dx.Kp, static_cast<const float*>(Dy.data), Dy.Kp,
                p, ux, uy, c2, nx, ny};
  const int nA = ((nx - 1 + TILE - 1) / TILE) * ((ny + TILE - 1) / TILE) +
                 ((nx + TILE - 1) / TILE) * ((ny - 1 + TILE - 1) / TILE);
  const int nB = ((nx + TILE - 1) / TILE) * ((ny + TILE - 1) / TILE);
  if (which == 0) hipLaunchKernelGGL(velocity2d_kernel, dim3(nA), dim3(NT), kLds, s, a);
  else hipLaunchKernelGGL(pressure2d_kernel, dim3(nB), dim3(NT), kLds, s, a);
  return hipGetLastError();
}

hipError_t launch_phase2d(const DevOperator& Gx, const DevOperator& Gy, const DevOperator& Dx, const DevOperator& Dy,
                          float* p, float* ux, float* uy, const float* c2, int nx, int ny, int64_t steps,
                          hipStream_t s) {
  if (!phase2d_supported(nx, ny)) return hipErrorInvalidValue;
  hipError_t e = configure(reinterpret_cast<const void*>(velocity2d_kernel));
  if (e == hipSuccess) e = configure(reinterpret_cast<const void*>(pressure2d_kernel));
  if (e != hipSuccess) return e;
  Phase2DArgs a{static_cast<const float*>(Gx.data), Gx.Kp, static_cast<const float*>(Gy.data), Gy.Kp,
                static_cast<const float*>(Dx.data), Dx.Kp, static_cast<const float*>(Dy.data), Dy.Kp,
                p, ux, uy, c2, nx, ny};
  const int nA = ((nx - 1 + TILE - 1) / TILE) * ((ny + TILE - 1) / TILE) +
                 ((nx + TILE - 1) / TILE) * ((ny - 1 + TILE - 1) / TILE);
  const int nB = ((nx + TILE - 1) / TILE) * ((ny + TILE - 1) / TILE);
  for (int64_t t = 0; t < steps; ++t) {
    hipLaunchKernelGGL(velocity2d_kernel, dim3(nA), dim3(NT), kLds, s, a);
    hipLaunchKernelGGL(pressure2d_kernel, dim3(nB), dim3(NT), kLds, s, a);
  }
  return hipGetLastError();
}

}  // namespace pstd
