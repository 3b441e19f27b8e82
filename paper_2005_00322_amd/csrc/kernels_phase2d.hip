// Two fused phase kernels per step for 2D FP32 plans with at most 512 nodes per axis.
//
// Eq. (dtt_pstd_solution) in its 2D form (§4.3) splits into a velocity phase and a pressure phase:
//   velocity  u_x += G~x p   and   u_y += p G~y^T           (one launch)
//   pressure  p += c2 .* (D~x u_x + u_y D~y^T)               (one launch)
// Each block owns one 16 x 16 output tile of the phase: in the velocity phase the u_x and the u_y tile at
// the same (i, j) position, in the pressure phase one p tile with both axes' terms.  Both phases are thus
// two contractions of the same shape,
//   contraction 0:  out0[i][j] = sum_k A0[i][k] X0[k][j]   (operator rows, columns of a field)
//   contraction 1:  out1[i][j] = sum_k X1[i][k] A1[j][k]   (rows of a field, operator rows)
// and the eight waves of a block split them as (contraction, quarter of k).  A box of a few hundred nodes a
// side is bound by latency, not by bandwidth or MFMA rate, so a block issues every load it needs (four
// full-k operand slices and the old output values of its epilogue) before the first LDS store: one
// round trip to memory per phase.  Small tiles give enough blocks to spread the MFMA work over the
// whole GPU (256 blocks of eight waves for 256 x 256).  The kernel boundary between the phases is the grid-wide
// dependency of the scheme; graph replay keeps the launch gaps short.
//
// MFMA v_mfma_f32_16x16x4: lane l supplies P[l%16][kslot l/16] and Q[l%16][kslot l/16] and receives
// C[4*(l/16)+r][l%16] in register r.  A lane reads four consecutive k of each operand with one LDS
// read and feeds component e to the e-th of four independent MFMAs, so MFMA e contracts the k set
// {k0 + 4s + e}; the four together cover k0 .. k0+15 once.  FP32 chain sums are flushed into FP64
// registers every 32 k, the halves and contractions are added in FP64, and the update is rounded once.
#include <algorithm>

#include "common.h"

namespace pstd {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;

constexpr int T = 16;                   // output tile edge
constexpr int NT = 512;                 // eight waves
constexpr uint32_t kOOB = 0x80000000u;  // buffer offset past every range: the load returns zero

// mx, my: staggered points along x and y, n - 1 between two walls and n on a periodic axis
struct Phase2DArgs {
  const float* Gx; int ldgx, mgx;   // mx x nx operator, row stride ldgx, mgx rows allocated (zero padded)
  const float* Gy; int ldgy, mgy;   // my x ny
  const float* Dx; int lddx, mdx;   // nx x mx
  const float* Dy; int lddy, mdy;   // ny x my
  float* p;                         // nx x ny
  float* ux;                        // mx x ny
  float* uy;                        // nx x my
  const float* c2;                  // nx x ny or null
  int nx, ny, mx, my;
  double sv, sp;                    // velocity / pressure factors on the contractions (1 for folded operators)
};

__device__ __forceinline__ rsrc_t make_rsrc(const void* ptr, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(ptr), 0, static_cast<int>(bytes), 0x00020000);
}
__device__ __forceinline__ float ld_f32(rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
}
__device__ __forceinline__ f32x4 ld_f32x4(rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0));
}

__host__ __device__ __forceinline__ int pad64(int k) { return (k + 63) & ~63; }

// One phase's operands in registers between the loads and the LDS stores (512 threads).
//   op0, op1: operator rows r0 .. r0+15, k < Kpad, thread t holds k = 4 (t%32) + 128 j of row t/32
//   col0:     X0[k][c0 + c], thread t holds c = t%16, k = t/16 + 32 u
//   row1:     X1[r0 + r][k], thread t holds r = t/64 + 8 q, k = t%64 + 64 j
template <int KMAX>
struct Slices {
  static constexpr int KC = KMAX / 64;
  f32x4 op0[KMAX / 128], op1[KMAX / 128];
  float col0[KMAX / 32];
  float row1[2 * KC];
};

template <int KMAX>
__device__ __forceinline__ void load_op(f32x4 (&v)[KMAX / 128], rsrc_t rs, int ld, int r0, int Kpad) {
  const int t = threadIdx.x;
  const uint32_t base = 4u * static_cast<uint32_t>((r0 + (t >> 5)) * ld + 4 * (t & 31));
#pragma unroll
  for (int j = 0; j < KMAX / 128; ++j)
    if (128 * j < Kpad) v[j] = ld_f32x4(rs, base + 512u * j);
}

template <int KMAX>
__device__ __forceinline__ void store_op(float* dst, const f32x4 (&v)[KMAX / 128], int Kpad) {
  constexpr int LD = KMAX + 4;
  const int t = threadIdx.x;
  float* d = dst + (t >> 5) * LD + 4 * (t & 31);
#pragma unroll
  for (int j = 0; j < KMAX / 128; ++j)
    if (128 * j < Kpad) *reinterpret_cast<f32x4*>(d + 128 * j) = v[j];
}

// columns c0 .. c0+15 of X (row stride ld; valid c < cols, k < K)
template <int KMAX>
__device__ __forceinline__ void load_cols(float (&v)[KMAX / 32], rsrc_t rs, int ld, int c0, int cols, int K, int Kpad) {
  const int t = threadIdx.x;
  const int c = c0 + (t & 15);
#pragma unroll
  for (int u = 0; u < KMAX / 32; ++u) {
    const int k = (t >> 4) + 32 * u;
    if (32 * u < Kpad) v[u] = ld_f32(rs, (c < cols && k < K) ? 4u * static_cast<uint32_t>(k * ld + c) : kOOB);
  }
}

template <int KMAX>
__device__ __forceinline__ void store_cols(float* dst, const float (&v)[KMAX / 32], int Kpad) {
  constexpr int LD = KMAX + 4;
  const int t = threadIdx.x;
  float* d = dst + (t & 15) * LD + (t >> 4);
#pragma unroll
  for (int u = 0; u < KMAX / 32; ++u)
    if (32 * u < Kpad) d[32 * u] = v[u];
}

// rows r0 .. r0+15 of X (row stride ld; valid r < rows, k < K)
template <int KMAX>
__device__ __forceinline__ void load_rows(float (&v)[2 * (KMAX / 64)], rsrc_t rs, int ld, int r0, int rows, int K,
                                          int Kpad) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = r0 + (t >> 6) + 8 * q;
#pragma unroll
    for (int j = 0; j < KMAX / 64; ++j) {
      const int k = (t & 63) + 64 * j;
      if (64 * j < Kpad)
        v[q * (KMAX / 64) + j] = ld_f32(rs, (r < rows && k < K) ? 4u * static_cast<uint32_t>(r * ld + k) : kOOB);
    }
  }
}

template <int KMAX>
__device__ __forceinline__ void store_rows(float* dst, const float (&v)[2 * (KMAX / 64)], int Kpad) {
  constexpr int LD = KMAX + 4;
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    float* d = dst + ((t >> 6) + 8 * q) * LD + (t & 63);
#pragma unroll
    for (int j = 0; j < KMAX / 64; ++j)
      if (64 * j < Kpad) d[64 * j] = v[q * (KMAX / 64) + j];
  }
}

// acc (this lane's four outputs of the 16 x 16 tile) += sum over k in [kb, ke) of P[row][k] Q[col][k];
// kb and ke multiples of 32.
template <int KMAX>
__device__ __forceinline__ void mma_range(const float* P, const float* Q, int kb, int ke, double (&acc)[4]) {
  constexpr int LD = KMAX + 4;
  const int lane = threadIdx.x & 63;
  const float* Pp = P + (lane & 15) * LD + 4 * (lane >> 4);
  const float* Qp = Q + (lane & 15) * LD + 4 * (lane >> 4);
  for (int k = kb; k < ke; k += 32) {
    const f32x4 a0 = *reinterpret_cast<const f32x4*>(Pp + k);
    const f32x4 b0 = *reinterpret_cast<const f32x4*>(Qp + k);
    const f32x4 a1 = *reinterpret_cast<const f32x4*>(Pp + k + 16);
    const f32x4 b1 = *reinterpret_cast<const f32x4*>(Qp + k + 16);
    const f32x4 z = {0, 0, 0, 0};
    f32x4 c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[0], b0[0], z, 0, 0, 0);
    f32x4 c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[1], b0[1], z, 0, 0, 0);
    f32x4 c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[2], b0[2], z, 0, 0, 0);
    f32x4 c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[3], b0[3], z, 0, 0, 0);
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[0], b1[0], c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[1], b1[1], c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[2], b1[2], c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[3], b1[3], c3, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      acc[r] += (static_cast<double>(c0[r]) + static_cast<double>(c1[r])) +
                (static_cast<double>(c2[r]) + static_cast<double>(c3[r]));
  }
}

template <int KMAX, bool ALIAS>
constexpr size_t lds_bytes() {
  return ALIAS ? std::max(sizeof(float) * 4 * T * (KMAX + 4), sizeof(double) * 8 * 4 * 64)
               : sizeof(float) * 4 * T * (KMAX + 4) + sizeof(double) * 8 * 4 * 64;
}

// PH 0: velocity phase, PH 1: pressure phase.
// ALIAS: the partial tiles reuse the operand slices' LDS once every wave has finished its products (one
// more barrier, less LDS: two blocks per CU where many blocks queue); otherwise they follow the slices.
template <int KMAX, int PH, bool ALIAS>
__device__ __forceinline__ void phase2d_body(const Phase2DArgs& a) {
  constexpr int SL = T * (KMAX + 4);
  extern __shared__ float lds[];
  double* red = reinterpret_cast<double*>(ALIAS ? lds : lds + 4 * SL);   // [wave][reg][lane], eight waves
  const int nx = a.nx, ny = a.ny, mx = a.mx, my = a.my;
  const int tiles_y = (ny + T - 1) / T;
  const int nb = gridDim.x;
  int b = blockIdx.x;
  if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);   // consecutive tiles on one XCD
  const int i0 = (b / tiles_y) * T, j0 = (b % tiles_y) * T;
  // the wave index through readfirstlane keeps per-wave buffer descriptors in scalar registers
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);

  // the two contractions of this phase
  const float* A0 = PH == 0 ? a.Gx : a.Dx;
  const int lda0 = PH == 0 ? a.ldgx : a.lddx, ma0 = PH == 0 ? a.mgx : a.mdx;
  const float* A1 = PH == 0 ? a.Gy : a.Dy;
  const int lda1 = PH == 0 ? a.ldgy : a.lddy, ma1 = PH == 0 ? a.mgy : a.mdy;
  const float* X0 = PH == 0 ? a.p : a.ux;                   // ld ny, K0 rows
  const float* X1 = PH == 0 ? a.p : a.uy;                   // nx rows of K1
  const int K0 = PH == 0 ? nx : mx, K1 = PH == 0 ? ny : my;
  const int ld1 = PH == 0 ? ny : my;
  const int Kp0 = pad64(K0), Kp1 = pad64(K1);

  const rsrc_t rA0 = make_rsrc(A0, 4u * static_cast<uint32_t>(ma0 * lda0));
  const rsrc_t rA1 = make_rsrc(A1, 4u * static_cast<uint32_t>(ma1 * lda1));
  const rsrc_t rX0 = make_rsrc(X0, 4u * static_cast<uint32_t>(K0 * ny));
  const rsrc_t rX1 = make_rsrc(X1, 4u * static_cast<uint32_t>(nx * ld1));

  // old output value of this wave's share of the epilogue, loaded with the operands
  //   velocity: wave w finishes register w%4 of the u_x (w < 4) or u_y (w >= 4) tile
  //   pressure: wave w < 4 finishes register w of the p tile
  float old = 0.f, cfac = 1.f;
  const int oj = j0 + (lane & 15);
  if (PH == 0) {
    float* Y = wave < 4 ? a.ux : a.uy;
    const int rows = wave < 4 ? mx : nx, cols = wave < 4 ? ny : my;
    const rsrc_t rY = make_rsrc(Y, 4u * static_cast<uint32_t>(rows * cols));
    const int oi = i0 + 4 * (lane >> 4) + (wave & 3);
    old = ld_f32(rY, (oi < rows && oj < cols) ? 4u * static_cast<uint32_t>(oi * cols + oj) : kOOB);
  } else if (wave < 4) {
    const rsrc_t rP = make_rsrc(a.p, 4u * static_cast<uint32_t>(nx * ny));
    const int oi = i0 + 4 * (lane >> 4) + wave;
    const bool ok = oi < nx && oj < ny;
    old = ld_f32(rP, ok ? 4u * static_cast<uint32_t>(oi * ny + oj) : kOOB);
    if (a.c2) {
      const rsrc_t rC = make_rsrc(a.c2, 4u * static_cast<uint32_t>(nx * ny));
      cfac = ld_f32(rC, ok ? 4u * static_cast<uint32_t>(oi * ny + oj) : kOOB);
    }
  }

  Slices<KMAX> s;
  load_op<KMAX>(s.op0, rA0, lda0, i0, Kp0);
  load_cols<KMAX>(s.col0, rX0, ny, j0, ny, K0, Kp0);
  load_rows<KMAX>(s.row1, rX1, ld1, i0, nx, K1, Kp1);
  load_op<KMAX>(s.op1, rA1, lda1, j0, Kp1);
  float* S0 = lds;            // A0 rows       [i][k]
  float* S1 = lds + SL;       // X0 columns    [j][k]
  float* S2 = lds + 2 * SL;   // X1 rows       [i][k]
  float* S3 = lds + 3 * SL;   // A1 rows       [j][k]
  store_op<KMAX>(S0, s.op0, Kp0);
  store_cols<KMAX>(S1, s.col0, Kp0);
  store_rows<KMAX>(S2, s.row1, Kp1);
  store_op<KMAX>(S3, s.op1, Kp1);
  __syncthreads();

  double acc[4] = {0, 0, 0, 0};
  {
    // wave w: contraction w / 4, quarter w % 4 of its 32-wide k chunks
    const int c = wave >> 2, h = wave & 3;
    const int nch = (c == 0 ? Kp0 : Kp1) >> 5;
    mma_range<KMAX>(c == 0 ? S0 : S2, c == 0 ? S1 : S3, 32 * ((h * nch) >> 2), 32 * (((h + 1) * nch) >> 2), acc);
  }
  if (ALIAS) __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) red[(wave * 4 + r) * 64 + lane] = acc[r];
  __syncthreads();

  auto part = [&](int w, int r) { return red[(w * 4 + r) * 64 + lane]; };
  if (PH == 0) {
    const int c = wave >> 2, r = wave & 3;
    float* Y = c == 0 ? a.ux : a.uy;
    const int rows = c == 0 ? mx : nx, cols = c == 0 ? ny : my;
    const double v = (part(4 * c, r) + part(4 * c + 1, r)) + (part(4 * c + 2, r) + part(4 * c + 3, r));
    const int oi = i0 + 4 * (lane >> 4) + r;
    if (oi < rows && oj < cols)
      Y[static_cast<int64_t>(oi) * cols + oj] = static_cast<float>(static_cast<double>(old) + a.sv * v);
  } else if (wave < 4) {
    const int r = wave;
    const double v = ((part(0, r) + part(1, r)) + (part(2, r) + part(3, r))) +
                     ((part(4, r) + part(5, r)) + (part(6, r) + part(7, r)));
    const int oi = i0 + 4 * (lane >> 4) + r;
    if (oi < nx && oj < ny)
      a.p[static_cast<int64_t>(oi) * ny + oj] =
          static_cast<float>(static_cast<double>(old) + a.sp * v * static_cast<double>(cfac));
  }
}

template <int KMAX, int PH>
__global__ __launch_bounds__(NT) void phase2d_kernel(Phase2DArgs a) {
  phase2d_body<KMAX, PH, false>(a);
}

// One phase of many solves of one shape: block (tile, solve), the solve's unscaled operators and
// factors from the batch's solve table.
template <int KMAX, int PH>
__global__ __launch_bounds__(NT) void phase2d_batch_kernel(const BatchSolve* __restrict__ solves) {
  const BatchSolve& S = solves[blockIdx.y];
  const Phase2DArgs a{S.Gx, S.ldgx, S.mgx, S.Gy, S.ldgy, S.mgy, S.Dx, S.lddx, S.mdx, S.Dy, S.lddy, S.mdy,
                      S.p, S.ux, S.uy, S.c2, S.nx, S.ny, S.nx - 1, S.ny - 1, S.sG, S.sD};
  phase2d_body<KMAX, PH, true>(a);
}

// the dynamic LDS size above 64 KB is an attribute of each kernel instance, set once per device
template <typename F>
hipError_t configure(F* fn, size_t lds, int* configured) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (*configured == dev) return hipSuccess;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                          static_cast<int>(lds));
  if (e == hipSuccess) *configured = dev;
  return e;
}

template <int KMAX>
hipError_t launch_one(int which, const Phase2DArgs& a, hipStream_t s) {
  static int conf[2] = {-1, -1};
  const int nb = ((a.nx + T - 1) / T) * ((a.ny + T - 1) / T);
  constexpr size_t lds = lds_bytes<KMAX, false>();
  hipError_t e = which == 0 ? configure(phase2d_kernel<KMAX, 0>, lds, &conf[0])
                            : configure(phase2d_kernel<KMAX, 1>, lds, &conf[1]);
  if (e != hipSuccess) return e;
  if (which == 0) hipLaunchKernelGGL((phase2d_kernel<KMAX, 0>), dim3(nb), dim3(NT), lds, s, a);
  else hipLaunchKernelGGL((phase2d_kernel<KMAX, 1>), dim3(nb), dim3(NT), lds, s, a);
  return hipGetLastError();
}

template <int KMAX>
hipError_t launch_batch(int which, const BatchSolve* solves, int count, int nx, int ny, hipStream_t s) {
  static int conf[2] = {-1, -1};
  const int nb = ((nx + T - 1) / T) * ((ny + T - 1) / T);
  constexpr size_t lds = lds_bytes<KMAX, true>();
  hipError_t e = which == 0 ? configure(phase2d_batch_kernel<KMAX, 0>, lds, &conf[0])
                            : configure(phase2d_batch_kernel<KMAX, 1>, lds, &conf[1]);
  if (e != hipSuccess) return e;
  if (which == 0) hipLaunchKernelGGL((phase2d_batch_kernel<KMAX, 0>), dim3(nb, count), dim3(NT), lds, s, solves);
  else hipLaunchKernelGGL((phase2d_batch_kernel<KMAX, 1>), dim3(nb, count), dim3(NT), lds, s, solves);
  return hipGetLastError();
}

Phase2DArgs make_args(const DevOperator& Gx, const DevOperator& Gy, const DevOperator& Dx, const DevOperator& Dy,
                      float* p, float* ux, float* uy, const float* c2, int nx, int ny) {
  return Phase2DArgs{static_cast<const float*>(Gx.data), Gx.Kp, Gx.Mp, static_cast<const float*>(Gy.data), Gy.Kp,
                     Gy.Mp, static_cast<const float*>(Dx.data), Dx.Kp, Dx.Mp, static_cast<const float*>(Dy.data), Dy.Kp,
                     Dy.Mp, p, ux, uy, c2, nx, ny, Gx.M, Gy.M, 1.0, 1.0};
}

// The operator slices are read as 16-byte rows of the zero-padded device matrices: every k < pad64(K)
// lies inside a row, and rows past the allocation read as zero.  The staggered extent of an axis (the
// rows of G, the columns of D) is n - 1 between walls or n on a periodic axis.
bool operators_fit(const DevOperator& Gx, const DevOperator& Gy, const DevOperator& Dx, const DevOperator& Dy,
                   int nx, int ny) {
  const int mx = Gx.M, my = Gy.M;
  return Gx.K == nx && Gy.K == ny && Dx.M == nx && Dy.M == ny && Dx.K == mx && Dy.K == my &&
         (mx == nx - 1 || mx == nx) && (my == ny - 1 || my == ny) && Gx.Kp >= pad64(nx) && Gy.Kp >= pad64(ny) &&
         Dx.Kp >= pad64(mx) && Dy.Kp >= pad64(my) && Gx.Kp % 4 == 0 && Gy.Kp % 4 == 0 && Dx.Kp % 4 == 0 &&
         Dy.Kp % 4 == 0;
}

}  // namespace

bool phase2d_supported(int nx, int ny) { return nx >= 3 && ny >= 3 && nx <= 512 && ny <= 512; }

hipError_t launch_phase2d_one(int which, const DevOperator& Gx, const DevOperator& Gy, const DevOperator& Dx,
                              const DevOperator& Dy, float* p, float* ux, float* uy, const float* c2, int nx, int ny,
                              hipStream_t s) {
  if (!phase2d_supported(nx, ny) || !operators_fit(Gx, Gy, Dx, Dy, nx, ny)) return hipErrorInvalidValue;
  const Phase2DArgs a = make_args(Gx, Gy, Dx, Dy, p, ux, uy, c2, nx, ny);
  return (nx <= 256 && ny <= 256) ? launch_one<256>(which, a, s) : launch_one<512>(which, a, s);
}

hipError_t launch_phase2d(const DevOperator& Gx, const DevOperator& Gy, const DevOperator& Dx, const DevOperator& Dy,
                          float* p, float* ux, float* uy, const float* c2, int nx, int ny, int64_t steps,
                          hipStream_t s) {
  if (!phase2d_supported(nx, ny) || !operators_fit(Gx, Gy, Dx, Dy, nx, ny)) return hipErrorInvalidValue;
  const Phase2DArgs a = make_args(Gx, Gy, Dx, Dy, p, ux, uy, c2, nx, ny);
  const bool small = nx <= 256 && ny <= 256;
  for (int64_t t = 0; t < steps; ++t) {
    hipError_t e = small ? launch_one<256>(0, a, s) : launch_one<512>(0, a, s);
    if (e == hipSuccess) e = small ? launch_one<256>(1, a, s) : launch_one<512>(1, a, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One phase of `count` solves of one shape from the batch's device solve table (unscaled operators; the
// factors sG, sD and the c0^2 maps of the table apply in the epilogue).  The caller checks that the
// operators' padded rows cover pad64(K) columns (batch2d_phase_fits).
hipError_t launch_phase2d_batch(int which, const BatchSolve* solves, int count, int nx, int ny, hipStream_t s) {
  if (!phase2d_supported(nx, ny) || count < 1 || count > 65535) return hipErrorInvalidValue;
  return (nx <= 256 && ny <= 256) ? launch_batch<256>(which, solves, count, nx, ny, s)
                                  : launch_batch<512>(which, solves, count, nx, ny, s);
}

bool batch2d_phase_fits(int ldgx, int ldgy, int lddx, int lddy, int nx, int ny) {
  return ldgx >= pad64(nx) && ldgy >= pad64(ny) && lddx >= pad64(nx - 1) && lddy >= pad64(ny - 1) && ldgx % 4 == 0 &&
         ldgy % 4 == 0 && lddx % 4 == 0 && lddy % 4 == 0;
}

}  // namespace pstd
