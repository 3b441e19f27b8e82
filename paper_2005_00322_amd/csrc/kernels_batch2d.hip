// Batched 2D solver: many independent 2D boxes of different sizes stepped by one persistent launch.
//
// Every solve advances with Eq. (dtt_pstd_solution) in its 2D form (§4.3).  One launch of at most as many
// blocks as the GPU holds at once runs all the steps: each step is a velocity phase over the velocity
// tiles of every solve, a grid-wide barrier, a pressure phase over the pressure tiles of every solve
// (each p tile takes both axes' terms), and a second barrier.  Within a phase blocks take tiles from a
// per-phase atomic ticket, largest tiles first, so the uneven sizes balance; the tickets are kept per
// XCD, each XCD's queue holding whole solves so their data stays in that XCD's L2.  Output tiles are 32 x 32
// (FP32 MFMA 16x16x4) or 64 x 64 (FP32 MFMA 32x32x2), chosen per batch by the autotuner.  The grid barrier is an
// arrival counter per (step, phase) with agent-scope release/acquire ordering (the L2 of every XCD is
// written back and invalidated around it); it gives up after a bounded wait and flags the launch, so a
// launch whose blocks were not all resident ends instead of hanging.  An ordinary launch, it can be
// captured in a HIP graph with the kernel that zeroes the counters.
//
// Operators are unscaled (dx = 1) FP32 matrices shared by all solves with the same (n, boundary pair);
// each solve's constants -dt/(rho0 dx) and -dt rho0 c0^2/dx are applied in the FP64 epilogue.  A tile is
// 32 x 32 outputs; its K extent is streamed through LDS in slices of 32 with a double buffer and a
// register prefetch; each wave computes a 16 x 16 quarter with MFMA 16x16x4 FP32, four independent
// chains per slice whose sums are flushed into FP64 registers.
//
// MFMA v_mfma_f32_16x16x4: lane l supplies P[l%16][l/16] and Q[l%16][l/16] (both staged as [row][k])
// and receives C[4*(l/16)+r][l%16] in register r.
#include "common.h"

namespace pstd {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t rsrc_t;

constexpr int BK = 32;
constexpr int LDB = BK + 1;      // LDS row stride (floats)
constexpr int NT = 256;
constexpr uint32_t kOOB = 0x80000000u;
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Every descriptor here is the same for the whole wave (it comes from the task of the block); passing
// base and size through readfirstlane keeps it in scalar registers, where a buffer access needs it,
// instead of a per-lane loop over distinct descriptors.
__device__ __forceinline__ rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(a >> 32));
  void* u = reinterpret_cast<void*>((static_cast<uint64_t>(hi) << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(u, 0, static_cast<int>(__builtin_amdgcn_readfirstlane(bytes)), 0x00020000);
}
__device__ __forceinline__ float ld_f32(rsrc_t r, uint32_t voff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
}

// Stage one BK slice of a TILE-row tile operand into LDS [row][k].  KIND:
//   0 operator rows: A[(r0 + r) * lda + k], zero padded on the host to its allocated rows and stride
//   1 field rows (contiguous):  X[(r0 + r) * ldx + k] for r0 + r < rows, k < K
//   2 field columns (strided):  X[k * ldx + c0 + c]   for c0 + c < cols, k < K   (transposed into [c][k])
// Every access is a buffer load whose out-of-range offset reads zero, so a thread issues the same loads
// for every slice (past the last one too) and the compiler can count them exactly.  A thread holds
// V = TILE/8 values of a slice between its load and its LDS store.
template <int TILE, int KIND>
struct Stager {
  static constexpr int V = TILE / 8;
  rsrc_t rs;
  int ld, r0, lim, K;

  __device__ void load(int k0, float (&v)[V]) const {
    const int t = threadIdx.x;
    if (KIND == 0) {
#pragma unroll
      for (int h = 0; h < V / 4; ++h) {
        const int r = (t >> 3) + 32 * h, kk = (t & 7) * 4;
        const f32x4 x = __builtin_bit_cast(
            f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, 4u * static_cast<uint32_t>((r0 + r) * ld + k0 + kk), 0, 0));
        v[4 * h] = x[0]; v[4 * h + 1] = x[1]; v[4 * h + 2] = x[2]; v[4 * h + 3] = x[3];
      }
    } else if (KIND == 1) {
#pragma unroll
      for (int h = 0; h < V / 4; ++h) {
        const int r = (t >> 3) + 32 * h, kk = (t & 7) * 4;
        const bool rv = r0 + r < lim;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = k0 + kk + j;
          v[4 * h + j] = ld_f32(rs, (rv && k < K) ? 4u * static_cast<uint32_t>((r0 + r) * ld + k) : kOOB);
        }
      }
    } else {
      const int k = t >> 3, c = (t & 7) * V;
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const bool ok = r0 + c + j < lim && k0 + k < K;
        v[j] = ld_f32(rs, ok ? 4u * static_cast<uint32_t>((k0 + k) * ld + r0 + c + j) : kOOB);
      }
    }
  }
  __device__ void store(float* lds, const float (&v)[V]) const {
    const int t = threadIdx.x;
    if (KIND == 2) {
      const int k = t >> 3, c = (t & 7) * V;
#pragma unroll
      for (int j = 0; j < V; ++j) lds[(c + j) * LDB + k] = v[j];
    } else {
#pragma unroll
      for (int h = 0; h < V / 4; ++h) {
        const int r = (t >> 3) + 32 * h, kk = (t & 7) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) lds[r * LDB + kk + j] = v[4 * h + j];
      }
    }
  }
};

// FP32 MFMA per slice into FP32 partial sums, which flush() adds into the FP64 accumulators every
// kFlush slices (64 terms of k): TILE 32 = four waves of 16 x 16 (v_mfma_f32_16x16x4f32, four chains);
// TILE 64 = four waves of 32 x 32 (v_mfma_f32_32x32x2f32, two chains).
constexpr int kFlush = 2;
template <int TILE>
struct Acc;
template <>
struct Acc<32> {
  static constexpr int R = 4;
  struct Part {
    f32x4 c0, c1, c2, c3;
  };
  __device__ static void zero(Part& p) {
    p.c0 = p.c1 = p.c2 = p.c3 = f32x4{0, 0, 0, 0};
  }
  __device__ static void slice(const float* Pl, const float* Ql, Part& p) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kl = lane >> 4;
    const float* Pp = Pl + ((wave & 1) * 16 + (lane & 15)) * LDB + kl;
    const float* Qp = Ql + ((wave >> 1) * 16 + (lane & 15)) * LDB + kl;
#pragma unroll
    for (int k = 0; k < BK; k += 16) {
      p.c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(Pp[k], Qp[k], p.c0, 0, 0, 0);
      p.c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(Pp[k + 4], Qp[k + 4], p.c1, 0, 0, 0);
      p.c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(Pp[k + 8], Qp[k + 8], p.c2, 0, 0, 0);
      p.c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(Pp[k + 12], Qp[k + 12], p.c3, 0, 0, 0);
    }
  }
  __device__ static void flush(Part& p, double (&accd)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      accd[r] += (static_cast<double>(p.c0[r]) + static_cast<double>(p.c1[r])) +
                 (static_cast<double>(p.c2[r]) + static_cast<double>(p.c3[r]));
    zero(p);
  }
  // tile-local output coordinates of register r (lane l receives C[4 (l/16) + r][l%16])
  __device__ static int row(int r) { return ((threadIdx.x >> 6) & 1) * 16 + 4 * ((threadIdx.x & 63) >> 4) + r; }
  __device__ static int col() { return (threadIdx.x >> 7) * 16 + (threadIdx.x & 15); }
};
template <>
struct Acc<64> {
  static constexpr int R = 16;
  struct Part {
    f32x16 c0, c1;
  };
  __device__ static void zero(Part& p) {
#pragma unroll
    for (int r = 0; r < 16; ++r) p.c0[r] = p.c1[r] = 0.f;
  }
  __device__ static void slice(const float* Pl, const float* Ql, Part& p) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kl = lane >> 5;
    // lane l supplies P[l%32][k + l/32] and Q[l%32][k + l/32]
    const float* Pp = Pl + ((wave & 1) * 32 + (lane & 31)) * LDB + kl;
    const float* Qp = Ql + ((wave >> 1) * 32 + (lane & 31)) * LDB + kl;
#pragma unroll
    for (int k = 0; k < BK; k += 4) {
      p.c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(Pp[k], Qp[k], p.c0, 0, 0, 0);
      p.c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(Pp[k + 2], Qp[k + 2], p.c1, 0, 0, 0);
    }
  }
  __device__ static void flush(Part& p, double (&accd)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) accd[r] += static_cast<double>(p.c0[r]) + static_cast<double>(p.c1[r]);
    zero(p);
  }
  // lane l receives C[8 (r/4) + 4 (l/32) + r%4][l%32]
  __device__ static int row(int r) {
    return ((threadIdx.x >> 6) & 1) * 32 + 8 * (r >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (r & 3);
  }
  __device__ static int col() { return (threadIdx.x >> 7) * 32 + (threadIdx.x & 31); }
};

// accd += P . Q^T over K (zero filled to a multiple of BK), P and Q described by their stagers.  Two LDS
// buffers and a ring of D register sets: while slice t is multiplied out of one buffer, slice t+1 is
// stored into the other and the loads of slice t+D are issued into the set slice t came from, so a
// slice's loads have D-1 slices of MFMA work to arrive.  The loop is unrolled by D so every set and
// buffer index is a constant; a tile whose slice count is not a multiple of D runs up to D-1 steps
// without MFMA work at its end.
template <int TILE, int PK, int QK>
__device__ __forceinline__ void tile_contract(const Stager<TILE, PK>& P, const Stager<TILE, QK>& Q, int K, float* lds,
                                              double (&accd)[Acc<TILE>::R]) {
  constexpr int V = TILE / 8, D = 4;
  static_assert(D % kFlush == 0, "the partial sums are flushed within each unrolled group");
  typename Acc<TILE>::Part part;
  Acc<TILE>::zero(part);
  float* Pl[2] = {lds, lds + 2 * TILE * LDB};
  float* Ql[2] = {lds + TILE * LDB, lds + 3 * TILE * LDB};
  const int nsl = (K + BK - 1) / BK;
  float rp[D][V], rq[D][V];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    P.load(i * BK, rp[i]);
    Q.load(i * BK, rq[i]);
  }
  lds_barrier();  // the previous user of the LDS buffers is done
  P.store(Pl[0], rp[0]);
  Q.store(Ql[0], rq[0]);
  lds_barrier();
  // Only the MFMA work is conditional: the stores and loads run in every step (past the last slice they
  // move zeros or unused values into the buffer that is not read), so each load stays where it is issued
  // instead of being sunk into a conditional block next to its store.
  for (int s0 = 0; s0 < nsl; s0 += D) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const int t = s0 + i;   // wave-uniform
      if (t < nsl) Acc<TILE>::slice(Pl[i & 1], Ql[i & 1], part);
      if (i % kFlush == kFlush - 1) Acc<TILE>::flush(part, accd);
      P.store(Pl[(i + 1) & 1], rp[(i + 1) % D]);
      Q.store(Ql[(i + 1) & 1], rq[(i + 1) % D]);
      P.load((t + D) * BK, rp[i]);
      Q.load((t + D) * BK, rq[i]);
      lds_barrier();
    }
  }
}

template <int TILE>
__device__ void run_task(const BatchSolve& S, const BatchTask& T, float* lds) {
  constexpr int R = Acc<TILE>::R;
  double accd[R];
#pragma unroll
  for (int r = 0; r < R; ++r) accd[r] = 0.0;
  const int nx = S.nx, ny = S.ny;
  float* Y;
  int rows, cols;
  double scale;
  if (T.kind == 0) {
    // u_x[i][j] += sG * sum_k Gx[i][k] p[k][j]
    const Stager<TILE, 0> P{make_rsrc(S.Gx, 4u * S.mgx * S.ldgx), S.ldgx, T.i0, nx - 1, nx};
    const Stager<TILE, 2> Q{make_rsrc(S.p, 4u * nx * ny), ny, T.j0, ny, nx};
    tile_contract<TILE>(P, Q, nx, lds, accd);
    Y = S.ux; rows = nx - 1; cols = ny; scale = S.sG;
  } else if (T.kind == 1) {
    // u_y[i][j] += sG_y * sum_k p[i][k] Gy[j][k]
    const Stager<TILE, 1> P{make_rsrc(S.p, 4u * nx * ny), ny, T.i0, nx, ny};
    const Stager<TILE, 0> Q{make_rsrc(S.Gy, 4u * S.mgy * S.ldgy), S.ldgy, T.j0, ny - 1, ny};
    tile_contract<TILE>(P, Q, ny, lds, accd);
    Y = S.uy; rows = nx; cols = ny - 1; scale = S.sG;
  } else {
    // p[i][j] += sD * (sum_k Dx[i][k] u_x[k][j] + sum_k u_y[i][k] Dy[j][k])
    const Stager<TILE, 0> P{make_rsrc(S.Dx, 4u * S.mdx * S.lddx), S.lddx, T.i0, nx, nx - 1};
    const Stager<TILE, 2> Q{make_rsrc(S.ux, 4u * (nx - 1) * ny), ny, T.j0, ny, nx - 1};
    tile_contract<TILE>(P, Q, nx - 1, lds, accd);
    const Stager<TILE, 1> P2{make_rsrc(S.uy, 4u * nx * (ny - 1)), ny - 1, T.i0, nx, ny - 1};
    const Stager<TILE, 0> Q2{make_rsrc(S.Dy, 4u * S.mdy * S.lddy), S.lddy, T.j0, ny, ny - 1};
    tile_contract<TILE>(P2, Q2, ny - 1, lds, accd);
    Y = S.p; rows = nx; cols = ny; scale = S.sD;
  }
  const int j = T.j0 + Acc<TILE>::col();
  // pressure tiles of a heterogeneous solve take c0(x)^2 pointwise
  const float* c2 = T.kind == 2 ? S.c2 : nullptr;
  float yv[R], cv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = T.i0 + Acc<TILE>::row(r);
    const bool ok = i < rows && j < cols;
    yv[r] = ok ? Y[static_cast<int64_t>(i) * cols + j] : 0.f;
    cv[r] = (ok && c2) ? c2[static_cast<int64_t>(i) * cols + j] : 1.f;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = T.i0 + Acc<TILE>::row(r);
    if (i < rows && j < cols)
      Y[static_cast<int64_t>(i) * cols + j] =
          static_cast<float>(static_cast<double>(yv[r]) + scale * static_cast<double>(cv[r]) * accd[r]);
  }
}

// All blocks of the grid meet here.  Bounded wait: about 2^22 polls (well over a second) before the
// launch is flagged and the block moves on.
__device__ void grid_barrier(unsigned* arrivals, unsigned* timeout) {
  __syncthreads();   // the block's stores are complete
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(arrivals, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned polls = 0;
    // relaxed polls (they read the counter past the caches without invalidating them), one acquire after
    while (__hip_atomic_load(arrivals, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x) {
      __builtin_amdgcn_s_sleep(4);
      if (++polls > (1u << 22)) {
        __hip_atomic_store(timeout, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

template <int TILE>
__global__ __launch_bounds__(NT, 2) void batch2d_kernel(BatchArgs a) {
  __shared__ float lds[4 * TILE * LDB];
  const int home = blockIdx.x % kBatchQueues;
  for (int64_t s = 0; s < a.steps; ++s) {
    unsigned* cs = a.counters + kBatchCountersPerStep * s;
    for (int phase = 0; phase < 2; ++phase) {
      const BatchTask* tasks = phase == 0 ? a.tasksA : a.tasksB;
      const int* seg = phase == 0 ? a.segA : a.segB;
      __shared__ int t_shared;
      // the home queue first, then the others in turn
      for (int qi = 0; qi < kBatchQueues; ++qi) {
        const int q = (home + qi) % kBatchQueues;
        const int beg = __builtin_amdgcn_readfirstlane(seg[q]);
        const int len = __builtin_amdgcn_readfirstlane(seg[q + 1]) - beg;
        unsigned* ctr = cs + phase * kBatchQueues + q;
        for (;;) {
          if (threadIdx.x == 0) t_shared = static_cast<int>(atomicAdd(ctr, 1u));
          lds_barrier();
          // uniform by construction; readfirstlane lets the compiler keep the task, the solve and the
          // buffer descriptors built from them in scalar registers (no per-lane descriptor loops)
          const int t = __builtin_amdgcn_readfirstlane(t_shared);
          lds_barrier();
          if (t >= len) break;
          const BatchTask L = tasks[beg + t];
          const BatchTask T{__builtin_amdgcn_readfirstlane(L.solve), __builtin_amdgcn_readfirstlane(L.kind),
                            __builtin_amdgcn_readfirstlane(L.i0), __builtin_amdgcn_readfirstlane(L.j0)};
          run_task<TILE>(a.solves[T.solve], T, lds);
        }
      }
      grid_barrier(cs + 2 * kBatchQueues + phase, a.timeout);
    }
  }
}

__global__ void zero_u32(unsigned* p, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

}  // namespace

int batch2d_max_blocks(int tile, int* out) {
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  const hipError_t e = tile == 64 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch2d_kernel<64>, NT, 0)
                                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch2d_kernel<32>, NT, 0);
  if (e != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  *out = per_cu * cus;
  return 0;
}

hipError_t launch_batch2d(const BatchArgs& a, int tile, int blocks, hipStream_t s) {
  // fresh tickets and barrier counters for every launch (a fill kernel, not a memset, so the pair of
  // launches can be captured in a graph)
  hipLaunchKernelGGL(zero_u32, dim3(64), dim3(256), 0, s, a.counters, kBatchCountersPerStep * a.steps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (tile == 64) hipLaunchKernelGGL(batch2d_kernel<64>, dim3(blocks), dim3(NT), 0, s, a);
  else hipLaunchKernelGGL(batch2d_kernel<32>, dim3(blocks), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace pstd
