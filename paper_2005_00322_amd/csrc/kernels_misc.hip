// Single-workgroup 1D stepper, wall handling, the reflection-coefficient combination and checks.
#include "common.h"

namespace pstd {
namespace {

// Whole 1D time loop in one workgroup: p and u live in LDS for all steps, the operators (stored
// transposed, K x M with row stride ldt, so that consecutive lanes read consecutive rows' entries)
// stream from L2.  Each step is Eq. (dtt_pstd_solution): u += G~ p, then p += D~ u (scaled pointwise by
// c0(x)^2 when a sound-speed map is given).  Threads split every dot product 4 ways; the sums and the
// update are formed in FP64 for both state types and rounded once into the state.
template <typename T>
__global__ __launch_bounds__(1024) void step1d_kernel(const T* __restrict__ GT, int ldg, const T* __restrict__ DT,
                                                      int ldd, T* __restrict__ p, T* __restrict__ u, int n,
                                                      int64_t steps, const T* __restrict__ scale) {
  extern __shared__ unsigned char smem_raw[];
  T* sp = reinterpret_cast<T*>(smem_raw);
  T* su = sp + n;
  // 4 partial sums per row, 8-byte aligned after the two state vectors
  double* part = reinterpret_cast<double*>(smem_raw + ((2 * n * sizeof(T) + 7) & ~static_cast<size_t>(7)));
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  for (int i = tid; i < n; i += nt) sp[i] = p[i];
  for (int i = tid; i < n - 1; i += nt) su[i] = u[i];
  const int nm = n - 1;
  for (int64_t s = 0; s < steps; ++s) {
    __syncthreads();
    // u_i += sum_k G~[i][k] p_k, k split in 4 interleaved quarters
    for (int e = tid; e < 4 * nm; e += nt) {
      const int i = e % nm, q = e / nm;
      double acc = 0;
      for (int k = q; k < n; k += 4) acc += static_cast<double>(GT[static_cast<int64_t>(k) * ldg + i]) * sp[k];
      part[q * n + i] = acc;
    }
    __syncthreads();
    for (int i = tid; i < nm; i += nt)
      su[i] = static_cast<T>(su[i] + ((part[i] + part[n + i]) + (part[2 * n + i] + part[3 * n + i])));
    __syncthreads();
    // p_i += c(x_i) * sum_k D~[i][k] u_k
    for (int e = tid; e < 4 * n; e += nt) {
      const int i = e % n, q = e / n;
      double acc = 0;
      for (int k = q; k < nm; k += 4) acc += static_cast<double>(DT[static_cast<int64_t>(k) * ldd + i]) * su[k];
      part[q * n + i] = acc;
    }
    __syncthreads();
    for (int i = tid; i < n; i += nt) {
      double d = (part[i] + part[n + i]) + (part[2 * n + i] + part[3 * n + i]);
      if (scale) d *= static_cast<double>(scale[i]);
      sp[i] = static_cast<T>(sp[i] + d);
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += nt) p[i] = sp[i];
  for (int i = tid; i < n - 1; i += nt) u[i] = su[i];
}

// The same time loop for n <= 128 with both operators in registers for all steps: thread t owns row
// t / 8 of each operator and its 16 entries in columns 16 (t % 8) .. 16 (t % 8) + 15, so a step reads no
// global memory.  A row's eight partial dot products are added across its eight lanes (xor shuffles, a
// fixed order); the state vectors live in LDS.  Per step: u += G~ p, a barrier, p += D~ u (times c0(x)^2
// with a map), a barrier.  Sums and updates in FP64, rounded once into the state, as above.
template <typename T>
__global__ __launch_bounds__(1024) void step1d_reg_kernel(const T* __restrict__ G, int ldg, const T* __restrict__ D,
                                                          int ldd, T* __restrict__ p, T* __restrict__ u, int n,
                                                          int64_t steps, const T* __restrict__ scale) {
  __shared__ T sp[128], su[128];
  const int tid = threadIdx.x, i = tid >> 3, q = tid & 7;
  const int nm = n - 1;
  T g[16], d[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int k = 16 * q + j;
    g[j] = (i < nm && k < n) ? G[static_cast<int64_t>(i) * ldg + k] : T(0);
    d[j] = (i < n && k < nm) ? D[static_cast<int64_t>(i) * ldd + k] : T(0);
  }
  const double sc = (scale && i < n) ? static_cast<double>(scale[i]) : 1.0;
  if (tid < 128) {
    sp[tid] = tid < n ? p[tid] : T(0);
    su[tid] = tid < nm ? u[tid] : T(0);
  }
  __syncthreads();
  for (int64_t s = 0; s < steps; ++s) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) acc += static_cast<double>(g[j]) * static_cast<double>(sp[16 * q + j]);
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 4);
    if (q == 0 && i < nm) su[i] = static_cast<T>(su[i] + acc);
    __syncthreads();
    acc = 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) acc += static_cast<double>(d[j]) * static_cast<double>(su[16 * q + j]);
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 4);
    if (q == 0 && i < n) sp[i] = static_cast<T>(sp[i] + acc * sc);
    __syncthreads();
  }
  if (tid < n) p[tid] = sp[tid];
  if (tid < nm) u[tid] = su[tid];
}

template <typename T>
__global__ void zero_dirichlet_kernel(T* p, int ndim, int64_t n0, int64_t n1, int64_t n2, int lo0, int hi0, int lo1,
                                      int hi1, int lo2, int hi2) {
  const int64_t total = n0 * n1 * n2;
  for (int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t i2 = idx % n2;
    const int64_t i1 = (idx / n2) % n1;
    const int64_t i0 = idx / (n1 * n2);
    bool wall = (lo0 && i0 == 0) || (hi0 && i0 == n0 - 1);
    if (ndim > 1) wall = wall || (lo1 && i1 == 0) || (hi1 && i1 == n1 - 1);
    if (ndim > 2) wall = wall || (lo2 && i2 == 0) || (hi2 && i2 == n2 - 1);
    if (wall) p[idx] = T(0);
  }
}

template <typename T>
__global__ void fill_zero_kernel(T* x, int64_t count) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    x[i] = T(0);
}

template <typename T>
__global__ void square_kernel(const float* in, T* out, int64_t count) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const T v = static_cast<T>(in[i]);
    out[i] = v * v;
  }
}

constexpr int kMaxFields = 64;
struct CombineArgs {
  const float* f[kMaxFields];
  float w[kMaxFields];
  int nf;
};

// out = sum_i w_i f_i (§5), 4 elements per lane with a scalar tail.
__global__ __launch_bounds__(256) void combine_kernel(CombineArgs a, float* out, int64_t count) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t nvec = count / 4;
  bool aligned = (reinterpret_cast<uintptr_t>(out) & 15) == 0;
  for (int i = 0; i < a.nf; ++i) aligned = aligned && ((reinterpret_cast<uintptr_t>(a.f[i]) & 15) == 0);
  const int64_t start = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (aligned) {
    for (int64_t v = start; v < nvec; v += stride) {
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int i = 0; i < a.nf; ++i) {
        const float4 x = reinterpret_cast<const float4*>(a.f[i])[v];
        acc.x += a.w[i] * x.x;
        acc.y += a.w[i] * x.y;
        acc.z += a.w[i] * x.z;
        acc.w += a.w[i] * x.w;
      }
      reinterpret_cast<float4*>(out)[v] = acc;
    }
    for (int64_t e = 4 * nvec + start; e < count; e += stride) {
      float acc = 0.f;
      for (int i = 0; i < a.nf; ++i) acc += a.w[i] * a.f[i][e];
      out[e] = acc;
    }
  } else {
    for (int64_t e = start; e < count; e += stride) {
      float acc = 0.f;
      for (int i = 0; i < a.nf; ++i) acc += a.w[i] * a.f[i][e];
      out[e] = acc;
    }
  }
}

template <typename T>
__global__ void nonfinite_kernel(const T* x, int64_t count, int* flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const T v = x[i];
    bad = bad || !(v - v == T(0));
  }
  if (bad) atomicOr(flag, 1);
}

unsigned blocks_for(int64_t count, int threads) {
  int64_t b = (count + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return static_cast<unsigned>(b);
}

}  // namespace

hipError_t launch_step1d(int prec, const DevOperator& G, const DevOperator& D, void* p, void* u, int n,
                         int64_t steps, const void* scale, hipStream_t s) {
  if (n <= 128) {
    if (prec == PSTD_FP64)
      hipLaunchKernelGGL(step1d_reg_kernel<double>, dim3(1), dim3(1024), 0, s, static_cast<const double*>(G.data),
                         G.Kp, static_cast<const double*>(D.data), D.Kp, static_cast<double*>(p),
                         static_cast<double*>(u), n, steps, static_cast<const double*>(scale));
    else
      hipLaunchKernelGGL(step1d_reg_kernel<float>, dim3(1), dim3(1024), 0, s, static_cast<const float*>(G.data),
                         G.Kp, static_cast<const float*>(D.data), D.Kp, static_cast<float*>(p),
                         static_cast<float*>(u), n, steps, static_cast<const float*>(scale));
    return hipGetLastError();
  }
  const size_t esz = prec == PSTD_FP64 ? 8 : 4;
  const size_t shmem = ((esz * 2 * static_cast<size_t>(n) + 7) & ~static_cast<size_t>(7)) + 8 * static_cast<size_t>(4) * n;
  if (shmem > 64 * 1024) return hipErrorInvalidConfiguration;
  int threads = 4 * n;
  threads = threads > 1024 ? 1024 : ((threads + 63) / 64) * 64;
  if (prec == PSTD_FP64)
    hipLaunchKernelGGL(step1d_kernel<double>, dim3(1), dim3(threads), shmem, s, static_cast<const double*>(G.dataT),
                       G.Mp, static_cast<const double*>(D.dataT), D.Mp, static_cast<double*>(p),
                       static_cast<double*>(u), n, steps, static_cast<const double*>(scale));
  else
    hipLaunchKernelGGL(step1d_kernel<float>, dim3(1), dim3(threads), shmem, s, static_cast<const float*>(G.dataT),
                       G.Mp, static_cast<const float*>(D.dataT), D.Mp, static_cast<float*>(p),
                       static_cast<float*>(u), n, steps, static_cast<const float*>(scale));
  return hipGetLastError();
}

hipError_t launch_zero_dirichlet(int prec, void* p, int ndim, const int64_t* n, const int* lo, const int* hi,
                                 hipStream_t s) {
  const int64_t total = n[0] * n[1] * n[2];
  const unsigned nb = blocks_for(total, 256);
  if (prec == PSTD_FP64)
    hipLaunchKernelGGL(zero_dirichlet_kernel<double>, dim3(nb), dim3(256), 0, s, static_cast<double*>(p), ndim, n[0],
                       n[1], n[2], lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]);
  else
    hipLaunchKernelGGL(zero_dirichlet_kernel<float>, dim3(nb), dim3(256), 0, s, static_cast<float*>(p), ndim, n[0],
                       n[1], n[2], lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]);
  return hipGetLastError();
}

hipError_t launch_fill_zero(int prec, void* x, int64_t count, hipStream_t s) {
  const unsigned nb = blocks_for(count, 256);
  if (prec == PSTD_FP64)
    hipLaunchKernelGGL(fill_zero_kernel<double>, dim3(nb), dim3(256), 0, s, static_cast<double*>(x), count);
  else
    hipLaunchKernelGGL(fill_zero_kernel<float>, dim3(nb), dim3(256), 0, s, static_cast<float*>(x), count);
  return hipGetLastError();
}

hipError_t launch_square(int prec, const float* in, void* out, int64_t count, hipStream_t s) {
  if (prec == PSTD_FP64)
    hipLaunchKernelGGL(square_kernel<double>, dim3(blocks_for(count, 256)), dim3(256), 0, s, in,
                       static_cast<double*>(out), count);
  else
    hipLaunchKernelGGL(square_kernel<float>, dim3(blocks_for(count, 256)), dim3(256), 0, s, in,
                       static_cast<float*>(out), count);
  return hipGetLastError();
}

hipError_t launch_combine(const float* const* f, const float* w, int nf, float* out, int64_t count, hipStream_t s) {
  if (nf < 1 || nf > kMaxFields) return hipErrorInvalidValue;
  CombineArgs a;
  for (int i = 0; i < nf; ++i) {
    a.f[i] = f[i];
    a.w[i] = w[i];
  }
  a.nf = nf;
  hipLaunchKernelGGL(combine_kernel, dim3(blocks_for((count + 3) / 4, 256)), dim3(256), 0, s, a, out, count);
  return hipGetLastError();
}

hipError_t launch_nonfinite(int prec, const void* x, int64_t count, int* flag, hipStream_t s) {
  const unsigned nb = blocks_for(count, 256);
  if (prec == PSTD_FP64)
    hipLaunchKernelGGL(nonfinite_kernel<double>, dim3(nb), dim3(256), 0, s, static_cast<const double*>(x), count, flag);
  else
    hipLaunchKernelGGL(nonfinite_kernel<float>, dim3(nb), dim3(256), 0, s, static_cast<const float*>(x), count, flag);
  return hipGetLastError();
}

}  // namespace pstd
