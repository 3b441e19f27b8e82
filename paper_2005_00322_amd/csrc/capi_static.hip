// libpstd C ABI: relative L2 errors of a batch of device fields without any allocation.
//
// The same measure as pstd_nop_relative_errors (the surrogate's error against the solver, and the parity
// measure of the tests), for callers that cannot allocate device memory: the per-block partial sums live
// in a file-scope device array instead of a buffer the library allocates, and the result is written to a
// caller-owned device array, so the call enqueues two kernels and nothing else (no allocation, no copy,
// no synchronisation).  Every call on a GPU shares that GPU's copy of the array: calls that overlap on
// one GPU (two streams, two host threads) race on it.
#include <algorithm>
#include <mutex>

#include "common.h"

namespace pstd {
namespace {

constexpr int kPairsMax = 65536;      // partial (squared error, squared reference) pairs: 1 MiB per GPU
constexpr int kBlocksPerSample = 256;
constexpr int kThreads = 256;

// Partial sums of every call: pair i holds (sum d^2, sum t^2) of one block of one sample.
static __device__ __align__(256) double scratch[2 * kPairsMax];

// Device address of each GPU's copy of `scratch`, looked up once per device with that device current.
// In host code the array's name is not a device address; only these pointers are passed to kernels.
double* g_ptr[64] = {nullptr};
std::mutex g_mu;

int scratch_for_current_device(double** out) {
  int dev = 0;
  PSTD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(PSTD_E_UNSUPPORTED, "device index %d above 63", dev);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PSTD_E_HIP, "hipGetSymbolAddress of the partial-sum array failed: %s", hipGetErrorString(e));
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return PSTD_OK;
}

// Block b * nb + x sums chunk x of sample b: (pred - target)^2 and target^2 in FP64.
__global__ __launch_bounds__(kThreads) void rel_err_partial_kernel(const float* __restrict__ pred,
                                                                   const float* __restrict__ tgt, int64_t count,
                                                                   int nb, double* __restrict__ part) {
  const int b = blockIdx.x / nb, x = blockIdx.x % nb;
  const int64_t chunk = (count + nb - 1) / nb;
  const int64_t lo = x * chunk, hi = min<int64_t>(count, lo + chunk);
  const float* o = pred + b * count;
  const float* t = tgt + b * count;
  double sn = 0.0, sd = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const double tv = static_cast<double>(t[i]);
    const double d = static_cast<double>(o[i]) - tv;
    sn += d * d;
    sd += tv * tv;
  }
  __shared__ double rn[kThreads], rd[kThreads];
  rn[threadIdx.x] = sn;
  rd[threadIdx.x] = sd;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) {
      rn[threadIdx.x] += rn[threadIdx.x + w];
      rd[threadIdx.x] += rd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t slot = static_cast<int64_t>(b) * nb + x;
    part[2 * slot] = rn[0];
    part[2 * slot + 1] = rd[0];
  }
}

// err[b] = sqrt(sum over the sample's blocks of d^2 / sum of t^2), 0 where the reference is zero.
__global__ __launch_bounds__(kThreads) void rel_err_final_kernel(const double* __restrict__ part, int nb,
                                                                 double* __restrict__ err) {
  const int b = blockIdx.x;
  double sn = 0.0, sd = 0.0;
  for (int x = threadIdx.x; x < nb; x += kThreads) {
    const int64_t slot = static_cast<int64_t>(b) * nb + x;
    sn += part[2 * slot];
    sd += part[2 * slot + 1];
  }
  __shared__ double rn[kThreads], rd[kThreads];
  rn[threadIdx.x] = sn;
  rd[threadIdx.x] = sd;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) {
      rn[threadIdx.x] += rn[threadIdx.x + w];
      rd[threadIdx.x] += rd[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) err[b] = rd[0] > 0.0 ? sqrt(rn[0] / rd[0]) : 0.0;
}

}  // namespace
}  // namespace pstd

using namespace pstd;

extern "C" {

int pstd_relative_errors_static(const float* pred, const float* target, int32_t batch, int64_t count, double* err,
                                void* hip_stream) {
  if (!pred || !target || !err) return fail(PSTD_E_INVALID_ARG, "null pointer");
  if (batch < 1 || count < 1) return fail(PSTD_E_INVALID_ARG, "batch and count must be >= 1");
  if (batch > kPairsMax)
    return fail(PSTD_E_UNSUPPORTED, "batch %d above the %d samples the partial-sum array holds", batch, kPairsMax);
  if (count > (int64_t(1) << 40)) return fail(PSTD_E_UNSUPPORTED, "count above 2^40");
  double* part = nullptr;
  const int st = scratch_for_current_device(&part);
  if (st != PSTD_OK) return st;
  // blocks per sample: enough to stream a large field, within the array's kPairsMax pairs
  int64_t nb = std::min<int64_t>(kBlocksPerSample, (count + 8 * kThreads - 1) / (8 * kThreads));
  nb = std::max<int64_t>(1, std::min<int64_t>(nb, kPairsMax / batch));
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(rel_err_partial_kernel, dim3(static_cast<unsigned>(nb * batch)), dim3(kThreads), 0, s, pred,
                     target, count, static_cast<int>(nb), part);
  PSTD_HIP(hipGetLastError());
  hipLaunchKernelGGL(rel_err_final_kernel, dim3(static_cast<unsigned>(batch)), dim3(kThreads), 0, s, part,
                     static_cast<int>(nb), err);
  PSTD_HIP(hipGetLastError());
  return PSTD_OK;
}

}  // extern "C"
