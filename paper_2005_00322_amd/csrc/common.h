// Internal declarations shared by the libpstd sources (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pstd.h"

namespace pstd {

// ---- error reporting ------------------------------------------------------------------------------
void set_error(const char* fmt, ...);
int fail(int status, const char* fmt, ...);

#define PSTD_HIP(expr)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::pstd::fail(PSTD_E_HIP, "%s failed: %s (%s:%d)", #expr,                    \
                          hipGetErrorString(e_), __FILE__, __LINE__);                    \
  } while (0)

// ---- host operator tables (tables.cpp) ------------------------------------------------------------
// Per-axis boundary case of Table transform_choices.
// CASE_PP: a periodic axis (the Fourier basis).  CASE_NNH .. CASE_DDH: a Neumann or Dirichlet wall on
// node 0 and a Neumann or Dirichlet wall half a step beyond node n-1 (groups III/IV, types V-VIII).
enum AxisCase {
  CASE_NN = 0, CASE_ND = 1, CASE_DN = 2, CASE_DD = 3, CASE_PP = 4,
  CASE_NNH = 5, CASE_NDH = 6, CASE_DNH = 7, CASE_DDH = 8
};

inline bool half_wall(int face) { return face == PSTD_NEUMANN_HALF || face == PSTD_DIRICHLET_HALF; }

inline AxisCase axis_case(int left, int right) {
  if (left == PSTD_PERIODIC) return CASE_PP;
  if (half_wall(right))
    return static_cast<AxisCase>(CASE_NNH + 2 * (left == PSTD_DIRICHLET) + (right == PSTD_DIRICHLET_HALF));
  return static_cast<AxisCase>(2 * (left == PSTD_DIRICHLET) + (right == PSTD_DIRICHLET));
}

// Staggered points of an axis: n - 1 between two walls on nodes, n on a periodic axis or one whose right
// wall lies on the last staggered point.
inline int staggered_points(int n, AxisCase c) { return c >= CASE_PP ? n : n - 1; }

// Unscaled FP64 operators of one axis for dx = 1 (scale by 1/dx), with m = staggered_points(n, case):
//   G: m x n row-major, velocity operator T2^{-1} diag(a1) T1 (periodic: F^{-1} diag(i k e^{i k/2}) F)
//   D: n x m row-major, pressure operator T1^{-1} diag(a2) T2 (periodic: F^{-1} diag(i k e^{-i k/2}) F)
struct AxisTables {
  int n = 0;
  AxisCase c = CASE_NN;
  std::vector<double> G, D;
  double kmax = 0.0;  // largest |k| the pressure basis carries (dx = 1)
};

// Returns a cached table (built once per (n, case) in the process).
const AxisTables& axis_tables(int n, AxisCase c);

// Largest |k| of the pressure basis for dx = 1 (the value AxisTables::kmax holds), without building the
// tables.
double axis_kmax(int n, AxisCase c);

// Collocated differentiation and half-step interpolation along one wall-bounded axis (not CASE_PP),
// dx = 1, row-major, m = n - 1 staggered points.  kind 2: d/dx on the nodes (n x n); 3: d/dx on the
// staggered points (m x m); 4: nodes -> staggered points (m x n); 5: staggered points -> nodes (n x m).
std::vector<double> resample_table(int n, AxisCase c, int kind, int* rows, int* cols);

// ---- device helpers ------------------------------------------------------------------------------
// Block barrier ordering only LDS accesses.  __syncthreads() also orders global memory, which makes the
// compiler drain every outstanding global load (s_waitcnt vmcnt(0)) at each barrier and so defeats
// prefetching across it.  The kernels here exchange data between waves only through LDS.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Padding of every device operator matrix: rows to a multiple of kRowPad, columns to kColPad.
constexpr int kRowPad = 128;
constexpr int kColPad = 64;

// One operator (an M x K row-major matrix, zero padded) in the precision of its plan.
struct DevOperator {
  int M = 0, K = 0;        // logical size
  int Mp = 0, Kp = 0;      // padded size (row stride = Kp)
  void* data = nullptr;    // FP64: double[Mp*Kp]; FP32: float[Mp*Kp]; SPLIT: bf16 hi[Mp*Kp] then lo[Mp*Kp]
  void* dataT = nullptr;   // 1D plans: transposed copy, Kp x Mp (row stride Mp)
  // SPLIT only, operators with a Toeplitz-plus-Hankel form and kThRowsMin < M <= kThRowsMax, Kp <= kThColsMax:
  // FP32 f and g windows of th_len values each (see kernels_split.hip) and the end weights
  // {first row, last row, first column, last column}
  float* th = nullptr;
  int th_len = 0;
  float thw[4] = {1.f, 1.f, 1.f, 1.f};
};

// Operators whose slices the split-bf16 contraction forms from their Toeplitz and Hankel parts.
constexpr int kThRowsMin = 192, kThRowsMax = 384, kThColsMax = 512;
constexpr int kThLen = kThRowsMax + kThColsMax + 8;   // upper bound of th_len
// Largest entry error of the form, relative to max|A|: far below FP32 rounding, so the slices formed on
// the chip equal the stored operator to the rounding of their FP32 sum.
constexpr double kThTol = 1e-9;

// A (R x C, row-major, FP64) = diag(wr) (F + H) diag(wc) with F[r][c] = f[r - c + C - 1],
// H[r][c] = g[r + c] (f and g of R + C - 1 values), wr and wc one except w = {wr[0], wr[R-1], wc[0],
// wc[C-1]}, to tol * max|A|; false (outputs untouched except resid) when A has no such form.
bool toeplitz_hankel(const double* A, int R, int C, double tol, std::vector<double>* f, std::vector<double>* g,
                     double w[4], double* resid);

struct ContractArgs {
  const void* A;        // operator, row-major, row stride lda, zero padded
  const void* A_lo;     // SPLIT_BF16 only: low part
  int lda;
  int M, K;             // output length and input length along the contracted axis
  const void* X;        // input field
  void* Y;              // output field (read-modify-write)
  int64_t ncols;        // strided: contiguous extent C; contiguous: number of rows R
  int64_t batch;        // strided: number of outer blocks; contiguous: 1
  int64_t x_bstride;    // strided: elements between outer blocks of X (= K*C)
  int64_t y_bstride;    // strided: elements between outer blocks of Y (= M*C)
  float alpha, beta;    // Y = beta*Y + alpha * scale * (A X)
  double alpha_d, beta_d;
  const void* scale;    // optional per-point factor with Y's layout (c0(x)^2 map, state dtype), may be null
  const float* th;      // SPLIT_BF16: Toeplitz/Hankel windows of the operator (null: read A and A_lo)
  int th_len;
  float thw[4];
};

// Launchers (kernels_*.hip).  contiguous = the contracted axis is the last (unit-stride) one.
hipError_t launch_contract_fp32(const ContractArgs& a, bool contiguous, hipStream_t s);
hipError_t launch_contract_fp64(const ContractArgs& a, bool contiguous, hipStream_t s);
hipError_t launch_contract_split(const ContractArgs& a, bool contiguous, hipStream_t s);
hipError_t launch_step1d(int prec, const DevOperator& G, const DevOperator& D, void* p, void* u, int n,
                         int64_t steps, const void* scale, hipStream_t s);
hipError_t launch_zero_dirichlet(int prec, void* p, int ndim, const int64_t* n, const int* dir_lo,
                                 const int* dir_hi, hipStream_t s);
hipError_t launch_fill_zero(int prec, void* x, int64_t count, hipStream_t s);
hipError_t launch_square(int prec, const float* in, void* out, int64_t count, hipStream_t s);
hipError_t launch_combine(const float* const* f, const float* w, int nf, float* out, int64_t count,
                          hipStream_t s);
bool phase2d_supported(int nx, int ny);
hipError_t launch_phase2d(const DevOperator& Gx, const DevOperator& Gy, const DevOperator& Dx, const DevOperator& Dy,
                          float* p, float* ux, float* uy, const float* c2, int nx, int ny, int64_t steps,
                          hipStream_t s);
hipError_t launch_phase2d_one(int which, const DevOperator& Gx, const DevOperator& Gy, const DevOperator& Dx,
                              const DevOperator& Dy, float* p, float* ux, float* uy, const float* c2, int nx, int ny,
                              hipStream_t s);
// ---- batched 2D solves (kernels_batch2d.hip, capi_batch.hip) --------------------------------------
struct BatchSolve {
  float* p;                 // nx x ny
  float* ux;                // (nx-1) x ny
  float* uy;                // nx x (ny-1)
  const float* Gx; const float* Dx; const float* Gy; const float* Dy;   // unscaled (dx = 1) operators
  int ldgx, lddx, ldgy, lddy;                                          // their row strides
  int mgx, mdx, mgy, mdy;                                              // their allocated (padded) rows
  int nx, ny;
  double sG;                // -dt / (rho0 dx)
  double sD;                // -dt rho0 c0^2 / dx, or -dt rho0 / dx with a c0^2 map
  const float* c2;          // nx x ny map of c0(x)^2, or null for a homogeneous medium
};
// One fused phase of many solves of one shape (kernels_phase2d.hip): grid (tiles, count).
hipError_t launch_phase2d_batch(int which, const BatchSolve* solves, int count, int nx, int ny, hipStream_t s);
bool batch2d_phase_fits(int ldgx, int ldgy, int lddx, int lddy, int nx, int ny);
struct BatchTask {
  int solve;
  int kind;                 // 0 u_x tile, 1 u_y tile, 2 p tile
  int i0, j0;
};
// Tiles of each phase are kept in kBatchQueues queues, one per XCD (blocks of XCD x are those with
// blockIdx % 8 == x): queue q holds the tiles of the solves assigned to XCD q, so a solve's operator rows
// and field strips are fetched into one L2; a block drains its own queue, then takes tiles from the others.
constexpr int kBatchQueues = 8;
constexpr int kBatchCountersPerStep = 2 * kBatchQueues + 2;   // tickets per queue and phase, two arrivals
struct BatchArgs {
  const BatchSolve* solves;
  const BatchTask* tasksA;  // velocity-phase tiles, queue after queue
  int segA[kBatchQueues + 1];   // queue q is tasksA[segA[q] .. segA[q + 1])
  const BatchTask* tasksB;  // pressure-phase tiles
  int segB[kBatchQueues + 1];
  unsigned* counters;       // kBatchCountersPerStep per step, zeroed by the launcher
  unsigned* timeout;        // set to 1 when a grid barrier gives up waiting (sticky; cleared by the host)
  int64_t steps;
};
int batch2d_max_blocks(int tile, int* out);   // tile: 32 or 64 (output tile edge)
hipError_t launch_batch2d(const BatchArgs& a, int tile, int blocks, hipStream_t s);

hipError_t launch_nonfinite(int prec, const void* x, int64_t count, int* flag, hipStream_t s);

// ---- FFT path of one axis (kernels_fft.hip, fft_plan.cpp) ------------------------------------------
// Device tables of one axis whose extended period L = 2(n-1) is 16 x 2^a 3^b 5^c (in the state dtype:
// complex float, or complex double for FP64 plans).
struct FftAxis {
  bool ok = false;              // the axis can use the FFT path
  int N = 0, L = 0;             // N = n - 1, L = 2N
  int npass = 0;
  int radix[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int sL = 1, sR = 1;           // +1 Neumann wall, -1 Dirichlet wall
  void* tab = nullptr;          // 64 + L/16 entries: w^l (l < 64) then w^{64 h}, w = e^{-2 pi i / 4L}
  double kfac[2] = {0, 0};      // pi c / (N L) with c the velocity (0) or pressure (1) constant
  // FP32 plans with L = 2^m, 256 <= L <= 8192 (fft_pow2_kernel): complex FP32 tables
  void* tw = nullptr;           // w, w^2, w^4, w^8 of each Stockham pass after the first, per j mod Ns
  void* hb = nullptr;           // e^{i pi (2t + a) / (2L)}, t < L/16 (a = 1 for mixed walls)
  void* pre = nullptr;          // e^{-i pi t / L}, t < L/16 (mixed walls)
  bool periodic = false;        // a periodic axis: L = n, no extension (fft_pow2_kernel only)
};

struct FftArgs {
  const void* X;                // input field
  void* Y;                      // output field (read-modify-write)
  const void* scale;            // optional per-point factor with Y's layout, may be null
  const void* tab;              // root table (FftAxis::tab)
  const void* tw;               // fft_pow2_kernel: FftAxis::tw, FftAxis::hb, FftAxis::pre
  const void* h;
  const void* pre;
  double kfac;                  // FftAxis::kfac of this direction
  double alpha, beta;           // Y = beta Y + alpha scale (op X)
  int N, L;
  int nin, nout;                // extents of X and Y along the axis
  int dir;                      // 0: G (nodes -> half nodes), 1: D (half nodes -> nodes)
  int sL, sR, anti;
  int periodic;                 // a periodic axis (fft_pow2_kernel): L = n input and output values per line
  int F;                        // transforms per block (2F lines)
  int npass;
  int radix[8];
  int contig;                   // 1: the axis is the unit-stride one (lines are rows)
  int xcd_spread;               // launch is padded to a multiple of 8 blocks and line groups spread per XCD
  int64_t ncols;                // contig: number of rows; strided: extent of the unit-stride block
  int64_t gpb;                  // strided: line groups per outer block
  int64_t groups;               // line groups (working blocks)
  int64_t x_bstride, y_bstride; // strided: elements between outer blocks
};

// Radix passes for a transform of length L (all 16, 8, 4, 2, 3, 5); false if L is not 16 x 2^a 3^b 5^c or
// needs more than 8 passes.
bool fft_factor(int L, int* npass, int* radix);
int fft_capacity(bool dbl);     // complex entries per block (F L at most)
int fft_max_per_block(bool dbl, int L);   // transforms per block that keep a block within 64 KB of LDS
bool fft_axis_possible(int n, int prec);
void fft_axis_free(FftAxis* f);
hipError_t launch_fft_axis(bool dbl, const FftArgs& a, hipStream_t s);
// FP32 power-of-two lengths 256 <= L <= 8192: lines per block of fft_pow2_kernel (0: not supported), and
// its launch (F = lines / 2 transforms per block, tables tw, h, pre set)
int fft_pow2_lines(int L);
hipError_t launch_fft_pow2(const FftArgs& a, hipStream_t s);
// the launches of up to three axes as one (one transform length, all periodic or none; each a[i] as for
// launch_fft_pow2); the axes must write different outputs
hipError_t launch_fft_pow2_multi(const FftArgs* a, int count, hipStream_t s);

// ---- neural-operator surrogate (kernels_nop.hip, capi_nop.hip) ----------------------------------------
// C[z] = alpha A[z] B[z] (+ beta C[z]) (+ bias_m[m]) (+ D[z]) (* GELU'(dgelu[z])), then with act set
// pre[z] = value (if pre is given) and C[z] = GELU(value).  A is M x K, B is K x N, C is M x N, all FP32
// with element strides; the batch index z = z1 nb2 + z2 adds z1 b*1 + z2 b*2 to each operand.  pre and
// dgelu use C's strides.
struct NopGemm {
  const float* A; const float* B; float* C;
  int M, N, K;
  int64_t sAm, sAk, sBk, sBn, sCm, sCn;
  int nb1, nb2;
  int64_t bA1, bA2, bB1, bB2, bC1, bC2;
  float alpha, beta;
  const float* bias_m;
  const float* add;
  int64_t sDm, sDn, bD1, bD2;
  float* pre;
  const float* dgelu;
  int act;              // apply GELU
  int split;            // 1: hi*hi + hi*lo + lo*hi bf16 products (near FP32); 0: one bf16 product
};
hipError_t launch_nop_gemm(const NopGemm& g, hipStream_t s);
// Y[b][o][p] = sum_i A[o][i] X[b][i][p] (+ bias[o]) (+ D[b][o][p]) (+ sum_k T[b][h][o][k] Cw[k][w] at
// p = (h, w)) (-> pre, GELU) for O <= 32 over an H x W grid, on the bf16 matrix cores (split: hi/lo
// parts); A is O x I row-major, or I x O (its transpose) with transA; T ([b][h][o][Mm]) and Cw (Mm x W)
// optional.  act_types: 0 X, Y, T in FP32; 1 X in FP32, Y in bf16; 2 X, Y, T in bf16 (inference
// activations, which every consumer rounds to bf16 before its product).
hipError_t launch_nop_mix(const float* A, bool transA, const void* X, void* Y, const float* bias, const float* D,
                          float* pre, const void* T, const float* Cw, int Mm, int O, int I, int H, int W, int B, bool act,
                          bool split, int act_types, hipStream_t s);
// out = Q2 GELU(Q1 v + q1b) + q2b per position (C <= 32); qpre and q stored when non-null; v in bf16 with
// half.
hipError_t launch_nop_project(const float* Q1, const float* q1b, const float* Q2, const float* q2b, const void* v,
                              float* out, float* qpre, float* q, int C, int Hp, int64_t P, int B, bool split, bool half,
                              hipStream_t s);
// A[pl][kh][kw] = sum_h sum_w Ch[kh][h] V[pl][h][w] Cw[kw][w] for every plane (the truncated 2D DCT, Ch:
// Mm x H, Cw: Mm x W), one plane per wave on the bf16 matrix cores; W <= 128, Mm <= 64.
// The per-plane DCT kernels read their tables from images (bf16, remainders with split) built once:
// sizes, and the kernel that builds them from the FP32 tables Ch (Mm x H) and Cw (Mm x W).
void nop_table_bytes(int H, int W, int Mm, bool split, size_t* dct2_bytes, size_t* idct_bytes);
hipError_t launch_nop_tables(const float* Ch, const float* Cw, void* dct2_img, void* idct_img, int H, int W, int Mm,
                             bool split, hipStream_t s);
bool nop_dct2_supported(int H, int W, int Mm);
hipError_t launch_nop_dct2(const void* V, float* A, const void* img, int planes, int H, int W, int Mm, bool split,
                           bool half, hipStream_t s);   // V in bf16 with half
// T[b][h][c][kw] = sum_kh Ch[kh][h] Z[b][c][kh][kw] (first inverse-DCT stage), one plane per wave on the
// bf16 matrix cores; Mm <= 64 and H <= 512 (LDS).
hipError_t launch_nop_idct_h(const float* Z, void* T, const void* img, int B, int C, int H, int Mm, bool split,
                             bool half, hipStream_t s);   // T in bf16 with half
hipError_t launch_nop_mode_transpose(const float* in, float* out, int B, int C, int Mm, bool to_block, hipStream_t s);
hipError_t launch_nop_features(const float* p0, const float* c0, float* f, int B, int H, int W, hipStream_t s);
hipError_t launch_nop_gelu_bwd(const float* gin, const float* pre, float* d, int64_t n, hipStream_t s);
hipError_t launch_nop_rowsum(const float* x, float* out, int nb, int rows, int64_t P, hipStream_t s);
hipError_t launch_nop_partial_sum(const float* part, float* out, int nz, int n, hipStream_t s);
hipError_t launch_nop_loss(const float* out, const float* tgt, double* terms, float* dout, int B, int64_t P,
                           hipStream_t s);
hipError_t launch_nop_input_stats(const float* p0, const float* c0, double* stats, int B, int H, int W, int margin,
                                  hipStream_t s);
hipError_t launch_nop_adam(float* th, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t s);

}  // namespace pstd

// ---- the plan --------------------------------------------------------------------------------------
struct pstd_plan_s {
  int ndim = 0;
  int64_t n[3] = {1, 1, 1};
  int bc[6] = {0, 0, 0, 0, 0, 0};
  double dx = 0, dt = 0, c0 = 0, rho0 = 1000.0;
  int prec = PSTD_FP32;
  hipStream_t stream = nullptr;
  int device = 0;
  pstd::DevOperator G[3], D[3];  // dense operators (built when an axis runs the dense path)
  pstd::DevOperator R[3][4];     // collocated-derivative and interpolation operators (built on first use)
  pstd::FftAxis fft[3];
  void* c2map = nullptr;       // c0(x)^2 in the state dtype (owned), null for a homogeneous medium
  int* flag = nullptr;         // device int for reductions (owned)
  int path = 0;                // PSTD_PATH_* (0 = automatic)
  bool use_th = true;          // split-bf16 contractions form Toeplitz-plus-Hankel operators on the chip
  bool fft_pow2 = true;        // FP32 power-of-two FFT axes use fft_pow2_kernel
  // captured step graphs: slot 0 holds a full chunk of steps, slot 1 the last other length used
  struct StepGraph {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int64_t steps = 0;
    void* key[4] = {nullptr, nullptr, nullptr, nullptr};
  } graphs[2];
};

namespace pstd {
// Build the FFT tables of axis a (no-op when the axis cannot use the FFT path).  sG, sD: the constants
// -dt/(rho0 dx) and -dt rho0 c0^2/dx of the velocity and pressure operators.
int fft_axis_setup(pstd_plan_s* P, int a, double sG, double sD);
}  // namespace pstd
