// libpstd C ABI: plan creation (operator tables), state initialisation, stepping, combination.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "common.h"

namespace pstd {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int fail(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return status;
}

namespace {

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

float bf16_to_float(uint16_t h) {
  uint32_t u = static_cast<uint32_t>(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Round the FP64 matrix (M x K, already scaled) to the plan precision and upload it zero padded.
int upload_operator(pstd_plan_s* P, const std::vector<double>& m, int M, int K, double scale, DevOperator* op) {
  op->M = M;
  op->K = K;
  op->Mp = static_cast<int>(round_up(M, kRowPad));
  op->Kp = static_cast<int>(round_up(K, kColPad));
  const size_t cnt = static_cast<size_t>(op->Mp) * op->Kp;
  const bool want_t = (P->ndim == 1);
  if (P->prec == PSTD_FP64 || P->prec == PSTD_FP32) {
    const size_t esz = P->prec == PSTD_FP64 ? 8 : 4;
    std::vector<unsigned char> host(cnt * esz, 0), hostT(want_t ? cnt * esz : 0, 0);
    for (int i = 0; i < M; ++i)
      for (int k = 0; k < K; ++k) {
        const double v = scale * m[static_cast<size_t>(i) * K + k];
        const size_t a = static_cast<size_t>(i) * op->Kp + k;
        const size_t t = static_cast<size_t>(k) * op->Mp + i;
        if (esz == 8) {
          reinterpret_cast<double*>(host.data())[a] = v;
          if (want_t) reinterpret_cast<double*>(hostT.data())[t] = v;
        } else {
          reinterpret_cast<float*>(host.data())[a] = static_cast<float>(v);
          if (want_t) reinterpret_cast<float*>(hostT.data())[t] = static_cast<float>(v);
        }
      }
    if (hipMalloc(&op->data, cnt * esz) != hipSuccess) return fail(PSTD_E_OOM, "hipMalloc of an operator failed");
    PSTD_HIP(hipMemcpy(op->data, host.data(), cnt * esz, hipMemcpyHostToDevice));
    if (want_t) {
      if (hipMalloc(&op->dataT, cnt * esz) != hipSuccess) return fail(PSTD_E_OOM, "hipMalloc of an operator failed");
      PSTD_HIP(hipMemcpy(op->dataT, hostT.data(), cnt * esz, hipMemcpyHostToDevice));
    }
    return PSTD_OK;
  }
  // split bf16: hi = bf16(v), lo = bf16(v - hi), both rounded from the FP64 value
  std::vector<uint16_t> host(2 * cnt, 0);
  for (int i = 0; i < M; ++i)
    for (int k = 0; k < K; ++k) {
      const double v = scale * m[static_cast<size_t>(i) * K + k];
      const uint16_t hi = bf16_rne(static_cast<float>(v));
      const uint16_t lo = bf16_rne(static_cast<float>(v - static_cast<double>(bf16_to_float(hi))));
      host[static_cast<size_t>(i) * op->Kp + k] = hi;
      host[cnt + static_cast<size_t>(i) * op->Kp + k] = lo;
    }
  if (hipMalloc(&op->data, 2 * cnt * 2) != hipSuccess) return fail(PSTD_E_OOM, "hipMalloc of an operator failed");
  PSTD_HIP(hipMemcpy(op->data, host.data(), 2 * cnt * 2, hipMemcpyHostToDevice));
  // operators the contraction forms on the chip from f and g: windows Fr[i] = f(kThRowsMax - 1 - i) and
  // G[i] = g(i), i < th_len, zero past the operator
  std::vector<double> f, g;
  double w[4], resid = 0.0;
  if (M > kThRowsMin && M <= kThRowsMax && op->Kp <= kThColsMax &&
      toeplitz_hankel(m.data(), M, K, kThTol, &f, &g, w, &resid)) {
    const int len = kThRowsMax + op->Kp + 8;
    std::vector<float> win(2 * static_cast<size_t>(len), 0.f);
    for (int i = 0; i < len; ++i) {
      const int d = kThRowsMax - 1 - i;
      if (d >= 1 - K && d <= M - 1) win[i] = static_cast<float>(scale * f[d + K - 1]);
      if (i <= M + K - 2) win[len + i] = static_cast<float>(scale * g[i]);
    }
    if (hipMalloc(&op->th, win.size() * sizeof(float)) != hipSuccess)
      return fail(PSTD_E_OOM, "hipMalloc of an operator failed");
    PSTD_HIP(hipMemcpy(op->th, win.data(), win.size() * sizeof(float), hipMemcpyHostToDevice));
    op->th_len = len;
    for (int i = 0; i < 4; ++i) op->thw[i] = static_cast<float>(w[i]);
  }
  return PSTD_OK;
}

void drop_graphs(pstd_plan_s* P) {
  for (auto& g : P->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = pstd_plan_s::StepGraph{};
  }
}

void free_plan(pstd_plan_s* P) {
  if (!P) return;
  for (int a = 0; a < 3; ++a) {
    if (P->G[a].data) (void)hipFree(P->G[a].data);
    if (P->G[a].dataT) (void)hipFree(P->G[a].dataT);
    if (P->G[a].th) (void)hipFree(P->G[a].th);
    if (P->D[a].data) (void)hipFree(P->D[a].data);
    if (P->D[a].dataT) (void)hipFree(P->D[a].dataT);
    if (P->D[a].th) (void)hipFree(P->D[a].th);
    fft_axis_free(&P->fft[a]);
    for (int k = 0; k < 4; ++k) {
      if (P->R[a][k].data) (void)hipFree(P->R[a][k].data);
      if (P->R[a][k].dataT) (void)hipFree(P->R[a][k].dataT);
      if (P->R[a][k].th) (void)hipFree(P->R[a][k].th);
    }
  }
  if (P->c2map) (void)hipFree(P->c2map);
  if (P->flag) (void)hipFree(P->flag);
  drop_graphs(P);
  delete P;
}

int64_t numel_p(const pstd_plan_s* P) { return P->n[0] * P->n[1] * P->n[2]; }
bool axis_periodic(const pstd_plan_s* P, int a) { return P->bc[2 * a] == PSTD_PERIODIC; }
bool axis_half_wall(const pstd_plan_s* P, int a) { return half_wall(P->bc[2 * a + 1]); }
// n staggered points on a periodic axis and on one with a half-step wall, n - 1 otherwise
int64_t numel_u(const pstd_plan_s* P, int a) {
  return numel_p(P) / P->n[a] * (P->n[a] - (axis_periodic(P, a) || axis_half_wall(P, a) ? 0 : 1));
}

// Geometry of the contraction along axis a for a field whose extent along a is `len`.
void axis_geometry(const pstd_plan_s* P, int a, int64_t* outer, int64_t* inner) {
  int64_t o = 1, i = 1;
  for (int b = 0; b < a; ++b) o *= P->n[b];
  for (int b = a + 1; b < P->ndim; ++b) i *= P->n[b];
  *outer = o;
  *inner = i;
}

// Constants folded into the operators: velocity -dt/(rho0 dx), pressure -dt rho0 c0^2/dx (c0^2 from the
// map, applied pointwise, when the plan has one).
double const_G(const pstd_plan_s* P) { return -P->dt / P->rho0 / P->dx; }
double const_D(const pstd_plan_s* P) { return -P->dt * P->rho0 * (P->c2map ? 1.0 : P->c0 * P->c0) / P->dx; }

// Dense operators of axis a, built on first use for axes that start on the FFT path.
int ensure_dense(pstd_plan_s* P, int a) {
  if (P->G[a].data) return PSTD_OK;
  const int n = static_cast<int>(P->n[a]);
  if (n > 4097) return fail(PSTD_E_UNSUPPORTED, "axis %d: dense operators are limited to 4097 nodes", a);
  const AxisCase c = axis_case(P->bc[2 * a], P->bc[2 * a + 1]);
  const AxisTables& t = axis_tables(n, c);
  const int m = staggered_points(n, c);
  int st = upload_operator(P, t.G, m, n, const_G(P), &P->G[a]);
  if (st == PSTD_OK) st = upload_operator(P, t.D, n, m, const_D(P), &P->D[a]);
  return st;
}

// Whether axis a runs on the FFT path under the plan's current path setting.  AUTO: axes above 512
// nodes (1D plans keep the single-workgroup kernel up to 1365 nodes).
bool axis_fft(const pstd_plan_s* P, int a) {
  if (!P->fft[a].ok) return false;
  if (P->fft[a].periodic && !P->fft_pow2) return false;   // the mixed-radix kernel extends symmetrically
  if (P->path == PSTD_PATH_FFT || P->path == PSTD_PATH_FFT_GENERIC) return true;
  if (P->path != PSTD_PATH_AUTO) return false;
  if (P->ndim == 1) return P->n[0] > 1365;
  return P->n[a] > 512;
}

// Make sure every axis has what its path needs (called before any capture).
int prepare_axes(pstd_plan_s* P) {
  for (int a = 0; a < P->ndim; ++a)
    if (!axis_fft(P, a)) {
      const int st = ensure_dense(P, a);
      if (st != PSTD_OK) return st;
    }
  return PSTD_OK;
}

hipError_t contract(const pstd_plan_s* P, const DevOperator& op, int a, const void* X, void* Y, double alpha,
                    double beta, const void* scale, hipStream_t s) {
  ContractArgs c{};
  c.A = op.data;
  c.A_lo = nullptr;
  c.lda = op.Kp;
  c.M = op.M;
  c.K = op.K;
  c.X = X;
  c.Y = Y;
  c.alpha = static_cast<float>(alpha);
  c.beta = static_cast<float>(beta);
  c.alpha_d = alpha;
  c.beta_d = beta;
  c.scale = scale;
  int64_t outer, inner;
  axis_geometry(P, a, &outer, &inner);
  const bool contiguous = (a == P->ndim - 1);
  if (contiguous) {
    c.ncols = outer;
    c.batch = 1;
    c.x_bstride = 0;
    c.y_bstride = 0;
  } else {
    c.ncols = inner;
    c.batch = outer;
    c.x_bstride = static_cast<int64_t>(op.K) * inner;
    c.y_bstride = static_cast<int64_t>(op.M) * inner;
  }
  c.th = nullptr;
  c.th_len = 0;
  if (P->prec == PSTD_FP64) return launch_contract_fp64(c, contiguous, s);
  if (P->prec == PSTD_FP32) return launch_contract_fp32(c, contiguous, s);
  c.A_lo = static_cast<const uint16_t*>(op.data) + static_cast<size_t>(op.Mp) * op.Kp;
  if (op.th && P->use_th) {
    c.th = op.th;
    c.th_len = op.th_len;
    for (int i = 0; i < 4; ++i) c.thw[i] = op.thw[i];
  }
  return launch_contract_split(c, contiguous, s);
}

// The launch arguments of Y = beta Y + alpha scale (op X) along FFT axis a; true when the axis runs on the
// power-of-two kernel.
bool fft_args(const pstd_plan_s* P, int a, int which, const void* X, void* Y, double alpha, double beta,
              const void* scale, FftArgs* out) {
  const FftAxis& f = P->fft[a];
  FftArgs& x = *out;
  x = FftArgs{};
  x.X = X;
  x.Y = Y;
  x.scale = scale;
  x.tab = f.tab;
  x.kfac = f.kfac[which];
  x.alpha = alpha;
  x.beta = beta;
  x.N = f.N;
  x.L = f.L;
  const int n = static_cast<int>(P->n[a]);
  x.periodic = f.periodic;
  x.nin = which == 0 || f.periodic ? n : n - 1;
  x.nout = which == 1 || f.periodic ? n : n - 1;
  x.dir = which;
  x.sL = f.sL;
  x.sR = f.sR;
  x.anti = f.sL * f.sR < 0;
  x.npass = f.npass;
  for (int i = 0; i < 8; ++i) x.radix[i] = f.radix[i];
  int64_t outer, inner;
  axis_geometry(P, a, &outer, &inner);
  x.contig = a == P->ndim - 1;
  const int64_t lines = x.contig ? outer : outer * inner;
  // transforms per block: enough blocks to fill the chip first (about 1024), then as many lines per
  // block as 64 KB of LDS holds; at least 64 threads (F L / 16) where that allows
  const bool pow2 = f.tw != nullptr && P->fft_pow2;
  int F;
  if (pow2) {
    F = fft_pow2_lines(f.L) / 2;   // fixed by the kernel
    x.tw = f.tw;
    x.h = f.hb;
    x.pre = f.pre;
  } else {
    const int fmax = fft_max_per_block(P->prec == PSTD_FP64, f.L);
    F = static_cast<int>(std::min<int64_t>(fmax, std::max<int64_t>(1, lines / 2048)));
    F = std::max(F, std::min(fmax, std::max(1, 1024 / f.L)));
    F = static_cast<int>(std::min<int64_t>(F, (lines + 1) / 2));
    F = std::max(F, 1);
  }
  x.F = F;
  const int W = 2 * F;
  if (x.contig) {
    x.ncols = outer;
    x.gpb = 0;
    x.groups = (outer + W - 1) / W;
    x.x_bstride = x.y_bstride = 0;
  } else {
    x.ncols = inner;
    x.gpb = (inner + W - 1) / W;
    x.groups = outer * x.gpb;
    x.x_bstride = static_cast<int64_t>(x.nin) * inner;
    x.y_bstride = static_cast<int64_t>(x.nout) * inner;
  }
  x.xcd_spread = x.groups >= 64;
  return pow2;
}

// Y = beta Y + alpha scale (op X) along axis a with the velocity (which = 0) or pressure (which = 1)
// operator, on the axis's FFT or dense path.
hipError_t apply_op(const pstd_plan_s* P, int a, int which, const void* X, void* Y, double alpha, double beta,
                    const void* scale, hipStream_t s) {
  if (!axis_fft(P, a)) return contract(P, which == 0 ? P->G[a] : P->D[a], a, X, Y, alpha, beta, scale, s);
  FftArgs x;
  return fft_args(P, a, which, X, Y, alpha, beta, scale, &x) ? launch_fft_pow2(x, s)
                                                                : launch_fft_axis(P->prec == PSTD_FP64, x, s);
}

// The velocity half step of every axis as one launch when all of them run on the power-of-two FFT
// kernel with one transform length (each reads p and writes its own u_a); false: not applicable.
bool velocity_fft_multi(const pstd_plan_s* P, pstd_state* st, hipStream_t s, hipError_t* err) {
  if (P->ndim < 2) return false;
  FftArgs x[3];
  for (int a = 0; a < P->ndim; ++a) {
    if (!axis_fft(P, a) || !fft_args(P, a, 0, st->p, st->u[a], 1.0, 1.0, nullptr, &x[a])) return false;
    if (x[a].L != x[0].L || x[a].periodic != x[0].periodic) return false;
  }
  *err = launch_fft_pow2_multi(x, P->ndim, s);
  return true;
}

bool use_fused2d(const pstd_plan_s* P) {
  return P->ndim == 2 && P->prec == PSTD_FP32 && (P->path == PSTD_PATH_AUTO || P->path == PSTD_PATH_FUSED) &&
         phase2d_supported(static_cast<int>(P->n[0]), static_cast<int>(P->n[1]));
}

// Enqueue n steps of the 2D/3D scheme: all velocity contractions, then all pressure contractions
// (two fused phase kernels per step for small 2D FP32 plans, one kernel per axis and phase otherwise).
hipError_t enqueue_steps(pstd_plan_s* P, pstd_state* st, int64_t nsteps, hipStream_t s) {
  if (use_fused2d(P))
    return launch_phase2d(P->G[0], P->G[1], P->D[0], P->D[1], static_cast<float*>(st->p),
                          static_cast<float*>(st->u[0]), static_cast<float*>(st->u[1]),
                          static_cast<const float*>(P->c2map), static_cast<int>(P->n[0]), static_cast<int>(P->n[1]),
                          nsteps, s);
  for (int64_t t = 0; t < nsteps; ++t) {
    hipError_t e = hipSuccess;
    if (velocity_fft_multi(P, st, s, &e)) {
      if (e != hipSuccess) return e;
    } else {
      for (int a = 0; a < P->ndim; ++a) {
        e = apply_op(P, a, 0, st->p, st->u[a], 1.0, 1.0, nullptr, s);
        if (e != hipSuccess) return e;
      }
    }
    for (int a = 0; a < P->ndim; ++a) {
      e = apply_op(P, a, 1, st->u[a], st->p, 1.0, 1.0, P->c2map, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

constexpr int64_t kGraphChunk = 50;  // steps captured per graph launch

// The captured graph of `steps` steps on this state's buffers (captured on first use, kept per plan:
// slot 0 for a full chunk, slot 1 for the last other length).  Capturing runs nothing.
int step_graph(pstd_plan_s* P, const pstd_state* st, int64_t steps, hipGraphExec_t* out) {
  pstd_plan_s::StepGraph& g = P->graphs[steps == kGraphChunk ? 0 : 1];
  const bool same = g.exec && g.steps == steps && g.key[0] == st->p && g.key[1] == st->u[0] &&
                    g.key[2] == st->u[1] && g.key[3] == st->u[2];
  if (!same) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = pstd_plan_s::StepGraph{};
    hipStream_t cs;
    PSTD_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      pstd_state tmp = *st;
      const hipError_t le = enqueue_steps(P, &tmp, steps, cs);
      e = hipStreamEndCapture(cs, &g.graph);
      if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
      if (g.graph) (void)hipGraphDestroy(g.graph);
      g = pstd_plan_s::StepGraph{};
      return fail(PSTD_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    }
    g.steps = steps;
    g.key[0] = st->p;
    g.key[1] = st->u[0];
    g.key[2] = st->u[1];
    g.key[3] = st->u[2];
  }
  *out = g.exec;
  return PSTD_OK;
}

// Whether pstd_step runs the whole time loop in the single-workgroup 1D kernel (walls on nodes, at most
// 1365 nodes, not on the FFT path); other 1D plans step through the dense contractions.
bool use_step1d(const pstd_plan_s* P) {
  return P->ndim == 1 && !axis_fft(P, 0) && !axis_periodic(P, 0) && !axis_half_wall(P, 0) && P->n[0] <= 1365;
}

}  // namespace
}  // namespace pstd

using namespace pstd;

extern "C" {

const char* pstd_status_string(int status) {
  switch (status) {
    case PSTD_OK: return "ok";
    case PSTD_E_INVALID_ARG: return "invalid argument";
    case PSTD_E_UNSTABLE: return "time step above the stability limit";
    case PSTD_E_UNSUPPORTED: return "unsupported size or mode";
    case PSTD_E_HIP: return "HIP runtime error";
    case PSTD_E_OOM: return "out of device memory";
    case PSTD_E_NONFINITE: return "non-finite values in the state";
    default: return "unknown status";
  }
}

const char* pstd_last_error(void) { return g_err; }

int pstd_plan_create(const pstd_grid* grid, double dx, double dt, double c0, const int32_t bc_per_face[6],
                     pstd_plan* out) {
  return pstd_plan_create_ex(grid, dx, dt, c0, bc_per_face, 1000.0, PSTD_FP32, nullptr, nullptr, out);
}

int pstd_plan_create_ex(const pstd_grid* grid, double dx, double dt, double c0, const int32_t bc_per_face[6],
                        double rho0, int32_t precision, const float* c0_map_dev, void* hip_stream, pstd_plan* out) {
  if (!out) return fail(PSTD_E_INVALID_ARG, "out is null");
  *out = nullptr;
  if (!grid || !bc_per_face) return fail(PSTD_E_INVALID_ARG, "grid or bc_per_face is null");
  if (grid->ndim < 1 || grid->ndim > 3) return fail(PSTD_E_INVALID_ARG, "ndim must be 1, 2 or 3");
  if (!(dx > 0) || !(dt > 0) || !(c0 > 0) || !(rho0 > 0) || !std::isfinite(dx) || !std::isfinite(dt) ||
      !std::isfinite(c0) || !std::isfinite(rho0))
    return fail(PSTD_E_INVALID_ARG, "dx, dt, c0 and rho0 must be positive and finite");
  if (precision < PSTD_FP64 || precision > PSTD_SPLIT_BF16) return fail(PSTD_E_INVALID_ARG, "bad precision");
  for (int a = 0; a < grid->ndim; ++a) {
    if (grid->n[a] < 3) return fail(PSTD_E_INVALID_ARG, "axis %d has %lld nodes (need >= 3)", a, (long long)grid->n[a]);
    const bool per_fft = bc_per_face[2 * a] == PSTD_PERIODIC && precision != PSTD_FP64 && grid->n[a] <= 8192 &&
                         fft_pow2_lines(static_cast<int>(grid->n[a])) > 0;
    if (grid->n[a] > 4097 && bc_per_face[2 * a] != PSTD_PERIODIC &&
        !(grid->n[a] <= 16385 && fft_axis_possible(static_cast<int>(grid->n[a]), precision)))
      return fail(PSTD_E_UNSUPPORTED,
                  "axis %d: %lld nodes; above 4097 the FFT path needs 2(n-1) = 16 x 2^a 3^b 5^c within %d (%s)", a,
                  (long long)grid->n[a], fft_capacity(precision == PSTD_FP64),
                  precision == PSTD_FP64 ? "FP64" : "FP32 state");
    for (int f = 0; f < 2; ++f)
      if (bc_per_face[2 * a + f] != PSTD_NEUMANN && bc_per_face[2 * a + f] != PSTD_DIRICHLET &&
          bc_per_face[2 * a + f] != PSTD_PERIODIC && !(f == 1 && half_wall(bc_per_face[2 * a + f])))
        return fail(PSTD_E_INVALID_ARG, "bad boundary condition on face %d (half-step walls are right faces)",
                    2 * a + f);
    if (half_wall(bc_per_face[2 * a + 1]) && bc_per_face[2 * a] == PSTD_PERIODIC)
      return fail(PSTD_E_INVALID_ARG, "axis %d: a periodic axis has both faces periodic", a);
    if (half_wall(bc_per_face[2 * a + 1]) && grid->n[a] > 4097)
      return fail(PSTD_E_UNSUPPORTED, "axis %d: half-step walls run on the dense path (at most 4097 nodes)", a);
    if ((bc_per_face[2 * a] == PSTD_PERIODIC) != (bc_per_face[2 * a + 1] == PSTD_PERIODIC))
      return fail(PSTD_E_INVALID_ARG, "axis %d: a periodic axis has both faces periodic", a);
    if (bc_per_face[2 * a] == PSTD_PERIODIC && grid->n[a] > 4097 && !per_fft)
      return fail(PSTD_E_UNSUPPORTED,
                  "axis %d: periodic axes above 4097 points need n a power of two up to 8192 and a float state", a);
  }
  // a single line has no matrix-matrix product for the bf16 matrix cores: a 1D split-bf16 plan (float
  // state) computes as an FP32 plan
  if (grid->ndim == 1 && precision == PSTD_SPLIT_BF16) precision = PSTD_FP32;
  // 1D walls on nodes: the single-workgroup kernel up to 1365 nodes, above that the FFT path where 2(n-1)
  // factors and the dense contraction path otherwise (up to 4097 nodes, checked above)
  int64_t total = 1;
  for (int a = 0; a < grid->ndim; ++a) total *= grid->n[a];
  if (total > (int64_t(1) << 31)) return fail(PSTD_E_UNSUPPORTED, "grid above 2^31 points");
  if (precision == PSTD_SPLIT_BF16 && 4 * total >= (int64_t(1) << 31))
    return fail(PSTD_E_UNSUPPORTED, "split-bf16 plans need fields below 2 GiB (32-bit buffer offsets)");

  // stability: c0 dt |k|_max / 2 <= 1 with |k|_max^2 the sum of the per-axis maxima
  double kmax2 = 0.0;
  for (int a = 0; a < grid->ndim; ++a) {
    const double km = axis_kmax(static_cast<int>(grid->n[a]), axis_case(bc_per_face[2 * a], bc_per_face[2 * a + 1]));
    kmax2 += (km / dx) * (km / dx);
  }
  if (c0 * dt * std::sqrt(kmax2) / 2.0 > 1.0)
    return fail(PSTD_E_UNSTABLE, "c0*dt/dx = %g above the limit %g", c0 * dt / dx, 2.0 / (dx * std::sqrt(kmax2)));

  pstd_plan_s* P = new pstd_plan_s();
  P->ndim = grid->ndim;
  for (int a = 0; a < 3; ++a) P->n[a] = a < grid->ndim ? grid->n[a] : 1;
  for (int f = 0; f < 2 * grid->ndim; ++f) P->bc[f] = bc_per_face[f];
  P->dx = dx;
  P->dt = dt;
  P->c0 = c0;
  P->rho0 = rho0;
  P->prec = precision;
  P->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&P->device) != hipSuccess) {
    free_plan(P);
    return fail(PSTD_E_HIP, "hipGetDevice failed");
  }

  // velocity: u += -(dt/rho0) G p ; pressure: p += -(dt rho0 c0^2) D u (c0^2 from the map if given)
  const double sG = -dt / rho0 / dx;
  const double sD = -dt * rho0 * (c0_map_dev ? 1.0 : c0 * c0) / dx;
  for (int a = 0; a < P->ndim; ++a) {
    int st = fft_axis_setup(P, a, sG, sD);
    if (st != PSTD_OK) {
      free_plan(P);
      return st;
    }
  }
  if (hipMalloc(&P->flag, sizeof(int)) != hipSuccess) {
    free_plan(P);
    return fail(PSTD_E_OOM, "hipMalloc failed");
  }
  if (c0_map_dev) {
    if (hipMalloc(&P->c2map, (precision == PSTD_FP64 ? 8 : 4) * total) != hipSuccess) {
      free_plan(P);
      return fail(PSTD_E_OOM, "hipMalloc of the c0^2 map failed");
    }
    if (launch_square(precision, c0_map_dev, P->c2map, total, P->stream) != hipSuccess) {
      free_plan(P);
      return fail(PSTD_E_HIP, "squaring the c0 map failed");
    }
  }
  const int st = prepare_axes(P);
  if (st != PSTD_OK) {
    free_plan(P);
    return st;
  }
  *out = P;
  return PSTD_OK;
}

int pstd_plan_destroy(pstd_plan plan) {
  if (!plan) return PSTD_OK;
  if (plan->stream) (void)hipStreamSynchronize(plan->stream);
  else (void)hipDeviceSynchronize();
  free_plan(plan);
  return PSTD_OK;
}

int64_t pstd_plan_numel(pstd_plan plan, int32_t field) {
  if (!plan) return -1;
  if (field < 0) return numel_p(plan);
  if (field >= plan->ndim) return -1;
  return numel_u(plan, field);
}

int pstd_state_init(pstd_plan P, pstd_state* st, int32_t u_mode) {
  if (!P || !st || !st->p) return fail(PSTD_E_INVALID_ARG, "null plan/state/p");
  for (int a = 0; a < P->ndim; ++a)
    if (!st->u[a]) return fail(PSTD_E_INVALID_ARG, "u[%d] is null", a);
  if (u_mode < 0 || u_mode > 2) return fail(PSTD_E_INVALID_ARG, "u_mode must be 0, 1 or 2");
  const int pst = prepare_axes(P);
  if (pst != PSTD_OK) return pst;
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int a = 0; a < P->ndim; ++a) {
    lo[a] = P->bc[2 * a] == PSTD_DIRICHLET;
    hi[a] = P->bc[2 * a + 1] == PSTD_DIRICHLET;
  }
  PSTD_HIP(launch_zero_dirichlet(P->prec, st->p, P->ndim, P->n, lo, hi, P->stream));
  for (int a = 0; a < P->ndim; ++a) {
    if (u_mode == 2) break;
    if (u_mode == 1) {
      PSTD_HIP(launch_fill_zero(P->prec, st->u[a], numel_u(P, a), P->stream));
      continue;
    }
    // u^{-1/2} = +(dt/(2 rho0)) G p = -1/2 * (folded operator) p  (beta = 0: u is not read)
    PSTD_HIP(apply_op(P, a, 0, st->p, st->u[a], -0.5, 0.0, nullptr, P->stream));
  }
  st->step = 0;
  return PSTD_OK;
}

int pstd_step(pstd_plan P, pstd_state* st, int64_t n_steps) {
  if (!P || !st || !st->p) return fail(PSTD_E_INVALID_ARG, "null plan/state/p");
  for (int a = 0; a < P->ndim; ++a)
    if (!st->u[a]) return fail(PSTD_E_INVALID_ARG, "u[%d] is null", a);
  if (n_steps < 0) return fail(PSTD_E_INVALID_ARG, "n_steps < 0");
  if (n_steps == 0) return PSTD_OK;
  const int pst = prepare_axes(P);
  if (pst != PSTD_OK) return pst;
  if (use_step1d(P)) {
    PSTD_HIP(launch_step1d(P->prec, P->G[0], P->D[0], st->p, st->u[0], static_cast<int>(P->n[0]), n_steps,
                           P->c2map, P->stream));
    st->step += n_steps;
    return PSTD_OK;
  }
  // every step runs from a captured graph: whole chunks of kGraphChunk steps, then one graph of the rest
  const int64_t full = n_steps / kGraphChunk, rest = n_steps % kGraphChunk;
  hipGraphExec_t g = nullptr;
  if (full > 0) {
    const int gst = step_graph(P, st, kGraphChunk, &g);
    if (gst != PSTD_OK) return gst;
    for (int64_t i = 0; i < full; ++i) PSTD_HIP(hipGraphLaunch(g, P->stream));
  }
  if (rest > 0) {
    const int gst = step_graph(P, st, rest, &g);
    if (gst != PSTD_OK) return gst;
    PSTD_HIP(hipGraphLaunch(g, P->stream));
  }
  st->step += n_steps;
  return PSTD_OK;
}

int pstd_step_prepare(pstd_plan P, const pstd_state* st, int64_t n_steps) {
  if (!P || !st || !st->p) return fail(PSTD_E_INVALID_ARG, "null plan/state/p");
  for (int a = 0; a < P->ndim; ++a)
    if (!st->u[a]) return fail(PSTD_E_INVALID_ARG, "u[%d] is null", a);
  if (n_steps < 0) return fail(PSTD_E_INVALID_ARG, "n_steps < 0");
  const int pst = prepare_axes(P);
  if (pst != PSTD_OK) return pst;
  if (n_steps == 0 || use_step1d(P)) return PSTD_OK;
  hipGraphExec_t g = nullptr;
  if (n_steps >= kGraphChunk) {
    const int gst = step_graph(P, st, kGraphChunk, &g);
    if (gst != PSTD_OK) return gst;
  }
  if (n_steps % kGraphChunk) return step_graph(P, st, n_steps % kGraphChunk, &g);
  return PSTD_OK;
}

int pstd_plan_set_path(pstd_plan P, int32_t path) {
  if (!P) return fail(PSTD_E_INVALID_ARG, "null plan");
  if (path < PSTD_PATH_AUTO || path > PSTD_PATH_FFT_GENERIC) return fail(PSTD_E_INVALID_ARG, "bad path");
  if (path == PSTD_PATH_FFT || path == PSTD_PATH_FFT_GENERIC) {
    bool any = false;
    for (int a = 0; a < P->ndim; ++a) any = any || P->fft[a].ok;
    if (!any) return fail(PSTD_E_UNSUPPORTED, "no axis has 2(n-1) = 16 x 2^a 3^b 5^c within the FFT capacity");
  }
  if (path == PSTD_PATH_FUSED &&
      !(P->ndim == 2 && P->prec == PSTD_FP32 &&
        phase2d_supported(static_cast<int>(P->n[0]), static_cast<int>(P->n[1]))))
    return fail(PSTD_E_UNSUPPORTED, "the fused path needs a 2D FP32 plan of at most 512 x 512 nodes");
  const int old = P->path;
  P->path = path;
  const int pst = prepare_axes(P);
  if (pst != PSTD_OK) {
    P->path = old;
    return pst;
  }
  P->use_th = path != PSTD_PATH_STORED;
  P->fft_pow2 = path != PSTD_PATH_FFT_GENERIC;
  drop_graphs(P);  // captured graphs may belong to the other path
  return PSTD_OK;
}

int pstd_apply_axis(pstd_plan P, pstd_state* st, int32_t axis, int32_t which) {
  if (!P || !st || !st->p) return fail(PSTD_E_INVALID_ARG, "null plan/state/p");
  if (axis < -1 || axis >= P->ndim || which < 0 || which > 1) return fail(PSTD_E_INVALID_ARG, "bad axis/which");
  if (axis == -1) {
    for (int a = 0; a < P->ndim; ++a)
      if (!st->u[a]) return fail(PSTD_E_INVALID_ARG, "u[%d] is null", a);
    if (use_fused2d(P)) {
      PSTD_HIP(launch_phase2d_one(which, P->G[0], P->G[1], P->D[0], P->D[1], static_cast<float*>(st->p),
                                  static_cast<float*>(st->u[0]), static_cast<float*>(st->u[1]),
                                  static_cast<const float*>(P->c2map), static_cast<int>(P->n[0]),
                                  static_cast<int>(P->n[1]), P->stream));
      return PSTD_OK;
    }
    const int pst = prepare_axes(P);
    if (pst != PSTD_OK) return pst;
    hipError_t e = hipSuccess;
    if (which == 0 && velocity_fft_multi(P, st, P->stream, &e)) {
      PSTD_HIP(e);
      return PSTD_OK;
    }
    for (int a = 0; a < P->ndim; ++a) {
      const int st2 = pstd_apply_axis(P, st, a, which);
      if (st2 != PSTD_OK) return st2;
    }
    return PSTD_OK;
  }
  if (!st->u[axis]) return fail(PSTD_E_INVALID_ARG, "u[%d] is null", axis);
  const int pst = prepare_axes(P);
  if (pst != PSTD_OK) return pst;
  if (which == 0) PSTD_HIP(apply_op(P, axis, 0, st->p, st->u[axis], 1.0, 1.0, nullptr, P->stream));
  else PSTD_HIP(apply_op(P, axis, 1, st->u[axis], st->p, 1.0, 1.0, P->c2map, P->stream));
  return PSTD_OK;
}

int pstd_combine_R(const float* p_dirichlet, const float* p_neumann, double R, float* p_out, int64_t count,
                   void* hip_stream) {
  if (count < 0) return fail(PSTD_E_INVALID_ARG, "count < 0");
  if (!std::isfinite(R)) return fail(PSTD_E_INVALID_ARG, "R must be finite");
  if (count == 0) return PSTD_OK;
  if (!p_dirichlet || !p_neumann || !p_out) return fail(PSTD_E_INVALID_ARG, "null pointer");
  const float* f[2] = {p_neumann, p_dirichlet};
  const float w[2] = {static_cast<float>(0.5 * (1.0 + R)), static_cast<float>(0.5 * (1.0 - R))};
  PSTD_HIP(launch_combine(f, w, 2, p_out, count, static_cast<hipStream_t>(hip_stream)));
  return PSTD_OK;
}

int pstd_face_weights(int32_t ndim, const double* R, int32_t* bc_out, double* w_out) {
  if (ndim < 1 || ndim > 3) return fail(PSTD_E_INVALID_ARG, "ndim must be 1..3");
  if (!R || !bc_out || !w_out) return fail(PSTD_E_INVALID_ARG, "null pointer");
  for (int i = 0; i < 2 * ndim; ++i)
    if (!std::isfinite(R[i])) return fail(PSTD_E_INVALID_ARG, "R[%d] is not finite", i);
  // per axis: the four basic walls (N,N), (N,D), (D,N), (D,D) are the columns of the image matrix; the
  // weight of column c is (1/4) sum_j M[j][c] r[j] with r = (R_L, 1, R_R, R_L R_R)
  static const int M[4][4] = {{1, 1, -1, -1}, {1, 1, 1, 1}, {1, -1, 1, -1}, {1, -1, -1, 1}};
  static const int walls[4][2] = {{PSTD_NEUMANN, PSTD_NEUMANN}, {PSTD_NEUMANN, PSTD_DIRICHLET},
                                  {PSTD_DIRICHLET, PSTD_NEUMANN}, {PSTD_DIRICHLET, PSTD_DIRICHLET}};
  double w1[3][4];
  for (int a = 0; a < ndim; ++a) {
    const double RL = R[2 * a], RR = R[2 * a + 1];
    const double r[4] = {RL, 1.0, RR, RL * RR};
    for (int c = 0; c < 4; ++c) {
      double acc = 0.0;
      for (int j = 0; j < 4; ++j) acc += M[j][c] * r[j];
      w1[a][c] = 0.25 * acc;
    }
  }
  // field f = sum_a c_a 4^(ndim-1-a): its weight is the product of the axes' weights
  const int nf = 1 << (2 * ndim);
  for (int f = 0; f < nf; ++f) {
    double w = 1.0;
    for (int a = 0; a < ndim; ++a) {
      const int c = (f >> (2 * (ndim - 1 - a))) & 3;
      w *= w1[a][c];
      bc_out[f * 2 * ndim + 2 * a] = walls[c][0];
      bc_out[f * 2 * ndim + 2 * a + 1] = walls[c][1];
    }
    w_out[f] = w;
  }
  return PSTD_OK;
}

int pstd_combine_fields(const float* const* fields, const double* w, int32_t nfields, float* p_out, int64_t count,
                        void* hip_stream) {
  if (!fields || !w || !p_out) return fail(PSTD_E_INVALID_ARG, "null pointer");
  if (nfields < 1 || nfields > 64) return fail(PSTD_E_INVALID_ARG, "nfields must be 1..64");
  if (count < 0) return fail(PSTD_E_INVALID_ARG, "count < 0");
  for (int i = 0; i < nfields; ++i)
    if (!fields[i]) return fail(PSTD_E_INVALID_ARG, "fields[%d] is null", i);
  if (count == 0) return PSTD_OK;
  float wf[64];
  for (int i = 0; i < nfields; ++i) wf[i] = static_cast<float>(w[i]);
  PSTD_HIP(launch_combine(fields, wf, nfields, p_out, count, static_cast<hipStream_t>(hip_stream)));
  return PSTD_OK;
}

int pstd_check_finite(pstd_plan P, const pstd_state* st) {
  if (!P || !st || !st->p) return fail(PSTD_E_INVALID_ARG, "null plan/state");
  PSTD_HIP(hipMemsetAsync(P->flag, 0, sizeof(int), P->stream));
  PSTD_HIP(launch_nonfinite(P->prec, st->p, numel_p(P), P->flag, P->stream));
  for (int a = 0; a < P->ndim; ++a)
    if (st->u[a]) PSTD_HIP(launch_nonfinite(P->prec, st->u[a], numel_u(P, a), P->flag, P->stream));
  int h = 0;
  PSTD_HIP(hipMemcpyAsync(&h, P->flag, sizeof(int), hipMemcpyDeviceToHost, P->stream));
  PSTD_HIP(hipStreamSynchronize(P->stream));
  return h ? fail(PSTD_E_NONFINITE, "non-finite value in the state") : PSTD_OK;
}

int pstd_axis_operator(int64_t n, int32_t bc_left, int32_t bc_right, double dx, int32_t which, double* out) {
  if (!out) return fail(PSTD_E_INVALID_ARG, "out is null");
  if (n < 3 || n > 4097) return fail(PSTD_E_INVALID_ARG, "n must be in [3, 4097]");
  const bool per = bc_left == PSTD_PERIODIC && bc_right == PSTD_PERIODIC;
  const bool half = half_wall(bc_right);
  if (!per && ((bc_left != PSTD_NEUMANN && bc_left != PSTD_DIRICHLET) ||
               (bc_right != PSTD_NEUMANN && bc_right != PSTD_DIRICHLET && !half)))
    return fail(PSTD_E_INVALID_ARG, "bad boundary condition");
  if (!(dx > 0) || which < 0 || which > 5) return fail(PSTD_E_INVALID_ARG, "bad dx or which");
  if (which >= 2) {
    if (per || half) return fail(PSTD_E_UNSUPPORTED, "collocated and interpolation operators need walls on nodes");
    int rows = 0, cols = 0;
    const std::vector<double> m = resample_table(static_cast<int>(n), axis_case(bc_left, bc_right), which, &rows, &cols);
    const double s = which <= 3 ? 1.0 / dx : 1.0;
    for (size_t i = 0; i < m.size(); ++i) out[i] = m[i] * s;
    return PSTD_OK;
  }
  const AxisTables& t = axis_tables(static_cast<int>(n), axis_case(bc_left, bc_right));
  const std::vector<double>& m = which == 0 ? t.G : t.D;
  for (size_t i = 0; i < m.size(); ++i) out[i] = m[i] / dx;
  return PSTD_OK;
}

int pstd_axis_operator_structure(int64_t n, int32_t bc_left, int32_t bc_right, double dx, int32_t which, double* f,
                                 double* g, double* w, double* resid) {
  if (!f || !g || !w) return fail(PSTD_E_INVALID_ARG, "null output");
  if (n < 3 || n > 4097) return fail(PSTD_E_INVALID_ARG, "n must be in [3, 4097]");
  const bool per = bc_left == PSTD_PERIODIC && bc_right == PSTD_PERIODIC;
  const int m = (per || half_wall(bc_right)) ? static_cast<int>(n) : static_cast<int>(n) - 1;
  int rows = 0, cols = 0;
  switch (which) {
    case 0: rows = m; cols = static_cast<int>(n); break;
    case 1: rows = static_cast<int>(n); cols = m; break;
    case 2: rows = cols = static_cast<int>(n); break;
    case 3: rows = cols = m; break;
    case 4: rows = m; cols = static_cast<int>(n); break;
    case 5: rows = static_cast<int>(n); cols = m; break;
    default: return fail(PSTD_E_INVALID_ARG, "bad which");
  }
  std::vector<double> A(static_cast<size_t>(rows) * cols);
  const int st = pstd_axis_operator(n, bc_left, bc_right, dx, which, A.data());
  if (st != PSTD_OK) return st;
  std::vector<double> fv, gv;
  double wv[4], r = 0.0;
  const bool ok = toeplitz_hankel(A.data(), rows, cols, kThTol, &fv, &gv, wv, &r);
  if (resid) *resid = r;
  if (!ok) return fail(PSTD_E_UNSUPPORTED, "operator has no Toeplitz-plus-Hankel form (residual %g)", r);
  for (size_t i = 0; i < fv.size(); ++i) {
    f[i] = fv[i];
    g[i] = gv[i];
  }
  for (int i = 0; i < 4; ++i) w[i] = wv[i];
  return PSTD_OK;
}

int pstd_apply_axis_operator(pstd_plan P, int32_t axis, int32_t which, const void* in, void* out) {
  if (!P || !in || !out) return fail(PSTD_E_INVALID_ARG, "null plan/in/out");
  if (axis < 0 || axis >= P->ndim || which < 2 || which > 5) return fail(PSTD_E_INVALID_ARG, "bad axis/which");
  if (in == out) return fail(PSTD_E_INVALID_ARG, "in and out must be different buffers");
  if (axis_periodic(P, axis) || axis_half_wall(P, axis))
    return fail(PSTD_E_UNSUPPORTED, "collocated and interpolation operators need walls on nodes");
  const int n = static_cast<int>(P->n[axis]);
  if (n > 4097) return fail(PSTD_E_UNSUPPORTED, "axis %d: dense operators are limited to 4097 nodes", axis);
  DevOperator& op = P->R[axis][which - 2];
  if (!op.data) {
    int rows = 0, cols = 0;
    const std::vector<double> m =
        resample_table(n, axis_case(P->bc[2 * axis], P->bc[2 * axis + 1]), which, &rows, &cols);
    const int st = upload_operator(P, m, rows, cols, which <= 3 ? 1.0 / P->dx : 1.0, &op);
    if (st != PSTD_OK) return st;
  }
  PSTD_HIP(contract(P, op, axis, in, out, 1.0, 0.0, nullptr, P->stream));
  return PSTD_OK;
}

int pstd_plan_get_operator(pstd_plan P, int32_t axis, int32_t which, double* out) {
  if (!P || !out) return fail(PSTD_E_INVALID_ARG, "null pointer");
  if (axis < 0 || axis >= P->ndim || which < 0 || which > 1) return fail(PSTD_E_INVALID_ARG, "bad axis/which");
  const int est = ensure_dense(P, axis);
  if (est != PSTD_OK) return est;
  const DevOperator& op = which == 0 ? P->G[axis] : P->D[axis];
  const size_t cnt = static_cast<size_t>(op.Mp) * op.Kp;
  if (P->prec == PSTD_FP64) {
    std::vector<double> h(cnt);
    PSTD_HIP(hipMemcpy(h.data(), op.data, cnt * 8, hipMemcpyDeviceToHost));
    for (int i = 0; i < op.M; ++i)
      for (int k = 0; k < op.K; ++k) out[static_cast<size_t>(i) * op.K + k] = h[static_cast<size_t>(i) * op.Kp + k];
  } else if (P->prec == PSTD_FP32) {
    std::vector<float> h(cnt);
    PSTD_HIP(hipMemcpy(h.data(), op.data, cnt * 4, hipMemcpyDeviceToHost));
    for (int i = 0; i < op.M; ++i)
      for (int k = 0; k < op.K; ++k) out[static_cast<size_t>(i) * op.K + k] = h[static_cast<size_t>(i) * op.Kp + k];
  } else {
    std::vector<uint16_t> h(2 * cnt);
    PSTD_HIP(hipMemcpy(h.data(), op.data, cnt * 4, hipMemcpyDeviceToHost));
    for (int i = 0; i < op.M; ++i)
      for (int k = 0; k < op.K; ++k) {
        const size_t a = static_cast<size_t>(i) * op.Kp + k;
        out[static_cast<size_t>(i) * op.K + k] =
            static_cast<double>(bf16_to_float(h[a])) + static_cast<double>(bf16_to_float(h[cnt + a]));
      }
  }
  return PSTD_OK;
}

}  // extern "C"
